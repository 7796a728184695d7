"""Differentiation and least-squares migration on top of the C ABI.

Migration (data -> image, Algorithm 1) is linear in the surface plane, and
mig_demigrate is its exact transpose for the real inner product
<a, b> = Re sum conj(a) b.  This module exposes both as
``torch.autograd.Function`` objects (each one's backward is the other kernel),
least-squares migration by CGLS, and depth checkpoints of the extrapolated
wavefield.  All operator applications run in the library's kernels; the CG
vector updates and scalars are device tensor arithmetic between them.
"""
from __future__ import annotations

import torch

from . import mig


class Migrate(torch.autograd.Function):
    """image = A(data): forward mig_migrate, backward mig_demigrate."""

    @staticmethod
    def forward(ctx, data, vel, omega, tab32, desc):
        ctx.save_for_backward(vel, omega, tab32)
        ctx.desc = desc
        ctx.nw = data.shape[1]
        return mig.migrate(data.contiguous(), vel, omega, tab32, desc)

    @staticmethod
    def backward(ctx, grad_image):
        vel, omega, tab32 = ctx.saved_tensors
        g = mig.demigrate(grad_image.contiguous().to(torch.float64), vel, omega, tab32, ctx.desc)
        return g, None, None, None, None


class Demigrate(torch.autograd.Function):
    """data = A^T(image): forward mig_demigrate, backward mig_migrate."""

    @staticmethod
    def forward(ctx, image, vel, omega, tab32, desc):
        ctx.save_for_backward(vel, omega, tab32)
        ctx.desc = desc
        return mig.demigrate(image.contiguous(), vel, omega, tab32, desc)

    @staticmethod
    def backward(ctx, grad_data):
        vel, omega, tab32 = ctx.saved_tensors
        g = mig.migrate(grad_data.contiguous().to(torch.complex64), vel, omega, tab32, ctx.desc)
        return g, None, None, None, None


def migrate_fn(data, vel, omega, tab32, desc):
    return Migrate.apply(data, vel, omega, tab32, desc)


def demigrate_fn(image, vel, omega, tab32, desc):
    return Demigrate.apply(image, vel, omega, tab32, desc)


def _dot_data(a, b):
    """Re <a, b> on planes, as a 0-d float64 device tensor (no host sync)."""
    return torch.sum(a.real.double() * b.real.double() + a.imag.double() * b.imag.double())


def _dot_img(a, b):
    return torch.sum(a * b)


def cgls(d_obs, vel, omega, tab32, desc, niter=10, m0=None):
    """Least-squares migration: minimize ||A^T m - d_obs||^2 over real images m
    ([nz][nx] float64) by conjugate gradients on the normal equations (CGLS),
    with modelling A^T = mig_demigrate and its adjoint A = mig_migrate.

    The CG scalars stay on the device (0-d tensors), so the iterations queue
    without host round trips; the history is read back once at the end.
    Started from zero, CGLS converges to the minimum-norm least-squares
    solution, i.e. for noise-free data to the part of the true model that the
    operator can recover (its projection onto the range of A).

    Returns (m, history) where history holds ||r|| / ||d_obs|| per iteration."""
    nz, nx = vel.shape
    if m0 is None:
        m = torch.zeros((nz, nx), dtype=torch.float64, device=d_obs.device)
        r = d_obs.clone()
    else:
        m = m0.clone()
        r = d_obs - mig.demigrate(m, vel, omega, tab32, desc)
    s = mig.migrate(r, vel, omega, tab32, desc)
    p = s.clone()
    gamma = _dot_img(s, s)
    dn = torch.sqrt(_dot_data(d_obs, d_obs))
    hist = [torch.sqrt(_dot_data(r, r)) / dn]
    zero = torch.zeros((), dtype=torch.float64, device=d_obs.device)
    for _ in range(niter):
        q = mig.demigrate(p, vel, omega, tab32, desc)
        qq = _dot_data(q, q)
        # a zero direction (converged exactly) leaves everything unchanged
        alpha = torch.where(qq > 0, gamma / torch.where(qq > 0, qq, 1.0), zero)
        m = m + alpha * p
        r = (r - alpha * q).to(torch.complex64)
        s = mig.migrate(r, vel, omega, tab32, desc)
        gnew = _dot_img(s, s)
        beta = torch.where(gamma > 0, gnew / torch.where(gamma > 0, gamma, 1.0), zero)
        p = s + beta * p
        gamma = gnew
        hist.append(torch.sqrt(_dot_data(r, r)) / dn)
    return m, [float(h) for h in torch.stack(hist).cpu()]


def migrate_checkpointed(data, vel, omega, tab32, desc, every=32, ws=None):
    """mig_migrate in segments of `every` depth steps, keeping the wavefield
    plane at depths 0, every, 2*every, ... and the last depth.  Returns
    (image, {depth index: plane}).
    A later call of mig.extrapolate from any checkpoint reproduces the same
    planes and rows (bit for bit: the kernels are deterministic)."""
    nx, nw = data.shape
    nz = vel.shape[0]
    image = torch.empty((nz, nx), dtype=torch.float64, device=data.device)
    mig.image_into(data, image[0])
    cps = {0: data.clone()}
    cur = data
    k = 0
    while k < nz - 1:
        n = min(every, nz - 1 - k)
        nxt, _ = mig.extrapolate(cur, vel[k:k + n].contiguous(), omega, tab32, desc, n,
                                 rows_out=image[k + 1:k + 1 + n], ws=ws)
        k += n
        cur = nxt
        cps[k] = nxt
    return image, cps
