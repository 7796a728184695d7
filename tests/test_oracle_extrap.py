"""Pins of the oracle's extrapolation (Eq. 1), recursion (Algorithm 1) and imaging.

* P4: in constant velocity, with the wavenumber on a table entry, n steps of the
  zero-boundary Eq. 1 on an interior packet equal F^-1 H^n F u (convolution
  theorem), and stay within n * design error of the exact phase shift
  exp(i kz dz) (coded here in physical units, with dz != dx so a wrong dz/dx
  factor shows).
* P5: tiny grids against dense matrices E_k(omega) built from a random table
  and an exact-rational nearest-entry look-up.
* P12: constant velocity never increases the wavefield energy.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1912_05529_amd import synth


def _nearest_exact(desc, omega, v):
    """Nearest table entry to omega/v in exact rational arithmetic (ties up)."""
    if not (v > 0) or math.isnan(v):
        return 0
    kmin = Fraction(desc.kmin)
    dk = (Fraction(desc.kmax) - kmin) / (desc.nk - 1)
    dk_f = Fraction((desc.kmax - desc.kmin) / (desc.nk - 1))
    t = (Fraction(omega) / Fraction(float(v)) - kmin) / dk_f
    j = math.floor(t + Fraction(1, 2))
    del dk
    return min(max(j, 0), desc.nk - 1), t


def _resp(h, theta):
    H = np.full(theta.shape, h[0], dtype=np.complex128)
    for n in range(1, h.size):
        H = H + 2.0 * h[n] * np.cos(n * theta)
    return H


def test_p4_constant_velocity_matches_convolution_theorem_and_phase_shift():
    dx, dz = 10.0, 5.0
    desc = synth.TableDesc(ntaps=25, nk=64, kmin=0.03, kmax=0.25, dx=dx, dz=dz)
    tab, _, pe, _ = oracle.design_table(desc)
    j0 = 30
    dk = (desc.kmax - desc.kmin) / (desc.nk - 1)
    k0 = desc.kmin + j0 * dk
    v = 1000.0
    om = np.array([k0 * v])
    nx, nsteps = 400, 8
    x = np.arange(nx)
    win = np.where((x >= 150) & (x < 250), np.sin(math.pi * (x - 150) / 100.0) ** 2, 0.0)
    theta0 = 0.3 * k0 * dx
    u = (win * np.exp(1j * theta0 * x))[:, None]
    vel = np.full((nsteps, nx), v, np.float32)
    assert oracle.table_index(desc, om, vel[:1])[0, :, 0].tolist() == [j0] * nx

    out, _ = oracle.extrapolate(desc, tab, om, vel, u, nsteps, rows=False)

    npad = 1024
    theta = 2.0 * math.pi * np.fft.fftfreq(npad)
    U = np.fft.fft(u[:, 0], npad)
    exact_fir = np.fft.ifft(_resp(tab[j0], theta) ** nsteps * U)[:nx]
    err = np.linalg.norm(out[:, 0] - exact_fir) / np.linalg.norm(exact_fir)
    assert err < 1e-13, err

    kx = theta / dx
    kz2 = k0 ** 2 - kx ** 2
    D = np.where(kz2 >= 0, np.exp(1j * np.sqrt(np.abs(kz2)) * dz),
                 np.exp(-np.sqrt(np.abs(kz2)) * dz))
    exact_ps = np.fft.ifft(D ** nsteps * U)[:nx]
    passband = np.abs(theta) <= k0 * dx * math.sin(math.radians(desc.theta_max_deg))
    eps = np.abs(_resp(tab[j0], theta) - D)[passband].max()
    u_out = np.sqrt(np.sum(np.abs(U[~passband]) ** 2) / npad)
    bound = nsteps * eps * np.linalg.norm(u) + 2.0 * nsteps * u_out
    diff = np.linalg.norm(out[:, 0] - exact_ps)
    assert diff <= bound, (diff, bound)
    assert diff / np.linalg.norm(u) < 0.05
    # the conjugate (wrong-sign) propagator is far away
    wrong = np.fft.ifft(np.conj(D) ** nsteps * U)[:nx]
    assert np.linalg.norm(out[:, 0] - wrong) / np.linalg.norm(u) > 0.5


def _brute_force_image(desc, tab, om, vel, data):
    nz, nx = vel.shape
    nw = om.size
    M = tab.shape[1] - 1
    img = np.zeros((nz, nx))
    P = data.astype(np.complex128).copy()
    img[0] = P.real.sum(axis=1)
    for k in range(nz - 1):
        Q = np.zeros_like(P)
        for r in range(nw):
            E = np.zeros((nx, nx), np.complex128)
            for xo in range(nx):
                j, _ = _nearest_exact(desc, om[r], float(vel[k, xo]))
                for xi in range(nx):
                    n = xo - xi
                    if abs(n) <= M:
                        E[xo, xi] = tab[j, abs(n)]
            Q[:, r] = E @ P[:, r]
        P = Q
        img[k + 1] = P.real.sum(axis=1)
    return img, P


@pytest.mark.parametrize("nx,nw,nz,ntaps", [(16, 4, 5, 5), (8, 3, 5, 25), (1, 1, 3, 3),
                                             (5, 2, 1, 7), (13, 4, 4, 1), (16, 2, 5, 9)])
def test_p5_brute_force_dense_matrices(nx, nw, nz, ntaps):
    rng = np.random.default_rng(100 + nx * 7 + nw * 3 + nz + ntaps)
    desc = synth.TableDesc(ntaps=ntaps, nk=8, kmin=0.02, kmax=0.45, dx=10.0, dz=10.0)
    K = (ntaps - 1) // 2 + 1
    tab = (rng.standard_normal((desc.nk, K)) + 1j * rng.standard_normal((desc.nk, K))) / K
    om = synth.omegas(nw, 5.0, 55.0)
    vel = rng.uniform(700.0, 2500.0, (nz, nx)).astype(np.float32)
    data = rng.standard_normal((nx, nw)) + 1j * rng.standard_normal((nx, nw))
    ref, Pref = _brute_force_image(desc, tab, om, vel, data)
    img = oracle.migrate(desc, tab, om, vel, data)
    scale = np.abs(ref).max()
    assert np.abs(img - ref).max() <= 1e-13 * scale
    if nz > 1:
        out, rows = oracle.extrapolate(desc, tab, om, vel, data, nz - 1)
        assert np.abs(out - Pref).max() <= 1e-13 * np.abs(Pref).max()
        assert np.abs(rows - ref[1:]).max() <= 1e-13 * scale


def test_p12_energy_never_grows_in_constant_velocity(cfg1, cfg1_table):
    tab = cfg1_table[0]
    rng = np.random.default_rng(9)
    nx, nw = 128, 6
    om = cfg1.omega[::11][:nw]
    vel = np.full((1, nx), 1000.0, np.float32)
    P = rng.standard_normal((nx, nw)) + 1j * rng.standard_normal((nx, nw))
    for _ in range(30):
        Q, _ = oracle.extrapolate(cfg1.desc, tab, om, vel, P, 1, rows=False)
        e0 = np.linalg.norm(P, axis=0)
        e1 = np.linalg.norm(Q, axis=0)
        assert np.all(e1 <= e0 * (1 + 1e-14))
        P = Q


def test_image_is_real_part_sum_over_frequencies():
    rng = np.random.default_rng(3)
    P = rng.standard_normal((7, 5)) + 1j * rng.standard_normal((7, 5))
    row = oracle.image(P)
    for x in range(7):
        s = 0.0
        for r in range(5):
            s += P[x, r].real
        assert row[x] == s
