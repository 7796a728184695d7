"""Pins for the 3-D extension of the oracle (Sec. II: the explicit method
extends to 3-D, where Eq. (1) becomes a 2-D sum over a square stencil of
circularly symmetric filters).

* the 2-D design against a closed form (one coefficient: the weighted mean of
  the phase-shift target) and against a textbook weighted least-squares solve
  built from the *expanded* (2M+1)^2 filter;
* stability and passband error re-evaluated by FFT of the expanded filter on
  a grid finer than the oracle's own check grid;
* the 3-D step against brute force (numpy, per output point), against
  scipy's 2-D convolution for constant velocity, and against the convolution
  theorem for an impulse carried several steps;
* a single y line collapsing to the 2-D path, and a diffraction hyperboloid
  focusing on its scatterer.
"""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
from paper_1912_05529_amd import synth


def expand(c, M):
    """(2M+1) x (2M+1) filter h[n1+M][n2+M] = c[a(a+1)/2 + b], a = max, b = min."""
    h = np.zeros((2 * M + 1, 2 * M + 1), np.complex128)
    for n1 in range(-M, M + 1):
        for n2 in range(-M, M + 1):
            a, b = max(abs(n1), abs(n2)), min(abs(n1), abs(n2))
            h[n1 + M, n2 + M] = c[a * (a + 1) // 2 + b]
    return h


def target(desc, j, tx, ty):
    """Phase-shift operator and band weights of entry j at (tx, ty)."""
    dk = (desc.kmax - desc.kmin) / (desc.nk - 1)
    kappa = (desc.kmin + j * dk) * desc.dx
    zeta = desc.dz / desc.dx
    r2 = tx ** 2 + ty ** 2
    prop = r2 <= kappa ** 2
    D = np.where(prop, np.exp(1j * zeta * np.sqrt(np.where(prop, kappa ** 2 - r2, 0.0))),
                 np.exp(-zeta * np.sqrt(np.where(prop, 0.0, r2 - kappa ** 2))))
    r = np.sqrt(r2)
    edge = kappa * math.sin(math.radians(desc.theta_max_deg))
    w = np.where(r <= edge, desc.w_pass, np.where(r <= kappa, desc.w_trans, desc.w_evan))
    return D, w, r <= edge


def grid(L):
    t = (np.arange(L) + 0.5) * math.pi / L
    return np.meshgrid(t, t, indexing="ij")


def response(c, M, tx, ty):
    """H = sum over all (n1, n2) of h exp(-i (n1 tx + n2 ty)), expanded filter."""
    h = expand(c, M)
    n = np.arange(-M, M + 1)
    ex = np.exp(-1j * n[:, None, None] * tx.ravel()[None, None, :])
    ey = np.exp(-1j * n[None, :, None] * ty.ravel()[None, None, :])
    return np.einsum("ab,abp->p", h, ex * ey).reshape(tx.shape)


def small_desc(ntaps, nk=8, **kw):
    return synth.table2d_for(ntaps, nk, 5.0, 40.0, 750.0, 2000.0, 10.0, 10.0,
                             ngrid=kw.pop("ngrid", 40), ncheck=kw.pop("ncheck", 160), **kw)


def test_design2d_single_coefficient_is_weighted_mean():
    desc = small_desc(1, nreweight=0, lam=1e-3)
    tab, _, _, _ = oracle.design_table_2d(desc, apply_scale=False)
    tx, ty = grid(desc.ngrid)
    for j in range(desc.nk):
        D, w, _ = target(desc, j, tx, ty)
        want = np.sum(w * D) / (np.sum(w) + 1e-3)
        assert abs(tab[j, 0] - want) <= 1e-13 * max(1.0, abs(want))


@pytest.mark.parametrize("ntaps,nreweight", [(3, 0), (5, 0), (7, 0), (5, 2), (7, 1), (7, 3)])
def test_design2d_matches_weighted_lstsq_of_expanded_filter(ntaps, nreweight):
    """Weighted least squares with the basis built from the expanded filter,
    solved by numpy's lstsq, followed by `nreweight` passes that multiply the
    weight of every design point with |H| > 1 by 1 + beta (|H| - 1) / tau
    and solve again."""
    M = (ntaps - 1) // 2
    NU = (M + 1) * (M + 2) // 2
    lam = 1e-6
    desc = small_desc(ntaps, nreweight=nreweight, lam=lam)
    tab, _, _, _ = oracle.design_table_2d(desc, apply_scale=False)
    tx, ty = grid(desc.ngrid)
    # columns: response of the expanded filter with one unique coefficient set
    cols = []
    for u in range(NU):
        e = np.zeros(NU)
        e[u] = 1.0
        cols.append(response(e, M, tx, ty).ravel())
    A = np.stack(cols, axis=1)
    assert np.max(np.abs(A.imag)) < 1e-12          # the expanded filters are real-symmetric
    A = A.real
    moved = 0.0
    for j in (0, desc.nk // 2, desc.nk - 1):
        D, w, _ = target(desc, j, tx, ty)
        w = w.ravel().astype(np.float64)

        def solve(wt):
            sw = np.sqrt(wt)
            Aw = np.vstack([A * sw[:, None], math.sqrt(lam) * np.eye(NU)])
            bw = np.concatenate([D.ravel() * sw, np.zeros(NU)])
            return np.linalg.lstsq(Aw, bw, rcond=None)[0]

        want = solve(w)
        first = want
        for _ in range(nreweight):
            excess = np.abs(A @ want) - 1.0
            w = w * (1.0 + desc.beta * np.maximum(excess, 0.0) / desc.tau)
            want = solve(w)
        moved = max(moved, float(np.max(np.abs(want - first)) / np.max(np.abs(want))))
        err = np.max(np.abs(tab[j] - want)) / np.max(np.abs(want))
        assert err <= 1e-10, (j, err)
    if nreweight:
        # the passes change the taps far beyond the agreement asked for above
        assert moved > 1e-6, moved


@pytest.mark.parametrize("ntaps", [5, 11])
def test_design2d_stable_on_fine_grid_and_passerr_consistent(ntaps):
    M = (ntaps - 1) // 2
    desc = small_desc(ntaps, nk=6, ngrid=48, ncheck=96)
    tab, maxgain, passerr, scale = oracle.design_table_2d(desc)
    Lf = 1024
    for j in range(desc.nk):
        H = np.fft.fft2(expand(tab[j], M), s=(Lf, Lf))     # every (theta_x, theta_y) on a 1024^2 grid
        assert np.abs(H).max() <= 1.0, (j, np.abs(H).max())
        assert maxgain[j] <= 1.0 - desc.margin + 1e-15
        assert 0.0 < scale[j] <= 1.0
        tx, ty = grid(desc.ngrid)
        D, _, pas = target(desc, j, tx, ty)
        Hd = response(tab[j], M, tx, ty)
        mine = np.max(np.abs(Hd - D)[pas]) if pas.any() else 0.0
        assert abs(mine - passerr[j]) <= 1e-12


def test_design2d_beats_the_identity_filter_in_the_passband():
    desc = small_desc(11, nk=4, ngrid=48, ncheck=96)
    tab, _, passerr, _ = oracle.design_table_2d(desc)
    tx, ty = grid(desc.ngrid)
    for j in range(desc.nk):
        D, _, pas = target(desc, j, tx, ty)
        if not pas.any():
            continue
        ident = np.max(np.abs(1.0 - D)[pas])
        assert passerr[j] < 0.5 * ident


def _brute_force(desc, tab, omega, vel, data):
    """Per output point, the expanded filter of its (omega, v) applied to the
    zero-padded plane, one depth step after another."""
    M = (desc.ntaps - 1) // 2
    nx, ny, nw = data.shape
    nz = vel.shape[0]
    idx = oracle.table_index(desc, omega, vel.reshape(nz, nx * ny)).reshape(nz, nx, ny, nw)
    H = [expand(tab[j], M) for j in range(tab.shape[0])]
    P = data.copy()
    img = np.zeros((nz, nx, ny))
    img[0] = P.real.sum(axis=2)
    for k in range(1, nz):
        Pp = np.zeros((nx + 2 * M, ny + 2 * M, nw), np.complex128)
        Pp[M:M + nx, M:M + ny] = P
        Q = np.zeros_like(P)
        for x in range(nx):
            for y in range(ny):
                for r in range(nw):
                    # out(x, y) = sum h[n1][n2] P(x - n1, y - n2); h is symmetric
                    patch = Pp[x:x + 2 * M + 1, y:y + 2 * M + 1, r][::-1, ::-1]
                    Q[x, y, r] = np.sum(H[idx[k - 1, x, y, r]] * patch)
        P = Q
        img[k] = P.real.sum(axis=2)
    return img


@pytest.mark.parametrize("ntaps,nx,ny", [(5, 7, 6), (11, 6, 13), (3, 1, 5)])
def test_migrate3d_matches_brute_force(ntaps, nx, ny):
    vol = synth.random_volume(31 + nx, nx, ny, 4, 3, ntaps=ntaps, nk=16, layered=False)
    tab = oracle.design_table_2d(vol.desc)[0]
    got = oracle.migrate3d(vol.desc, tab, vol.omega, vol.vel, vol.data)
    want = _brute_force(vol.desc, tab, vol.omega, vol.vel, vol.data)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_migrate3d_constant_velocity_is_scipy_convolution():
    vol = synth.random_volume(41, 17, 12, 3, 4, ntaps=7, nk=16)
    vol.vel[:] = 1100.0
    tab = oracle.design_table_2d(vol.desc)[0]
    got = oracle.migrate3d(vol.desc, tab, vol.omega, vol.vel, vol.data)
    idx = oracle.table_index(vol.desc, vol.omega, np.full((1, 1), 1100.0, np.float32))[0, 0]
    P = vol.data.copy()
    for k in range(1, 3):
        for r in range(vol.nw):
            P[:, :, r] = scipy.signal.convolve2d(P[:, :, r], expand(tab[idx[r]], 3), mode="same")
        assert np.max(np.abs(got[k] - P.real.sum(axis=2))) <= 1e-12 * np.max(np.abs(got[k]))


def test_migrate3d_impulse_obeys_convolution_theorem():
    """An impulse far from the edges, k steps of one filter: the wavefield is
    the inverse 2-D DFT of H^k (exactly, since the support never reaches the
    boundary).  Image rows are the real parts summed over frequencies."""
    M, nx, nsteps = 5, 61, 4
    desc = small_desc(11, nk=8, ngrid=48, ncheck=96)
    tab = oracle.design_table_2d(desc)[0]
    omega = np.array([2 * math.pi * 12.0, 2 * math.pi * 31.0])
    vel = np.full((nsteps + 1, nx, nx), 900.0, np.float32)
    data = np.zeros((nx, nx, 2), np.complex128)
    data[nx // 2, nx // 2, :] = [1.0, 0.5 - 0.25j]
    got = oracle.migrate3d(desc, tab, omega, vel, data)
    idx = oracle.table_index(desc, omega, vel[0, :1, :1])[0, 0]
    for k in range(1, nsteps + 1):
        want = np.zeros((nx, nx))
        for r in range(2):
            Hk = np.fft.fft2(expand(tab[idx[r]], M), s=(nx, nx)) ** k
            # the filter's centre sits at index (M, M): undo that shift k times
            field = np.roll(np.fft.ifft2(Hk), (-k * M + nx // 2, -k * M + nx // 2), axis=(0, 1))
            want += (data[nx // 2, nx // 2, r] * field).real
        assert np.max(np.abs(got[k] - want)) <= 1e-12 * np.max(np.abs(want))


def test_migrate3d_single_line_collapses_to_2d_path():
    """ny = 1: only the n2 = 0 column of each filter touches the data, so the
    result equals the 2-D migration with the 1-D filter h[n] = c(|n|, 0)."""
    vol = synth.random_volume(51, 23, 1, 6, 5, ntaps=9, nk=16)
    tab2 = oracle.design_table_2d(vol.desc)[0]
    M = 4
    tab1 = np.stack([tab2[:, a * (a + 1) // 2] for a in range(M + 1)], axis=1)
    got = oracle.migrate3d(vol.desc, tab2, vol.omega, vol.vel, vol.data)
    want = oracle.migrate(vol.desc, tab1, vol.omega, vol.vel[:, :, 0], vol.data[:, 0, :])
    assert np.max(np.abs(got[:, :, 0] - want)) <= 1e-12 * np.max(np.abs(want))


def test_migrate3d_diffraction_hyperboloid_focuses():
    vol = synth.point_scatterer_3d()
    tab = oracle.design_table_2d(vol.desc)[0]
    img = oracle.migrate3d(vol.desc, tab, vol.omega, vol.vel, vol.data)
    k, x, y = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    e = vol.extra
    assert abs(k - e["iz0"]) <= 1 and abs(x - e["ix0"]) <= 1 and abs(y - e["iy0"]) <= 1
    en = img ** 2
    box = en[k - 5:k + 6, x - 3:x + 4, y - 3:y + 4].sum() / en.sum()
    assert box >= 0.7
    # control: the medium velocity instead of the propagation velocity does not focus
    bad = oracle.migrate3d(vol.desc, tab, vol.omega, 2.0 * vol.vel, vol.data)
    kb, xb, yb = np.unravel_index(np.argmax(np.abs(bad)), bad.shape)
    eb = bad ** 2
    assert eb[e["iz0"] - 5:e["iz0"] + 6, e["ix0"] - 3:e["ix0"] + 4,
              e["iy0"] - 3:e["iy0"] + 4].sum() / eb.sum() < 0.5 * box
