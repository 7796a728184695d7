"""Seeded synthetic inputs: velocity models, frequency sets and f-x sections.

This module serves both the GPU path and the FP64 oracle and holds none of the
migration arithmetic (no extrapolation filters, no table look-up, no imaging).
All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64) and all
generation is FP64.

The paper images the SEG/EAGE salt zero-offset section (Sec. IV); that dataset
is not available here, so these models stand in for it:

* :func:`config1` -- constant medium velocity 2000 m/s, one point scatterer at a
  seeded position; the zero-offset data are the analytic two-way diffraction
  hyperbola convolved with a 20 Hz Ricker wavelet, transformed to omega by a
  direct DFT (forward sign exp(-i omega t)).
* :func:`config2` -- 6-10 seeded dipping layers (1500-4500 m/s) plus a 4800 m/s
  blob-shaped body; +-1 reflectivity at the interfaces; exploding-reflector data
  modelled by phase-shift upward continuation in the laterally averaged
  propagation velocity (an f-k model, not the f-x method), shaped by a 20 Hz
  Ricker amplitude spectrum.
* :func:`random_case` -- small random layered models with random complex data for
  parity sweeps.
* :func:`config3` -- a batch of sections of uneven size (band-limited random data).
* :func:`point_scatterer_3d`, :func:`config5` -- 3-D volumes for the extension to
  2-D extrapolators: an analytic diffraction hyperboloid in constant velocity,
  and a seeded layered volume (1500-4000 m/s) with an ellipsoidal body whose
  exploding-reflector data are modelled by phase shift in the velocity profile
  of the undisturbed layering at the centre of the volume.

Velocities handed to the migration are *propagation* velocities: for zero-offset
(exploding-reflector) data that is half the medium velocity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class TableDesc:
    """Extrapolator-table descriptor (mirrors the C struct ``mig_table_desc``).

    ``kmin``/``kmax`` bound the table axis k = omega / v_prop (rad/m).  The
    remaining fields parameterize the weighted least-squares design; the
    defaults are the ones every configuration uses.
    """

    ntaps: int
    nk: int
    kmin: float
    kmax: float
    dx: float
    dz: float
    theta_max_deg: float = 60.0
    w_pass: float = 1.0
    w_trans: float = 0.01
    w_evan: float = 0.01
    ngrid: int = 1024
    ncheck: int = 8192
    nreweight: int = 30
    lam: float | None = None  # None -> 1e-9 * ngrid
    beta: float = 1.0
    tau: float = 5e-4
    margin: float = 1e-5

    @property
    def half(self) -> int:
        return (self.ntaps - 1) // 2

    @property
    def lam_value(self) -> float:
        return self.lam if self.lam is not None else 1e-9 * self.ngrid


@dataclass
class Section:
    """One 2-D zero-offset section ready for migration."""

    name: str
    nx: int
    nz: int
    dx: float
    dz: float
    omega: np.ndarray          # [nw] float64, rad/s
    vel: np.ndarray            # [nz][nx] float32 propagation velocity, m/s
    data: np.ndarray           # [nx][nw] complex128 surface plane
    desc: TableDesc
    extra: dict = field(default_factory=dict)

    @property
    def nw(self) -> int:
        return int(self.omega.size)


def omegas(nw: int, fmin: float, fmax: float) -> np.ndarray:
    """omega_r = 2 pi (fmin + r (fmax - fmin)/(nw - 1)), endpoints included."""
    r = np.arange(nw, dtype=np.float64)
    if nw == 1:
        return np.array([TWO_PI * fmin])
    return TWO_PI * (fmin + r * (fmax - fmin) / (nw - 1))


def ricker(t: np.ndarray, f: float) -> np.ndarray:
    a = (math.pi * f * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ricker_spectrum(freq: np.ndarray, fp: float) -> np.ndarray:
    """Amplitude spectrum of a Ricker wavelet with peak frequency fp."""
    return (2.0 / math.sqrt(math.pi)) * (freq ** 2 / fp ** 3) * np.exp(-(freq ** 2) / fp ** 2)


def table_for(ntaps: int, nk: int, fmin: float, fmax: float, vmin_prop: float,
              vmax_prop: float, dx: float, dz: float, **kw) -> TableDesc:
    """Table spanning k = omega/v over [omega_min/vmax, omega_max/vmin]."""
    return TableDesc(ntaps=ntaps, nk=nk, kmin=TWO_PI * fmin / vmax_prop,
                     kmax=TWO_PI * fmax / vmin_prop, dx=dx, dz=dz, **kw)


# --------------------------------------------------------------------------- #
# Configuration 1: constant velocity, one point scatterer.
# --------------------------------------------------------------------------- #
def config1(seed: int = 1, nx: int = 128, nz: int = 128, nw: int = 64,
            dx: float = 10.0, dz: float = 10.0, nt: int = 256, dt: float = 0.004,
            v_medium: float = 2000.0, fmin: float = 5.0, fmax: float = 40.0,
            f_ricker: float = 20.0, ntaps: int = 25, nk: int = 512) -> Section:
    rng = np.random.default_rng(seed)
    ix0 = int(rng.integers(32, 97))
    iz0 = int(rng.integers(20, 61))
    x = np.arange(nx) * dx
    x0, z0 = ix0 * dx, iz0 * dz
    t_d = 2.0 * np.sqrt((x - x0) ** 2 + z0 ** 2) / v_medium          # [nx]
    t = np.arange(nt) * dt                                             # [nt]
    p = ricker(t[None, :] - t_d[:, None], f_ricker)                    # [nx][nt]
    om = omegas(nw, fmin, fmax)
    kern = np.exp(-1j * np.outer(t, om))                               # [nt][nw]
    data = p @ kern                                                    # [nx][nw]
    v_prop = v_medium / 2.0
    vel = np.full((nz, nx), v_prop, dtype=np.float32)
    desc = table_for(ntaps, nk, fmin, fmax, v_prop, v_prop, dx, dz)
    return Section("config1_diffraction", nx, nz, dx, dz, om, vel, data, desc,
                   extra={"ix0": ix0, "iz0": iz0, "nt": nt, "dt": dt,
                          "seed": seed, "section": p.astype(np.float32)})


# --------------------------------------------------------------------------- #
# Configuration 2: dipping layers plus a high-velocity body.
# --------------------------------------------------------------------------- #
def layered_model(rng: np.random.Generator, nx: int, nz: int, dx: float, dz: float,
                  vlo: float = 1500.0, vhi: float = 4500.0, vbody: float = 4800.0,
                  nlayer_range=(6, 11), body: bool = True) -> np.ndarray:
    """Medium velocity [nz][nx] float64 (draw order is part of the recipe)."""
    X, Z = nx * dx, nz * dz
    nl = int(rng.integers(nlayer_range[0], nlayer_range[1]))
    base = np.sort(rng.uniform(0.05, 0.95, nl)) * Z
    dip = np.deg2rad(rng.uniform(-15.0, 15.0, nl))
    vlay = np.sort(rng.uniform(vlo, vhi, nl + 1))
    xs = np.arange(nx) * dx
    zs = np.arange(nz) * dz
    zif = base[:, None] + np.tan(dip)[:, None] * (xs[None, :] - X / 2.0)   # [nl][nx]
    layer = (zif[None, :, :] <= zs[:, None, None]).sum(axis=1)             # [nz][nx]
    v = vlay[layer]
    if body:
        xc = rng.uniform(0.3, 0.7) * X
        zc = rng.uniform(0.35, 0.65) * Z
        a = rng.uniform(0.08, 0.18) * X
        b = rng.uniform(0.06, 0.15) * Z
        c = rng.uniform(-0.12, 0.12, 3)
        psi = rng.uniform(0.0, TWO_PI, 3)
        ex = (xs[None, :] - xc) / a
        ez = (zs[:, None] - zc) / b
        rho = np.sqrt(ex ** 2 + ez ** 2)
        phi = np.arctan2(ez, ex)
        lim = 1.0 + sum(c[m] * np.cos((m + 2) * phi + psi[m]) for m in range(3))
        v = np.where(rho <= lim, vbody, v)
    return v


def reflectivity(v: np.ndarray) -> np.ndarray:
    """+-1 where the velocity changes going down, 0 elsewhere; [nz][nx]."""
    r = np.zeros_like(v)
    r[:-1] = np.sign(v[1:] - v[:-1])
    return r


def phase_shift_model(refl: np.ndarray, v_prop_z: np.ndarray, omega: np.ndarray,
                      wavelet: np.ndarray, dx: float, dz: float, pad: int = 2,
                      chunk: int = 25) -> np.ndarray:
    """Exploding-reflector zero-offset data by upward continuation in v(z).

    U_{nz-1} = W R^_{nz-1};  U_k = U_{k+1} exp(-i kz_k dz) + W R^_k, with
    kz_k = sqrt(omega^2/v_k^2 - kx^2) and evanescent components removed; the
    surface plane is the inverse x-transform of U_0.  Returns [nx][nw].
    """
    nz, nx = refl.shape
    nxp = pad * nx
    R = np.fft.fft(refl, n=nxp, axis=1)                   # [nz][nxp]
    kx = TWO_PI * np.fft.fftfreq(nxp, d=dx)
    out = np.zeros((nx, omega.size), np.complex128)
    for c0 in range(0, omega.size, chunk):
        om = omega[c0:c0 + chunk]
        W = wavelet[c0:c0 + chunk][:, None]
        U = np.zeros((om.size, nxp), np.complex128)
        for k in range(nz - 1, -1, -1):
            if k < nz - 1:
                kz2 = (om[:, None] / v_prop_z[k]) ** 2 - kx[None, :] ** 2
                prop = kz2 > 0.0
                ph = np.where(prop, np.exp(-1j * np.sqrt(np.where(prop, kz2, 0.0)) * dz), 0.0)
                U *= ph
            U += W * R[k][None, :]
        out[:, c0:c0 + chunk] = np.fft.ifft(U, axis=1)[:, :nx].T
    return out


def config2(seed: int = 2, nx: int = 1024, nz: int = 512, nw: int = 200,
            dx: float = 10.0, dz: float = 10.0, fmin: float = 5.0, fmax: float = 55.0,
            f_ricker: float = 20.0, ntaps: int = 35, nk: int = 2048,
            with_data: bool = True) -> Section:
    rng = np.random.default_rng(seed)
    v = layered_model(rng, nx, nz, dx, dz)
    vel = (v / 2.0).astype(np.float32)
    om = omegas(nw, fmin, fmax)
    refl = reflectivity(v)
    if with_data:
        W = ricker_spectrum(om / TWO_PI, f_ricker)
        vz = vel.astype(np.float64).mean(axis=1)
        data = phase_shift_model(refl, vz, om, W, dx, dz)
    else:
        data = np.zeros((nx, nw), np.complex128)
    desc = table_for(ntaps, nk, fmin, fmax, 750.0, 2400.0, dx, dz)
    return Section("config2_layers_body", nx, nz, dx, dz, om, vel, data, desc,
                   extra={"refl": refl, "seed": seed})


# --------------------------------------------------------------------------- #
# Small random cases for parity sweeps.
# --------------------------------------------------------------------------- #
def random_case(seed: int, nx: int, nz: int, nw: int, ntaps: int = 25, nk: int = 256,
                dx: float = 10.0, dz: float = 10.0, fmin: float = 5.0,
                fmax: float = 55.0, layered: bool = True, ngrid: int = 512,
                ncheck: int = 4096) -> Section:
    """Random velocity (layered or per-point random) and random complex data."""
    rng = np.random.default_rng(seed)
    if layered:
        v = layered_model(rng, nx, nz, dx, dz, nlayer_range=(2, 6))
    else:
        v = rng.uniform(1500.0, 4800.0, (nz, nx))
    vel = (v / 2.0).astype(np.float32)
    om = omegas(nw, fmin, fmax)
    data = rng.standard_normal((nx, nw)) + 1j * rng.standard_normal((nx, nw))
    desc = table_for(ntaps, nk, fmin, fmax, 750.0, 2400.0, dx, dz,
                     ngrid=ngrid, ncheck=ncheck)
    return Section("random_%d" % seed, nx, nz, dx, dz, om, vel, data, desc,
                   extra={"seed": seed})


# --------------------------------------------------------------------------- #
# Configuration 3: a batch of independent sections of uneven size.
# --------------------------------------------------------------------------- #
def bandlimited_data(rng: np.random.Generator, nx: int, nw: int, dx: float,
                     kx_max: float) -> np.ndarray:
    """Random complex f-x plane whose lateral spectrum is confined to
    |kx| <= kx_max (rad/m): white Gaussian spectra, zeroed outside the band,
    transformed back along x.  [nx][nw] complex128."""
    spec = rng.standard_normal((nx, nw)) + 1j * rng.standard_normal((nx, nw))
    kx = TWO_PI * np.fft.fftfreq(nx, d=dx)
    spec[np.abs(kx) > kx_max] = 0.0
    return np.fft.ifft(spec, axis=0)


def config3(seed: int = 3, nsec: int = 64, nx_range=(256, 2048), nz_range=(200, 800),
            nw_range=(100, 300), dx: float = 10.0, dz: float = 10.0, fmin: float = 5.0,
            fmax: float = 55.0, ntaps: int = 35, nk: int = 2048) -> list:
    """Batch of `nsec` sections with seed-drawn nx, nz, nw (inclusive ranges),
    velocity models drawn like configuration 2, and band-limited random
    complex data (propagating band of the slowest medium at fmax), all
    sharing configuration 2's table."""
    rng = np.random.default_rng(seed)
    desc = table_for(ntaps, nk, fmin, fmax, 750.0, 2400.0, dx, dz)
    out = []
    for i in range(nsec):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nz = int(rng.integers(nz_range[0], nz_range[1] + 1))
        nw = int(rng.integers(nw_range[0], nw_range[1] + 1))
        v = layered_model(rng, nx, nz, dx, dz)
        vel = (v / 2.0).astype(np.float32)
        om = omegas(nw, fmin, fmax)
        data = bandlimited_data(rng, nx, nw, dx, TWO_PI * fmax / 750.0)
        out.append(Section("config3_%02d" % i, nx, nz, dx, dz, om, vel, data, desc,
                           extra={"seed": seed, "index": i}))
    return out


def with_desc(sec: Section, **kw) -> Section:
    sec.desc = replace(sec.desc, **kw)
    return sec


# --------------------------------------------------------------------------- #
# 3-D volumes (extension with 2-D extrapolators).
# --------------------------------------------------------------------------- #
@dataclass
class Volume:
    """One 3-D zero-offset volume ready for migration."""

    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dz: float
    omega: np.ndarray          # [nw] float64
    vel: np.ndarray            # [nz][nx][ny] float32 propagation velocity
    data: np.ndarray           # [nx][ny][nw] complex128 surface plane
    desc: TableDesc            # 2-D table: ntaps = 2M+1 per axis
    extra: dict = field(default_factory=dict)

    @property
    def nw(self) -> int:
        return int(self.omega.size)


def table2d_for(ntaps: int, nk: int, fmin: float, fmax: float, vmin_prop: float,
                vmax_prop: float, dx: float, dz: float, ngrid: int = 48,
                ncheck: int = 192, tau: float = 1e-2, beta: float = 0.3,
                **kw) -> TableDesc:
    """2-D table descriptor; ngrid/ncheck are points per axis of the 2-D grids.
    The reweighting is gentler than in 1-D (tau 1e-2, beta 0.3): with beta 1
    and tau of order 1e-4 the 2-D fit becomes ill-conditioned at large kappa
    (1-ulp input changes move some entries by 1e-4) and its worst passband
    error grows."""
    return table_for(ntaps, nk, fmin, fmax, vmin_prop, vmax_prop, dx, dz, ngrid=ngrid,
                     ncheck=ncheck, tau=tau, beta=beta, **kw)


def point_scatterer_3d(seed: int = 5, nx: int = 40, ny: int = 40, nz: int = 40, nw: int = 24,
                       dx: float = 10.0, dz: float = 10.0, nt: int = 192, dt: float = 0.004,
                       v_medium: float = 2000.0, fmin: float = 5.0, fmax: float = 30.0,
                       f_ricker: float = 15.0, ntaps: int = 11, nk: int = 64) -> Volume:
    """Constant medium velocity, one point scatterer at a seeded (x, y, z):
    two-way diffraction times over the surface, a Ricker wavelet on each, and
    a direct DFT along t (forward sign exp(-i omega t))."""
    rng = np.random.default_rng(seed)
    ix0 = int(rng.integers(nx // 3, 2 * nx // 3))
    iy0 = int(rng.integers(ny // 3, 2 * ny // 3))
    iz0 = int(rng.integers(nz // 3, 2 * nz // 3))
    xs = np.arange(nx) * dx
    ys = np.arange(ny) * dx
    r = np.sqrt((xs[:, None] - ix0 * dx) ** 2 + (ys[None, :] - iy0 * dx) ** 2 + (iz0 * dz) ** 2)
    t_d = 2.0 * r / v_medium                                           # [nx][ny]
    t = np.arange(nt) * dt
    p = ricker(t[None, None, :] - t_d[:, :, None], f_ricker)           # [nx][ny][nt]
    om = omegas(nw, fmin, fmax)
    data = p @ np.exp(-1j * np.outer(t, om))                           # [nx][ny][nw]
    v_prop = v_medium / 2.0
    vel = np.full((nz, nx, ny), v_prop, dtype=np.float32)
    desc = table2d_for(ntaps, nk, fmin, fmax, v_prop, v_prop, dx, dz)
    return Volume("point_scatterer_3d", nx, ny, nz, dx, dz, om, vel, data, desc,
                  extra={"ix0": ix0, "iy0": iy0, "iz0": iz0, "seed": seed})


def layered_volume(rng: np.random.Generator, nx: int, ny: int, nz: int, dx: float, dz: float,
                   vlo: float = 1500.0, vhi: float = 3500.0, vbody: float = 4000.0,
                   nlayer_range=(6, 11)):
    """Medium velocity [nz][nx][ny] float64 of planar dipping layers plus one
    ellipsoidal body, and the undisturbed layer velocity down the centre
    column [nz] (draw order is part of the recipe)."""
    X, Y, Z = nx * dx, ny * dx, nz * dz
    nl = int(rng.integers(nlayer_range[0], nlayer_range[1]))
    base = np.sort(rng.uniform(0.05, 0.95, nl)) * Z
    dipx = np.tan(np.deg2rad(rng.uniform(-12.0, 12.0, nl)))
    dipy = np.tan(np.deg2rad(rng.uniform(-12.0, 12.0, nl)))
    vlay = np.sort(rng.uniform(vlo, vhi, nl + 1))
    xs = np.arange(nx) * dx - X / 2.0
    ys = np.arange(ny) * dx - Y / 2.0
    zs = np.arange(nz) * dz
    v = np.empty((nz, nx, ny))
    for k in range(nz):
        zif = base[:, None, None] + dipx[:, None, None] * xs[None, :, None] \
            + dipy[:, None, None] * ys[None, None, :]                  # [nl][nx][ny]
        v[k] = vlay[(zif <= zs[k]).sum(axis=0)]
    centre = vlay[(base[:, None] <= zs[None, :]).sum(axis=0)]          # [nz]
    c = np.array([rng.uniform(0.3, 0.7) * X, rng.uniform(0.3, 0.7) * Y,
                  rng.uniform(0.35, 0.65) * Z])
    ax = np.array([rng.uniform(0.08, 0.18) * X, rng.uniform(0.08, 0.18) * Y,
                   rng.uniform(0.06, 0.15) * Z])
    e = ((np.arange(nx) * dx - c[0]) / ax[0])[None, :, None] ** 2 \
        + ((np.arange(ny) * dx - c[1]) / ax[1])[None, None, :] ** 2 \
        + ((zs - c[2]) / ax[2])[:, None, None] ** 2
    v = np.where(e <= 1.0, vbody, v)
    return v, centre


def phase_shift_model_3d(refl: np.ndarray, v_prop_z: np.ndarray, omega: np.ndarray,
                         wavelet: np.ndarray, dx: float, dz: float,
                         chunk: int = 16) -> np.ndarray:
    """Exploding-reflector data by upward continuation in v(z) on the periodic
    (kx, ky) grid of the volume: U_k = U_{k+1} exp(-i kz_k dz) + W R^_k with
    evanescent components removed.  refl [nz][nx][ny] -> [nx][ny][nw]."""
    nz, nx, ny = refl.shape
    R = np.fft.fft2(refl, axes=(1, 2))                                # [nz][nx][ny]
    kx = TWO_PI * np.fft.fftfreq(nx, d=dx)
    ky = TWO_PI * np.fft.fftfreq(ny, d=dx)
    kr2 = kx[:, None] ** 2 + ky[None, :] ** 2
    out = np.zeros((nx, ny, omega.size), np.complex128)
    for c0 in range(0, omega.size, chunk):
        om = omega[c0:c0 + chunk]
        W = wavelet[c0:c0 + chunk][:, None, None]
        U = np.zeros((om.size, nx, ny), np.complex128)
        ph, v_ph = None, None
        for k in range(nz - 1, -1, -1):
            if k < nz - 1:
                if v_prop_z[k] != v_ph:
                    kz2 = (om[:, None, None] / v_prop_z[k]) ** 2 - kr2[None]
                    prop = kz2 > 0.0
                    ph = np.where(prop, np.exp(-1j * np.sqrt(np.where(prop, kz2, 0.0)) * dz), 0.0)
                    v_ph = v_prop_z[k]
                U *= ph
            U += W * R[k][None]
        out[:, :, c0:c0 + chunk] = np.moveaxis(np.fft.ifft2(U, axes=(1, 2)), 0, 2)
    return out


def config5(seed: int = 5, nx: int = 256, ny: int = 256, nz: int = 200, nw: int = 128,
            dx: float = 10.0, dz: float = 10.0, fmin: float = 5.0, fmax: float = 40.0,
            f_ricker: float = 20.0, ntaps: int = 11, nk: int = 1024,
            with_data: bool = True) -> Volume:
    """3-D layered volume with an ellipsoidal body; 11 x 11 extrapolators."""
    rng = np.random.default_rng(seed)
    v, centre = layered_volume(rng, nx, ny, nz, dx, dz)
    vel = (v / 2.0).astype(np.float32)
    om = omegas(nw, fmin, fmax)
    refl = np.zeros_like(v)
    refl[:-1] = np.sign(v[1:] - v[:-1])
    if with_data:
        W = ricker_spectrum(om / TWO_PI, f_ricker)
        data = phase_shift_model_3d(refl, centre / 2.0, om, W, dx, dz)
    else:
        data = np.zeros((nx, ny, nw), np.complex128)
    desc = table2d_for(ntaps, nk, fmin, fmax, 750.0, 2000.0, dx, dz)
    return Volume("config5_layers_ellipsoid", nx, ny, nz, dx, dz, om, vel, data, desc,
                  extra={"refl": refl, "seed": seed})


def random_volume(seed: int, nx: int, ny: int, nz: int, nw: int, ntaps: int = 11,
                  nk: int = 64, layered: bool = True, fmin: float = 5.0,
                  fmax: float = 40.0, dx: float = 10.0, dz: float = 10.0) -> Volume:
    """Random velocity volume (layered or per-point random) and random complex
    data, for parity sweeps."""
    rng = np.random.default_rng(seed)
    if layered:
        v, _ = layered_volume(rng, nx, ny, nz, dx, dz, nlayer_range=(2, 6))
    else:
        v = rng.uniform(1500.0, 4000.0, (nz, nx, ny))
    vel = (v / 2.0).astype(np.float32)
    om = omegas(nw, fmin, fmax)
    data = rng.standard_normal((nx, ny, nw)) + 1j * rng.standard_normal((nx, ny, nw))
    desc = table2d_for(ntaps, nk, fmin, fmax, 750.0, 2000.0, dx, dz, ngrid=48, ncheck=192)
    return Volume("random_volume_%d" % seed, nx, ny, nz, dx, dz, om, vel, data, desc,
                  extra={"seed": seed})
