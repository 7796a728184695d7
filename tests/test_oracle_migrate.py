"""Migration-level pins of the oracle (Algorithm 1 end to end).

* P8: the analytic two-way diffraction hyperbola of one point scatterer (config
  1) collapses to the scatterer: the image peak is within one sample of the
  truth and most of the image energy sits in a small box around it.  The
  wrong-velocity control (medium instead of propagation velocity) must fail.
* P9: the adjoint passes the dot-product test.
* P7: the image stays close to textbook phase-shift (Gazdag) migration, coded
  here with numpy FFTs; the difference is recorded.
"""
import math

import numpy as np

import oracle
from paper_1912_05529_amd import synth


def _box_fraction(img, iz, ix, hx=3, hz=5):
    e = img ** 2
    return e[max(iz - hz, 0):iz + hz + 1, max(ix - hx, 0):ix + hx + 1].sum() / e.sum()


def test_p8_diffraction_collapses_to_scatterer(cfg1, cfg1_table):
    img = oracle.migrate(cfg1.desc, cfg1_table[0], cfg1.omega, cfg1.vel, cfg1.data)
    iz, ix = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    assert abs(iz - cfg1.extra["iz0"]) <= 1 and abs(ix - cfg1.extra["ix0"]) <= 1
    assert _box_fraction(img, cfg1.extra["iz0"], cfg1.extra["ix0"]) >= 0.80


def test_p8_control_wrong_velocity_does_not_focus(cfg1, cfg1_table):
    desc = synth.table_for(25, 512, 5.0, 40.0, 2000.0, 2000.0, 10.0, 10.0)
    tab = oracle.design_table(desc)[0]
    vel = np.full_like(cfg1.vel, 2000.0)
    img = oracle.migrate(desc, tab, cfg1.omega, vel, cfg1.data)
    iz, ix = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    assert abs(iz - cfg1.extra["iz0"]) > 5
    assert _box_fraction(img, cfg1.extra["iz0"], cfg1.extra["ix0"]) < 0.5


def test_p9_adjoint_dot_product():
    rng = np.random.default_rng(21)
    nx, nz, nw, ntaps = 24, 9, 5, 7
    desc = synth.TableDesc(ntaps=ntaps, nk=16, kmin=0.02, kmax=0.45, dx=10.0, dz=10.0)
    K = (ntaps - 1) // 2 + 1
    tab = (rng.standard_normal((desc.nk, K)) + 1j * rng.standard_normal((desc.nk, K))) / K
    om = synth.omegas(nw, 5.0, 55.0)
    vel = rng.uniform(700.0, 2500.0, (nz, nx)).astype(np.float32)
    d = rng.standard_normal((nx, nw)) + 1j * rng.standard_normal((nx, nw))
    m = rng.standard_normal((nz, nx))
    Ld = oracle.migrate(desc, tab, om, vel, d)
    Ltm = oracle.demigrate(desc, tab, om, vel, m)
    lhs = float(np.sum(Ld * m))
    rhs = float(np.sum((np.conj(d) * Ltm).real))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Ld) * np.linalg.norm(m)


def test_p7_close_to_gazdag_phase_shift(cfg1, cfg1_table):
    img = oracle.migrate(cfg1.desc, cfg1_table[0], cfg1.omega, cfg1.vel, cfg1.data)
    nx, nz, dx, dz = cfg1.nx, cfg1.nz, cfg1.dx, cfg1.dz
    npad = 512
    kx = 2 * np.pi * np.fft.fftfreq(npad, dx)
    U = np.fft.fft(cfg1.data, npad, axis=0)
    k = cfg1.omega[None, :] / float(cfg1.vel[0, 0])
    kz2 = k ** 2 - kx[:, None] ** 2
    keep = np.abs(kx[:, None]) <= k * math.sin(math.radians(60.0))
    shift = np.where(keep, np.exp(1j * np.sqrt(np.maximum(kz2, 0.0)) * dz), 0.0)
    g = np.zeros((nz, nx))
    g[0] = np.fft.ifft(U, axis=0)[:nx].real.sum(axis=1)
    for iz in range(1, nz):
        U = U * shift
        g[iz] = np.fft.ifft(U, axis=0)[:nx].real.sum(axis=1)
    sl = (slice(10, 100), slice(20, 108))
    rel = np.linalg.norm(img[sl] - g[sl]) / np.linalg.norm(g[sl])
    print("P7 relative interior difference FIR vs phase shift: %.4f" % rel)
    assert rel < 0.2
    assert np.unravel_index(np.argmax(np.abs(g)), g.shape) == \
        np.unravel_index(np.argmax(np.abs(img)), img.shape)
