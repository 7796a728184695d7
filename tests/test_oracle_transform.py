"""Pins of the oracle's transform along t (Algorithm 1, first step): at FFT bin
frequencies it equals numpy's FFT (textbook routine); a delayed unit spike
transforms to exp(-i omega n0 dt) exactly (closed form) at any frequency."""
import math

import numpy as np

import oracle


def test_transform_equals_fft_at_bins():
    rng = np.random.default_rng(1)
    nx, nt, dt = 5, 64, 0.004
    p = rng.standard_normal((nx, nt)).astype(np.float32)
    bins = np.array([0, 1, 7, 31, 32])
    om = 2 * math.pi * bins / (nt * dt)
    got = oracle.transform_t(p, dt, om)
    ref = np.fft.fft(p.astype(np.float64), axis=1)[:, bins]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_transform_of_delayed_spike():
    nx, nt, dt = 3, 50, 0.002
    p = np.zeros((nx, nt), np.float32)
    n0 = [0, 7, 49]
    for x in range(nx):
        p[x, n0[x]] = 1.0
    om = np.array([3.0, 100.0, 2 * math.pi * 37.3])
    got = oracle.transform_t(p, dt, om)
    for x in range(nx):
        assert np.abs(got[x] - np.exp(-1j * om * n0[x] * dt)).max() <= 1e-14
