"""Pin of the table look-up (the look-up step of Algorithm 1; Sec. III: filter
chosen by the wavenumber omega/v): the oracle's IEEE-double index must be the
exact-rational nearest entry wherever the exact position is not within 1e-6 of
a tie, and must follow the stated clamps."""
import math
from fractions import Fraction

import numpy as np

import oracle
from paper_1912_05529_amd import synth


def _exact_position(desc, omega, v):
    kmin = Fraction(desc.kmin)
    dk = Fraction((desc.kmax - desc.kmin) / (desc.nk - 1))
    return (Fraction(float(omega)) / Fraction(float(v)) - kmin) / dk


def test_index_is_exact_nearest_entry():
    desc = synth.table_for(35, 2048, 5.0, 55.0, 750.0, 2400.0, 10.0, 10.0)
    rng = np.random.default_rng(11)
    om = synth.omegas(200, 5.0, 55.0)
    vel = rng.uniform(700.0, 2500.0, (3, 97)).astype(np.float32)
    idx = oracle.table_index(desc, om, vel)
    checked = 0
    for k in range(vel.shape[0]):
        for x in range(vel.shape[1]):
            for r in range(0, om.size, 7):
                t = _exact_position(desc, om[r], vel[k, x])
                frac = t - math.floor(t)
                if abs(frac - Fraction(1, 2)) < Fraction(1, 10 ** 6):
                    continue
                j = min(max(math.floor(t + Fraction(1, 2)), 0), desc.nk - 1)
                assert idx[k, x, r] == j, (k, x, r, float(t))
                checked += 1
    assert checked > 8000


def test_index_on_entries_and_clamps():
    desc = synth.TableDesc(ntaps=5, nk=10, kmin=0.1, kmax=1.0, dx=10.0, dz=10.0)
    # omega chosen so omega/v lands on entries (v = 1): exact grid points
    dk = (desc.kmax - desc.kmin) / (desc.nk - 1)
    om = np.array([desc.kmin + j * dk for j in range(desc.nk)])
    idx = oracle.table_index(desc, om, np.ones((1, 1), np.float32))[0, 0]
    assert idx.tolist() == list(range(desc.nk))
    # below the axis -> 0, above -> nk-1, non-positive / NaN velocity -> 0
    v = np.array([[1e9, 1e-9, 0.0, -0.0, -5.0, np.nan, np.inf]], np.float32)
    idx = oracle.table_index(desc, np.array([0.5]), v)[0, :, 0]
    assert idx.tolist() == [0, desc.nk - 1, 0, 0, 0, 0, 0]
