"""Transform along t on the matrix cores (Algorithm 1, first step) vs the FP64
oracle, the closed form of delayed spikes, and migration from a t-x section.

FP32 tolerance: the DFT matrix entries are FP64 values rounded to FP32 and
the nt-term sums accumulate in FP32, so the relative error is a few ulp times
a modest growth factor: 1e-5 relative L2 (1e-4 for the migrated image)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1912_05529_amd import mig, synth
from gpu_helpers import dev, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,nt,nw", [(37, 100, 13), (64, 256, 64), (1024, 1024, 200), (1, 5, 1),
                                      (130, 17, 33)])
def test_transform_matches_oracle(nx, nt, nw):
    rng = np.random.default_rng(nx + nt)
    p = rng.standard_normal((nx, nt)).astype(np.float32)
    om = synth.omegas(nw, 5.0, 55.0)
    got = mig.transform_t(torch.from_numpy(p).to(dev()), 0.004, torch.from_numpy(om).to(dev()))
    ref = oracle.transform_t(p, 0.004, om)
    assert rel_l2(got.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("nx,nt,nw", [(2048, 131076, 8), (1024, 262147, 3)])
def test_transform_large_sections_sampled(nx, nt, nw):
    """Sections of over 2^30 bytes (the product's buffer offsets are taken from
    per-chunk bases): sampled traces against the FP64 oracle, 16-byte copy path
    (nt and 2 nw multiples of 4) and 4-byte copy path."""
    print("large transform nx=%d nt=%d nw=%d" % (nx, nt, nw), flush=True)
    rng = np.random.default_rng(nt)
    p = rng.standard_normal((nx, nt), dtype=np.float32)
    om = synth.omegas(nw, 5.0, 55.0)
    got = mig.transform_t(torch.from_numpy(p).to(dev()), 0.001, torch.from_numpy(om).to(dev()))
    idx = [0, 1, 777, nx - 1]
    ref = oracle.transform_t(np.ascontiguousarray(p[idx]), 0.001, om)
    assert rel_l2(got[idx].cpu().numpy(), ref) <= 1e-4


def test_transform_of_spikes_is_closed_form():
    nx, nt, dt = 70, 90, 0.002
    p = np.zeros((nx, nt), np.float32)
    n0 = (np.arange(nx) * 7) % nt
    p[np.arange(nx), n0] = 1.0
    om = np.linspace(3.0, 300.0, 21)
    got = mig.transform_t(torch.from_numpy(p).to(dev()), dt, torch.from_numpy(om).to(dev()))
    ref = np.exp(-1j * np.outer(n0 * dt, om))
    assert np.abs(got.cpu().numpy() - ref).max() <= 2e-6


def test_migrate_from_tx_section_focuses(cfg1, cfg1_table):
    sec = cfg1
    tab = mig.design_table(sec.desc, dev())
    d = dev()
    section = torch.from_numpy(sec.extra["section"]).to(d)
    om = torch.from_numpy(sec.omega).to(d)
    plane = mig.transform_t(section, sec.extra["dt"], om)
    assert rel_l2(plane.cpu().numpy(), sec.data) <= 1e-5
    img = mig.migrate_tx(section, sec.extra["dt"], torch.from_numpy(sec.vel).to(d), om,
                         tab["tab32"], sec.desc).cpu().numpy()
    ref = oracle.migrate(sec.desc, cfg1_table[0], sec.omega, sec.vel, sec.data)
    assert rel_l2(img, ref) <= 1e-4
    iz, ix = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    assert abs(iz - sec.extra["iz0"]) <= 1 and abs(ix - sec.extra["ix0"]) <= 1
