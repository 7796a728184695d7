"""Adjoint (demigration), autograd wrappers, least-squares migration and depth
checkpoints, through the C ABI.

Checks: FP32 GPU adjoint vs the FP64 oracle adjoint on a 64x64 grid; the
dot-product test <A d, m> = <d, A^T m>; autograd gradients vs central finite
differences of a quadratic loss (exact for any step, so only rounding
remains); CGLS on the layered model with 5 % noise; checkpointed migration
bit-identical to the single call and resumable.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1912_05529_amd import lsm, mig, synth
from gpu_helpers import assert_rows_close, dev, rel_l2, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    sec = synth.random_case(64, 64, 64, 16, ntaps=35, nk=256)
    tab = mig.design_table(sec.desc, dev())
    return sec, tab, upload(sec)


def test_demigrate_matches_oracle_adjoint(small):
    sec, tab, t = small
    rng = np.random.default_rng(7)
    img = rng.standard_normal((sec.nz, sec.nx))
    got = mig.demigrate(torch.from_numpy(img).to(dev()), t["vel"], t["omega"], tab["tab32"],
                        sec.desc).cpu().numpy()
    ot = oracle.design_table(sec.desc)[0]
    ref = oracle.demigrate(sec.desc, ot, sec.omega, sec.vel, img)
    err = rel_l2(got, ref)
    print("demigrate vs FP64 oracle rel L2 %.3e" % err)
    assert err <= 1e-5


@pytest.mark.parametrize("nx,nz,nw,ntaps,layered", [
    (64, 2, 4, 35, True), (64, 3, 4, 35, True), (130, 4, 5, 35, True), (257, 5, 3, 35, False),
    (1024, 40, 6, 35, True), (1023, 37, 5, 11, True), (300, 20, 4, 41, True)])
def test_demigrate_shapes_match_oracle(nx, nz, nw, ntaps, layered):
    """Demigration against the FP64 oracle for one to a few dozen depth steps
    (both tap sets of the register-tap kernel, odd and even step counts), a
    layered model (taps kept across steps where the slowness repeats), an odd
    nx, and the general kernel (N = 41)."""
    sec = synth.random_case(1700 + nx + nz, nx, nz, nw, ntaps=ntaps, nk=256, layered=layered)
    print("demigrate nx=%d nz=%d nw=%d N=%d layered=%s" % (nx, nz, nw, ntaps, layered), flush=True)
    tab = mig.design_table(sec.desc, dev())
    t = upload(sec)
    rng = np.random.default_rng(nx + nz)
    img = rng.standard_normal((nz, nx))
    got = mig.demigrate(torch.from_numpy(img).to(dev()), t["vel"], t["omega"], tab["tab32"],
                        sec.desc).cpu().numpy()
    ot = oracle.design_table(sec.desc)[0]
    ref = oracle.demigrate(sec.desc, ot, sec.omega, sec.vel, img)
    err = rel_l2(got, ref)
    print("  rel L2 %.3e" % err)
    assert err <= 1e-5


@pytest.mark.parametrize("nx,nz,nw,ntaps", [(64, 64, 16, 35), (1024, 40, 12, 35),
                                            (300, 33, 7, 25), (2100, 5, 3, 35), (1, 4, 2, 35)])
def test_dot_product(nx, nz, nw, ntaps):
    sec = synth.random_case(900 + nx, nx, nz, nw, ntaps=ntaps, nk=256, layered=False)
    tab = mig.design_table(sec.desc, dev())
    t = upload(sec)
    rng = np.random.default_rng(nx)
    m = torch.from_numpy(rng.standard_normal((nz, nx))).to(dev())
    Ad = mig.migrate(t["data"], t["vel"], t["omega"], tab["tab32"], sec.desc)
    Atm = mig.demigrate(m, t["vel"], t["omega"], tab["tab32"], sec.desc)
    lhs = float(torch.sum(Ad * m))
    d = t["data"]
    rhs = float(torch.sum(d.real.double() * Atm.real.double() + d.imag.double() * Atm.imag.double()))
    scale = float(torch.linalg.norm(Ad)) * float(torch.linalg.norm(m))
    print("dot test nx=%d: |lhs-rhs|/scale = %.3e" % (nx, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_autograd_gradient_matches_finite_differences(small):
    sec, tab, t = small
    rng = np.random.default_rng(11)
    target = torch.from_numpy(rng.standard_normal((sec.nz, sec.nx))).to(dev())
    d = t["data"].clone().requires_grad_(True)
    img = lsm.migrate_fn(d, t["vel"], t["omega"], tab["tab32"], sec.desc)
    loss = 0.5 * torch.sum((img - target) ** 2)
    loss.backward()
    g = d.grad
    for seed in range(3):
        r = np.random.default_rng(100 + seed)
        v = torch.from_numpy((r.standard_normal(d.shape) + 1j * r.standard_normal(d.shape))
                             .astype(np.complex64)).to(dev())

        def L(x):
            im = mig.migrate(x, t["vel"], t["omega"], tab["tab32"], sec.desc)
            return 0.5 * float(torch.sum((im - target) ** 2))

        with torch.no_grad():
            fd = (L(d.detach() + v) - L(d.detach() - v)) / 2.0
        an = float(torch.sum(g.real.double() * v.real.double() + g.imag.double() * v.imag.double()))
        print("FD %.6e autograd %.6e" % (fd, an))
        assert abs(fd - an) <= 1e-4 * max(abs(fd), 1e-30) + 1e-6 * float(torch.linalg.norm(g))


def test_demigrate_autograd_backward_is_migrate(small):
    sec, tab, t = small
    m = torch.zeros((sec.nz, sec.nx), dtype=torch.float64, device=dev(), requires_grad=True)
    d = lsm.demigrate_fn(m, t["vel"], t["omega"], tab["tab32"], sec.desc)
    w = t["data"]
    loss = torch.sum(d.real.double() * w.real.double() + d.imag.double() * w.imag.double())
    loss.backward()
    ref = mig.migrate(w, t["vel"], t["omega"], tab["tab32"], sec.desc)
    assert torch.allclose(m.grad, ref, rtol=0, atol=0)


def test_lsm_cgls_on_layered_model():
    sec = synth.config2(with_data=False)
    tab = mig.design_table(sec.desc, dev())
    t = upload(sec)
    refl = torch.from_numpy(sec.extra["refl"]).to(dev())
    d_clean = mig.demigrate(refl, t["vel"], t["omega"], tab["tab32"], sec.desc)
    g = torch.Generator(device="cpu").manual_seed(5)
    rms = float(torch.sqrt(torch.mean(torch.abs(d_clean.cpu()) ** 2)))
    noise = (torch.randn(d_clean.shape, generator=g) + 1j * torch.randn(d_clean.shape, generator=g))
    d_obs = d_clean + (0.05 * rms / np.sqrt(2.0) * noise).to(torch.complex64).to(dev())
    m, hist = lsm.cgls(d_obs, t["vel"], t["omega"], tab["tab32"], sec.desc, niter=10)
    err0 = 1.0
    err = float(torch.linalg.norm(m - refl) / torch.linalg.norm(refl))
    # the migrated image itself (first CG direction) for reference
    mig_img = mig.migrate(d_obs, t["vel"], t["omega"], tab["tab32"], sec.desc)
    a = float(torch.sum(mig_img * refl) / torch.sum(mig_img * mig_img))
    err_mig = float(torch.linalg.norm(a * mig_img - refl) / torch.linalg.norm(refl))
    print("CGLS residual history", ["%.4f" % h for h in hist])
    print("model error: best-scaled migration %.4f, CGLS(10) %.4f" % (err_mig, err))
    assert all(h2 <= h1 + 1e-6 for h1, h2 in zip(hist, hist[1:]))
    assert hist[-1] < 0.5 * hist[0]
    assert err < err_mig < err0


def test_checkpointed_migration_is_identical_and_resumable(small):
    sec, tab, t = small
    ref = mig.migrate(t["data"], t["vel"], t["omega"], tab["tab32"], sec.desc)
    img, cps = lsm.migrate_checkpointed(t["data"], t["vel"], t["omega"], tab["tab32"], sec.desc,
                                        every=16)
    assert torch.equal(img, ref)
    assert sorted(cps) == [0, 16, 32, 48, 63]
    nxt, rows = mig.extrapolate(cps[16], t["vel"][16:32].contiguous(), t["omega"], tab["tab32"],
                                sec.desc, 16)
    assert torch.equal(nxt, cps[32])
    assert torch.equal(rows, ref[17:33])


def test_demigrate_config2_full_matches_oracle():
    """Demigration at the benchmarked size (1024 x 512, 200 frequencies, 35
    taps, the layered model with its body) against the FP64 oracle adjoint."""
    sec = synth.config2(with_data=False)
    tab = mig.design_table(sec.desc, dev())
    refl = sec.extra["refl"]
    got = mig.demigrate(torch.from_numpy(refl).to(dev()), torch.from_numpy(sec.vel).to(dev()),
                        torch.from_numpy(sec.omega).to(dev()), tab["tab32"], sec.desc)
    ot = oracle.design_table(sec.desc)[0]
    ref = oracle.demigrate(sec.desc, ot, sec.omega, sec.vel, refl)
    got = got.cpu().numpy()
    err = rel_l2(got, ref)
    print("config2 demigrate rel L2 vs FP64 oracle %.3e" % err, flush=True)
    assert err <= 1e-4
    # element by element, per frequency (each frequency is its own recursion)
    assert_rows_close(got, ref, 1e-4, "config2 demigrate per frequency", axis=1)
