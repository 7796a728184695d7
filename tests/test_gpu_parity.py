"""GPU parity against the FP64 oracle, through the C ABI (libmig.so).

Tolerances
  * table design (FP64 on both sides, same formulas, same accumulation order;
    only libm vs device cos/sin/exp/sqrt differ in the last bit): 1e-10
    relative.  The reweighting passes multiply weights by
    1 + beta (|H|-1)/tau; with tau = 5e-4 a 1-ulp change of dx, dz or tau
    moves the oracle's own table by at most ~2e-11, so last-bit differences
    of the transcendental functions stay well inside the bound (the test
    prints that sensitivity next to the measured difference);
  * table look-up: bit-exact (same IEEE-double operation sequence);
  * FP32 extrapolation vs FP64 oracle: relative L2 <= 1e-5 after a few steps
    (FP32 taps and arithmetic, ~1e-7 per operation, ~2N operations per output
    per step), and relative image L2 <= 1e-4 over a full section (the target);
  * imaging of the same complex64 plane: FP64 sums in a different order,
    1e-13 relative.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1912_05529_amd import mig, synth
from gpu_helpers import assert_rows_close, data64, dev, rel_l2, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tables():
    cache = {}

    def get(desc):
        if desc not in cache:
            cache[desc] = (oracle.design_table(desc), mig.design_table(desc, dev()))
        return cache[desc]
    return get


def _ulp_sensitivity(desc, ot):
    """Largest relative change of the oracle's table under 1-ulp changes of
    (dx, dz) and of tau."""
    worst = 0.0
    for kw in ({"dx": np.nextafter(desc.dx, np.inf), "dz": np.nextafter(desc.dz, np.inf)},
               {"tau": np.nextafter(desc.tau, np.inf)}):
        t1 = oracle.design_table(dataclasses.replace(desc, **kw))[0]
        worst = max(worst, float(np.abs(t1 - ot).max() / np.abs(ot).max()))
    return worst


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
def test_design_table_matches_oracle(which, tables, cfg1, cfg2_model):
    desc = (cfg1 if which == "cfg1" else cfg2_model).desc
    (ot, omg, ope, _), g = tables(desc)
    t64 = g["tab64"].cpu().numpy()
    err = np.abs(t64 - ot).max() / np.abs(ot).max()
    sens = _ulp_sensitivity(desc, ot)
    tol = 1e-10
    print("%s table max rel diff %.3e; oracle 1-ulp sensitivity %.3e" % (which, err, sens))
    assert err <= tol
    assert np.abs(g["maxgain"].cpu().numpy() - omg).max() <= tol
    assert np.abs(g["passerr"].cpu().numpy() - ope).max() <= tol
    assert float(g["maxgain"].max()) <= 1.0
    assert torch.equal(g["tab32"], g["tab64"].to(torch.complex64))


def test_table_index_bit_exact(cfg2_model):
    desc = cfg2_model.desc
    rng = np.random.default_rng(4)
    vel = rng.uniform(700.0, 2500.0, (5, 300)).astype(np.float32)
    vel[0, :7] = [0.0, -0.0, -3.0, np.nan, np.inf, 1e-30, 3e38]
    vel[1] = cfg2_model.vel[100, :300]
    om = cfg2_model.omega
    ref = oracle.table_index(desc, om, vel)
    got = mig.table_index(torch.from_numpy(vel).to(dev()), torch.from_numpy(om).to(dev()), desc)
    assert np.array_equal(got.cpu().numpy(), ref)


CASES = [
    # nx, nw, nsteps, ntaps, layered velocity
    (64, 8, 7, 25, True),
    (100, 5, 6, 35, False),
    (1000, 4, 5, 35, True),
    (1024, 3, 4, 35, False),
    (1025, 3, 4, 35, True),
    (1500, 2, 5, 25, False),
    (1280, 3, 6, 35, True),
    (1536, 2, 4, 35, False),
    (1537, 2, 3, 35, True),
    (2048, 2, 3, 35, True),
    (2049, 2, 3, 35, False),
    (300, 3, 4, 37, False),
    (1, 2, 3, 25, False),
    (2, 1, 2, 35, False),
    (129, 3, 1, 1, False),
    (77, 2, 2, 3, True),
]


@pytest.mark.parametrize("nx,nw,nsteps,ntaps,layered", CASES)
def test_extrapolate_matches_oracle(nx, nw, nsteps, ntaps, layered, tables):
    sec = synth.random_case(1000 + nx + ntaps, nx, nsteps + 1, nw, ntaps=ntaps, nk=256,
                            layered=layered)
    (ot, _, _, _), g = tables(sec.desc)
    print("case nx=%d nw=%d nsteps=%d N=%d kind=%d" % (nx, nw, nsteps, ntaps,
                                                       mig.kernel_kind(nx, ntaps)), flush=True)
    t = upload(sec)
    vel = t["vel"][:nsteps].contiguous()
    plane, rows = mig.extrapolate(t["data"], vel, t["omega"], g["tab32"], sec.desc, nsteps)
    torch.cuda.synchronize()
    ref_plane, ref_rows = oracle.extrapolate(sec.desc, ot, sec.omega, sec.vel[:nsteps],
                                             data64(sec), nsteps)
    p = plane.cpu().numpy()
    assert rel_l2(p, ref_plane) <= 1e-5
    assert np.abs(p - ref_plane).max() <= 1e-4 * np.abs(ref_plane).max()
    assert rel_l2(rows.cpu().numpy(), ref_rows) <= 1e-5
    # rows off: same plane bit for bit
    plane2, none = mig.extrapolate(t["data"], vel, t["omega"], g["tab32"], sec.desc, nsteps,
                                   rows=False)
    assert none is None and torch.equal(plane2, plane)


def test_image_matches_oracle():
    rng = np.random.default_rng(8)
    for nx, nw in [(1, 1), (7, 300), (130, 64), (1024, 200)]:
        P = (rng.standard_normal((nx, nw)) + 1j * rng.standard_normal((nx, nw))).astype(np.complex64)
        row = mig.image(torch.from_numpy(P).to(dev())).cpu().numpy()
        ref = oracle.image(P.astype(np.complex128))
        assert np.abs(row - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1.0)


def test_migrate_config1_matches_oracle_and_focuses(cfg1, cfg1_table, tables):
    g = tables(cfg1.desc)[1]
    t = upload(cfg1)
    img = mig.migrate(t["data"], t["vel"], t["omega"], g["tab32"], cfg1.desc).cpu().numpy()
    ref = oracle.migrate(cfg1.desc, cfg1_table[0], cfg1.omega, cfg1.vel, data64(cfg1))
    err = rel_l2(img, ref)
    print("config1 image rel L2 %.3e" % err)
    assert err <= 1e-4
    assert_rows_close(img, ref, 1e-4, "config1 image")
    iz, ix = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    assert abs(iz - cfg1.extra["iz0"]) <= 1 and abs(ix - cfg1.extra["ix0"]) <= 1


@pytest.fixture(scope="module")
def cfg2_full():
    return synth.config2()


def test_migrate_config2_full_matches_oracle(cfg2_full, tables):
    sec = cfg2_full
    (ot, _, _, _), g = tables(sec.desc)
    t = upload(sec)
    img = mig.migrate(t["data"], t["vel"], t["omega"], g["tab32"], sec.desc).cpu().numpy()
    ref = oracle.migrate(sec.desc, ot, sec.omega, sec.vel, data64(sec))
    err = rel_l2(img, ref)
    print("config2 image rel L2 %.3e" % err)
    assert err <= 1e-4
    assert_rows_close(img, ref, 1e-4, "config2 image")
    # the rows through the 4800 m/s body, element by element on their own scale
    body = np.nonzero((sec.vel * 2.0 == 4800.0).any(axis=1))[0]
    assert body.size > 0
    assert_rows_close(img[body], ref[body], 1e-4, "config2 rows crossing the body",
                      energy_floor=0.0)


def test_migrate_is_deterministic_and_chunking_is_exact(tables):
    sec = synth.random_case(77, 300, 40, 24, ntaps=35, nk=256)
    g = tables(sec.desc)[1]
    t = upload(sec)
    args = (t["data"], t["vel"], t["omega"], g["tab32"], sec.desc)
    a = mig.migrate(*args)
    b = mig.migrate(*args)
    assert torch.equal(a, b)
    for nbytes in (mig.workspace_min_size(300, 24, sec.desc),
                   mig.workspace_min_size(300, 24, sec.desc) + 7 * 24 * 320 * 4 + 5):
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev())
        c = mig.migrate(*args, ws=ws)
        assert torch.equal(a, c)


def test_extrapolate_zero_steps_and_errors(tables):
    sec = synth.random_case(5, 50, 3, 4, ntaps=25, nk=64)
    g = tables(sec.desc)[1]
    t = upload(sec)
    out, _ = mig.extrapolate(t["data"], t["vel"], t["omega"], g["tab32"], sec.desc, 0,
                             rows=False)
    assert torch.equal(out, t["data"])
    with pytest.raises(mig.MigError) as e:
        mig.extrapolate(t["data"], t["vel"], t["omega"], g["tab32"], sec.desc, 2, rows=False,
                        out=t["data"])
    assert e.value.code == mig.MIG_E_ARG
    small = torch.empty(16, dtype=torch.uint8, device=dev())
    with pytest.raises(mig.MigError) as e:
        mig.extrapolate(t["data"], t["vel"], t["omega"], g["tab32"], sec.desc, 2, ws=small)
    assert e.value.code == mig.MIG_E_WORKSPACE


@pytest.mark.parametrize("nx,nw,nsteps,ntaps", [(1024, 600, 20, 35), (130, 37, 33, 35),
                                               (2000, 9, 17, 35), (1024, 300, 97, 35),
                                               (2100, 40, 40, 35), (300, 60, 70, 41),
                                               (1280, 50, 40, 35)])
def test_fused_reduction_rows_match_oracle(nx, nw, nsteps, ntaps, tables):
    """Image rows formed inside the depth-stepping launch (reducer workgroups)
    and, for the last published block, after it: more frequency workgroups than
    CUs, several publish blocks with a ragged last block, the
    three- and four-outputs-per-thread kernels (1280 points: three outputs per
    thread reach past the row stride) and the general kernel (nx > 2048,
    N > 35)."""
    sec = synth.random_case(3000 + nx + nw, nx, nsteps + 1, nw, ntaps=ntaps, nk=256)
    (ot, _, _, _), g = tables(sec.desc)
    print("fused rows nx=%d nw=%d nsteps=%d N=%d kind=%d" % (nx, nw, nsteps, ntaps,
                                                           mig.kernel_kind(nx, ntaps)),
          flush=True)
    t = upload(sec)
    vel = t["vel"][:nsteps].contiguous()
    ws = torch.empty(mig.workspace_size(nx, nsteps, nw, sec.desc), dtype=torch.uint8,
                     device=dev())
    _, rows = mig.extrapolate(t["data"], vel, t["omega"], g["tab32"], sec.desc, nsteps,
                              want_plane=False, ws=ws)
    assert mig.workspace_status(ws) == mig.MIG_OK
    r = rows.cpu().numpy()
    assert np.isfinite(r).all()
    _, ref = oracle.extrapolate(sec.desc, ot, sec.omega, sec.vel[:nsteps], data64(sec), nsteps)
    assert rel_l2(r, ref) <= 1e-5


def _bad_velocity_case(seed, nx, nz, nw):
    """Layered section whose velocity holds values that are not > 0: NaN, +0,
    -0, negative numbers, and a whole NaN row; each selects table entry 0."""
    sec = synth.random_case(seed, nx, nz, nw, ntaps=35, nk=256)
    v = sec.vel.copy()
    v[1, 3:40] = np.nan
    v[2, :] = np.nan
    v[3, 10:20] = 0.0
    v[3, 20:25] = -0.0
    v[4, nx // 2:] = -1500.0
    v[5, ::7] = np.nan
    v[nz - 2, -5:] = -np.inf
    sec.vel = v
    return sec


@pytest.mark.parametrize("nx,nw", [(300, 7), (1024, 5), (1300, 4), (2100, 3)])
def test_non_positive_and_nan_velocity_select_entry_0(nx, nw, tables):
    """The look-up contract (velocity not > 0 -> entry 0) through the
    depth-stepping kernels of migrate, the adjoint and the batched form,
    against the oracle (which makes the same choice explicitly)."""
    sec = _bad_velocity_case(5000 + nx, nx, 12, nw)
    (ot, _, _, _), g = tables(sec.desc)
    print("bad velocity nx=%d kind=%d" % (nx, mig.kernel_kind(nx, 35)), flush=True)
    t = upload(sec)
    img = mig.migrate(t["data"], t["vel"], t["omega"], g["tab32"], sec.desc).cpu().numpy()
    ref = oracle.migrate(sec.desc, ot, sec.omega, sec.vel, data64(sec))
    assert_rows_close(img, ref, 1e-5, "migrate with bad velocities nx=%d" % nx)
    b = [dict(t)]
    mig.migrate_batched(b, g["tab32"], sec.desc)
    torch.cuda.synchronize()
    assert torch.equal(b[0]["image"].cpu(), torch.from_numpy(img))
    rng = np.random.default_rng(nx)
    m = rng.standard_normal((sec.nz, nx))
    dem = mig.demigrate(torch.from_numpy(m).to(dev()), t["vel"], t["omega"], g["tab32"],
                        sec.desc).cpu().numpy()
    dref = oracle.demigrate(sec.desc, ot, sec.omega, sec.vel, m)
    assert_rows_close(dem, dref, 1e-5, "demigrate with bad velocities nx=%d" % nx, axis=1)
