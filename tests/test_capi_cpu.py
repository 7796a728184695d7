"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/mig.h declares, and rejects bad arguments on the host before launching."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mig.h")).read()
    return sorted(set(re.findall(r"MIG_API[^;(]*?\b(mig_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_1912_05529_amd import mig
    return mig.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_strerror_and_version(L):
    from paper_1912_05529_amd import mig
    assert mig.strerror(0) == "success"
    assert "argument" in mig.strerror(-1)
    assert "gfx950" in mig.version()


def _desc(**kw):
    from paper_1912_05529_amd import synth
    base = dict(ntaps=25, nk=64, kmin=0.01, kmax=0.4, dx=10.0, dz=10.0)
    base.update(kw)
    return synth.TableDesc(**base)


def test_host_validation_rejects_bad_arguments(L):
    from paper_1912_05529_amd import mig
    fake = C.c_void_p(4096)
    good = mig.cdesc(_desc())
    # NULL descriptor, even N, inverted table range, NULL plane
    assert L.mig_extrapolate(fake, fake, fake, fake, fake, None, 8, 2, 1, None, None, 0, None) == -1
    even = mig.cdesc(_desc(ntaps=24))
    assert L.mig_extrapolate(fake, C.c_void_p(8192), fake, fake, fake, C.byref(even), 8, 2, 1,
                             None, None, 0, None) == -1
    inv = mig.cdesc(_desc(kmin=0.5, kmax=0.1))
    assert L.mig_migrate(fake, fake, fake, fake, C.byref(inv), 8, 4, 2, fake, fake, 1 << 20,
                         None) == -1
    assert L.mig_extrapolate(None, fake, fake, fake, fake, C.byref(good), 8, 2, 1, None, None, 0,
                             None) == -1
    # aliasing planes
    assert L.mig_extrapolate(fake, C.c_void_p(4096 + 8), fake, fake, fake, C.byref(good), 8, 2,
                             1, None, None, 0, None) == -1
    # sizes out of range
    assert L.mig_image(fake, fake, 0, 4, None) == -1
    assert L.mig_image(fake, fake, 8193, 4, None) == -1
    # rows requested without workspace
    assert L.mig_extrapolate(fake, C.c_void_p(1 << 30), fake, fake, fake, C.byref(good), 8, 2, 3,
                             fake, None, 0, None) == -4
    # design descriptor checks (zero weight breaks reweighting; ngrid too large)
    bad = mig.cdesc(_desc(w_trans=0.0))
    assert L.mig_design_workspace_size(C.byref(bad)) == 0
    assert L.mig_design_table(C.byref(bad), fake, None, None, None, fake, 1 << 20, None) == -1
    big = mig.cdesc(_desc(ngrid=4096))
    assert L.mig_design_table(C.byref(big), fake, None, None, None, fake, 1 << 30, None) == -1
    small = mig.cdesc(_desc())
    assert L.mig_design_table(C.byref(small), fake, None, None, None, fake, 16, None) == -4
    # status query without a workspace
    assert L.mig_workspace_status(None, None) == -1


def test_noalloc_entry_is_validated_on_the_host(L):
    """The allocation-free call rejects bad arguments and sizes whose one depth
    step does not fit its static workspace before touching the device."""
    from paper_1912_05529_amd import mig
    fake = C.c_void_p(4096)
    good = mig.cdesc(_desc(ntaps=35, nk=2048))
    inv = mig.cdesc(_desc(kmin=0.5, kmax=0.1))
    assert L.mig_migrate_noalloc(fake, fake, fake, fake, C.byref(inv), 8, 4, 2, fake, None) == -1
    assert L.mig_migrate_noalloc(None, fake, fake, fake, C.byref(good), 8, 4, 2, fake, None) == -1
    assert L.mig_migrate_noalloc(fake, fake, fake, fake, C.byref(good), 8, 0, 2, fake, None) == -1
    static = 64 * 1024 * 1024
    assert mig.workspace_min_size(8192, 2048, _desc(ntaps=35, nk=2048)) > static
    assert L.mig_migrate_noalloc(fake, fake, fake, fake, C.byref(good), 8192, 4, 2048, fake,
                                 None) == -4
    assert mig.workspace_min_size(1024, 200, _desc(ntaps=35, nk=2048)) < static


def test_batched_tuning_is_validated_on_the_host(L):
    from paper_1912_05529_amd import mig
    fake = C.c_void_p(4096)
    d = mig.cdesc(_desc())
    sec = (mig.CSection * 1)()
    sec[0] = mig.CSection(4096, 8192, 12288, 16384, 64, 8, 4, 0)
    ok = mig.CTuning(0, 0, 0, 0, 0)
    assert L.mig_batch_workspace_size(sec, 1, C.byref(d), C.byref(ok)) > 0
    for q in (3, 4):
        assert L.mig_batch_workspace_size(sec, 1, C.byref(d), C.byref(mig.CTuning(0, 0, 0, 0, q))) > 0
    for bad in (mig.CTuning(-1, 0, 0, 0, 0), mig.CTuning(0, -2, 0, 0, 0),
                mig.CTuning(0, 0, -5, 0, 0), mig.CTuning(0, 0, 0, 2, 0),
                mig.CTuning(0, 0, 0, 0, 2), mig.CTuning(0, 0, 0, 0, 5)):
        assert L.mig_batch_workspace_size(sec, 1, C.byref(d), C.byref(bad)) == 0
        assert L.mig_migrate_batched(sec, 1, fake, C.byref(d), C.byref(bad), fake, 1 << 30,
                                     None) == -1


def test_workspace_sizes_and_kernel_kinds(L):
    from paper_1912_05529_amd import mig
    d = _desc(ntaps=35, nk=2048)
    full = mig.workspace_size(1024, 511, 200, d)
    one = mig.workspace_min_size(1024, 200, d)
    # status word + scratch plane + block counters + sink row
    plane = 256 + 1024 * 200 * 8 + 16384 + 1024 * 4
    step = 1024 * 8 + 200 * 1024 * 4          # slowness row + partial rows
    assert one == plane + step
    assert full == plane + 511 * step
    plane_1000 = 256 + (1000 * 7 * 8 + 255) // 256 * 256 + 16384 + 1024 * 4
    assert mig.workspace_size(1000, 3, 7, d) == plane_1000 + 3 * (1024 * 8 + 7 * 1024 * 4)
    assert mig.kernel_kind(1024, 35) == 1
    assert mig.kernel_kind(1025, 35) == 3
    assert mig.kernel_kind(1536, 35) == 3
    assert mig.kernel_kind(1537, 35) == 2
    assert mig.kernel_kind(2048, 25) == 2
    assert mig.kernel_kind(2049, 25) == 0
    assert mig.kernel_kind(512, 37) == 0
    assert mig.kernel_kind(512, 36) == -1
    # demigration: slowness rows, the dense flag, per-row change points (80 bytes
    # each) and (left, right) entries per row, frequency and change point (16)
    al = lambda n: (n + 255) // 256 * 256
    assert mig.demigrate_workspace_size(1024, 512, 200, d) == (
        al(511 * 1024 * 8) + 256 + al(511 * 80) + al(511 * 200 * 16 * 4))
    assert mig.demigrate_workspace_size(1024, 0, 200, d) == 0
    assert mig.demigrate_workspace_size(1024, 4, 0, d) == 0
    # transform along t: the FP32 DFT matrix [nt][2 nw], nt <= 2^22
    assert mig.transform_workspace_size(1024, 200) == 1024 * 400 * 4
    assert mig.transform_workspace_size(4194304, 1) == 4194304 * 2 * 4
    assert mig.transform_workspace_size(4194305, 1) == 0
    assert mig.transform_workspace_size(0, 1) == 0


def test_3d_host_checks_and_workspace_sizes(L):
    from paper_1912_05529_amd import mig, synth
    fake = C.c_void_p(4096)
    d2 = synth.table2d_for(11, 64, 5.0, 40.0, 750.0, 2000.0, 10.0, 10.0)
    # 2-D design workspace: basis on the design grid, cosines on the check
    # grid, one status word per entry (each region 256-byte aligned)
    al = lambda n: (n + 255) // 256 * 256
    assert L.mig_design2d_workspace_size(C.byref(mig.cdesc(d2))) == (
        al(48 * 48 * 21 * 8) + al(192 * 6 * 8) + al(64 * 4))
    for bad in (dict(ntaps=13), dict(ngrid=65), dict(ncheck=4097)):
        import dataclasses
        cd = mig.cdesc(dataclasses.replace(d2, **bad))
        assert L.mig_design2d_workspace_size(C.byref(cd)) == 0
        assert L.mig_design_table_2d(C.byref(cd), fake, None, None, None, fake, 1 << 30,
                                     None) == -1
    # migration workspace: two planes + two groups of partial image slices
    nx, ny, nw = 100, 70, 13
    for wpg in (1, 4, 13, 50):
        ng = (nw + min(wpg, nw) - 1) // min(wpg, nw)
        assert mig.omegas_per_group_3d(nx, ny, nw, wpg) == min(wpg, nw)
        assert mig.migrate3d_workspace_size(nx, ny, nw, 5, wpg) == (
            2 * al(nx * ny * nw * 8) + 2 * al(ng * nx * ny * 8))
    assert mig.migrate3d_workspace_size(0, 8, 2, 3) == 0
    assert mig.migrate3d_workspace_size(16384, 8193, 1, 2) == 0      # plane over 2^27 points
    assert mig.migrate3d_workspace_size(16384, 8192, 1, 2) > 0
    assert mig.migrate3d_workspace_size(8, 8, 2, 0) == 0
    assert mig.omegas_per_group_3d(8, 8, 2, -1) == -1
    cd = mig.cdesc(d2)
    # NULL data, too-wide filters, too-small workspace
    assert L.mig_migrate3d(None, fake, fake, fake, C.byref(cd), 8, 8, 2, 3, 0, fake, None, fake,
                           1 << 30, None) == -1
    wide = mig.cdesc(synth.table2d_for(13, 64, 5.0, 40.0, 750.0, 2000.0, 10.0, 10.0))
    assert L.mig_migrate3d(fake, fake, fake, fake, C.byref(wide), 8, 8, 2, 3, 0, fake, None,
                           fake, 1 << 30, None) == -1
    assert L.mig_migrate3d(fake, fake, fake, fake, C.byref(cd), 8, 8, 2, 3, 1, C.c_void_p(1 << 40),
                           None, C.c_void_p(1 << 41), 16, None) == -4
