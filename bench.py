#!/usr/bin/env python3
"""Throughput of explicit f-x poststack depth migration on one MI355X.

Headline workload: the 2-D laterally varying section (nx=1024, nz=512,
dx=dz=10 m, 200 frequencies 5-55 Hz, 6-10 dipping layers 1500-4500 m/s plus
a 4800 m/s body, 35-tap extrapolators, 2048-entry table), seeded synthetic
inputs.

One step = Algorithm 1 end to end on the section, inputs resident in HBM:
image row 0, then all 511 depth steps of Eq. (1) with FP32 complex
wavefields, per-point table look-up, and FP64 image rows (the two C-ABI
stages of mig_migrate).  The table is designed once on the GPU beforehand
(reported as design_ms).

Prints ONE JSON line.  value = G complex tap-MAC/s = nx*nw*(nz-1)*N / t.
roofline: the depth-stepping launch's algorithmic FP32 FLOP
(nx*nw*(nz-1)*(8(M+1)+2M)) over its event-timed average duration, against
the MI355X FP32 vector peak.  cpu_baseline: the FP64 oracle on the host
cores (also the FP64 reference for the image error).

Extras on the same line (each against the plain per-section GPU path):
  batched  - 64 sections of uneven size in the batched form with autotuned
             knobs, vs 64 separate mig_migrate calls;
  adjoint  - demigration (the adjoint) vs migration on the headline model,
             the dot-product test at full size, and CGLS least-squares
             migration (10 iterations, 5 % noise);
  volume3d - the 3-D extension on a 256 x 256 x 200 volume with 128
             frequencies and 11 x 11 circularly symmetric extrapolators,
             with the FP64 oracle timed on its first depth steps;
  transform - the transform along t of a 1024 x 1024 t-x section to the 200
             migration frequencies on the matrix cores, with the FP64 oracle
             timed on a sample of traces.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector peak (packed FMA, 256 CU, 2.4 GHz)
# Without packed FP32 the VALU issues 64 FP32 lane-ops per clock per CU (78.6
# TFLOP/s of FMA); the folded Eq. (1) step takes 4(M+1)+2M instructions for
# 8(M+1)+2M FLOP (178 in 106 at 35 taps), so 178/106 x 39.3 T lane-op/s = 66
# TFLOP/s is this instruction mix's ceiling, and 200 frequencies on 256 CUs
# (one per workgroup) leave 200/256 of it: 51.6 TFLOP/s.
CEIL_MIX_TFLOPS = 66.0
CEIL_MIX_200CU_TFLOPS = 51.6
METRIC = "f-x extrapolation G complex tap-MAC/s + image err vs FP64; batched/adjoint vs plain"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the FP64 oracle legs (no image error, no cpu_baseline)")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no batched / adjoint / 3-D extras)")
    ap.add_argument("--traffic", default=None,
                    help="JSON file with rocprofv3-derived HBM bytes per launch "
                         "(default profiles/traffic.json)")
    ap.add_argument("--profile", choices=["plain", "batched", "adjoint", "volume3d", "transform"],
                    default=None,
                    help="short run of one part for profilers: warmup + steps, no oracle, "
                         "prints timings only")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--batched-tune", default="4,32,3",
                    help="omegas_per_group,reducers,outputs_mid for --profile batched (no "
                         "autotuning inside a profiled run)")
    ap.add_argument("--oracle-one-core", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


def profiled_traffic(args, key):
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE and WRITE_SIZE
    scaled by a copy calibration; see profiles/), or None when the kernel's
    source has changed since the counters were taken."""
    import hashlib
    path = args.traffic or os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        e = json.load(f).get(key)
    if not e:
        return None
    h = hashlib.sha1()
    for src in e["source"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return e["bytes_per_launch"] if h.hexdigest() == e["source_sha1"] else None


class Timer:
    """Event pair on the current stream."""

    def __init__(self, torch):
        self.t = torch
        self.s = torch.cuda.current_stream()
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.e0.record(self.s)
        return self

    def __exit__(self, *a):
        self.e1.record(self.s)
        self.e1.synchronize()
        self.ms = self.e0.elapsed_time(self.e1)


def timed(torch, fn, reps, warmup=1):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    with Timer(torch) as t:
        for _ in range(reps):
            fn()
    return t.ms / reps


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_one_core():
    """The oracle on one host core: the headline workload's first 40 of 200
    frequencies (all 511 depth steps), in a child process with
    OMP_NUM_THREADS=1 that touches no GPU; scaled to the whole workload it
    is the one-core throughput (frequencies are independent)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-core"],
                             env=env, capture_output=True, text=True, timeout=600, check=True)
        return json.loads(out.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError, OSError) as e:
        print("one-core oracle run failed: %s" % e, file=sys.stderr, flush=True)
        return None


def oracle_one_core_child():
    import oracle
    from paper_1912_05529_amd import synth
    sec = synth.config2()
    nsub = 40
    otab = oracle.design_table(sec.desc)[0]
    d64 = sec.data[:, :nsub].astype(np.complex64).astype(np.complex128)
    t0 = time.time()
    oracle.migrate(sec.desc, otab, sec.omega[:nsub].copy(), sec.vel, np.ascontiguousarray(d64))
    t = time.time() - t0
    macs = sec.nx * nsub * (sec.nz - 1) * sec.desc.ntaps
    print(json.dumps({"cores": oracle.num_threads(), "frequencies_run": nsub,
                      "seconds_run": round(t, 3), "seconds": round(t * sec.nw / nsub, 3),
                      "value": round(macs / t / 1e9, 4), "unit": "G complex tap-MAC/s"}))


def config1_line(torch, mig, synth, dev, args):
    """Configuration 1 (128 x 128, 64 frequencies, 25 taps): small enough that
    the step is latency, reported beside the headline."""
    sec = synth.config1()
    desc = sec.desc
    N = desc.ntaps
    M = (N - 1) // 2
    tab = mig.design_table(desc, dev)
    data = torch.from_numpy(sec.data.astype(np.complex64)).to(dev)
    vel = torch.from_numpy(sec.vel).to(dev)
    omega = torch.from_numpy(sec.omega).to(dev)
    ws = torch.empty(mig.workspace_size(sec.nx, sec.nz - 1, sec.nw, desc), dtype=torch.uint8,
                     device=dev)
    img = torch.empty((sec.nz, sec.nx), dtype=torch.float64, device=dev)
    reps = max(20, args.steps)
    ms = timed(torch, lambda: mig.migrate(data, vel, omega, tab["tab32"], desc, ws=ws, out=img),
               reps, warmup=max(3, args.warmup))
    outputs = sec.nx * sec.nw * (sec.nz - 1)
    tflops = outputs * (8 * (M + 1) + 2 * M) / (ms * 1e-3) / 1e12
    out = {
        "workload": "2-D constant velocity 2000 m/s (1000 m/s propagation), one diffraction "
                    "hyperbola: nx=128, nz=128, 64 frequencies 5-40 Hz, 25-tap extrapolators, "
                    "512-entry table, seed 1",
        "ms_per_migration": round(ms, 4),
        "G_tap_mac_per_s": round(outputs * N / (ms * 1e-3) / 1e9, 2),
        "tflops_algorithmic": round(tflops, 3),
        "frac_of_peak": round(tflops / PEAK_FP32_TFLOPS, 5),
    }
    if not args.no_cpu_baseline:
        import oracle
        otab = oracle.design_table(desc)[0]
        ref = oracle.migrate(desc, otab, sec.omega, sec.vel,
                             sec.data.astype(np.complex64).astype(np.complex128))
        got = img.cpu().numpy()
        out["image_rel_l2_vs_fp64"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["table_rel_err_vs_fp64"] = float(np.abs(tab["tab64"].cpu().numpy() - otab).max() /
                                             np.abs(otab).max())
    print("config1: %.4f ms per migration" % ms, file=sys.stderr, flush=True)
    return out


# --------------------------------------------------------------------------- #
# Headline: configuration 2, plain path.
# --------------------------------------------------------------------------- #
def headline(torch, mig, synth, dev, args):
    t_gen = time.time()
    sec = synth.config2()
    gen_s = time.time() - t_gen
    desc = sec.desc
    nx, nz, nw, N = sec.nx, sec.nz, sec.nw, desc.ntaps
    M = (N - 1) // 2
    data = torch.from_numpy(sec.data.astype(np.complex64)).to(dev)
    vel = torch.from_numpy(sec.vel).to(dev)
    omega = torch.from_numpy(sec.omega).to(dev)
    stream = torch.cuda.current_stream()

    torch.cuda.synchronize()
    with Timer(torch) as t:
        tab = mig.design_table(desc, dev)
    design_ms = t.ms

    ws = torch.empty(mig.workspace_size(nx, nz - 1, nw, desc), dtype=torch.uint8, device=dev)
    img = torch.empty((nz, nx), dtype=torch.float64, device=dev)
    rows_view = img[1:]

    # One step = mig_migrate's two C-ABI stages, called separately so that the
    # dominant launch (all depth steps with fused image rows) is event-timed
    # inside the timed region: image row 0, then mig_extrapolate with rows.
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def step(pair=None):
        mig.image_into(data, img[0])
        if pair:
            pair[0].record(stream)
        mig.extrapolate(data, vel, omega, tab["tab32"], desc, nz - 1, ws=ws,
                        rows_out=rows_view, want_plane=False)
        if pair:
            pair[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.time()
    with Timer(torch) as t:
        for i in range(args.steps):
            step(ev[i])
    wall = time.time() - t0
    ms_step = t.ms / args.steps
    ms_kernel = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    print("plain: %d steps, %.3f ms/step (events), %.3f ms/step (wall), depth-stepping "
          "launch %.3f ms" % (args.steps, ms_step, 1e3 * wall / args.steps, ms_kernel),
          file=sys.stderr, flush=True)
    ref_img = mig.migrate(data, vel, omega, tab["tab32"], desc, ws=ws)
    assert torch.equal(ref_img, img), "staged step differs from mig_migrate"
    # the extrapolation alone (image rows off), reported beside the step
    plane = torch.empty_like(data)
    ms_rows_off = timed(torch, lambda: mig.extrapolate(data, vel, omega, tab["tab32"], desc,
                                                       nz - 1, rows=False, out=plane, ws=ws),
                        args.steps, warmup=args.warmup)
    if args.calib_copy:
        # plain copy kernel of known size, for scaling HBM byte counters
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    outputs = nx * nw * (nz - 1)
    tap_macs = outputs * N
    flop_alg = outputs * (8 * (M + 1) + 2 * M)
    value = tap_macs / (ms_step * 1e-3) / 1e9
    achieved = flop_alg / (ms_kernel * 1e-3) / 1e12
    traffic = profiled_traffic(args, "mig_extrapolate config2")
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G complex tap-MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "2-D layered section with high-velocity body: nx=1024, nz=512, "
                        "dx=dz=10 m, 200 frequencies 5-55 Hz, 35-tap extrapolators, "
                        "2048-entry table, seed 2",
            "nx": nx, "nz": nz, "nw": nw, "ntaps": N, "nk": desc.nk,
            "kernel_kind": mig.kernel_kind(nx, N),
        },
        "design_ms": round(design_ms, 3),
        "gen_s": round(gen_s, 2),
        "extrapolate_rows_off": {
            "ms": round(ms_rows_off, 4),
            "tflops_algorithmic": round(flop_alg / (ms_rows_off * 1e-3) / 1e12, 3),
            "frac_of_peak": round(flop_alg / (ms_rows_off * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "depth-stepping launch: register-tap kernel, all %d depth steps, fused "
                      "image rows (mig_extrapolate with rows: its small slowness pre-kernel, "
                      "the depth-stepping kernel with reducer workgroups, and the row "
                      "kernel of the last published block)" % (nz - 1),
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": traffic,
            "ms_per_launch": round(ms_kernel, 4),
            "flop_per_launch": flop_alg,
            "frac_of_mix_ceiling": round(achieved / CEIL_MIX_TFLOPS, 4),
            "frac_of_mix_ceiling_200_of_256_cus": round(achieved / CEIL_MIX_200CU_TFLOPS, 4),
            "mix_ceiling_note": "66 TFLOP/s = unpacked FP32 issue with 178 FLOP per 106 "
                                "instructions per output; 51.6 = the same with 200 of 256 CUs "
                                "busy (one frequency per workgroup)",
        },
    }
    if not args.no_cpu_baseline:
        # cpu_baseline leg: the FP64 oracle, as it stands, on the host cores.
        import oracle
        omp = oracle.num_threads()
        t0 = time.time()
        otab = oracle.design_table(desc)[0]
        t_design = time.time() - t0
        d64 = sec.data.astype(np.complex64).astype(np.complex128)
        times = []
        for _ in range(3):   # median of three runs of the full workload
            t0 = time.time()
            ref = oracle.migrate(desc, otab, sec.omega, sec.vel, d64)
            times.append(time.time() - t0)
        t_mig = sorted(times)[1]
        gimg = img.cpu().numpy()
        res["image_rel_l2_vs_fp64"] = float(np.linalg.norm(gimg - ref) / np.linalg.norm(ref))
        res["image_worst_elem_err_vs_fp64"] = float(np.abs(gimg - ref).max() / np.abs(ref).max())
        t64 = tab["tab64"].cpu().numpy()
        res["table_rel_err_vs_fp64"] = float(np.abs(t64 - otab).max() / np.abs(otab).max())
        one = oracle_one_core()
        res["cpu_baseline"] = {
            "value": round(tap_macs / t_mig / 1e9, 4),
            "unit": "G complex tap-MAC/s",
            "cores": omp,
            "kind": "oracle",
            "sample": "the full workload (all 200 frequencies, 511 depth steps, unfolded "
                      "FP64 Eq. 1, OpenMP over frequencies), median of 3 runs; table "
                      "design %.1f s not included; one_core: the first 40 frequencies on "
                      "one thread in a child process, scaled by 200/40" % t_design,
            "seconds": round(t_mig, 3),
            "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "one_core": one,
        }
        res["speedup_vs_cpu_oracle"] = round(value / res["cpu_baseline"]["value"], 1)
        if one and one.get("seconds"):
            res["speedup_vs_cpu_oracle_one_core"] = round(value / (tap_macs / one["seconds"] / 1e9), 1)
    if not args.profile:
        res["config1"] = config1_line(torch, mig, synth, dev, args)
    ctx = {"sec": sec, "tab": tab, "data": data, "vel": vel, "omega": omega, "ws": ws,
           "ms_plain": ms_step}
    return res, ctx


# --------------------------------------------------------------------------- #
# Batched form: configuration 3.
# --------------------------------------------------------------------------- #
def batched(torch, mig, synth, dev, args, profile=False):
    from paper_1912_05529_amd import tune
    secs = synth.config3()
    desc = secs[0].desc
    tab = mig.design_table(desc, dev)
    batch = [{"data": torch.from_numpy(s.data.astype(np.complex64)).to(dev),
              "vel": torch.from_numpy(s.vel).to(dev),
              "omega": torch.from_numpy(s.omega).to(dev)} for s in secs]
    if profile:
        g, nred, qm = (int(v) for v in args.batched_tune.split(","))
        best, table = {"omegas_per_group": g, "reducers": nred, "outputs_mid": qm}, []
    else:
        best, table = tune.autotune(batch, tab["tab32"], desc, reps=1)
    ws_b = torch.empty(max(mig.batch_workspace_size(batch, desc, best), 1), dtype=torch.uint8,
                       device=dev)
    reps = max(1, args.steps // 4)
    ms_b = timed(torch, lambda: mig.migrate_batched(batch, tab["tab32"], desc, tune=best,
                                                    ws=ws_b), reps)
    if profile:
        print(json.dumps({"part": "batched", "ms": ms_b, "tune": best}))
        return None
    need = max(mig.workspace_size(b["data"].shape[0], b["vel"].shape[0] - 1,
                                  b["data"].shape[1], desc) for b in batch)
    ws_p = torch.empty(need, dtype=torch.uint8, device=dev)
    outs = [torch.empty_like(b["image"]) for b in batch]

    def plain():
        for b, o in zip(batch, outs):
            mig.migrate(b["data"], b["vel"], b["omega"], tab["tab32"], desc, ws=ws_p, out=o)
    ms_p = timed(torch, plain, reps)
    plain()
    mig.migrate_batched(batch, tab["tab32"], desc, tune=best, ws=ws_b)
    torch.cuda.synchronize()
    same = all(torch.equal(b["image"], o) for b, o in zip(batch, outs))
    tap_macs = sum(s.nx * s.nw * (s.nz - 1) * desc.ntaps for s in secs)
    M = (desc.ntaps - 1) // 2
    flop = sum(s.nx * s.nw * (s.nz - 1) for s in secs) * (8 * (M + 1) + 2 * M)
    out = {
        "workload": "64 sections, seed-drawn nx 256-2048, nz 200-800, nw 100-300, 35-tap "
                    "table, seed 3",
        "ms_batched": round(ms_b, 3),
        "ms_plain_64_calls": round(ms_p, 3),
        "speedup_vs_plain": round(ms_p / ms_b, 3),
        "G_tap_mac_per_s_batched": round(tap_macs / ms_b / 1e6, 1),
        "G_tap_mac_per_s_plain": round(tap_macs / ms_p / 1e6, 1),
        "tune": best,
        "tune_candidates": len(table),
        "tune_spread_pct": round(100.0 * (max(r["ms"] for r in table) /
                                          min(r["ms"] for r in table) - 1.0), 2),
        "tune_best_by_outputs_mid": {
            str(q): round(min(r["ms"] for r in table if r["tune"]["outputs_mid"] == q), 3)
            for q in (3, 4)},
        "images_bit_identical_to_plain": bool(same),
        "roofline": {
            "bound": "alu",
            "kernel": "the batched launches (one per kernel variant) with their small "
                      "pre-kernels, folded Eq. 1 FLOP of every section",
            "achieved": round(flop / (ms_b * 1e-3) / 1e12, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(flop / (ms_b * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            "traffic": profiled_traffic(args, "mig_migrate_batched config3"),
            "traffic_note": "HBM bytes per batched call (tuning 2, 32, 4), mostly the partial "
                            "image rows: 4 B per output written and read, rows padded to 256 "
                            "points",
        },
    }
    print("batched: %.3f ms vs plain %.3f ms (%s)" % (ms_b, ms_p, best), file=sys.stderr,
          flush=True)
    return out


# --------------------------------------------------------------------------- #
# Adjoint and least-squares migration: configuration 2's model.
# --------------------------------------------------------------------------- #
def adjoint(torch, mig, synth, dev, args, ctx=None, profile=False):
    from paper_1912_05529_amd import lsm
    if ctx is None:
        sec = synth.config2(with_data=False)
        tab = mig.design_table(sec.desc, dev)
        ctx = {"sec": sec, "tab": tab, "vel": torch.from_numpy(sec.vel).to(dev),
               "omega": torch.from_numpy(sec.omega).to(dev)}
    sec, tab, vel, omega = ctx["sec"], ctx["tab"], ctx["vel"], ctx["omega"]
    desc = sec.desc
    refl = torch.from_numpy(sec.extra["refl"]).to(dev)
    nz, nx = refl.shape
    ws_a = torch.empty(max(mig.demigrate_workspace_size(nx, nz, sec.nw, desc), 1), dtype=torch.uint8,
                       device=dev)
    d = torch.empty((nx, sec.nw), dtype=torch.complex64, device=dev)
    reps = max(1, args.steps // 4)
    ms_adj = timed(torch, lambda: mig.demigrate(refl, vel, omega, tab["tab32"], desc, out=d,
                                                ws=ws_a), reps)
    if profile:
        print(json.dumps({"part": "adjoint", "ms": ms_adj}))
        return None
    ws_m = torch.empty(mig.workspace_size(nx, nz - 1, sec.nw, desc), dtype=torch.uint8,
                       device=dev)
    img = torch.empty((nz, nx), dtype=torch.float64, device=dev)
    ms_fwd = timed(torch, lambda: mig.migrate(d, vel, omega, tab["tab32"], desc, ws=ws_m,
                                              out=img), reps)
    # dot-product test at full size: <A d, m> = <d, A^T m>
    g = torch.Generator(device="cpu").manual_seed(9)
    dd = (torch.randn((nx, sec.nw), generator=g) + 1j * torch.randn((nx, sec.nw), generator=g))
    dd = dd.to(torch.complex64).to(dev)
    mm = torch.randn((nz, nx), generator=g, dtype=torch.float64).to(dev)
    Ad = mig.migrate(dd, vel, omega, tab["tab32"], desc)
    Atm = mig.demigrate(mm, vel, omega, tab["tab32"], desc)
    lhs = float(torch.sum(Ad * mm))
    rhs = float(torch.sum(dd.real.double() * Atm.real.double() + dd.imag.double() * Atm.imag.double()))
    dot_rel = abs(lhs - rhs) / (float(torch.linalg.norm(Ad)) * float(torch.linalg.norm(mm)))
    # CGLS on the layered model's reflectivity with 5 % noise
    d_clean = mig.demigrate(refl, vel, omega, tab["tab32"], desc)
    rms = float(torch.sqrt(torch.mean(torch.abs(d_clean) ** 2)))
    noise = (torch.randn(d_clean.shape, generator=g) + 1j * torch.randn(d_clean.shape, generator=g))
    d_obs = d_clean + (0.05 * rms / np.sqrt(2.0) * noise).to(torch.complex64).to(dev)
    lsm.cgls(d_obs, vel, omega, tab["tab32"], desc, niter=1)   # warm-up (first-use kernels)
    torch.cuda.synchronize()
    with Timer(torch) as t:
        m, hist = lsm.cgls(d_obs, vel, omega, tab["tab32"], desc, niter=10)
    err = float(torch.linalg.norm(m - refl) / torch.linalg.norm(refl))
    # what the operator can recover: CGLS from zero converges to the
    # minimum-norm least-squares solution, so on the noise-free data it
    # tends to the reflectivity projected onto the range of A (the part the
    # 5-55 Hz band and the propagating wavenumbers carry); 200 iterations
    m_rec, hist_rec = lsm.cgls(d_clean, vel, omega, tab["tab32"], desc, niter=200)
    nrec = float(torch.linalg.norm(m_rec))
    err_rec = float(torch.linalg.norm(m - m_rec)) / nrec
    mig_img = mig.migrate(d_obs, vel, omega, tab["tab32"], desc)
    sc = float(torch.sum(mig_img * m_rec) / torch.sum(mig_img * mig_img))
    err_mig_rec = float(torch.linalg.norm(sc * mig_img - m_rec)) / nrec
    sc_t = float(torch.sum(mig_img * refl) / torch.sum(mig_img * mig_img))
    err_mig = float(torch.linalg.norm(sc_t * mig_img - refl) / torch.linalg.norm(refl))
    # algorithmic FLOP as for migration: the folded Eq. (1) count per output
    # and step (the corrections at lateral changes are overhead)
    M = (desc.ntaps - 1) // 2
    flop_adj = nx * sec.nw * (nz - 1) * (8 * (M + 1) + 2 * M)
    out = {
        "workload": "adjoint of the headline section's migration (reflectivity -> data), "
                    "and CGLS least-squares migration with 5 % Gaussian noise, 10 iterations",
        "ms_demigrate": round(ms_adj, 3),
        "ms_migrate": round(ms_fwd, 3),
        "adjoint_vs_plain_time": round(ms_adj / ms_fwd, 3),
        "dot_product_rel_err": dot_rel,
        "cgls_ms_total": round(t.ms, 2),
        "cgls_ms_operators": round(11 * ms_fwd + 10 * ms_adj, 2),
        "cgls_residual_history": [round(h, 4) for h in hist],
        "cgls_model_rel_err": round(err, 4),
        "best_scaled_migration_rel_err": round(err_mig, 4),
        "recoverable": {
            "definition": "CGLS, 200 iterations from zero on the noise-free data: the "
                          "minimum-norm solution, i.e. the reflectivity projected onto the "
                          "range of the migration operator",
            "norm_fraction_of_true": round(nrec / float(torch.linalg.norm(refl)), 4),
            "rel_residual_after_200": round(hist_rec[-1], 5),
            "cgls10_rel_err_vs_recoverable": round(err_rec, 4),
            "best_scaled_migration_rel_err_vs_recoverable": round(err_mig_rec, 4),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "demigration: slowness and change-point pre-kernels, the folded adjoint "
                      "kernel (all depth steps; exact corrections at lateral changes) and the "
                      "product kernel's immediate return",
            "achieved": round(flop_adj / (ms_adj * 1e-3) / 1e12, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(flop_adj / (ms_adj * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            "flop_per_output": 8 * (M + 1) + 2 * M,
            "traffic": profiled_traffic(args, "mig_demigrate config2"),
        },
    }
    print("adjoint: %.3f ms vs migrate %.3f ms; CGLS %.1f ms" % (ms_adj, ms_fwd, t.ms),
          file=sys.stderr, flush=True)
    return out


# --------------------------------------------------------------------------- #
# 3-D extension: configuration 5.
# --------------------------------------------------------------------------- #
def volume3d(torch, mig, synth, dev, args, profile=False):
    t0 = time.time()
    vol = synth.config5(with_data=not profile)
    gen_s = time.time() - t0
    desc = vol.desc
    nx, ny, nz, nw = vol.nx, vol.ny, vol.nz, vol.nw
    M = (desc.ntaps - 1) // 2
    nu = (M + 1) * (M + 2) // 2
    if profile:
        rng = np.random.default_rng(5)
        vol.data = rng.standard_normal((nx, ny, nw)) + 1j * rng.standard_normal((nx, ny, nw))
    data = torch.from_numpy(np.ascontiguousarray(
        np.moveaxis(vol.data.astype(np.complex64), 2, 0))).to(dev)
    vel = torch.from_numpy(vol.vel).to(dev)
    omega = torch.from_numpy(vol.omega).to(dev)
    with Timer(torch) as t:
        tab = mig.design_table_2d(desc, dev)
    design_ms = t.ms
    ws = torch.empty(mig.migrate3d_workspace_size(nx, ny, nw, nz), dtype=torch.uint8, device=dev)
    img = torch.empty((nz, nx, ny), dtype=torch.float64, device=dev)
    reps = max(1, args.steps // 5)
    ms = timed(torch, lambda: mig.migrate3d(data, vel, omega, tab["tab32"], desc, ws=ws, out=img),
               reps)
    if profile:
        print(json.dumps({"part": "volume3d", "ms": ms}))
        return None
    outputs = nx * ny * nw * (nz - 1)
    flop_out = 8 * nu + 2 * ((2 * M + 1) ** 2 - nu)   # folded form: unique MACs + orbit adds
    achieved = outputs * flop_out / (ms * 1e-3) / 1e12
    out = {
        "workload": "3-D layered volume with an ellipsoidal body: nx=ny=256, nz=200, "
                    "dx=dy=dz=10 m, 128 frequencies 5-40 Hz, 11x11 circularly symmetric "
                    "extrapolators (21 unique taps), 1024-entry table, seed 5",
        "ms_per_volume": round(ms, 3),
        "us_per_depth_step": round(1e3 * ms / (nz - 1), 2),
        "G_outputs_per_s": round(outputs / ms / 1e6, 2),
        "G_tap_mac_per_s_nominal": round(outputs * (2 * M + 1) ** 2 / ms / 1e6, 1),
        "design_ms": round(design_ms, 2),
        "gen_s": round(gen_s, 2),
        "omegas_per_group": mig.omegas_per_group_3d(nx, ny, nw, 0),
        "roofline": {
            "bound": "alu",
            "kernel": "3-D depth step (one launch per step), averaged over the volume "
                      "including the image and reduction launches",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "flop_per_output": flop_out,
            "traffic": profiled_traffic(args, "k_step3d<5> config5"),
        },
    }
    if not args.no_cpu_baseline:
        import oracle
        k = 3
        otab = oracle.design_table_2d(desc)[0]   # the oracle's own table
        t0 = time.time()
        ref = oracle.migrate3d(desc, otab, vol.omega, np.ascontiguousarray(vol.vel[:k + 1]),
                               vol.data.astype(np.complex64).astype(np.complex128))
        t_or = time.time() - t0
        sub = torch.empty((k + 1, nx, ny), dtype=torch.float64, device=dev)
        mig.migrate3d(data, vel[:k + 1].contiguous(), omega, tab["tab32"], desc, out=sub)
        got = sub.cpu().numpy()
        out["image_rel_l2_vs_fp64_first_steps"] = float(
            np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["cpu_baseline"] = {
            "value": round(nx * ny * nw * k / t_or / 1e9, 4),
            "unit": "G outputs/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "the first %d depth steps of the volume (all frequencies, unfolded "
                      "FP64 2-D Eq. 1)" % k,
            "seconds": round(t_or, 3),
        }
        out["speedup_vs_cpu_oracle"] = round(out["G_outputs_per_s"] /
                                             out["cpu_baseline"]["value"], 1)
    print("volume3d: %.3f ms per volume (%.1f us/step)" % (ms, out["us_per_depth_step"]),
          file=sys.stderr, flush=True)
    return out


# --------------------------------------------------------------------------- #
# Transform along t (Algorithm 1, first step) on the matrix cores.
# --------------------------------------------------------------------------- #
def transform(torch, mig, synth, dev, args, profile=False):
    nx, nt, dt = 1024, 1024, 0.004
    om = synth.omegas(200, 5.0, 55.0)
    nw = om.size
    rng = np.random.default_rng(12)
    p = rng.standard_normal((nx, nt)).astype(np.float32)
    sec = torch.from_numpy(p).to(dev)
    omega = torch.from_numpy(om).to(dev)
    out = torch.empty((nx, nw), dtype=torch.complex64, device=dev)
    ws = torch.empty(max(mig.transform_workspace_size(nt, nw), 1), dtype=torch.uint8,
                     device=dev)
    reps = max(1, args.steps)
    ms = timed(torch, lambda: mig.transform_t(sec, dt, omega, out=out, ws=ws), reps)
    if profile:
        print(json.dumps({"part": "transform", "ms": ms}))
        return None
    flop = 2.0 * nx * nt * 2 * nw      # real [nx][nt] x [nt][2 nw]
    res = {
        "workload": "t-x section nx=1024, nt=1024, dt=4 ms (seeded Gaussian samples) to the "
                    "200 migration frequencies 5-55 Hz: DFT matrix built in FP64, product on "
                    "FP32 MFMA",
        "ms": round(ms, 4),
        "roofline": {
            "bound": "mfma",
            "kernel": "mig_transform_t: DFT-matrix kernel + v_mfma_f32_16x16x4f32 product",
            "achieved": round(flop / (ms * 1e-3) / 1e12, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(flop / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            "flop_per_launch": flop,
            "traffic": profiled_traffic(args, "mig_transform_t 1024x1024x200"),
        },
    }
    if not args.no_cpu_baseline:
        import oracle
        k = 64                               # sampled traces
        t0 = time.time()
        ref = oracle.transform_t(p[:k], dt, om)
        t_or = time.time() - t0
        got = out[:k].cpu().numpy()
        res["rel_l2_vs_fp64_sample"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        res["cpu_baseline"] = {
            "value": round(2.0 * k * nt * 2 * nw / t_or / 1e9, 3),
            "unit": "GFLOP/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "the first %d of the 1024 traces (FP64 direct DFT)" % k,
            "seconds": round(t_or, 4),
        }
    print("transform: %.4f ms (%.1f TFLOP/s)" % (ms, res["roofline"]["achieved"]),
          file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.oracle_one_core:
        oracle_one_core_child()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU; runs over several GPUs are not supported "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_05529_amd import mig, synth

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")

    if args.profile == "batched":
        batched(torch, mig, synth, dev, args, profile=True)
        return
    if args.profile == "adjoint":
        adjoint(torch, mig, synth, dev, args, profile=True)
        return
    if args.profile == "volume3d":
        volume3d(torch, mig, synth, dev, args, profile=True)
        return
    if args.profile == "transform":
        transform(torch, mig, synth, dev, args, profile=True)
        return
    if args.profile == "plain":
        args.no_cpu_baseline = True
    res, ctx = headline(torch, mig, synth, dev, args)
    if args.profile == "plain":
        print(json.dumps({"part": "plain", "ms_per_step": res["ms_per_step"],
                          "ms_kernel": res["roofline"]["ms_per_launch"]}))
        return
    if not args.no_extras:
        res["batched"] = batched(torch, mig, synth, dev, args)
        res["adjoint"] = adjoint(torch, mig, synth, dev, args, ctx)
        res["volume3d"] = volume3d(torch, mig, synth, dev, args)
        res["transform"] = transform(torch, mig, synth, dev, args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
