#!/usr/bin/env python3
"""Throughput of explicit f-x poststack depth migration on one MI355X.

Workload: the 2-D laterally varying section (nx=1024, nz=512, dx=dz=10 m,
200 frequencies 5-55 Hz, 6-10 dipping layers 1500-4500 m/s plus a 4800 m/s
body, 35-tap extrapolators, 2048-entry table), seeded synthetic inputs.

One step = Algorithm 1 end to end on the section, inputs resident in HBM:
image row 0, then all 511 depth steps of Eq. (1) with FP32 complex
wavefields, per-point table look-up, and FP64 image rows (mig_migrate).
The table is designed once on the GPU beforehand (reported as design_ms).

Prints ONE JSON line.  value = G complex tap-MAC/s = nx*nw*(nz-1)*N / t.
roofline: the extrapolation kernel's algorithmic FP32 FLOP per launch
(nx*nw*(nz-1)*(8(M+1)+2M)) over its event-timed average duration, against
the MI355X FP32 vector peak.  cpu_baseline: the FP64 oracle on the host
cores (this is also where the FP64 reference image for the error comes
from).
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
METRIC = "f-x extrapolation G complex tap-MAC/s + image err vs FP64; batched/adjoint vs plain"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the FP64 oracle leg (no image error, no cpu_baseline)")
    ap.add_argument("--traffic", default=None,
                    help="JSON file with rocprofv3-derived HBM bytes per launch")
    ap.add_argument("--profile-only", action="store_true",
                    help="short run for profilers: warmup + steps, no oracle, no JSON extras")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB device copy (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_05529_amd import mig, synth

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")
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

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    tab = mig.design_table(desc, dev)
    e1.record(stream)
    torch.cuda.synchronize()
    design_ms = e0.elapsed_time(e1)

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
    e0.record(stream)
    for i in range(args.steps):
        step(ev[i])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    ms_kernel = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    print("timed %d steps: %.3f ms/step (events), %.3f ms/step (wall), depth-stepping launch "
          "%.3f ms" % (args.steps, ms_step, 1e3 * wall / args.steps, ms_kernel),
          file=sys.stderr, flush=True)
    # same result as the single-call entry point
    ref_img = mig.migrate(data, vel, omega, tab["tab32"], desc, ws=ws)
    assert torch.equal(ref_img, img), "staged step differs from mig_migrate"
    if args.calib_copy:
        # plain copy kernel of known size, for scaling HBM byte counters
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if args.profile_only:
        print(json.dumps({"ms_per_step": ms_step, "ms_kernel": ms_kernel}))
        return

    outputs = nx * nw * (nz - 1)
    tap_macs = outputs * N
    flop_alg = outputs * (8 * (M + 1) + 2 * M)
    value = tap_macs / (ms_step * 1e-3) / 1e9
    achieved = flop_alg / (ms_kernel * 1e-3) / 1e12
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as f:
            traffic = json.load(f).get("bytes_per_launch")

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
        "roofline": {
            "bound": "alu",
            "kernel": "depth-stepping launch: register-tap kernel, all %d depth steps, fused "
                      "image rows (mig_extrapolate with rows; includes its two small "
                      "pre-kernels)" % (nz - 1),
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": traffic,
            "ms_per_launch": round(ms_kernel, 4),
            "flop_per_launch": flop_alg,
        },
    }

    if not args.no_cpu_baseline:
        # cpu_baseline leg: the FP64 oracle, as it stands, on the host cores.
        import oracle
        omp = oracle.num_threads()
        t0 = time.time()
        otab = oracle.design_table(desc)[0]
        t_design = time.time() - t0
        t0 = time.time()
        ref = oracle.migrate(desc, otab, sec.omega, sec.vel,
                             sec.data.astype(np.complex64).astype(np.complex128))
        t_mig = time.time() - t0
        gimg = img.cpu().numpy()
        res["image_rel_l2_vs_fp64"] = float(np.linalg.norm(gimg - ref) / np.linalg.norm(ref))
        res["cpu_baseline"] = {
            "value": round(tap_macs / t_mig / 1e9, 4),
            "unit": "G complex tap-MAC/s",
            "cores": omp,
            "kind": "oracle",
            "sample": "the full workload once (all 200 frequencies, 511 depth steps, "
                      "unfolded FP64 Eq. 1, OpenMP over frequencies); table design "
                      "%.1f s not included" % t_design,
            "seconds": round(t_mig, 3),
        }
        res["speedup_vs_cpu_oracle"] = round(value / res["cpu_baseline"]["value"], 1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
