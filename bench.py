"""Throughput of the fused Shan-Chen D3Q19 step on one MI355X.

Workload (default): the elongated sessile cap on the 256 x 128 x 64 lattice
(footprint 150 x 36, height 24, stripe 160 x 40, reservoir plane on top),
FP32 populations.  One step = one pass of the hot path over the lattice.
Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line with the metric (MLUPS over fluid nodes), a roofline
object for the fused step kernel (algorithmic bytes / average launch time,
measured with HIP events on the launch stream) and the FP64 oracle timed on
the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import os

# the oracle's baseline is single-threaded by construction; pin BLAS pools too
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse  # noqa: E402
import json  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
BYTES_PER_ELEM = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}
METRIC = "MLUPS + % HBM roofline: plain vs FP16-storage vs batched; surrogate speedup"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_lu(prec):
    # every population of both components read once and written once
    return 2 * 19 * 2 * BYTES_PER_ELEM[prec]


def time_fluid(case, prec, steps, warmup, tile, autotune):
    import torch

    from paper_2607_06794_amd.sim import Lattice
    from tests import cases

    lat = Lattice(cases.lattice_params(case, prec, **tile), case["rho"], case["mat"])
    obs0 = lat.observables()
    n_fluid = int(obs0["fluid_nodes"])
    chosen = dict(tile)
    if autotune:
        # tile shape picked by the library's autotuner (its trial steps are
        # ordinary steps, run before the timed region)
        t = lat.autotune(trial_steps=10, cache=os.path.join(ROOT, "gpurun_out", "tiles.json"))
        chosen = {k: t[k] for k in ("tile_y", "rows_per_thread", "zchunk")}
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        lat.step(1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    obs = lat.observables()
    lat.close()
    return ms / steps, n_fluid, obs, chosen


def cpu_baseline(case, sample_steps):
    from oracle import lbm
    from tests import cases

    run = lbm.Run(case["rho"], case["mat"], cases.oracle_params(case))
    n_fluid = int((case["mat"] == 0).sum())
    t0 = time.perf_counter()
    run.step(sample_steps)
    dt = time.perf_counter() - t0
    return n_fluid * sample_steps / dt / 1e6, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--prec", default="f32", choices=list(BYTES_PER_ELEM))
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--rows-per-thread", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=5, help="oracle steps in the CPU baseline sample (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from tests import cases

    torch.cuda.init()
    case = cases.cap_case()
    tile = dict(tile_y=args.tile_y, rows_per_thread=args.rows_per_thread, zchunk=args.zchunk)
    log(f"[bench] workload cap 256x128x64 prec={args.prec} steps={args.steps} warmup={args.warmup}")
    autotune = args.tile_y == 0 and args.rows_per_thread == 0 and args.zchunk == 0
    ms, n_fluid, obs, chosen = time_fluid(case, args.prec, args.steps, args.warmup, tile, autotune)
    mlups = n_fluid / (ms * 1e-3) / 1e6
    bpl = algorithmic_bytes_per_lu(args.prec)
    achieved = bpl * n_fluid / (ms * 1e-3) / 1e9
    log(f"[bench] {ms * 1e3:.1f} us/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic")

    cpu = None
    if args.cpu_steps > 0:
        log(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps of the same lattice")
        v, dt = cpu_baseline(case, args.cpu_steps)
        cpu = {"value": v, "unit": "MLUPS", "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_steps} FP64 NumPy oracle steps of the full 256x128x64 cap from t=0 "
                         f"({dt:.1f} s, 1 of {os.cpu_count()} host cores)"}

    out = {
        "metric": METRIC,
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {
            "workload": "elongated sessile cap 256x128x64, Shan-Chen D3Q19 two-component, G=3.6, tau=1, "
                        "striped bounce-back wall, reservoir plane (rho_A=0), fused pull step",
            "lattice": [256, 128, 64],
            "fluid_nodes": n_fluid,
            "prec": args.prec,
            "rods": 0,
            "tile": chosen,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "sc_step_kernel",
            "bytes_per_lu": bpl,
        },
        "cpu_baseline": cpu,
        "status": int(obs["status"]),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
