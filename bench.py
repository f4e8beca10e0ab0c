"""Throughput benchmark of the fused D2Q4 x 6 collide-stream step on one MI355X.

Workload (default): 8192 x 8192 periodic grid, log-neo-Hookean mu = 0.1, lam = 0.2,
F0 = I, initial velocity a seeded Gaussian random field with power spectrum ~ k^-3 and
rms 5e-3 (seeds 301, 302), c = 2, omega = 2, populations in FP32 with F carried as F - I.
A "step" is one time level of the whole hot path (pull streaming, moments, constitutive
update, equilibrium, collision, store, displacement quadrature) over the whole grid; inputs
are resident in HBM before timing.  The headline runs the steps in pairs through lbm_step2
(two levels per pass over HBM, bit for bit the result of two lbm_step calls); the single-
level lbm_step is timed beside it.  Also measured: FP64 and FP16 storage of the same step,
and forward + adjoint with every-K checkpointing on per-node mu, lam fields.

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
# algorithmic bytes per lattice update of one step, averaged over the 16-step cycle of the
# displacement accumulator: 24 populations read + written; u* = U + S with S (float)
# read + written every step and U (double) read + written every 16th step (FP64: u* read
# + written every step)
BYTES_PER_LU = {"f32": 96 + 96 + 16 + 32 / 16, "f16": 48 + 48 + 16 + 32 / 16, "f64": 192 + 192 + 32}
# the same per launch of the two-level kernel (lbm_step2): populations read and written
# once per two levels, S read + written once, U folded once per 8 launches
BYTES_PER_LU_PAIR = {"f32": 96 + 96 + 16 + 32 / 8, "f16": 48 + 48 + 16 + 32 / 8, "f64": 192 + 192 + 32}


PROFILE_PMC = {"step": os.path.join(ROOT, "profiles", "step_f32_lognh_periodic_8192_pmc.txt"),
               "step2": os.path.join(ROOT, "profiles", "step2_f32_lognh_periodic_8192_pmc.txt")}
STEP_SOURCES = ("lbm_forward.hip", "lbm_pair.hip", "lbm_collide.hpp", "lbm_device.hpp", "lbm_kernel_util.hpp",
                "lbm_internal.hpp")


def step_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_26677_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n, kernel="step"):
    """HBM bytes per launch of the step ("step") or two-level ("step2") kernel from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the same counters on a
    copy of known size), or None when the summary is missing, was taken at another size,
    or the kernel source changed since."""
    path = PROFILE_PMC[kernel]
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != step_source_hash() or kv.get("grid") != f"{n}x{n}":
        return None
    return float(kv["traffic_bytes_per_launch"])


def copy_ceiling():
    """Bandwidth of a plain device copy (torch elementwise kernel, 4 GiB read + 4 GiB
    written): the practical ceiling beside the published 8 TB/s."""
    import torch
    a = torch.ones(2 ** 30, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    torch.cuda.empty_cache()
    return 2 * 2 ** 32 / (ms * 1e-3) / 1e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(n):
    import lbm_inputs as li
    v0 = np.stack([li.gaussian_random_field(n, n, 301, 5e-3), li.gaussian_random_field(n, n, 302, 5e-3)])
    return v0


def time_forward(n, storage, steps, warmup, v0, law="lognh", pairs=False):
    """ms per level of `steps` levels after `warmup` untimed ones: single lbm_step calls, or
    lbm_step2 calls of two levels each (`pairs`; steps and warmup rounded up to even)."""
    import torch
    from paper_2605_26677_amd.solver import Solver
    sv = Solver(n, n, c=2.0, omega=2.0, material=law, storage=storage, mu=0.1, lam=0.2)
    sv.init(v0)
    if pairs:
        steps, warmup = steps + steps % 2, warmup + warmup % 2

    def run(k0, count):
        if pairs:
            for k in range(k0, k0 + count, 2):
                sv.step2(k)
        else:
            for k in range(k0, k0 + count):
                sv.step(k)
    run(0, warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    run(warmup, steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    faults = sv.faults()
    del sv
    torch.cuda.empty_cache()
    return ms, faults, steps


def time_block(n=1024, steps=2000, start=512):
    """The walled block workload: n x n, velocity wall (v = 0) on the left, traction-free
    elsewhere, log-NH mu = 0.1, lam = 0.3, b = (0, -1e-5) ramped over 500 steps, c = 10,
    omega = 2 - 1.6/n, FP32.  Timed from level ``start`` (past the ramp, where the block
    arguments repeat): eager lbm_step and lbm_step2 calls, and Solver.advance with single
    steps and in pairs, both replaying captured HIP graphs."""
    import torch
    import lbm_inputs as li
    from paper_2605_26677_amd.solver import Solver
    v0 = np.stack([li.gaussian_random_field(n, n, 403, 1e-3), li.gaussian_random_field(n, n, 404, 1e-3)])
    ramp = lambda k: min(1.0, k / 500)
    edges = lambda k: [(0.0, 0.0)] * 4
    out = {"grid": [n, n], "steps": steps, "start": start}
    for mode in ("eager", "eager_pairs", "graph_single", "graph_pairs"):
        sv = Solver(n, n, c=10.0, omega=2.0 - 1.6 / n, material="lognh", storage="f32", mu=0.1, lam=0.3,
                    body=(0.0, -1e-5), bc=("velocity", "traction", "traction", "traction"))
        sv.init(v0, r0=0.0)
        pairs, graph = mode.endswith("pairs"), mode.startswith("graph")
        sv.advance(0, start, ramp=ramp, edges=edges, block=64, fused=pairs, graph=graph)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if mode == "eager":
            for k in range(start, start + steps):
                sv.step(k, ramp(k), ramp(k + 1), edges=edges(k))
        elif mode == "eager_pairs":
            for k in range(start, start + steps, 2):
                sv.step2(k, ramp(k + 1), ramp(k + 2), r_n=ramp(k), edges=edges(k), edges_next=edges(k + 1))
        else:
            sv.advance(start, steps, ramp=ramp, edges=edges, block=64, fused=pairs, graph=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"{mode}_ms_per_step"] = ms
        out[f"{mode}_mlups"] = n * n / (ms * 1e-3) / 1e6
        out[f"{mode}_faults"] = sv.faults()
        del sv
        torch.cuda.empty_cache()
    return out


def time_launch_bound(n=256, steps=4000, block=100):
    """The same step on a small grid where the host launch cost dominates: per-step eager
    lbm_step calls against blocks of the same single steps replayed from a captured HIP
    graph (Solver.advance)."""
    import torch
    from paper_2605_26677_amd.solver import Solver
    v0 = make_inputs(n)
    out = {}
    for mode in ("eager", "graph"):
        sv = Solver(n, n, c=2.0, omega=2.0, storage="f32", mu=0.1, lam=0.2)
        sv.init(v0)
        for k in range(20):
            sv.step(k)
        if mode == "graph":
            sv.advance(20, 2 * block, block=block, fused=False, graph=True)   # capture outside the timed region
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if mode == "eager":
            for k in range(steps):
                sv.step(k)
        else:
            sv.advance(0, steps, block=block, fused=False, graph=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"{mode}_ms_per_step"] = ms
        out[f"{mode}_mlups"] = n * n / (ms * 1e-3) / 1e6
        assert sv.faults() == 0
        del sv
    out["grid"] = [n, n]
    out["speedup"] = out["eager_ms_per_step"] / out["graph_ms_per_step"]
    return out


def time_forward_adjoint(n, steps, K, nprobe=16, storage="f32"):
    """Forward + checkpointed adjoint of the probe-displacement loss with per-node mu, lam
    (log-normal, median 0.1 / 0.2, sigma_log 0.3, correlation length 32), every-K
    checkpoints on the device."""
    import torch
    import lbm_inputs as li
    from paper_2605_26677_amd.rollout import RolloutConfig, rollout
    torch.cuda.empty_cache()                  # the blocks of an earlier rollout
    torch.cuda.reset_peak_memory_stats()
    mu = torch.tensor(li.lognormal_field(n, n, 401, 0.1, 0.3, 32.0), device="cuda", requires_grad=True)
    lam = torch.tensor(li.lognormal_field(n, n, 402, 0.2, 0.3, 32.0), device="cuda", requires_grad=True)
    body = torch.zeros((2, n, n), dtype=torch.float64, device="cuda", requires_grad=True)
    v0 = torch.tensor(make_inputs(n), device="cuda", requires_grad=True)
    ys, xs = li.random_probes(n, n, nprobe, 405)
    probes = torch.tensor(ys * n + xs, dtype=torch.int64)
    # c from the audit bound sqrt(lam_max + 2 mu_max) / c <= 1/2 with margin
    c = float(np.ceil(2.0 * np.sqrt(float(lam.max()) + 2 * float(mu.max())) * 1.1 * 4) / 4)
    cfg = RolloutConfig(nx=n, ny=n, c=c, omega=2.0, nsteps=steps, probes=probes, storage=storage,
                        checkpoint_every=K)
    # one untimed rollout first, so that the timed one reuses the allocator's blocks
    (rollout(mu, lam, body, v0, cfg) ** 2).sum().backward()
    for t in (mu, lam, body, v0):
        t.grad = None
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    u = rollout(mu, lam, body, v0, cfg)
    e1.record()
    (u ** 2).sum().backward()
    e2.record()
    torch.cuda.synchronize()
    t_f, t_b = e0.elapsed_time(e1), e1.elapsed_time(e2)
    mem = torch.cuda.max_memory_allocated() / 2 ** 30
    ok = all(torch.isfinite(t.grad).all().item() for t in (mu, lam, v0))
    out = dict(ms_fwd=t_f, ms_bwd=t_b, mlups=n * n * steps / ((t_f + t_b) * 1e-3) / 1e6,
               bwd_over_fwd=t_b / t_f, peak_mem_GiB=mem, grads_finite=ok, steps=steps, K=K, c=c,
               storage=storage)
    del u, mu, lam, body, v0
    torch.cuda.empty_cache()
    return out


def adjoint_at_scale(n, steps, budget_gib, fd_dirs, c=10.0, host_gib=0.0):
    """The large adjoint workload: n x n, velocity wall (v = 0) at the bottom, traction
    (0, -2e-4 min(1, t/(2000 dt))) on the top evaluated at t^{m+1/2}, traction-free sides,
    per-node log-NH mu, lam log-normal fields (median 0.1 / 0.4, sigma_log 0.3, correlation
    length 32), c = 10 (traction-free corners go unstable over thousands of steps at
    lattice speeds near the P-wave bound), omega = 2 - 1.6/n, loss sum |u|^2 at 256
    random probes after `steps` steps, FP32 forward and
    adjoint with FP64 gradient accumulation, checkpoint levels planned for a device-memory
    budget.  Reports forward + adjoint throughput, peak device memory against the budget
    and the relative error of directional derivatives against FP64 central differences."""
    import torch
    import lbm_inputs as li
    from paper_2605_26677_amd.rollout import RolloutConfig, plan_checkpoints, rollout
    budget = int(budget_gib * 2 ** 30)
    plan = plan_checkpoints(n, n, "f32", steps, budget, int(host_gib * 2 ** 30))
    levels, host_top, model = plan["levels"], plan["host_top"], plan["model"]
    log(f"bench: adjoint at scale {n}^2 x {steps}, levels {levels}, outer level on host {host_top}, "
        f"model device peak {model['peak'] / 2**30:.1f} GiB, host {model['host'] / 2**30:.1f} GiB")
    mu0 = li.lognormal_field(n, n, 401, 0.1, 0.3, 32.0)
    lam0 = li.lognormal_field(n, n, 402, 0.4, 0.3, 32.0)
    ys, xs = li.random_probes(n, n, 256, 405)
    probes = torch.tensor(ys * n + xs, dtype=torch.int64)
    top = lambda m: (0.0, -2e-4 * min(1.0, (m + 0.5) / 2000.0))
    common = dict(nx=n, ny=n, c=c, omega=2.0 - 1.6 / n, nsteps=steps, probes=probes,
                  bc=("traction", "traction", "velocity", "traction"),
                  edges=lambda m: [(0.0, 0.0), (0.0, 0.0), (0.0, 0.0), top(m)])
    dev = "cuda"
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    mu = torch.tensor(mu0, dtype=torch.float64, device=dev, requires_grad=True)
    lam = torch.tensor(lam0, dtype=torch.float64, device=dev, requires_grad=True)
    body = torch.zeros((2, n, n), dtype=torch.float64, device=dev, requires_grad=True)
    v0 = torch.zeros((2, n, n), dtype=torch.float64, device=dev, requires_grad=True)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    u = rollout(mu, lam, body, v0, RolloutConfig(storage="f32", levels=levels, host_top=host_top, **common))
    e1.record()
    torch.cuda.synchronize()
    log(f"bench: forward done, {e0.elapsed_time(e1) / 1e3:.1f} s")
    (u.double() ** 2).sum().backward()
    e2.record()
    torch.cuda.synchronize()
    t_f, t_b = e0.elapsed_time(e1), e1.elapsed_time(e2)
    peak = torch.cuda.max_memory_allocated() - base_mem
    log(f"bench: backward done, {t_b / 1e3:.1f} s, peak {peak / 2**30:.1f} GiB")
    g = {k: t.grad.cpu().numpy() for k, t in (("mu", mu), ("lam", lam), ("body", body), ("v0", v0))}
    del mu, lam, body, v0, u
    torch.cuda.empty_cache()
    cfg64 = RolloutConfig(storage="f64", **common)

    def loss(p):
        with torch.no_grad():
            uu = rollout(*(torch.tensor(p[k], device=dev, dtype=torch.float32 if k != "v0" else torch.float64)
                           for k in ("mu", "lam", "body", "v0")), cfg64)
        return float((uu.double() ** 2).sum())

    base = dict(mu=mu0, lam=lam0, body=np.zeros((2, n, n)), v0=np.zeros((2, n, n)))
    scale = dict(mu=0.1, lam=0.4, body=1e-6, v0=1e-4)
    errs = []
    for d in li.fd_directions({k: base[k].shape for k in base}, fd_dirs, 406):
        plus, minus = {}, {}
        for k in base:
            step = 1e-3 * scale[k] * d[k]
            if k == "v0":
                plus[k], minus[k] = base[k] + step, base[k] - step
            else:
                plus[k], minus[k] = li.round_f32(base[k] + step), li.round_f32(base[k] - step)
        fd = loss(plus) - loss(minus)
        an = sum((g[k] * (plus[k] - minus[k])).sum() for k in base)
        errs.append(abs(fd - an) / abs(fd))
        log(f"bench: FD {fd:.6e} adjoint {an:.6e} rel {errs[-1]:.2e}")
    return dict(grid=[n, n], steps=steps, levels=levels, host_top=host_top, budget_GiB=budget_gib,
                host_budget_GiB=host_gib, model_host_GiB=model["host"] / 2 ** 30,
                model_peak_GiB=model["peak"] / 2 ** 30, peak_mem_GiB=peak / 2 ** 30,
                forward_passes=model["forward_passes"], ms_fwd=t_f, ms_bwd=t_b, bwd_over_fwd=t_b / t_f,
                mlups=n * n * steps / ((t_f + t_b) * 1e-3) / 1e6, fd_rel_err=errs, c=c)


def profile_run(n, steps):
    """Short run for rocprofv3: a plain device copy of known size (counter calibration)
    followed by FP32 steps of the benchmark workload."""
    import torch
    a = torch.ones(2 ** 29, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    v0 = make_inputs(n)
    ms, faults, _ = time_forward(n, "f32", steps, 3, v0)
    ms2, faults2, _ = time_forward(n, "f32", steps, 4, v0, pairs=True)
    adj = time_forward_adjoint(n, 20, 10)
    print(json.dumps({"profile": True, "copy_bytes_each_way": 2 ** 31, "ms_per_step": ms, "faults": faults,
                      "ms_per_level_pairs": ms2, "faults_pairs": faults2, "fwd_adj": adj}))


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
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--adjoint-every", type=int, default=50)
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3 (copy + 20 f32 steps)")
    ap.add_argument("--block", action="store_true",
                    help="only the walled 1024^2 block (single steps and pairs; separate JSON line)")
    ap.add_argument("--adjoint-at-scale", action="store_true",
                    help="the 4096^2 adjoint workload under a 64 GiB checkpoint budget (separate JSON line)")
    ap.add_argument("--scale-size", type=int, default=4096)
    ap.add_argument("--scale-steps", type=int, default=20000)
    ap.add_argument("--scale-budget-gib", type=float, default=64.0)
    ap.add_argument("--scale-fd-dirs", type=int, default=1)
    ap.add_argument("--scale-host-gib", type=float, default=48.0,
                    help="pinned host memory for the outermost checkpoints (0: device only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.size
    if args.profile:
        profile_run(n, 20)
        return
    if args.block:
        print(json.dumps({"block_1024_walls": time_block()}), flush=True)
        return
    if args.adjoint_at_scale:
        r = adjoint_at_scale(args.scale_size, args.scale_steps, args.scale_budget_gib, args.scale_fd_dirs,
                             host_gib=args.scale_host_gib)
        print(json.dumps({"adjoint_at_scale": r}), flush=True)
        return
    log(f"bench: generating {n}x{n} inputs")
    v0 = make_inputs(n)
    only = [s for s in args.only.split(",") if s] or ["f32", "f64", "f16"]
    res = {}

    def record(key, storage, ms, faults, steps, pairs):
        mlups = n * n / (ms * 1e-3) / 1e6
        bpl = BYTES_PER_LU_PAIR[storage] if pairs else BYTES_PER_LU[storage]
        launch_ms = 2 * ms if pairs else ms
        gbs = bpl * n * n / (launch_ms * 1e-3) / 1e9
        res[key] = dict(ms_per_step=ms, mlups=mlups, kernel="step2_kernel" if pairs else "step_kernel",
                        launch_ms=launch_ms, bytes_per_lu_per_launch=bpl, algorithmic_GBps=gbs,
                        frac_hbm=gbs * 1e9 / PEAK_HBM, faults=faults, steps=steps)
        log(f"bench: {key}: {ms:.3f} ms/step, {mlups:.0f} MLUPS, {gbs:.0f} GB/s per launch")

    for storage in only:
        for pairs in (True, False):
            steps = args.steps if storage == "f32" else args.variant_steps
            key = storage + ("_pairs" if pairs else "")
            log(f"bench: timing {key} forward, {steps} steps")
            ms, faults, steps = time_forward(n, storage, steps, args.warmup, v0, pairs=pairs)
            record(key, storage, ms, faults, steps, pairs)
    if "f32" in only:
        # the St. Venant-Kirchhoff variant of the same workload (FP32 storage)
        for pairs in (True, False):
            key = "svk_f32" + ("_pairs" if pairs else "")
            log(f"bench: timing {key} forward, {args.variant_steps} steps")
            ms, faults, steps = time_forward(n, "f32", args.variant_steps, args.warmup, v0, law="svk", pairs=pairs)
            record(key, "f32", ms, faults, steps, pairs)
    log("bench: walled 1024^2 block, single steps vs advance in pairs")
    res["block_1024_walls"] = time_block()
    log(f"bench: block: {res['block_1024_walls']}")
    log("bench: launch-bound grid, eager vs captured graph")
    res["launch_bound_256"] = time_launch_bound()
    log(f"bench: launch-bound: {res['launch_bound_256']}")
    if not args.no_adjoint:
        log(f"bench: forward + adjoint, {args.adjoint_steps} steps, checkpoint every {args.adjoint_every}")
        res["fwd_adj_f32"] = time_forward_adjoint(n, args.adjoint_steps, args.adjoint_every)
        log(f"bench: fwd+adj: {res['fwd_adj_f32']}")
        # FP64: half the levels and half the segment length, so that the every-K schedule
        # (the same levels per segment) fits the 268 GiB of HBM (212 GiB modelled)
        log(f"bench: forward + adjoint FP64, {args.adjoint_steps // 2} steps, "
            f"checkpoint every {args.adjoint_every // 2}")
        res["fwd_adj_f64"] = time_forward_adjoint(n, args.adjoint_steps // 2, args.adjoint_every // 2, storage="f64")
        log(f"bench: fwd+adj f64: {res['fwd_adj_f64']}")
    log("bench: copy ceiling")
    copy_gbs = copy_ceiling()
    main_storage = "f32" if "f32" in only else only[0]
    main_key = main_storage + "_pairs"
    r = res[main_key]
    traffic = measured_traffic(n, "step2") if main_storage == "f32" else None
    out = {
        "metric": METRIC, "value": r["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": r["steps"], "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": main_storage,
        "data": "synthetic",
        "config": {"workload": f"{n}x{n} periodic random-field elastic waves (k^-3 spectrum, rms 5e-3), "
                               f"log-NH mu=0.1 lam=0.2, c=2, omega=2, {main_storage} storage, "
                               f"two levels per pass (lbm_step2)",
                   "grid": [n, n], "storage": main_storage},
        "roofline": {"bound": "hbm", "kernel": "step2_kernel", "achieved": r["algorithmic_GBps"],
                     "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": r["frac_hbm"], "traffic": traffic,
                     "algorithmic_bytes_per_launch": BYTES_PER_LU_PAIR[main_storage] * n * n,
                     "launch_ms": r["launch_ms"], "copy_ceiling_GBps": copy_gbs},
        "single_step_roofline": None,
        "variants": res,
    }
    if main_storage in res:
        r1 = res[main_storage]
        out["single_step_roofline"] = {
            "bound": "hbm", "kernel": "step_kernel", "achieved": r1["algorithmic_GBps"], "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": r1["frac_hbm"],
            "traffic": measured_traffic(n, "step") if main_storage == "f32" else None,
            "algorithmic_bytes_per_launch": BYTES_PER_LU[main_storage] * n * n, "mlups": r1["mlups"]}
    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
