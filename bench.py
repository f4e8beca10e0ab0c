"""Throughput benchmark of the fused D2Q4 x 6 collide-stream step on one MI355X.

Workload (default): 8192 x 8192 periodic grid, log-neo-Hookean mu = 0.1, lam = 0.2,
F0 = I, initial velocity a seeded Gaussian random field with power spectrum ~ k^-3 and
rms 5e-3 (seeds 301, 302), c = 2, omega = 2, populations in FP32 with F carried as F - I.
A "step" is one time level of the whole hot path (pull streaming, moments, constitutive
update, equilibrium, collision, store, displacement quadrature) over the whole grid; inputs
are resident in HBM before timing.  The headline runs the steps four at a time through
lbm_step_multi (four levels per pass over HBM, bit for bit the result of four lbm_step
calls); pairs through lbm_step2 and the single-level lbm_step are timed beside it.  Also
measured:
  - FP64 and FP16 storage of the same step, and the St. Venant-Kirchhoff law;
  - forward + adjoint at 8192^2 with every-K checkpointing on per-node mu, lam fields
    (FP32 200 levels every 50; FP32 and FP64 on one schedule, 100 levels every 25), with
    the HBM roofline fraction of the whole run from the kernels' algorithmic bytes;
  - the walled 1024^2 block, a launch-bound 256^2 grid with and without HIP graphs;
  - the walled 4096^2 adjoint workload (20 000 steps, 256 probes, 64 GiB device budget,
    device only and with the outermost checkpoints in pinned host memory), its gradient
    checked against FP64 central differences on 8 directions;
  - the FP64 numpy oracle on one host core.

Prints one JSON line.  Only --gpus 1 is supported.
"""
import argparse
import json
import os
import sys
import time

# the CPU baseline runs the numpy oracle on one core; set before numpy is imported
os.environ["OMP_NUM_THREADS"] = "1"
os.environ["OPENBLAS_NUM_THREADS"] = "1"
os.environ["MKL_NUM_THREADS"] = "1"

import numpy as np  # noqa: E402

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
# levels per launch of the headline (lbm_step_multi)
MULTI_LEVELS = 4


def bytes_per_lu_multi(storage, levels=MULTI_LEVELS):
    """Algorithmic bytes per node and launch of the multi-level kernel (lbm_step_multi):
    populations read and written once per launch, S read + written once, U folded on
    levels / 16 of the launches (FP64: u* read + written once)."""
    if storage == "f64":
        return 192 + 192 + 32
    pops = {"f32": 96 + 96, "f16": 48 + 48}[storage]
    return pops + 16 + 32 * levels / 16


# Single-pass algorithmic bytes per lattice update of the path (one level, every value
# through HBM once): 24 populations read + written, the compensated u* pair read + written
BYTES_PER_LU_SINGLE_PASS = {"f32": 96 + 96 + 32, "f16": 48 + 48 + 32, "f64": 192 + 192 + 32}

# Algorithmic bytes per node and launch of the kernels of the forward + adjoint run (FP32,
# per-node mu, lam and body force b, two levels per launch):
#   forward step2_kernel: populations 96 + 96, u* block sum S 8 + 8, U fold 32 / 8, mu lam 8,
#     b 8 -> 228
#   replay step2_kernel with the records of both levels, no u*: 96 + 96, records 2 x 24,
#     mu lam 8, b 8 -> 256
#   adjoint2_kernel: adjoint populations 96 + 96, F - I of two records 2 x 16, mu lam 8,
#     FP32 block sums 4 x 4 read + written 32, FP64 fold 64 / 8 -> 272
#   every-K snapshot: populations and record copied (read + written) once per K levels
# (FP64: populations 192 + 192, u* 16 + 16, records 2 x 48, adjoint F - I 2 x 32, mu lam 8,
# b 8; gradients added to the FP64 planes directly, 4 x 8 read + written per level)
# and in the multi-level kernels the rollout takes on periodic FP32 grids, T levels per launch
# (fwd_adj_multi_bytes):
#   forward march_kernel: populations 96 + 96, S 8 + 8, U fold 32 T / 16, mu lam 8, b 8
#     -> 224 + 2 T (232 at T = 4)
#   replay march_kernel with the F - I planes of the record of each level (the rollout's
#     record_planes = 4): 96 + 96, records T x 16, mu lam 8, b 8 -> 208 + 16 T (272 at T = 4)
#   march_adj_kernel: adjoint populations 96 + 96, F - I of T records T x 16, mu lam 8, FP32
#     block sums 16 + 16, FP64 fold 64 T / 16 -> 232 + 20 T (312 at T = 4)
FWD_ADJ_BYTES = {
    "f32": dict(fwd=228, replay=256, adj=272, snapshot=2 * (96 + 24)),
    "f64": dict(fwd=192 + 192 + 32 + 8 + 8, replay=192 + 192 + 96 + 8 + 8,
                adj=192 + 192 + 64 + 8 + 2 * 64, snapshot=2 * (192 + 48)),
}


# The same run in the single-pass model (every level of every pass through HBM once, per
# node and level): forward (populations, u* pair, mu lam 8, b 8) + replay (populations, the
# record of U written, mu lam, b) + adjoint (adjoint populations, U of the record, mu lam,
# FP64 gradients of mu, lam, b1, b2 read + written 64)
SINGLE_PASS_FWD_ADJ = {"f32": (224 + 16) + (192 + 24 + 16) + (192 + 24 + 8 + 64),
                       "f64": (416 + 16) + (384 + 48 + 16) + (384 + 48 + 8 + 64)}


def fwd_adj_multi_bytes(kind, levels):
    """Algorithmic bytes per node and launch of a multi-level kernel of the FP32 rollout:
    kind "fwd" (forward march), "replay" (recorded replay march) or "adj" (adjoint march)."""
    return {"fwd": 224 + 2 * levels, "replay": 208 + 16 * levels, "adj": 232 + 20 * levels}[kind]


def fwd_adj_bytes_per_level(storage, K, multi=None):
    """Algorithmic bytes per node and level of the every-K forward + adjoint run: the forward
    sweep, the recorded replay and the adjoint in launches of multi = (forward, replay,
    adjoint) levels (the multi-level kernels), or all in pairs (multi None)."""
    b = FWD_ADJ_BYTES[storage]
    if multi:
        f, r, a = multi
        return (fwd_adj_multi_bytes("fwd", f) / f + fwd_adj_multi_bytes("replay", r) / r
                + fwd_adj_multi_bytes("adj", a) / a + b["snapshot"] / K)
    return (b["fwd"] + b["replay"] + b["adj"]) / 2 + b["snapshot"] / K


PROFILE_PMC = {"step": os.path.join(ROOT, "profiles", "step_f32_lognh_periodic_8192_pmc.txt"),
               "step2": os.path.join(ROOT, "profiles", "step2_f32_lognh_periodic_8192_pmc.txt"),
               "march": os.path.join(ROOT, "profiles", "march4_f32_lognh_periodic_8192_pmc.txt")}
STEP_SOURCES = ("lbm_forward.hip", "lbm_pair.hip", "lbm_collide.hpp", "lbm_device.hpp", "lbm_kernel_util.hpp",
                "lbm_internal.hpp")
# the march kernel's sources and lbm_api.hip, which sets its launch geometry (segment length)
MARCH_SOURCES = ("lbm_march.hip", "lbm_march.hpp", "lbm_collide.hpp", "lbm_device.hpp", "lbm_kernel_util.hpp",
                 "lbm_internal.hpp", "lbm_api.hip")


def step_source_hash(files=STEP_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2605_26677_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n, kernel="step"):
    """HBM bytes per launch of the step ("step"), two-level ("step2") or four-level
    ("march") kernel from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by
    the same counters on a copy of known size), or None when the summary is missing, was
    taken at another size, or the kernel source changed since."""
    path = PROFILE_PMC[kernel]
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    files = MARCH_SOURCES if kernel == "march" else STEP_SOURCES
    if kv.get("source_sha256") != step_source_hash(files) or kv.get("grid") != f"{n}x{n}":
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


def time_forward(n, storage, steps, warmup, v0, law="lognh", mode="single"):
    """ms per level of `steps` levels after `warmup` untimed ones: single lbm_step calls
    ("single"), lbm_step2 calls of two levels each ("pairs") or lbm_step_multi calls of
    MULTI_LEVELS levels each ("multi"); steps and warmup rounded up to whole calls."""
    import torch
    from paper_2605_26677_amd.solver import Solver
    sv = Solver(n, n, c=2.0, omega=2.0, material=law, storage=storage, mu=0.1, lam=0.2)
    sv.init(v0)
    per = {"single": 1, "pairs": 2, "multi": MULTI_LEVELS}[mode]
    steps, warmup = -(-steps // per) * per, -(-warmup // per) * per

    def run(k0, count):
        for k in range(k0, k0 + count, per):
            if mode == "multi":
                sv.step_multi(k, per)
            elif mode == "pairs":
                sv.step2(k)
            else:
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
    graph (Solver.advance), and blocks of fused launches replayed the same way (the fused
    form advance takes on this grid: pairs; four-level launches pay from 1024^2)."""
    import torch
    from paper_2605_26677_amd.solver import Solver
    v0 = make_inputs(n)
    out = {}
    for mode in ("eager", "graph", "graph_fused"):
        fused = mode == "graph_fused"
        sv = Solver(n, n, c=2.0, omega=2.0, storage="f32", mu=0.1, lam=0.2)
        sv.init(v0)
        for k in range(20):
            sv.step(k)
        if mode != "eager":
            sv.advance(20, 2 * block, block=block, fused=fused, graph=True)   # capture outside the timed region
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if mode == "eager":
            for k in range(steps):
                sv.step(k)
        else:
            sv.advance(0, steps, block=block, fused=fused, graph=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"{mode}_ms_per_step"] = ms
        out[f"{mode}_mlups"] = n * n / (ms * 1e-3) / 1e6
        assert sv.faults() == 0
        del sv
    out["grid"] = [n, n]
    out["speedup"] = out["eager_ms_per_step"] / out["graph_ms_per_step"]
    out["speedup_fused"] = out["eager_ms_per_step"] / out["graph_fused_ms_per_step"]
    return out


def time_forward_adjoint(n, steps, K, nprobe=16, storage="f32", multi=None):
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
    c = float(np.ceil(2.0 * np.sqrt(float(lam.detach().max()) + 2 * float(mu.detach().max())) * 1.1 * 4) / 4)
    cfg = RolloutConfig(nx=n, ny=n, c=c, omega=2.0, nsteps=steps, probes=probes, storage=storage,
                        checkpoint_every=K, multi=multi)
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
    # the rollout's forward sweep, replay and adjoint go through the multi-level kernels on
    # this periodic grid in the shifted storages (Solver.multi_levels, replay_multi_levels,
    # adj_multi_levels), in pairs in FP64 or when turned off
    from paper_2605_26677_amd.solver import Solver
    multi = ((Solver.MULTI_LEVELS, Solver.REPLAY_MULTI_LEVELS, Solver.ADJ_MULTI_LEVELS)
             if (storage != "f64" and cfg.multi is not False) else None)
    bpl = fwd_adj_bytes_per_level(storage, K, multi)
    gbs = bpl * n * n * steps / ((t_f + t_b) * 1e-3) / 1e9
    single = SINGLE_PASS_FWD_ADJ[storage]
    out = dict(ms_fwd=t_f, ms_bwd=t_b, mlups=n * n * steps / ((t_f + t_b) * 1e-3) / 1e6,
               bwd_over_fwd=t_b / t_f, peak_mem_GiB=mem, grads_finite=ok, steps=steps, K=K, c=c,
               storage=storage,
               roofline={"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": gbs * 1e9 / PEAK_HBM,
                         "bytes_per_node_level": bpl,
                         "byte_model": (("multi-level kernels, B per node and launch / levels per launch: "
                                         f"forward march_kernel {fwd_adj_multi_bytes('fwd', multi[0])} / {multi[0]}, "
                                         f"recorded replay march_kernel {fwd_adj_multi_bytes('replay', multi[1])} / "
                                         f"{multi[1]}, march_adj_kernel {fwd_adj_multi_bytes('adj', multi[2])} / "
                                         f"{multi[2]}")
                                        if multi else
                                        ("two-level kernels, B per node and launch / 2: forward step2 "
                                         f"{FWD_ADJ_BYTES[storage]['fwd']}, recorded replay step2 "
                                         f"{FWD_ADJ_BYTES[storage]['replay']}, adjoint2 {FWD_ADJ_BYTES[storage]['adj']}"))
                                       + f"; snapshots {FWD_ADJ_BYTES[storage]['snapshot']} B per node every K levels",
                         "single_pass_bytes_per_node_level": single,
                         "single_pass_effective_GBps": single * n * n * steps / ((t_f + t_b) * 1e-3) / 1e9})
    del u, mu, lam, body, v0
    torch.cuda.empty_cache()
    return out


def adjoint_at_scale(n, steps, budget_gib, fd_dirs, c=10.0, host_gibs=(0.0,)):
    """The large adjoint workload: n x n, velocity wall (v = 0) at the bottom, traction
    (0, -2e-4 min(1, t/(2000 dt))) on the top evaluated at t^{m+1/2}, traction-free sides,
    per-node log-NH mu, lam log-normal fields (median 0.1 / 0.4, sigma_log 0.3, correlation
    length 32), c = 10 (at c near twice the P-wave speed the walled runs go unstable after
    some thousands of steps when omega is this close to 2), omega = 2 - 1.6/n, loss sum |u|^2
    at 256 random probes after `steps` steps, FP32 forward and adjoint with FP64 gradient
    accumulation, checkpoint levels planned for a device-memory budget (and, for each entry
    of host_gibs above 0, with the outermost level in that much pinned host memory).
    Reports forward + adjoint throughput, peak device memory against the budget and the
    relative error of directional derivatives against FP64 central differences: half of
    the directions perturb every parameter group at once, the others one group each (mu,
    lam, b, v0 in turn)."""
    import torch
    import lbm_inputs as li
    from paper_2605_26677_amd.rollout import RolloutConfig, plan_checkpoints, rollout
    budget = int(budget_gib * 2 ** 30)
    mu0 = li.lognormal_field(n, n, 501, 0.1, 0.3, 32.0)
    lam0 = li.lognormal_field(n, n, 502, 0.4, 0.3, 32.0)
    ys, xs = li.random_probes(n, n, 256, 505)
    probes = torch.tensor(ys * n + xs, dtype=torch.int64)
    top = lambda m: (0.0, -2e-4 * min(1.0, (m + 0.5) / 2000.0))
    common = dict(nx=n, ny=n, c=c, omega=2.0 - 1.6 / n, nsteps=steps, probes=probes,
                  bc=("traction", "traction", "velocity", "traction"),
                  edges=lambda m: [(0.0, 0.0), (0.0, 0.0), (0.0, 0.0), top(m)])
    dev = "cuda"
    runs = []
    g = None
    for host_gib in host_gibs:
        plan = plan_checkpoints(n, n, "f32", steps, budget, int(host_gib * 2 ** 30))
        levels, host_top, model = plan["levels"], plan["host_top"], plan["model"]
        log(f"bench: adjoint at scale {n}^2 x {steps}, levels {levels}, outer level on host {host_top}, "
            f"model device peak {model['peak'] / 2**30:.1f} GiB, host {model['host'] / 2**30:.1f} GiB")
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
        if g is None:
            g = {k: t.grad.cpu().numpy() for k, t in (("mu", mu), ("lam", lam), ("body", body), ("v0", v0))}
        runs.append(dict(levels=levels, host_top=host_top, host_budget_GiB=host_gib,
                         model_host_GiB=model["host"] / 2 ** 30, model_peak_GiB=model["peak"] / 2 ** 30,
                         peak_mem_GiB=peak / 2 ** 30, forward_passes=model["forward_passes"], ms_fwd=t_f,
                         ms_bwd=t_b, bwd_over_fwd=t_b / t_f, mlups=n * n * steps / ((t_f + t_b) * 1e-3) / 1e6))
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
    groups = list(base)
    dirs = li.fd_directions({k: base[k].shape for k in base}, fd_dirs, 406)
    errs, kinds, scaled, cancel = [], [], [], []
    for j, d in enumerate(dirs):
        # the first half joint, the rest one group each
        only = None if j < (fd_dirs + 1) // 2 else groups[(j - (fd_dirs + 1) // 2) % len(groups)]
        plus, minus = {}, {}
        for k in base:
            step = 1e-3 * scale[k] * d[k] * (1.0 if only in (None, k) else 0.0)
            if k == "v0":
                plus[k], minus[k] = base[k] + step, base[k] - step
            else:
                plus[k], minus[k] = li.round_f32(base[k] + step), li.round_f32(base[k] - step)
        fd = loss(plus) - loss(minus)
        an = sum((g[k] * (plus[k] - minus[k])).sum() for k in base)
        # the sum of |dL/dp_i dp_i|: where the terms of the directional derivative cancel,
        # the rounding of the FP32 adjoint shows relative to this sum, not to the result
        mag = sum(np.abs(g[k] * (plus[k] - minus[k])).sum() for k in base)
        errs.append(abs(fd - an) / abs(fd))
        scaled.append(abs(fd - an) / mag)
        cancel.append(mag / abs(an))
        kinds.append(only or "all")
        log(f"bench: FD ({kinds[-1]}) {fd:.6e} adjoint {an:.6e} rel {errs[-1]:.2e} "
            f"(sum |terms| / |result| {cancel[-1]:.1f}, error / sum |terms| {scaled[-1]:.2e})")
    best = min(runs, key=lambda r: r["ms_bwd"])
    return dict(grid=[n, n], steps=steps, budget_GiB=budget_gib, runs=runs, c=c,
                ms_fwd=best["ms_fwd"], ms_bwd=best["ms_bwd"], bwd_over_fwd=best["bwd_over_fwd"],
                mlups=best["mlups"], fd_rel_err=[float(e) for e in errs], fd_groups=kinds,
                fd_cancellation=[float(x) for x in cancel], fd_err_over_term_sum=[float(x) for x in scaled],
                fd_max_rel_err=float(max(errs)) if errs else None,
                fd_max_err_over_term_sum=float(max(scaled)) if scaled else None)


def time_levels(n=8192, steps=48, N=24):
    """ms per level against the levels each call takes, on the n x n periodic FP32 workload
    (log-NH; `steps` timed levels after 12 untimed ones, rounded up to whole calls):
    - forward, uniform mu, lam: lbm_step, lbm_step2, lbm_step_multi of 3 and 4 levels;
    - recorded replay, per-node mu, lam (the fields of the forward + adjoint run), the
      record of every level, no u*: lbm_step2 (whole records) and lbm_step_multi of 3 and 4
      levels (the F - I planes of the records, as the rollout asks);
    - adjoint with the gradients of mu, lam and b, per-node mu, lam, 16 probes: levels
      N .. 1 by lbm_adjoint_step, _step2 and _step_multi of 3 and 4 levels (best of 3)."""
    import torch
    import lbm_inputs as li
    from paper_2605_26677_amd.rollout import RolloutConfig, _Adjoint
    from paper_2605_26677_amd.solver import Solver
    v0 = make_inputs(n)
    out = {"grid": [n, n], "storage": "f32"}

    def timed(call, per, count):
        count = -(-count // per) * per
        for k in range(0, 12, per):
            call(k, per)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(12, 12 + count, per):
            call(k, per)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / count

    sv = Solver(n, n, c=2.0, omega=2.0, material="lognh", storage="f32", mu=0.1, lam=0.2)
    sv.init(v0)
    fwd = {"single": timed(lambda k, p: sv.step(k), 1, steps),
           "pairs": timed(lambda k, p: sv.step2(k), 2, steps)}
    for L in (3, 4):
        fwd[f"multi{L}"] = timed(lambda k, p: sv.step_multi(k, p), L, steps)
    fwd["faults"] = sv.faults()
    out["forward_ms_per_level"] = fwd
    del sv
    torch.cuda.empty_cache()

    mu = torch.tensor(li.lognormal_field(n, n, 401, 0.1, 0.3, 32.0), dtype=torch.float64, device="cuda")
    lam = torch.tensor(li.lognormal_field(n, n, 402, 0.2, 0.3, 32.0), dtype=torch.float64, device="cuda")
    body = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    c = float(np.ceil(2.0 * np.sqrt(float(lam.max()) + 2 * float(mu.max())) * 1.1 * 4) / 4)
    sv = Solver(n, n, c=c, omega=2.0, material="lognh", storage="f32", mu=mu, lam=lam, body=body)
    sv.init(v0)
    recs = [sv.new_record() for _ in range(4)]
    rep = {"pairs": timed(lambda k, p: sv.step2(k, record1=recs[0], record2=recs[1], ustar=False), 2, steps)}
    for L in (3, 4):
        rep[f"multi{L}"] = timed(lambda k, p: sv.step_multi(k, p, [1.0] * p, records=recs[:p], ustar=False,
                                                            record_planes=4), L, steps)
    rep["faults"] = sv.faults()
    out["replay_ms_per_level"] = rep
    del recs

    # the adjoint: records of levels 0 .. N from a fresh forward run
    sv.init(v0)
    recs = [sv.record_state(1.0, sv.new_record())]
    for k in range(N):
        r = sv.new_record()
        sv.step(k, record=r)
        recs.append(r)
    ys, xs = li.random_probes(n, n, 16, 405)
    cfg = RolloutConfig(nx=n, ny=n, c=c, omega=2.0, nsteps=N + 1, probes=torch.tensor(ys * n + xs),
                        storage="f32")
    adj = _Adjoint(sv, cfg, torch.ones((2, 16), dtype=torch.float64))
    res = {}
    for mode, per in (("single", 1), ("pairs", 2), ("multi3", 3), ("multi4", 4)):
        best = None
        for _ in range(3):
            m = N
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            while m - (per - 1) >= 1:
                if per == 1:
                    adj.step(sv, cfg, m, recs[m])
                elif per == 2:
                    adj.step2(sv, cfg, m, recs[m], recs[m - 1])
                else:
                    adj.step_multi(sv, cfg, m, [recs[m - t] for t in range(per)])
                m -= per
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (N - m)
            best = ms if best is None else min(best, ms)
        res[mode] = best
    out["adjoint_ms_per_level"] = res
    del adj, recs, sv
    torch.cuda.empty_cache()
    return out


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
    ms2, faults2, _ = time_forward(n, "f32", steps, 4, v0, mode="pairs")
    ms4, faults4, _ = time_forward(n, "f32", steps, 4, v0, mode="multi")
    adj = time_forward_adjoint(n, 20, 10)
    adj_pairs = time_forward_adjoint(n, 20, 10, multi=False)   # the two-level kernels
    print(json.dumps({"profile": True, "fwd_adj_pairs": adj_pairs, "copy_bytes_each_way": 2 ** 31, "ms_per_step": ms, "faults": faults,
                      "ms_per_level_pairs": ms2, "faults_pairs": faults2, "ms_per_level_multi": ms4,
                      "faults_multi": faults4, "fwd_adj": adj}))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s=20.0):
    """The FP64 oracle on the host, one core (OMP_NUM_THREADS=1 before numpy's import; the
    process CPU time over the wall time confirms it): the 64 x 64 shear-wave workload in full
    (200 steps) and a bounded sample of the headline workload, the 1024 x 1024 periodic
    random-field grid (at most 50 steps or budget_s seconds).  The value is the 1024^2
    sample's rate, in the headline's unit."""
    from oracle import lbm as olbm
    import lbm_inputs as li
    out = {}
    # the 64 x 64 shear wave of the plain-method workload, in full
    pb = olbm.Problem(nx=64, ny=64, c=2.0, omega=2.0, law="lognh", mu=0.1, lam=0.2)
    st = olbm.initial_state(pb, li.shear_wave_v0(64, 64))
    t0, c0 = time.perf_counter(), time.process_time()
    for _ in range(200):
        olbm.step(pb, st)
    dt1, ct1 = time.perf_counter() - t0, time.process_time() - c0
    out["shear_wave_64"] = dict(steps=200, seconds=dt1, mlups=64 * 64 * 200 / dt1 / 1e6)
    n = 1024
    v0 = make_inputs(n)
    pb = olbm.Problem(nx=n, ny=n, c=2.0, omega=2.0, law="lognh", mu=0.1, lam=0.2)
    st = olbm.initial_state(pb, v0)
    t0, c0 = time.perf_counter(), time.process_time()
    steps = 0
    while True:
        olbm.step(pb, st)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 50:
            break
    dt, ct = time.perf_counter() - t0, time.process_time() - c0
    return dict(value=n * n * steps / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"1024x1024 periodic random-field workload (the 8192^2 headline's setup on a "
                       f"1024^2 grid), {steps} FP64 numpy oracle steps, {dt:.1f} s",
                cpu_time_over_wall=(ct + ct1) / (dt + dt1), omp_num_threads=os.environ.get("OMP_NUM_THREADS"),
                cpu_model=_cpu_model(), os_cpu_count=os.cpu_count(), **out)


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
    ap.add_argument("--scale-fd-dirs", type=int, default=8)
    ap.add_argument("--scale-host-gib", default="0,48",
                    help="comma list of pinned host memory sizes (GiB) for the outermost checkpoints, "
                         "one timed run each (0: device only)")
    ap.add_argument("--no-scale", action="store_true", help="skip the 4096^2 adjoint workload")
    ap.add_argument("--fwd-adj", action="store_true",
                    help="only the FP32 forward + adjoint leg (one untimed and one timed rollout), for rocprofv3")
    ap.add_argument("--levels", action="store_true",
                    help="ms per level of forward, recorded replay and adjoint against the levels per call")
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
                             host_gibs=[float(x) for x in args.scale_host_gib.split(",")])
        print(json.dumps({"adjoint_at_scale": r}), flush=True)
        return
    if args.levels:
        print(json.dumps({"levels": time_levels(n)}), flush=True)
        return
    if args.fwd_adj:
        print(json.dumps({"fwd_adj": time_forward_adjoint(n, args.adjoint_steps, args.adjoint_every)}), flush=True)
        return
    log(f"bench: generating {n}x{n} inputs")
    v0 = make_inputs(n)
    only = [s for s in args.only.split(",") if s] or ["f32", "f64", "f16"]
    res = {}

    kernels = {"single": "step_kernel", "pairs": "step2_kernel", "multi": "march_kernel"}

    def record(key, storage, ms, faults, steps, mode):
        mlups = n * n / (ms * 1e-3) / 1e6
        per = {"single": 1, "pairs": 2, "multi": MULTI_LEVELS}[mode]
        bpl = {"single": BYTES_PER_LU[storage], "pairs": BYTES_PER_LU_PAIR[storage],
               "multi": bytes_per_lu_multi(storage)}[mode]
        launch_ms = per * ms
        gbs = bpl * n * n / (launch_ms * 1e-3) / 1e9
        res[key] = dict(ms_per_step=ms, mlups=mlups, kernel=kernels[mode], levels_per_launch=per,
                        launch_ms=launch_ms, bytes_per_lu_per_launch=bpl, algorithmic_GBps=gbs,
                        frac_hbm=gbs * 1e9 / PEAK_HBM, faults=faults, steps=steps)
        log(f"bench: {key}: {ms:.3f} ms/step, {mlups:.0f} MLUPS, {gbs:.0f} GB/s per launch")

    suffix = {"single": "", "pairs": "_pairs", "multi": f"_multi{MULTI_LEVELS}"}
    for storage in only:
        # FP64: pairs are its fastest fused form (its multi-level kernel runs short of registers)
        modes = ("pairs", "single") if storage == "f64" else ("multi", "pairs", "single")
        for mode in modes:
            steps = args.steps if (storage == "f32" and mode == "multi") else args.variant_steps
            key = storage + suffix[mode]
            log(f"bench: timing {key} forward, {steps} steps")
            ms, faults, steps = time_forward(n, storage, steps, args.warmup, v0, mode=mode)
            record(key, storage, ms, faults, steps, mode)
    if "f32" in only:
        # the St. Venant-Kirchhoff variant of the same workload (FP32 storage)
        for mode in ("multi", "single"):
            key = "svk_f32" + suffix[mode]
            log(f"bench: timing {key} forward, {args.variant_steps} steps")
            ms, faults, steps = time_forward(n, "f32", args.variant_steps, args.warmup, v0, law="svk", mode=mode)
            record(key, "f32", ms, faults, steps, mode)
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
        # the same run with the two-level kernels only (the multi-level kernels turned off)
        res["fwd_adj_f32_pairs"] = time_forward_adjoint(n, args.adjoint_steps, args.adjoint_every, multi=False)
        log(f"bench: fwd+adj pairs: {res['fwd_adj_f32_pairs']}")
        # FP32 against FP64 on one schedule: FP64 takes half the levels and half the segment
        # length, because 200 levels every 50 do not fit the 288 GB of HBM in FP64 (5
        # snapshots of 16.1 GB, 51 records of 3.2 GB, about 60 GB of working buffers)
        half_n, half_k = args.adjoint_steps // 2, args.adjoint_every // 2
        for st in ("f32", "f64"):
            log(f"bench: forward + adjoint {st}, {half_n} steps, checkpoint every {half_k}")
            res[f"fwd_adj_{st}_{half_n}"] = time_forward_adjoint(n, half_n, half_k, storage=st)
            log(f"bench: fwd+adj {st}: {res[f'fwd_adj_{st}_{half_n}']}")
    if not args.no_scale:
        log("bench: the 4096^2 walled adjoint workload")
        res["adjoint_at_scale"] = adjoint_at_scale(args.scale_size, args.scale_steps, args.scale_budget_gib,
                                                   args.scale_fd_dirs,
                                                   host_gibs=[float(x) for x in args.scale_host_gib.split(",")])
        log(f"bench: adjoint at scale: {res['adjoint_at_scale']}")
    log("bench: copy ceiling")
    copy_gbs = copy_ceiling()
    main_storage = "f32" if "f32" in only else only[0]
    main_key = main_storage + (suffix["pairs"] if main_storage == "f64" else suffix["multi"])
    r = res[main_key]
    main_kernel = "march" if r["kernel"] == "march_kernel" else "step2"
    traffic = measured_traffic(n, main_kernel) if main_storage == "f32" else None
    per = r["levels_per_launch"]
    how = (f"{per} levels per pass (lbm_step_multi)" if r["kernel"] == "march_kernel"
           else "two levels per pass (lbm_step2)")
    out = {
        "metric": METRIC, "value": r["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": r["steps"], "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": main_storage,
        "data": "synthetic",
        "config": {"workload": f"{n}x{n} periodic random-field elastic waves (k^-3 spectrum, rms 5e-3), "
                               f"log-NH mu=0.1 lam=0.2, c=2, omega=2, {main_storage} storage, {how}",
                   "grid": [n, n], "storage": main_storage},
        "roofline": {"bound": "hbm", "kernel": r["kernel"], "achieved": r["algorithmic_GBps"],
                     "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": r["frac_hbm"], "traffic": traffic,
                     "algorithmic_bytes_per_launch": r["bytes_per_lu_per_launch"] * n * n,
                     "launch_ms": r["launch_ms"], "copy_ceiling_GBps": copy_gbs,
                     "byte_models": {
                         "blocked_per_launch": {
                             "bytes_per_node": r["bytes_per_lu_per_launch"], "levels_per_launch": per,
                             "achieved_GBps": r["algorithmic_GBps"], "frac": r["frac_hbm"],
                             "note": f"what {r['kernel']} itself moves per launch ({per} levels)"},
                         "single_pass_per_level": {
                             "bytes_per_node": BYTES_PER_LU_SINGLE_PASS[main_storage],
                             "effective_GBps": BYTES_PER_LU_SINGLE_PASS[main_storage] * n * n
                             / (r["ms_per_step"] * 1e-3) / 1e9,
                             "frac": BYTES_PER_LU_SINGLE_PASS[main_storage] * n * n
                             / (r["ms_per_step"] * 1e-3) / PEAK_HBM,
                             "note": "bytes one level would move in a single pass, per level time; above 1 "
                                     f"because {per} levels share one pass"}}},
        "pairs_roofline": None,
        "single_step_roofline": None,
        "variants": res,
    }
    pk = main_storage + suffix["pairs"]
    if pk in res and pk != main_key:
        r2 = res[pk]
        out["pairs_roofline"] = {
            "bound": "hbm", "kernel": "step2_kernel", "achieved": r2["algorithmic_GBps"], "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": r2["frac_hbm"],
            "traffic": measured_traffic(n, "step2") if main_storage == "f32" else None,
            "algorithmic_bytes_per_launch": BYTES_PER_LU_PAIR[main_storage] * n * n, "mlups": r2["mlups"]}
    if main_storage in res:
        r1 = res[main_storage]
        out["single_step_roofline"] = {
            "bound": "hbm", "kernel": "step_kernel", "achieved": r1["algorithmic_GBps"], "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": r1["frac_hbm"],
            "traffic": measured_traffic(n, "step") if main_storage == "f32" else None,
            "algorithmic_bytes_per_launch": BYTES_PER_LU[main_storage] * n * n, "mlups": r1["mlups"]}
    fa = {}
    for key, label in (("fwd_adj_f32", "f32"), ("fwd_adj_f32_pairs", "f32_two_level_kernels"),
                       (f"fwd_adj_f32_{args.adjoint_steps // 2}", "f32_same_schedule_as_f64"),
                       (f"fwd_adj_f64_{args.adjoint_steps // 2}", "f64")):
        if key in res:
            v = res[key]
            fa[label] = dict(mlups=v["mlups"], frac_hbm=v["roofline"]["frac"], steps=v["steps"], K=v["K"],
                             bwd_over_fwd=v["bwd_over_fwd"])
    if fa:
        out["fwd_adjoint"] = fa
    if "f64_pairs" in res:
        out["fwd_f64"] = dict(mlups=res["f64_pairs"]["mlups"], frac_hbm=res["f64_pairs"]["frac_hbm"],
                              mlups_single=res.get("f64", {}).get("mlups"))
    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
