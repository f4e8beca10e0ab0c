"""Differentiable rollout: forward steps through lbm_step, gradients through the
hand-written adjoint kernels (lbm_adjoint_step, lbm_adjoint_init) with checkpointed
recomputation.

The quantity differentiated is the displacement at probe nodes after N steps,
u^N(X_p) (eq:trapezoid-u), with respect to per-node mu and lam fields, the per-node body
force field b (the force at level n is r(n) b) and the initial velocity v0.

Checkpointing: the forward pass keeps the post-collision populations every K levels
("every-K"); the backward pass walks the segments in reverse, restores the segment's
snapshot, replays it while recording the state U^m of each level (lbm_step(record)),
then runs the adjoint steps of that segment from its last level down to its first.
Memory: floor(N / K) + 1 snapshots of lbm_pop_bytes() + lbm_record_bytes() plus K + 1
records.  ``levels=[K0, K1, ...]`` splits the replay recursively (segment lengths
K0 > K1 > ...): each extra level re-runs the forward once more and divides the number of
live snapshots; ``checkpoint_plan`` picks the shallowest nesting whose peak device memory
fits a byte budget (``memory_model`` is the accounting it uses).
"""
import math
import ctypes
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import torch

from . import _lib as L
from .solver import EdgeData, Solver, _ptr, _stream, host_matrix


@dataclass
class RolloutConfig:
    nx: int
    ny: int
    c: float
    omega: float
    nsteps: int
    probes: torch.Tensor                              # (P,) int node indices b * nx + a
    dx: float = 1.0
    material: str = "lognh"
    storage: str = "f32"
    bc: Sequence[str] = ("periodic",) * 4
    ramp: Callable[[int], float] = lambda n: 1.0      # r(n)
    edges: Optional[Callable[[int], Sequence]] = None  # n -> data at t^{n+1/2} (4 pairs)
    u0: Optional[torch.Tensor] = None
    checkpoint_every: int = 100
    levels: Sequence[int] = field(default_factory=list)   # nested segment lengths, outermost first
    newton_max_iter: int = 0
    law_k: Optional[Sequence[float]] = None            # invariant-law constants (lbm.h law_k)
    Fbar: Optional[Sequence[Sequence[float]]] = None   # uniform predeformation at t = 0
    host_top: bool = False                             # outermost snapshots in pinned host memory
    revolve: int = 0                                   # binomial checkpointing with this many
                                                       # snapshot slots (0: every K or levels)
    pairs: Optional[bool] = None                       # forward levels in pairs (lbm_step2):
                                                       # None where faster (Solver.pairs_pay),
                                                       # True wherever they apply, False never
    force_unstable: bool = False                       # skip the lattice-speed audit (short
                                                       # runs outside its long-run region)
    multi: Optional[bool] = None                       # several levels per call (lbm_step_multi,
                                                       # lbm_adjoint_step_multi) where they apply
                                                       # and pay (Solver.multi_levels ...): None
                                                       # there, False never (pairs instead)

    def __post_init__(self):
        check_probes(self.probes, self.nx, self.ny)


def check_probes(probes, nx, ny):
    """Raises ValueError unless ``probes`` is a 1-D integer tensor of node indices in
    [0, nx * ny).  The adjoint kernels index device memory with them, and the library cannot
    inspect device memory before it launches, so the check happens here, on the host."""
    if not isinstance(probes, torch.Tensor) or probes.dim() != 1:
        raise ValueError("probes must be a 1-D tensor of node indices")
    if probes.dtype.is_floating_point or probes.dtype.is_complex or probes.dtype == torch.bool:
        raise ValueError(f"probes must hold integers, not {probes.dtype}")
    if probes.numel() == 0:
        return
    lo, hi = int(probes.min()), int(probes.max())
    if lo < 0 or hi >= int(nx) * int(ny):
        raise ValueError(f"probe indices must lie in [0, {int(nx) * int(ny)}), got [{lo}, {hi}]")


def _sizes(nx, ny, storage):
    p = L.lbm_params()
    p.nx, p.ny, p.storage = int(nx), int(ny), L.STORAGE[storage]
    lib = L.lib()
    nodes = int(nx) * int(ny)
    return dict(pop=lib.lbm_pop_bytes(ctypes.byref(p)), rec=lib.lbm_record_bytes(ctypes.byref(p)),
                ustar=lib.lbm_ustar_bytes(ctypes.byref(p)), adj=lib.lbm_adj_bytes(ctypes.byref(p)),
                gsum=lib.lbm_adj_sum_bytes(ctypes.byref(p)),
                aux=lib.lbm_aux_bytes(ctypes.byref(p)), nodes=nodes)


def memory_model(nx, ny, storage, nsteps, levels, leaf_bytes_per_node=48, host_top=False):
    """Peak device bytes of ``rollout`` with nested segment lengths ``levels`` (outermost
    first; [K] is every-K), as the sum of
      fixed:     two population buffers, u*, the float32 mu, lam, b planes, the FP64 v0,
                 u and gradient planes, two adjoint buffers and the gradient block sums,
                 and the caller's leaf tensors
                 (leaf_bytes_per_node: FP64 mu, lam, b, v0 = 48);
      snapshots: the forward's floor(N / K0) + 1 (f*, record) pairs, plus, while the
                 first top segment is reversed, ceil(K_{l-1} / K_l) - 1 more per level;
      records:   K_last + 1 records for the innermost replay.
    With host_top the forward's snapshots (the outermost level) live in pinned host
    memory instead (``host`` bytes) and leave the device; the backward then holds device
    copies of two of them (the one in use and the next one, fetched ahead)."""
    z = _sizes(nx, ny, storage)
    n, N = z["nodes"], int(nsteps)
    fixed = (2 * z["pop"] + z["ustar"] + 2 * z["aux"] + 16 * n + 16 * n + 16 * n
             + 2 * z["adj"] + z["gsum"] + 48 * n + leaf_bytes_per_node * n)
    pair = z["pop"] + z["rec"]
    K = [int(k) for k in levels]
    top = (N // K[0] + 1) * pair
    snaps = 2 * pair if host_top else top
    for a, b in zip(K[:-1], K[1:]):
        snaps += (math.ceil((a + 1) / b) - 1) * pair
    records = (K[-1] + 1) * z["rec"]
    return dict(fixed=fixed, snapshots=snaps, records=records, peak=fixed + snaps + records,
                host=top if host_top else 0, forward_passes=len(K) + 1)


def checkpoint_plan(nx, ny, storage, nsteps, budget_bytes, max_depth=8, leaf_bytes_per_node=48):
    """Segment lengths for ``RolloutConfig.levels`` whose ``memory_model`` peak fits
    budget_bytes with the fewest nesting levels (each level costs one forward replay).
    For depth d the segment lengths follow the geometric split K_l ~ N / x^(l+1) that
    balances the snapshot and record terms, refined by a small scan of x.  Raises
    ValueError when even max_depth levels do not fit."""
    N = int(nsteps)
    z = _sizes(nx, ny, storage)
    ratio = z["rec"] / (z["pop"] + z["rec"])
    best = None
    for d in range(1, max_depth + 1):
        x0 = max(1.0 + 1e-9, (N * ratio) ** (1.0 / (d + 1)))
        cands = []
        for f in (0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1, 1.25, 1.4, 1.6, 1.8, 2.0):
            x = max(1.0 + 1e-9, x0 * f)
            K = []
            for lvl in range(d):
                k = max(1, int(round(N / x ** (lvl + 1))))
                if K and k >= K[-1]:
                    k = K[-1] - 1
                if k < 1:
                    break
                K.append(k)
            if len(K) != d:
                continue
            m = memory_model(nx, ny, storage, N, K, leaf_bytes_per_node)
            cands.append((m["peak"], K, m))
        if not cands:
            continue
        peak, K, m = min(cands, key=lambda t: t[0])
        if best is None or peak < best[0]:
            best = (peak, K, m)
        if peak <= budget_bytes:
            return K
    raise ValueError(f"no nesting up to depth {max_depth} fits {budget_bytes / 2**30:.1f} GiB "
                     f"(best {best[0] / 2**30:.1f} GiB with levels {best[1]})")


def plan_checkpoints(nx, ny, storage, nsteps, device_budget_bytes, host_budget_bytes=0, max_depth=8,
                     leaf_bytes_per_node=48):
    """Checkpoint schedule with the fewest forward replays whose device peak fits
    device_budget_bytes, optionally keeping the outermost level in pinned host memory
    (at most host_budget_bytes; one host-to-device copy of a snapshot per outer segment).
    Returns dict(levels=[...], host_top=bool, model=memory_model(...))."""
    N = int(nsteps)
    best = None
    for d in range(1, max_depth + 1):
        options = []
        try:
            K = checkpoint_plan(nx, ny, storage, N, device_budget_bytes, max_depth=d,
                                leaf_bytes_per_node=leaf_bytes_per_node)
            if len(K) == d:
                options.append((K, False))
        except ValueError:
            pass
        if host_budget_bytes > 0:
            z = _sizes(nx, ny, storage)
            pair = z["pop"] + z["rec"]
            k0_min = max(1, math.ceil(N / max(1, host_budget_bytes // pair - 1)))
            for K0 in sorted({int(k0_min * f) for f in (1.0, 1.1, 1.25, 1.5, 2.0, 3.0, 4.0)} | {k0_min}):
                if K0 > N:
                    continue
                if d == 1:
                    K = [K0]
                else:
                    # inner levels split one outer segment as the device-only plan would
                    try:
                        inner = checkpoint_plan(nx, ny, storage, K0 + 1, device_budget_bytes, max_depth=d - 1,
                                                leaf_bytes_per_node=leaf_bytes_per_node)
                    except ValueError:
                        continue
                    if len(inner) != d - 1 or inner[0] >= K0:
                        continue
                    K = [K0] + inner
                m = memory_model(nx, ny, storage, N, K, leaf_bytes_per_node, host_top=True)
                if m["host"] <= host_budget_bytes:
                    options.append((K, True))
        fits = []
        for K, host in options:
            m = memory_model(nx, ny, storage, N, K, leaf_bytes_per_node, host_top=host)
            if m["peak"] <= device_budget_bytes:
                fits.append((m["peak"], K, host, m))
        if fits:
            peak, K, host, m = min(fits, key=lambda t: t[0])
            return dict(levels=K, host_top=host, model=m)
    raise ValueError(f"no schedule up to depth {max_depth} fits {device_budget_bytes / 2**30:.1f} GiB of device "
                     f"memory and {host_budget_bytes / 2**30:.1f} GiB of host memory")


def revolve_actions(start, end, leaf, slots):
    """Binomial checkpointing (Griewank's treeverse) of the reversal of levels [start, end)
    (adjoint steps end-1 .. start), holding the snapshot of `start` and `slots` more
    snapshot slots; the unit is a leaf segment of at most `leaf` levels, reversed from one
    replay that records every level.  With l units and c free slots, r is the smallest
    repetition count with beta(c, r) = C(c + r, c) >= l; the first checkpoint goes m units
    in, m in [l - beta(c - 1, r), beta(c, r - 1)], so that the part after it is reversed
    with c - 1 slots and the part before with c slots and one repetition less.

    Yields ("take", a, m): restore the snapshot of level a, step to level m and keep its
    snapshot; ("leaf", a, b): reverse levels [a, b) from the snapshot of level a;
    ("free", m): drop the snapshot of level m."""
    units = -(-(end - start) // leaf)
    if units <= 1:
        yield ("leaf", start, end)
        return
    if slots < 1:
        raise ValueError("binomial checkpointing needs a free snapshot slot for more than one leaf segment")
    r = 1
    while math.comb(slots + r, slots) < units:
        r += 1
    m_units = max(1, units - math.comb(slots - 1 + r, slots - 1))
    m_units = min(m_units, math.comb(slots + r - 1, slots), units - 1)
    mid = start + m_units * leaf
    yield ("take", start, mid)
    yield from revolve_actions(mid, end, leaf, slots - 1)
    yield ("free", mid)
    yield from revolve_actions(start, mid, leaf, slots)


class _HostPrefetch:
    """Device copies of the pinned host snapshots the backward uses, in its order of use:
    each crosses PCIe once, on a copy stream of its own (default priority), and the copy
    of the next one starts when the current one is taken, so that it overlaps the current
    segment's compute.  The copy stream first waits for the work already queued on the
    current stream, which itself waits for the forward's host copies (_HostSaver.finish)."""

    def __init__(self, device, snaps, keys):
        self.device, self.snaps, self.keys = device, snaps, list(keys)
        self.stream = torch.cuda.Stream(device=device)
        self.stream.wait_stream(torch.cuda.current_stream(device))
        self.pending = {}

    def _start(self, key):
        if key in self.pending:
            return
        with torch.cuda.stream(self.stream):
            dev = tuple(t.to(self.device, non_blocking=True) for t in self.snaps[key])
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.pending[key] = (dev, ev)

    def take(self, j):
        """The device copy of snapshot keys[j], ordered before the current stream's next
        work; starts the copy of keys[j + 1]."""
        key = self.keys[j]
        self._start(key)
        if j + 1 < len(self.keys):
            self._start(self.keys[j + 1])
        dev, ev = self.pending.pop(key)
        cur = torch.cuda.current_stream(self.device)
        cur.wait_event(ev)
        for t in dev:
            t.record_stream(cur)
        return dev


class _HostSaver:
    """Pinned host copies of the forward's snapshots on a copy stream of its own (default
    priority), so that they overlap the forward's compute: each copy starts after the work
    already queued on the current stream (the step that wrote the snapshot), the device
    tensor stays allocated until its copy is done, and ``finish`` makes the current stream
    wait for every copy, so that all later work (the backward's fetches among it) sees
    complete host snapshots."""

    def __init__(self, device):
        self.device = device
        self.stream = torch.cuda.Stream(device=device)

    def save(self, snap):
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        out = []
        with torch.cuda.stream(self.stream):
            for t in snap:
                h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
                h.copy_(t, non_blocking=True)
                t.record_stream(self.stream)
                out.append(h)
        return tuple(out)

    def finish(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)


def _edges(cfg, n):
    return EdgeData(None if cfg.edges is None else cfg.edges(n))


class _Adjoint:
    """Device buffers and the C struct of the adjoint state."""

    def __init__(self, sv: Solver, cfg: RolloutConfig, ubar: torch.Tensor):
        dev = sv.device
        nb = sv.lib.lbm_adj_bytes(ctypes.byref(sv.p))
        self.buf = [torch.zeros(nb, dtype=torch.uint8, device=dev) for _ in range(2)]
        n = sv.nx * sv.ny
        self.g_mu = torch.zeros(n, dtype=torch.float64, device=dev)
        self.g_lam = torch.zeros(n, dtype=torch.float64, device=dev)
        self.g_body = torch.zeros(2 * n, dtype=torch.float64, device=dev)
        self.g_v0 = torch.zeros(2 * n, dtype=torch.float64, device=dev)
        self.aux = torch.zeros(sv.lib.lbm_aux_bytes(ctypes.byref(sv.p)), dtype=torch.uint8, device=dev)
        self.gsum = torch.zeros(sv.lib.lbm_adj_sum_bytes(ctypes.byref(sv.p)), dtype=torch.uint8, device=dev)
        self.probe = cfg.probes.to(device=dev, dtype=torch.int32).contiguous()
        self.ubar = ubar.to(device=dev, dtype=torch.float64).contiguous()
        a = L.lbm_adj_state()
        a.adj[0], a.adj[1] = self.buf[0].data_ptr(), self.buf[1].data_ptr()
        a.cur = 0
        a.g_mu, a.g_lam, a.g_body = self.g_mu.data_ptr(), self.g_lam.data_ptr(), self.g_body.data_ptr()
        a.probe, a.ubar = self.probe.data_ptr(), self.ubar.data_ptr()
        a.nprobe = int(self.probe.numel())
        a.nsteps = int(cfg.nsteps)
        a.aux = self.aux.data_ptr()
        a.gsum = self.gsum.data_ptr()
        self.a = a
        # the probe table: the adjoint kernels add the probe sources where they write the
        # probe nodes (both levels of the two-level adjoint; the single step through the
        # state's probe_mask / probe_field)
        self.periodic = sv.periodic
        self.pmask = torch.empty(sv.lib.lbm_probe_mask_bytes(ctypes.byref(sv.p)), dtype=torch.uint8, device=dev)
        self.pfield = torch.empty(2 * n, dtype=torch.float64, device=dev)
        L.check(sv.lib.lbm_adjoint_probe_table(ctypes.byref(sv.p), ctypes.byref(self.a), _ptr(self.pmask),
                                               _ptr(self.pfield), _stream()), "lbm_adjoint_probe_table")
        a.probe_mask, a.probe_field = self.pmask.data_ptr(), self.pfield.data_ptr()

    def step(self, sv, cfg, m, record):
        L.check(sv.lib.lbm_adjoint_step(ctypes.byref(sv.p), ctypes.byref(sv.s), ctypes.byref(self.a), int(m),
                                        float(cfg.ramp(m)), ctypes.byref(_edges(cfg, m).c), _ptr(record),
                                        _stream()), "lbm_adjoint_step")

    def pair_ok(self, sv, cfg, m, lowest):
        """Levels m and m - 1 can go through lbm_adjoint_step2 (unless the configuration
        turns pairs off)."""
        return cfg.pairs is not False and lowest <= m - 1 and 1 <= m < cfg.nsteps

    def step2(self, sv, cfg, m, record_m, record_mm1):
        L.check(sv.lib.lbm_adjoint_step2(ctypes.byref(sv.p), ctypes.byref(sv.s), ctypes.byref(self.a), int(m),
                                         float(cfg.ramp(m)), float(cfg.ramp(m - 1)), ctypes.byref(_edges(cfg, m).c),
                                         ctypes.byref(_edges(cfg, m - 1).c), _ptr(record_m), _ptr(record_mm1),
                                         _ptr(self.pmask), _ptr(self.pfield), _stream()),
                "lbm_adjoint_step2")

    def step_multi(self, sv, cfg, m, records):
        """lbm_adjoint_step_multi: levels m, m - 1, ..., m - len(records) + 1 in one pass;
        records[t] holds U^{m-t}."""
        k = len(records)
        r = (ctypes.c_double * k)(*[float(cfg.ramp(m - t)) for t in range(k)])
        recs = (ctypes.c_void_p * k)(*[rec.data_ptr() for rec in records])
        L.check(sv.lib.lbm_adjoint_step_multi(ctypes.byref(sv.p), ctypes.byref(sv.s), ctypes.byref(self.a), int(m),
                                              int(k), ctypes.cast(r, ctypes.c_void_p),
                                              ctypes.cast(recs, ctypes.c_void_p), _ptr(self.pmask),
                                              _ptr(self.pfield), _stream()),
                "lbm_adjoint_step_multi")

    def init(self, sv, cfg, v0, u0):
        L.check(sv.lib.lbm_adjoint_init(ctypes.byref(sv.p), ctypes.byref(sv.s), ctypes.byref(self.a), _ptr(v0),
                                        _ptr(u0), host_matrix(cfg.Fbar), float(cfg.ramp(0)), _ptr(self.g_v0),
                                        _stream()),
                "lbm_adjoint_init")


def _restore(sv, snap):
    """Level of the snapshot as the solver's current level: its populations are lent to the
    next launch, which reads them in place (no copy), and are left unchanged.  A snapshot in
    host memory (the forward's level 0 with host_top, as binomial checkpointing reads it)
    is copied to the device first.  Returns the snapshot as the device holds it."""
    if snap[0].device.type != sv.pop[sv.s.cur].device.type:
        snap = tuple(t.to(sv.pop[sv.s.cur].device, non_blocking=True) for t in snap)
    sv.lend(snap[0])
    return snap


def _steps_to_snapshot(sv, cfg, n0, n, ustar=True):
    """Steps n0 .. n - 1 as _plain_steps, then step n -> n + 1, and keep (f*^{n+1}, U^{n+1});
    the record comes from the step kernel itself, exactly as a replay would produce it, so
    every schedule sees the same records.  Where the rollout fuses levels and a plain step
    precedes, that step and step n run as one pair that records its second level (bit for
    bit the two single steps).  The snapshot takes over the buffer the last step wrote
    (Solver.detach_current) rather than a copy of it."""
    rec = sv.new_record()
    if n > n0 and _pairs(sv, cfg):
        _plain_steps(sv, cfg, n0, n - 1, ustar=ustar)
        _pair(sv, cfg, n - 1, record2=rec, ustar=ustar)
    else:
        _plain_steps(sv, cfg, n0, n, ustar=ustar)
        sv.step(n, cfg.ramp(n), cfg.ramp(n + 1), _edges(cfg, n), record=rec, ustar=ustar)
    return (sv.detach_current(), rec)


def _pairs(sv, cfg):
    """Whether the forward levels of this rollout go two per lbm_step2 call."""
    return sv.pairs_pay if cfg.pairs is None else (bool(cfg.pairs) and sv.pairs_ok)


def _pair(sv, cfg, n, record1=None, record2=None, ustar=True):
    sv.step2(n, cfg.ramp(n + 1), cfg.ramp(n + 2), record1=record1, record2=record2, ustar=ustar,
             r_n=cfg.ramp(n), edges=_edges(cfg, n), edges_next=_edges(cfg, n + 1))


def _plain_steps(sv, cfg, n0, n1, ustar=True):
    """Steps n0 .. n1 - 1 without records: where the rollout fuses levels (_pairs), in
    groups through lbm_step_multi where that applies (Solver.multi_levels; it updates u*,
    so not where u* is skipped; a shorter group where fewer levels remain, and never a
    single level left over where two groups can share the rest) and else in pairs through
    lbm_step2; bit for bit the same result as single steps."""
    n = n0
    pairs = _pairs(sv, cfg)
    multi = sv.multi_levels if (pairs and ustar and cfg.multi is not False) else 0
    while n < n1:
        if multi and n + 1 < n1:
            L = min(multi, n1 - n)
            if n1 - n - L == 1 and L > 2:
                L -= 1
            sv.step_multi(n, L, [cfg.ramp(n + 1 + t) for t in range(L)])
            n += L
        elif pairs and n + 1 < n1:
            _pair(sv, cfg, n, ustar=ustar)
            n += 2
        else:
            sv.step(n, cfg.ramp(n), cfg.ramp(n + 1), _edges(cfg, n), ustar=ustar)
            n += 1


def _reverse_segment(sv, cfg, adj, start, end, snap, recs):
    """Adjoint levels end-1 .. start, starting from the snapshot of level `start`.  The
    replay skips the displacement quadrature (the adjoint does not read u*) and records
    U of every level, several levels per call (Solver.replay_multi_levels, else pairs;
    the multi-level calls write only the F - I planes, which is all the adjoint reads);
    the adjoint takes several levels per call (Solver.adj_multi_levels, else pairs).  The
    snapshot's populations and record are read in place: the replay's first launch reads
    the former, the adjoint's last level the latter."""
    snap = _restore(sv, snap)
    recs = [snap[1]] + recs[1:]
    n = start
    pairs = _pairs(sv, cfg)
    rmulti = sv.replay_multi_levels if (pairs and cfg.multi is not False) else 0
    while n < end - 1:
        if rmulti and n + rmulti <= end - 1:
            sv.step_multi(n, rmulti, [cfg.ramp(n + 1 + t) for t in range(rmulti)],
                          records=[recs[n + 1 + t - start] for t in range(rmulti)], ustar=False,
                          record_planes=4)
            n += rmulti
        elif pairs and n + 1 < end - 1:
            _pair(sv, cfg, n, record1=recs[n + 1 - start], record2=recs[n + 2 - start], ustar=False)
            n += 2
        else:
            sv.step(n, cfg.ramp(n), cfg.ramp(n + 1), _edges(cfg, n), record=recs[n + 1 - start], ustar=False)
            n += 1
    m = end - 1
    multi = sv.adj_multi_levels if (cfg.pairs is not False and cfg.multi is not False) else 0
    while m >= start:
        if multi and m - (multi - 1) >= start and m < cfg.nsteps:
            adj.step_multi(sv, cfg, m, [recs[m - t - start] for t in range(multi)])
            m -= multi
        elif adj.pair_ok(sv, cfg, m, start):
            adj.step2(sv, cfg, m, recs[m - start], recs[m - 1 - start])
            m -= 2
        else:
            adj.step(sv, cfg, m, recs[m - start])
            m -= 1


def _reverse_nested(sv, cfg, adj, start, end, snap, lengths, recs):
    """Reverse levels [start, end) holding only the snapshot of `start`: split into
    sub-segments of lengths[0], re-run forward to take their snapshots, recurse."""
    if not lengths or end - start <= len(recs):
        _reverse_segment(sv, cfg, adj, start, end, snap, recs)
        return
    K = lengths[0]
    bounds = list(range(start, end, K)) + [end]
    snaps = [snap]
    _restore(sv, snap)
    for i in range(len(bounds) - 2):
        snaps.append(_steps_to_snapshot(sv, cfg, bounds[i], bounds[i + 1] - 1, ustar=False))
    for i in range(len(bounds) - 2, -1, -1):
        _reverse_nested(sv, cfg, adj, bounds[i], bounds[i + 1], snaps[i], lengths[1:], recs)
        snaps.pop()


class LBMRollout(torch.autograd.Function):
    """u^N at the probes (2, P) as a differentiable function of (mu, lam, body, v0).

    mu, lam (ny, nx) and body (2, ny, nx) are used by the library in float32 (pass float64
    leaves holding float32-representable values to receive FP64 gradients); v0 (2, ny, nx)
    is used in float64.  Gradients are accumulated in FP64 and returned in each input's
    dtype."""

    @staticmethod
    def forward(ctx, mu, lam, body, v0, cfg: RolloutConfig):
        sv = Solver(cfg.nx, cfg.ny, c=cfg.c, omega=cfg.omega, dx=cfg.dx, material=cfg.material,
                    storage=cfg.storage, bc=tuple(cfg.bc), mu=mu.detach(), lam=lam.detach(),
                    body=body.detach(), newton_max_iter=cfg.newton_max_iter, law_k=cfg.law_k,
                    force_unstable=cfg.force_unstable, device=mu.device)
        v0d = v0.detach().to(torch.float64).contiguous()
        u0 = None if cfg.u0 is None else cfg.u0.to(device=mu.device, dtype=torch.float64).contiguous()
        sv.init(v0d, u0, r0=cfg.ramp(0), Fbar=cfg.Fbar)
        N = cfg.nsteps
        K = cfg.levels[0] if cfg.levels else cfg.checkpoint_every
        # checkpoints only when a gradient will be asked for (a no-grad evaluation, such as
        # a finite-difference probe, keeps nothing)
        keep = any(ctx.needs_input_grad[:4])
        snaps = {0: (sv.detach_current(), sv.record_state(cfg.ramp(0), sv.new_record()))} if keep else {}
        saver = _HostSaver(sv.device) if keep and cfg.host_top else None
        if saver:
            snaps[0] = saver.save(snaps[0])
        n = 0
        while n < N:
            # plain steps up to the next snapshot step (the one that reaches a multiple of K;
            # binomial checkpointing keeps only level 0 here)
            end = min(N, (n // K + 1) * K - 1) if keep and not cfg.revolve else N
            if end < N:
                snap = _steps_to_snapshot(sv, cfg, n, end)
                snaps[end + 1] = saver.save(snap) if saver else snap
                n = end + 1
            else:
                _plain_steps(sv, cfg, n, end)
                n = end
        if saver:
            saver.finish()
        u = sv.displacement(cfg.ramp(N))
        probes = cfg.probes.to(device=mu.device, dtype=torch.long)
        out = u.reshape(2, -1)[:, probes]
        ctx.sv, ctx.cfg, ctx.snaps, ctx.v0, ctx.u0 = sv, cfg, snaps, v0d, u0
        ctx.dtypes = (mu.dtype, lam.dtype, body.dtype, v0.dtype)
        ctx.faults = sv.faults
        return out

    @staticmethod
    def backward(ctx, grad_out):
        sv, cfg, snaps = ctx.sv, ctx.cfg, ctx.snaps
        N = cfg.nsteps
        adj = _Adjoint(sv, cfg, grad_out.detach())
        if cfg.revolve:
            K = cfg.checkpoint_every
            recs = [sv.new_record() for _ in range(K + 1)]
            for act in revolve_actions(0, N + 1, K, cfg.revolve):
                if act[0] == "take":
                    a, m = act[1], act[2]
                    _restore(sv, snaps[a])
                    snaps[m] = _steps_to_snapshot(sv, cfg, a, m - 1, ustar=False)
                elif act[0] == "free":
                    del snaps[act[1]]
                else:
                    _reverse_segment(sv, cfg, adj, act[1], act[2], snaps[act[1]], recs)
        elif cfg.levels:
            K0 = cfg.levels[0]
            inner = list(cfg.levels[1:])
            nrec = (inner[-1] if inner else K0) + 1
            recs = [sv.new_record() for _ in range(nrec)]
            bounds = list(range(0, N + 1, K0))
            if bounds[-1] != N + 1:
                bounds.append(N + 1)
            order = list(range(len(bounds) - 2, -1, -1))
            fetch = _HostPrefetch(sv.device, snaps, [bounds[i] for i in order]) if cfg.host_top else None
            for j, i in enumerate(order):
                snap = fetch.take(j) if fetch else snaps[bounds[i]]
                _reverse_nested(sv, cfg, adj, bounds[i], bounds[i + 1], snap, inner, recs)
                del snap
        else:
            K = cfg.checkpoint_every
            recs = [sv.new_record() for _ in range(K + 1)]
            starts = list(range(0, N + 1, K))
            order = list(range(len(starts) - 1, -1, -1))
            fetch = _HostPrefetch(sv.device, snaps, [starts[i] for i in order]) if cfg.host_top else None
            for j, i in enumerate(order):
                start = starts[i]
                end = min(start + K, N + 1)
                snap = fetch.take(j) if fetch else snaps[start]
                _reverse_segment(sv, cfg, adj, start, end, snap, recs)
                del snap
        adj.init(sv, cfg, ctx.v0, ctx.u0)
        ny, nx = cfg.ny, cfg.nx
        g_mu = adj.g_mu.view(ny, nx).to(ctx.dtypes[0])
        g_lam = adj.g_lam.view(ny, nx).to(ctx.dtypes[1])
        g_body = adj.g_body.view(2, ny, nx).to(ctx.dtypes[2])
        g_v0 = adj.g_v0.view(2, ny, nx).to(ctx.dtypes[3])
        return g_mu, g_lam, g_body, g_v0, None


def rollout(mu, lam, body, v0, cfg: RolloutConfig):
    return LBMRollout.apply(mu, lam, body, v0, cfg)
