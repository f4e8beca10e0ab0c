"""Device-resident solver state and thin wrappers of the C ABI (include/lbm.h).

PyTorch supplies device memory and the stream; every compute step is a call into the
HIP library.  A ``Solver`` owns the two population buffers, the displacement accumulator,
the traction staging buffer, the fault word and the optional per-node parameter fields.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class EdgeData:
    """Boundary data at one half step: per edge either a pair (uniform along the edge) or
    a (2, L) float64 device tensor."""

    def __init__(self, values=None):
        self.c = L.lbm_edge_data()
        self._keep = []
        for e in range(4):
            v = None if values is None else values[e]
            if v is None:
                continue
            if isinstance(v, torch.Tensor):
                t = v.to(torch.float64).contiguous()
                self._keep.append(t)
                self.c.field[e] = t.data_ptr()
            else:
                self.c.value[e][0] = float(v[0])
                self.c.value[e][1] = float(v[1])


def host_matrix(F):
    """A (2, 2) matrix as a host array of 4 doubles (row-major), or None."""
    if F is None:
        return None
    vals = [float(v) for v in torch.as_tensor(F, dtype=torch.float64).reshape(-1).tolist()]
    if len(vals) != 4:
        raise ValueError("a 2 x 2 matrix is expected")
    return (ctypes.c_double * 4)(*vals)


def _edge_key(edges):
    """Hashable description of wall data: values, or tensor identities (a captured graph
    holds the tensor's address)."""
    if edges is None:
        return None
    key = []
    for v in edges:
        if v is None:
            key.append(None)
        elif isinstance(v, torch.Tensor):
            key.append(("t", v.data_ptr(), tuple(v.shape)))
        else:
            key.append((float(v[0]), float(v[1])))
    return tuple(key)


class StepGraph:
    """A fixed sequence of lbm_step / lbm_step2 calls recorded once as a HIP graph (the
    library's launches are captured from torch's capture stream) and replayed as one launch.

    Every argument is frozen at capture: step factors, wall data (values, or the addresses
    of field tensors, which the graph keeps alive), record buffers, and the two population
    buffers in the order they had then.  ``replay`` therefore requires the solver to hold
    the same current buffer as at capture, and afterwards sets it to the buffer the
    sequence ends in.  The fold of the displacement accumulator (every 16th level) is
    frozen with the step indices.  The library records no memset and allocates nothing,
    so its launches are capture-safe; the capture itself executes nothing."""

    def __init__(self, solver, steps):
        if solver._lent is not None:
            raise RuntimeError("StepGraph: the current level is in a lent buffer; advance once before capturing")
        self.sv = solver
        self.start_cur = solver.s.cur
        self._keep = ([st.get("edges") for st in steps] + [st.get("edges_next") for st in steps]
                      + [st.get("record") for st in steps])
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for st in steps:
                solver._run(st)
        self.end_cur = solver.s.cur
        solver.s.cur = self.start_cur
        self.nsteps = sum(st["multi"] if st.get("multi") else 2 if st.get("pair") else 1 for st in steps)

    def replay(self):
        if self.sv._lent is not None:
            raise RuntimeError("StepGraph.replay: the current level is in a lent buffer, which the graph does not read")
        if self.sv.s.cur != self.start_cur:
            raise RuntimeError("StepGraph.replay: the solver's current buffer differs from the capture's")
        self.graph.replay()
        self.sv.s.cur = self.end_cur


def _as_device(a, device):
    """A contiguous FP64 copy (or view) of a field on the device; a read-only numpy array is
    copied on the host first (torch does not wrap read-only memory)."""
    if isinstance(a, np.ndarray) and not a.flags.writeable:
        a = a.copy()
    return torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()


class Solver:
    """One grid's device state and the library calls on it (torch's current stream).

    Parameters mirror lbm_params: grid size, lattice speed c and BGK rate omega, spacing
    dx, law ("lognh", "nh", "svk", "mr", "yeoh", "gent") with optional law_k constants,
    storage ("f32", "f16", "f64"), edge kinds, uniform or per-node mu, lam and body force."""

    # Defaults of advance() and of the checkpointed rollout, from timings on one MI355X
    # (FP32, log-NH, us per level): a captured graph beats eager launches only where the
    # host launch cost dominates (256^2 periodic pairs 3.42 against 4.44, 384^2 4.37
    # against 4.52; from 512^2 up a replay adds a few microseconds per kernel node); on
    # walled grids a pair adds latency-bound launches and loses on small grids (384^2:
    # 16.2 against 15.6 single; 512^2: 20.4 against 22.9).
    GRAPH_MAX_NODES = 400 * 400
    PAIR_MIN_WALLED_NODES = 416 * 416
    # levels per lbm_step_multi call, and the grid size from which it beats pairs (bench.py
    # --levels, FP32, ms per level, four levels against pairs: 512^2 0.0125 against 0.0083,
    # 1024^2 0.0212 against 0.0228, 8192^2 0.705 against 1.301: a small grid leaves compute
    # units idle)
    MULTI_LEVELS = 4
    MULTI_MIN_NODES = 1024 * 1024
    # the same for the recorded replay and the adjoint, which pay clearly only from a larger
    # grid (four levels against pairs, replay: 1024^2 0.0262 against 0.0269, 2048^2 0.0701
    # against 0.1121; adjoint: 1024^2 0.0298 against 0.0311, 2048^2 0.0770 against 0.1193)
    BACKWARD_MULTI_MIN_NODES = 2048 * 2048
    # adjoint levels per lbm_adjoint_step_multi call (8192^2 FP32 log-NH, per-node mu lam,
    # gradients: pairs through lbm_adjoint_step2 1.77 ms per level, three levels 1.23, four
    # 1.00); three for the invariant-based laws, whose four-level kernel runs out of registers
    ADJ_MULTI_LEVELS = 4
    ADJ_MULTI_LEVELS_INVARIANT = 3
    # levels per lbm_step_multi call in the replay form (records of every level; 8192^2 FP32,
    # per-node mu lam: pairs 1.63 ms per level, three levels 1.10, four 0.90)
    REPLAY_MULTI_LEVELS = 4

    def __init__(self, nx, ny, *, c, omega, dx=1.0, material="lognh", storage="f32",
                 bc=("periodic",) * 4, mu=0.1, lam=0.2, body=None, newton_max_iter=0,
                 newton_tol=0.0, force_unstable=False, law_k=None, device="cuda"):
        self.device = torch.device(device)
        p = L.lbm_params()
        p.nx, p.ny = int(nx), int(ny)
        p.material = L.MATERIAL[material]
        p.storage = L.STORAGE[storage]
        for e in range(4):
            p.bc[e] = L.BC[bc[e]]
        p.newton_max_iter = int(newton_max_iter)
        p.force_unstable = int(bool(force_unstable))
        p.dx, p.c, p.omega, p.newton_tol = float(dx), float(c), float(omega), float(newton_tol)
        k = law_k if law_k is not None else L.LAW_K_DEFAULT.get(material, (0.0, 0.0, 0.0))
        k = tuple(float(v) for v in k) + (0.0,) * (3 - len(k))
        for i in range(3):
            p.law_k[i] = k[i]
        self.law_k = k
        self.p = p
        self.lib = L.lib()
        L.check(self.lib.lbm_check_params(ctypes.byref(p)), "lbm_check_params")
        self.nx, self.ny = int(nx), int(ny)
        self.storage, self.material = storage, material
        self.dt = float(dx) / float(c)
        pb = self.lib.lbm_pop_bytes(ctypes.byref(p))
        self.pop = [torch.empty(pb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.ustar = torch.zeros(self.lib.lbm_ustar_bytes(ctypes.byref(p)), dtype=torch.uint8, device=self.device)
        self.aux = torch.zeros(self.lib.lbm_aux_bytes(ctypes.byref(p)), dtype=torch.uint8, device=self.device)
        self.fault = torch.zeros(1, dtype=torch.int32, device=self.device)
        s = L.lbm_state()
        s.pop[0], s.pop[1] = self.pop[0].data_ptr(), self.pop[1].data_ptr()
        s.cur = 0
        s.ustar = self.ustar.data_ptr()
        s.aux = self.aux.data_ptr()
        s.fault = self.fault.data_ptr()
        self.s = s
        self._lent = None          # (slot, own buffer) while a lent buffer holds the current level
        self.set_parameters(mu, lam, body)

    # ------------------------------------------------------------ parameters
    def set_parameters(self, mu, lam, body=None):
        s = self.s
        self.mu_t = self.lam_t = self.body_t = None
        if np.isscalar(mu):
            s.mu, s.mu0, s.mu_max = None, float(mu), float(mu)
        else:
            self.mu_t = torch.as_tensor(mu, dtype=torch.float32, device=self.device).contiguous()
            s.mu, s.mu_max = self.mu_t.data_ptr(), float(self.mu_t.max())
        if np.isscalar(lam):
            s.lam, s.lam0, s.lam_max = None, float(lam), float(lam)
        else:
            self.lam_t = torch.as_tensor(lam, dtype=torch.float32, device=self.device).contiguous()
            s.lam, s.lam_max = self.lam_t.data_ptr(), float(self.lam_t.max())
        if body is None:
            s.body, s.b0[0], s.b0[1] = None, 0.0, 0.0
        elif isinstance(body, (tuple, list)):
            s.body, s.b0[0], s.b0[1] = None, float(body[0]), float(body[1])
        else:
            self.body_t = torch.as_tensor(body, dtype=torch.float32, device=self.device).contiguous()
            s.body = self.body_t.data_ptr()

    def set_body_levels(self, body_prev, body_next):
        """Per-step body force fields: body_prev for level n, body_next for level n + 1
        of the next lbm_step (float32 device tensors (2, ny, nx); use r = 1)."""
        self._body_prev = torch.as_tensor(body_prev, dtype=torch.float32, device=self.device).contiguous()
        self.body_t = torch.as_tensor(body_next, dtype=torch.float32, device=self.device).contiguous()
        self.s.body = self.body_t.data_ptr()
        self.s.body_prev = self._body_prev.data_ptr()

    # ------------------------------------------------------------ sizes
    @property
    def tiles_per_row(self):
        w = int(self.lib.lbm_tile_width())
        return (self.nx + w - 1) // w

    @property
    def record_bytes(self):
        return int(self.lib.lbm_record_bytes(ctypes.byref(self.p)))

    @property
    def real_dtype(self):
        return torch.float64 if self.storage == "f64" else torch.float32

    def new_record(self):
        """A state record (6 tiled planes of the compute type, see lbm.h)."""
        return torch.empty(self.record_bytes // self.real_dtype.itemsize, dtype=self.real_dtype, device=self.device)

    # ------------------------------------------------------------ lent buffers
    def lend(self, buf):
        """Take the current level from `buf`, a population buffer of lbm_pop_bytes() that the
        caller keeps (a snapshot), in place of copying it in: the next call that advances
        the state reads buf and writes the solver's other buffer, and the solver's own buffer
        is back in its slot after that call.  No launch writes the buffer that holds the
        current level, so buf is left as it was."""
        self._give_back()
        slot = self.s.cur
        self._lent = (slot, self.pop[slot])
        self.pop[slot] = buf
        self.s.pop[slot] = buf.data_ptr()

    def detach_current(self):
        """The buffer that holds the current level, handed over to the caller (a snapshot,
        in place of a copy): the solver's slot gets a fresh buffer, and the next call that
        advances the state still reads the level from the handed-over one (see lend)."""
        slot = self.s.cur
        if self._lent is not None:
            return self.pop[slot]          # already the caller's buffer
        cur = self.pop[slot]
        self.pop[slot] = torch.empty_like(cur)
        self.lend(cur)
        return cur

    def _give_back(self):
        if self._lent is not None:
            slot, own = self._lent
            self._lent = None
            self.pop[slot] = own
            self.s.pop[slot] = own.data_ptr()

    # ------------------------------------------------------------ entry points
    def init(self, v0, u0=None, r0=0.0, Fbar=None):
        """lbm_init; Fbar (2, 2) is an optional uniform predeformation (F = Fbar + grad u0)."""
        self._give_back()
        self._v0 = _as_device(v0, self.device)
        self._u0 = None if u0 is None else _as_device(u0, self.device)
        self.s.cur = 0
        self.fault.zero_()
        self.ustar.zero_()
        L.check(self.lib.lbm_init(ctypes.byref(self.p), ctypes.byref(self.s), _ptr(self._v0), _ptr(self._u0),
                                  host_matrix(Fbar), float(r0), _stream()), "lbm_init")

    def init_state(self, U0, dUdX, dUdY, u0=None, r0=0.0):
        """lbm_init_state: the initialisation from U0 = (v, F - I) (6, ny, nx) and its X and Y
        derivatives given by the caller."""
        def dev(a):
            return torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        self._give_back()
        self._U0, self._dUdX, self._dUdY = dev(U0), dev(dUdX), dev(dUdY)
        self._u0 = None if u0 is None else dev(u0)
        self.s.cur = 0
        self.fault.zero_()
        self.ustar.zero_()
        L.check(self.lib.lbm_init_state(ctypes.byref(self.p), ctypes.byref(self.s), _ptr(self._U0),
                                        _ptr(self._dUdX), _ptr(self._dUdY), _ptr(self._u0), float(r0),
                                        _stream()), "lbm_init_state")

    def step(self, n, r_n=1.0, r_np1=1.0, edges=None, record=None, ustar=True):
        """lbm_step; ustar=False skips the displacement quadrature (replays)."""
        ed = edges if isinstance(edges, EdgeData) else EdgeData(edges)
        keep = self.s.ustar
        if not ustar:
            self.s.ustar = None
        try:
            L.check(self.lib.lbm_step(ctypes.byref(self.p), ctypes.byref(self.s), int(n), float(r_n),
                                      float(r_np1), ctypes.byref(ed.c), _ptr(record), _stream()), "lbm_step")
            self._give_back()
        finally:
            self.s.ustar = keep

    def step2(self, n, r_np1=1.0, r_np2=1.0, record1=None, record2=None, ustar=True, r_n=1.0, edges=None,
              edges_next=None):
        """lbm_step2: levels n -> n + 2 in one pass, bit for bit the same as step(n, r_n, r_np1,
        edges) then step(n + 1, r_np1, r_np2, edges_next); record1 / record2 receive U^{n+1}
        and U^{n+2}."""
        e1 = edges if isinstance(edges, EdgeData) else EdgeData(edges)
        e2 = edges_next if isinstance(edges_next, EdgeData) else EdgeData(edges_next)
        keep = self.s.ustar
        if not ustar:
            self.s.ustar = None
        try:
            L.check(self.lib.lbm_step2(ctypes.byref(self.p), ctypes.byref(self.s), int(n), float(r_n), float(r_np1),
                                       float(r_np2), ctypes.byref(e1.c), ctypes.byref(e2.c), _ptr(record1),
                                       _ptr(record2), _stream()), "lbm_step2")
            self._give_back()
        finally:
            self.s.ustar = keep

    def step_multi(self, n, levels, r_next=None, records=None, ustar=True, record_planes=6):
        """lbm_step_multi: levels n -> n + levels in one pass on a periodic grid, bit for bit
        the same as `levels` calls of step; r_next[t] is the body factor of level n + 1 + t.
        With records (one record tensor per level) the replay form: records of every level
        and no accumulator update (then ustar must be False); record_planes = 4 writes only
        their F - I planes (what the adjoint reads)."""
        r = [1.0] * levels if r_next is None else [float(x) for x in r_next]
        if len(r) != levels:
            raise ValueError("r_next needs one factor per level")
        arr = (ctypes.c_double * levels)(*r)
        recs = None
        if records is not None:
            if len(records) != levels:
                raise ValueError("one record per level")
            recs = (ctypes.c_void_p * levels)(*[t.data_ptr() for t in records])
        keep = self.s.ustar
        if not ustar:
            self.s.ustar = None
        try:
            L.check(self.lib.lbm_step_multi(ctypes.byref(self.p), ctypes.byref(self.s), int(n), int(levels),
                                            ctypes.cast(arr, ctypes.c_void_p),
                                            ctypes.cast(recs, ctypes.c_void_p) if recs is not None else None,
                                            int(record_planes), _stream()), "lbm_step_multi")
            self._give_back()
        finally:
            self.s.ustar = keep

    @property
    def multi_levels(self):
        """Levels per lbm_step_multi call where that is the fastest way to advance: periodic
        grids of at least MULTI_MIN_NODES nodes in the shifted storages (FP32, FP16) with a
        body field shared by all levels; 0 elsewhere (walls: lbm_step2; FP64: pairs are
        faster, its multi-level kernel has too few registers for the levels it holds)."""
        ok = (self.periodic and self.pairs_ok and self.storage != "f64" and self.s.ustar
              and self.nx * self.ny >= self.MULTI_MIN_NODES)
        return self.MULTI_LEVELS if ok else 0

    @property
    def replay_multi_levels(self):
        """Levels per lbm_step_multi call in the replay form (records, no accumulator) where
        that is faster than pairs: periodic grids of at least BACKWARD_MULTI_MIN_NODES nodes
        in the shifted storages; 0 elsewhere."""
        ok = (self.periodic and self.pairs_ok and self.storage != "f64"
              and self.nx * self.ny >= self.BACKWARD_MULTI_MIN_NODES)
        return self.REPLAY_MULTI_LEVELS if ok else 0

    @property
    def adj_multi_levels(self):
        """Adjoint levels per lbm_adjoint_step_multi call where that is the fastest way:
        periodic grids of at least BACKWARD_MULTI_MIN_NODES nodes, FP32 or FP16; else 0."""
        ok = self.periodic and self.storage != "f64" and self.nx * self.ny >= self.BACKWARD_MULTI_MIN_NODES
        if not ok:
            return 0
        if self.material in ("mr", "yeoh", "gent"):
            return self.ADJ_MULTI_LEVELS_INVARIANT
        return self.ADJ_MULTI_LEVELS

    @property
    def periodic(self):
        return all(int(b) == L.BC["periodic"] for b in self.p.bc)

    @property
    def pairs_ok(self):
        """lbm_step2 equals two lbm_step calls unless per-level body fields are in use."""
        return not self.s.body_prev

    @property
    def pairs_pay(self):
        """lbm_step2 applies (pairs_ok) and is faster than two lbm_step calls: on periodic
        grids always, on walled grids from PAIR_MIN_WALLED_NODES nodes."""
        return self.pairs_ok and (self.periodic or self.nx * self.ny >= self.PAIR_MIN_WALLED_NODES)

    def _run(self, st):
        if st.get("multi"):
            self.step_multi(st["n"], st["multi"], st["r_next"])
        elif st.get("pair"):
            self.step2(st["n"], st["r_np1"], st["r_np2"], r_n=st["r_n"], edges=st.get("edges"),
                       edges_next=st.get("edges_next"))
        else:
            self.step(**st)

    def capture(self, steps):
        """Records a fixed sequence of lbm_step calls as one HIP graph (``StepGraph``).
        ``steps`` is a list of dicts with the keyword arguments of ``step``, or, with
        ``pair=True``, of ``step2`` (n, r_n, r_np1, r_np2, edges, edges_next)."""
        return StepGraph(self, steps)

    def advance(self, n0, count, ramp=None, edges=None, block=64, fused=None, graph=None):
        """Steps n0 .. n0 + count - 1 with ramp factors ``ramp(n)`` (default 1) and wall data
        ``edges(n)`` (default zero).  With ``graph`` True, whole blocks of ``block`` steps
        whose arguments equal those of the first captured block replay one captured graph
        and the rest run eagerly; this removes the per-step host cost where it dominates.
        ``graph`` None captures only grids of at most GRAPH_MAX_NODES nodes: on larger ones
        eager launches already follow each other without a gap, and a graph replay adds a
        few microseconds between its kernel nodes.  With ``fused`` True the steps go in
        groups of multi_levels through lbm_step_multi where that applies, else in pairs
        through lbm_step2 (where pairs_ok), with the same result bit for bit; None fuses
        where it is faster (pairs_pay)."""
        ramp = ramp or (lambda n: 1.0)
        edges = edges or (lambda n: None)
        fused = self.pairs_pay if fused is None else (bool(fused) and self.pairs_ok)
        if graph is None:
            graph_on = self.nx * self.ny <= self.GRAPH_MAX_NODES
        else:
            graph_on = bool(graph)

        multi = self.multi_levels if fused else 0

        def block_calls(n, m):
            # the calls for steps n .. m - 1
            calls = []
            while n < m:
                if multi and n + multi <= m:
                    calls.append(dict(multi=multi, n=n, r_next=tuple(float(ramp(n + 1 + t)) for t in range(multi))))
                    n += multi
                elif fused and n + 1 < m:
                    calls.append(dict(pair=True, n=n, r_n=float(ramp(n)), r_np1=float(ramp(n + 1)),
                                      r_np2=float(ramp(n + 2)), edges=edges(n), edges_next=edges(n + 1)))
                    n += 2
                else:
                    calls.append(dict(n=n, r_n=float(ramp(n)), r_np1=float(ramp(n + 1)), edges=edges(n)))
                    n += 1
            return calls

        graph, proto = None, None
        n, end = n0, n0 + count
        # whole multiples of 16 steps keep both the buffer parity and the phase of the
        # displacement accumulator's 16-step fold (lbm.h, lbm_state.ustar)
        block = max(16, -(-block // 16) * 16)
        while n < end:
            m = min(end, n + block)
            blk = block_calls(n, m)
            # a graph holds the solver's own buffers: a block that starts from a lent buffer
            # runs eagerly (and gives the buffer back)
            eager = self._lent is not None
            if graph_on and m - n == block and graph is None and not eager and self._graph_ok(blk):
                proto = blk
                graph = self.capture(blk)
            if (graph is not None and not eager and m - n == block and self.s.cur == graph.start_cur
                    and all(self._same(a, b) for a, b in zip(blk, proto))):
                graph.replay()
            else:
                for a in blk:
                    self._run(a)
            n = m

    @staticmethod
    def _same(a, b):
        keys = ("multi", "r_next", "pair", "r_n", "r_np1", "r_np2")
        return (all(a.get(k) == b.get(k) for k in keys)
                and _edge_key(a.get("edges")) == _edge_key(b.get("edges"))
                and _edge_key(a.get("edges_next")) == _edge_key(b.get("edges_next")))

    @classmethod
    def _graph_ok(cls, blk):
        # a block is capturable when its per-call arguments repeat exactly: the step index
        # reaches the kernels only through the accumulator's fold, whose 16-level phase a
        # block of a multiple of 16 steps keeps
        return all(cls._same(a, blk[0]) for a in blk)

    def moments(self, r_n=1.0):
        out = torch.empty((6, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.check(self.lib.lbm_moments(ctypes.byref(self.p), ctypes.byref(self.s), float(r_n), _ptr(out),
                                     _stream()), "lbm_moments")
        return out

    def displacement(self, r_n=1.0):
        out = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.check(self.lib.lbm_displacement(ctypes.byref(self.p), ctypes.byref(self.s), float(r_n), _ptr(out),
                                          _stream()), "lbm_displacement")
        return out

    def stress(self, r_n=1.0):
        """(P (2, 2, ny, nx), sigma (2, 2, ny, nx)) in FP64 at the current level."""
        P = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device=self.device)
        S = torch.empty((3, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.check(self.lib.lbm_stress(ctypes.byref(self.p), ctypes.byref(self.s), float(r_n), _ptr(P), _ptr(S),
                                    _stream()), "lbm_stress")
        sig = torch.stack([S[0], S[1], S[1], S[2]])
        return P.view(2, 2, self.ny, self.nx), sig.view(2, 2, self.ny, self.nx)

    def record_state(self, r_n, out):
        L.check(self.lib.lbm_record_state(ctypes.byref(self.p), ctypes.byref(self.s), float(r_n), _ptr(out),
                                          _stream()), "lbm_record_state")
        return out

    def diagnostics(self, r_n=1.0):
        out = torch.empty(L.LBM_DIAG_COUNT, dtype=torch.float64, device=self.device)
        scratch = torch.empty(self.lib.lbm_diag_scratch_bytes(ctypes.byref(self.p)), dtype=torch.uint8,
                              device=self.device)
        L.check(self.lib.lbm_diagnostics(ctypes.byref(self.p), ctypes.byref(self.s), float(r_n), _ptr(out),
                                         _ptr(scratch), _stream()), "lbm_diagnostics")
        return out

    def populations(self):
        """Current post-collision populations as a (4, 6, ny, nx) tensor in the storage dtype
        (shifted storages hold f* - (0, 0, 1/4, 0, 0, 1/4)), gathered from the tiled layout."""
        dt = {"f32": torch.float32, "f16": torch.float16, "f64": torch.float64}[self.storage]
        w = int(self.lib.lbm_tile_width())
        T = self.tiles_per_row
        buf = self.pop[self.s.cur].view(dt).view(self.ny, T, 24, w)
        planes = buf.permute(2, 0, 1, 3).reshape(24, self.ny, T * w)[:, :, : self.nx]
        return planes.reshape(4, 6, self.ny, self.nx)

    def faults(self):
        return int(self.fault.item())
