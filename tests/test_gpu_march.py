"""Several fused steps per pass (lbm_step_multi, temporal blocking of the step of Sec. 3.7 on
periodic grids) against single steps (lbm_step) and against the FP64 oracle.

lbm_step_multi promises the result of `levels` calls of lbm_step, bit for bit: the
populations, both words of the displacement accumulator across its 16-level folds (or the
FP64 planes) and the fault word.  The cases cover 2, 3 and 4 levels per pass; every storage
and law; uniform and per-node mu, lam and body force with a body ramp that differs at every
level; grids that are multiples neither of the kernel's window of output columns (64 minus
2 per extra level) nor of its segment of rows, grids narrower than one window (the lanes
then wrap the periodic axis several times) down to 3 x 3; start levels that put the fold on
each level of a pass; a run that blows up (the fault words must agree); and the 8192 x 8192
benchmark grid in the launch configuration that bench.py times.
"""
import ctypes

import numpy as np
import pytest
import torch

import lbm_inputs as li
from gpu_cases import ALL_LAWS, Case, make_solver, oracle_law, rel_l2, shifted_state

pytestmark = pytest.mark.gpu


def _case(nx, ny, law="lognh", fields=False, rms=5e-3, c=2.5, omega=1.9):
    if min(nx, ny) >= 4:
        v0 = np.stack([li.gaussian_random_field(nx, ny, 601, rms), li.gaussian_random_field(nx, ny, 602, rms)])
    else:                                     # too small for a smooth field: white noise
        v0 = rms * np.random.default_rng(601).standard_normal((2, ny, nx))
    mu = li.lognormal_field(nx, ny, 603, 0.1, 0.3, 4.0) if fields else 0.1
    lam = li.lognormal_field(nx, ny, 604, 0.2, 0.3, 4.0) if fields else 0.2
    body = li.uniform_body(nx, ny, (2e-4, -3e-4)) if fields else (1e-4, -2e-4)
    return Case(f"multi_{law}_{nx}x{ny}_{'fields' if fields else 'uniform'}", nx, ny, c, omega, 0, law=law,
                mu=mu, lam=lam, body=body, ramp_steps=7, v0=v0)


def _ustar_words(sv):
    w = int(sv.lib.lbm_tile_width())
    T, ny, nx = sv.tiles_per_row, sv.ny, sv.nx
    padded = T * w * ny

    def planes(flat):
        return flat.view(ny, T, 2, w).permute(2, 0, 1, 3).reshape(2, ny, T * w)[:, :, :nx]
    if sv.storage == "f64":
        return planes(sv.ustar.view(torch.float64)[: 2 * padded]), None
    S = planes(sv.ustar[: 8 * padded].view(torch.float32))
    U = planes(sv.ustar[8 * padded: 24 * padded].view(torch.float64))
    return S, U


def _multi_vs_single(case, storage, levels, start, passes, check_faults_only=False):
    single = make_solver(case, storage)
    multi = make_solver(case, storage)
    for sv in (single, multi):
        sv.init(case.v0, r0=case.ramp(0))
        for m in range(start):
            sv.step(m, case.ramp(m), case.ramp(m + 1))
    n = start
    for _ in range(passes):
        for t in range(levels):
            single.step(n + t, case.ramp(n + t), case.ramp(n + t + 1))
        multi.step_multi(n, levels, [case.ramp(n + 1 + t) for t in range(levels)])
        n += levels
    torch.cuda.synchronize()
    if check_faults_only:
        return single.faults(), multi.faults()
    assert torch.equal(single.populations(), multi.populations())
    for a, b in zip(_ustar_words(single), _ustar_words(multi)):
        if a is not None:
            assert torch.equal(a, b)
    assert torch.equal(single.displacement(case.ramp(n)), multi.displacement(case.ramp(n)))
    assert single.faults() == multi.faults() == 0
    return single, multi


@pytest.mark.parametrize("fields", [False, True])
@pytest.mark.parametrize("nx,ny", [(64, 64), (121, 13), (200, 9), (5, 3), (3, 3)])
@pytest.mark.parametrize("levels", [2, 3, 4])
@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_multi_bitwise_equals_single_steps(storage, levels, nx, ny, fields):
    case = _case(nx, ny, fields=fields)
    # 12 levels per run; the start puts the fold at level 16 on each level of a pass
    for start in range(16 - levels, 16):
        _multi_vs_single(case, storage, levels, start, passes=12 // levels)


def _replay_vs_single(case, storage, levels, start, passes, planes=6):
    """The replay form: single steps with a record each and no accumulator against
    lbm_step_multi with the records of every level; with planes = 4 only the F - I planes
    of the records are written, and the velocity planes keep what they held."""
    single = make_solver(case, storage)
    multi = make_solver(case, storage)
    for sv in (single, multi):
        sv.init(case.v0, r0=case.ramp(0))
        for m in range(start):
            sv.step(m, case.ramp(m), case.ramp(m + 1))
    n = start
    for _ in range(passes):
        ra = [single.new_record() for _ in range(levels)]
        rb = [multi.new_record().fill_(1234.5) for _ in range(levels)]
        for t in range(levels):
            single.step(n + t, case.ramp(n + t), case.ramp(n + t + 1), record=ra[t], ustar=False)
        multi.step_multi(n, levels, [case.ramp(n + 1 + t) for t in range(levels)], records=rb, ustar=False,
                         record_planes=planes)
        n += levels
        torch.cuda.synchronize()
        for a, b in zip(ra, rb):
            ua, ub = _record_nodes(single, a), _record_nodes(multi, b)
            if planes == 6:
                assert torch.equal(ua, ub)
            else:
                assert torch.equal(ua[2:], ub[2:])
                assert bool((ub[:2] == 1234.5).all())
    assert torch.equal(single.populations(), multi.populations())
    assert single.faults() == multi.faults() == 0


def _record_nodes(sv, rec):
    """The 6 planes of a record at the grid's nodes (its tiled layout without padding)."""
    w = int(sv.lib.lbm_tile_width())
    T = sv.tiles_per_row
    r = rec.view(torch.float32).view(sv.ny, T, 6, w)
    return r.permute(2, 0, 1, 3).reshape(6, sv.ny, T * w)[:, :, : sv.nx]


@pytest.mark.parametrize("fields", [False, True])
@pytest.mark.parametrize("nx,ny", [(64, 64), (121, 13), (500, 9), (5, 3), (3, 3)])
@pytest.mark.parametrize("levels", [2, 3, 4])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_multi_replay_bitwise_equals_single_steps(storage, levels, nx, ny, fields):
    _replay_vs_single(_case(nx, ny, fields=fields), storage, levels, 1, passes=12 // levels)


@pytest.mark.parametrize("nx,ny", [(2500, 23), (4160, 70)])
@pytest.mark.parametrize("levels", [2, 3, 4])
def test_multi_bitwise_wide_grids(nx, ny, levels):
    """Many windows per row, and with 70 rows more than one segment of rows."""
    _multi_vs_single(_case(nx, ny, fields=True), "f32", levels, 1, passes=3)


@pytest.mark.parametrize("nx,ny", [(64, 64), (121, 13), (3, 3)])
@pytest.mark.parametrize("levels", [2, 3, 4])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_multi_replay_strain_planes(storage, levels, nx, ny):
    """record_planes = 4: the F - I planes bit for bit those of single steps, the velocity
    planes untouched."""
    _replay_vs_single(_case(nx, ny, fields=True), storage, levels, 1, passes=12 // levels, planes=4)


@pytest.mark.parametrize("nx,ny", [(2500, 23), (4160, 70)])
def test_multi_replay_bitwise_wide_grids(nx, ny):
    """The replay form at four levels (one LDS buffer of records) on many windows per row and
    more than one segment of rows."""
    _replay_vs_single(_case(nx, ny, fields=True), "f32", 4, 1, passes=3)


@pytest.mark.parametrize("law", [l for l in ALL_LAWS if l != "lognh"])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_multi_bitwise_every_law(storage, law):
    _multi_vs_single(_case(97, 20, law=law, fields=True), storage, 3, 1, passes=4)


@pytest.mark.parametrize("law", [l for l in ALL_LAWS if l != "lognh"])
def test_multi_replay_bitwise_every_law(law):
    _replay_vs_single(_case(97, 20, law=law, fields=True), "f32", 4, 1, passes=3)


def test_multi_fault_words_agree():
    """A run that leaves the stable range (c below the P-wave speed bound, large velocities):
    the fault words of single steps and of passes of three levels are equal and non-zero."""
    case = _case(40, 24, rms=0.4, c=1.0, omega=2.0)
    case.force_unstable = True
    single, multi = _multi_vs_single(case, "f32", 3, 0, passes=20, check_faults_only=True)
    print(f"\n[multi faults] single {single:#x} multi {multi:#x}")
    assert single != 0 and single == multi


@pytest.mark.parametrize("storage,bar", [("f64", 1e-10), ("f32", 1e-5)])
def test_multi_matches_oracle(storage, bar):
    """36 levels in passes of three on a 96 x 70 random field against the FP64 oracle."""
    from oracle import lbm
    case = _case(96, 70, fields=True)
    sv = make_solver(case, storage)
    sv.init(case.v0, r0=case.ramp(0))
    N = 36
    for n in range(0, N, 3):
        sv.step_multi(n, 3, [case.ramp(n + 1 + t) for t in range(3)])
    U = sv.moments(case.ramp(N)).cpu().numpy()
    u = sv.displacement(case.ramp(N)).cpu().numpy()
    assert sv.faults() == 0
    body = np.broadcast_to(np.asarray(case.body, dtype=np.float64), (2, case.ny, case.nx))
    pb = lbm.Problem(nx=case.nx, ny=case.ny, c=case.c, omega=case.omega, law=oracle_law(case.law), mu=case.mu,
                     lam=case.lam, body=body, ramp=case.ramp)
    st = lbm.initial_state(pb, case.v0)
    Uo, uo = lbm.run(pb, st, N)
    Uo = shifted_state(Uo)
    ev, eF, eu = rel_l2(U[0:2], Uo[0:2]), rel_l2(U[2:6], Uo[2:6]), rel_l2(u, uo)
    print(f"\n[multi {storage}] v={ev:.2e} F-I={eF:.2e} u={eu:.2e}")
    assert ev <= bar and eF <= bar and eu <= bar


def test_multi_refuses_bad_arguments():
    from paper_2605_26677_amd import _lib as L
    case = _case(32, 16)
    sv = make_solver(case, "f32")
    sv.init(case.v0)
    r = (ctypes.c_double * 5)(1, 1, 1, 1, 1)
    for levels in (0, 1, 5):
        st = sv.lib.lbm_step_multi(ctypes.byref(sv.p), ctypes.byref(sv.s), 0, levels,
                                   ctypes.cast(r, ctypes.c_void_p), None, 6, None)
        assert st == L.LBM_ERR_ARG
    st = sv.lib.lbm_step_multi(ctypes.byref(sv.p), ctypes.byref(sv.s), 0, 3, None, None, 6, None)
    assert st == L.LBM_ERR_ARG
    # the replay form: records need no accumulator, no FP64
    recs = [sv.new_record() for _ in range(4)]
    rp = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in recs])
    st = sv.lib.lbm_step_multi(ctypes.byref(sv.p), ctypes.byref(sv.s), 0, 3, ctypes.cast(r, ctypes.c_void_p),
                               ctypes.cast(rp, ctypes.c_void_p), 6, None)
    assert st == L.LBM_ERR_UNSUPPORTED                  # s->ustar is set
    for planes in (0, 5, 7):
        st = sv.lib.lbm_step_multi(ctypes.byref(sv.p), ctypes.byref(sv.s), 0, 3, ctypes.cast(r, ctypes.c_void_p),
                                   ctypes.cast(rp, ctypes.c_void_p), planes, None)
        assert st == L.LBM_ERR_ARG                      # records of 6 or 4 planes only
    s64 = make_solver(case, "f64")
    s64.init(case.v0)
    keep = s64.s.ustar
    s64.s.ustar = None
    st = s64.lib.lbm_step_multi(ctypes.byref(s64.p), ctypes.byref(s64.s), 0, 3, ctypes.cast(r, ctypes.c_void_p),
                                ctypes.cast(rp, ctypes.c_void_p), 6, None)
    assert st == L.LBM_ERR_UNSUPPORTED                  # records of FP64 states
    s64.s.ustar = keep
    walled = Case("multi_walled", 32, 16, 10.0, 1.95, 0, kinds=("velocity", "traction", "periodic", "periodic"),
                  mu=0.1, lam=0.2, v0=np.zeros((2, 16, 32)))
    sw = make_solver(walled, "f32")
    sw.init(walled.v0)
    st = sw.lib.lbm_step_multi(ctypes.byref(sw.p), ctypes.byref(sw.s), 0, 3, ctypes.cast(r, ctypes.c_void_p), None,
                               6, None)
    assert st == L.LBM_ERR_UNSUPPORTED


def test_multi_full_size_bitwise():
    """The 8192 x 8192 benchmark workload (FP32, log-NH, uniform parameters, no body force):
    twelve levels in passes of three against twelve single steps, every node, across the
    fold at level 16."""
    n = 8192
    v0 = np.stack([li.gaussian_random_field(n, n, 301, 5e-3), li.gaussian_random_field(n, n, 302, 5e-3)])
    case = Case("multi_8192", n, n, 2.0, 2.0, 0, v0=v0)
    case.body = None
    single, multi = _multi_vs_single(case, "f32", 3, 14, passes=4)
    del single, multi
    torch.cuda.empty_cache()


def test_multi_replay_full_size_four_planes():
    """The replay of the 8192^2 forward + adjoint benchmark (per-node mu, lam log-normal with
    correlation length 32, a uniform body force under a ramp): four-level passes writing
    the F - I planes of every record against single steps with records, bit for bit."""
    n = 8192
    mu = li.lognormal_field(n, n, 401, 0.1, 0.3, 32.0)
    lam = li.lognormal_field(n, n, 402, 0.2, 0.3, 32.0)
    c = float(np.ceil(2.0 * np.sqrt(float(lam.max()) + 2 * float(mu.max())) * 1.1 * 4) / 4)
    v0 = np.stack([li.gaussian_random_field(n, n, 301, 5e-3), li.gaussian_random_field(n, n, 302, 5e-3)])
    case = Case("replay_8192", n, n, c, 2.0, 0, mu=mu, lam=lam, body=li.uniform_body(n, n, (1e-5, -2e-5)),
                ramp_steps=7, v0=v0)
    _replay_vs_single(case, "f32", 4, 1, passes=2, planes=4)
    torch.cuda.empty_cache()


def test_multi_in_captured_graphs():
    """Solver.advance on a 1024^2 grid takes four-level launches (multi_levels) and, with
    graph=True, replays captured blocks of them: bitwise equal to eager single steps after
    every replay, with eager work and host synchronisation between the replays."""
    n = 1024
    case = _case(n, n)                               # uniform mu, lam: per-node fields this large
    eager = make_solver(case, "f32")                 # reach the lattice-speed bound at c = 2.5
    graph = make_solver(case, "f32")
    assert graph.multi_levels == 4
    for sv in (eager, graph):
        sv.init(case.v0, r0=case.ramp(0))
        for m in range(16):                          # past the ramp, also loads the kernels
            sv.step(m, case.ramp(m), case.ramp(m + 1))
    blk = 32
    n0 = 16
    for rep in range(3):
        for m in range(n0, n0 + blk):
            eager.step(m, case.ramp(m), case.ramp(m + 1))
        graph.advance(n0, blk, ramp=case.ramp, block=blk, fused=True, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(eager.populations(), graph.populations()), rep
        assert torch.equal(eager.displacement(case.ramp(n0 + blk)), graph.displacement(case.ramp(n0 + blk))), rep
        n0 += blk
    assert eager.faults() == graph.faults() == 0
