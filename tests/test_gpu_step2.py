"""Two fused steps (lbm_step2, temporal blocking of the step of Sec. 3.7) against two single
steps (lbm_step) and against the FP64 oracle.

lbm_step2 promises the result of lbm_step(n) followed by lbm_step(n + 1), bit for bit: the
populations, both words of the displacement accumulator across its 16-level folds (or the
FP64 planes), the records and the fault word, on periodic grids and on grids with
velocity and traction walls (corners, walls along one axis only, wall data that change
every half step, per-node wall data).  The cases cover every storage and law; uniform and
per-node mu, lam and body force, with different ramp factors at the two levels; grids that
are multiples of neither the 64-node strip nor the block of rows of the kernel, grids
narrower than one strip (the lanes then wrap the periodic axis several times) down to the
3 x 3 minimum; start levels of both parities, so that the fold falls on the first and on
the second level of a pair; and the 8192 x 8192 benchmark grid in the launch
configuration that bench.py times.
"""
import numpy as np
import pytest
import torch

import lbm_inputs as li
from gpu_cases import ALL_LAWS, Case, make_solver, oracle_law, rel_l2, shifted_state

pytestmark = pytest.mark.gpu


def _case(nx, ny, law="lognh", fields=False, rms=5e-3):
    if min(nx, ny) >= 4:
        v0 = np.stack([li.gaussian_random_field(nx, ny, 501, rms), li.gaussian_random_field(nx, ny, 502, rms)])
    else:                                     # too small for a smooth field: white noise
        v0 = rms * np.random.default_rng(501).standard_normal((2, ny, nx))
    mu = li.lognormal_field(nx, ny, 503, 0.1, 0.3, 4.0) if fields else 0.1
    lam = li.lognormal_field(nx, ny, 504, 0.2, 0.3, 4.0) if fields else 0.2
    body = li.uniform_body(nx, ny, (2e-4, -3e-4)) if fields else (1e-4, -2e-4)
    return Case(f"pair_{law}_{nx}x{ny}_{'fields' if fields else 'uniform'}", nx, ny, 2.5, 1.9, 0, law=law,
                mu=mu, lam=lam, body=body, ramp_steps=7, v0=v0)


def _ustar_words(sv):
    """Valid nodes of the displacement accumulator: (S, U) for the shifted storages (float32
    and float64 planes, lbm.h), (u*, None) for FP64."""
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


def _pair_vs_single(case, storage, start, pairs):
    single = make_solver(case, storage)
    pair = make_solver(case, storage)
    for sv in (single, pair):
        sv.init(case.v0, r0=case.ramp(0))
        for m in range(start):
            sv.step(m, case.ramp(m), case.ramp(m + 1))
    n = start
    for _ in range(pairs):
        single.step(n, case.ramp(n), case.ramp(n + 1))
        single.step(n + 1, case.ramp(n + 1), case.ramp(n + 2))
        pair.step2(n, case.ramp(n + 1), case.ramp(n + 2))
        n += 2
    torch.cuda.synchronize()
    assert torch.equal(single.populations(), pair.populations())
    for a, b in zip(_ustar_words(single), _ustar_words(pair)):
        if a is not None:
            assert torch.equal(a, b)
    assert torch.equal(single.displacement(case.ramp(n)), pair.displacement(case.ramp(n)))
    assert single.faults() == pair.faults() == 0
    return single, pair


@pytest.mark.parametrize("fields", [False, True])
@pytest.mark.parametrize("nx,ny", [(64, 64), (130, 13), (200, 7), (5, 3), (3, 3)])
@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_step2_bitwise_equals_two_steps(storage, nx, ny, fields):
    case = _case(nx, ny, fields=fields)
    for start in (0, 1):                      # the fold on the second, then the first level of a pair
        _pair_vs_single(case, storage, start, pairs=20)


@pytest.mark.parametrize("nx,ny", [(2500, 23), (4160, 11)])
def test_step2_bitwise_wide_grids(nx, ny):
    """More strips than one chunk of the workgroup order (32), with a narrower last chunk
    (40 strips: 32 + 8; 65 strips: 2 x 32 + 1), so the block map divides by both widths."""
    _pair_vs_single(_case(nx, ny, fields=True), "f32", 1, pairs=4)


@pytest.mark.parametrize("law", [l for l in ALL_LAWS if l != "lognh"])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_step2_bitwise_every_law(storage, law):
    _pair_vs_single(_case(97, 20, law=law, fields=True), storage, 1, pairs=10)


@pytest.mark.parametrize("storage,bar", [("f64", 1e-10), ("f32", 1e-5)])
def test_step2_matches_oracle(storage, bar):
    """40 levels in pairs on a 96 x 70 random field against the FP64 oracle."""
    from oracle import lbm
    case = _case(96, 70, fields=True)
    sv = make_solver(case, storage)
    sv.init(case.v0, r0=case.ramp(0))
    N = 40
    for n in range(0, N, 2):
        sv.step2(n, case.ramp(n + 1), case.ramp(n + 2))
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
    print(f"\n[step2 {storage}] v={ev:.2e} F-I={eF:.2e} u={eu:.2e}")
    assert ev <= bar and eF <= bar and eu <= bar


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_step2_records_equal_single_step_records(storage):
    """The records of both levels (the checkpointed adjoint replays through them) are bit
    for bit those of two lbm_step calls; also with the displacement quadrature skipped."""
    case = _case(150, 37, fields=True)
    single = make_solver(case, storage)
    pair = make_solver(case, storage)
    for sv in (single, pair):
        sv.init(case.v0, r0=case.ramp(0))
    for n in range(0, 12, 2):
        ra, rb = single.new_record(), single.new_record()
        pa, pb = pair.new_record(), pair.new_record()
        ustar = n % 4 == 0
        single.step(n, case.ramp(n), case.ramp(n + 1), record=ra, ustar=ustar)
        single.step(n + 1, case.ramp(n + 1), case.ramp(n + 2), record=rb, ustar=ustar)
        pair.step2(n, case.ramp(n + 1), case.ramp(n + 2), record1=pa, record2=pb, ustar=ustar)
        torch.cuda.synchronize()
        w = int(single.lib.lbm_tile_width())
        T = single.tiles_per_row

        def valid(r):
            return r.view(case.ny, T, 6, w).permute(2, 0, 1, 3).reshape(6, case.ny, T * w)[:, :, :case.nx]
        assert torch.equal(valid(ra), valid(pa)), n
        assert torch.equal(valid(rb), valid(pb)), n
    assert torch.equal(single.populations(), pair.populations())
    assert single.faults() == pair.faults() == 0


WALL_KINDS = {
    "block": ("velocity", "traction", "traction", "traction"),
    "mixed": ("velocity", "traction", "traction", "velocity"),
    "traction4": ("traction",) * 4,
    "y_walls": ("periodic", "periodic", "traction", "velocity"),
    "x_walls": ("velocity", "traction", "periodic", "periodic"),
}


def _wall_data(kinds, n, nx, ny, field_edge=None):
    """Wall data of half step n: uniform values that change every half step, and on one
    edge optionally a per-node field."""
    base = {"velocity": (1e-4, -2e-4), "traction": (3e-4, -1e-4), "periodic": None}
    out = []
    for e, k in enumerate(kinds):
        if base[k] is None:
            out.append(None)
            continue
        f = 1.0 + 0.05 * n
        if e == field_edge:
            L = ny if e < 2 else nx
            s = np.linspace(0.5, 1.5, L)
            out.append(torch.tensor(np.stack([base[k][0] * f * s, base[k][1] * f * s[::-1]]), device="cuda"))
        else:
            out.append((base[k][0] * f, base[k][1] * f))
    return out


def _walls_pair_vs_single(kinds, nx, ny, storage, fields, start, pairs, law="lognh", field_edge=None, records=False):
    case = _case(nx, ny, law=law, fields=fields, rms=1e-3)
    case.kinds = kinds
    single = make_solver(case, storage)
    pair = make_solver(case, storage)
    data = lambda n: _wall_data(kinds, n, nx, ny, field_edge)
    for sv in (single, pair):
        sv.init(case.v0, r0=case.ramp(0))
        for m in range(start):
            sv.step(m, case.ramp(m), case.ramp(m + 1), edges=data(m))
    n = start
    for _ in range(pairs):
        ra = rb = pa = pb = None
        if records:
            ra, rb, pa, pb = (single.new_record() for _ in range(4))
        single.step(n, case.ramp(n), case.ramp(n + 1), edges=data(n), record=ra)
        single.step(n + 1, case.ramp(n + 1), case.ramp(n + 2), edges=data(n + 1), record=rb)
        pair.step2(n, case.ramp(n + 1), case.ramp(n + 2), record1=pa, record2=pb, r_n=case.ramp(n),
                   edges=data(n), edges_next=data(n + 1))
        if records:
            w = int(single.lib.lbm_tile_width())
            T = single.tiles_per_row

            def valid(r):
                return r.view(ny, T, 6, w).permute(2, 0, 1, 3).reshape(6, ny, T * w)[:, :, :nx]
            assert torch.equal(valid(ra), valid(pa)) and torch.equal(valid(rb), valid(pb)), n
        n += 2
    torch.cuda.synchronize()
    diff = (single.populations().double() - pair.populations().double()).abs()
    assert torch.equal(single.populations(), pair.populations()), (
        f"{int((diff > 0).sum())} differences, first at {(diff > 0).nonzero()[:4].tolist()}")
    for a, b in zip(_ustar_words(single), _ustar_words(pair)):
        if a is not None:
            assert torch.equal(a, b)
    assert torch.equal(single.displacement(case.ramp(n)), pair.displacement(case.ramp(n)))
    assert single.faults() == pair.faults() == 0


@pytest.mark.parametrize("kind", list(WALL_KINDS))
@pytest.mark.parametrize("nx,ny", [(64, 40), (130, 13), (5, 6)])
@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_step2_walls_bitwise_equals_two_steps(kind, nx, ny, storage):
    for start, fields in ((0, False), (1, True)):
        _walls_pair_vs_single(WALL_KINDS[kind], nx, ny, storage, fields, start, pairs=10)


@pytest.mark.parametrize("storage,records", [("f32", False), ("f32", True), ("f16", True)])
def test_step2_walls_bitwise_wide_grid(storage, records):
    """A walled grid whose interior spans more than one chunk of strips (41 strips, 39 of
    them interior: 32 + 7): interior and rim blocks in one launch, with per-node fields,
    and with the records of both levels (as the checkpointed replays write them)."""
    _walls_pair_vs_single(WALL_KINDS["block"], 2600, 40, storage, True, 1, pairs=3, records=records)


@pytest.mark.parametrize("law", ["svk", "gent", "nh"])
def test_step2_walls_every_law_field_edge_records(law):
    """Other laws, per-node wall data on one edge, and the records of both levels."""
    _walls_pair_vs_single(WALL_KINDS["mixed"], 97, 20, "f32", True, 1, pairs=8, law=law, field_edge=1,
                          records=True)


def test_advance_in_pairs_with_walls_equals_single_steps():
    """Solver.advance on a grid with walls (captured pairs and an eager tail)."""
    case = _case(100, 70, fields=True, rms=1e-3)
    case.kinds = WALL_KINDS["block"]
    data = lambda n: _wall_data(case.kinds, 0, case.nx, case.ny)
    eager = make_solver(case, "f32")
    adv = make_solver(case, "f32")
    for sv in (eager, adv):
        sv.init(case.v0, r0=case.ramp(0))
    N = 83
    for m in range(N):
        eager.step(m, case.ramp(m), case.ramp(m + 1), edges=data(m))
    adv.advance(0, N, ramp=case.ramp, edges=data, block=32, fused=True, graph=True)
    assert torch.equal(eager.populations(), adv.populations())
    assert torch.equal(eager.displacement(case.ramp(N)), adv.displacement(case.ramp(N)))
    assert eager.faults() == adv.faults() == 0


def test_advance_in_pairs_equals_single_steps():
    """Solver.advance on a periodic grid goes through lbm_step2 (captured blocks and an eager
    tail with one single step at the end); bitwise equal to single steps."""
    case = _case(256, 200, fields=True)
    eager = make_solver(case, "f32")
    adv = make_solver(case, "f32")
    for sv in (eager, adv):
        sv.init(case.v0, r0=case.ramp(0))
    N = 151
    for m in range(N):
        eager.step(m, case.ramp(m), case.ramp(m + 1))
    adv.advance(0, N, ramp=case.ramp, block=32, fused=True, graph=True)   # a pair flips the buffers once per two levels
    assert torch.equal(eager.populations(), adv.populations())
    assert torch.equal(eager.displacement(case.ramp(N)), adv.displacement(case.ramp(N)))


def test_step2_full_size_bitwise():
    """The 8192 x 8192 benchmark workload (FP32, log-NH, uniform parameters, no body force):
    four levels in pairs against four single steps, every node."""
    n = 8192
    v0 = np.stack([li.gaussian_random_field(n, n, 301, 5e-3), li.gaussian_random_field(n, n, 302, 5e-3)])
    case = Case("pair_8192", n, n, 2.0, 2.0, 0, v0=v0)
    case.body = None
    single, pair = _pair_vs_single(case, "f32", 14, pairs=2)      # folds at level 16
    del single, pair
    torch.cuda.empty_cache()
