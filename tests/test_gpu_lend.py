"""Snapshots without copies: Solver.detach_current hands the buffer that holds the current
level to the caller and Solver.lend gives such a buffer back as the current level, read in
place by the next launch.  Whatever advances the state afterwards (a single step, a pair,
a multi-level pass), the snapshot stays bit for bit what it was, the levels reached from
it equal those reached without it, and the solver's own buffers never alias it.
"""
import pytest
import torch

from test_gpu_step2 import _case
from gpu_cases import make_solver

pytestmark = pytest.mark.gpu


def _pop(sv):
    """The current level's populations at the grid's nodes, as bits (the padding columns of
    a tile that the last column cuts are not part of the state: not every kernel writes
    them)."""
    return sv.populations().contiguous().view(torch.int32).clone()


@pytest.mark.parametrize("advance", ["step", "pair", "multi"])
def test_lend_and_detach_keep_the_snapshot(advance):
    case = _case(200, 136, fields=True)
    sv = make_solver(case, "f32")
    sv.init(case.v0, r0=case.ramp(0))
    sv.step(0, case.ramp(0), case.ramp(1))

    def go(n):
        if advance == "step":
            sv.step(n, case.ramp(n), case.ramp(n + 1))
            return n + 1
        if advance == "pair":
            sv.step2(n, case.ramp(n + 1), case.ramp(n + 2), r_n=case.ramp(n))
            return n + 2
        sv.step_multi(n, 4, [case.ramp(n + 1 + t) for t in range(4)])
        return n + 4

    snap = sv.detach_current()
    kept = snap.clone()
    assert all(p.data_ptr() != snap.data_ptr() for i, p in enumerate(sv.pop) if i != sv.s.cur)
    n = go(1)
    after = _pop(sv)
    n = go(n)
    later = _pop(sv)
    torch.cuda.synchronize()
    assert torch.equal(snap, kept)
    assert all(p.data_ptr() != snap.data_ptr() for p in sv.pop)
    # back to level 1 from the snapshot, twice: the same levels each time
    for _ in range(2):
        sv.lend(snap)
        assert torch.equal(sv.pop[sv.s.cur], kept)
        m = go(1)
        assert torch.equal(_pop(sv), after)
        m = go(m)
        assert m == n and torch.equal(_pop(sv), later)
        assert torch.equal(snap, kept)
        assert all(p.data_ptr() != snap.data_ptr() for p in sv.pop)
    # a detach right after a lend hands back the lent buffer itself
    sv.lend(snap)
    assert sv.detach_current() is snap
    go(1)
    assert torch.equal(_pop(sv), after) and torch.equal(snap, kept)
    assert sv.faults() == 0


def test_init_after_a_lend_leaves_the_snapshot():
    case = _case(96, 80)
    sv = make_solver(case, "f32")
    sv.init(case.v0, r0=case.ramp(0))
    sv.step(0, case.ramp(0), case.ramp(1))
    snap = sv.detach_current()
    kept = snap.clone()
    sv.init(case.v0, r0=case.ramp(0))     # writes the solver's own buffers only
    torch.cuda.synchronize()
    assert torch.equal(snap, kept)
    assert all(p.data_ptr() != snap.data_ptr() for p in sv.pop)


def test_graph_advance_from_a_lent_snapshot():
    """Solver.advance with captured graphs starting from a lent snapshot: the block that
    reads the snapshot runs eagerly, the next ones replay a graph; the levels equal those of
    eager steps from a copy of the snapshot."""
    case = _case(200, 136, fields=True)
    ref = make_solver(case, "f32")
    ref.init(case.v0, r0=case.ramp(0))
    ref.step(0, case.ramp(0), case.ramp(1))
    ref.advance(1, 192, ramp=case.ramp, graph=False)
    want = _pop(ref)
    sv = make_solver(case, "f32")
    sv.init(case.v0, r0=case.ramp(0))
    sv.step(0, case.ramp(0), case.ramp(1))
    snap = sv.detach_current()
    kept = snap.clone()
    for i in range(2):
        if i:
            sv.lend(snap)
        sv.advance(1, 192, ramp=case.ramp, graph=True)
        assert torch.equal(_pop(sv), want)
        assert torch.equal(snap, kept)
    # a captured graph reads the solver's own buffers, never a lent one
    g = sv.capture([dict(n=193, r_n=case.ramp(193), r_np1=case.ramp(194))])
    sv.lend(snap)
    with pytest.raises(RuntimeError, match="lent buffer"):
        g.replay()
    assert sv.faults() == 0
