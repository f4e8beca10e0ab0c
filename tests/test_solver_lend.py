"""Host bookkeeping of lent and detached population buffers (Solver.lend,
Solver.detach_current): which buffer each slot of the C state points to before and after
the next call that advances the state.  No kernel runs: the solver's buffers live in host
memory here and the advance is stood in for by its give-back step; the GPU test
test_gpu_lend.py runs the launches themselves."""
import pytest
import torch

from paper_2605_26677_amd.solver import Solver, StepGraph


def _solver():
    return Solver(64, 48, c=2.0, omega=1.9, device="cpu")


def _slots_match(sv):
    return all(sv.s.pop[i] == sv.pop[i].data_ptr() for i in range(2))


def test_lend_points_the_current_slot_at_the_buffer_until_the_advance():
    sv = _solver()
    own = list(sv.pop)
    buf = torch.empty_like(own[0])
    cur = sv.s.cur
    sv.lend(buf)
    assert sv.pop[cur] is buf and sv.pop[1 - cur] is own[1 - cur] and _slots_match(sv)
    sv._give_back()                         # what a successful advance does after its launch
    assert sv.pop[0] is own[0] and sv.pop[1] is own[1] and _slots_match(sv)
    sv._give_back()                         # nothing lent: no change
    assert sv.pop[0] is own[0] and sv.pop[1] is own[1]


def test_a_second_lend_replaces_the_first():
    sv = _solver()
    own = list(sv.pop)
    a, b = torch.empty_like(own[0]), torch.empty_like(own[0])
    sv.lend(a)
    sv.lend(b)
    cur = sv.s.cur
    assert sv.pop[cur] is b and _slots_match(sv)
    sv._give_back()
    assert sv.pop[cur] is own[cur] and _slots_match(sv)


def test_detach_hands_over_the_current_buffer_and_takes_a_fresh_one():
    sv = _solver()
    own = list(sv.pop)
    cur = sv.s.cur
    snap = sv.detach_current()
    assert snap is own[cur]
    assert sv.pop[cur] is snap and _slots_match(sv)          # still read by the next advance
    assert sv.detach_current() is snap                         # pending: the same buffer
    sv._give_back()
    fresh = sv.pop[cur]
    assert fresh is not snap and fresh.data_ptr() != snap.data_ptr()
    assert fresh.shape == snap.shape and fresh.dtype == snap.dtype
    assert sv.pop[1 - cur] is own[1 - cur] and _slots_match(sv)


def test_graph_capture_refuses_a_pending_lend():
    sv = _solver()
    buf = torch.empty_like(sv.pop[0])
    sv.lend(buf)
    with pytest.raises(RuntimeError, match="lent buffer"):
        StepGraph(sv, [])
    sv._give_back()
    assert sv._lent is None and _slots_match(sv)
