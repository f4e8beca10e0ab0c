"""Binomial checkpointing schedule (rollout.revolve_actions), simulated on the host.

The schedule must reverse every level exactly once, in descending order (the adjoint steps
m = end - 1 .. start); every action must start from a snapshot that is held at that moment;
no more than `slots` snapshots beyond the first may be held at once; and no leaf unit may
be re-advanced more often than the binomial bound allows: with l units and c slots, the
smallest r with C(c + r, c) >= l (Griewank's treeverse)."""
import math

import pytest

from paper_2605_26677_amd.rollout import revolve_actions


def simulate(start, end, leaf, slots):
    held = {start}
    peak = 0
    reversed_levels = []
    advanced = {}                  # leaf unit -> times it was stepped through by "take"
    steps = 0
    for act in revolve_actions(start, end, leaf, slots):
        kind = act[0]
        if kind == "take":
            a, m = act[1], act[2]
            assert a in held and a < m <= end and m not in held
            for u in range((a - start) // leaf, (m - 1 - start) // leaf + 1):
                advanced[u] = advanced.get(u, 0) + 1
            steps += m - a
            held.add(m)
            peak = max(peak, len(held) - 1)
        elif kind == "free":
            assert act[1] in held and act[1] != start
            held.remove(act[1])
        else:
            a, b = act[1], act[2]
            assert a in held and 0 < b - a <= leaf
            steps += b - a - 1              # the recorded replay of the leaf
            reversed_levels.extend(range(b - 1, a - 1, -1))
    assert held == {start}
    return reversed_levels, peak, advanced, steps


@pytest.mark.parametrize("N,leaf,slots", [(1, 5, 1), (5, 5, 0), (6, 5, 1), (37, 4, 2), (100, 10, 3), (1000, 7, 4),
                                          (20001, 65, 3), (50, 1, 5), (13, 3, 10)])
def test_schedule_reverses_every_level_once_in_order(N, leaf, slots):
    levels, peak, advanced, steps = simulate(0, N, leaf, slots)
    assert levels == list(range(N - 1, -1, -1))
    assert peak <= slots
    units = -(-N // leaf)
    if units > 1:
        r = 1
        while math.comb(slots + r, slots) < units:
            r += 1
        assert max(advanced.values()) <= r


def test_fewer_forward_steps_than_replaying_every_segment_from_the_start():
    """With 3 slots over 2000 levels in leaves of 10, the schedule advances far fewer steps
    than replaying every leaf from level 0 (the cost with no slot), and not more than
    (r + 1) times the chain."""
    N, leaf, slots = 2000, 10, 3
    _, _, advanced, steps = simulate(0, N, leaf, slots)
    quadratic = sum(range(0, N, leaf))
    assert steps < quadratic / 10
    units = N // leaf
    r = 1
    while math.comb(slots + r, slots) < units:
        r += 1
    assert steps <= (r + 1) * N


def test_needs_a_slot_beyond_one_leaf():
    with pytest.raises(ValueError):
        list(revolve_actions(0, 12, 5, 0))
