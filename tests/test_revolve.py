"""The binomial checkpoint schedule (host logic of the differentiable
rollout) against what fixes it: Griewank's closed form for the minimal
number of forward steps, and a simulation that checks every schedule is
executable (each step reversed once, in reverse order, from the right
state, within the slot budget)."""
from math import comb

import pytest

from paper_2401_09843_amd import revolve as rv


def simulate(actions, l, c):
    """Run a schedule on a symbolic chain; returns the number of forward
    steps.  Fails on any action that the state of the chain does not allow."""
    cur = 0          # index of the current state, None once consumed
    slots = {}
    next_rev = l - 1
    steps = 0
    for a in actions:
        kind = a[0]
        if kind == rv.ADVANCE:
            i, j = a[1], a[2]
            assert cur == i and j > i
            steps += j - i
            cur = j
        elif kind == rv.TAKESHOT:
            assert cur == a[1] and a[1] not in slots
            slots[a[1]] = True
            assert len(slots) <= c
        elif kind == rv.RESTORE:
            assert a[1] == 0 or a[1] in slots
            cur = a[1]
        elif kind == rv.FREE:
            del slots[a[1]]
        elif kind == rv.REVERSE:
            assert cur == a[1] == next_rev
            next_rev -= 1
            cur = None
        else:
            raise AssertionError(kind)
    assert next_rev == -1
    return steps


def test_closed_form_small_cases():
    # values that follow from the definition by hand: no slot means every
    # step is reached again from the start; one step needs no forward step;
    # with a slot for every intermediate state one sweep suffices
    assert rv.binomial_forward_steps(1, 0) == 0
    assert rv.binomial_forward_steps(5, 0) == 10
    assert rv.binomial_forward_steps(2, 1) == 1
    assert rv.binomial_forward_steps(3, 1) == 2
    for l in range(1, 30):
        assert rv.binomial_forward_steps(l, l - 1) == l - 1
        assert rv.binomial_forward_steps(l, l + 5) == l - 1


@pytest.mark.parametrize("l", list(range(1, 41)) + [100, 200])
@pytest.mark.parametrize("c", [0, 1, 2, 3, 5, 9])
def test_schedule_is_executable_and_optimal(l, c):
    acts = rv.schedule(l, c)
    steps = simulate(acts, l, c)
    assert steps == rv.forward_steps(acts)
    assert steps == rv.binomial_forward_steps(l, c)


def test_binomial_count_against_beta():
    # r l - C(s + r, s + 1) at the points where beta(s, r) = l exactly:
    # l = C(s + r, s) steps with s checkpoints take r l - C(s + r, s + 1)
    for s in range(1, 6):
        for r in range(1, 6):
            l = comb(s + r, s)
            assert rv.binomial_forward_steps(l, s - 1) == r * l - comb(s + r, s + 1)
