"""Binomial (revolve) checkpoint schedules for reversing a chain of steps.

Reversing l steps u_0 -> u_1 -> ... -> u_l needs the state at the start of
each step, in reverse order.  With s checkpoints (one of them holding the
initial state), the schedule that runs the fewest forward steps is the
binomial one of Griewank (1992) and Griewank & Walther (2000, "Algorithm
799: revolve"): with r the smallest integer such that beta(s, r) =
C(s + r, s) >= l, it takes r l - beta(s + 1, r - 1) forward steps in all
(the first sweep included), and no schedule with s checkpoints takes fewer.

This module only plans: it produces the sequence of actions, and the
caller (the differentiable rollout of ns.py) carries them out on the GPU.
The plan is found by a dynamic programme over the split point of each
interval (the recursion of the binomial schedule), which reaches that
count.
"""
from __future__ import annotations

from functools import lru_cache
from math import comb

ADVANCE, TAKESHOT, RESTORE, REVERSE, FREE = "advance", "takeshot", "restore", "reverse", "free"


def binomial_forward_steps(l: int, c: int) -> int:
    """Griewank's minimal number of forward steps to reverse l steps with c
    checkpoint slots beside the initial state (l >= 1, c >= 0).  With
    s = c + 1 checkpoints counting the one that holds the initial state and
    r the smallest integer with beta(s, r) = C(s + r, s) >= l, it is
    r l - beta(s + 1, r - 1) = r l - C(s + r, s + 1).  Counts every step
    advanced, the first sweep included; the reversal of each step (which
    evaluates the step once more) is not counted."""
    if l < 1:
        return 0
    s = c + 1
    r = 0
    while comb(s + r, s) < l:
        r += 1
    return r * l - comb(s + r, s + 1)


@lru_cache(maxsize=None)
def _cost(l: int, c: int) -> int:
    """Forward steps of the best schedule reversing l steps from a held
    start state with c free slots (the sweep to the end included)."""
    if l <= 1:
        return 0
    if c == 0:
        return l * (l - 1) // 2
    return min(k + _cost(l - k, c - 1) + _cost(k, c) for k in range(1, l))


@lru_cache(maxsize=None)
def _split(l: int, c: int) -> int:
    """Steps to advance before the first checkpoint of the best schedule."""
    best, arg = None, 1
    for k in range(1, l):
        v = k + _cost(l - k, c - 1) + _cost(k, c)
        if best is None or v < best:
            best, arg = v, k
    return arg


def schedule(l: int, c: int):
    """Actions that reverse steps l-1, ..., 0 of a chain whose state 0 the
    caller holds, using at most c checkpoint slots beside it.  Actions:
      (ADVANCE, i, j)   step the current state from index i to j (j > i)
      (TAKESHOT, i)     store the current state, at index i, in a slot
      (RESTORE, i)      make the stored state at index i (or state 0) current
      (REVERSE, i)      reverse step i from the current state, at index i
      (FREE, i)         release the slot of index i
    The current state is consumed by ADVANCE and REVERSE."""
    if l < 0 or c < 0:
        raise ValueError("need l >= 0 and c >= 0")
    out = []

    def rec(i: int, j: int, c: int):
        # the state at index i is current and also kept (slot or state 0)
        l = j - i
        if l == 0:
            return
        if l == 1:
            out.append((REVERSE, i))
            return
        if c == 0:
            for k in range(j - 1, i - 1, -1):
                if k > i:
                    out.append((ADVANCE, i, k))
                out.append((REVERSE, k))
                if k > i:
                    out.append((RESTORE, i))
            return
        m = i + _split(l, c)
        out.append((ADVANCE, i, m))
        out.append((TAKESHOT, m))
        rec(m, j, c - 1)
        out.append((FREE, m))
        out.append((RESTORE, i))
        rec(i, m, c)

    rec(0, l, c)
    return out


def forward_steps(actions) -> int:
    """Forward steps advanced by a schedule."""
    return sum(a[2] - a[1] for a in actions if a[0] == ADVANCE)
