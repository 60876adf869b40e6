"""The bulge chasing's inter-sweep waits, checked on the CPU by brute force.

A model of the stage-2 kernel's schedule: sweep s (s = 0 .. n-3) makes column
s tridiagonal in steps k = 0 .. K_s - 1; step k touches the band store in two
parts, its rows rx .. rx+L-1 (part A: the reflector's column, the bulge
block, the diagonal block) and its block below (part B), with rx, L and the
block shapes as the kernel forms them.  One workgroup runs a sweep's parts in
order and publishes step k (progress k+1) once its part A is done; part A of
step k of sweep s starts once sweep s-1 has published min(k+2, K_{s-1}) steps,
part B (when the step has a block below) once it has published
min(k+3, K_{s-1}).  These waits, with program order, define a partial order
on all parts.  The sequential algorithm runs sweep after sweep,
so every element two sweeps touch must be touched by the earlier sweep's part
first: the test checks that for every such pair the earlier part precedes the
later one in the partial order (which also keeps valid the block a sweep
holds in LDS from one step's part B to the next step's part A, since that
part B touches the same elements).  A schedule one step tighter is shown to
fail the same check."""
import itertools

import pytest


def sweep_steps(n, w, s):
    rem = n - 1 - s
    return 1 + ((rem - 1) // w if rem > w else 0)


def step_parts(n, w, s, k):
    """(elements of part A, elements of part B) of step k of sweep s, as
    sets of (row, column) with row >= column (the stored triangle)."""
    if k == 0:
        cx, rx, L = s, s + 1, min(w, n - 1 - s)
    else:
        cx, rx = s + 1 + (k - 1) * w, s + 1 + k * w
        L = min(w, n - rx)
    if L < 2:
        return set(), set()
    A = {(rx + t, cx) for t in range(L)}
    if k >= 1:
        A |= {(rx + t, cx + 1 + j) for t in range(L) for j in range(w - 1)}
    A |= {(rx + t, rx + u) for t in range(L) for u in range(t + 1)}
    r2 = rx + w
    m2 = min(rx + 2 * w, n) - r2
    B = {(r2 + i, rx + u) for i in range(max(m2, 0)) for u in range(L)}
    return A, B


def check_schedule(n, w, lag_a=2, lag_b=3, publish_after_a=True):
    """Returns the list of element conflicts the waits fail to order
    (publish_after_a=False: a step published only once both parts are done)."""
    S = max(0, n - 2)
    K = [sweep_steps(n, w, s) for s in range(S)]
    parts = {}
    for s in range(S):
        for k in range(K[s]):
            parts[(s, k)] = step_parts(n, w, s, k)

    # event index within a sweep: part A of step k is 2k, part B 2k+1.
    # before[s][e] = for each earlier sweep q, the largest event index of q
    # that precedes event e of sweep s (-1: none).
    before = []
    for s in range(S):
        rows = []
        cur = [-1] * S
        for k in range(K[s]):
            for part in (0, 1):
                e = 2 * k + part
                if s > 0:
                    lag = lag_a if part == 0 else lag_b
                    has_wait = part == 0 or len(parts[(s, k)][1]) > 0
                    if has_wait:
                        need = min(k + lag, K[s - 1])
                        if need >= 1:
                            # the event after which step need-1 is published
                            src = 2 * (need - 1) + (0 if publish_after_a else 1)
                            cur[s - 1] = max(cur[s - 1], src)
                            # and everything that precedes that event
                            for q, idx in enumerate(before[s - 1][src]):
                                cur[q] = max(cur[q], idx)
                rows.append(list(cur))
        before.append(rows)

    touch = {}
    for (s, k), (A, B) in parts.items():
        for part, elems in ((0, A), (1, B)):
            for el in elems:
                touch.setdefault(el, []).append((s, 2 * k + part))
    bad = []
    for el, evs in touch.items():
        for (s1, e1), (s2, e2) in itertools.combinations(sorted(evs), 2):
            if s1 < s2 and before[s2][e2][s1] < e1:
                bad.append((el, (s1, e1), (s2, e2)))
    return bad


@pytest.mark.parametrize("n,w", [(6, 2), (12, 2), (17, 3), (25, 3), (33, 4), (40, 5), (47, 6),
                                 (64, 8), (70, 16)])
def test_stage2_waits_order_every_shared_element(n, w):
    bad = check_schedule(n, w)
    assert not bad, bad[:5]


@pytest.mark.parametrize("n,w", [(33, 4), (64, 8)])
def test_stage2_earlier_schedules_are_also_safe(n, w):
    # publication after the whole step, and every part 3 steps behind
    assert not check_schedule(n, w, publish_after_a=False)
    assert not check_schedule(n, w, lag_a=3, lag_b=3, publish_after_a=False)


@pytest.mark.parametrize("n,w", [(17, 3), (33, 4), (64, 8)])
def test_stage2_one_step_tighter_is_caught(n, w):
    # the check has teeth: part A only 1 step behind, or part B only 2
    assert check_schedule(n, w, lag_a=1, lag_b=3)
    assert check_schedule(n, w, lag_a=2, lag_b=2)
