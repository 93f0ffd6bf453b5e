"""Pins for the CPU oracle: checks against what the paper and the mathematics fix.

Each ``pin_*`` takes ``lib`` (None = the oracle as built, or the path of another build of
``oracle/oracle.c``) and raises AssertionError (or the oracle's error) when the oracle
disagrees with:
  - brute force over all segmentations of tiny tours (the plain definition behind Eq. (1)),
  - an independent O(n) monotone-deque Split (Vidal 2016, C&OR 69), written here,
  - closed forms (one route when Q covers everything, singletons when every q > Q/2, n = 1),
  - invariants (monotone in Q, scenario permutation, tour reversal for symmetric costs),
  - the paper's Example 1 (Section 2) from tests/golden/example1.json,
  - exact integer arithmetic for distances and the sample-average moments.
The same pins are run against deliberately broken copies of the oracle
(tests/test_oracle_mutants.py) to show that each plausible mistake is caught.
"""
from __future__ import annotations

import json
import math
import os
from collections import deque
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
INF = float("inf")


# ---------------------------------------------------------------- independent references

def route_cost(route, d) -> int:
    """Depot -> route customers in order -> depot, arcs directed."""
    c = int(d[0][route[0]])
    for a, b in zip(route[:-1], route[1:]):
        c += int(d[a][b])
    return c + int(d[route[-1]][0])


def brute_force(tour, d, q_pos, Q):
    """Min over all 2^(n-1) segmentations of the tour into feasible consecutive routes.

    Returns (cost, min_route_count, best_segmentations) or (None, None, []) if infeasible.
    """
    n = len(tour)
    best, best_routes, best_segs = None, None, []
    min_routes = None
    for mask_bits in range(1 << (n - 1)):
        cuts = [k + 1 for k in range(n - 1) if mask_bits >> k & 1]
        bounds = [0] + cuts + [n]
        ok, total = True, 0
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            if sum(q_pos[lo:hi]) > Q:
                ok = False
                break
            total += route_cost([int(x) for x in tour[lo:hi]], d)
        if not ok:
            continue
        nr = len(bounds) - 1
        min_routes = nr if min_routes is None else min(min_routes, nr)
        seg = [[int(x) for x in tour[lo:hi]] for lo, hi in zip(bounds[:-1], bounds[1:])]
        if best is None or total < best:
            best, best_segs = total, [seg]
        elif total == best:
            best_segs.append(seg)
    return best, min_routes, best_segs


def deque_split(tour, d, q_pos, Q):
    """O(n) Split with a monotone deque of predecessors (unlimited fleet).

    The cost of route (p+1..i) splits into a term of p and a term of i:
        c(0, s_{p+1}) - D[p+1]   +   D[i] + c(s_i, 0),   D[k] = sum of tour arcs up to k,
    so the best predecessor of i is the one minimising f(p) + c(0, s_{p+1}) - D[p+1] among
    the capacity-feasible p; a deque kept increasing in that key gives it at its front.
    """
    n = len(tour)
    t = [0] + [int(x) for x in tour]  # 1-based positions
    D = [0] * (n + 2)
    for k in range(2, n + 1):
        D[k] = D[k - 1] + int(d[t[k - 1]][t[k]])
    P = [0] * (n + 1)
    for k in range(1, n + 1):
        P[k] = P[k - 1] + int(q_pos[k - 1])
    f = [None] * (n + 1)
    f[0] = 0

    def key(p):
        return f[p] + int(d[0][t[p + 1]]) - D[p + 1]

    dq = deque([0])
    for i in range(1, n + 1):
        while dq and P[i] - P[dq[0]] > Q:
            dq.popleft()
        if not dq:
            return None
        p = dq[0]
        f[i] = key(p) + D[i] + int(d[t[i]][0])
        if i < n:
            ki = key(i)
            while dq and key(dq[-1]) >= ki:
                dq.pop()
            dq.append(i)
    return f[n]


def q_positions(demand, tour, s):
    return [int(demand[int(c) - 1, s]) for c in tour]


def metric_matrix(rng, V, symmetric=False, lo=1, hi=100):
    """Random positive arc weights closed under shortest paths (triangle inequality holds)."""
    w = rng.integers(lo, hi, size=(V, V)).astype(np.int64)
    if symmetric:
        w = np.minimum(w, w.T)
    np.fill_diagonal(w, 0)
    for k in range(V):
        w = np.minimum(w, w[:, [k]] + w[[k], :])
    return w.astype(np.int32)


def random_instance(rng, N, asymmetric):
    if asymmetric:
        d = rng.integers(0, 200, size=(N + 1, N + 1)).astype(np.int32)
        np.fill_diagonal(d, 0)
        return d
    xy = rng.integers(0, 100, size=(N + 1, 2)).astype(np.int32)
    return oracle.dist_matrix(xy)


def random_demand(rng, N, S, Q, zero_frac=0.15):
    dem = rng.integers(0, Q + 1, size=(N, S))
    dem[rng.random((N, S)) < zero_frac] = 0
    return np.ascontiguousarray(dem.astype(np.int16))


# ---------------------------------------------------------------- pins

def pin_isqrt(lib=None):
    rng = np.random.default_rng(11)
    cases = list(range(0, 5000))
    for k in list(range(1, 3000)) + [int(x) for x in rng.integers(1, 1 << 30, size=2000)]:
        cases += [k * k - 1, k * k, k * k + 1, k * k + k, k * k + k + 1, k * k + 2 * k]
    for m in cases:
        assert oracle.isqrt(m, lib=lib) == math.isqrt(m), m


def _nearest_ok(m, k):
    # k >= 0 is the integer nearest to sqrt(m)  <=>  max(2k - 1, 0)^2 <= 4m <= (2k + 1)^2
    return k >= 0 and max(2 * k - 1, 0) ** 2 <= 4 * m <= (2 * k + 1) ** 2


def pin_nint_dist(lib=None):
    for dx in range(-45, 46):
        for dy in range(-45, 46):
            k = oracle.nint_dist(0, 0, dx, dy, lib=lib)
            assert _nearest_ok(dx * dx + dy * dy, k), (dx, dy, k)
    rng = np.random.default_rng(12)
    pts = rng.integers(-(1 << 20), 1 << 20, size=(3000, 4))
    for x1, y1, x2, y2 in pts:
        k = oracle.nint_dist(x1, y1, x2, y2, lib=lib)
        m = int(x1 - x2) ** 2 + int(y1 - y2) ** 2
        assert _nearest_ok(m, k), (x1, y1, x2, y2, k)


def pin_dist_matrix(lib=None):
    rng = np.random.default_rng(13)
    xy = rng.integers(0, 1000, size=(31, 2)).astype(np.int32)
    d = oracle.dist_matrix(xy, lib=lib)
    for a in range(31):
        for b in range(31):
            m = int(xy[a, 0] - xy[b, 0]) ** 2 + int(xy[a, 1] - xy[b, 1]) ** 2
            assert _nearest_ok(m, int(d[a, b])), (a, b)
    assert (d == d.T).all() and (np.diag(d) == 0).all()


def pin_brute_force(lib=None):
    rng = np.random.default_rng(14)
    for trial in range(70):
        n = int(rng.integers(1, 10))
        N = n + int(rng.integers(0, 3))
        asym = trial % 2 == 1
        d = random_instance(rng, N, asym)
        tour = rng.permutation(np.arange(1, N + 1))[:n].astype(np.int32)
        Q = int(rng.integers(1, 60))
        S = 6
        dem = random_demand(rng, N, S, Q)
        got = oracle.split(tour, d, dem, Q, lib=lib)
        for s in range(S):
            want, _, _ = brute_force(tour, d, q_positions(dem, tour, s), Q)
            assert int(got[s]) == want, (trial, s, int(got[s]), want)


def pin_deque(lib=None):
    rng = np.random.default_rng(15)
    for trial in range(16):
        n = int(rng.integers(10, 70))
        N = n + int(rng.integers(0, 5))
        asym = trial % 2 == 1
        d = random_instance(rng, N, asym)
        tour = rng.permutation(np.arange(1, N + 1))[:n].astype(np.int32)
        Q = int(rng.integers(20, 120))
        S = 24
        dem = random_demand(rng, N, S, Q, zero_frac=0.1)
        dem = np.ascontiguousarray(np.minimum(dem, Q // 3 + 1).astype(np.int16))
        got = oracle.split(tour, d, dem, Q, threads=3, lib=lib)
        for s in range(S):
            want = deque_split(tour, d, q_positions(dem, tour, s), Q)
            assert int(got[s]) == want, (trial, s, int(got[s]), want)


def pin_closed_forms(lib=None):
    rng = np.random.default_rng(16)
    for trial in range(20):
        N = int(rng.integers(1, 40))
        # a single route is optimal when Q covers the tour only under the triangle inequality
        d = metric_matrix(rng, N + 1, symmetric=trial % 2 == 0)
        tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
        n = len(tour)
        S = 5
        # Q covers the whole tour: a single route
        dem = rng.integers(0, 10, size=(N, S)).astype(np.int16)
        Q = int(dem.sum(axis=0).max()) + int(rng.integers(0, 3))
        one = route_cost([int(x) for x in tour], d)
        got = oracle.split(tour, d, np.ascontiguousarray(dem), max(Q, 1), lib=lib)
        assert (got == one).all(), (trial, got, one)
        # every demand above Q/2: singletons only
        Q2 = 50
        dem2 = rng.integers(26, 51, size=(N, S)).astype(np.int16)
        single = sum(int(d[0][c]) + int(d[c][0]) for c in tour)
        got2 = oracle.split(tour, d, np.ascontiguousarray(dem2), Q2, lib=lib)
        assert (got2 == single).all(), (trial, got2, single)
        # n = 1
        c = int(tour[0])
        got3 = oracle.split(tour[:1], d, np.ascontiguousarray(dem2), Q2, lib=lib)
        assert (got3 == int(d[0][c]) + int(d[c][0])).all()
        assert n == N


def pin_equal_scenarios(lib=None):
    rng = np.random.default_rng(17)
    for trial in range(8):
        N = int(rng.integers(5, 9))
        d = random_instance(rng, N, trial % 2 == 1)
        tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
        Q = int(rng.integers(10, 40))
        col = rng.integers(0, Q + 1, size=(N, 1))
        dem = np.ascontiguousarray(np.repeat(col, 37, axis=1).astype(np.int16))
        got = oracle.split(tour, d, dem, Q, lib=lib)
        want, _, _ = brute_force(tour, d, q_positions(dem, tour, 0), Q)
        assert (got == want).all(), (trial, got[:3], want)


def pin_monotone_in_Q(lib=None):
    rng = np.random.default_rng(18)
    N = 40
    d = metric_matrix(rng, N + 1, symmetric=False)
    tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
    dem = random_demand(rng, N, 50, 30)
    prev = None
    top = int(dem.astype(np.int64).sum(axis=0).max())
    for Q in list(range(30, top, 7)) + [top]:
        cur = oracle.split(tour, d, dem, Q, lib=lib)
        if prev is not None:
            assert (cur <= prev).all()
        prev = cur
    # with Q at the total demand a single route is reached
    assert (prev == route_cost([int(x) for x in tour], d)).all()


def pin_scenario_permutation(lib=None):
    rng = np.random.default_rng(19)
    N = 30
    d = random_instance(rng, N, True)
    tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
    dem = random_demand(rng, N, 64, 40)
    perm = rng.permutation(64)
    a = oracle.split(tour, d, dem, 40, lib=lib)
    b = oracle.split(tour, d, np.ascontiguousarray(dem[:, perm]), 40, lib=lib)
    assert (a[perm] == b).all()


def pin_reversal(lib=None):
    rng = np.random.default_rng(20)
    for _ in range(4):
        N = 35
        d = random_instance(rng, N, False)
        tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
        dem = random_demand(rng, N, 40, 45)
        a = oracle.split(tour, d, dem, 45, lib=lib)
        b = oracle.split(np.ascontiguousarray(tour[::-1]), d, dem, 45, lib=lib)
        assert (a == b).all()


def pin_mask(lib=None):
    rng = np.random.default_rng(21)
    for _ in range(200):
        n = int(rng.integers(1, 25))
        Q = int(rng.integers(1, 50))
        q = rng.integers(0, Q + 1, size=n)
        if rng.random() < 0.2:
            q[rng.integers(0, n)] = Q + 1 + int(rng.integers(0, 5))
        got = oracle.mask(q, Q, lib=lib)
        for i in range(1, n + 1):
            want = next((p for p in range(i) if sum(q[p:i]) <= Q), -1)
            assert int(got[i - 1]) == want, (q, Q, i)


def pin_eq1_equals_eq3(lib=None):
    rng = np.random.default_rng(22)
    for trial in range(30):
        N = int(rng.integers(3, 30))
        d = random_instance(rng, N, trial % 2 == 0)
        tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
        Q = int(rng.integers(5, 60))
        dem = random_demand(rng, N, 4, Q)
        got = oracle.split(tour, d, dem, Q, lib=lib)
        for s in range(4):
            m = oracle.mask(q_positions(dem, tour, s), Q, lib=lib)
            assert oracle.split_masked(tour, d, m, lib=lib) == int(got[s])


def pin_example1(lib=None):
    with open(os.path.join(GOLDEN, "example1.json")) as fh:
        ex = json.load(fh)
    tour = np.array(ex["tour"], dtype=np.int32)
    Q = ex["Q"]
    N = 5
    rng = np.random.default_rng(23)
    for sc in ex["scenarios"]:
        qpos = sc["demand_by_position"]
        assert list(oracle.mask(qpos, Q, lib=lib)) == sc["mask"]
        dem = np.zeros((N, 1), dtype=np.int16)
        for c, qv in zip(ex["tour"], qpos):
            dem[c - 1, 0] = qv
        for trial in range(60):
            d = metric_matrix(rng, N + 1, symmetric=trial % 2 == 0)
            got = int(oracle.split(tour, d, dem, Q, lib=lib)[0])
            want, min_routes, segs = brute_force(tour, d, qpos, Q)
            assert got == want and min_routes == sc["min_routes"]
            if sc["min_routes"] == 3:
                # the unique 3-route split; under the triangle inequality it is optimal
                assert got == sum(route_cost(r, d) for r in sc["paper_routes"])
            else:
                cands = [sum(route_cost(r, d) for r in split)
                         for split in sc["feasible_two_route_splits"]]
                assert sc["paper_routes"] in sc["feasible_two_route_splits"]
                assert got == min(cands)


def pin_errors(lib=None):
    rng = np.random.default_rng(24)
    N = 12
    d = random_instance(rng, N, False)
    tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
    dem = random_demand(rng, N, 8, 30)
    bad = dem.copy()
    bad[int(tour[4]) - 1, 3] = 31
    _expect_status(lambda: oracle.split(tour, d, np.ascontiguousarray(bad), 30, lib=lib),
                   oracle.E_DEMAND)
    neg = dem.copy()
    neg[int(tour[7]) - 1, 5] = -1
    _expect_status(lambda: oracle.split(tour, d, np.ascontiguousarray(neg), 30, lib=lib),
                   oracle.E_DEMAND)
    dup = tour.copy()
    dup[3] = dup[2]
    _expect_status(lambda: oracle.split(dup, d, dem, 30, lib=lib), oracle.E_TOUR)
    oob = tour.copy()
    oob[0] = N + 1
    _expect_status(lambda: oracle.split(oob, d, dem, 30, lib=lib), oracle.E_TOUR)


def _expect_status(fn, status):
    try:
        fn()
    except oracle.OracleError as e:
        assert e.status == status, (e.status, status)
        return
    raise AssertionError(f"expected oracle status {status}")


def pin_moments(lib=None):
    rng = np.random.default_rng(25)
    for S in (1, 2, 3, 17, 1000, 65536):
        c = rng.integers(0, 3_000_000, size=S).astype(np.int32)
        _check_moments(c, lib)
    # large values: the sum of squares exceeds 64 bits
    c = np.full(1 << 20, (1 << 31) - 1, dtype=np.int32)
    c[::3] = (1 << 30) + 12345
    _check_moments(c, lib)


def _check_moments(c, lib):
    got = oracle.moments(c, lib=lib)
    vals = [int(x) for x in c]
    S = len(vals)
    s1 = sum(vals)
    s2 = sum(v * v for v in vals)
    assert got["sum"] == s1 and got["sumsq"] == s2
    assert got["mean"] == float(Fraction(s1, S))
    if S == 1:
        assert got["var"] == 0.0
        return
    exact = Fraction(S * s2 - s1 * s1, S * (S - 1))
    if exact == 0:
        assert got["var"] == 0.0
    else:
        assert abs(Fraction(got["var"]) - exact) <= exact * Fraction(4, 1 << 52)


def pin_work_count(lib=None):
    rng = np.random.default_rng(26)
    N = 25
    d = random_instance(rng, N, False)
    tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
    Q = 40
    dem = random_demand(rng, N, 30, Q)
    _, work = oracle.split(tour, d, dem, Q, return_work=True, lib=lib)
    want = 0
    for s in range(30):
        q = q_positions(dem, tour, s)
        for i in range(1, N + 1):
            w = sum(1 for p in range(i) if sum(q[p:i]) <= Q)
            want += w - 1
    assert work == want


ALL_PINS = [
    pin_isqrt, pin_nint_dist, pin_dist_matrix, pin_brute_force, pin_deque, pin_closed_forms,
    pin_equal_scenarios, pin_monotone_in_Q, pin_scenario_permutation, pin_reversal, pin_mask,
    pin_eq1_equals_eq3, pin_example1, pin_errors, pin_moments, pin_work_count,
]
