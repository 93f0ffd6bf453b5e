"""The strong CPU baseline that the benchmark times beside the oracle: the linear-time Split
with a monotone deque of predecessors (oracle.split_deque, C, threaded). It must return the
oracle's Eq. (1) costs on every scenario and report the same errors. CPU only."""
import numpy as np
import pytest

import oracle
from oracle_pins import deque_split, q_positions, random_demand, random_instance


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


@pytest.mark.parametrize("seed", range(12))
def test_deque_baseline_matches_the_oracle(seed):
    rng = np.random.default_rng(900 + seed)
    for case in range(8):
        N = int(rng.integers(1, 70))
        n = int(rng.integers(1, N + 1))
        S = int(rng.integers(1, 200))
        Q = int(rng.integers(1, 120))
        d = random_instance(rng, N, asymmetric=bool(case % 2))
        tour = rng.permutation(np.arange(1, N + 1))[:n].astype(np.int32)
        # demands up to Q (binding capacity), up to Q/2 + 1, or tiny (long windows)
        hi = [Q, Q // 2 + 1, 2][case % 3]
        dem = random_demand(rng, N, S, hi)
        want = oracle.split(tour, d, dem, Q)
        for threads in (1, 3):
            got = oracle.split_deque(tour, d, dem, Q, threads=threads)
            assert np.array_equal(got, want), (seed, case, threads)


def test_deque_baseline_on_a_padded_leading_dimension_and_block_tails():
    # scenario ranges that are not multiples of the 32-scenario copy blocks, read from a
    # demand matrix whose rows are longer than S
    rng = np.random.default_rng(77)
    N, n, Q = 50, 45, 60
    d = random_instance(rng, N, asymmetric=False)
    tour = rng.permutation(np.arange(1, N + 1))[:n].astype(np.int32)
    dem = random_demand(rng, N, 200, Q)
    for S in (1, 31, 32, 33, 95, 150):
        want = oracle.split(tour, d, np.ascontiguousarray(dem[:, :S]), Q)
        for threads in (1, 4):
            got = oracle.split_deque(tour, d, dem, Q, S=S, threads=threads)
            assert np.array_equal(got[:S], want), (S, threads)


def test_deque_baseline_matches_the_python_deque_pin():
    rng = np.random.default_rng(5)
    N, n, S, Q = 30, 30, 20, 40
    d = random_instance(rng, N, asymmetric=True)
    tour = rng.permutation(np.arange(1, N + 1)).astype(np.int32)
    dem = random_demand(rng, N, S, Q)
    got = oracle.split_deque(tour, d, dem, Q)
    for s in range(S):
        assert got[s] == deque_split(tour, d, q_positions(dem, tour, s), Q)


@pytest.mark.parametrize("bad", ["over_capacity", "negative", "repeated_id", "id_range", "n_gt_N"])
def test_deque_baseline_reports_the_oracle_errors(bad):
    rng = np.random.default_rng(3)
    N, S, Q = 12, 40, 30
    d = random_instance(rng, N, asymmetric=False)
    tour = np.arange(1, N + 1, dtype=np.int32)
    dem = random_demand(rng, N, S, Q)
    if bad == "over_capacity":
        dem[4, 17] = Q + 1
    elif bad == "negative":
        dem[7, 33] = -1
    elif bad == "repeated_id":
        tour[5] = tour[2]
    elif bad == "id_range":
        tour[0] = N + 1
    else:
        tour = np.arange(1, N + 2, dtype=np.int32)
    with pytest.raises(oracle.OracleError) as e1:
        oracle.split(tour, d, dem, Q)
    with pytest.raises(oracle.OracleError) as e2:
        oracle.split_deque(tour, d, dem, Q, threads=2)
    assert e1.value.status == e2.value.status
