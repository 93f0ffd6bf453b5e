"""Seeded input generators: Philox4x32-10 known answers, determinism, thread independence and
the marginal statistics of each demand law. CPU only."""
import numpy as np
import pytest

import gen

# Known-answer vectors published with the Random123 library for Philox4x32-10.
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.fixture(scope="module", autouse=True)
def _built():
    gen.build(force=False)


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert list(gen.philox4x32_10(ctr, key)) == want


def test_coords_and_tours():
    xy = gen.coords(5, 300)
    assert xy.shape == (301, 2) and xy.min() >= 0 and xy.max() <= 999
    t = gen.tour(5, 300)
    assert sorted(t.tolist()) == list(range(1, 301))
    sub = gen.tour(5, 300, n=120, variant=3)
    assert len(set(sub.tolist())) == 120 and sub.min() >= 1 and sub.max() <= 300
    assert not np.array_equal(gen.tour(5, 300), gen.tour(6, 300))
    assert np.array_equal(gen.tour(5, 300), t)


@pytest.mark.parametrize("law", ["uniform", "poisson", "copula"])
def test_thread_count_does_not_change_values(law):
    def make(seed, threads):
        if law == "uniform":
            return gen.demand_uniform(seed, 50, 3001, 1, 20, threads=threads)
        if law == "poisson":
            return gen.demand_poisson(seed, 50, 3001, 5.0, 25.0, 200, threads=threads)
        return gen.demand_copula(seed, 50, 3001, 0.6, 20.0, 0.5, 500, threads=threads)
    a, b = make(7, 1), make(7, 5)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, make(8, 3))


def test_leading_dimension_pads_rows():
    a = gen.demand_uniform(3, 10, 100, 1, 20)
    b = gen.demand_uniform(3, 10, 100, 1, 20, ld=128)
    assert b.shape == (10, 128) and np.array_equal(a, b[:, :100])


def test_uniform_law():
    q = gen.demand_uniform(1, 20, 20000, 1, 20)
    assert q.min() == 1 and q.max() == 20
    assert abs(q.mean() - 10.5) < 0.05
    counts = np.bincount(q.ravel(), minlength=21)[1:]
    assert counts.min() > 0.9 * counts.mean()


def test_poisson_law():
    q, lam = gen.demand_poisson(2, 40, 20000, 5.0, 25.0, 200, return_lambda=True)
    assert lam.min() >= 5.0 and lam.max() <= 25.0
    m = q.astype(np.float64).mean(axis=1)
    v = q.astype(np.float64).var(axis=1)
    assert np.all(np.abs(m - lam) < 4 * np.sqrt(lam / 20000) + 1e-9)
    assert np.all(np.abs(v / lam - 1.0) < 0.08)
    assert q.min() >= 0 and q.max() <= 200


def test_copula_law():
    q = gen.demand_copula(3, 60, 40000, 0.6, 20.0, 0.5, 500)
    x = q.astype(np.float64)
    assert abs(x.mean() - 20.0) < 0.1
    assert abs(x.std() / x.mean() - 0.5) < 0.01
    lq = np.log(np.maximum(x, 0.5))
    r = [np.corrcoef(lq[c], lq[c + 1])[0, 1] for c in range(59)]
    assert abs(np.mean(r) - 0.6) < 0.02
    far = [np.corrcoef(lq[c], lq[c + 10])[0, 1] for c in range(49)]
    assert abs(np.mean(far) - 0.6 ** 10) < 0.02
    assert q.min() >= 0 and q.max() <= 500


def test_named_workloads_small():
    w = gen.make_workload("uniform-n20")
    assert w.demand.shape == (20, 1000) and w.Q == 100 and len(w.tour) == 20
    w2 = gen.make_workload("poisson-n200", S=1000)
    assert w2.demand.shape == (200, 1000) and w2.Q == 200
    w3 = gen.make_workload("copula-n1000", S=512)
    assert w3.demand.shape == (1000, 512) and w3.Q == 500


def _cycle_len(xy, t):
    p = np.r_[0, t, 0]
    return float(np.hypot(*(xy[p[1:]] - xy[p[:-1]]).T).sum())


def test_two_opt_base_tour_is_a_short_permutation():
    xy = gen.coords(5, 300)
    t = gen.two_opt_tour(xy)
    assert sorted(t.tolist()) == list(range(1, 301))
    # 2-opt local optimum: no single reversal shortens the depot cycle
    L = _cycle_len(xy, t)
    rng = np.random.default_rng(0)
    for _ in range(300):
        i, j = sorted(rng.choice(300, 2, replace=False))
        u = t.copy()
        u[i:j + 1] = u[i:j + 1][::-1]
        assert _cycle_len(xy, u) >= L - 1e-6
    assert L < 0.2 * _cycle_len(xy, gen.tour(5, 300))


def test_perturbed_candidates_are_permutations_and_thread_independent():
    xy = gen.coords(6, 200)
    base = gen.two_opt_tour(xy)
    a = gen.perturb(11, base, 500, 1, 20, threads=1)
    b = gen.perturb(11, base, 500, 1, 20, threads=7)
    assert np.array_equal(a, b)
    assert all(sorted(row.tolist()) == list(range(1, 201)) for row in a)
    assert not np.array_equal(a, gen.perturb(12, base, 500, 1, 20))
    # zero moves reproduce the base tour
    assert np.array_equal(gen.perturb(11, base, 3, 0, 0), np.stack([base] * 3))
