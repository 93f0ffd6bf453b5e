"""Sample-average estimates of a tour's expected recourse cost (the appendix's Monte Carlo
proposition): for a fixed first-stage tour the scenario mean over m i.i.d. scenarios is
asymptotically normal around the true expectation with variance sigma^2 / m (its rate-of-
convergence statement), so

- two independent scenario sets give means within a few standard errors of each other;
- the means of k disjoint slices of one set (independent sets of size m / k) scatter with a
  sample variance close to sigma^2 / (m / k), and their average is the whole set's mean exactly
  (sums are exact integers).

The tour and demand law are the n = 1000, S = 2^20 copula workload's; the scenario sets use other
seeds. The library's own variances (sample variance of the costs) supply sigma^2.
"""
import numpy as np
import pytest

import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import paper_2511_18022_amd as sg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return sg


def _copula_set(seed, w, S):
    law = gen.RECIPES["copula-n1000"]["law"]
    return gen.demand_copula(seed, w.N, S, law[1], law[2], law[3], w.Q, threads=16)


def test_independent_scenario_sets_agree_within_standard_errors(sg):
    w = gen.make_workload("copula-n1000", S=64)  # the instance and tour; scenarios below
    S = 1 << 20
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    means, vars_ = [], []
    for seed in (1003, 2003):
        print(f"[saa] scenario set seed {seed}, S = {S}", flush=True)
        dem = torch.from_numpy(_copula_set(seed, w, S)).cuda()
        _, st = ctx.eval(w.tour, dem, w.Q)
        assert st.n_fallback == 0
        means.append(st.mean)
        vars_.append(st.var)
        del dem
    se = np.sqrt((vars_[0] + vars_[1]) / S)
    gap = abs(means[0] - means[1])
    print(f"[saa] means {means}, sd {np.sqrt(vars_)}, |gap| = {gap:.3f} = {gap / se:.2f} se",
          flush=True)
    assert gap <= 4.0 * se
    # the two sets estimate the same spread as well (relative gap of sample variances)
    assert abs(vars_[0] - vars_[1]) <= 0.05 * max(vars_)
    ctx.close()


def test_slice_means_scatter_as_sigma_over_root_m(sg):
    scipy_stats = pytest.importorskip("scipy.stats")
    w = gen.make_workload("copula-n1000", S=64)
    S, k = 1 << 20, 32
    m = S // k
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    dem = torch.from_numpy(_copula_set(3003, w, S)).cuda()
    _, whole = ctx.eval(w.tour, dem, w.Q)
    sums, means = [], []
    for j in range(k):
        # a column slice: leading dimension S, m scenarios starting at column j * m
        _, st = ctx.eval(w.tour, dem[:, j * m:(j + 1) * m], w.Q)
        sums.append(st.sum)
        means.append(st.mean)
    assert sum(sums) == whole.sum  # exact integer sums: the slices partition the set
    assert abs(float(np.mean(means)) - whole.mean) <= 1e-9 * whole.mean
    # (k - 1) s^2 / (sigma^2 / m) is chi-square with k - 1 degrees of freedom; two-sided 1e-4
    ratio = float(np.var(means, ddof=1)) / (whole.var / m)
    lo = scipy_stats.chi2.ppf(1e-4, k - 1) / (k - 1)
    hi = scipy_stats.chi2.ppf(1 - 1e-4, k - 1) / (k - 1)
    print(f"[saa] {k} slices of {m}: var(means) / (sigma^2 / m) = {ratio:.3f} "
          f"(accepted [{lo:.3f}, {hi:.3f}])", flush=True)
    assert lo <= ratio <= hi
    ctx.close()
