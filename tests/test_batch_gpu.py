"""GPU parity of the batched evaluation (split_eval_batch) against the CPU oracle, tour by tour.

Every tour of a batch must get exactly the costs, exact moments and mean/variance doubles that
the oracle computes for that tour alone. Inputs are seeded and synthetic (see gen/).
"""
import os

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_18022_amd as sg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = sg.SplitContext(0)
    yield c
    c.close()


def check_batch(ctx, tours, dem_np, Q, d_oracle, form="auto", xy=None, d=None, ldc=None):
    if xy is not None:
        ctx.set_coords(xy)
    if d is not None:
        ctx.set_dist(d)
    ctx.set_form(form)
    S = dem_np.shape[1]
    dem = torch.from_numpy(np.ascontiguousarray(dem_np)).cuda()
    cost = None
    if ldc is not None:
        cost = torch.full((len(tours), ldc), -7, dtype=torch.int32, device="cuda")
    cost, stats, status = ctx.eval_batch(tours, dem, Q, cost=cost)
    torch.cuda.synchronize()
    got = cost.cpu().numpy()
    for t, tour in enumerate(tours):
        want = oracle.split(np.asarray(tour, dtype=np.int32), d_oracle,
                            np.ascontiguousarray(dem_np), Q, threads=ORACLE_THREADS)
        bad = np.nonzero(got[t, :S] != want)[0]
        assert bad.size == 0, (f"tour {t} (n={len(tour)}): {bad.size} mismatches, first "
                               f"{bad[:5]}: gpu {got[t, bad[:5]]} oracle {want[bad[:5]]}")
        mom = oracle.moments(want)
        assert stats[t].sum == mom["sum"] and stats[t].sumsq == mom["sumsq"]
        assert stats[t].mean == mom["mean"] and stats[t].var == mom["var"]
        assert status[t] == 0
        if ldc is not None:
            assert np.all(got[t, S:] == -7), "cost padding past S was written"
    return got, stats


@pytest.mark.parametrize("form", ["lane", "wave", "mask"])
def test_uneven_subset_tours(ctx, form):
    b = gen.make_batch_workload("batch-256", T=12, S=3000)
    print(f"[batch] T=12 S=3000 form={form} lengths={[len(t) for t in b.tours]}", flush=True)
    d = oracle.dist_matrix(b.xy)
    check_batch(ctx, b.tours, b.demand, b.Q, d, form=form, xy=b.xy)


def test_batch_shape_full_scenarios_sampled_tours(ctx):
    # the batched workload at its full scenario count, tours checked on a sample of scenarios
    b = gen.make_batch_workload("batch-256", T=24)
    print(f"[batch] T=24 S={b.S}", flush=True)
    d = oracle.dist_matrix(b.xy)
    ctx.set_coords(b.xy)
    ctx.set_form("auto")
    dem = torch.from_numpy(b.demand).cuda()
    cost, stats, status = ctx.eval_batch(b.tours, dem, b.Q)
    torch.cuda.synchronize()
    got = cost.cpu().numpy()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(b.S, size=512, replace=False))
    sub = np.ascontiguousarray(b.demand[:, idx])
    for t, tour in enumerate(b.tours):
        want = oracle.split(tour, d, sub, b.Q, threads=ORACLE_THREADS)
        assert np.array_equal(got[t, idx], want), f"tour {t}"
        assert status[t] == 0
        # the exact moments of the whole row agree with the row the GPU wrote
        mom = oracle.moments(got[t])
        assert stats[t].sum == mom["sum"] and stats[t].sumsq == mom["sumsq"]


def test_padded_cost_rows_and_single_tour_batch(ctx):
    w = gen.make_workload("poisson-n200", S=2500)
    d = oracle.dist_matrix(w.xy)
    tours = [w.tour, w.tour[:37], w.tour[::-1][:150]]
    check_batch(ctx, tours, w.demand, w.Q, d, form="lane", xy=w.xy, ldc=2500 + 41)
    # a batch of one is split_eval
    dem = torch.from_numpy(w.demand).cuda()
    c1, s1 = ctx.eval(w.tour, dem, w.Q)
    cb, sb, _ = ctx.eval_batch([w.tour], dem, w.Q)
    torch.cuda.synchronize()
    assert np.array_equal(c1.cpu().numpy(), cb.cpu().numpy()[0])
    assert s1.sum == sb[0].sum and s1.var == sb[0].var


@pytest.mark.parametrize("form", ["lane", "wave", "mask"])
def test_infeasible_tour_is_isolated(ctx, form):
    import paper_2511_18022_amd as sg
    w = gen.make_workload("uniform-n20", S=700)
    dem = w.demand.copy()
    bad_customer = int(w.tour[15])
    dem[bad_customer - 1, 321] = 101  # > Q = 100
    tours = [w.tour[:10], w.tour, np.array([c for c in w.tour if c != bad_customer],
                                           dtype=np.int32)]
    ctx.set_coords(w.xy)
    ctx.set_form(form)
    with pytest.raises(sg.SplitError) as ei:
        ctx.eval_batch(tours, torch.from_numpy(dem).cuda(), w.Q)
    assert ei.value.status == sg.SPLIT_E_DEMAND
    stats, status = ctx.batch_stats()
    assert status == [0, sg.SPLIT_E_DEMAND, 0]
    d = oracle.dist_matrix(w.xy)
    cost, _, _ = ctx.eval_batch([tours[0], tours[2]], torch.from_numpy(dem).cuda(), w.Q)
    got = cost.cpu().numpy()
    for k, tour in enumerate([tours[0], tours[2]]):
        assert np.array_equal(got[k], oracle.split(tour, d, dem, w.Q))


def test_fallback_scenarios_in_a_batch(ctx):
    # long zero-demand runs make windows longer than the lane kernel keeps: those scenarios
    # are marked and finished by the general kernel, tour by tour
    N = 600
    xy = gen.coords(11, N)
    d = oracle.dist_matrix(xy)
    dem = gen.demand_uniform(11, N, 1500, 0, 40)
    rng = np.random.default_rng(3)
    cols = rng.choice(1500, size=200, replace=False)
    for c in cols:
        lo = int(rng.integers(0, N - 200))
        dem[lo:lo + int(rng.integers(60, 200)), c] = 0
    dem[:, cols[:15]] = 0  # scenarios without demand: one route, a window over the whole tour
    tours = [gen.tour(11, N, n, variant=v) for v, n in [(1, 600), (2, 333), (3, 480), (4, 90)]]
    _, stats = check_batch(ctx, tours, dem, 200, d, form="lane", xy=xy)
    assert sum(s.n_fallback for s in stats) > 0


def test_batch_argument_errors(ctx):
    import paper_2511_18022_amd as sg
    w = gen.make_workload("uniform-n20", S=100)
    ctx.set_coords(w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    for tours, code in [([w.tour, np.array([1, 2, 2], dtype=np.int32)], sg.SPLIT_E_TOUR),
                        ([w.tour, np.array([], dtype=np.int32)], sg.SPLIT_E_INVAL)]:
        with pytest.raises(sg.SplitError) as ei:
            ctx.eval_batch(tours, dem, w.Q)
        assert ei.value.status == code


def test_every_tail_length_stays_in_the_lane_kernel(ctx):
    # short capacity windows (copula demands, mean 20, Q = 500): the lane kernel finishes every
    # scenario itself whatever n mod 16 is, including a last block that ends at state n
    b = gen.make_batch_workload("batch-256", T=1, S=1024)
    d = oracle.dist_matrix(b.xy)
    lens = [16 * k + r for r, k in zip(range(16), (1, 2, 3, 5, 8, 13, 21, 34, 55, 40, 20, 10,
                                                    6, 4, 3, 61))]
    tours = [gen.tour(b.seed, b.N, n, variant=100 + n) for n in lens]
    print(f"[batch] tail lengths {lens}", flush=True)
    _, stats = check_batch(ctx, tours, b.demand, b.Q, d, form="lane", xy=b.xy)
    assert [s.n_fallback for s in stats] == [0] * len(tours)


@pytest.mark.parametrize("k", range(8))
def test_seeded_random_batches_under_launch_choices(ctx, k):
    # random batches (uneven subset tours, some of a single customer) under a different launch
    # choice each: one workgroup per item or a persistent queue, longest-first or given order,
    # 16- or 8-state blocks, the lane or the wave form; every tour matches the oracle
    import paper_2511_18022_amd as sg
    rng = np.random.default_rng(7000 + k)
    N = int(rng.integers(2, 300))
    S = int(rng.integers(1, 2500))
    T = int(rng.integers(1, 40))
    xy = gen.coords(7000 + k, N)
    Q = int(rng.integers(60, 600))
    dem = np.clip(gen.demand_uniform(7000 + k, N, S, 0, Q // int(rng.integers(3, 30))), 0, Q)
    tours = [gen.tour(7000 + k, N, int(rng.integers(1, N + 1)), variant=v) for v in range(T)]
    choices = [(sg.FORM_LANE, 0, 0, 0), (sg.FORM_LANE, 8, 1, 8), (sg.FORM_LANE, 2, 0, 16),
               (sg.FORM_LANE, 1, 1, 8), (sg.FORM_WAVE, 0, 0, 0), (sg.FORM_LANE, 4, 0, 8),
               (sg.FORM_LANE, 0, 1, 8), (sg.FORM_WAVE, 0, 1, 0)]
    form, per_cu, order, block = choices[k]
    print(f"[batch] random case {k}: N={N} S={S} T={T} Q={Q} form {form} per_cu {per_cu} "
          f"order {order} lane_block {block}", flush=True)
    ctx.set_coords(xy)
    ctx.set_tuning(sg.SplitTuning(form, per_cu, order, 0, block))
    try:
        check_batch(ctx, tours, np.ascontiguousarray(dem.astype(np.int16)), Q,
                    oracle.dist_matrix(xy), form={sg.FORM_LANE: "lane", sg.FORM_WAVE: "wave"}[form])
    finally:
        ctx.set_tuning(sg.SplitTuning(sg.FORM_AUTO, 0, 0, 0))
