"""split_eval_noalloc (the entry point for callers that cannot allocate device memory) against
split_eval, the entry point whose kernels it shares: identical costs, exact moments and mean /
variance doubles on two calls in a row, the second with a smaller input, and the oracle's costs
on a sample. Run alone in a fresh process and after the other GPU tests."""
import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import paper_2511_18022_amd as sg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return sg


def _pair(ctx, tour, dem, Q, S):
    """(costs, stats) of split_eval and of split_eval_noalloc on the same input."""
    ref_cost, ref = ctx.eval(tour, dem, Q, S=S)
    ref_cost = ref_cost[:S].cpu().numpy()
    cost = torch.full((S + 7,), -5, dtype=torch.int32, device="cuda")
    st = ctx.eval_noalloc(tour, dem, Q, cost, S=S)
    got = cost.cpu().numpy()
    assert np.all(got[S:] == -5), "written past S"
    return ref_cost, ref, got[:S], st


@pytest.mark.parametrize("form", ["auto", "lane", "lane8", "wave"])
def test_noalloc_matches_split_eval_on_two_calls_the_second_smaller(sg, form):
    big = gen.make_workload("copula-n1000", S=300_000, threads=16)
    small = gen.make_workload("poisson-n200", S=5000)
    ctx = sg.SplitContext(0)
    if form == "lane8":  # 8-state blocks: the copula tour's long windows go to the wave kernel
        ctx.set_tuning(sg.SplitTuning(sg.FORM_LANE, lane_block=8))
    else:
        ctx.set_form(form)
    for w in (big, small):
        ctx.set_coords(w.xy)
        dem = torch.from_numpy(w.demand).cuda()
        print(f"[noalloc] form {form}, n={w.n}, S={w.S}", flush=True)
        ref_cost, ref, got, st = _pair(ctx, w.tour, dem, w.Q, w.S)
        assert np.array_equal(got, ref_cost)
        assert (st.sum, st.sumsq, st.mean, st.var, st.n_fallback) == (
            ref.sum, ref.sumsq, ref.mean, ref.var, ref.n_fallback)
        # the oracle on a sample of the scenarios
        d = oracle.dist_matrix(w.xy)
        k = min(w.S, 4096)
        want = oracle.split(w.tour, d, np.ascontiguousarray(w.demand[:, :k]), w.Q, threads=16)
        assert np.array_equal(got[:k], want)
    ctx.close()


def test_noalloc_asynchronous_call_then_a_shorter_tour(sg):
    # a call that only enqueues, then a shorter tour on a column slice; the scratch keeps the
    # last call's contents, and each call's result block is cleared by its own prep kernel
    w = gen.make_workload("copula-n1000", S=20000)
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    cost = torch.empty(w.S, dtype=torch.int32, device="cuda")
    assert ctx.eval_noalloc(w.tour, dem, w.Q, cost, sync=False) is None
    torch.cuda.synchronize()
    want, ref = ctx.eval(w.tour, dem, w.Q)
    assert np.array_equal(cost.cpu().numpy(), want.cpu().numpy())
    short = np.ascontiguousarray(w.tour[:137])
    sl = dem[:, 1000:1000 + 3333]
    cost2 = torch.empty(3333, dtype=torch.int32, device="cuda")
    st = ctx.eval_noalloc(short, sl, w.Q, cost2)
    want2, ref2 = ctx.eval(short, sl, w.Q)
    assert np.array_equal(cost2.cpu().numpy(), want2.cpu().numpy())
    assert (st.sum, st.sumsq, st.mean, st.var) == (ref2.sum, ref2.sumsq, ref2.mean, ref2.var)
    ctx.close()


def test_noalloc_errors(sg):
    w = gen.make_workload("uniform-n20", S=500)
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    bad = w.demand.copy()
    bad[int(w.tour[2]) - 1, 9] = 101  # above Q = 100
    cost = torch.empty(w.S, dtype=torch.int32, device="cuda")
    with pytest.raises(sg.SplitError) as ei:
        ctx.eval_noalloc(w.tour, torch.from_numpy(bad).cuda(), w.Q, cost)
    assert ei.value.status == sg.SPLIT_E_DEMAND
    ctx.set_form("mask")
    with pytest.raises(sg.SplitError) as ei:
        ctx.eval_noalloc(w.tour, torch.from_numpy(w.demand).cuda(), w.Q, cost)
    assert ei.value.status == sg.SPLIT_E_INVAL
    ctx.set_form("auto")
    # the next good call is unaffected by the failed ones
    dem = torch.from_numpy(w.demand).cuda()
    st = ctx.eval_noalloc(w.tour, dem, w.Q, cost)
    want, ref = ctx.eval(w.tour, dem, w.Q)
    assert np.array_equal(cost.cpu().numpy(), want.cpu().numpy()) and st.sum == ref.sum
    ctx.close()
