"""GPU tests of the launch choices, the autotuner and captured evaluation graphs: none of them
may change a single cost. Every result is compared with the CPU oracle (or with an eager
evaluation that is itself compared with the oracle)."""
import os

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def sg():
    import paper_2511_18022_amd as sg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return sg


@pytest.fixture(scope="module")
def batch():
    b = gen.make_batch_workload("batch-256", T=7, S=2500)
    d = oracle.dist_matrix(b.xy)
    want = [oracle.split(t, d, b.demand, b.Q, threads=ORACLE_THREADS) for t in b.tours]
    return b, d, want


def fresh_ctx(sg, xy):
    c = sg.SplitContext(0)
    c.set_coords(xy)
    return c


def test_every_launch_choice_gives_the_oracle_costs(sg, batch):
    b, d, want = batch
    ctx = fresh_ctx(sg, b.xy)
    dem = torch.from_numpy(b.demand).cuda()
    choices = [sg.SplitTuning(sg.FORM_LANE, pc, order, 0, lb)
               for lb in (0, 8) for pc in (0, 1, 2, 4, 8) for order in (0, 1)]
    choices += [sg.SplitTuning(sg.FORM_WAVE, 0, 0, wg) for wg in (0, 1024)]
    for tu in choices:
        print(f"[tuning] {tu}", flush=True)
        ctx.set_tuning(tu)
        assert ctx.tuning() == tu
        cost, stats, status = ctx.eval_batch(b.tours, dem, b.Q)
        got = cost.cpu().numpy()
        for t in range(len(b.tours)):
            assert np.array_equal(got[t], want[t]), (tu, t)
            assert stats[t].sum == int(want[t].astype(np.int64).sum())
        assert status == [0] * len(b.tours)
    ctx.close()


def test_tuning_fields_are_checked(sg, batch):
    b, _, _ = batch
    ctx = fresh_ctx(sg, b.xy)
    for bad in (sg.SplitTuning(7, 0, 0, 0), sg.SplitTuning(1, 9, 0, 0),
                sg.SplitTuning(1, -1, 0, 0), sg.SplitTuning(1, 0, 2, 0),
                sg.SplitTuning(2, 0, 0, -5), sg.SplitTuning(1, 0, 0, 0, 4),
                sg.SplitTuning(1, 0, 0, 0, 12)):
        with pytest.raises(sg.SplitError) as ei:
            ctx.set_tuning(bad)
        assert ei.value.status == sg.SPLIT_E_INVAL
    assert ctx.tuning() == sg.SplitTuning()
    ctx.close()


def test_autotune_installs_a_choice_and_keeps_the_costs(sg, batch):
    b, _, want = batch
    ctx = fresh_ctx(sg, b.xy)
    dem = torch.from_numpy(b.demand).cuda()
    tu, ms, cost = ctx.autotune(b.tours, dem, b.Q, reps=2)
    print(f"[autotune] {tu} {ms:.4f} ms", flush=True)
    assert ms > 0 and ctx.tuning() == tu
    got = cost.cpu().numpy()
    for t in range(len(b.tours)):
        assert np.array_equal(got[t], want[t])
    stats, status = ctx.batch_stats()
    assert status == [0] * len(b.tours)
    assert [s.sum for s in stats] == [int(w.astype(np.int64).sum()) for w in want]
    # later calls run under the installed choice and still agree
    cost2, _, _ = ctx.eval_batch(b.tours[::-1], dem, b.Q)
    got2 = cost2.cpu().numpy()
    for k, t in enumerate(range(len(b.tours) - 1, -1, -1)):
        assert np.array_equal(got2[k], want[t])
    ctx.close()


def test_autotune_small_scenario_count_considers_the_wave_form(sg):
    w = gen.make_workload("uniform-n20", S=1000)
    d = oracle.dist_matrix(w.xy)
    ctx = fresh_ctx(sg, w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    tu, ms, cost = ctx.autotune([w.tour], dem, w.Q, reps=3)
    print(f"[autotune] uniform-n20: {tu} {ms:.4f} ms", flush=True)
    assert np.array_equal(cost.cpu().numpy()[0], oracle.split(w.tour, d, w.demand, w.Q))
    ctx.close()


@pytest.mark.parametrize("name,block", [("poisson-n200", 8), ("copula-n1000", 16)])
def test_autotune_block_length_follows_the_window_lengths(sg, name, block):
    # windows of about 13 positions (poisson-n200) mostly start inside 16-state blocks: 8-state
    # blocks keep them in older blocks and win. Windows of about 24 (copula-n1000) outgrow
    # three 8-state blocks: the fallback probe drops 8 and 16 stays.
    w = gen.make_workload(name, S=65536, threads=ORACLE_THREADS)
    ctx = fresh_ctx(sg, w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    tu, ms, cost = ctx.autotune([w.tour], dem, w.Q, reps=5)
    print(f"[autotune] {name}: {tu} {ms:.4f} ms", flush=True)
    assert tu.form == sg.FORM_LANE and tu.lane_block == block
    _, stats, _ = ctx.eval_batch([w.tour], dem, w.Q)
    assert stats[0].n_fallback == 0
    # the costs under the choice, on a sample against the oracle
    idx = np.random.default_rng(5).choice(w.S, size=2048, replace=False)
    want = oracle.split(w.tour, oracle.dist_matrix(w.xy),
                        np.ascontiguousarray(w.demand[:, idx]), w.Q, threads=ORACLE_THREADS)
    assert np.array_equal(cost.cpu().numpy()[0, idx], want)
    ctx.close()


def test_graph_replays_match_eager_evaluations(sg, batch):
    b, d, want = batch
    ctx = fresh_ctx(sg, b.xy)
    dem = torch.from_numpy(b.demand).cuda()
    N = b.N
    rng = np.random.default_rng(17)
    g = ctx.graph(max_T=8, max_total_n=8 * 700, demand=dem, Q=b.Q)
    eager_cost = torch.empty((8, b.S), dtype=torch.int32, device="cuda")
    for rep in range(5):
        T = int(rng.integers(1, 9))
        lens = rng.integers(1, 700, size=T)
        tours = [gen.tour(b.seed, N, int(n), variant=1000 + 10 * rep + k)
                 for k, n in enumerate(lens)]
        print(f"[graph] replay {rep}: T={T} lengths={lens.tolist()}", flush=True)
        cost = g.launch(tours)
        gstats, gstatus = g.stats()
        torch.cuda.synchronize()
        got = cost[:T].cpu().numpy()
        # eager work between replays, on the same stream
        ec, estats, estatus = ctx.eval_batch(tours, dem, b.Q, cost=eager_cost)
        torch.cuda.synchronize()
        exp = ec[:T].cpu().numpy()
        assert np.array_equal(got, exp), f"replay {rep}"
        assert gstatus == estatus == [0] * T
        assert [s.sum for s in gstats] == [s.sum for s in estats]
        assert [s.var for s in gstats] == [s.var for s in estats]
        # the eager result itself against the oracle, on a sample of scenarios
        idx = np.arange(0, b.S, 37)
        sub = np.ascontiguousarray(b.demand[:, idx])
        for k, t in enumerate(tours):
            assert np.array_equal(exp[k, idx], oracle.split(t, d, sub, b.Q))
    # the batch the fixture checked in full, through the graph
    cost = g.launch(b.tours)
    g.stats()
    got = cost[:len(b.tours)].cpu().numpy()
    for t in range(len(b.tours)):
        assert np.array_equal(got[t], want[t])
    g.close()
    ctx.close()


def test_graph_with_8_state_blocks_and_the_persistent_queue(sg):
    # the graph captures the context's launch choices: here 8-state blocks and 2 persistent
    # workgroups per CU, over short-window Poisson demands (the case 8-state blocks are for);
    # every replay equals an eager evaluation under the same choice and the oracle
    w = gen.make_workload("poisson-n200", S=20000)
    d = oracle.dist_matrix(w.xy)
    ctx = fresh_ctx(sg, w.xy)
    ctx.set_tuning(sg.SplitTuning(sg.FORM_LANE, 2, 0, 0, 8))
    dem = torch.from_numpy(w.demand).cuda()
    rng = np.random.default_rng(23)
    g = ctx.graph(max_T=4, max_total_n=4 * w.N, demand=dem, Q=w.Q)
    for rep in range(3):
        T = int(rng.integers(1, 5))
        tours = [gen.tour(w.seed, w.N, int(rng.integers(1, w.N + 1)), variant=500 + 10 * rep + k)
                 for k in range(T)]
        print(f"[graph-lb8] replay {rep}: T={T} lengths={[len(t) for t in tours]}", flush=True)
        cost = g.launch(tours)
        gstats, gstatus = g.stats()
        got = cost[:T].cpu().numpy()
        ec, estats, estatus = ctx.eval_batch(tours, dem, w.Q)
        assert np.array_equal(got, ec.cpu().numpy()), f"replay {rep}"
        assert gstatus == estatus == [0] * T
        assert [s.sum for s in gstats] == [s.sum for s in estats]
        assert sum(s.n_fallback for s in gstats) == 0
        for k, t in enumerate(tours):
            assert np.array_equal(got[k], oracle.split(t, d, w.demand, w.Q,
                                                       threads=ORACLE_THREADS)), (rep, k)
    g.close()
    ctx.close()


def test_block_length_takes_effect_in_eager_calls_and_graphs(sg):
    # windows of 24..38 positions (copula-n1000) fit three 16-state blocks but not three 8-state
    # ones: under 8-state blocks the lane kernel hands scenarios to the wave kernel, which shows
    # that the choice reaches the launch, eager and captured alike; the costs stay exact
    w = gen.make_workload("copula-n1000", S=4096, threads=ORACLE_THREADS)
    d = oracle.dist_matrix(w.xy)
    want = oracle.split(w.tour, d, w.demand, w.Q, threads=ORACLE_THREADS)
    ctx = fresh_ctx(sg, w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    for block, falls_back in ((16, False), (8, True)):
        ctx.set_tuning(sg.SplitTuning(sg.FORM_LANE, 0, 0, 0, block))
        cost, stats, status = ctx.eval_batch([w.tour], dem, w.Q)
        assert status == [0]
        assert np.array_equal(cost.cpu().numpy()[0], want)
        assert (stats[0].n_fallback > 0) == falls_back, (block, stats[0].n_fallback)
        g = ctx.graph(1, w.n, dem, w.Q)
        gcost = g.launch([w.tour])
        gstats, gstatus = g.stats()
        assert gstatus == [0]
        assert np.array_equal(gcost[:1].cpu().numpy()[0], want)
        assert gstats[0].n_fallback == stats[0].n_fallback, (block, gstats[0].n_fallback)
        g.close()
    ctx.close()


def test_graph_back_to_back_launches_keep_each_batch(sg, batch):
    # two launches in flight use the two host slots; each batch's result is read after the
    # stream reaches it
    b, _, want = batch
    ctx = fresh_ctx(sg, b.xy)
    dem = torch.from_numpy(b.demand).cuda()
    g = ctx.graph(max_T=7, max_total_n=7 * 1000, demand=dem, Q=b.Q)
    snaps = []
    for rep in range(4):
        tours = b.tours if rep % 2 == 0 else b.tours[::-1]
        cost = g.launch(tours)
        snaps.append((rep, cost[:7].clone()))
    torch.cuda.synchronize()
    for rep, c in snaps:
        got = c.cpu().numpy()
        order = range(7) if rep % 2 == 0 else range(6, -1, -1)
        for k, t in enumerate(order):
            assert np.array_equal(got[k], want[t]), (rep, k)
    g.close()
    ctx.close()


def test_graph_keeps_its_instance_and_checks_capacity(sg, batch):
    b, d, want = batch
    ctx = fresh_ctx(sg, b.xy)
    dem = torch.from_numpy(b.demand).cuda()
    g = ctx.graph(max_T=3, max_total_n=1500, demand=dem, Q=b.Q)
    # a later instance on the context does not reach the graph
    ctx.set_coords(gen.coords(99, b.N))
    picks = [i for i, t in enumerate(b.tours) if len(t) <= 500][:3]
    assert picks, "the fixture batch has tours of at most 500 customers"
    cost = g.launch([b.tours[i] for i in picks])
    g.stats()
    got = cost[:len(picks)].cpu().numpy()
    for k, i in enumerate(picks):
        assert np.array_equal(got[k], want[i])
    long2 = [gen.tour(b.seed, b.N, 800, variant=501), gen.tour(b.seed, b.N, 800, variant=502)]
    for tours, code in [([b.tours[picks[0]]] * 4, sg.SPLIT_E_INVAL),  # T over capacity
                        (long2, sg.SPLIT_E_INVAL),                    # 1600 positions > 1500
                        ([np.array([1, 2, 1], dtype=np.int32)], sg.SPLIT_E_TOUR)]:
        with pytest.raises(sg.SplitError) as ei:
            g.launch(tours)
        assert ei.value.status == code
    # the failed launches left the graph usable
    cost = g.launch([b.tours[picks[0]]])
    g.stats()
    assert np.array_equal(cost[0].cpu().numpy(), want[picks[0]])
    g.close()
    ctx.close()


def test_graph_reports_an_infeasible_tour(sg):
    w = gen.make_workload("uniform-n20", S=300)
    d = oracle.dist_matrix(w.xy)
    dem = w.demand.copy()
    bad = int(w.tour[4])
    dem[bad - 1, 77] = 150  # > Q = 100
    ctx = fresh_ctx(sg, w.xy)
    ddem = torch.from_numpy(dem).cuda()
    g = ctx.graph(max_T=2, max_total_n=40, demand=ddem, Q=w.Q)
    ok_tour = np.array([c for c in w.tour if c != bad], dtype=np.int32)
    cost = g.launch([ok_tour, w.tour])
    stats, status = g.stats()
    assert status == [0, sg.SPLIT_E_DEMAND]
    assert np.array_equal(cost[0].cpu().numpy(), oracle.split(ok_tour, d, dem, w.Q))
    g.close()
    ctx.close()


def test_graphs_reject_the_two_kernel_ablation(sg, batch):
    b, _, _ = batch
    ctx = fresh_ctx(sg, b.xy)
    ctx.set_form("mask")
    dem = torch.from_numpy(b.demand).cuda()
    with pytest.raises(sg.SplitError) as ei:
        ctx.graph(max_T=2, max_total_n=2000, demand=dem, Q=b.Q)
    assert ei.value.status == sg.SPLIT_E_INVAL
    ctx.close()


def test_graph_at_full_size_in_the_timed_configuration(sg):
    # one 1000-customer tour over 2^20 copula scenarios, replayed from a captured graph as the
    # throughput line times it (automatic form choice, cost viewed as one row): every cost of
    # every replay against the eager evaluation, and a sample of scenarios against the oracle
    w = gen.make_workload("copula-n1000", threads=ORACLE_THREADS)
    ctx = fresh_ctx(sg, w.xy)
    ctx.set_form("auto")
    dem = torch.from_numpy(w.demand).cuda()
    eager, est = ctx.eval(w.tour, dem, w.Q)
    exp = eager.cpu().numpy()
    cost = torch.empty(w.S, dtype=torch.int32, device="cuda")
    g = ctx.graph(1, len(w.tour), dem, w.Q, cost=cost.view(1, -1))
    for rep in range(3):
        cost.fill_(-1)
        print(f"[graph] copula-n1000 S={w.S} replay {rep}", flush=True)
        got = g.launch([w.tour])
        gstats, gstatus = g.stats()
        torch.cuda.synchronize()
        assert np.array_equal(got[0].cpu().numpy(), exp), f"replay {rep}"
        assert gstatus == [0]
        assert (gstats[0].sum, gstats[0].var) == (est.sum, est.var)
        # eager work between replays, on the same stream
        ctx.eval(w.tour[:500], dem, w.Q)
    g.close()
    idx = np.arange(0, w.S, 97)
    sub = np.ascontiguousarray(w.demand[:, idx])
    d = oracle.dist_matrix(w.xy)
    assert np.array_equal(exp[idx], oracle.split(w.tour, d, sub, w.Q, threads=ORACLE_THREADS))
    assert est.sum == int(exp.astype(np.int64).sum())
    ctx.close()



@pytest.mark.parametrize("block", [16, 8])
def test_fixed_stride_grid_with_ragged_items(sg, block):
    # One tour over more work items than the default one-tour grid of 8 workgroups per compute
    # unit: 150,001 scenarios are 2344 items (the last holds one scenario), so the first
    # workgroups take a second item at the fixed stride and the others one. Eager calls, a
    # captured graph and the allocation-free call all against the oracle on every scenario.
    w = gen.make_workload("copula-n1000", S=150_001, threads=ORACLE_THREADS)
    tour = np.ascontiguousarray(w.tour[:300])
    ctx = fresh_ctx(sg, w.xy)
    ctx.set_tuning(sg.SplitTuning(sg.FORM_LANE, lane_block=block))
    dem = torch.from_numpy(w.demand).cuda()
    want = oracle.split(tour, oracle.dist_matrix(w.xy), w.demand, w.Q, threads=ORACLE_THREADS)
    print(f"[stride] lane_block {block}: n=300 S={w.S}", flush=True)
    eager, est = ctx.eval(tour, dem, w.Q)
    assert np.array_equal(eager.cpu().numpy(), want)
    assert est.sum == int(want.astype(np.int64).sum())
    g = ctx.graph(1, len(tour), dem, w.Q)
    for rep in range(2):
        got = g.launch([tour])
        torch.cuda.synchronize()
        assert np.array_equal(got[0].cpu().numpy(), want), f"replay {rep}"
        ctx.eval(tour[:100], dem, w.Q)  # eager work between replays
    g.close()
    cost = torch.full((w.S,), -1, dtype=torch.int32, device="cuda")
    st = ctx.eval_noalloc(tour, dem, w.Q, cost)
    assert np.array_equal(cost.cpu().numpy(), want)
    assert (st.sum, st.var) == (est.sum, est.var)
    ctx.close()
