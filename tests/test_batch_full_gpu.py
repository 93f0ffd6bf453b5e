"""The batched workload at its full size and in its timed launch configuration.

256 candidate tours of uneven length (n ~ U[100, 1000]) over one 1000-customer instance, against
S = 65,536 copula scenarios, evaluated by the scenario-per-lane kernel with 8 persistent
workgroups per compute unit taking (tour, 64-scenario) work items from a queue, and replayed
from a captured graph (the configuration the batch benchmark times). Every cost row is compared
with an eager evaluation, with the wavefront-per-scenario kernel (an independent kernel form
over all 65,536 scenarios of every tour) and with the CPU oracle on a sample of scenarios of
every tour; the moments are compared with the oracle's on the sample's rows and with the eager
evaluation's over all rows.
"""
import os

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))
SAMPLE = 4096  # scenarios per tour checked against the oracle


@pytest.fixture(scope="module")
def sg():
    import paper_2511_18022_amd as sg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return sg


def test_full_batch_persistent_queue_graph_replay(sg):
    b = gen.make_batch_workload("batch-256", threads=ORACLE_THREADS)
    T, S = len(b.tours), b.S
    assert T == 256 and S == 65536
    print(f"[batch-full] T={T} S={S} n in [{min(map(len, b.tours))}, "
          f"{max(map(len, b.tours))}]", flush=True)
    ctx = sg.SplitContext(0)
    ctx.set_coords(b.xy)
    dem = torch.from_numpy(b.demand).cuda()
    tuned = sg.SplitTuning(sg.FORM_LANE, 8, 0, 0)
    # 8 workgroups per CU take 2048 items first; the other items go through the queue
    assert T * ((S + 63) // 64) > 8 * torch.cuda.get_device_properties(0).multi_processor_count

    # eager evaluation under the timed choice
    ctx.set_tuning(tuned)
    eager, stats_e, status_e = ctx.eval_batch(b.tours, dem, b.Q)
    eager = eager.cpu().numpy()
    assert status_e == [0] * T
    assert sum(s.n_fallback for s in stats_e) == 0

    # graph replays (three, with eager work between them), each equal to the eager rows
    cost = torch.full((T, S), -1, dtype=torch.int32, device="cuda")
    g = ctx.graph(T, sum(len(t) for t in b.tours), dem, b.Q, cost=cost)
    for rep in range(3):
        print(f"[batch-full] graph replay {rep}", flush=True)
        cost.fill_(-1)
        g.launch(b.tours)
        gstats, gstatus = g.stats()
        assert gstatus == [0] * T
        assert np.array_equal(cost.cpu().numpy(), eager), f"replay {rep} differs from eager"
        for t in range(T):
            assert (gstats[t].sum, gstats[t].sumsq, gstats[t].mean, gstats[t].var) == (
                stats_e[t].sum, stats_e[t].sumsq, stats_e[t].mean, stats_e[t].var)
        ctx.eval_batch(b.tours[:3], dem, b.Q)  # unrelated eager work between replays
    g.close()

    # the other kernel form over every scenario of every tour
    print("[batch-full] wave form, all rows", flush=True)
    ctx.set_tuning(sg.SplitTuning(sg.FORM_WAVE, 0, 0, 0))
    wave, stats_w, _ = ctx.eval_batch(b.tours, dem, b.Q)
    wave = wave.cpu().numpy()
    bad = np.nonzero((wave != eager).any(axis=1))[0]
    assert bad.size == 0, f"lane and wave forms differ on tours {bad[:8]}"
    assert [s.sum for s in stats_w] == [s.sum for s in stats_e]

    # the oracle on a sample of scenarios of every tour; moments over the whole row from the
    # exact integers of the (now cross-checked) row
    rng = np.random.default_rng(256)
    d = oracle.dist_matrix(b.xy)
    for t, tour in enumerate(b.tours):
        idx = np.sort(rng.choice(S, size=SAMPLE, replace=False))
        sub = np.ascontiguousarray(b.demand[:, idx])
        want = oracle.split(np.asarray(tour, dtype=np.int32), d, sub, b.Q,
                            threads=ORACLE_THREADS)
        mism = np.nonzero(eager[t, idx] != want)[0]
        assert mism.size == 0, (f"tour {t} (n={len(tour)}): {mism.size} of {SAMPLE} sampled "
                                f"scenarios differ from the oracle, first {idx[mism[:5]]}")
        mom = oracle.moments(eager[t])
        assert (stats_e[t].sum, stats_e[t].sumsq, stats_e[t].mean, stats_e[t].var) == (
            mom["sum"], mom["sumsq"], mom["mean"], mom["var"])
    ctx.close()


def test_queue_path_at_the_timed_choice(sg):
    # a small batch with more work items than 8 workgroups per CU: the queue hands out the rest;
    # every scenario of every tour against the oracle
    b = gen.make_batch_workload("batch-256", T=5, S=40000, threads=ORACLE_THREADS)
    items = len(b.tours) * ((b.S + 63) // 64)
    grid = 8 * torch.cuda.get_device_properties(0).multi_processor_count
    assert items > grid
    print(f"[batch-queue] T=5 S=40000 items={items} grid={grid}", flush=True)
    ctx = sg.SplitContext(0)
    ctx.set_coords(b.xy)
    ctx.set_tuning(sg.SplitTuning(sg.FORM_LANE, 8, 0, 0))
    dem = torch.from_numpy(b.demand).cuda()
    cost, stats, status = ctx.eval_batch(b.tours, dem, b.Q)
    got = cost.cpu().numpy()
    d = oracle.dist_matrix(b.xy)
    for t, tour in enumerate(b.tours):
        want = oracle.split(np.asarray(tour, dtype=np.int32), d, b.demand, b.Q,
                            threads=ORACLE_THREADS)
        assert np.array_equal(got[t], want), f"tour {t}"
        mom = oracle.moments(want)
        assert (stats[t].sum, stats[t].sumsq, stats[t].mean, stats[t].var) == (
            mom["sum"], mom["sumsq"], mom["mean"], mom["var"])
    assert status == [0] * len(b.tours)
    ctx.close()
