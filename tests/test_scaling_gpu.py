"""Runtime against the number of scenarios (Section 4.1, the scenario-scaling experiment) on one
GPU: once the grid fills the chip for more than one round (2^17 scenarios = 2048 work items of
64 scenarios = two wavefronts on every SIMD), the lane kernel's time grows linearly in S. Checked
on the n = 1000 copula workload at S = 2^16 .. 2^20 (column slices of one scenario matrix):

- the marginal time per scenario of the doublings from 2^18 agree within 15%;
- the time per scenario at 2^19 and 2^20 agrees within 15% (the fixed cost per launch is small
  there);
- every timed launch gives the costs of the others (the slices share their first columns).
"""
import numpy as np
import pytest

import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_kernel_time_is_linear_in_the_scenarios_once_the_chip_is_full():
    import paper_2511_18022_amd as sg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    w = gen.make_workload("copula-n1000", threads=16)
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    ctx.set_form("lane")
    dem = torch.from_numpy(w.demand).cuda()
    sizes = [1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20]
    times, ref = {}, None
    for S in sizes:
        sl = dem[:, :S]
        for _ in range(30):  # clocks settle, caches warm
            ctx.eval(w.tour, sl, w.Q, sync=False)
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_reset()
        for _ in range(15):
            cost, _ = ctx.eval(w.tour, sl, w.Q, sync=False)
        torch.cuda.synchronize()
        samples = ctx.timing_samples()
        ctx.timing(False)
        times[S] = float(np.median(samples))
        got = cost[:S].cpu().numpy()
        if ref is not None:
            assert np.array_equal(got[:ref.size], ref)
        ref = got
        print(f"[scaling] S={S}: kernel median {times[S]:.4f} ms, "
              f"{times[S] * 1e6 / S:.3f} ns per scenario", flush=True)
    slopes = [(times[b] - times[a]) / (b - a) for a, b in zip(sizes[2:], sizes[3:])]
    print(f"[scaling] marginal ns per scenario per doubling from 2^18: "
          f"{[round(s * 1e6, 3) for s in slopes]}", flush=True)
    for s in slopes:
        assert abs(s / slopes[-1] - 1.0) <= 0.15
    per19, per20 = times[1 << 19] / (1 << 19), times[1 << 20] / (1 << 20)
    assert abs(per19 / per20 - 1.0) <= 0.15
    ctx.close()
