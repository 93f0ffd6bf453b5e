#!/usr/bin/env python3
"""Benchmark of the scenario-batched Split.

Default: one giant tour, n = 1000 customers, S = 2^20 copula scenarios (copula-n1000). One step
is one full evaluation (split_eval): the per-tour prep kernel, the Split DP of every scenario,
the exact moments and their copy to the host.

--workload batch-256: 256 candidate tours of uneven length (n uniform in [100, 1000]) over one
1000-customer instance x S = 65,536 copula scenarios. One step is one split_eval_batch of all
256 tours (one persistent lane-kernel launch); one scenario-eval is one (tour, scenario) pair.

Demands are generated on the host (seeded, gen/) and uploaded once; they are resident in HBM
before the timed region starts. Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Split scenario-evals/s at n=1000,S=2^20 (% roofline)"
METRIC_BATCH = "Split scenario-evals/s, 256 tours n~U[100,1000] x S=65536 (% roofline)"
METRIC_SCREEN = "screened tours/s at regret (1000 customers, S=65536, top 1% re-evaluated)"
MFMA_BF16_PEAK_TFLOPS = 2500.0
METRIC_SEARCH = "expected cost after a timed local search (1000 customers, 10^4 in-sample scenarios)"
HBM_PEAK_GBS = 8000.0
SETTLE_S = 0.5  # untimed sustained work before the warm-up steps (clock ramp)
# INT32 VALU lane-ops: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
KERNEL_SRC = os.path.join(ROOT, "paper_2511_18022_amd", "csrc", "split_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")
COPULA_DESC = ("int16 [N][S]; Gaussian copula, AR(1) 0.6 along customer id, lognormal mean 20 "
               "CV 0.5")


def metric_name(workload: str, batch: bool, T: int, S: int, sum_n: int) -> str:
    """The headline metric's name for the recipes it is quoted on; otherwise one that names the
    workload that was run."""
    if not batch and workload == "copula-n1000" and S == 1 << 20:
        return METRIC
    if batch and workload == "batch-256" and T == 256 and S == 65536:
        return METRIC_BATCH
    if batch:
        return f"Split scenario-evals/s, {workload} ({T} tours, {sum_n} positions, S={S})"
    return f"Split scenario-evals/s, {workload} (n={sum_n}, S={S})"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


LANE_BEGIN = b"// ------------------------------------------------------------------------- lane kernel"
LANE_END = b"// ------------------------------------------------------------------------- wave kernel"
INTERNAL_H = os.path.join(ROOT, "paper_2511_18022_amd", "csrc", "split_internal.h")


def kernel_source_sha() -> str:
    """Hash of the lane kernel's source: its section of the kernel file and the shared internal
    header (other kernels in the file do not change it)."""
    with open(KERNEL_SRC, "rb") as fh:
        src = fh.read()
    i, j = src.index(LANE_BEGIN), src.index(LANE_END)
    with open(INTERNAL_H, "rb") as fh:
        hdr = fh.read()
    return hashlib.sha256(src[i:j] + hdr).hexdigest()[:16]


NN_SRC = os.path.join(ROOT, "paper_2511_18022_amd", "csrc", "nn_kernels.hip")
NN_H = os.path.join(ROOT, "paper_2511_18022_amd", "csrc", "nn_internal.h")


NN_MARK = b"// " + b"-" * 73 + b" "


def nn_source_sha() -> str:
    """Hash of the fused prediction kernel's source: its section of the surrogate's kernel file,
    the section that packs its fragment-ordered weights, and the internal header."""
    with open(NN_SRC, "rb") as fh:
        src = fh.read()
    h = hashlib.sha256()
    for name in (b"fused inference", b"Adam and weights"):
        i = src.index(NN_MARK + name)
        j = src.index(NN_MARK, i + len(NN_MARK))
        h.update(src[i:j])
    with open(NN_H, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_nn_traffic(n: int):
    """HBM bytes per predicted tour of the fused prediction kernel from committed rocprofv3
    counter runs, if they match this source and tour length."""
    try:
        with open(os.path.join(PROFILES, "traffic_nn_fwd_fused_kernel_screen.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != nn_source_sha() or t.get("n") != n:
        return None
    return t.get("bytes_per_tour")


def measured_traffic(workload: str, launch_scenarios: int):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they match this source."""
    path = os.path.join(PROFILES, f"traffic_split_lane_kernel_{workload}.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha() or t.get("S") != launch_scenarios:
        return None
    return t.get("bytes_per_launch")


def window_work(dem, tours, Q: int, chunk: int = 16384) -> int:
    """M = sum over tours, scenarios and states i of (w_i - 1), w_i the size of state i's
    capacity window (Eq. (2)): the two-input minima a plain Eq. (3) scan performs. It sizes the
    ALU roofline only (algorithmic ops = M/2 + 4n per scenario-eval: v_min3 retires two minima,
    and each state needs a prefix-load add, a window compare and the two DP adds). `dem` is an
    int16 torch tensor [N, ld] with non-negative demands; any device."""
    import torch
    total = 0
    S = dem.shape[1]
    for tour in tours:
        idx = torch.as_tensor(tour, dtype=torch.long, device=dem.device) - 1
        n = idx.numel()
        ii = torch.arange(n + 1, device=dem.device, dtype=torch.int64)
        for s0 in range(0, S, chunk):
            q = dem[idx, s0:s0 + chunk].to(torch.int32).t()  # [c, n]
            P = torch.zeros((q.shape[0], n + 1), dtype=torch.int32, device=dem.device)
            P[:, 1:] = torch.cumsum(q, 1, dtype=torch.int32)
            # window start: first p with P_p >= P_i - Q (P is non-decreasing)
            start = torch.searchsorted(P, P - Q, side="left")
            total += int((ii[1:] - start[:, 1:] - 1).sum())
    return total


def host_cpu() -> dict:
    """The host the CPU baselines ran on: CPU model (from /proc/cpuinfo) and logical CPUs."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(tours, d, demand, Q, S, threads: int, got_cost, target_cpu_s: float = 20.0):
    """The oracle as it stands, on the host cores, over a bounded sample of the scenarios (the
    first `sample` scenarios of every tour, about target_cpu_s of single-core work). Its output
    on the sample is also compared with the GPU's costs of the timed run."""
    import numpy as np
    import oracle
    probe = 256
    dem = np.ascontiguousarray(demand[:, :probe])
    t0 = time.perf_counter()
    for t in tours:
        oracle.split(t, d, dem, Q, threads=1)
    per_scen = (time.perf_counter() - t0) / (probe * len(tours))
    sample = int(min(S, max(probe, target_cpu_s / len(tours) / max(per_scen, 1e-9))))
    sample -= sample % 64
    dem = np.ascontiguousarray(demand[:, :sample])
    parity = True
    t0 = time.perf_counter()
    outs = [oracle.split(t, d, dem, Q, threads=threads) for t in tours]
    el = time.perf_counter() - t0
    for k, want in enumerate(outs):
        parity &= bool(np.array_equal(got_cost[k][:sample], want))
    evals = sample * len(tours)
    what = "the tour" if len(tours) == 1 else f"each of the {len(tours)} tours"
    # the same oracle on one thread (the paper's single-threaded CPU comparison), over a
    # quarter of the sample: about target_cpu_s / 4 of work
    sample1 = max(64, (sample // 4) - (sample // 4) % 64)
    dem1 = np.ascontiguousarray(demand[:, :sample1])
    t0 = time.perf_counter()
    for t in tours:
        oracle.split(t, d, dem1, Q, threads=1)
    el1 = time.perf_counter() - t0
    # the strong CPU baseline: the linear-time Split (monotone deque) on the same sample and
    # threads, its costs also compared with the GPU's
    t0 = time.perf_counter()
    outs_d = [oracle.split_deque(t, d, dem, Q, threads=threads) for t in tours]
    eld = time.perf_counter() - t0
    parity_d = all(bool(np.array_equal(got_cost[k][:sample], o)) for k, o in enumerate(outs_d))
    return {"value": evals / el, "unit": "scenario-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} of {S} scenarios of {what}, {threads} threads, "
                      f"{el:.2f} s wall",
            "parity_vs_gpu_on_sample": parity,
            "single_thread": {"value": sample1 * len(tours) / el1, "unit": "scenario-evals/s",
                              "sample": f"first {sample1} scenarios of {what}, 1 thread, "
                                        f"{el1:.2f} s"},
            "strong": {"value": evals / eld, "unit": "scenario-evals/s", "cores": threads,
                       "kind": "linear-time Split (monotone deque, Vidal 2016), C, threads over "
                               "scenario ranges",
                       "sample": f"the same {sample} scenarios, {eld:.2f} s wall",
                       "parity_vs_gpu_on_sample": parity_d},
            "host": host_cpu()}


def calibrate_copy(nbytes: int = 2 << 30, reps: int = 3):
    """A plain copy kernel of known size: reads nbytes and writes nbytes per launch. Profiling
    it with the same hardware counters gives the scale between counter readings and bytes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(7)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
                      "ms_per_copy": el * 1e3, "GBps_read_plus_write": 2 * nbytes / el / 1e9}))


def timed_steps(ctx, step, wait, steps: int, warmup: int, settle_s: float = SETTLE_S):
    """Warm-up steps, then `steps` timed steps between device synchronizations, with the
    dominant kernel of eager evaluations timed by HIP events on their stream. Returns
    (ms per step, dominant-kernel average ms, kernel name, timed launches, median ms)."""
    import torch
    # the GPU's clocks ramp over the first few hundred milliseconds of sustained work: untimed
    # evaluations for at least settle_s seconds come before the warm-up steps
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < settle_s:
        for _ in range(10):
            step()
        wait()
        torch.cuda.synchronize()
    for _ in range(warmup):
        step()
    wait()
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    wait()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern_ms, launches, kname = ctx.timing_get()
    samples = ctx.timing_samples()
    ctx.timing(False)
    median = float(sorted(samples)[len(samples) // 2]) if len(samples) else None
    return el * 1e3 / steps, kern_ms / max(launches, 1), kname, launches, median


def exact_means(ctx, tours, dem, Q, chunk: int = 256):
    """Exact expected cost (mean over the scenarios) of every tour, chunk tours per batch."""
    import numpy as np
    out = np.empty(len(tours))
    t0 = last = time.perf_counter()
    for k0 in range(0, len(tours), chunk):
        if time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            log(f"exact evaluation: {k0} of {len(tours)} tours, {last - t0:.0f}s")
        _, stats, status = ctx.eval_batch(tours[k0:k0 + chunk], dem, Q)
        assert all(x == 0 for x in status)
        out[k0:k0 + len(stats)] = [st.mean for st in stats]
    return out


def run_screen(args, threads):
    """Surrogate screening against exact-only search on the same candidates."""
    import numpy as np
    import torch

    import gen
    import paper_2511_18022_amd as sg
    t0 = time.perf_counter()
    w = gen.make_screen_workload("screen", train=args.train, candidates=args.candidates,
                                 threads=threads)
    C, ntrain = len(w.cands), len(w.train)
    log(f"generated screen: N={w.N} S={w.S} Q={w.Q}, {ntrain} training tours, {C} candidates, "
        f"keep {w.keep} ({time.perf_counter() - t0:.1f}s)")
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    tr = torch.from_numpy(w.train).cuda()
    ca = torch.from_numpy(w.cands).cuda()
    tu, tune_ms, _ = ctx.autotune(list(w.cands[:256]), dem, w.Q, reps=2)
    log(f"autotune on 256 candidates: {tu} {tune_ms:.3f} ms")
    # labels: exact expected costs of the training tours from the GPU Split
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    labels = exact_means(ctx, w.train, dem, w.Q)
    label_s = time.perf_counter() - t0
    log(f"labelled {ntrain} tours in {label_s:.2f}s; mean {labels.mean():.1f} std {labels.std():.1f}")
    net = sg.SplitNN(ctx, seed=1, length_scale=1000.0)
    net.set_scenarios(dem, w.Q)
    net.set_norm(float(labels.mean()), float(labels.std()))
    lab = torch.from_numpy(labels.astype(np.float32)).cuda()
    steps = args.epochs * (ntrain // args.batch)
    t0 = time.perf_counter()
    loss = net.train(tr, lab, batch=args.batch, steps=steps, lr=args.lr, seed=3)
    train_s = time.perf_counter() - t0
    log(f"trained {steps} steps (batch {args.batch}) in {train_s:.2f}s, mean loss {loss:.4f}")
    # MFMA work of one training step, per tour of n positions (8 input features, 128 channels,
    # 5 taps): forward 2n*128*(5*8 + 3*5*128), data gradients of layers 2-4 2n*128*(3*5*128),
    # weight gradients 2n*128*(5*8 + 3*5*128)
    n_tr = int(w.train.shape[1])
    train_flops_step = 2.0 * n_tr * 128 * (2 * (5 * 8 + 3 * 5 * 128) + 3 * 5 * 128) * args.batch
    train_tflops = train_flops_step * steps / train_s / 1e12
    # screening, timed: predict every candidate, keep the top 1%, evaluate those exactly
    res = net.screen(ca[:min(C, 4096)], max(1, min(C, 4096) // 100), dem, w.Q)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = net.screen(ca, w.keep, dem, w.Q)
    torch.cuda.synchronize()
    screen_s = time.perf_counter() - t0
    # forward pass alone (HIP events on its stream): the conv layers' MFMA rate
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    net.timing(True)
    net.timing_reset()
    e0.record()
    net.predict(ca, out=res["pred"])
    e1.record()
    torch.cuda.synchronize()
    predict_ms = e0.elapsed_time(e1)
    fused_ms, fused_launches = net.timing_get()
    net.timing(False)
    # exact-only, timed
    t0 = time.perf_counter()
    means = exact_means(ctx, w.cands, dem, w.Q)
    exact_s = time.perf_counter() - t0
    best = int(np.argmin(means))
    regret = (res["best_mean"] - means[best]) / means[best]
    pred = res["pred"].cpu().numpy()
    rank_corr = float(np.corrcoef(np.argsort(np.argsort(pred)), np.argsort(np.argsort(means)))[0, 1])
    rank_of_best = int((pred < pred[best]).sum())
    log(f"screen {screen_s:.3f}s ({C / screen_s:.0f} tours/s), exact-only {exact_s:.3f}s "
        f"({C / exact_s:.0f} tours/s), regret {regret:.5f}, best exact mean {means[best]:.2f} at "
        f"predicted rank {rank_of_best}, Spearman {rank_corr:.4f}")
    n = w.N
    flops_per_tour = 2.0 * n * 128 * (5 * 8 + 3 * 5 * 128)
    # the dominant kernel: the fused convolution kernel, HIP-event timed per launch; a launch
    # is one forward pass of up to 1024 tours
    per_launch = C / fused_launches
    # HBM bytes per launch from the committed counter runs (same source and tour length)
    traffic_per_tour = measured_nn_traffic(int(ca.shape[1]))
    achieved = flops_per_tour * per_launch / (fused_ms / fused_launches * 1e-3) / 1e12
    out = {
        "metric": METRIC_SCREEN,
        "value": C / screen_s,
        "unit": "tours/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": screen_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (surrogate), int32 (exact Split)",
        "data": "synthetic",
        "regret": regret,
        "regret_target": 0.005,
        "exact_only": {"tours_per_s": C / exact_s, "seconds": exact_s, "best_mean": means[best]},
        "train_roofline": {"bound": "mfma", "achieved": train_tflops,
                           "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": train_tflops / MFMA_BF16_PEAK_TFLOPS,
                           "flops_per_step": train_flops_step, "steps": steps,
                           "ms_per_step": train_s * 1e3 / steps,
                           "what": "whole training steps by wall time (features, conv forward, "
                                   "data and weight gradients, head, Adam); per-kernel times "
                                   "in the committed rocprofv3 summary"},
        "speedup_vs_exact_only": exact_s / screen_s,
        "config": {"workload": "screen", "N": n, "S": w.S, "Q": w.Q, "candidates": C,
                   "keep": w.keep, "train_tours": ntrain, "train_steps": steps,
                   "batch": args.batch, "lr": args.lr, "train_seconds": train_s,
                   "label_seconds": label_s, "final_mean_loss": loss,
                   "best_screened_mean": res["best_mean"], "spearman_pred_vs_exact": rank_corr,
                   "predicted_rank_of_exact_best": rank_of_best,
                   "candidates_recipe": "2-opt base tour with 1..60 random segment reversals"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFLOPS,
                     "traffic": (None if traffic_per_tour is None
                                 else traffic_per_tour * per_launch),
                     "kernel": "nn_fwd_fused_kernel",
                     "kernel_avg_ms": fused_ms / fused_launches, "launches": fused_launches,
                     "tours_per_launch": per_launch, "flops_per_tour": flops_per_tour,
                     "predict_ms_all_kernels": predict_ms},
    }
    if not args.no_cpu_baseline:
        import oracle
        d = oracle.dist_matrix(w.xy)
        k = 0
        t0 = time.perf_counter()
        ok = True
        while time.perf_counter() - t0 < 15.0 and k < C:
            m = oracle.moments(oracle.split(w.cands[k], d, w.demand, w.Q, threads=threads))["mean"]
            ok &= m == means[k]
            k += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": k / el, "unit": "tours/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"exact evaluation of the first {k} candidates at "
                                         f"S={w.S}, {threads} threads, {el:.1f} s wall",
                               "parity_vs_gpu_on_sample": bool(ok), "host": host_cpu()}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    net.close()
    ctx.close()


def run_search(args, threads):
    """Exact-only and surrogate-assisted local search under the same wall-clock budget, then an
    out-of-sample evaluation of the start and the two results on held-out scenarios."""
    import numpy as np
    import torch

    import gen
    import paper_2511_18022_amd as sg
    S_in, S_out = args.search_scenarios, args.holdout_scenarios
    w = gen.make_screen_workload("screen", train=args.train, candidates=1, S=S_in, threads=threads)
    law = gen.SCREEN_RECIPES["screen"]["law"]
    t0 = time.perf_counter()
    held = gen.demand_copula(w.seed + 1000, w.N, S_out, law[1], law[2], law[3], w.Q,
                             threads=threads)
    log(f"search: N={w.N}, {S_in} in-sample scenarios, {S_out} held-out (generated in "
        f"{time.perf_counter() - t0:.1f}s), budget {args.budget}s per search")
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    base = w.base
    tu, _, _ = ctx.autotune([base] * args.search_batch, dem, w.Q, reps=2)
    log(f"autotune: {tu}")
    exact = sg.search(ctx, base, dem, w.Q, batch=args.search_batch, budget_s=args.budget,
                      seed=21)
    log(f"exact-only search: {exact['iterations']} iterations, {exact['evaluated']} exact "
        f"evaluations, {exact['start_mean']:.2f} -> {exact['best_mean']:.2f}")
    # surrogate trained on the in-sample scenarios
    tr = torch.from_numpy(w.train).cuda()
    t0 = time.perf_counter()
    labels = exact_means(ctx, w.train, dem, w.Q)
    nn = sg.SplitNN(ctx, seed=1, length_scale=1000.0)
    nn.set_scenarios(dem, w.Q)
    nn.set_norm(float(labels.mean()), float(labels.std()))
    steps = args.epochs * (len(w.train) // args.batch)
    nn.train(tr, torch.from_numpy(labels.astype(np.float32)).cuda(), batch=args.batch,
             steps=steps, lr=args.lr, seed=3)
    prep_s = time.perf_counter() - t0
    log(f"surrogate: labels and {steps} training steps in {prep_s:.1f}s")
    assisted = sg.search(ctx, base, dem, w.Q, batch=args.search_batch, pool=args.search_pool,
                         nn=nn, budget_s=args.budget, seed=21)
    log(f"surrogate search: {assisted['iterations']} iterations, {assisted['predicted']} "
        f"predicted, {assisted['evaluated']} exact, {assisted['start_mean']:.2f} -> "
        f"{assisted['best_mean']:.2f}")
    hdem = torch.from_numpy(held).cuda()
    oos, saa = {}, {}
    for name, t in (("start", base), ("exact_only", exact["best_tour"]),
                    ("surrogate", assisted["best_tour"])):
        _, st = ctx.eval(t, hdem, w.Q)
        _, st_in = ctx.eval(t, dem, w.Q)
        oos[name] = st.mean
        # sample-average check (the appendix's rate of convergence): in-sample and held-out
        # means of one tour differ by N(0, var_in / S_in + var_out / S_out) when the tour was
        # not chosen on the in-sample scenarios; a searched tour's in-sample mean is optimistic
        se = float(np.sqrt(st_in.var / S_in + st.var / S_out))
        saa[name] = {"in_sample": st_in.mean, "held_out": st.mean, "se": se,
                     "gap_in_se": (st_in.mean - st.mean) / se}
    saa["start_within_4se"] = abs(saa["start"]["gap_in_se"]) <= 4.0
    log(f"out-of-sample means: {oos}; start tour in-sample minus held-out = "
        f"{saa['start']['gap_in_se']:.2f} standard errors")

    def summary(r):
        return {k: r[k] for k in ("iterations", "evaluated", "predicted", "improvements",
                                  "start_mean", "best_mean", "seconds")}
    out = {
        "metric": METRIC_SEARCH,
        "value": assisted["best_mean"],
        "unit": "expected cost (in-sample mean)",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": assisted["seconds"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 (exact Split), bf16 (surrogate)",
        "data": "synthetic",
        "exact_only": summary(exact),
        "surrogate": summary(assisted),
        "out_of_sample": {"scenarios": S_out, **oos},
        "saa_check": saa,
        "config": {"workload": "search", "N": w.N, "S": S_in, "Q": w.Q, "budget_s": args.budget,
                   "batch": args.search_batch, "pool": args.search_pool,
                   "surrogate_prep_seconds": prep_s, "train_tours": len(w.train),
                   "start": "nearest neighbour + 2-opt tour (straight-line distances)",
                   "moves": "2-opt or relocate, uniform positions"},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    nn.close()
    ctx.close()


SCALING_S = (10_000, 65_536, 100_000, 131_072, 262_144, 524_288, 1_000_000, 1 << 20)


def run_scaling(args, threads):
    """Runtime against the number of scenarios for one giant tour (n = 1000, copula demands):
    the paper's first experiment (Section 4.1, Fig. 3) on one GPU, with the CPU oracle on one
    thread and on every host core and the linear-time CPU Split beside every point. The
    scenario sets are the first S columns of the 2^20-scenario matrix (the generator is keyed by
    scenario), each launch reading a column slice of the resident matrix."""
    import numpy as np
    import torch

    import gen
    import oracle
    import paper_2511_18022_amd as sg
    Smax = max(SCALING_S)
    t0 = time.perf_counter()
    w = gen.make_workload("copula-n1000", S=Smax, threads=threads)
    log(f"generated copula-n1000 at S={Smax} in {time.perf_counter() - t0:.1f}s")
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    d = oracle.dist_matrix(w.xy)
    cost = torch.empty(Smax, dtype=torch.int32, device="cuda")
    points = []
    for S in SCALING_S:
        sl = dem[:, :S]

        def step():
            ctx.eval(w.tour, sl, w.Q, cost=cost, sync=False)
        ms, kern_ms, kname, launches, kern_med = timed_steps(ctx, step, ctx.batch_stats,
                                                             args.steps, args.warmup,
                                                             args.settle)
        stats, _ = ctx.batch_stats()
        M = window_work(sl, [w.tour], w.Q)
        ops = M / 2 + 4 * w.n * S
        alu = ops / (kern_ms * 1e-3) / 1e12
        hbm = (2 * w.n + 4) * S / (kern_ms * 1e-3) / 1e9
        pt = {"S": S, "kernel": kname, "kernel_ms": kern_ms, "kernel_median_ms": kern_med,
              "ms_per_step": ms, "evals_per_s": S / (ms * 1e-3),
              "kernel_ns_per_scenario": kern_ms * 1e6 / S,
              "alu_frac": alu / ALU_PEAK_TOPS, "hbm_frac": hbm / HBM_PEAK_GBS,
              "fallback_scenarios": stats[0].n_fallback}
        # CPU baselines on the same columns (layout [N][S]: the oracle strides over the whole
        # S-wide rows as the GPU does): time a bounded prefix of scenarios, report evals/s and
        # the time the whole set takes at that rate
        got = cost[:S].cpu().numpy()
        sub = np.ascontiguousarray(w.demand[:, :S])
        for key, fn, thr, budget in (("cpu_1t", oracle.split, 1, 2.0),
                                     ("cpu_mt", oracle.split, threads, 2.0),
                                     ("cpu_deque_mt", oracle.split_deque, threads, 1.0)):
            k = min(S, 1024)
            while True:
                t1 = time.perf_counter()
                out = fn(w.tour, d, sub, w.Q, S=k, threads=thr)
                el = time.perf_counter() - t1
                if el >= budget / 4 or k == S:
                    break
                k = min(S, k * 4)
            assert np.array_equal(out, got[:k]), f"{key}: CPU and GPU costs differ at S={S}"
            rate = k / el
            pt[key] = {"evals_per_s": rate, "scenarios_timed": k, "threads": thr,
                       "seconds_for_S": S / rate}
        pt["speedup_vs_cpu_1t"] = pt["evals_per_s"] / pt["cpu_1t"]["evals_per_s"]
        pt["speedup_vs_cpu_mt"] = pt["evals_per_s"] / pt["cpu_mt"]["evals_per_s"]
        pt["speedup_vs_cpu_deque_mt"] = pt["evals_per_s"] / pt["cpu_deque_mt"]["evals_per_s"]
        log(f"S={S}: kernel {kern_ms:.4f} ms ({pt['kernel_ns_per_scenario']:.3f} ns/scenario), "
            f"step {ms:.4f} ms, ALU {pt['alu_frac']:.3f}, x{pt['speedup_vs_cpu_1t']:.0f} vs 1T, "
            f"x{pt['speedup_vs_cpu_mt']:.0f} vs {threads}T")
        points.append(pt)
    big = points[-1]
    out = {
        "metric": "Split runtime against the number of scenarios (n=1000, copula demands)",
        "value": big["evals_per_s"],
        "unit": "scenario-evals/s at the largest S",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": big["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "scaling", "n": w.n, "Q": w.Q, "demand": COPULA_DESC,
                   "S": list(SCALING_S), "host": host_cpu(),
                   "paper_claim": "near-linear GPU time in the number of scenarios over 10^4-10^6 "
                                  "(NVIDIA RTX 2080 Ti; CPU baselines on an AMD Ryzen 7 9700X, "
                                  "1 and 8 threads)"},
        "points": points,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def run_crossover(args, threads):
    """Whole evaluations (prep, Split DP, moments, statistics copy) in both kernel forms for
    short tours over few scenarios: the first n positions of the n = 1000 copula tour, over its
    first S scenarios. The crossover sets the automatic form choice."""
    import numpy as np
    import torch

    import gen
    import paper_2511_18022_amd as sg
    w = gen.make_workload("copula-n1000", S=4096, threads=threads)
    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    dem = torch.from_numpy(w.demand).cuda()
    cost = torch.empty(w.S, dtype=torch.int32, device="cuda")

    def timed(tour, S, form):
        ctx.set_form(form)
        sl = dem[:, :S]
        for _ in range(10):
            ctx.eval(tour, sl, w.Q, cost=cost, sync=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            ctx.eval(tour, sl, w.Q, cost=cost, sync=False)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps * 1e3, cost[:S].cpu().numpy()

    for _ in range(200):  # clock ramp
        ctx.eval(w.tour, dem, w.Q, cost=cost, sync=False)
    torch.cuda.synchronize()
    points = []
    for S in (256, 1024, 4096):
        for n in (8, 16, 24, 32, 48, 64, 96, 128, 256):
            tour = np.ascontiguousarray(w.tour[:n])
            us_lane, c_lane = timed(tour, S, "lane")
            us_wave, c_wave = timed(tour, S, "wave")
            assert np.array_equal(c_lane, c_wave)
            points.append({"S": S, "n": n, "lane_us": us_lane, "wave_us": us_wave,
                           "faster": "wave" if us_wave < us_lane else "lane"})
            log(f"S={S} n={n}: lane {us_lane:.1f} us, wave {us_wave:.1f} us")
    print(json.dumps({"metric": "whole-evaluation time per kernel form (form crossover)",
                      "unit": "us", "steps": args.steps, "data": "synthetic",
                      "config": {"workload": "crossover", "instance": "copula-n1000"},
                      "points": points}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU's clocks need a few tens of milliseconds of work to settle
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--settle", type=float, default=SETTLE_S,
                    help="seconds of untimed evaluations before the warm-up steps (clock ramp)")
    ap.add_argument("--workload", default="copula-n1000")
    ap.add_argument("--form", default="auto", choices=["auto", "lane", "wave", "mask"])
    ap.add_argument("--tours", type=int, default=None, help="batch workloads: number of tours")
    ap.add_argument("--scenarios", type=int, default=None,
                    help="evaluate the workload's first S scenarios instead of all (a profiling "
                         "and form-comparison run; the headline uses the full recipe)")
    ap.add_argument("--launch", default="graph", choices=["eager", "graph"],
                    help="time eager calls or replays of a captured graph of the same "
                         "evaluation (the kernel's HIP-event duration always comes from eager "
                         "calls)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch workloads: keep the default launch choices")
    ap.add_argument("--tuning", default=None, metavar="PER_CU,ORDER",
                    help="lane form with these launch choices instead of autotuning")
    ap.add_argument("--lane-block", type=int, default=0, choices=[0, 8, 16],
                    help="lane form: states per block of the scenario-per-lane kernel (0: the "
                         "library default, 16; 8 suits windows shorter than about 24); batch "
                         "workloads take it with --tuning, else the autotuner chooses")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-alu-count", action="store_true",
                    help="skip counting the window work that sizes the ALU roofline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device-to-device copy of 2 GiB (HBM counter scale)")
    ap.add_argument("--candidates", type=int, default=1_000_000,
                    help="screen workload: candidate tours")
    ap.add_argument("--train", type=int, default=100_000, help="screen workload: training tours")
    ap.add_argument("--epochs", type=int, default=2, help="screen workload: training epochs")
    ap.add_argument("--batch", type=int, default=128, help="screen workload: training batch")
    ap.add_argument("--lr", type=float, default=1e-3, help="screen workload: Adam learning rate")
    ap.add_argument("--budget", type=float, default=10.0, help="search workload: seconds per search")
    ap.add_argument("--search-batch", type=int, default=256,
                    help="search workload: tours evaluated exactly per iteration")
    ap.add_argument("--search-pool", type=int, default=4096,
                    help="search workload: neighbours scored by the surrogate per iteration")
    ap.add_argument("--search-scenarios", type=int, default=10_000)
    ap.add_argument("--holdout-scenarios", type=int, default=1 << 20)
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported (a multi-GPU "
              "run would shard the scenarios and all-reduce 24 bytes of moments; it is not "
              "built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2511_18022_amd as sg

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    threads = max(1, min(16, os.cpu_count() or 1))
    if args.workload == "screen":
        run_screen(args, threads)
        return
    if args.workload == "search":
        run_search(args, threads)
        return
    if args.workload == "scaling":
        run_scaling(args, threads)
        return
    if args.workload == "crossover":
        run_crossover(args, threads)
        return
    batch = args.workload in gen.BATCH_RECIPES
    t0 = time.perf_counter()
    if batch:
        w = gen.make_batch_workload(args.workload, T=args.tours, S=args.scenarios,
                                    threads=threads)
        tours = w.tours
        lens = [len(t) for t in tours]
        log(f"generated {args.workload}: T={len(tours)} n in [{min(lens)}, {max(lens)}] "
            f"(sum {sum(lens)}) S={w.S} Q={w.Q} in {time.perf_counter() - t0:.1f}s")
    else:
        w = gen.make_workload(args.workload, S=args.scenarios, threads=threads)
        tours = [w.tour]
        log(f"generated {args.workload}: n={w.n} S={w.S} Q={w.Q} in "
            f"{time.perf_counter() - t0:.1f}s")
    T = len(tours)

    ctx = sg.SplitContext(0)
    ctx.set_coords(w.xy)
    ctx.set_tuning(sg.SplitTuning(lane_block=args.lane_block))
    ctx.set_form(args.form)
    t0 = time.perf_counter()
    dem = torch.from_numpy(w.demand).cuda()
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    log(f"uploaded {dem.numel() * 2 / 1e9:.3f} GB in {h2d_s:.3f}s")

    launch = args.launch
    tuning, tune_ms = None, None
    if batch:
        cost = torch.empty((T, w.S), dtype=torch.int32, device="cuda")
        if args.tuning:
            pc, order = (int(x) for x in args.tuning.split(","))
            ctx.set_tuning(sg.SplitTuning(sg.FORM_LANE, pc, order, 0, args.lane_block))
            tuning = {"form": sg.FORM_LANE, "lane_per_cu": pc, "order": order, "wave_grid": 0,
                      "lane_block": args.lane_block}
        elif not args.no_autotune:
            t0 = time.perf_counter()
            tu, tune_ms, _ = ctx.autotune(tours, dem, w.Q, reps=3)
            tuning = {"form": tu.form, "lane_per_cu": tu.lane_per_cu, "order": tu.order,
                      "wave_grid": tu.wave_grid, "lane_block": tu.lane_block}
            log(f"autotune: {tu} {tune_ms:.4f} ms per evaluation "
                f"({time.perf_counter() - t0:.1f}s)")

        def step():
            ctx.eval_batch(tours, dem, w.Q, cost=cost, sync=False)
    else:
        cost = torch.empty(w.S, dtype=torch.int32, device="cuda")

        def step():
            ctx.eval(w.tour, dem, w.Q, cost=cost, sync=False)

    # eager evaluations: the dominant kernel's duration for the roofline
    ms_eager, kern_avg_ms, kname, launches, kern_med_ms = timed_steps(
        ctx, step, ctx.batch_stats, args.steps, args.warmup, args.settle)
    stats, status = ctx.batch_stats()
    ms_step = ms_eager
    if launch == "graph":
        g = ctx.graph(T, sum(len(t) for t in tours), dem, w.Q,
                      cost=cost if batch else cost.view(1, -1))
        ms_step, _, _, _, _ = timed_steps(ctx, lambda: g.launch(tours), g.stats, args.steps,
                                          args.warmup, args.settle)
        gstats, gstatus = g.stats()
        assert [s.sum for s in gstats] == [s.sum for s in stats] and gstatus == status
        g.close()
        log(f"graph replays: {ms_step:.4f} ms/step (eager {ms_eager:.4f})")
    n_fallback = sum(s.n_fallback for s in stats)
    log(f"{args.steps} steps: {ms_step:.4f} ms/step, {kname} avg {kern_avg_ms:.4f} ms "
        f"({launches} launches), fallback scenarios {n_fallback}, bad tours "
        f"{sum(1 for x in status if x != 0)}")

    evals = T * w.S
    sum_n = sum(len(t) for t in tours)
    algo_bytes = (2 * sum_n + 4 * T) * w.S  # int16 demand column per tour + int32 cost
    alu = None
    if not args.no_alu_count:
        t0 = time.perf_counter()
        M = window_work(dem, tours, w.Q)
        ops = M / 2 + 4 * sum_n * w.S
        alu = {"bound": "alu", "window_work_M": M, "ops_per_launch": ops,
               "achieved": ops / (kern_avg_ms * 1e-3) / 1e12, "peak": ALU_PEAK_TOPS,
               "unit": "Tops/s (int32 lane-ops)"}
        alu["frac"] = alu["achieved"] / ALU_PEAK_TOPS
        log(f"window work M = {M} ({time.perf_counter() - t0:.1f}s); ALU view "
            f"{alu['achieved']:.2f} Tops/s = {alu['frac']:.3f} of peak")
    hbm_achieved = algo_bytes / (kern_avg_ms * 1e-3) / 1e9
    hbm = {"bound": "hbm", "achieved": hbm_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": hbm_achieved / HBM_PEAK_GBS}

    config = {"workload": w.name, "S": w.S, "Q": w.Q, "seed": w.seed, "demand": COPULA_DESC,
              "coords": "integer uniform 1000x1000, rounded Euclidean int32 costs",
              "kernel": kname, "form": args.form, "lane_block": ctx.tuning().lane_block or 16,
              "fallback_scenarios": n_fallback,
              "launch": launch, "eager_ms_per_step": ms_eager,
              "h2d_GBps": dem.numel() * 2 / h2d_s / 1e9}
    if tuning is not None:
        config["tuning"] = tuning
        config["autotune_ms"] = tune_ms
    if batch:
        config.update({"N": w.N, "tours": T, "n_min": min(len(t) for t in tours),
                       "n_max": max(len(t) for t in tours), "n_sum": sum_n})
        # the scenario matrix (131 MB) stays in the last-level cache across tours: the
        # binding floor is the VALU, and the HBM figure is what re-reading it would cost
        roof = dict(alu) if alu else None
        if roof is not None:
            roof["hbm_equivalent"] = hbm
            # bytes the kernel fetched from the memory fabric (HBM or the last-level cache)
            roof["traffic"] = measured_traffic(w.name, w.S)
    else:
        config["n"] = w.n
        # the binding roofline is the one with the larger floor: the algorithmic bytes at the
        # HBM peak, or the algorithmic int32 ops at the VALU peak
        t_hbm = algo_bytes / (HBM_PEAK_GBS * 1e9)
        t_alu = alu["ops_per_launch"] / (ALU_PEAK_TOPS * 1e12) if alu else 0.0
        if alu and t_alu >= t_hbm:
            roof = dict(alu)
            roof["hbm_view"] = hbm
        else:
            roof = dict(hbm)
            if alu:
                roof["alu_view"] = alu
        roof["floor_ms"] = {"hbm": t_hbm * 1e3, "alu": t_alu * 1e3 if alu else None}
        roof["traffic"] = measured_traffic(w.name, w.S)
    if roof is not None:
        roof.update({"kernel": kname, "kernel_avg_ms": kern_avg_ms,
                     "kernel_median_ms": kern_med_ms,
                     "algorithmic_bytes_per_launch": algo_bytes})
    out = {
        "metric": metric_name(w.name, batch, T, w.S, sum_n),
        "value": evals / (ms_step * 1e-3),
        "unit": "scenario-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        import oracle
        log("timing the oracle on the host cores")
        d = oracle.dist_matrix(w.xy)
        got = cost.cpu().numpy().reshape(T, -1)
        out["cpu_baseline"] = cpu_baseline(tours, d, w.demand, w.Q, w.S, threads, got)
        log(f"oracle parity on its sample: {out['cpu_baseline']['parity_vs_gpu_on_sample']}")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
