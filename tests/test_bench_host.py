"""Host-side pieces of bench.py: the window-work count that sizes the ALU roofline agrees with
the oracle's count of Eq. (3)'s window minima, the multi-GPU request is refused, and the source
hashes that guard committed traffic figures track their own kernels."""
import subprocess
import sys
import os

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_window_work_matches_oracle_count():
    import bench
    b = gen.make_batch_workload("batch-256", T=5, S=700)
    d = oracle.dist_matrix(b.xy)
    want = 0
    for t in b.tours:
        _, work = oracle.split(t, d, b.demand, b.Q, return_work=True)
        want += work
    got = bench.window_work(torch.from_numpy(b.demand), b.tours, b.Q, chunk=256)
    assert got == want


def test_window_work_single_tour_workload():
    import bench
    w = gen.make_workload("poisson-n200", S=300)
    d = oracle.dist_matrix(w.xy)
    _, work = oracle.split(w.tour, d, w.demand, w.Q, return_work=True)
    assert bench.window_work(torch.from_numpy(w.demand), [w.tour], w.Q) == work


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_source_hashes_cover_only_their_kernels(tmp_path, monkeypatch):
    # a committed traffic figure stays valid while other kernels of the same file change, and
    # is dropped as soon as its own kernel's source changes
    import bench
    src = open(bench.NN_SRC, "rb").read()
    base = bench.nn_source_sha()
    mark = bench.NN_MARK + b"weight gradients"
    assert mark in src
    edits = {
        "other": src.replace(mark, mark + b"\n// edited", 1),
        "fused": src.replace(bench.NN_MARK + b"fused inference",
                             bench.NN_MARK + b"fused inference\n// edited", 1),
    }
    shas = {}
    for name, text in edits.items():
        p = tmp_path / f"{name}.hip"
        p.write_bytes(text)
        monkeypatch.setattr(bench, "NN_SRC", str(p))
        shas[name] = bench.nn_source_sha()
    assert shas["other"] == base and shas["fused"] != base
