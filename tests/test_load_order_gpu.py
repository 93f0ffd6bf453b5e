"""One HIP runtime per process, whatever the import order.

torch ships a HIP runtime of its own under the soname the library links against; the binding
loads torch before the library so that both use that one. The check runs in a fresh process
that creates a context before it imports torch itself, then evaluates device demands and
compares every cost with the oracle.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import paper_2511_18022_amd as sg
ctx = sg.SplitContext(0)            # loads the library before this script imports torch
import torch
d = np.load(sys.argv[1])
ctx.set_coords(d["xy"])
dem = torch.from_numpy(d["demand"]).cuda()
cost, st = ctx.eval(d["tour"], dem, int(d["Q"]))
np.save(sys.argv[2], cost.cpu().numpy())
ctx.close()
print("child ok", flush=True)
"""


def test_context_created_before_torch_import(tmp_path):
    n, S, Q = 60, 3000, 100
    xy = gen.coords(71, n)
    tour = gen.tour(72, n)
    demand = gen.demand_uniform(73, n, S, 0, 30)
    inp, out = tmp_path / "in.npz", tmp_path / "out.npy"
    np.savez(inp, xy=xy, tour=tour, demand=demand, Q=Q)
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    res = subprocess.run([sys.executable, "-c", CHILD, str(inp), str(out)], env=env,
                         capture_output=True, text=True, timeout=110)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    got = np.load(out)
    want = oracle.split(tour, oracle.dist_matrix(xy), demand, Q, threads=4)
    np.testing.assert_array_equal(got, want)
