"""The PCG iterations between two convergence polls run as a captured HIP
graph that is replayed, with the host's poll (a kernel, a copy and a
synchronisation) between the replays.  The kernels are deterministic (fixed
summation orders), so the replayed graphs must give bit-identical results to
the same solves launched kernel by kernel (GLM_GRAPHS=0, in a child process),
and both must match the oracle."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from test_gpu_parity import check_against_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
import paper_2510_14471_amd as glm
from test_gpu_graphs import batch, solve
out = {}
for prec, red in (("fp64", False), ("mixed", False), ("mixed", True)):
    insts = batch()
    beta, u, it = solve(glm, insts, prec, red)
    out[f"{prec}-{red}"] = [beta.tolist(), float(np.abs(u).sum()), it.tolist()]
print(json.dumps(out))
"""


def batch():
    return list(synth.small_batch(seed=501, B=5, G_rng=(2, 9), M_rng=(200, 900),
                                  n_rng=(2, 9), K_rng=(1, 6)))


def solve(glm, insts, precision, reduce):
    lay, d = glm.pack_instances(insts)
    s = glm.SURSolver(lay, precision, reduce=reduce)
    s.factor(d["X"])
    beta, u, _, info, iters = s.solve(d["Omega"], d["y"], tol=1e-13 if precision == "mixed"
                                      else 1e-12)
    torch.cuda.synchronize()
    s.close()
    return beta.cpu().numpy(), u.cpu().numpy(), iters.cpu().numpy()


def test_graph_replays_match_eager_launches(tmp_path):
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    assert os.environ.get("GLM_GRAPHS", "1") != "0"
    got = {}
    for prec, red in (("fp64", False), ("mixed", False), ("mixed", True)):
        insts = batch()
        beta, u, it = solve(glm, insts, prec, red)
        assert it.max() > 16, "needs several replays of the 8-iteration graph"
        lay, _ = glm.pack_instances(insts)
        out = dict(beta=glm.unpack(lay, torch.tensor(beta), "beta"),
                   u=glm.unpack(lay, torch.tensor(u), "u"),
                   info=[[0] * i.K for i in insts])
        check_against_oracle(insts, out)
        got[f"{prec}-{red}"] = (beta, float(np.abs(u).sum()), it)
    print("[case] eager launches in a child process (GLM_GRAPHS=0)", flush=True)
    env = dict(os.environ, GLM_GRAPHS="0")
    res = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True,
                         text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    ref = json.loads(res.stdout.strip().splitlines()[-1])
    for key, (beta, usum, it) in got.items():
        rb, ru, rit = ref[key]
        assert np.array_equal(beta, np.array(rb)), key
        assert usum == ru, key
        assert np.array_equal(it, np.array(rit)), key
