import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def rel_err(a, b):
    """||a - b|| / ||b|| (Frobenius over all entries); 0 when both vanish."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


@pytest.fixture
def relerr():
    return rel_err


_BATCH512 = {}


def batch512_with_oracle():
    """The batched workload (512 instances x 16 rhs) and the oracle's
    (beta, U) of every instance, computed once per test process (about a
    minute of host time) and shared by the full-size tests."""
    if "v" not in _BATCH512:
        import sys
        import time
        import synth
        from oracle import gls
        t0 = time.time()
        insts = list(synth.config2())
        refs = []
        for b, inst in enumerate(insts):
            refs.append(gls.sur_gls(inst))
            if b % 128 == 127:
                sys.stderr.write(f"[oracle] {b + 1}/512 instances, {time.time() - t0:.0f}s\n")
                sys.stderr.flush()
        _BATCH512["v"] = (insts, refs)
    return _BATCH512["v"]


def assert_all_pairs(insts, refs, beta, U, info, tol=1e-10):
    """Every (instance, rhs): beta and u against the oracle, normwise
    (||x - x_o|| <= tol ||x_o||) and element-wise (|x - x_o| <= tol ||x_o||_inf),
    and a converged or stagnated status.  Returns the worst errors."""
    import numpy as np
    worst = {"beta": 0.0, "u": 0.0, "beta_elem": 0.0, "u_elem": 0.0}
    for b, inst in enumerate(insts):
        beta_o, U_o = refs[b]
        assert all(v in (0, 1) for v in info[b]), (b, info[b])
        for k in range(inst.K):
            for key, got, want in (("beta", beta[b][:, k], beta_o[:, k]),
                                   ("u", U[b][:, :, k], U_o[:, :, k])):
                e = rel_err(got, want)
                ee = float(np.abs(got - want).max() / np.abs(want).max())
                worst[key] = max(worst[key], e)
                worst[key + "_elem"] = max(worst[key + "_elem"], ee)
                assert e <= tol and ee <= tol, (b, k, key, e, ee)
    return worst
