"""Scale robustness of the factorizations on the GPU: regressors multiplied
by 1e-140, 1e150, 1e-160 or 1e160 as a whole, or column by column by powers of ten in
[1e-120, 1e120], give beta scaled back by the same factors and the same u
(exact identities: X S beta_S = X beta with beta_S = S^-1 beta, and u does
not change).  Both precisions, with and without the model reduction,
restricted instances included (R_c scaled with X, so that the restricted
solution is the same up to S).  Without the power-of-two column scaling of
the QR the squared Householder norms overflow at 1e160 and fall below the
zero-subcolumn threshold (1e-250) at 1e-140, where every reflector would be
skipped."""
import copy

import numpy as np
import pytest

import synth
from conftest import rel_err
from oracle import gls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


def _instances():
    insts = list(synth.small_batch(seed=601, B=4, G_rng=(2, 6), M_rng=(30, 300),
                                   n_rng=(2, 6), K_rng=(1, 3)))
    insts += list(synth.small_batch(seed=603, B=2, G_rng=(2, 5), M_rng=(40, 200),
                                    n_rng=(2, 5), K_rng=(1, 2), constraints=2))
    insts += list(synth.small_batch(seed=605, B=1, G_rng=(3, 3), M_rng=(1500, 1500),
                                    n_rng=(20, 30), K_rng=(4, 4)))
    return insts


def _scaled(inst, sc):
    si = copy.deepcopy(inst)
    si.W = si.W * sc
    if si.Rc is not None:
        si.Rc = si.Rc * sc
    return si


def _run(glm, insts, precision, reduce):
    lay, d = glm.pack_instances(insts)
    s = glm.SURSolver(lay, precision, reduce=reduce)
    s.factor(d["X"], d["Rc"])
    tol = 1e-13 if precision == "mixed" else 1e-12
    beta, u, _, info, _ = s.solve(d["Omega"], d["y"], d["r"], tol=tol)
    torch.cuda.synchronize()
    out = (glm.unpack(lay, beta, "beta"), glm.unpack(lay, u, "u"), glm.unpack(lay, info, "rhs"))
    s.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("reduce", [False, True])
@pytest.mark.parametrize("mode", ["1e-140", "1e150", "1e-160", "1e160", "columns"])
def test_scaled_regressors(glmlib, precision, reduce, mode):
    insts = _instances()
    rng = np.random.default_rng(607)
    scales = []
    for inst in insts:
        if mode == "columns":
            scales.append(10.0 ** rng.uniform(-120, 120, inst.n))
        else:
            scales.append(np.full(inst.n, float(mode)))
    print(f"[case] scaled regressors {mode} {precision} reduce={reduce}", flush=True)
    beta, u, info = _run(glmlib, [_scaled(i, s) for i, s in zip(insts, scales)], precision,
                         reduce)
    for b, inst in enumerate(insts):
        beta_o, U_o, _ = gls.sur_solution(inst)
        for k in range(inst.K):
            eb = rel_err(beta[b][:, k] * scales[b], beta_o[:, k])
            eu = rel_err(u[b][:, :, k], U_o[:, :, k])
            assert eb <= TOL and eu <= TOL, (mode, b, k, eb, eu, info[b][k])
            assert info[b][k] in (0, 1), (b, k, info[b][k])
