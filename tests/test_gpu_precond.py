"""The per-equation preconditioner D = diag(omega_11 .. omega_GG) (x) I_M
(GLM_PRECOND_EQ) on the GPU: beta and u match the oracle at 1e-10 in both
precisions and through the model reduction (beta does not depend on D), a
diagonal Omega is solved in one PCG step (the preconditioner is then the
exact inverse of the augmented matrix), and the iteration count follows the
oracle's PCG-Aug with the same D."""
import numpy as np
import pytest

import synth
from conftest import rel_err
from oracle import gls, pcg_aug
from test_gpu_parity import check_against_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


def run(glm, insts, precision, reduce=False, precond="equation", tol=None):
    print(f"[case] precond={precond} {precision} reduce={reduce} B={len(insts)} "
          f"G={[i.G for i in insts]} K={[i.K for i in insts]} k={[i.kc for i in insts]}",
          flush=True)
    lay, d = glm.pack_instances(insts)
    s = glm.SURSolver(lay, precision, reduce=reduce, precond=precond)
    s.factor(d["X"], d["Rc"])
    if tol is None:
        tol = 1e-13 if precision == "mixed" else 1e-12
    beta, u, _, info, iters = s.solve(d["Omega"], d["y"], d["r"], tol=tol)
    torch.cuda.synchronize()
    out = dict(beta=glm.unpack(lay, beta, "beta"), u=glm.unpack(lay, u, "u"),
               info=glm.unpack(lay, info, "rhs"), iters=glm.unpack(lay, iters, "rhs"),
               stats=s.stats())
    s.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_equation_d_ragged_and_restricted(glmlib, precision):
    insts = list(synth.small_batch(seed=401, B=6, G_rng=(1, 7), M_rng=(30, 400),
                                   n_rng=(1, 7), K_rng=(1, 5)))
    insts += list(synth.small_batch(seed=403, B=2, G_rng=(2, 5), M_rng=(40, 200),
                                    n_rng=(2, 5), K_rng=(1, 3), constraints=3))
    out = run(glmlib, insts, precision)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_equation_d_sixteen_rhs_and_wide_omega(glmlib, precision):
    """Sixteen rhs with G up to 20 (matrix-core Omega apply of the FP32
    passes), and G = 70 (column-slot passes)."""
    insts = list(synth.small_batch(seed=405, B=3, G_rng=(4, 20), M_rng=(300, 1200),
                                   n_rng=(3, 12), K_rng=(16, 16)))
    out = run(glmlib, insts, precision)
    check_against_oracle(insts, out)
    wide = list(synth.small_batch(seed=407, B=1, G_rng=(70, 70), M_rng=(150, 150),
                                  n_rng=(2, 4), K_rng=(16, 16)))
    out = run(glmlib, wide, precision)
    assert out["stats"]["fp64_passes"]["rowvec"] == 0
    check_against_oracle(wide, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_equation_d_through_the_model_reduction(glmlib, precision):
    insts = list(synth.small_batch(seed=409, B=4, G_rng=(3, 12), M_rng=(200, 900),
                                   n_rng=(3, 12), K_rng=(1, 16)))
    out = run(glmlib, insts, precision, reduce=True)
    check_against_oracle(insts, out)


def test_diagonal_omega_takes_one_step(glmlib):
    """Sigma = D: one PCG step per rhs, at blockwise OLS; D = alpha I needs
    one step per distinct omega_ii."""
    insts = list(synth.small_batch(seed=411, B=3, G_rng=(3, 6), M_rng=(60, 300),
                                   n_rng=(2, 5), K_rng=(1, 4)))
    rng = np.random.default_rng(412)
    for inst in insts:
        inst.Omega = np.diag(rng.uniform(0.5, 4.0, inst.G))
    out = run(glmlib, insts, "fp64", tol=1e-12)
    check_against_oracle(insts, out)
    for b, inst in enumerate(insts):
        assert all(int(v) == 1 for v in out["iters"][b]), (b, out["iters"][b])
    out_a = run(glmlib, insts, "fp64", precond="scalar", tol=1e-12)
    for b, inst in enumerate(insts):
        assert all(int(v) >= inst.G - 1 for v in out_a["iters"][b]), (b, out_a["iters"][b])


def test_per_equation_d_iterations_follow_the_oracle(glmlib):
    inst = list(synth.config0())[0]
    out = run(glmlib, [inst], "fp64", tol=1e-12)
    check_against_oracle([inst], out)
    ref = pcg_aug.pcg_aug_projected(inst, tol=1e-12, alpha=pcg_aug.per_equation_d(inst.Omega))
    assert abs(int(out["iters"][0][0]) - ref.iterations) <= 2, (out["iters"], ref.iterations)
