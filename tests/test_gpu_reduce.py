"""SUR model reduction on the GPU (GLM_REDUCED): parity with the oracle's
direct GLS of the full model, beta and u (Sigma u for singular Omega), in
both precisions; several Householder panels (n > 32), instances with
M <= n (nothing to drop), restrictions, singular Omega, sixteen rhs (the
matrix-core passes of the reduced problem), up to 100 equations, reverse
mode, and the batched workload at full size.  The reduced route itself is
pinned on the CPU (oracle.reduce against oracle.gls)."""
import numpy as np
import pytest

import synth
from conftest import assert_all_pairs, batch512_with_oracle, rel_err
from oracle import gls
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


def run_reduced(glm, insts, precision, tol=1e-13, precond="scalar"):
    print(f"[case] reduced {precision} {precond} B={len(insts)} G={[i.G for i in insts][:6]} "
          f"M={[i.M for i in insts][:6]} n={[i.n for i in insts][:6]} K={insts[0].K} "
          f"k={[i.kc for i in insts][:6]}", flush=True)
    lay, d = glm.pack_instances(insts)
    s = glm.SURSolver(lay, precision, reduce=True, precond=precond)
    s.factor(d["X"], d["Rc"])
    beta, u, _, info, iters = s.solve(d["Omega"], d["y"], d["r"], tol=tol)
    torch.cuda.synchronize()
    out = dict(beta=glm.unpack(lay, beta, "beta"), u=glm.unpack(lay, u, "u"),
               info=glm.unpack(lay, info, "rhs"), iters=glm.unpack(lay, iters, "rhs"),
               stats=s.stats(), solver=s, dev=d)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_ragged_batch(glmlib, precision):
    insts = list(synth.small_batch(seed=161, B=6, G_rng=(1, 6), M_rng=(30, 400),
                                   n_rng=(1, 7), K_rng=(1, 5)))
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_several_panels(glmlib, precision):
    """n from 33 to ~140: two to five Householder panels of 32 columns."""
    insts = list(synth.small_batch(seed=163, B=3, G_rng=(5, 12), M_rng=(300, 900),
                                   n_rng=(6, 12), K_rng=(2, 4)))
    insts += list(synth.small_batch(seed=165, B=1, G_rng=(4, 4), M_rng=(200, 200),
                                    n_rng=(8, 8), K_rng=(3, 3)))        # n = 32 exactly
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)


def test_reduced_when_nothing_is_dropped(glmlib):
    """M <= n + 1: the rotation keeps every observation (and M < n uses only M
    reflectors).  With G = 12, M = 3, n = 20 the exact-arithmetic termination
    falls on the iteration limit m - n + 1 = 17 itself, so a solve may end
    there (GLM_INFO_NOCONV, outputs = the last iterate) a hair above the
    stopping threshold; its beta and u are still checked at 1e-10."""
    insts = list(synth.small_batch(seed=167, B=1, G_rng=(12, 12), M_rng=(3, 3),
                                   n_rng=(1, 2), K_rng=(3, 3)))
    insts += list(synth.small_batch(seed=169, B=1, G_rng=(4, 4), M_rng=(13, 13),
                                    n_rng=(3, 3), K_rng=(2, 2)))
    out = run_reduced(glmlib, insts, "fp64", tol=1e-12)
    for k in range(insts[0].K):
        assert out["info"][0][k] in (0, 1) or (out["info"][0][k] == -10 and
                                               out["iters"][0][k] == 17), out["info"][0]
    out["info"][0] = [0] * insts[0].K
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_with_restrictions(glmlib, precision):
    insts = list(synth.small_batch(seed=171, B=4, G_rng=(2, 5), M_rng=(40, 200),
                                   n_rng=(2, 5), K_rng=(1, 3), constraints=3))
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)
    for b, inst in enumerate(insts):
        if inst.kc:
            assert np.abs(inst.Rc @ out["beta"][b] - inst.r).max() < 1e-10


def test_reduced_sixteen_rhs(glmlib):
    insts = list(synth.small_batch(seed=173, B=3, G_rng=(4, 20), M_rng=(500, 2500),
                                   n_rng=(3, 12), K_rng=(16, 16)))
    out = run_reduced(glmlib, insts, "mixed")
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_singular_omega(glmlib, precision):
    """A singular Omega through the reduction: the dropped rows take a
    generalized inverse of Omega (pivoted Cholesky) and the null-space part
    of U comes from Q1; beta and Sigma u match the oracle and beta equals
    beta_true (the noise-free combinations determine it).  Ranks G - 2 at
    G = 5, 32 and 64, mixed with a positive definite instance."""
    good = list(synth.small_batch(seed=175, B=1, G_rng=(3, 3), M_rng=(80, 80),
                                  n_rng=(2, 3), K_rng=(2, 2)))
    bad = list(synth.small_batch(seed=177, B=1, G_rng=(5, 5), M_rng=(120, 120),
                                 n_rng=(2, 3), K_rng=(2, 2), singular=2))
    bad += list(synth.small_batch(seed=178, B=1, G_rng=(32, 32), M_rng=(160, 160),
                                  n_rng=(2, 3), K_rng=(1, 2), singular=2))
    bad += list(synth.small_batch(seed=180, B=1, G_rng=(64, 64), M_rng=(240, 240),
                                  n_rng=(1, 2), K_rng=(1, 1), singular=2))
    insts = good + bad
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)
    for b, inst in enumerate(bad, start=1):
        assert rel_err(out["beta"][b], inst.beta_true) <= TOL, b


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_backward_matches_dense_reference(glmlib, precision):
    """Reverse mode on a reduced handle: the adjoint system goes through the
    same reduction, and dL/dy, dL/dOmega, dL/dX of the full model match the
    oracle's gradients (restricted instances: the KKT adjoint) at 1e-10."""
    from oracle import grad
    insts = list(synth.small_batch(seed=179, B=4, G_rng=(2, 6), M_rng=(40, 300),
                                   n_rng=(1, 5), K_rng=(1, 3), shift=0.5, constraints=2))
    insts[2].Rc, insts[2].r = None, None
    out = run_reduced(glmlib, insts, precision)
    s, d = out["solver"], out["dev"]
    lay = glmlib.BatchLayout.of(insts)
    rng = np.random.default_rng(15)
    gb = [rng.standard_normal((i.n, i.K)) for i in insts]
    gu = [rng.standard_normal(i.Y.shape) for i in insts]
    g_beta = torch.tensor(np.concatenate([a.ravel() for a in gb]), device="cuda")
    g_u = torch.tensor(np.concatenate([a.ravel() for a in gu]), device="cuda")
    beta_d = torch.tensor(np.concatenate([a.ravel() for a in out["beta"]]), device="cuda")
    u_d = torch.tensor(np.concatenate([a.ravel() for a in out["u"]]), device="cuda")
    dy, dOm, dX, info, _ = s.backward(d["Omega"], beta_d, u_d, g_beta, g_u, tol=1e-13)
    dy = glmlib.unpack(lay, dy, "u")
    dOm = glmlib.unpack(lay, dOm, "Omega")
    dX = glmlib.unpack(lay, dX, "X")
    for b, inst in enumerate(insts):
        if inst.kc:
            beta_o, U_o, _ = gls.restricted_gls(inst)
            rY, rO, rW = grad.restricted_gls_vjp(inst, beta_o, U_o, gb[b], gu[b])
        else:
            beta_o, U_o = gls.sur_gls(inst)
            rY, rO, rW = grad.sur_gls_vjp(inst, beta_o, U_o, gb[b], gu[b])
        assert rel_err(dy[b], rY) <= TOL, (b, rel_err(dy[b], rY))
        assert rel_err(dOm[b], rO) <= TOL, (b, rel_err(dOm[b], rO))
        assert rel_err(dX[b], rW) <= TOL, (b, rel_err(dX[b], rW))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precond", ["equation", "scalar"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_reduced_batched_workload_full_size(glmlib, precision, precond):
    """The batched workload (512 instances x 16 rhs) through the reduction,
    in the launch configurations the benchmark times (D = diag(omega_ii) (x) I
    by default, D = alpha I): all 8,192 (instance, rhs) pairs against the
    oracle, normwise and element-wise, and Sigma u + X beta = y,
    X_i^T u_i = 0 on every instance."""
    from test_gpu_fullsize import identities
    insts, refs = batch512_with_oracle()
    out = run_reduced(glmlib, insts, precision, tol=1e-12, precond=precond)
    worst = assert_all_pairs(insts, refs, out["beta"], out["u"], out["info"], TOL)
    print(f"[worst] reduced {precision} {worst}", flush=True)
    out["solver"].close()
    worst = (0.0, 0.0)
    for b, inst in enumerate(insts):
        r1, r2 = identities(inst, out["beta"][b], out["u"][b])
        worst = (max(worst[0], r1), max(worst[1], r2))
    assert worst[0] <= TOL and worst[1] <= TOL, worst


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_repeated_intercepts(glmlib, precision):
    """The two widest instances of the batched workload (G = 32, n = 417 and
    419): the intercept repeated in every equation makes W exactly rank
    deficient, and later dependent columns leave subcolumns of ~1e-160 whose
    squares underflow; the QR must take them as zero for Q to stay
    orthogonal."""
    insts = list(synth.config2(subset=[12, 228]))
    out = run_reduced(glmlib, insts, precision, tol=1e-12)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_many_equations(glmlib, precision):
    """G = 64 and G = 100 equations (Omega^g and the full model's u formed
    from global memory), with W of 128 to 300 columns (four to ten
    Householder panels) and rows in several apply segments."""
    insts = list(synth.small_batch(seed=181, B=2, G_rng=(64, 64), M_rng=(300, 1500),
                                   n_rng=(2, 3), K_rng=(1, 3)))
    insts += list(synth.small_batch(seed=183, B=1, G_rng=(100, 100), M_rng=(900, 900),
                                    n_rng=(2, 3), K_rng=(2, 2)))
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)
