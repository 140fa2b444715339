"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: the FP64 path and the mixed path after refinement must match
the oracle within 1e-10 relative error per (instance, rhs) for beta and u
(for singular Omega: Sigma u, since u is not unique there)."""
import numpy as np
import pytest

import synth
from conftest import rel_err
from oracle import gls, grad, pcg_aug

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


def run(glm, instances, precision, tol=1e-12, max_iter=0, want_uc=False):
    print(f"[case] {precision} B={len(instances)} "
          f"G={[i.G for i in instances]} M={[i.M for i in instances]} "
          f"K={[i.K for i in instances]} k={[i.kc for i in instances]}", flush=True)
    lay, d = glm.pack_instances(instances)
    s = glm.SURSolver(lay, precision)
    s.factor(d["X"], d["Rc"])
    beta, u, uc, info, iters = s.solve(d["Omega"], d["y"], d["r"], tol=tol, max_iter=max_iter,
                                       want_uc=want_uc)
    torch.cuda.synchronize()
    out = dict(beta=glm.unpack(lay, beta, "beta"), u=glm.unpack(lay, u, "u"),
               info=glm.unpack(lay, info, "rhs"), iters=glm.unpack(lay, iters, "rhs"),
               stats=s.stats(), solver=s, dev=d, lay=lay)
    if uc is not None:
        out["uc"] = glm.unpack(lay, uc, "uc")
    return out


def check_against_oracle(instances, out, tol=TOL):
    for b, inst in enumerate(instances):
        beta_o, U_o, SU_o = gls.sur_solution(inst)
        for k in range(inst.K):
            eb = rel_err(out["beta"][b][:, k], beta_o[:, k])
            if U_o is not None:
                eu = rel_err(out["u"][b][:, :, k], U_o[:, :, k])
            else:
                SU = np.einsum("ti,ij->tj", out["u"][b][:, :, k], inst.Omega)
                eu = rel_err(SU, SU_o[:, :, k])
            assert eb <= tol and eu <= tol, (b, k, eb, eu, out["info"][b][k])
            assert out["info"][b][k] in (0, 1), (b, k, out["info"][b][k])


# -- the small workload, FP64 ----------------------------------------------------

def test_sur_small_fp64_matches_oracle_and_reference_iterations(glmlib):
    insts = list(synth.config0())
    out = run(glmlib, insts, "fp64")
    check_against_oracle(insts, out)
    ref = pcg_aug.pcg_aug_projected(insts[0], tol=1e-12)
    assert abs(int(out["iters"][0][0]) - ref.iterations) <= 2, (out["iters"], ref.iterations)


def test_sur_small_mixed_matches_oracle(glmlib):
    insts = list(synth.config0())
    out = run(glmlib, insts, "mixed", tol=1e-13)
    check_against_oracle(insts, out)
    assert out["stats"]["outer_steps"] >= 2


# -- ragged batches ---------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ragged_batch(glmlib, precision):
    insts = list(synth.small_batch(seed=7, B=7, G_rng=(1, 6), M_rng=(20, 300),
                                   n_rng=(1, 7), K_rng=(1, 5)))
    out = run(glmlib, insts, precision, tol=1e-12 if precision == "fp64" else 1e-13)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_with_sixteen_rhs_and_long_tiles(glmlib, precision):
    insts = list(synth.small_batch(seed=11, B=3, G_rng=(4, 9), M_rng=(900, 2500),
                                   n_rng=(3, 12), K_rng=(16, 16)))
    out = run(glmlib, insts, precision, tol=1e-12 if precision == "fp64" else 1e-13)
    check_against_oracle(insts, out)


def test_degenerate_shapes(glmlib):
    insts = list(synth.small_batch(seed=13, B=1, G_rng=(1, 1), M_rng=(7, 7),
                                   n_rng=(1, 1), K_rng=(1, 1)))          # G=1, n=1
    rng = np.random.default_rng(14)
    insts.append(synth.sur._instance(rng, 5, [5, 2], np.array([[2.0, 0.5], [0.5, 1.0]]),
                                     2))                                  # n_i = M
    insts += list(synth.small_batch(seed=15, B=1, G_rng=(12, 12), M_rng=(3, 3),
                                    n_rng=(1, 2), K_rng=(3, 3)))         # M < G
    out = run(glmlib, insts, "fp64")
    check_against_oracle(insts, out)


# -- QR factors --------------------------------------------------------------------

def test_householder_factors(glmlib):
    insts = list(synth.small_batch(seed=17, B=4, G_rng=(1, 5), M_rng=(30, 700),
                                   n_rng=(1, 40), K_rng=(1, 1)))
    lay, d = glmlib.pack_instances(insts)
    s = glmlib.SURSolver(lay, "fp64")
    s.factor(d["X"])
    Q, R, rank = s.factors()
    Q = glmlib.unpack(lay, Q, "X")
    R = R.cpu().numpy()
    rank = rank.cpu().numpy()
    assert not rank.any()
    ro = 0
    for b, inst in enumerate(insts):
        for i in range(inst.G):
            ni = inst.n_i[i]
            Qi = Q[b][:, inst.col_off[i]:inst.col_off[i] + ni]
            Ri = R[ro:ro + ni * ni].reshape(ni, ni)
            ro += ni * ni
            Xi = inst.X(i)
            eps = np.finfo(float).eps
            assert np.abs(Qi.T @ Qi - np.eye(ni)).max() <= 20 * ni * eps * np.sqrt(inst.M)
            assert np.abs(Xi - Qi @ Ri).max() <= 20 * eps * np.abs(Xi).max() * np.sqrt(inst.M)
            assert np.allclose(np.tril(Ri, -1), 0.0)
            Rl = np.linalg.qr(Xi)[1]
            assert np.allclose(Ri.T @ Ri, Rl.T @ Rl, rtol=1e-11, atol=1e-11 * np.abs(Rl).max() ** 2)


# -- failure modes forced from the host ----------------------------------------------

def test_rank_deficient_block_is_reported(glmlib):
    insts = list(synth.small_batch(seed=19, B=2, G_rng=(3, 3), M_rng=(40, 60),
                                   n_rng=(3, 4), K_rng=(2, 2)))
    inst = insts[1]
    inst.W[:, inst.col_off[1] + 1] = inst.W[:, inst.col_off[1]]   # duplicated column
    out = run(glmlib, insts, "fp64")
    assert all(v == -12 for v in out["info"][1])
    check_against_oracle(insts[:1], {k: v[:1] if isinstance(v, list) else v
                                     for k, v in out.items()})


def test_iteration_limit_is_reported(glmlib):
    insts = list(synth.config0())
    out = run(glmlib, insts, "fp64", max_iter=2)
    assert out["info"][0][0] == -10 and out["iters"][0][0] == 2


# -- restrictions and singular Omega ---------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_restricted_batch(glmlib, precision):
    insts = list(synth.small_batch(seed=23, B=4, G_rng=(2, 5), M_rng=(40, 200),
                                   n_rng=(2, 5), K_rng=(1, 3), constraints=3))
    out = run(glmlib, insts, precision, tol=1e-13, want_uc=True)
    check_against_oracle(insts, out)
    for b, inst in enumerate(insts):
        if inst.kc:
            assert np.abs(inst.Rc @ out["beta"][b] - inst.r).max() < 1e-10
            _, _, wc = gls.restricted_gls(inst)
            assert rel_err(out["uc"][b], wc) < 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_singular_omega(glmlib, precision):
    insts = list(synth.small_batch(seed=29, B=3, G_rng=(4, 6), M_rng=(200, 400),
                                   n_rng=(2, 4), K_rng=(1, 2), singular=2))
    out = run(glmlib, insts, precision, tol=1e-13)
    check_against_oracle(insts, out)
    for b, inst in enumerate(insts):
        assert rel_err(out["beta"][b], inst.beta_true) < 1e-10


# -- gradients -------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_backward_matches_dense_reference(glmlib, precision):
    insts = list(synth.small_batch(seed=31, B=3, G_rng=(2, 5), M_rng=(30, 120),
                                   n_rng=(1, 4), K_rng=(1, 3), shift=0.5))
    out = run(glmlib, insts, precision, tol=1e-13)
    s, d, lay = out["solver"], out["dev"], out["lay"]
    rng = np.random.default_rng(5)
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
        beta_o, U_o = gls.sur_gls(inst)
        rY, rO, rW = grad.sur_gls_vjp(inst, beta_o, U_o, gb[b], gu[b])
        assert rel_err(dy[b], rY) <= TOL
        assert rel_err(dOm[b], rO) <= TOL
        assert rel_err(dX[b], rW) <= TOL


def test_autograd_loss_with_likelihood_matches_oracle_and_fd(glmlib):
    inst = synth.small_batch(seed=37, B=1, G_rng=(3, 3), M_rng=(60, 60), n_rng=(2, 4),
                             K_rng=(1, 1), shift=0.5)[0]
    lay, d = glmlib.pack_instances([inst])
    s = glmlib.SURSolver(lay, "fp64")
    X = d["X"].clone().requires_grad_(True)
    Om = d["Omega"].clone().requires_grad_(True)
    y = d["y"].clone().requires_grad_(True)
    beta, u = glmlib.gls(s, X, Om, y, tol=1e-13)
    M, G, n = inst.M, inst.G, inst.n
    Omm = Om.view(G, G)
    W = X.view(M, n)
    fit = torch.stack([W[:, o:o + ni] @ beta[o:o + ni] for o, ni in
                       zip(inst.col_off, inst.n_i)], 1)
    E = y.view(M, G) - fit
    bt = torch.tensor(inst.beta_true[:, 0], device="cuda")
    L = 0.5 * torch.sum((beta - bt) ** 2) + 0.5 * (
        M * torch.logdet(Omm) + torch.trace(torch.linalg.solve(Omm, E.T @ E)))
    L.backward()
    rY, rO, rW = grad.loss_grad(inst, inst.beta_true)
    assert rel_err(y.grad.cpu().numpy().reshape(M, G), rY[:, :, 0]) <= TOL
    gO = Om.grad.cpu().numpy().reshape(G, G)
    assert rel_err(0.5 * (gO + gO.T), rO) <= TOL
    assert rel_err(X.grad.cpu().numpy().reshape(M, n), rW) <= TOL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_backward_of_restricted_instances(glmlib, precision):
    """Reverse mode through restricted instances (eq. GRGLM): the adjoint
    solve runs in the restricted geometry, and dL/dy, dL/dOmega, dL/dX
    match the oracle's restricted-GLS gradient (KKT adjoint) at 1e-10; the
    batch mixes restricted and unrestricted instances."""
    insts = list(synth.small_batch(seed=43, B=4, G_rng=(2, 5), M_rng=(40, 160),
                                   n_rng=(2, 5), K_rng=(1, 3), shift=0.5, constraints=3))
    insts[1].Rc, insts[1].r = None, None
    out = run(glmlib, insts, precision, tol=1e-13)
    s, d, lay = out["solver"], out["dev"], out["lay"]
    rng = np.random.default_rng(9)
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
