"""Parity of the HIP path at the full sizes of the workloads (GPU).

The batched workload runs in the launch configuration bench.py times; all
of its 8,192 (instance, rhs) pairs are compared with the oracle, normwise and
element by element, and every instance is checked for the two defining
identities of the augmented system (Sigma u + X beta = y and X^T u = 0).  The
single large instances are compared with the oracle outright."""
import numpy as np
import pytest

import synth
from conftest import assert_all_pairs, batch512_with_oracle, rel_err
from oracle import gls, grad

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


def solve(glm, insts, precision, tol=1e-12, max_iter=0, reduce=False):
    print(f"[case] {precision} reduce={reduce} B={len(insts)} G={[i.G for i in insts][:4]} "
          f"M={[i.M for i in insts][:4]} K={insts[0].K} k={insts[0].kc}", flush=True)
    lay, d = glm.pack_instances(insts)
    s = glm.SURSolver(lay, precision, reduce=reduce)
    s.factor(d["X"], d["Rc"])
    beta, u, _, info, iters = s.solve(d["Omega"], d["y"], d["r"], tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    out = dict(beta=glm.unpack(lay, beta, "beta"), u=glm.unpack(lay, u, "u"),
               info=glm.unpack(lay, info, "rhs"), stats=s.stats())
    s.close()
    return out


def identities(inst, beta, U):
    """Relative residuals of Sigma u + X beta = y and of X_i^T u_i = 0."""
    fit = gls.fitted(inst, beta)                       # M x G x K
    SU = np.einsum("tjk,ji->tik", U, inst.Omega)
    r1 = np.linalg.norm(SU + fit - inst.Y) / np.linalg.norm(inst.Y)
    r2 = 0.0
    for i in range(inst.G):
        Xi = inst.X(i)
        r2 = max(r2, np.linalg.norm(Xi.T @ U[:, i, :]) /
                 (np.linalg.norm(Xi) * max(np.linalg.norm(U[:, i, :]), 1e-300)))
    return r1, r2


# -- the batched workload (512 instances x 16 right-hand sides) --------------------------

@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batched_workload_all_pairs_and_identities(glmlib, precision):
    """All 512 x 16 (instance, rhs) pairs against the oracle, normwise and
    element-wise, plus the two identities on every instance."""
    insts, refs = batch512_with_oracle()
    out = solve(glmlib, insts, precision)
    worst = assert_all_pairs(insts, refs, out["beta"], out["u"], out["info"], TOL)
    print(f"[worst] {precision} {worst}", flush=True)
    worst = (0.0, 0.0)
    for b, inst in enumerate(insts):
        r1, r2 = identities(inst, out["beta"][b], out["u"][b])
        worst = (max(worst[0], r1), max(worst[1], r2))
    assert worst[0] <= TOL and worst[1] <= TOL, worst


# -- one large SUR (G = 50, M = 10,000) ------------------------------------------------

@pytest.mark.parametrize("reduce", [False, True], ids=["full", "reduced"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_single_sur(glmlib, precision, reduce):
    insts = list(synth.config1())
    out = solve(glmlib, insts, precision, reduce=reduce)
    beta_o, U_o = gls.sur_gls(insts[0])
    assert out["info"][0][0] in (0, 1)
    assert rel_err(out["beta"][0], beta_o) <= TOL
    assert rel_err(out["u"][0], U_o) <= TOL


# -- singular Omega of rank G - 2 with 10 cross-equation restrictions -----------------

@pytest.mark.parametrize("reduce", [False, True], ids=["full", "reduced"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_singular_restricted_workload(glmlib, precision, reduce):
    """G = 100, M = 50,000, rank G - 2, ten restrictions; also through the
    model reduction (1,751 rotated rows instead of 50,000)."""
    inst = list(synth.config4())[0]
    out = solve(glmlib, [inst], precision, reduce=reduce)
    beta_o, _, SU_o = gls.sur_solution(inst)
    beta = out["beta"][0]
    SU = np.einsum("tjk,ji->tik", out["u"][0], inst.Omega)
    assert out["info"][0][0] in (0, 1), out
    assert rel_err(beta, beta_o) <= TOL
    assert rel_err(SU, SU_o) <= TOL
    # the noise-free combinations determine beta: it equals beta_true
    assert rel_err(beta, inst.beta_true) <= TOL
    assert np.linalg.norm(inst.Rc @ beta - inst.r) <= TOL * np.linalg.norm(inst.r)


# -- differentiation workload (G = 20, M = 20,000) ------------------------------------

@pytest.mark.parametrize("reduce", [False, True], ids=["full", "reduced"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_differentiation_workload(glmlib, precision, reduce):
    """dL/dy, dL/dOmega, dL/dX of L = 1/2 ||b - beta_true||^2 + the Gaussian
    negative log-likelihood in Omega, through the autograd binding (also
    through the model reduction): against the oracle's dense reference
    gradient, and against central finite differences of the oracle's loss
    (h = 1e-6) on 200 random coordinates."""
    inst = list(synth.config3())[0]
    lay, d = glmlib.pack_instances([inst])
    s = glmlib.SURSolver(lay, precision, reduce=reduce)
    X = d["X"].clone().requires_grad_(True)
    Om = d["Omega"].clone().requires_grad_(True)
    y = d["y"].clone().requires_grad_(True)
    beta, u = glmlib.gls(s, X, Om, y, tol=1e-12)
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
    s.close()
    gY = y.grad.cpu().numpy().reshape(M, G)
    gO = Om.grad.cpu().numpy().reshape(G, G)
    gO = 0.5 * (gO + gO.T)
    gW = X.grad.cpu().numpy().reshape(M, n)
    rY, rO, rW = grad.loss_grad(inst, inst.beta_true)
    assert rel_err(gY, rY[:, :, 0]) <= TOL
    assert rel_err(gO, rO) <= TOL
    assert rel_err(gW, rW) <= TOL
    if precision != "fp64":
        return
    # central differences of the oracle's loss
    h = 1e-6
    rng = np.random.default_rng(41)
    L0 = grad.loss_value(inst, inst.beta_true)
    floor = 10 * np.finfo(float).eps * abs(L0) / h

    def fd(perturb):
        perturb(+h)
        lp = grad.loss_value(inst, inst.beta_true)
        perturb(-2 * h)
        lm = grad.loss_value(inst, inst.beta_true)
        perturb(+h)
        return (lp - lm) / (2 * h)

    checks = []
    for _ in range(80):
        t, i = int(rng.integers(M)), int(rng.integers(G))

        def py(e, t=t, i=i):
            inst.Y[t, i, 0] += e
        checks.append((fd(py), gY[t, i]))
    for _ in range(80):
        t, c = int(rng.integers(M)), int(rng.integers(n))

        def pw(e, t=t, c=c):
            inst.W[t, c] += e
        checks.append((fd(pw), gW[t, c]))
    for _ in range(40):
        i, j = int(rng.integers(G)), int(rng.integers(G))

        def po(e, i=i, j=j):
            inst.Omega[i, j] += e
            if i != j:
                inst.Omega[j, i] += e
        an = gO[i, j] if i == j else 2 * gO[i, j]
        checks.append((fd(po), an))
    bad = [(f, a) for f, a in checks if abs(f - a) > 1e-6 * abs(a) + floor]
    assert not bad, (len(bad), bad[:5], floor)
