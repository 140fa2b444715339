"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check compares the oracle with something other than itself: a second
independent route (dense formula vs structured formula vs brute-force
least-squares KKT solve), a special case that reduces to OLS, exact
rational arithmetic, numbers printed in the paper, a theorem (unbiasedness,
monotone error), or finite differences.  Several tests plant a plausible
mistake in a copy of an oracle routine and check that a pin catches it.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import gls, grad, pcg_aug
from conftest import rel_err

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _nonsingular_batch():
    return synth.small_batch(seed=21, B=5, G_rng=(1, 4), M_rng=(8, 40),
                             n_rng=(1, 4), K_rng=(1, 3))


# -- P1: two independent routes to b_GLS and to the augmented solution --------

def test_structured_gls_matches_dense_formula_and_kkt():
    for inst in _nonsingular_batch():
        beta, U = gls.sur_gls(inst)
        for k in range(inst.K):
            X, S, y = gls.sur_dense(inst, k)
            b_dense = gls.gls_dense(X, S, y)
            w_kkt, b_kkt = gls.augmented_lstsq(X, S, y)
            assert rel_err(beta[:, k], b_dense) < 1e-11
            assert rel_err(beta[:, k], b_kkt) < 1e-10
            assert rel_err(U[:, :, k].T.reshape(-1), w_kkt) < 1e-10
            # u is the GLS residual mapped by Sigma^-1 and is orthogonal to X
            assert np.abs(X.T @ w_kkt).max() < 1e-9 * max(1, np.abs(w_kkt).max())


def test_eigsplit_equals_textbook_gls_for_nonsingular_omega():
    for inst in _nonsingular_batch():
        beta, U = gls.sur_gls(inst)
        beta2, SU = gls.sur_gls_eigsplit(inst)
        assert rel_err(beta2, beta) < 1e-10
        assert rel_err(SU, np.einsum("tik,ij->tjk", U, inst.Omega)) < 1e-10


# -- P3: Lemma AugBLUE closed form through the full QR ------------------------

def test_aug_blue_closed_form():
    inst = synth.small_batch(seed=3, B=1, G_rng=(3, 3), M_rng=(12, 12),
                             n_rng=(2, 3), K_rng=(1, 1))[0]
    X, S, y = gls.sur_dense(inst)
    w, b = gls.aug_blue_closed_form(X, S, y)
    w2, b2 = gls.augmented_lstsq(X, S, y)
    assert rel_err(b, b2) < 1e-11 and rel_err(w, w2) < 1e-10


# -- P2: special cases in which GLS reduces to OLS ----------------------------

def _blockwise_ols(inst):
    return np.concatenate([np.linalg.lstsq(inst.X(i), inst.Y[:, i, :], rcond=None)[0]
                           for i in range(inst.G)], 0)


def test_diagonal_omega_is_blockwise_ols_and_pcg_needs_G_steps():
    inst = synth.small_batch(seed=5, B=1, G_rng=(3, 3), M_rng=(50, 50),
                             n_rng=(2, 4), K_rng=(2, 2))[0]
    inst.Omega = np.diag([0.7, 1.9, 3.1])
    beta, _ = gls.sur_gls(inst)
    assert rel_err(beta, _blockwise_ols(inst)) < 1e-12
    for k in range(inst.K):
        res = pcg_aug.pcg_aug(inst, k=k, tol=1e-13)
        # with D = alpha I the reduced matrix Q_N^T Sigma Q_N has exactly G
        # distinct eigenvalues (omega_ii), hence G steps
        assert res.iterations <= inst.G
        assert rel_err(res.z_hat, beta[:, k]) < 1e-12


def test_identical_regressors_gls_equals_ols():
    inst = synth.small_batch(seed=6, B=1, G_rng=(4, 4), M_rng=(40, 40),
                             n_rng=(3, 3), K_rng=(2, 2))[0]
    X0 = inst.X(0).copy()
    for i in range(inst.G):
        inst.W[:, inst.col_off[i]:inst.col_off[i] + 3] = X0
    beta, _ = gls.sur_gls(inst)
    assert rel_err(beta, _blockwise_ols(inst)) < 1e-11


def test_scalar_omega_and_single_equation_are_ols():
    inst = synth.small_batch(seed=8, B=1, G_rng=(3, 3), M_rng=(30, 30),
                             n_rng=(2, 3), K_rng=(1, 1))[0]
    inst.Omega = 2.5 * np.eye(3)
    assert rel_err(gls.sur_gls(inst)[0], _blockwise_ols(inst)) < 1e-12
    one = synth.small_batch(seed=9, B=1, G_rng=(1, 1), M_rng=(30, 30),
                            n_rng=(3, 3), K_rng=(2, 2))[0]
    assert rel_err(gls.sur_gls(one)[0], _blockwise_ols(one)) < 1e-12


# -- P4: exact rational PCG-Aug terminates at #distinct eigenvalues -------------

@pytest.mark.parametrize("seed,n_i", [(5, (1, 2)), (6, (2, 1)), (7, (1, 1))])
def test_exact_pcg_aug_finite_termination(seed, n_i):
    Xs, Om, Y = synth.tiny_integer_sur(seed=seed, n_i=n_i)
    X, S, y = pcg_aug.dense_from_integer_sur(Xs, Om, Y)
    it, z_hat, w, status = pcg_aug.pcg_aug_exact(X, S, y)
    assert status == "converged"
    w_k, b_k = pcg_aug.kkt_exact(X, S, y)
    assert z_hat == b_k and w == w_k            # bit-identical rationals
    m, n = X.shape
    Q, _ = np.linalg.qr(X.astype(float), mode="complete")
    ev = np.sort(np.linalg.eigvalsh(Q[:, n:].T @ S @ Q[:, n:]))
    distinct = 1 + int(np.sum(np.diff(ev) > 1e-9 * ev[-1]))
    assert it <= m - n + 1
    assert it == distinct


# -- P5: FP64 reference iteration --------------------------------------------

def test_pcg_reference_converges_to_direct_solution_with_monotone_error():
    inst = synth.config0()[0]
    beta, U = gls.sur_gls(inst)
    res = pcg_aug.pcg_aug(inst, tol=1e-12, keep_w=True)
    assert res.status == "converged"
    assert rel_err(res.z_hat, beta[:, 0]) < 1e-12
    w_true = U[:, :, 0].T.reshape(-1)
    assert rel_err(res.w, w_true) < 1e-11
    ops = pcg_aug.SurOperators(inst, 1.0)
    errs = [float((wi - w_true) @ ops.Sigma(wi - w_true)) for wi in res.w_iterates]
    assert all(b <= a * (1 + 1e-9) + 1e-20 for a, b in zip(errs, errs[1:]))  # eq. wOptim
    for wi in res.w_iterates:                                            # X^T w_i = 0
        assert np.abs(ops.XT(wi)).max() < 1e-10 * max(1.0, np.abs(wi).max())
    q = np.linalg.matrix_rank(inst.W)
    G, n = inst.G, inst.n
    assert res.iterations <= G + G * q - n + 1


def test_pcg_reference_nonzero_lower_rhs():
    inst = _nonsingular_batch()[1]
    X, S, y = gls.sur_dense(inst, 0)
    h2 = np.random.default_rng(0).standard_normal(inst.n)
    res = pcg_aug.pcg_aug(inst, k=0, tol=1e-13, h2=h2)
    w_k, b_k = gls.augmented_lstsq(X, S, y, h2=h2)
    assert rel_err(res.z_hat, b_k) < 1e-10 and rel_err(res.w, w_k) < 1e-10


def test_pcg_reference_alpha_only_changes_iterates_not_solution():
    inst = synth.config0()[0]
    b0 = pcg_aug.pcg_aug(inst, tol=1e-12, alpha=1.0)
    b1 = pcg_aug.pcg_aug(inst, tol=1e-12)
    assert rel_err(b0.z_hat, b1.z_hat) < 1e-12
    assert abs(b0.iterations - b1.iterations) <= 2


# -- P7: condition numbers printed in the paper --------------------------------

def _cond_KG(X, Sigma):
    m, n = X.shape
    Gm = gls.augmented_matrix(X, Sigma)
    D = np.eye(m)
    # eq. prec with D = I: K = [[Pi, X*], [X*^T, -(X^T X)^-1]]
    XtXi = np.linalg.inv(X.T @ X)
    Xs = X @ XtXi
    Pi = np.eye(m) - Xs @ X.T
    K = np.block([[Pi, Xs], [Xs.T, -XtXi]])
    K_inv_form = np.linalg.inv(np.block([[D, X], [X.T, np.zeros((n, n))]]))  # eq. invprec
    assert np.abs(K - K_inv_form).max() < 1e-8 * np.abs(K).max()
    ev = np.abs(np.linalg.eigvals(K @ Gm))
    return ev.max() / ev.min()


def test_e1_condition_numbers_match_paper():
    golden = json.load(open(os.path.join(GOLDEN, "paper_condition_numbers.json")))
    for alpha_s, expected in golden["e1_scaling"]["cond_KG"].items():
        X, S = synth.e1_setup(float(alpha_s))
        assert abs(_cond_KG(X, S) - expected) < 1e-5 * expected


def test_e2_condition_number_consistent_with_paper():
    golden = json.load(open(os.path.join(GOLDEN, "paper_condition_numbers.json")))
    printed = golden["e2_monte_carlo"]["cond_KG"]
    X, S = synth.e2_setup()
    c = _cond_KG(X, S)
    # the nonunit spectrum lies inside [0.01, 50] (interlacing), and with
    # m = 80 no eigenvalue of Sigma survives the compression exactly
    assert c < 5000.0 * (1 - 1e-9)
    assert abs(c - printed) / printed < 0.02


# -- P8: unbiasedness of every PCG-Aug iterate (Theorem glmPcgUnbiased) ----

def test_pcg_aug_iterates_unbiased_monte_carlo():
    base = synth.small_batch(seed=31, B=1, G_rng=(3, 3), M_rng=(20, 20),
                             n_rng=(2, 3), K_rng=(1, 1))[0]
    rng = np.random.default_rng(99)
    L = np.linalg.cholesky(base.Omega)
    beta = base.beta_true[:, 0]
    R, iters = 600, (1, 2, 3)
    errs = {i: [] for i in iters}
    fit = gls.fitted(base, base.beta_true)[:, :, 0]
    for _ in range(R):
        E = rng.standard_normal((base.M, base.G)) @ L.T
        inst = synth.SURInstance(base.n_i, base.W, base.Omega,
                                 (fit + E)[:, :, None], base.beta_true)
        for i in iters:
            res = pcg_aug.pcg_aug(inst, tol=0.0, max_iter=i, stall=10**9)
            errs[i].append(res.z_hat - beta)
    for i in iters:
        e = np.array(errs[i])
        z = np.abs(e.mean(0)) / (e.std(0, ddof=1) / np.sqrt(R))
        assert z.max() < 4.0, (i, z)


# -- P9: singular Omega: the noise-free combinations pin beta exactly ---------

def test_singular_omega_recovers_beta_true_and_matches_kkt():
    b = synth.small_batch(seed=41, B=3, G_rng=(4, 5), M_rng=(30, 40),
                          n_rng=(1, 3), K_rng=(1, 2), singular=2)
    for inst in b:
        assert np.linalg.matrix_rank(inst.Omega) == inst.G - 2
        beta, SU = gls.sur_gls_eigsplit(inst)
        assert rel_err(beta, inst.beta_true) < 1e-10
        assert rel_err(SU, inst.noise) < 1e-9
        for k in range(inst.K):
            X, S, y = gls.sur_dense(inst, k)
            w_k, b_k = gls.augmented_lstsq(X, S, y)
            assert rel_err(beta[:, k], b_k) < 1e-9


def test_projected_form_has_the_same_iterates_as_the_algorithm():
    inst = synth.config0()[0]
    a = pcg_aug.pcg_aug(inst, tol=1e-12)
    b = pcg_aug.pcg_aug_projected(inst, tol=1e-12)
    assert a.iterations == b.iterations
    for i in range(8):
        assert abs(a.c[i] - b.c[i]) <= 1e-9 * a.c[i]
        assert abs(a.d[i] - b.d[i]) <= 1e-9 * a.d[i]
        assert abs(a.lam[i] - b.lam[i]) <= 1e-9 * a.lam[i]
    assert rel_err(a.z_hat, b.z_hat) < 1e-12 and rel_err(a.w, b.w) < 1e-11


@pytest.mark.parametrize("G,M,n_rng,k", [(5, 40, (2, 3), 0), (5, 100, (1, 3), 0),
                                         (8, 300, (2, 4), 3)])
def test_projected_pcg_on_singular_omega_reaches_beta_true(G, M, n_rng, k):
    inst = synth.small_batch(seed=42, B=1, G_rng=(G, G), M_rng=(M, M),
                             n_rng=n_rng, K_rng=(1, 1), singular=2,
                             constraints=k)[0]
    res = pcg_aug.pcg_aug_projected(inst, tol=1e-13)
    assert res.status == "converged"
    assert rel_err(res.z_hat, inst.beta_true[:, 0]) < 1e-11


def test_literal_recurrence_loses_accuracy_on_singular_omega():
    """Documents the floating-point failure of the literal recurrence that
    motivates carrying Pi r only (see pcg_aug_projected)."""
    inst = synth.small_batch(seed=42, B=1, G_rng=(5, 5), M_rng=(100, 100),
                             n_rng=(1, 3), K_rng=(1, 1), singular=2)[0]
    res = pcg_aug.pcg_aug(inst, tol=1e-13, stall=10**9, max_iter=120)
    assert res.status != "converged"
    assert rel_err(res.z_hat, inst.beta_true[:, 0]) > 1e-6


# -- P10: restrictions ------------------------------------------------------

def test_selection_restrictions_delete_columns():
    inst = synth.small_batch(seed=51, B=1, G_rng=(3, 3), M_rng=(40, 40),
                             n_rng=(3, 4), K_rng=(2, 2))[0]
    sel = [0, inst.col_off[1] + 1, inst.n - 1]
    inst.Rc = np.eye(inst.n)[sel]
    inst.r = np.zeros((len(sel), inst.K))
    beta_c, _, _ = gls.restricted_gls(inst)
    assert np.abs(beta_c[sel]).max() < 1e-12
    keep = [c for c in range(inst.n) if c not in sel]
    n_new = [sum(1 for c in keep if inst.col_off[i] <= c < inst.col_off[i] + inst.n_i[i])
             for i in range(inst.G)]
    red = synth.SURInstance(n_new, np.ascontiguousarray(inst.W[:, keep]),
                            inst.Omega, inst.Y, inst.beta_true[keep])
    beta_red, _ = gls.sur_gls(red)
    assert rel_err(beta_c[keep], beta_red) < 1e-11


def test_restricted_gls_three_routes():
    b = synth.small_batch(seed=52, B=3, G_rng=(2, 4), M_rng=(10, 30),
                          n_rng=(2, 4), K_rng=(1, 2), constraints=2)
    for inst in b:
        beta_c, U, wc = gls.restricted_gls(inst)
        assert np.abs(inst.Rc @ beta_c - inst.r).max() < 1e-10
        beta_e, SU = gls.sur_gls_eigsplit(inst)
        assert rel_err(beta_e, beta_c) < 1e-10
        for k in range(inst.K):
            X, S, y = gls.sur_dense(inst, k)
            w_k, b_k = gls.augmented_lstsq(X, S, y, inst.Rc, inst.r[:, k])
            assert rel_err(beta_c[:, k], b_k) < 1e-9
            m = X.shape[0]
            assert rel_err(U[:, :, k].T.reshape(-1), w_k[:m]) < 1e-9
            assert rel_err(wc[:, k], w_k[m:]) < 1e-8
        res = pcg_aug.pcg_aug_projected(inst, k=0, tol=1e-13)
        assert rel_err(res.z_hat, beta_c[:, 0]) < 1e-9


def test_singular_and_restricted_together():
    inst = synth.small_batch(seed=53, B=1, G_rng=(5, 5), M_rng=(20, 20),
                             n_rng=(2, 3), K_rng=(1, 1), singular=2,
                             constraints=2)[0]
    beta, SU = gls.sur_gls_eigsplit(inst)
    assert rel_err(beta, inst.beta_true) < 1e-10
    X, S, y = gls.sur_dense(inst, 0)
    _, b_k = gls.augmented_lstsq(X, S, y, inst.Rc, inst.r[:, 0])
    assert rel_err(beta[:, 0], b_k) < 1e-9


# -- P11: gradients against central finite differences -------------------------

def _fd_instance():
    inst = synth.small_batch(seed=61, B=1, G_rng=(3, 3), M_rng=(25, 25),
                             n_rng=(2, 3), K_rng=(1, 1), shift=0.5)[0]
    return inst


def _perturbed(inst, what, idx, h):
    W, Om, Y = inst.W.copy(), inst.Omega.copy(), inst.Y.copy()
    if what == "Y":
        Y[idx] += h
    elif what == "W":
        W[idx] += h
    else:
        i, j = idx
        Om[i, j] += h
        if i != j:
            Om[j, i] += h
    return synth.SURInstance(inst.n_i, W, Om, Y, inst.beta_true)


def _check_fd(inst, loss, grads, coords, h=1e-6):
    dY, dOm, dW = grads
    for what, idx in coords:
        fd = (loss(_perturbed(inst, what, idx, h)) -
              loss(_perturbed(inst, what, idx, -h))) / (2 * h)
        if what == "Y":
            an = dY[idx]
        elif what == "W":
            an = dW[idx]
        else:
            i, j = idx
            an = dOm[i, j] * (1 if i == j else 2)   # symmetric perturbation
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-7, (what, idx, fd, an)


def _coords(inst, rng, count=30):
    out = []
    for _ in range(count):
        kind = rng.integers(3)
        if kind == 0:
            out.append(("Y", (int(rng.integers(inst.M)), int(rng.integers(inst.G)), 0)))
        elif kind == 1:
            out.append(("W", (int(rng.integers(inst.M)), int(rng.integers(inst.n)))))
        else:
            i, j = sorted(rng.integers(inst.G, size=2))
            out.append(("O", (int(i), int(j))))
    return out


def test_vjp_of_linear_functional_matches_fd():
    inst = _fd_instance()
    rng = np.random.default_rng(1)
    gb = rng.standard_normal((inst.n, 1))
    gu = rng.standard_normal(inst.Y.shape)

    def loss(I):
        beta, U = gls.sur_gls(I)
        return float(np.sum(gb * beta) + np.sum(gu * U))

    beta, U = gls.sur_gls(inst)
    grads = grad.sur_gls_vjp(inst, beta, U, gb, gu)
    _check_fd(inst, loss, grads, _coords(inst, rng))


def test_loss_gradient_with_likelihood_term_matches_fd():
    inst = _fd_instance()
    rng = np.random.default_rng(2)
    beta_ref = inst.beta_true

    grads = grad.loss_grad(inst, beta_ref)
    _check_fd(inst, lambda I: grad.loss_value(I, beta_ref), grads, _coords(inst, rng))


# -- planted mistakes: each pin above must fail on a plausible error -----------

def test_planted_mistake_dropped_cross_equation_terms_is_caught():
    inst = _nonsingular_batch()[2]
    assert inst.G > 1

    def wrong_sur_gls(I):   # forgets the off-diagonal blocks of Omega^-1
        Oinv = np.diag(1.0 / np.diag(I.Omega))
        WtW, WtY = gls._cross_products(I)
        A, c = gls._kron_weighted(I, WtW, WtY, Oinv)
        return np.linalg.solve(A, c)

    X, S, y = gls.sur_dense(inst, 0)
    assert rel_err(wrong_sur_gls(inst)[:, 0], gls.gls_dense(X, S, y)) > 1e-6


def test_planted_mistake_wrong_sign_in_restriction_is_caught():
    inst = synth.small_batch(seed=52, B=1, G_rng=(2, 4), M_rng=(10, 30),
                             n_rng=(2, 4), K_rng=(1, 1), constraints=2)[0]
    beta_c, _, _ = gls.restricted_gls(inst)
    Oinv = np.linalg.inv(inst.Omega)
    WtW, WtY = gls._cross_products(inst)
    A, c = gls._kron_weighted(inst, WtW, WtY, Oinv)
    bu = np.linalg.solve(A, c)
    AiRt = np.linalg.solve(A, inst.Rc.T)
    wrong = bu + AiRt @ np.linalg.solve(inst.Rc @ AiRt, inst.Rc @ bu - inst.r)
    assert np.abs(inst.Rc @ wrong - inst.r).max() > 1e-6
    assert np.abs(inst.Rc @ beta_c - inst.r).max() < 1e-10


def test_planted_mistake_unsymmetrised_omega_gradient_is_caught():
    inst = _fd_instance()
    rng = np.random.default_rng(3)
    gb = rng.standard_normal((inst.n, 1))

    def loss(I):
        return float(np.sum(gb * gls.sur_gls(I)[0]))

    beta, U = gls.sur_gls(inst)
    dY, dOm, dW = grad.sur_gls_vjp(inst, beta, U, gb)
    S = np.einsum("tik,tjk->ij", dY, U)
    wrong = (dY, -S, dW)            # -W^T Lambda without symmetrisation
    with pytest.raises(AssertionError):
        _check_fd(inst, loss, wrong, [("O", (0, 1)), ("O", (0, 2)), ("O", (1, 2))])


def test_xv_term_of_residual_update_is_annihilated_by_pi():
    """Pi X = 0 (eq. Xstar), so the X v_i term of the residual update never
    reaches Pi r: the iteration without it produces identical Pi r, c, d and
    w.  This is the identity behind carrying only g = Pi r."""
    inst = synth.config0()[0]
    ops = pcg_aug.SurOperators(inst, pcg_aug.default_alpha(inst.Omega))
    v = np.random.default_rng(4).standard_normal(inst.n)
    assert np.abs(ops.Pi(ops.X(v))).max() < 1e-12 * np.abs(ops.X(v)).max()


def test_planted_mistake_inverted_mu_is_caught():
    inst = synth.config0()[0]
    beta, _ = gls.sur_gls(inst)
    ops = pcg_aug.SurOperators(inst, pcg_aug.default_alpha(inst.Omega))
    y = ops.pack(inst.Y[:, :, 0])
    w = np.zeros(ops.m)
    r = -y
    Pr = ops.Pi(r)
    c = r @ Pr
    u, v = Pr, ops.Xstar_T(r)
    for _ in range(60):
        Su = ops.Sigma(u)
        lam = c / (u @ Su)
        w = w - lam * u
        r = r - lam * (Su + ops.X(v))
        Pr = ops.Pi(r)
        c_new = r @ Pr
        mu = c / c_new                     # planted: should be c_new / c
        v = ops.Xstar_T(r) + mu * v
        u = Pr + mu * u
        c = c_new
    z_wrong = ops.Xstar_T(y - ops.Sigma(w))
    assert rel_err(z_wrong, beta[:, 0]) > 1e-6


# -- SUR model reduction: the reduced route is the GLS of the full model ----------

def test_model_reduction_preserves_gls():
    """The GLS of the reduced model (one QR of W = [X_1 ... X_G]) equals the
    direct GLS of the full model, beta and u, with and without restrictions,
    and when M < n + 1 leaves nothing to drop."""
    from oracle import reduce as ored
    insts = list(synth.small_batch(seed=31, B=4, G_rng=(1, 5), M_rng=(30, 200),
                                   n_rng=(1, 6), K_rng=(1, 3)))
    insts += list(synth.small_batch(seed=33, B=3, G_rng=(2, 4), M_rng=(40, 90),
                                    n_rng=(2, 5), K_rng=(1, 2), constraints=3))
    insts += list(synth.small_batch(seed=35, B=1, G_rng=(6, 6), M_rng=(9, 9),
                                    n_rng=(2, 3), K_rng=(2, 2)))
    for inst in insts:
        Mr = ored.reduced_rows(inst.M, inst.n)
        assert Mr == min(inst.M, inst.n + 1)
        beta_r, U_r = ored.sur_gls_reduced(inst)
        if inst.Rc is not None:
            beta_d, U_d, _ = gls.restricted_gls(inst)
        else:
            beta_d, U_d = gls.sur_gls(inst)
        assert rel_err(beta_r, beta_d) < 1e-11
        assert rel_err(U_r, U_d) < 1e-11


def test_model_reduction_drops_only_noise_rows():
    """Rotated regressors vanish below row n; the dropped rows still carry the
    part of u that the tail term (Q^T Y) Omega^-1 restores: leaving it out
    changes u but not beta."""
    from oracle import reduce as ored
    inst = synth.small_batch(seed=37, B=1, G_rng=(3, 3), M_rng=(60, 60),
                             n_rng=(2, 4), K_rng=(2, 2))[0]
    red, Q, QtY = ored.reduce_instance(inst)
    QtW = Q.T @ inst.W
    assert np.abs(QtW[inst.n:]).max() < 1e-12 * np.abs(inst.W).max()
    assert np.allclose(Q.T @ Q, np.eye(inst.M), atol=1e-13)
    beta_r, Ur = gls.sur_gls(red)
    beta_d, U_d = gls.sur_gls(inst)
    assert rel_err(beta_r, beta_d) < 1e-11
    Z = np.zeros_like(inst.Y)
    Z[:red.M] = Ur
    U_no_tail = np.einsum("ts,sik->tik", Q, Z)
    assert rel_err(U_no_tail, U_d) > 1e-2


# -- restricted gradients: FD of the restricted estimator, dense adjoint --------

def _restricted_fd_instance():
    return synth.small_batch(seed=67, B=1, G_rng=(3, 3), M_rng=(20, 20),
                             n_rng=(2, 3), K_rng=(1, 1), shift=0.5, constraints=2)[0]


def _perturbed_keep_rc(inst, what, idx, h):
    out = _perturbed(inst, what, idx, h)
    out.Rc, out.r = inst.Rc, inst.r
    return out


def test_restricted_vjp_matches_fd_and_dense_adjoint():
    inst = _restricted_fd_instance()
    rng = np.random.default_rng(3)
    gb = rng.standard_normal((inst.n, 1))
    gu = rng.standard_normal(inst.Y.shape)

    def loss(I):
        beta, U, _ = gls.restricted_gls(I)
        return float(np.sum(gb * beta) + np.sum(gu * U))

    beta, U, wc = gls.restricted_gls(inst)
    grads = grad.restricted_gls_vjp(inst, beta, U, gb, gu)
    coords = _coords(inst, rng, count=40)
    for what, idx in coords:
        fd = (loss(_perturbed_keep_rc(inst, what, idx, 1e-6)) -
              loss(_perturbed_keep_rc(inst, what, idx, -1e-6))) / 2e-6
        dY, dOm, dW = grads
        an = dY[idx] if what == "Y" else dW[idx] if what == "W" else \
            dOm[idx] * (1 if idx[0] == idx[1] else 2)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-7, (what, idx, fd, an)
    # the adjoint of the dense restricted augmented system (eq. GRGLM):
    # A [l_w; l_c; l_b] = [g_u; 0; g_b], solved by least squares
    X, S, _ = gls.sur_dense(inst, 0)
    lw, lb = gls.augmented_lstsq(X, S, gu[:, :, 0].T.reshape(-1), inst.Rc,
                                 np.zeros(inst.kc), h2=gb[:, 0])
    m = X.shape[0]
    dY = grads[0][:, :, 0].T.reshape(-1)
    assert rel_err(dY, lw[:m]) < 1e-9
    w = U[:, :, 0].T.reshape(-1)
    dX_dense = -(np.outer(lw[:m], beta[:, 0]) + np.outer(w, lb))
    dW = np.concatenate([dX_dense[i * inst.M:(i + 1) * inst.M,
                                  inst.col_off[i]:inst.col_off[i] + inst.n_i[i]]
                         for i in range(inst.G)], 1)
    assert rel_err(grads[2], dW) < 1e-9


def test_planted_mistake_unrestricted_adjoint_on_restricted_problem_is_caught():
    """The unrestricted adjoint (no KKT rows) is wrong for a restricted
    solution; the finite-difference pin sees it."""
    inst = _restricted_fd_instance()
    rng = np.random.default_rng(4)
    gb = rng.standard_normal((inst.n, 1))

    def loss(I):
        return float(np.sum(gb * gls.restricted_gls(I)[0]))

    beta, U, _ = gls.restricted_gls(inst)
    wrong = grad.sur_gls_vjp(inst, beta, U, gb)
    bad = 0
    for what, idx in _coords(inst, rng, count=30):
        fd = (loss(_perturbed_keep_rc(inst, what, idx, 1e-6)) -
              loss(_perturbed_keep_rc(inst, what, idx, -1e-6))) / 2e-6
        dY, dOm, dW = wrong
        an = dY[idx] if what == "Y" else dW[idx] if what == "W" else \
            dOm[idx] * (1 if idx[0] == idx[1] else 2)
        bad += abs(fd - an) > 1e-6 * abs(an) + 1e-7
    assert bad > 0


# -- per-equation preconditioner D = diag(d) (x) I_M ------------------------------

def test_per_equation_d_diagonal_omega_terminates_in_one_step():
    """With Sigma = D the preconditioner K is the exact inverse of the
    augmented matrix (eq. invprec / eq. prec), so PCG-Aug ends after one
    step, at blockwise OLS; D = alpha I needs one step per distinct
    omega_ii instead."""
    inst = synth.small_batch(seed=5, B=1, G_rng=(3, 3), M_rng=(50, 50),
                             n_rng=(2, 4), K_rng=(2, 2))[0]
    inst.Omega = np.diag([0.7, 1.9, 3.1])
    ols = _blockwise_ols(inst)
    for k in range(inst.K):
        res = pcg_aug.pcg_aug(inst, k=k, tol=1e-13, alpha=pcg_aug.per_equation_d(inst.Omega))
        assert res.status == "converged" and res.iterations == 1, res.iterations
        assert rel_err(res.z_hat, ols[:, k]) < 1e-12
        resp = pcg_aug.pcg_aug_projected(inst, k=k, tol=1e-13,
                                         alpha=pcg_aug.per_equation_d(inst.Omega))
        assert resp.iterations == 1 and rel_err(resp.z_hat, ols[:, k]) < 1e-12
        res_a = pcg_aug.pcg_aug(inst, k=k, tol=1e-13)
        assert res_a.iterations == inst.G


def test_per_equation_d_leaves_beta_unchanged():
    """beta does not depend on D (X* is D-free for block-diagonal X)."""
    for inst in _nonsingular_batch()[:3]:
        beta, U = gls.sur_gls(inst)
        d = pcg_aug.per_equation_d(inst.Omega)
        for k in range(inst.K):
            res = pcg_aug.pcg_aug_projected(inst, k=k, tol=1e-13, alpha=d)
            assert rel_err(res.z_hat, beta[:, k]) < 1e-10
            assert rel_err(res.w, U[:, :, k].T.reshape(-1)) < 1e-9


def test_planted_mistake_scalar_norm_with_per_equation_d_is_caught():
    """c = alpha ||Pi r||^2 is right only for D = alpha I; with a per-equation
    D the projected form must use g^T D g.  Using the scalar form breaks
    the one-step termination of the diagonal case."""
    inst = synth.small_batch(seed=5, B=1, G_rng=(3, 3), M_rng=(50, 50),
                             n_rng=(2, 4), K_rng=(1, 1))[0]
    inst.Omega = np.diag([0.7, 1.9, 3.1])
    d = pcg_aug.per_equation_d(inst.Omega)
    ops = pcg_aug.SurOperators(inst, d)
    y = ops.pack(inst.Y[:, :, 0])
    g = ops.Pi(-y)
    c_right = ops.Dnorm2(g)
    c_wrong = float(d.max() * (g @ g))
    u = g
    lam_right = c_right / float(u @ ops.Sigma(u))
    lam_wrong = c_wrong / float(u @ ops.Sigma(u))
    g1 = g - lam_right * ops.Pi(ops.Sigma(u))
    g1w = g - lam_wrong * ops.Pi(ops.Sigma(u))
    assert np.linalg.norm(g1) < 1e-12 * np.linalg.norm(g)
    assert np.linalg.norm(g1w) > 1e-3 * np.linalg.norm(g)


# -- PCG-NE: CG on the normal equations (the Monte Carlo comparator) -----------

def test_pcg_ne_converges_to_gls_with_monotone_a_norm_error():
    from oracle import pcg_ne
    for inst in _nonsingular_batch()[:3]:
        beta, _ = gls.sur_gls(inst)
        A, b, _ = pcg_ne.normal_system(inst, 0)
        for precond in ("block", "none"):
            res = pcg_ne.pcg_ne(inst, tol=1e-13, precond=precond, keep=True,
                                max_iter=4 * inst.n)
            assert res.status == "converged", (precond, res.status)
            assert rel_err(res.beta, beta[:, 0]) < 1e-10
            errs = [float((x - beta[:, 0]) @ A @ (x - beta[:, 0])) for x in res.iterates]
            assert all(e2 <= e1 * (1 + 1e-8) + 1e-18 for e1, e2 in zip(errs, errs[1:]))


def test_pcg_ne_block_jacobi_on_diagonal_omega_is_one_step_ols():
    """A diagonal Omega makes the normal matrix block diagonal, which the
    block-Jacobi preconditioner inverts exactly: one step, at blockwise OLS."""
    from oracle import pcg_ne
    inst = synth.small_batch(seed=5, B=1, G_rng=(3, 3), M_rng=(50, 50),
                             n_rng=(2, 4), K_rng=(1, 1))[0]
    inst.Omega = np.diag([0.7, 1.9, 3.1])
    res = pcg_ne.pcg_ne(inst, tol=1e-13)
    assert res.iterations == 1 and rel_err(res.beta, _blockwise_ols(inst)[:, 0]) < 1e-12


def test_pcg_ne_early_iterates_are_biased_unlike_pcg_aug():
    """Started from beta_0 = 0, the CG iterates on the normal equations are
    shrunk toward 0 (biased), while PCG-Aug's estimate is unbiased at every
    iteration (Theorem on the unbiasedness of the PCG-Aug iterates)."""
    from oracle import pcg_ne
    base = synth.small_batch(seed=73, B=1, G_rng=(3, 3), M_rng=(40, 40), n_rng=(2, 3),
                             K_rng=(1, 1), shift=0.5)[0]
    base.beta_true[:, 0] = 3.0 + np.arange(base.n)          # far from the start point 0
    rng = np.random.default_rng(11)
    L = np.linalg.cholesky(base.Omega)
    fit = gls.fitted(base, base.beta_true)[:, :, 0]
    R = 400
    e_ne, e_aug = [], []
    for _ in range(R):
        E = rng.standard_normal((base.M, base.G)) @ L.T
        inst = synth.SURInstance(base.n_i, base.W, base.Omega, (fit + E)[:, :, None],
                                 base.beta_true)
        e_ne.append(pcg_ne.pcg_ne(inst, tol=0.0, max_iter=1, precond="none").beta -
                    base.beta_true[:, 0])
        e_aug.append(pcg_aug.pcg_aug(inst, tol=0.0, max_iter=1, stall=10**9).z_hat -
                     base.beta_true[:, 0])
    for e, biased in ((np.array(e_ne), True), (np.array(e_aug), False)):
        z = np.abs(e.mean(0)) / (e.std(0, ddof=1) / np.sqrt(R))
        if biased:
            assert z.max() > 10.0, z
        else:
            assert z.max() < 4.0, z


def test_oracle_gls_is_scale_equivariant():
    """X -> X S (S diagonal: one factor for all columns, 1e-140 or 1e150, or
    one per column in [1e-120, 1e120]) with R_c -> R_c S maps the GLS
    estimate to S^-1 beta and leaves u unchanged: the oracle meets this at
    rounding level far outside the range where squared entries stay finite."""
    import copy
    insts = list(synth.small_batch(seed=601, B=3, G_rng=(2, 6), M_rng=(30, 300),
                                   n_rng=(2, 6), K_rng=(1, 3)))
    insts += list(synth.small_batch(seed=603, B=2, G_rng=(2, 5), M_rng=(40, 200),
                                    n_rng=(2, 5), K_rng=(1, 2), constraints=2))
    rng = np.random.default_rng(5)
    for inst in insts:
        b0, U0, _ = gls.sur_solution(inst)
        for sc in (np.full(inst.n, 1e-140), np.full(inst.n, 1e150),
                   10.0 ** rng.uniform(-120, 120, inst.n)):
            si = copy.deepcopy(inst)
            si.W = si.W * sc
            if si.Rc is not None:
                si.Rc = si.Rc * sc
            b1, U1, _ = gls.sur_solution(si)
            assert rel_err(b1 * sc[:, None], b0) < 1e-12
            assert rel_err(U1, U0) < 1e-12


def test_mvrglm_sur_form_is_the_restricted_gls_and_reduction_keeps_it():
    """Exclusion-restricted multivariate model: the SUR with kept columns and
    the full model with the exclusions as restriction rows give the same
    estimate; the reduced model (Q0^T Y with R0's kept columns) gives it too;
    and it differs from equation-wise OLS (the restrictions matter)."""
    from oracle import mvrglm
    for lam, sp in ((0.9, 0.26), (1.05, 0.8)):
        inst = synth.mvrglm_var(seed=33, B=1, K=2, G=4, M=80, N=10, sparsity=sp,
                                lam_max=lam, omega_cond=50.0)[0]
        b_sur, U_sur = mvrglm.mvrglm_gls(inst)
        full = mvrglm.full_restricted_form(inst)
        b_full, U_full, _ = gls.restricted_gls(full)
        assert rel_err(mvrglm.kept(inst, b_full), b_sur) < 1e-10
        assert rel_err(U_full, U_sur) < 1e-10
        excl = np.ones(inst.G * inst.N, bool)
        for j, sel in enumerate(inst.sel):
            excl[j * inst.N + sel] = False
        assert np.abs(b_full[excl]).max() < 1e-10 * np.abs(b_full).max()
        b_red, _ = gls.sur_gls(mvrglm.reduced_form(inst))
        assert rel_err(b_red, b_sur) < 1e-10
        if lam < 1.0:
            b_w, U_w = mvrglm.mvrglm_gls_whitened(inst)
            assert rel_err(b_w, b_sur) < 1e-10 and rel_err(U_w, U_sur) < 1e-10
        assert rel_err(mvrglm.equationwise_ols(inst), b_sur) > 1e-6


def test_var_regressors_have_the_requested_largest_root():
    """The generated VAR(4) regressors grow like lam_max^t when the largest
    root is explosive (1.05: about 1.7e4 over 200 steps, up to transients)
    and stay bounded when it is stationary (0.9)."""
    rng = np.random.default_rng(3)
    z = synth.var_regressors(rng, 400, 6, lam_max=1.05)
    n1, n2 = np.linalg.norm(z[199]), np.linalg.norm(z[399])
    # an explosive root 1.05 grows the state by about 1.05^200 = 1.7e4 over
    # 200 steps (up to the transient), a stationary one would not
    assert 1e3 < n2 / n1 < 1e6
    z = synth.var_regressors(np.random.default_rng(4), 400, 6, lam_max=0.9)
    assert np.linalg.norm(z[399]) / np.linalg.norm(z[199]) < 50.0
