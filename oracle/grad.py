"""Dense reference gradients of the SUR GLS solution (nonsingular Omega).

The solution x = [w; b] of eq. aug1,  A x = h  with the symmetric matrix
A = [[Sigma, X], [X^T, 0]] and h = [y; 0], has the reverse-mode rule

    lambda = A^-1 [g_w; g_b]            (A is symmetric, so A^-T = A^-1)
    dL/dy  = lambda_w
    dL/dA  = -lambda x^T,

and A depends on Omega through Sigma = Omega (x) I_M and on X through
both off-diagonal blocks.  Collecting the entries:

    dL/dOmega_ij = -sum_t lambda_w[t,i] w[t,j]   -> symmetrised for a symmetric Omega
    dL/dX_i      = -(lambda_w,i b_i^T + w_i lambda_b,i^T).

For nonsingular Omega the adjoint system is solved in closed form:
lambda_b = (X^T Sigma^-1 X)^-1 (X^T Sigma^-1 g_w - g_b),
lambda_w = Sigma^-1 (g_w - X lambda_b).

Symmetric convention: dOmega is returned symmetric, with dL = <dOmega, E>_F
for every symmetric perturbation E.

With restrictions R_c b = r (eq. GRGLM: the restriction rows are extra
observations of zero variance), x = [w; w_c; b] and the same rule holds:
A = [[Sigmabar, Xbar], [Xbar^T, 0]] with Xbar = [X; R_c], Sigmabar =
diag(Sigma, 0).  Sigma and X enter A exactly as before, so dL/dy, dL/dOmega
and dL/dX keep the formulas above with the restricted solution (w, b) and
the restricted adjoint (lambda_w, lambda_b); the adjoint of nonsingular
Omega is the (n + k) x (n + k) KKT system

    [ X^T Sigma^-1 X   -R_c^T ] [lambda_b]   [ X^T Sigma^-1 g_w - g_b ]
    [ R_c                0    ] [lambda_c] = [ 0                      ],

lambda_w = Sigma^-1 (g_w - X lambda_b)   (the first rows of A lambda = g and
its restriction rows R_c lambda_b = 0).

Parity status: pinned against central finite differences of the direct
estimators, and the restricted adjoint against the dense augmented system
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .gls import _cross_products, _kron_weighted, fitted, sur_gls


def sur_gls_vjp(inst, beta, U, g_beta, g_u=None):
    """Vector-Jacobian product of (beta, U) = GLS(y, Omega, X) for all K
    right-hand sides.  Returns (dY M x G x K, dOmega G x G, dW M x n)."""
    G, M, K = inst.G, inst.M, inst.K
    Oinv = sla.cho_solve(sla.cho_factor(inst.Omega), np.eye(G))
    WtW, WtY = _cross_products(inst)
    A, _ = _kron_weighted(inst, WtW, WtY, Oinv)
    if g_u is None:
        g_u = np.zeros_like(inst.Y)
    # X^T Sigma^-1 g_u, blockwise
    Gs = np.einsum("tik,ij->tjk", g_u, Oinv)
    XtSg = np.concatenate([inst.X(i).T @ Gs[:, i, :] for i in range(G)], 0)
    lam_b = sla.cho_solve(sla.cho_factor(A), XtSg - g_beta)
    lam_w = np.einsum("tik,ij->tjk", g_u - fitted(inst, lam_b), Oinv)
    dY = lam_w
    S = np.einsum("tik,tjk->ij", lam_w, U)
    dOmega = -0.5 * (S + S.T)
    dW = np.empty_like(inst.W)
    for i in range(G):
        o, ni = inst.col_off[i], inst.n_i[i]
        dW[:, o:o + ni] = -(lam_w[:, i, :] @ beta[o:o + ni, :].T
                            + U[:, i, :] @ lam_b[o:o + ni, :].T)
    return dY, dOmega, dW


def _grads_from_adjoint(inst, beta, U, lam_w, lam_b):
    """dY, dOmega (symmetric), dW from the solution (U, beta) and the adjoint."""
    S = np.einsum("tik,tjk->ij", lam_w, U)
    dOmega = -0.5 * (S + S.T)
    dW = np.empty_like(inst.W)
    for i in range(inst.G):
        o, ni = inst.col_off[i], inst.n_i[i]
        dW[:, o:o + ni] = -(lam_w[:, i, :] @ beta[o:o + ni, :].T
                            + U[:, i, :] @ lam_b[o:o + ni, :].T)
    return lam_w, dOmega, dW


def restricted_gls_vjp(inst, beta, U, g_beta, g_u=None):
    """Vector-Jacobian product of the restricted GLS solution (beta, U) of
    eq. GRGLM (nonsingular Omega, R_c of full row rank) for all K right-hand
    sides, through the KKT form of the adjoint system in the module
    docstring.  Returns (dY M x G x K, dOmega G x G, dW M x n); the
    gradients w.r.t. R_c and r are not formed."""
    G, K, n, kc = inst.G, inst.K, inst.n, inst.kc
    Oinv = sla.cho_solve(sla.cho_factor(inst.Omega), np.eye(G))
    WtW, WtY = _cross_products(inst)
    A, _ = _kron_weighted(inst, WtW, WtY, Oinv)
    if g_u is None:
        g_u = np.zeros_like(inst.Y)
    Gs = np.einsum("tik,ij->tjk", g_u, Oinv)
    XtSg = np.concatenate([inst.X(i).T @ Gs[:, i, :] for i in range(G)], 0)
    kkt = np.zeros((n + kc, n + kc))
    kkt[:n, :n] = A
    kkt[:n, n:] = -inst.Rc.T
    kkt[n:, :n] = inst.Rc
    rhs = np.zeros((n + kc, K))
    rhs[:n] = XtSg - g_beta
    lam_b = np.linalg.solve(kkt, rhs)[:n]
    lam_w = np.einsum("tik,ij->tjk", g_u - fitted(inst, lam_b), Oinv)
    return _grads_from_adjoint(inst, beta, U, lam_w, lam_b)


def nll_omega(inst, beta):
    """Gaussian negative log-likelihood in Omega without constants,
    1/2 [M log det Omega + tr(Omega^-1 E^T E)], E = Y - X beta (one RHS)."""
    E = (inst.Y - fitted(inst, beta))[:, :, 0]
    sign, logdet = np.linalg.slogdet(inst.Omega)
    assert sign > 0
    return 0.5 * (inst.M * logdet + np.trace(np.linalg.solve(inst.Omega, E.T @ E)))


def loss_value(inst, beta_ref):
    """L = 1/2 ||b_GLS - beta_ref||^2 + nll_omega(b_GLS) for K = 1."""
    beta, _ = sur_gls(inst)
    return 0.5 * float(np.sum((beta - beta_ref) ** 2)) + nll_omega(inst, beta)


def loss_grad(inst, beta_ref):
    """Gradient of loss_value w.r.t. (Y, Omega, W).

    The likelihood term contributes directly (dY += u, dX_i += -u_i b_i^T,
    dOmega += 1/2 (M Omega^-1 - Omega^-1 E^T E Omega^-1)); its path through
    b vanishes at the GLS solution (normal equations), so only the
    quadratic term is propagated through the solve with g_b = b - beta_ref."""
    beta, U = sur_gls(inst)
    dY, dOm, dW = sur_gls_vjp(inst, beta, U, beta - beta_ref)
    E = (inst.Y - fitted(inst, beta))[:, :, 0]
    Oinv = np.linalg.inv(inst.Omega)
    dY = dY + U
    for i in range(inst.G):
        o, ni = inst.col_off[i], inst.n_i[i]
        dW[:, o:o + ni] -= U[:, i, :] @ beta[o:o + ni, :].T
    dOm = dOm + 0.5 * (inst.M * Oinv - Oinv @ (E.T @ E) @ Oinv)
    dOm = 0.5 * (dOm + dOm.T)
    return dY, dOm, dW
