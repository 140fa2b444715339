"""Multivariate linear model with exclusion restrictions (section on
multivariate linear models with parameter restrictions, eq. MvGLM):

    Y = Z0 B + U,   vec(U) ~ (0, Omega0 (x) I_M),   b_ij = 0 for (i, j) in S.

Without restrictions OLS and GLS coincide; exclusions break that.  Equation
j then has the free coefficients of the columns sel_j of Z0, which makes the
model a SUR with X_j = Z0[:, sel_j]: its GLS estimate is the restricted GLS
estimate of the multivariate model (the excluded coefficients are zero).

Model reduction (same section): with the thin QR Z0 = Q0 R0 (R0 N x N),
Q0^T Y = R0 B + Q0^T U, and vec(Q0^T U) ~ (0, Omega0 (x) I_N); the reduced
model has N rows per equation and the same GLS estimate.  In SUR form its
regressors are X_j,red = R0[:, sel_j].

TEST INFRASTRUCTURE: used by the tests and never by the product package.
The GLS solves are oracle.gls (closed forms on dense numpy/scipy algebra).

Parity status: pinned by tests/test_oracle_pins.py (the SUR form agrees with
the restricted GLS of the full multivariate model, whose exclusions are
explicit restriction rows; the reduced model gives the same estimate; the
whitened least-squares route agrees on well-conditioned regressors; the
restricted estimate differs from equation-wise OLS).
"""
from __future__ import annotations

import copy

import numpy as np
import scipy.linalg as sla

from . import gls


def sur_form(inst):
    """The SUR with X_j = Z0[:, sel_j] (the instance's own column selection)."""
    return inst.to_sur()


def mvrglm_gls(inst):
    """(beta of the kept coefficients, equation-major, n x K; U, M x G x K)."""
    return gls.sur_gls(sur_form(inst))


def mvrglm_gls_whitened(inst):
    """The same estimate by least squares on the whitened model: with
    Omega = L L^T, (L^-1 (x) I_M) y = (L^-1 (x) I_M) X beta + white noise, solved
    by numpy's SVD least squares, whose error grows like cond(X) rather than
    cond(X)^2 (for regressors too ill-conditioned for the normal equations).
    Returns (beta n x K, U M x G x K) with U = (Y - fitted) Omega^-1."""
    sur = sur_form(inst)
    G, M, K = inst.G, inst.M, inst.K
    L = np.linalg.cholesky(inst.Omega)
    Li = sla.solve_triangular(L, np.eye(G), lower=True)
    X = sla.block_diag(*[sur.X(i) for i in range(G)])          # (G M) x n, equation-major rows
    Xw = np.kron(Li, np.eye(M)) @ X
    beta = np.empty((sur.n, K))
    for k in range(K):
        yw = (inst.Y[:, :, k] @ Li.T).T.reshape(-1)
        beta[:, k] = np.linalg.lstsq(Xw, yw, rcond=None)[0]
    E = inst.Y - gls.fitted(sur, beta)
    Oinv = Li.T @ Li
    U = np.einsum("tik,ij->tjk", E, Oinv)
    return beta, U


def full_restricted_form(inst):
    """The same model with all N columns in every equation and the
    exclusions as restriction rows e_(j, c)^T beta = 0 (R_c beta = r)."""
    s = copy.deepcopy(sur_form(inst))
    G, N = inst.G, inst.N
    s.n_i = [N] * G
    s.W = np.concatenate([inst.Z0] * G, axis=1)
    rows = []
    for j, sel in enumerate(inst.sel):
        for c in sorted(set(range(N)) - set(int(v) for v in sel)):
            e = np.zeros(G * N)
            e[j * N + c] = 1.0
            rows.append(e)
    s.Rc = np.array(rows).reshape(len(rows), G * N)
    s.r = np.zeros((len(rows), inst.K))
    s.beta_true = np.repeat(inst.B_true.T.reshape(-1)[:, None], inst.K, axis=1)
    return s


def kept(inst, beta_full):
    """The kept coefficients (equation-major) of a full G N x K estimate."""
    N = inst.N
    return np.concatenate([beta_full[j * N + sel] for j, sel in enumerate(inst.sel)])


def reduced_form(inst):
    """The reduced model: Q0^T Y (N rows) with X_j,red = R0[:, sel_j]."""
    Q0, R0 = sla.qr(inst.Z0, mode="economic")
    s = copy.deepcopy(sur_form(inst))
    s.W = np.concatenate([R0[:, sel] for sel in inst.sel], axis=1)
    s.Y = np.einsum("tn,tik->nik", Q0, inst.Y)
    return s


def equationwise_ols(inst):
    """OLS of each equation on its kept columns (n x K)."""
    out = []
    for j, sel in enumerate(inst.sel):
        Xj = inst.Z0[:, sel]
        out.append(np.linalg.lstsq(Xj, inst.Y[:, j, :], rcond=None)[0])
    return np.concatenate(out, axis=0)
