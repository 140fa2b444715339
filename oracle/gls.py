"""Direct FP64 estimators: the plain definition of what PCG-Aug converges to.

PCG-Aug terminates, in exact arithmetic, at the solution of the augmented
system (Section "Augmented System formulation", eq. aug1)

    [ Sigma  X ] [ w ]   [ y ]
    [ X^T    0 ] [ b ] = [ 0 ]

whose b-block is the GLS estimator (eq. GLS) when Sigma is nonsingular,
and whose w satisfies  Sigma w = y - X b,  X^T w = 0.  With linear
restrictions C b = gamma the system is eq. GRGLM (restricted GLM section):
the restrictions enter as k extra observations with zero variance.

Every routine here is a textbook direct method, written for readability,
and uses LAPACK through numpy/scipy as its only primitives.

Parity status
  gls_dense, augmented_lstsq, aug_blue_closed_form, sur_gls,
  sur_gls_eigsplit, restricted_gls  -- pinned by tests/test_oracle_pins.py
  (cross-route agreement, special cases that reduce to OLS, exact rational
  PCG-Aug, beta = beta_true for singular Omega, selection constraints).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# --------------------------------------------------------------------------
# dense GLM helpers (tiny sizes only)
# --------------------------------------------------------------------------

def sur_dense(inst, k=0):
    """Dense (X, Sigma, y) of one right-hand side of a SUR instance.

    vec layout: y = vec(Y) stacks the equations, X = direct sum of the X_i,
    Sigma = Omega (x) I_M (SUR section, eq. SURdefs)."""
    M, G = inst.M, inst.G
    X = sla.block_diag(*[inst.X(i) for i in range(G)])
    Sigma = np.kron(inst.Omega, np.eye(M))
    y = inst.Y[:, :, k].T.reshape(-1)  # column i of Y is equation i
    return X, Sigma, y


def gls_dense(X, Sigma, y):
    """b_GLS = (X^T Sigma^-1 X)^-1 X^T Sigma^-1 y  (eq. GLS), Sigma nonsingular."""
    Si_X = np.linalg.solve(Sigma, X)
    Si_y = np.linalg.solve(Sigma, y)
    return np.linalg.solve(X.T @ Si_X, X.T @ Si_y)


def augmented_matrix(X, Sigma, C=None):
    """Coefficient matrix of eq. aug1, or of eq. GRGLM when C is given."""
    m, n = X.shape
    if C is None:
        return np.block([[Sigma, X], [X.T, np.zeros((n, n))]])
    k = C.shape[0]
    Xb = np.vstack([X, C])
    Sb = np.zeros((m + k, m + k))
    Sb[:m, :m] = Sigma
    return np.block([[Sb, Xb], [Xb.T, np.zeros((n, n))]])


def augmented_lstsq(X, Sigma, y, C=None, gamma=None, h2=None):
    """Brute-force solve of the augmented system (eq. aug1 / eq. GRGLM) with a
    minimum-norm least-squares solver (SVD), which also handles a singular
    but consistent system.  ``h2`` is an optional nonzero lower right-hand
    side.  Returns (w, b) with w of length m (+k with restrictions)."""
    m, n = X.shape
    A = augmented_matrix(X, Sigma, C)
    top = y if C is None else np.concatenate([y, gamma])
    low = np.zeros(n) if h2 is None else h2
    sol = np.linalg.lstsq(A, np.concatenate([top, low]), rcond=None)[0]
    return sol[:-n], sol[-n:]


def aug_blue_closed_form(X, Sigma, y):
    """Lemma AugBLUE: with the full QR  Q^T X = [R; 0],  Q = [Q_R Q_N],

        w = Q_N (Q_N^T Sigma Q_N)^-1 Q_N^T y,
        b = R^-1 Q_R^T P_N y,   P_N = I - Sigma Q_N (Q_N^T Sigma Q_N)^-1 Q_N^T.
    """
    m, n = X.shape
    Q, R = np.linalg.qr(X, mode="complete")
    QR_, QN = Q[:, :n], Q[:, n:]
    R = R[:n, :]
    S = QN.T @ Sigma @ QN
    w = QN @ np.linalg.solve(S, QN.T @ y)
    PN_y = y - Sigma @ (QN @ np.linalg.solve(S, QN.T @ y))
    b = sla.solve_triangular(R, QR_.T @ PN_y)
    return w, b


# --------------------------------------------------------------------------
# structured SUR estimators (any size)
# --------------------------------------------------------------------------

def _cross_products(inst):
    """W^T W (n x n) and W^T Y (n x G x K), W = [X_1 ... X_G]."""
    W = inst.W
    WtW = W.T @ W
    M, G, K = inst.Y.shape
    WtY = (W.T @ inst.Y.reshape(M, G * K)).reshape(-1, G, K)
    return WtW, WtY


def _kron_weighted(inst, WtW, WtY, Wt):
    """Blocks [Wt_il X_i^T X_l] and [sum_l Wt_il X_i^T y_l] for a G x G weight."""
    off, n_i, G = inst.col_off, inst.n_i, inst.G
    n, K = inst.n, inst.K
    A = np.empty((n, n))
    c = np.zeros((n, K))
    for i in range(G):
        si = slice(off[i], off[i] + n_i[i])
        for l in range(G):
            sl = slice(off[l], off[l] + n_i[l])
            A[si, sl] = Wt[i, l] * WtW[si, sl]
            c[si, :] += Wt[i, l] * WtY[si, l, :]
    return A, c


def fitted(inst, beta):
    """[X_i beta_i]_i as an M x G x K array."""
    M, G, K = inst.Y.shape
    out = np.empty((M, G, K))
    for i in range(G):
        o, ni = inst.col_off[i], inst.n_i[i]
        out[:, i, :] = inst.X(i) @ beta[o:o + ni, :]
    return out


def sur_gls(inst):
    """Textbook SUR GLS for nonsingular Omega (Introduction; SUR section).

    Sigma^-1 = Omega^-1 (x) I_M, so X^T Sigma^-1 X = [w^{il} X_i^T X_l] and
    X^T Sigma^-1 y = [sum_l w^{il} X_i^T y_l] with [w^{il}] = Omega^-1;
    beta solves that SPD system by Cholesky.  u = Sigma^-1 (y - X beta), i.e.
    U = E_hat Omega^-1 row by row.

    Returns (beta n x K, U M x G x K)."""
    Oinv = sla.cho_solve(sla.cho_factor(inst.Omega), np.eye(inst.G))
    WtW, WtY = _cross_products(inst)
    A, c = _kron_weighted(inst, WtW, WtY, Oinv)
    beta = sla.cho_solve(sla.cho_factor(A), c)
    E = inst.Y - fitted(inst, beta)
    U = np.einsum("tik,ij->tjk", E, Oinv)
    return beta, U


def restricted_gls(inst):
    """Restricted GLS closed form for nonsingular Omega and C beta = gamma
    (here R_c beta = r):  beta_c = beta - A^-1 R_c^T (R_c A^-1 R_c^T)^-1 (R_c beta - r),
    with A = X^T Sigma^-1 X and beta the unrestricted GLS estimate.
    u = Sigma^-1 (y - X beta_c); multipliers w_c solve R_c^T w_c = -X^T u.

    Returns (beta, U, w_c)."""
    Oinv = sla.cho_solve(sla.cho_factor(inst.Omega), np.eye(inst.G))
    WtW, WtY = _cross_products(inst)
    A, c = _kron_weighted(inst, WtW, WtY, Oinv)
    cf = sla.cho_factor(A)
    beta_u = sla.cho_solve(cf, c)
    Rc, r = inst.Rc, inst.r
    AiRt = sla.cho_solve(cf, Rc.T)
    beta = beta_u - AiRt @ np.linalg.solve(Rc @ AiRt, Rc @ beta_u - r)
    E = inst.Y - fitted(inst, beta)
    U = np.einsum("tik,ij->tjk", E, Oinv)
    XtU = np.concatenate([inst.X(i).T @ U[:, i, :] for i in range(inst.G)], 0)
    wc = np.linalg.lstsq(Rc.T, -XtU, rcond=None)[0]
    return beta, U, wc


def sur_gls_eigsplit(inst, tau=1e-10):
    """Structured direct method for singular Omega and/or restrictions.

    Following the restricted-GLM idea of treating zero-variance observations
    as equality restrictions: with Omega = V diag(lam) V^T, the rotated
    equations along eigenvectors with lam_j <= tau * lam_max carry no noise,
    so  sum_i V_ij X_i beta_i = Y v_j  holds exactly; they are stacked with
    R_c beta = r into E beta = e.  The remaining directions give the
    weighted normal matrix P = [(Omega^+)_il X_i^T X_l], p likewise.  beta
    minimises 1/2 b^T P b - p^T b subject to E b = e (null-space method on
    E^T E).  For nonsingular Omega and no restrictions this is plain GLS.

    Returns (beta n x K, Sigma u = Y - X beta as M x G x K)."""
    lam, V = np.linalg.eigh(inst.Omega)
    pos = lam > tau * lam.max()
    Vp, lp, V0 = V[:, pos], lam[pos], V[:, ~pos]
    Oplus = (Vp / lp) @ Vp.T
    P0 = V0 @ V0.T
    WtW, WtY = _cross_products(inst)
    P, p = _kron_weighted(inst, WtW, WtY, Oplus)
    EG, eG = _kron_weighted(inst, WtW, WtY, P0)
    if inst.Rc is not None:
        EG = EG + inst.Rc.T @ inst.Rc
        eG = eG + inst.Rc.T @ inst.r
    n = inst.n
    if V0.shape[1] == 0 and inst.Rc is None:
        beta = sla.cho_solve(sla.cho_factor(P), p)
    else:
        ev, Ue = np.linalg.eigh(EG)
        rng_ = ev > 1e-12 * max(ev.max(), 1e-300)
        Ur, er = Ue[:, rng_], ev[rng_]
        beta_p = Ur @ ((Ur.T @ eG) / er[:, None])
        NE = Ue[:, ~rng_]
        if NE.shape[1] > 0:
            red = NE.T @ P @ NE
            beta = beta_p + NE @ np.linalg.solve(red, NE.T @ (p - P @ beta_p))
        else:
            beta = beta_p
    assert beta.shape[0] == n
    SigmaU = inst.Y - fitted(inst, beta)
    return beta, SigmaU


def sur_solution(inst):
    """Dispatch: (beta, U or None, Sigma U).  U is returned only where it is
    unique (nonsingular Omega); the multipliers of restrictions are omitted."""
    lam = np.linalg.eigvalsh(inst.Omega)
    singular = lam[0] <= 1e-10 * lam[-1]
    if singular:
        beta, SU = sur_gls_eigsplit(inst)
        return beta, None, SU
    if inst.Rc is not None:
        beta, U, _ = restricted_gls(inst)
    else:
        beta, U = sur_gls(inst)
    SU = np.einsum("tik,ij->tjk", U, inst.Omega)
    return beta, U, SU
