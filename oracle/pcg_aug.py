"""The PCG-Aug iteration, written in the paper's order and notation.

This is Algorithm "The PCG-Aug method" (alg. glmpcg2) applied to the
augmented system of eq. aug1 with the indefinite preconditioner of
eq. invprec / eq. prec.  The auxiliary matrix D is either alpha I or, for a
SUR model, one scalar per equation, D = diag(d_1..d_G) (x) I_M (the VAR
experiments use both: D_1 = alpha I and D_2 = diag Sigma).  For a SUR model
X is block diagonal, so in both cases

    X* = D^-1 X (X^T D^-1 X)^-1 = X (X^T X)^-1          (D cancels blockwise),
    Pi = (I - X* X^T) D^-1,  block i:  (I - X_i (X_i^T X_i)^-1 X_i^T) / d_i,

so that X*^T r and Pi r are the OLS estimate and the residual (scaled by
1/d_i) of an auxiliary regression of r on X (the "auxiliary GLM").
Both operators act block by block through thin QR factors X_i = Q_i R_i:
X_i*^T xi = R_i^-1 Q_i^T xi, Pi_i xi = (xi - Q_i Q_i^T xi) / d_i, and
Sigma u = vec(U Omega).
With restrictions (restricted GLM section) the restrictions are k extra
observations of zero variance: Xbar = [X; R_c], Sigmabar = diag(Sigma, 0),
D = alpha I_{m+k}, and X*, Pi follow eq. rglm1m (the per-equation D is
offered for unrestricted instances only).

Iterates kept exactly as in the algorithm: residual r, search direction
blocks u (w-space) and v (z-space), scalars c, d, lambda, mu; the
estimate is recovered at termination as  z_hat = X*^T (y - Sigma w).

A nonzero lower right-hand side h2 (needed by iterative refinement and by
the adjoint solve) is handled by starting from w_1 = X* h2, which gives
X^T w_1 = h2 because X^T X* = I; the lower block of the PCG residual is
then zero and the algorithm is unchanged.

The exact-arithmetic variant runs the same steps on Fractions for tiny
integer data (D = I) and stops when c becomes exactly zero.

Parity status: pinned (finite termination in exact arithmetic at the
number of distinct eigenvalues; agreement with the direct estimators;
error norm monotonicity; X^T w_i = 0; unbiasedness at every iteration).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional

import numpy as np
import scipy.linalg as sla


class SurOperators:
    """Sigma, X, X^T, X*^T, X*, Pi for one SUR instance (optionally restricted).

    Vectors in observation space are flat: vec(U) (equation-major, length
    G*M) followed by the k restriction entries."""

    def __init__(self, inst, alpha):
        self.inst = inst
        self.M, self.G, self.n = inst.M, inst.G, inst.n
        self.kc = inst.kc
        self.m = self.G * self.M + self.kc
        d = np.asarray(alpha, dtype=np.float64)
        if d.ndim == 0:
            d = np.full(self.G, float(d))
        if d.shape != (self.G,) or not np.all(d > 0):
            raise ValueError("D needs one positive scalar, or one per equation")
        if self.kc and not np.all(d == d[0]):
            raise ValueError("restricted instances take D = alpha I")
        self.d = d
        # the diagonal of D over the observation space (restriction rows: d_1)
        self.Ddiag = np.concatenate([np.repeat(d, self.M), np.full(self.kc, d[0])])
        self.QR = [np.linalg.qr(inst.X(i)) for i in range(self.G)]
        if self.kc:
            # X^T X + R_c^T R_c (the D's cancel when D_Z = D_C = alpha I)
            N = sla.block_diag(*[inst.X(i).T @ inst.X(i) for i in range(self.G)])
            N = N + inst.Rc.T @ inst.Rc
            self.NF = sla.cho_factor(N)

    # -- pieces ---------------------------------------------------------
    def top(self, xi):
        return xi[: self.G * self.M].reshape(self.G, self.M).T

    def pack(self, top_mat, bottom=None):
        out = np.zeros(self.m)
        out[: self.G * self.M] = top_mat.T.reshape(-1)
        if self.kc and bottom is not None:
            out[self.G * self.M:] = bottom
        return out

    def Sigma(self, xi):
        return self.pack(self.top(xi) @ self.inst.Omega)

    def X(self, v):
        off, n_i = self.inst.col_off, self.inst.n_i
        T = np.column_stack([self.inst.X(i) @ v[off[i]:off[i] + n_i[i]]
                             for i in range(self.G)])
        bottom = self.inst.Rc @ v if self.kc else None
        return self.pack(T, bottom)

    def XT(self, xi):
        T = self.top(xi)
        out = np.concatenate([self.inst.X(i).T @ T[:, i] for i in range(self.G)])
        if self.kc:
            out = out + self.inst.Rc.T @ xi[self.G * self.M:]
        return out

    def Xstar_T(self, xi):
        if self.kc:
            return sla.cho_solve(self.NF, self.XT(xi))
        T = self.top(xi)
        return np.concatenate([sla.solve_triangular(R, Q.T @ T[:, i])
                               for i, (Q, R) in enumerate(self.QR)])

    def Xstar(self, h):
        if self.kc:
            return self.X(sla.cho_solve(self.NF, h))
        off, n_i = self.inst.col_off, self.inst.n_i
        cols = []
        for i, (Q, R) in enumerate(self.QR):
            s = sla.solve_triangular(R, h[off[i]:off[i] + n_i[i]], trans="T")
            cols.append(Q @ s)
        return self.pack(np.column_stack(cols))

    def Pi(self, xi):
        return (xi - self.X(self.Xstar_T(xi))) / self.Ddiag

    def Dnorm2(self, g):
        """g^T D g, which equals r^T Pi r for g = Pi r (Pi D Pi = Pi)."""
        return float(g @ (self.Ddiag * g))


@dataclass
class PcgResult:
    z_hat: np.ndarray
    w: np.ndarray
    iterations: int
    status: str
    c: List[float] = field(default_factory=list)
    d: List[float] = field(default_factory=list)
    lam: List[float] = field(default_factory=list)
    w_iterates: Optional[list] = None


def default_alpha(Omega):
    """D = alpha I with alpha = max_i omega_ii (the reading used throughout)."""
    return float(np.max(np.diag(Omega)))


def per_equation_d(Omega):
    """D = diag(omega_11 .. omega_GG) (x) I_M, the SUR form of D_2 = diag Sigma."""
    return np.array(np.diag(Omega), dtype=np.float64)


def pcg_aug(inst, k: int = 0, tol: float = 1e-12, max_iter: Optional[int] = None,
            alpha: Optional[float] = None, y=None, h2=None, stall: int = 20,
            keep_w: bool = False) -> PcgResult:
    """Algorithm glmpcg2 for right-hand side k of a SUR instance.

    ``y`` overrides the observation vector (flat, length G*M+k) and ``h2``
    gives a nonzero lower right-hand side; ``alpha`` is the scalar of
    D = alpha I or a length-G vector (D = diag(d) (x) I_M).  The stopping
    rule of the algorithm is read as: stop once sqrt(c_{i+1}/c_1) <= tol, or
    once c has gone ``stall`` iterations without a new minimum (no further
    progress is possible in floating point), on breakdown (d <= 0 or not
    finite), or after max_iter = m - n + 1 iterations."""
    a = default_alpha(inst.Omega) if alpha is None else alpha
    ops = SurOperators(inst, a)
    if y is None:
        bottom = inst.r[:, k] if inst.kc else None
        y = ops.pack(inst.Y[:, :, k], bottom)
    n, m = ops.n, ops.m
    if max_iter is None:
        max_iter = m - n + 1
    z = np.zeros(n)
    w = ops.Xstar(h2) if h2 is not None else np.zeros(m)
    r = ops.Sigma(w) + ops.X(z) - y
    Pr = ops.Pi(r)
    c = float(r @ Pr)
    c1 = c
    u = Pr
    v = ops.Xstar_T(r)
    res = PcgResult(z_hat=None, w=None, iterations=0, status="max_iter")
    res.c.append(c)
    if keep_w:
        res.w_iterates = [w.copy()]
    if c1 == 0.0:
        res.status = "converged"
        res.z_hat, res.w = ops.Xstar_T(y - ops.Sigma(w)), w
        return res
    c_min, since_min = c, 0
    i = 0
    for i in range(1, max_iter + 1):
        Su = ops.Sigma(u)
        d = float(u @ Su)
        res.d.append(d)
        if not (d > 0.0 and np.isfinite(d)):
            res.status = "breakdown"
            i -= 1
            break
        lam = c / d
        res.lam.append(lam)
        w = w - lam * u
        if keep_w:
            res.w_iterates.append(w.copy())
        r = r - lam * (Su + ops.X(v))
        Pr = ops.Pi(r)
        c_new = float(r @ Pr)
        res.c.append(c_new)
        if np.sqrt(abs(c_new) / c1) <= tol:
            res.status = "converged"
            break
        if c_new < c_min:
            c_min, since_min = c_new, 0
        else:
            since_min += 1
            if since_min >= stall:
                res.status = "stagnated"
                break
        mu = c_new / c
        v = ops.Xstar_T(r) + mu * v
        u = Pr + mu * u
        c = c_new
    res.iterations = i
    res.z_hat = ops.Xstar_T(y - ops.Sigma(w))
    res.w = w
    return res


def pcg_aug_projected(inst, k: int = 0, tol: float = 1e-12,
                      max_iter: Optional[int] = None, alpha: Optional[float] = None,
                      y=None, h2=None, stall: int = 50,
                      keep_w: bool = False) -> PcgResult:
    """Algorithm glmpcg2 carrying only g_i = Pi r_i instead of r_i and v_i.

    Two identities stated next to eq. Xstar make this the same iteration:
    Pi X = 0 removes the X v_i term from  Pi r_{i+1} = Pi r_i - lambda_i Pi (Sigma u_i
    + X v_i), and Pi D Pi = Pi gives  c_i = r_i^T Pi r_i = g_i^T D g_i
    (alpha ||g_i||^2 for D = alpha I).  The
    z-direction v_i is then unused (the estimate is recovered from w at
    termination exactly as in the algorithm), so it is not carried.  In
    exact arithmetic every iterate (w_i, u_i, c_i, d_i, lambda_i, mu_i)
    equals that of ``pcg_aug``.

    In floating point the forms differ for rank-deficient Sigma: the
    literal recurrence keeps the range-space part of r_i, which grows with
    the unbounded z-direction v_i and swamps Pi r_i by cancellation, while
    this form stays accurate.  Each iteration applies one OLS projection:
    T = Q^T (Sigma u) and Sigma u - Q T."""
    a = default_alpha(inst.Omega) if alpha is None else alpha
    ops = SurOperators(inst, a)
    if y is None:
        bottom = inst.r[:, k] if inst.kc else None
        y = ops.pack(inst.Y[:, :, k], bottom)
    n, m = ops.n, ops.m
    if max_iter is None:
        max_iter = m - n + 1
    w = ops.Xstar(h2) if h2 is not None else np.zeros(m)
    g = ops.Pi(ops.Sigma(w) - y)          # z_1 = 0
    c = ops.Dnorm2(g)
    c1 = c
    u = np.zeros(m)
    mu = 0.0
    res = PcgResult(z_hat=None, w=None, iterations=0, status="max_iter")
    res.c.append(c)
    if keep_w:
        res.w_iterates = [w.copy()]
    if c1 == 0.0:
        res.status = "converged"
        res.z_hat, res.w = ops.Xstar_T(y - ops.Sigma(w)), w
        return res
    c_min, since_min = c, 0
    i = 0
    for i in range(1, max_iter + 1):
        u = g + mu * u
        Su = ops.Sigma(u)
        d = float(u @ Su)
        res.d.append(d)
        if not (d > 0.0 and np.isfinite(d)):
            res.status = "breakdown"
            i -= 1
            break
        lam = c / d
        res.lam.append(lam)
        w = w - lam * u
        if keep_w:
            res.w_iterates.append(w.copy())
        g = g - lam * ops.Pi(Su)
        c_new = ops.Dnorm2(g)
        res.c.append(c_new)
        if np.sqrt(c_new / c1) <= tol:
            res.status = "converged"
            break
        if c_new < c_min:
            c_min, since_min = c_new, 0
        else:
            since_min += 1
            if since_min >= stall:
                res.status = "stagnated"
                break
        mu = c_new / c
        c = c_new
    res.iterations = i
    res.z_hat = ops.Xstar_T(y - ops.Sigma(w))
    res.w = w
    return res


# --------------------------------------------------------------------------
# exact rational arithmetic (tiny integer data)
# --------------------------------------------------------------------------

def _fmat(A):
    return [[Fraction(int(x)) for x in row] for row in np.asarray(A)]


def _mm(A, B):
    Bt = list(zip(*B))
    return [[sum((a * b for a, b in zip(row, col)), Fraction(0)) for col in Bt]
            for row in A]


def _mv(A, x):
    return [sum((a * b for a, b in zip(row, x)), Fraction(0)) for row in A]


def _dot(x, y):
    return sum((a * b for a, b in zip(x, y)), Fraction(0))


def _T(A):
    return [list(r) for r in zip(*A)]


def _solve_exact(A, B):
    """Gauss-Jordan elimination over the rationals: A^-1 B (A square, nonsingular)."""
    n = len(A)
    nb = len(B[0])
    aug = [list(A[i]) + list(B[i]) for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        p = aug[col][col]
        aug[col] = [x / p for x in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[col])]
    return [row[n:n + nb] for row in aug]


def dense_from_integer_sur(Xs, Omega, Y):
    """Dense integer (X, Sigma, y) of a SUR model in the vec layout."""
    G = len(Xs)
    M = Xs[0].shape[0]
    X = sla.block_diag(*Xs).astype(np.int64)
    Sigma = np.kron(Omega, np.eye(M, dtype=np.int64))
    y = Y.T.reshape(-1)
    return X, Sigma, y


def pcg_aug_exact(X, Sigma, y, max_iter=None):
    """Algorithm glmpcg2 on Fractions with D = I and z_1 = 0, w_1 = 0.

    Returns (iterations until c is exactly 0, z_hat, w, status)."""
    m, n = X.shape
    Xf, Sf = _fmat(X), _fmat(Sigma)
    yf = [Fraction(int(v)) for v in y]
    XtX_inv = _solve_exact(_mm(_T(Xf), Xf), [[Fraction(int(i == j)) for j in range(n)]
                                             for i in range(n)])
    XsT = _mm(XtX_inv, _T(Xf))                 # X*^T = (X^T X)^-1 X^T
    XXsT = _mm(Xf, XsT)
    Pi = [[Fraction(int(i == j)) - XXsT[i][j] for j in range(m)] for i in range(m)]
    if max_iter is None:
        max_iter = m - n + 1
    w = [Fraction(0)] * m
    z = [Fraction(0)] * n
    r = [a + b - c for a, b, c in zip(_mv(Sf, w), _mv(Xf, z), yf)]
    Pr = _mv(Pi, r)
    c = _dot(r, Pr)
    u, v = Pr, _mv(XsT, r)
    status, it = "max_iter", 0
    for it in range(1, max_iter + 1):
        Su = _mv(Sf, u)
        d = _dot(u, Su)
        if d == 0:
            status = "breakdown"
            it -= 1
            break
        lam = c / d
        w = [a - lam * b for a, b in zip(w, u)]
        Xv = _mv(Xf, v)
        r = [a - lam * (b + e) for a, b, e in zip(r, Su, Xv)]
        Pr = _mv(Pi, r)
        c_new = _dot(r, Pr)
        if c_new == 0:
            status = "converged"
            break
        mu = c_new / c
        v = [a + mu * b for a, b in zip(_mv(XsT, r), v)]
        u = [a + mu * b for a, b in zip(Pr, u)]
        c = c_new
    ymSw = [a - b for a, b in zip(yf, _mv(Sf, w))]
    z_hat = _mv(XsT, ymSw)
    return it, z_hat, w, status


def kkt_exact(X, Sigma, y):
    """Exact solution of eq. aug1 over the rationals: (w, b)."""
    m, n = X.shape
    A = augmented_int(X, Sigma)
    rhs = [[Fraction(int(v))] for v in y] + [[Fraction(0)] for _ in range(n)]
    sol = _solve_exact(_fmat(A), rhs)
    flat = [s[0] for s in sol]
    return flat[:m], flat[m:]


def augmented_int(X, Sigma):
    m, n = X.shape
    return np.block([[Sigma, X], [X.T, np.zeros((n, n), dtype=np.int64)]])
