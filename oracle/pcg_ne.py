"""PCG-NE: conjugate gradients on the normal equations of the GLS problem,

    (X^T Sigma^-1 X) beta = X^T Sigma^-1 y,

the comparator of the PCG-Aug method in the paper's Monte Carlo experiment
and VAR experiments (Section "Statistical properties of the PCG-Aug
estimator"; the VAR experiments of the applications section).  For a SUR
model X^T Sigma^-1 X = [w^{ij} X_i^T X_j] with [w^{ij}] = Omega^-1, applied
as X^T (Omega^-1 (x) I_M) X p without forming it.

The preconditioner is not named for the Monte Carlo experiment (a
"classical" CG on the normal equations); the reading taken here offers the
plain CG (identity) and the block-Jacobi preconditioner built from the
diagonal blocks w^{ii} X_i^T X_i of the normal matrix (one OLS solve per
equation, the natural counterpart of PCG-Aug's OLS step).

TEST INFRASTRUCTURE: used by the tests and never by the product package.

Parity status: pinned (converges to the direct GLS; with block-Jacobi and a
diagonal Omega it ends in one step; the iterates minimise the error in the
normal-matrix norm over growing Krylov spaces, so that error never grows;
started from 0 its iterates are biased toward 0, unlike PCG-Aug's).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .gls import _cross_products, _kron_weighted


@dataclass
class NeResult:
    beta: np.ndarray
    iterations: int
    status: str
    rnorm: List[float] = field(default_factory=list)
    iterates: Optional[list] = None


def normal_system(inst, k: int = 0):
    """(A, b) = (X^T Sigma^-1 X, X^T Sigma^-1 y_k) of a SUR instance."""
    Oinv = sla.cho_solve(sla.cho_factor(inst.Omega), np.eye(inst.G))
    WtW, WtY = _cross_products(inst)
    A, c = _kron_weighted(inst, WtW, WtY, Oinv)
    return A, c[:, k], Oinv


def pcg_ne(inst, k: int = 0, tol: float = 1e-12, max_iter: Optional[int] = None,
           precond: str = "block", keep: bool = False) -> NeResult:
    """CG on the normal equations of right-hand side k from beta_0 = 0.
    Stops when ||r_i|| <= tol ||b|| or after max_iter (default n) steps."""
    A, b, Oinv = normal_system(inst, k)
    n = inst.n
    if max_iter is None:
        max_iter = n
    if precond == "block":
        blocks = []
        for i in range(inst.G):
            o, ni = inst.col_off[i], inst.n_i[i]
            blocks.append(sla.cho_factor(A[o:o + ni, o:o + ni]))

        def Minv(r):
            out = np.empty_like(r)
            for i, cf in enumerate(blocks):
                o, ni = inst.col_off[i], inst.n_i[i]
                out[o:o + ni] = sla.cho_solve(cf, r[o:o + ni])
            return out
    elif precond == "none":
        def Minv(r):
            return r.copy()
    else:
        raise ValueError(precond)
    x = np.zeros(n)
    r = b.copy()
    z = Minv(r)
    p = z.copy()
    rz = float(r @ z)
    bn = float(np.linalg.norm(b))
    res = NeResult(beta=x, iterations=0, status="max_iter", rnorm=[float(np.linalg.norm(r))],
                   iterates=[x.copy()] if keep else None)
    if bn == 0.0:
        res.status = "converged"
        return res
    i = 0
    for i in range(1, max_iter + 1):
        Ap = A @ p
        pAp = float(p @ Ap)
        if not (pAp > 0.0):
            res.status = "breakdown"
            i -= 1
            break
        a = rz / pAp
        x = x + a * p
        r = r - a * Ap
        res.rnorm.append(float(np.linalg.norm(r)))
        if keep:
            res.iterates.append(x.copy())
        if res.rnorm[-1] <= tol * bn:
            res.status = "converged"
            break
        z = Minv(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    res.iterations = i
    res.beta = x
    return res
