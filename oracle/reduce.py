"""SUR model reduction (the remark on reducing the SUR model in the SUR
section): one QR decomposition of W = [X_1 ... X_G] turns the M observations
of every equation into at most n + 1 without changing the GLS estimate.

With W = Q [R; 0] (Q orthogonal M x M), multiplying every equation by Q^T
keeps Sigma = Omega (x) I_M (Q^T I_M Q = I_M) and gives

    rows t <  n :  (Q^T y_i)_t = (R_i beta_i)_t + noise      (R_i: columns of R of block i)
    rows t >= n :  (Q^T y_i)_t = noise

The rows t >= n carry no information on beta, so the GLS estimate of the
first M' = min(M, n + 1) rows is the GLS estimate of the full model.  The
residual-like vector of the full model follows row by row in the rotated
coordinates:  U = Q [U_red ; (Q^T Y)_{t >= M'} Omega^-1].

This module is test infrastructure (the oracle): only the tests, smoke()
and the benchmark's CPU baseline use it.  The QR and the solves are
numpy/scipy LAPACK calls; the GLS of the reduced model is oracle.gls.

Parity status: pinned by tests/test_oracle_pins.py (the reduced route agrees
with the direct GLS of the full model, beta and u, for nonsingular Omega with
and without restrictions).
"""
from __future__ import annotations

import copy

import numpy as np
import scipy.linalg as sla

from . import gls


def reduced_rows(M: int, n: int) -> int:
    """Rows the reduced model keeps: n + 1 (one pure-noise row keeps the
    augmented system of a single equation nonsingular), at most M."""
    return min(M, n + 1)


def reduce_instance(inst):
    """(reduced instance, Q, Q^T Y) for one SUR instance.

    The reduced instance has M' = reduced_rows(M, n) observations, regressors
    W' = (Q^T W)[:M'] (upper trapezoidal) and responses (Q^T Y)[:M']; Omega,
    the restrictions and beta_true are those of the full instance."""
    M, G, K = inst.Y.shape
    n = inst.n
    Q, _ = np.linalg.qr(inst.W, mode="complete")          # M x M orthogonal
    QtW = Q.T @ inst.W
    QtY = np.einsum("st,sik->tik", Q, inst.Y)             # Q^T acting on the rows
    Mr = reduced_rows(M, n)
    red = copy.copy(inst)
    red.W = np.array(QtW[:Mr], copy=True)
    red.W[np.tril_indices(Mr, -1, n)] = 0.0                # exact zeros below R
    red.Y = np.array(QtY[:Mr], copy=True)
    return red, Q, QtY


def sur_gls_reduced(inst):
    """GLS of a SUR instance through the reduced model (nonsingular Omega).

    Returns (beta n x K, U M x G x K) of the full model."""
    red, Q, QtY = reduce_instance(inst)
    if inst.Rc is not None:
        beta, Ur, _ = gls.restricted_gls(red)
    else:
        beta, Ur = gls.sur_gls(red)
    Mr = red.Y.shape[0]
    Oinv = sla.cho_solve(sla.cho_factor(inst.Omega), np.eye(inst.G))
    Z = np.empty_like(inst.Y)
    Z[:Mr] = Ur
    Z[Mr:] = np.einsum("tik,ij->tjk", QtY[Mr:], Oinv)
    U = np.einsum("ts,sik->tik", Q, Z)
    return beta, U
