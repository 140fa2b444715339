"""Seeded synthetic SUR (seemingly unrelated regressions) workloads.

Model (Introduction and the SUR section of the paper): for equations
i = 1..G with M observations each,

    y_i = X_i beta_i + eps_i,   X_i in R^{M x n_i} of full column rank,
    rows of E = [eps_1 ... eps_G] i.i.d. with covariance Omega (G x G, PSD),

so that Sigma = Omega (x) I_M in the vec layout.  Optional equality
constraints R_c beta = r (the restricted GLM of the applications section)
are drawn for the singular/constrained workload.

Storage conventions (shared by every consumer):
  * ``W``     M x n float64, C-contiguous, the blocks side by side
              ``[X_1 X_2 ... X_G]`` (n = sum n_i); X_i = W[:, off_i:off_i+n_i].
  * ``Y``     M x G x K float64, ``Y[t, i, k]`` = observation t of equation i
              for right-hand side k (observation-major, K innermost).
  * ``beta_true``  n x K, blocks stacked in equation order.
  * ``Rc``    k x n (or None), ``r``  k x K (or None).

Draw order inside one instance (fixed; changing it changes every workload):
sizes -> Omega -> X_1..X_G -> beta -> noise z -> (Rc).  A batch draws all
sizes from the parent generator first, then each instance from its own
child stream ``SeedSequence(seed).spawn(B)[b]``, so any subset of a batch
can be regenerated alone.

Nothing here computes an estimator: the only linear algebra is what is
needed to *draw* data with a prescribed covariance (a Cholesky factor of
Omega for the noise, eigenvalues to calibrate a condition number).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class SURInstance:
    n_i: List[int]
    W: np.ndarray
    Omega: np.ndarray
    Y: np.ndarray
    beta_true: np.ndarray
    Rc: Optional[np.ndarray] = None
    r: Optional[np.ndarray] = None
    noise: Optional[np.ndarray] = None  # M x G x K, the drawn disturbances

    @property
    def G(self) -> int:
        return len(self.n_i)

    @property
    def M(self) -> int:
        return self.W.shape[0]

    @property
    def K(self) -> int:
        return self.Y.shape[2]

    @property
    def n(self) -> int:
        return int(sum(self.n_i))

    @property
    def kc(self) -> int:
        return 0 if self.Rc is None else self.Rc.shape[0]

    @property
    def col_off(self) -> List[int]:
        off, acc = [], 0
        for v in self.n_i:
            off.append(acc)
            acc += v
        return off

    def X(self, i: int) -> np.ndarray:
        o = self.col_off[i]
        return self.W[:, o:o + self.n_i[i]]


@dataclass
class SURBatch:
    instances: List[SURInstance] = field(default_factory=list)
    name: str = ""

    def __len__(self):
        return len(self.instances)

    def __getitem__(self, b):
        return self.instances[b]

    def __iter__(self):
        return iter(self.instances)

    @property
    def n_solves(self) -> int:
        return int(sum(inst.K for inst in self.instances))


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _regressors(rng, M, n_i, intercept=True):
    """X_i with a column of ones first (when ``intercept``) and N(0,1) entries."""
    n = int(sum(n_i))
    W = np.empty((M, n), dtype=np.float64)
    off = 0
    for ni in n_i:
        blk = rng.standard_normal((M, ni))
        if intercept:
            blk[:, 0] = 1.0
        W[:, off:off + ni] = blk
        off += ni
    return W


def _responses(W, n_i, beta, noise):
    """Y[:, i, k] = X_i beta_i^{(k)} + noise[:, i, k]  (data generation only)."""
    M, G, K = noise.shape
    Y = np.empty((M, G, K), dtype=np.float64)
    off = 0
    for i, ni in enumerate(n_i):
        Y[:, i, :] = W[:, off:off + ni] @ beta[off:off + ni, :] + noise[:, i, :]
        off += ni
    return Y


def _noise_from_factor(rng, M, F, K):
    """Rows of E ~ (0, F F^T): E[:, :, k] = Z_k F^T with Z_k ~ N(0, I)."""
    G, q = F.shape
    E = np.empty((M, G, K), dtype=np.float64)
    for k in range(K):
        Z = rng.standard_normal((M, q))
        E[:, :, k] = Z @ F.T
    return E


def _instance(rng, M, n_i, Omega, K, intercept=True, noise_factor=None):
    W = _regressors(rng, M, n_i, intercept)
    n = int(sum(n_i))
    beta = rng.standard_normal((n, K))
    F = np.linalg.cholesky(Omega) if noise_factor is None else noise_factor
    E = _noise_from_factor(rng, M, F, K)
    Y = _responses(W, n_i, beta, E)
    return SURInstance(n_i=list(map(int, n_i)), W=W, Omega=Omega, Y=Y,
                       beta_true=beta, noise=E)


def _aat_plus(rng, G, shift):
    A = rng.standard_normal((G, G))
    return A @ A.T + shift * np.eye(G)


def _scaled_equicorrelated(rng, G, rho, target_cond):
    """S C_rho S with C_rho = rho 11^T + (1-rho) I and S = diag(exp(s u)),
    u ~ U(0,1) i.i.d.; s is found by bisection so that cond = target_cond."""
    C = rho * np.ones((G, G)) + (1.0 - rho) * np.eye(G)
    u = rng.uniform(0.0, 1.0, size=G)

    def cond_of(s):
        d = np.exp(s * u)
        ev = np.linalg.eigvalsh(C * np.outer(d, d))
        return ev[-1] / ev[0]

    lo, hi = 0.0, 1.0
    if cond_of(lo) >= target_cond:
        raise ValueError("target condition number below that of C_rho")
    while cond_of(hi) < target_cond:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if cond_of(mid) < target_cond:
            lo = mid
        else:
            hi = mid
    d = np.exp(hi * u)
    return C * np.outer(d, d)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config0(seed: int = 0) -> SURBatch:
    """Single small SUR: G=3, M=200, n_i = (4, 6, 5), K=1; X_i intercept +
    N(0,1); Omega = A A^T + 0.5 I with A ~ N(0,1); beta ~ N(0,1);
    y = X beta + (chol(Omega) (x) I_M) z."""
    rng = np.random.default_rng(seed)
    n_i = [4, 6, 5]
    Omega = _aat_plus(rng, 3, 0.5)
    inst = _instance(rng, 200, n_i, Omega, 1)
    return SURBatch([inst], name="sur_small_G3_M200")


def config1(seed: int = 1, M: int = 10_000, G: int = 50) -> SURBatch:
    """Single large SUR: G=50, M=10,000, n_i ~ U{5..40}; X_i intercept + N(0,1);
    Omega = S C_0.5 S with cond(Omega) = 1e3; K=1."""
    rng = np.random.default_rng(seed)
    n_i = rng.integers(5, 41, size=G).tolist()
    Omega = _scaled_equicorrelated(rng, G, 0.5, 1e3)
    inst = _instance(rng, M, n_i, Omega, 1)
    return SURBatch([inst], name=f"sur_large_G{G}_M{M}")


def _batch(seed, B, G_rng, M_rng, n_rng, K, shift, name, subset=None,
           intercept=True):
    parent = np.random.default_rng(seed)
    Gs = parent.integers(G_rng[0], G_rng[1] + 1, size=B)
    Ms = parent.integers(M_rng[0], M_rng[1] + 1, size=B)
    n_lists = [parent.integers(n_rng[0], n_rng[1] + 1, size=int(g)).tolist()
               for g in Gs]
    children = np.random.SeedSequence(seed).spawn(B)
    idx = list(range(B)) if subset is None else list(subset)

    def one(b):
        rng = np.random.default_rng(children[b])
        G = int(Gs[b])
        Omega = _aat_plus(rng, G, shift)
        return _instance(rng, int(Ms[b]), n_lists[b], Omega, K, intercept)

    # each instance has its own stream, so drawing them concurrently gives the
    # same values as drawing them in order
    workers = max(1, min(8, os.cpu_count() or 1, len(idx)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        out = list(ex.map(one, idx))
    return SURBatch(out, name=name)


def config2(seed: int = 2, B: int = 512, K: int = 16, subset=None) -> SURBatch:
    """Batch of 512 independent SUR instances: G ~ U{4..32}, M ~ U{500..5000},
    n_i ~ U{3..20}, K = 16 right-hand sides (independent beta and z per RHS);
    X_i intercept + N(0,1); Omega = A A^T + 0.1 I per instance.
    ``subset`` regenerates only the listed instances (same values)."""
    return _batch(seed, B, (4, 32), (500, 5000), (3, 20), K, 0.1,
                  f"sur_batch{B}_K{K}", subset)


def config2_sizes(seed: int = 2, B: int = 512):
    """(G_b, M_b, n_{b,i}) of the batched workload without drawing data."""
    parent = np.random.default_rng(seed)
    Gs = parent.integers(4, 33, size=B)
    Ms = parent.integers(500, 5001, size=B)
    n_lists = [parent.integers(3, 21, size=int(g)).tolist() for g in Gs]
    return [(int(Gs[b]), int(Ms[b]), n_lists[b]) for b in range(B)]


def config3(seed: int = 3, M: int = 20_000, G: int = 20) -> SURBatch:
    """Differentiation workload: G=20, M=20,000, n_i ~ U{10..50};
    X_i intercept + N(0,1); Omega = A A^T + 0.5 I; K=1."""
    rng = np.random.default_rng(seed)
    n_i = rng.integers(10, 51, size=G).tolist()
    Omega = _aat_plus(rng, G, 0.5)
    inst = _instance(rng, M, n_i, Omega, 1)
    return SURBatch([inst], name=f"sur_grad_G{G}_M{M}")


def config4(seed: int = 4, M: int = 50_000, G: int = 100, k: int = 10,
            rank_deficit: int = 2) -> SURBatch:
    """Singular and constrained: G=100, M=50,000, n_i ~ U{5..30}; X_i N(0,1)
    (no intercept); Omega = B B^T with B ~ N(0,1) of shape G x (G-2) (rank
    G-2); noise E = Z B^T; constraints R_c beta = r with R_c ~ N(0,1) of
    shape k x n and r = R_c beta_true; K = 1."""
    rng = np.random.default_rng(seed)
    n_i = rng.integers(5, 31, size=G).tolist()
    Bf = rng.standard_normal((G, G - rank_deficit))
    Omega = Bf @ Bf.T
    inst = _instance(rng, M, n_i, Omega, 1, intercept=False, noise_factor=Bf)
    n = inst.n
    inst.Rc = rng.standard_normal((k, n))
    inst.r = inst.Rc @ inst.beta_true
    return SURBatch([inst], name=f"sur_singular_G{G}_M{M}_k{k}")


def small_batch(seed: int = 7, B: int = 6, G_rng=(1, 6), M_rng=(20, 300),
                n_rng=(1, 7), K_rng=(1, 5), shift=0.3, constraints=0,
                singular=0, intercept=None) -> SURBatch:
    """Small uneven batch for parity tests: every size drawn per instance
    (including K), ragged shapes, optional constraints and rank deficit.
    With a rank-deficient Omega the regressors have no intercept column by
    default (as in the singular workload), since intercepts in every block
    are not identified by the few noise-free combinations alone."""
    if intercept is None:
        intercept = not singular
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(B):
        G = int(rng.integers(G_rng[0], G_rng[1] + 1))
        M = int(rng.integers(M_rng[0], M_rng[1] + 1))
        K = int(rng.integers(K_rng[0], K_rng[1] + 1))
        n_i = rng.integers(n_rng[0], n_rng[1] + 1, size=G).tolist()
        n_i = [min(v, M) for v in n_i]
        if singular and G > singular:
            Bf = rng.standard_normal((G, G - singular))
            Omega = Bf @ Bf.T
            inst = _instance(rng, M, n_i, Omega, K, intercept, noise_factor=Bf)
        else:
            Omega = _aat_plus(rng, G, shift)
            inst = _instance(rng, M, n_i, Omega, K, intercept)
        if constraints:
            kc = min(constraints, inst.n - 1) if inst.n > 1 else 0
            if kc > 0:
                inst.Rc = rng.standard_normal((kc, inst.n))
                inst.r = inst.Rc @ inst.beta_true
        out.append(inst)
    return SURBatch(out, name=f"small_batch_s{seed}")


def mc_sur(seed: int = 21, B: int = 256, K: int = 16, G: int = 4, M: int = 20, ni: int = 5,
           eigvals=(0.01, 0.1, 10.0, 50.0)) -> SURBatch:
    """SUR counterpart of the Monte Carlo experiment comparing the PCG-Aug
    and PCG-NE estimators: m = G M = 80 observations and n = G ni = 20
    coefficients; Omega = V diag(eigvals) V^T with V a random orthogonal
    matrix, so that Sigma = Omega (x) I_M has the four eigenvalues 0.01, 0.1,
    10 and 50, each M times; the regressors follow the recipe of the
    convergence experiment (a constant first column, other entries of
    variance m).  X, Omega and beta are drawn once and shared by all B
    instances; each of the B K right-hand sides is one replication
    y = X beta + eps with eps ~ N(0, Sigma)."""
    rng = np.random.default_rng(seed)
    n_i = [ni] * G
    m = G * M
    W = rng.standard_normal((M, G * ni)) * np.sqrt(m)
    W[:, ::ni] = 1.0
    V, _ = np.linalg.qr(rng.standard_normal((G, G)))
    Omega = (V * np.asarray(eigvals, dtype=np.float64)) @ V.T
    Omega = 0.5 * (Omega + Omega.T)
    beta = 1.0 + rng.standard_normal((G * ni, 1))
    F = np.linalg.cholesky(Omega)
    out = []
    for _ in range(B):
        E = _noise_from_factor(rng, M, F, K)
        Y = _responses(W, n_i, np.repeat(beta, K, axis=1), E)
        out.append(SURInstance(n_i=list(n_i), W=W, Omega=Omega, Y=Y,
                               beta_true=np.repeat(beta, K, axis=1), noise=E))
    return SURBatch(out, name=f"mc_sur_s{seed}")


# --------------------------------------------------------------------------
# multivariate model with exclusion restrictions (common regressors)
# --------------------------------------------------------------------------

@dataclass
class MVRInstance:
    """Y = Z0 B + U with exclusions: equation i keeps the columns sel[i] of
    Z0 (its other coefficients are zero).  Rows of U ~ N(0, Omega)."""
    Z0: np.ndarray                 # M x N
    sel: List[np.ndarray]          # per equation, kept column indices (ascending)
    Omega: np.ndarray              # G x G
    Y: np.ndarray                  # M x G x K
    B_true: np.ndarray             # N x G (zeros at the exclusions)

    @property
    def G(self) -> int:
        return int(self.Omega.shape[0])

    @property
    def M(self) -> int:
        return int(self.Z0.shape[0])

    @property
    def N(self) -> int:
        return int(self.Z0.shape[1])

    @property
    def K(self) -> int:
        return int(self.Y.shape[2])

    def to_sur(self) -> SURInstance:
        """The same model as a SUR with X_i = Z0[:, sel_i] (column selection)."""
        W = np.concatenate([self.Z0[:, s] for s in self.sel], axis=1)
        beta = np.concatenate([self.B_true[s, i] for i, s in enumerate(self.sel)])
        return SURInstance(n_i=[int(len(s)) for s in self.sel], W=W, Omega=self.Omega,
                           Y=self.Y, beta_true=np.repeat(beta[:, None], self.K, axis=1))


def var_regressors(rng, M: int, N: int, lags: int = 4, lam_max: float = 0.9,
                   burn: int = 50) -> np.ndarray:
    """M x N regressors whose rows follow a VAR(lags) process: random
    coefficient matrices A_l scaled by s^l, s chosen so that the largest
    root modulus of the companion matrix is lam_max; N(0, I) innovations."""
    A = [rng.standard_normal((N, N)) / np.sqrt(N * lags) for _ in range(lags)]
    comp = np.zeros((N * lags, N * lags))
    comp[:N, :] = np.concatenate(A, axis=1)
    comp[N:, :-N] = np.eye(N * (lags - 1))
    rho = np.abs(np.linalg.eigvals(comp)).max()
    s = lam_max / rho
    A = [a * s ** (l + 1) for l, a in enumerate(A)]
    steps = M + (burn if lam_max < 1.0 else lags)
    z = np.zeros((steps + lags, N))
    for t in range(lags, steps + lags):
        z[t] = sum(A[l] @ z[t - 1 - l] for l in range(lags)) + rng.standard_normal(N)
    return z[-M:]


def _omega_with_condition(rng, G: int, cond: float) -> np.ndarray:
    V, _ = np.linalg.qr(rng.standard_normal((G, G)))
    ev = np.geomspace(1.0, cond, G)
    Om = (V * ev) @ V.T
    return 0.5 * (Om + Om.T)


def mvrglm_var(seed: int = 31, B: int = 6, K: int = 4, G: int = 12, M: int = 300,
               N: int = 60, sparsity: float = 0.26, lam_max: float = 0.9,
               omega_cond: float = 4.48) -> List[MVRInstance]:
    """Restricted multivariate models of the VAR experiments: Z0 (M x N)
    with VAR(4) rows of largest root lam_max, B (N x G) with a fraction
    `sparsity` of its entries excluded (zero; every equation keeps at least
    its first column), Omega with condition number omega_cond.  Each
    instance draws its own Z0, exclusions and Omega."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(B):
        Z0 = var_regressors(rng, M, N, lam_max=lam_max)
        Z0 = Z0 / np.abs(Z0).max()
        sel = []
        Btrue = np.zeros((N, G))
        for i in range(G):
            keep = rng.random(N) >= sparsity
            keep[0] = True
            idx = np.flatnonzero(keep)
            sel.append(idx)
            Btrue[idx, i] = rng.standard_normal(idx.size)
        Om = _omega_with_condition(rng, G, omega_cond)
        F = np.linalg.cholesky(Om)
        Y = np.empty((M, G, K))
        fit = Z0 @ Btrue
        for k in range(K):
            Y[:, :, k] = fit + rng.standard_normal((M, G)) @ F.T
        out.append(MVRInstance(Z0=Z0, sel=sel, Omega=Om, Y=Y, B_true=Btrue))
    return out


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}


# --------------------------------------------------------------------------
# plain (non-SUR) GLM setups of the paper's two synthetic experiments
# --------------------------------------------------------------------------

def _glm_setup(rng, m, n, eigvals_with_mult):
    """X: first column constant, other entries N(0, m) (variance m);
    Sigma = V diag(ev) V^T with V the orthogonal factor of a Gaussian matrix."""
    X = rng.standard_normal((m, n)) * np.sqrt(m)
    X[:, 0] = 1.0
    ev = np.concatenate([np.full(mult, val) for val, mult in eigvals_with_mult])
    assert ev.size == m
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Sigma = (V * ev) @ V.T
    Sigma = 0.5 * (Sigma + Sigma.T)
    return X, Sigma


def e1_setup(alpha: float, seed: int = 11):
    """Scaling experiment: m=300, n=50, Sigma eigenvalues alpha*(1/2, 1, 3/2, 2)
    each of multiplicity 75; D = I."""
    rng = np.random.default_rng(seed)
    return _glm_setup(rng, 300, 50,
                      [(0.5 * alpha, 75), (alpha, 75), (1.5 * alpha, 75),
                       (2.0 * alpha, 75)])


def e2_setup(seed: int = 12, m: int = 80, n: int = 20, mult: int = 20):
    """Monte Carlo experiment: Sigma eigenvalues (0.01, 0.1, 10, 50); the paper
    gives m = 80 but multiplicity 50, which is inconsistent; m = 80 with
    multiplicity 20 is used."""
    rng = np.random.default_rng(seed)
    return _glm_setup(rng, m, n,
                      [(0.01, mult), (0.1, mult), (10.0, mult), (50.0, mult)])


def tiny_integer_sur(seed: int = 5, G: int = 2, M: int = 5, n_i=(1, 2),
                     lo: int = -3, hi: int = 3):
    """Small integer-valued SUR for exact rational arithmetic: integer X_i with
    full column rank, integer SPD Omega (A A^T + I), integer y."""
    rng = np.random.default_rng(seed)
    while True:
        Xs = [rng.integers(lo, hi + 1, size=(M, ni)) for ni in n_i]
        if all(np.linalg.matrix_rank(X) == X.shape[1] for X in Xs):
            break
    A = rng.integers(-2, 3, size=(G, G))
    Omega = A @ A.T + np.eye(G, dtype=np.int64)
    Y = rng.integers(-5, 6, size=(M, G))
    return [X.astype(np.int64) for X in Xs], Omega.astype(np.int64), Y.astype(np.int64)
