"""Batch packing, a workspace-owning solver object and the autograd wrapper.

Everything here is marshalling around the C ABI: torch allocates device
memory (the packed inputs, the outputs and the library's workspace) and
provides the stream; the factorization, the PCG-Aug iterations, the
refinement and the gradients run in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib


@dataclass
class BatchLayout:
    """Sizes and element offsets of the concatenated per-instance arrays."""
    G: List[int]
    M: List[int]
    K: List[int]
    kc: List[int]
    n_i: List[List[int]]

    def __post_init__(self):
        self.B = len(self.G)
        self.n = [int(sum(v)) for v in self.n_i]
        self.off_X = np.cumsum([0] + [m * n for m, n in zip(self.M, self.n)]).tolist()
        self.off_Om = np.cumsum([0] + [g * g for g in self.G]).tolist()
        self.off_y = np.cumsum([0] + [m * g * k for m, g, k in zip(self.M, self.G, self.K)]).tolist()
        self.off_b = np.cumsum([0] + [n * k for n, k in zip(self.n, self.K)]).tolist()
        self.off_Rc = np.cumsum([0] + [c * n for c, n in zip(self.kc, self.n)]).tolist()
        self.off_r = np.cumsum([0] + [c * k for c, k in zip(self.kc, self.K)]).tolist()
        self.off_rhs = np.cumsum([0] + list(self.K)).tolist()

    @property
    def n_rhs(self) -> int:
        return self.off_rhs[-1]

    def shape(self) -> _lib.Shape:
        flat = [v for lst in self.n_i for v in lst]
        return _lib.Shape(self.G, self.M, self.K, flat, self.kc if any(self.kc) else None)

    @classmethod
    def of(cls, instances) -> "BatchLayout":
        return cls([i.G for i in instances], [i.M for i in instances],
                   [i.K for i in instances], [i.kc for i in instances],
                   [list(i.n_i) for i in instances])


def _put(dst, off, arr):
    a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
    dst[off:off + a.size].copy_(torch.from_numpy(a), non_blocking=False)


def pack_instances(instances, device="cuda:0"):
    """Uploads a list of SUR instances into the packed device layout.

    Returns (layout, dict with X, Omega, y, Rc, r tensors; Rc/r None when no
    instance is restricted)."""
    lay = BatchLayout.of(instances)
    dev = torch.device(device)
    f64 = torch.float64
    X = torch.empty(lay.off_X[-1], dtype=f64, device=dev)
    Om = torch.empty(lay.off_Om[-1], dtype=f64, device=dev)
    y = torch.empty(lay.off_y[-1], dtype=f64, device=dev)
    restricted = any(lay.kc)
    Rc = torch.empty(max(lay.off_Rc[-1], 1), dtype=f64, device=dev) if restricted else None
    r = torch.empty(max(lay.off_r[-1], 1), dtype=f64, device=dev) if restricted else None
    for b, inst in enumerate(instances):
        _put(X, lay.off_X[b], inst.W)
        _put(Om, lay.off_Om[b], inst.Omega)
        _put(y, lay.off_y[b], inst.Y)
        if restricted and inst.kc:
            _put(Rc, lay.off_Rc[b], inst.Rc)
            _put(r, lay.off_r[b], inst.r)
    return lay, {"X": X, "Omega": Om, "y": y, "Rc": Rc, "r": r}


def unpack(lay: BatchLayout, flat, kind: str):
    """Splits a packed device/host array into per-instance numpy arrays."""
    a = flat.detach().cpu().numpy() if isinstance(flat, torch.Tensor) else np.asarray(flat)
    out = []
    for b in range(lay.B):
        if kind == "beta":
            out.append(a[lay.off_b[b]:lay.off_b[b + 1]].reshape(lay.n[b], lay.K[b]))
        elif kind == "u":
            out.append(a[lay.off_y[b]:lay.off_y[b + 1]].reshape(lay.M[b], lay.G[b], lay.K[b]))
        elif kind == "Omega":
            out.append(a[lay.off_Om[b]:lay.off_Om[b + 1]].reshape(lay.G[b], lay.G[b]))
        elif kind == "X":
            out.append(a[lay.off_X[b]:lay.off_X[b + 1]].reshape(lay.M[b], lay.n[b]))
        elif kind == "rhs":
            out.append(a[lay.off_rhs[b]:lay.off_rhs[b + 1]])
        elif kind == "uc":
            out.append(a[lay.off_r[b]:lay.off_r[b + 1]].reshape(lay.kc[b], lay.K[b]))
        else:
            raise ValueError(kind)
    return out


def pack_mvr(instances, device="cuda:0"):
    """Uploads multivariate instances with exclusions (Z0, kept columns
    `sel`, Omega, Y).  Returns (layout, dict with Z0, Omega, y, Rc=None,
    r=None, N (host list), sel (host flat list)); the layout's n_i are the
    numbers of kept columns, so beta comes back as the kept coefficients."""
    lay = BatchLayout([i.G for i in instances], [i.M for i in instances],
                      [i.K for i in instances], [0] * len(instances),
                      [[int(len(s)) for s in i.sel] for i in instances])
    dev = torch.device(device)
    f64 = torch.float64
    N = [int(i.N) for i in instances]
    off_Z = np.cumsum([0] + [i.M * i.N for i in instances]).tolist()
    Z0 = torch.empty(off_Z[-1], dtype=f64, device=dev)
    Om = torch.empty(lay.off_Om[-1], dtype=f64, device=dev)
    y = torch.empty(lay.off_y[-1], dtype=f64, device=dev)
    for b, inst in enumerate(instances):
        _put(Z0, off_Z[b], inst.Z0)
        _put(Om, lay.off_Om[b], inst.Omega)
        _put(y, lay.off_y[b], inst.Y)
    sel = [int(v) for inst in instances for s in inst.sel for v in s]
    return lay, {"Z0": Z0, "Omega": Om, "y": y, "Rc": None, "r": None, "N": N, "sel": sel}


# kernel ids of glm_profile_read: the iteration launches of projection passes
# A and B, and (reduced solvers) the reduced responses Q1^T Y
PROFILED_KERNELS = (0, 1, 2)


class SURSolver:
    """Owns one workspace and one factor handle for a fixed batch shape."""

    def __init__(self, layout: BatchLayout, precision: str = "fp64", device="cuda:0",
                 reduce: bool = False, precond: str = "scalar"):
        """reduce: solve through the SUR model reduction (one QR of
        W = [X_1 ... X_G] per instance; the iteration runs on min(M, n + 1)
        rotated observations).  factors() raises on such a solver.
        precond: "scalar" (D = alpha I, alpha = max_i omega_ii) or "equation"
        (D = diag(omega_ii) (x) I_M, one scalar per equation)."""
        if precond not in ("scalar", "equation"):
            raise ValueError(precond)
        self.layout = layout
        self.reduce = bool(reduce)
        self.precision = (_lib.PRECISIONS[precision] | (_lib.GLM_REDUCED if reduce else 0)
                          | (_lib.GLM_PRECOND_EQ if precond == "equation" else 0))
        self.device = torch.device(device)
        self._shape = layout.shape()
        rc = _lib.glm_validate_shape(self._shape)
        if rc != _lib.GLM_OK:
            raise _lib.GLMError(f"shape rejected: {_lib.glm_strerror(rc)} ({rc})")
        nbytes = _lib.glm_workspace_bytes(self._shape, self.precision)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = None
        self._X = None
        self._Rc = None
        self._profile = False
        self._prof_acc = {kid: [0, 0.0, 0.0] for kid in PROFILED_KERNELS}

    @property
    def workspace_bytes(self) -> int:
        return self.workspace.numel()

    def _harvest_profile(self):
        if self._profile and self.handle is not None:
            for kid in PROFILED_KERNELS:
                n, ms, by = _lib.glm_profile_read(self.handle, kid)
                acc = self._prof_acc[kid]
                acc[0] += n
                acc[1] += ms
                acc[2] += by

    def factor(self, X, Rc=None, stream=None):
        if self.handle is not None:
            self._harvest_profile()
            _lib.glm_factor_destroy(self.handle)
            self.handle = None
        self._X, self._Rc = X, Rc   # the library reads them during later solves
        self.handle = _lib.glm_qr_factor(self._shape, self.precision, X, Rc, self.workspace,
                                         stream)
        if self._profile:
            _lib.glm_profile_enable(self.handle, True)
        return self

    def solve(self, Omega, y, r=None, tol=1e-12, max_iter=0, want_uc=False, stream=None):
        lay = self.layout
        f64 = torch.float64
        beta = torch.empty(lay.off_b[-1], dtype=f64, device=self.device)
        u = torch.empty(lay.off_y[-1], dtype=f64, device=self.device)
        uc = torch.empty(max(lay.off_r[-1], 1), dtype=f64, device=self.device) \
            if (want_uc and any(lay.kc)) else None
        info = torch.empty(lay.n_rhs, dtype=torch.int32, device=self.device)
        iters = torch.empty(lay.n_rhs, dtype=torch.int32, device=self.device)
        _lib.glm_gls_solve(self.handle, Omega, y, r, tol, max_iter, beta, u, uc, info, iters,
                           stream)
        return beta, u, uc, info, iters

    def solve_ne(self, Omega, y, tol=1e-12, max_iter=0, stream=None):
        """CG on the normal equations (block-Jacobi preconditioner), FP64:
        (beta, info, iters).  The comparator of the PCG-Aug estimator."""
        lay = self.layout
        beta = torch.empty(lay.off_b[-1], dtype=torch.float64, device=self.device)
        info = torch.empty(lay.n_rhs, dtype=torch.int32, device=self.device)
        iters = torch.empty(lay.n_rhs, dtype=torch.int32, device=self.device)
        _lib.glm_gls_solve_ne(self.handle, Omega, y, tol, max_iter, beta, info, iters, stream)
        return beta, info, iters

    def backward(self, Omega, beta, u, g_beta, g_u=None, tol=1e-12, max_iter=0,
                 want_dOmega=True, want_dX=True, stream=None):
        lay = self.layout
        f64 = torch.float64
        dy = torch.empty(lay.off_y[-1], dtype=f64, device=self.device)
        dOm = torch.empty(lay.off_Om[-1], dtype=f64, device=self.device) if want_dOmega else None
        dX = torch.empty(lay.off_X[-1], dtype=f64, device=self.device) if want_dX else None
        info = torch.empty(lay.n_rhs, dtype=torch.int32, device=self.device)
        iters = torch.empty(lay.n_rhs, dtype=torch.int32, device=self.device)
        _lib.glm_gls_backward(self.handle, Omega, beta, u, g_beta, g_u, tol, max_iter, dy,
                              dOm, dX, info, iters, stream)
        return dy, dOm, dX, info, iters

    def factors(self, stream=None):
        """(Q packed like X, R blocks concatenated, rank flags per block) as device tensors."""
        lay = self.layout
        Q = torch.empty(lay.off_X[-1], dtype=torch.float64, device=self.device)
        nR = sum(v * v for lst in lay.n_i for v in lst)
        R = torch.empty(max(nR, 1), dtype=torch.float64, device=self.device)
        nblk = sum(len(v) for v in lay.n_i)
        rank = torch.empty(nblk, dtype=torch.int32, device=self.device)
        _lib.glm_copy_factors(self.handle, Q, R, rank, stream)
        return Q, R, rank

    def stats(self) -> dict:
        return _lib.glm_get_stats(self.handle)

    def profile(self, on: bool):
        """Kernel timing of the projection passes; stays on across re-factoring.
        Counters accumulate per handle and are read (and cleared) by profile_read."""
        self._profile = bool(on)
        if self.handle is not None:
            _lib.glm_profile_enable(self.handle, on)

    def profile_read(self, kernel_id: int):
        """(launches, summed ms, summed algorithmic bytes) since the last read."""
        self._harvest_profile()
        acc = self._prof_acc[kernel_id]
        out = (acc[0], acc[1], acc[2])
        self._prof_acc[kernel_id] = [0, 0.0, 0.0]
        return out

    def close(self):
        if self.handle is not None:
            _lib.glm_factor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _GLSFunction(torch.autograd.Function):
    """(beta, u) = GLS(X, Omega, y) with the reverse rule of the augmented system."""

    @staticmethod
    def forward(ctx, solver, tol, max_iter, X, Omega, y):
        solver.factor(X)
        beta, u, _, info, _ = solver.solve(Omega, y, None, tol, max_iter)
        ctx.solver = solver
        ctx.tol = tol
        ctx.max_iter = max_iter
        ctx.info = info
        ctx.save_for_backward(X, Omega, beta, u)
        return beta, u

    @staticmethod
    def backward(ctx, g_beta, g_u):
        X, Omega, beta, u = ctx.saved_tensors
        solver = ctx.solver
        g_beta = torch.zeros_like(beta) if g_beta is None else g_beta.contiguous()
        g_u = None if g_u is None else g_u.contiguous()
        dy, dOm, dX, _, _ = solver.backward(
            Omega, beta, u, g_beta, g_u, ctx.tol, ctx.max_iter,
            want_dOmega=ctx.needs_input_grad[4], want_dX=ctx.needs_input_grad[3])
        return None, None, None, dX, dOm, (dy if ctx.needs_input_grad[5] else None)


def gls(solver: SURSolver, X, Omega, y, tol: float = 1e-12, max_iter: int = 0):
    """Differentiable batched SUR GLS: returns packed (beta, u)."""
    return _GLSFunction.apply(solver, tol, max_iter, X, Omega, y)


class MVRSolver(SURSolver):
    """Multivariate models with exclusion restrictions (common regressors
    Z0, equation i keeping the columns sel_i): one QR of Z0 per instance and
    the solve on min(M, N + 1) rotated rows.  Solve and solve_ne as on a
    reduced SURSolver; no backward() or factors()."""

    def __init__(self, layout: BatchLayout, N, sel, precision: str = "fp64",
                 device="cuda:0", precond: str = "scalar"):
        if precond not in ("scalar", "equation"):
            raise ValueError(precond)
        self.layout = layout
        self.reduce = True
        self.precision = (_lib.PRECISIONS[precision]
                          | (_lib.GLM_PRECOND_EQ if precond == "equation" else 0))
        self.device = torch.device(device)
        self._shape = layout.shape()
        self._N = list(N)
        self._sel = list(sel)
        nbytes = _lib.glm_workspace_bytes_common(self._shape, self.precision, self._N,
                                                 self._sel)
        if nbytes == 0:
            raise _lib.GLMError("shape or column selection rejected")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = None
        self._X = None
        self._Rc = None
        self._profile = False
        self._prof_acc = {kid: [0, 0.0, 0.0] for kid in PROFILED_KERNELS}

    def factor(self, Z0, Rc=None, stream=None):
        if self.handle is not None:
            self._harvest_profile()
            _lib.glm_factor_destroy(self.handle)
            self.handle = None
        self._X, self._Rc = Z0, Rc
        self.handle = _lib.glm_qr_factor_common(self._shape, self.precision, Z0, self._N,
                                                self._sel, Rc, self.workspace, stream)
        if self._profile:
            _lib.glm_profile_enable(self.handle, True)
        return self
