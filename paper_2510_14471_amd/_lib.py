"""ctypes binding of include/glm.h.

Functions keep the C names and only marshal arguments: torch tensors become
device pointers, Python sequences become host int32 arrays.  Every numeric
step runs in the HIP library; if the library is missing the import of this
module raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglm_hip.so")

GLM_FP64 = 0
GLM_MIXED = 1
GLM_REDUCED = 4      # flag OR-ed into the precision: SUR model reduction
GLM_PRECOND_EQ = 8   # flag OR-ed into the precision: D = diag(omega_ii) (x) I_M

GLM_OK = 0
GLM_EINVAL = -1
GLM_EWORKSPACE = -2
GLM_EHIP = -3
GLM_EUNSUPPORTED = -4
GLM_INFO_CONVERGED = 0
GLM_INFO_STAGNATED = 1
GLM_INFO_NOCONV = -10
GLM_INFO_BREAKDOWN = -11
GLM_INFO_RANK = -12

PRECISIONS = {"fp64": GLM_FP64, "mixed": GLM_MIXED}


class GlmShape(ctypes.Structure):
    _fields_ = [("batch", c_int32), ("G", POINTER(c_int32)), ("M", POINTER(c_int32)),
                ("K", POINTER(c_int32)), ("k", POINTER(c_int32)), ("n", POINTER(c_int32))]


class GlmStats(ctypes.Structure):
    _fields_ = [("outer_steps", c_int32), ("pcg_iterations", c_int64),
                ("max_iterations", c_int32), ("launches", c_int32),
                ("pass_rowvec", c_int32 * 2), ("pass_kv", c_int32 * 2),
                ("pass_ks", c_int32 * 2), ("pass_omega", c_int32 * 2),
                ("pass_nim", c_int32 * 2)]


class GLMError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
            "(or python -m paper_2510_14471_amd._build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    lib.glm_validate_shape.argtypes = [POINTER(GlmShape)]
    lib.glm_validate_shape.restype = c_int
    lib.glm_workspace_bytes.argtypes = [POINTER(GlmShape), c_int]
    lib.glm_workspace_bytes.restype = c_size_t
    lib.glm_qr_factor.argtypes = [POINTER(GlmShape), c_int, P, P, P, c_size_t, P,
                                  POINTER(c_void_p)]
    lib.glm_qr_factor.restype = c_int
    lib.glm_qr_factor_static.argtypes = [POINTER(GlmShape), c_int, P, P, P, POINTER(c_void_p)]
    lib.glm_qr_factor_static.restype = c_int
    lib.glm_workspace_bytes_common.argtypes = [POINTER(GlmShape), c_int, P, P]
    lib.glm_workspace_bytes_common.restype = c_size_t
    lib.glm_qr_factor_common.argtypes = [POINTER(GlmShape), c_int, P, P, P, P, P, c_size_t, P,
                                         POINTER(c_void_p)]
    lib.glm_qr_factor_common.restype = c_int
    lib.glm_gls_solve.argtypes = [P, P, P, P, c_double, c_int32, P, P, P, P, P, P]
    lib.glm_gls_solve.restype = c_int
    lib.glm_gls_solve_ne.argtypes = [P, P, P, c_double, c_int32, P, P, P, P]
    lib.glm_gls_solve_ne.restype = c_int
    lib.glm_gls_backward.argtypes = [P, P, P, P, P, P, c_double, c_int32, P, P, P, P, P, P]
    lib.glm_gls_backward.restype = c_int
    lib.glm_copy_factors.argtypes = [P, P, P, P, P]
    lib.glm_copy_factors.restype = c_int
    lib.glm_plan_passes.argtypes = [POINTER(GlmShape), c_int, POINTER(GlmStats)]
    lib.glm_plan_passes.restype = c_int
    lib.glm_get_stats.argtypes = [P, POINTER(GlmStats)]
    lib.glm_get_stats.restype = c_int
    lib.glm_profile_enable.argtypes = [P, c_int]
    lib.glm_profile_enable.restype = c_int
    lib.glm_profile_read.argtypes = [P, c_int, POINTER(c_int64), POINTER(c_double),
                                     POINTER(c_double)]
    lib.glm_profile_read.restype = c_int
    lib.glm_stream_mix.argtypes = [P, P, c_int32, P, c_int32, c_int64, P, c_int32, c_int64, P]
    lib.glm_stream_mix.restype = c_int
    lib.glm_factor_destroy.argtypes = [P]
    lib.glm_factor_destroy.restype = None
    lib.glm_strerror.argtypes = [c_int]
    lib.glm_strerror.restype = ctypes.c_char_p
    return lib


_lib = _load()

EXPORTED = ["glm_validate_shape", "glm_workspace_bytes", "glm_qr_factor",
            "glm_qr_factor_static", "glm_workspace_bytes_common", "glm_qr_factor_common",
            "glm_gls_solve", "glm_gls_solve_ne",
            "glm_gls_backward", "glm_copy_factors", "glm_plan_passes", "glm_get_stats",
            "glm_profile_enable", "glm_profile_read", "glm_stream_mix", "glm_factor_destroy",
            "glm_strerror"]


def glm_strerror(code: int) -> str:
    return _lib.glm_strerror(int(code)).decode()


def _check(rc: int, what: str):
    if rc != GLM_OK:
        raise GLMError(f"{what}: {glm_strerror(rc)} ({rc})")


class Shape:
    """Host-side glm_shape: keeps the int32 arrays alive for the ctypes struct."""

    def __init__(self, G, M, K, n_flat, k=None):
        B = len(G)
        self.B = B
        self._G = (c_int32 * B)(*map(int, G))
        self._M = (c_int32 * B)(*map(int, M))
        self._K = (c_int32 * B)(*map(int, K))
        self._k = (c_int32 * B)(*map(int, k)) if k is not None else None
        self._n = (c_int32 * len(n_flat))(*map(int, n_flat))
        self.struct = GlmShape(B, self._G, self._M, self._K, self._k, self._n)

    def ptr(self):
        return ctypes.byref(self.struct)


def _dp(t):
    """Device pointer of a tensor (or NULL for None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise GLMError("argument must be a device tensor")
    if not t.is_contiguous():
        raise GLMError("argument must be contiguous")
    return c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def glm_validate_shape(shape: Shape) -> int:
    return _lib.glm_validate_shape(shape.ptr())


def glm_workspace_bytes(shape: Shape, precision: int) -> int:
    return int(_lib.glm_workspace_bytes(shape.ptr(), int(precision)))


def glm_qr_factor(shape: Shape, precision: int, X, Rc, ws, stream=None) -> c_void_p:
    h = c_void_p()
    rc = _lib.glm_qr_factor(shape.ptr(), int(precision), _dp(X), _dp(Rc), _dp(ws),
                            ws.numel() * ws.element_size(), _stream(stream), ctypes.byref(h))
    _check(rc, "glm_qr_factor")
    return h


def glm_qr_factor_static(shape: Shape, precision: int, X, Rc, stream=None) -> c_void_p:
    h = c_void_p()
    rc = _lib.glm_qr_factor_static(shape.ptr(), int(precision), _dp(X), _dp(Rc),
                                   _stream(stream), ctypes.byref(h))
    _check(rc, "glm_qr_factor_static")
    return h


def _host_i32(values):
    """A host int32 array for a pointer argument (kept alive by the caller)."""
    arr = np.ascontiguousarray(np.asarray(values, dtype=np.int32))
    return arr, arr.ctypes.data_as(c_void_p)


def glm_workspace_bytes_common(shape: Shape, precision: int, N, sel) -> int:
    a_n, p_n = _host_i32(N)
    a_s, p_s = _host_i32(sel)
    return int(_lib.glm_workspace_bytes_common(shape.ptr(), int(precision), p_n, p_s))


def glm_qr_factor_common(shape: Shape, precision: int, Z0, N, sel, Rc, ws,
                         stream=None) -> c_void_p:
    a_n, p_n = _host_i32(N)
    a_s, p_s = _host_i32(sel)
    h = c_void_p()
    rc = _lib.glm_qr_factor_common(shape.ptr(), int(precision), _dp(Z0), p_n, p_s, _dp(Rc),
                                   _dp(ws), ws.numel() * ws.element_size(), _stream(stream),
                                   ctypes.byref(h))
    _check(rc, "glm_qr_factor_common")
    return h


def glm_gls_solve(h, Omega, y, r, tol, max_iter, beta, u, uc, info, iters, stream=None) -> int:
    rc = _lib.glm_gls_solve(h, _dp(Omega), _dp(y), _dp(r), float(tol), int(max_iter),
                            _dp(beta), _dp(u), _dp(uc), _dp(info), _dp(iters), _stream(stream))
    _check(rc, "glm_gls_solve")
    return rc


def glm_gls_solve_ne(h, Omega, y, tol, max_iter, beta, info, iters, stream=None) -> int:
    rc = _lib.glm_gls_solve_ne(h, _dp(Omega), _dp(y), float(tol), int(max_iter), _dp(beta),
                               _dp(info), _dp(iters), _stream(stream))
    _check(rc, "glm_gls_solve_ne")
    return rc


def glm_gls_backward(h, Omega, beta, u, g_beta, g_u, tol, max_iter, dy, dOmega, dX, info,
                     iters, stream=None) -> int:
    rc = _lib.glm_gls_backward(h, _dp(Omega), _dp(beta), _dp(u), _dp(g_beta), _dp(g_u),
                               float(tol), int(max_iter), _dp(dy), _dp(dOmega), _dp(dX),
                               _dp(info), _dp(iters), _stream(stream))
    _check(rc, "glm_gls_backward")
    return rc


def glm_copy_factors(h, Q, R, rank, stream=None) -> int:
    rc = _lib.glm_copy_factors(h, _dp(Q), _dp(R), _dp(rank), _stream(stream))
    _check(rc, "glm_copy_factors")
    return rc


def _passes(st) -> dict:
    # pass configuration per precision: keys "fp32" (inner solves) and "fp64"
    out = {}
    for pi, name in enumerate(("fp32", "fp64")):
        out[name + "_passes"] = {"rowvec": st.pass_rowvec[pi], "kv": st.pass_kv[pi],
                                 "ks": st.pass_ks[pi], "omega": st.pass_omega[pi],
                                 "nim": st.pass_nim[pi]}
    return out


def glm_plan_passes(shape: Shape, precision: int) -> dict:
    st = GlmStats()
    _check(_lib.glm_plan_passes(shape.ptr(), int(precision), ctypes.byref(st)),
           "glm_plan_passes")
    return _passes(st)


def glm_get_stats(h) -> dict:
    st = GlmStats()
    _check(_lib.glm_get_stats(h, ctypes.byref(st)), "glm_get_stats")
    out = {"outer_steps": st.outer_steps, "pcg_iterations": st.pcg_iterations,
           "max_iterations": st.max_iterations, "launches": st.launches}
    out.update(_passes(st))
    return out


def glm_profile_enable(h, on: bool):
    _check(_lib.glm_profile_enable(h, int(bool(on))), "glm_profile_enable")


def glm_profile_read(h, kernel_id: int):
    n = c_int64()
    ms = c_double()
    by = c_double()
    _check(_lib.glm_profile_read(h, int(kernel_id), ctypes.byref(n), ctypes.byref(ms),
                                 ctypes.byref(by)), "glm_profile_read")
    return int(n.value), float(ms.value), float(by.value)


def glm_stream_mix(ro=(), rw=(), wo=(), stream=None):
    """Streaming-ceiling kernel: `ro` read-only, `rw` read and overwritten in
    place (all of one length), `wo` write-only (all of one length); float32
    device tensors."""
    for t in (*ro, *rw, *wo):
        if t.dtype.itemsize != 4:
            raise GLMError("glm_stream_mix takes float32 tensors")
    rw_len = {t.numel() for t in rw}
    wo_len = {t.numel() for t in wo}
    if len(rw_len) > 1 or len(wo_len) > 1:
        raise GLMError("glm_stream_mix: read-write and write-only streams each of one length")
    ro_p = (c_void_p * max(1, len(ro)))(*[_dp(t).value for t in ro])
    ro_n = (c_int64 * max(1, len(ro)))(*[t.numel() for t in ro])
    rw_p = (c_void_p * max(1, len(rw)))(*[_dp(t).value for t in rw])
    wo_p = (c_void_p * max(1, len(wo)))(*[_dp(t).value for t in wo])
    _check(_lib.glm_stream_mix(ro_p, ro_n, len(ro), rw_p, len(rw), rw_len.pop() if rw else 0,
                               wo_p, len(wo), wo_len.pop() if wo else 0, _stream(stream)),
           "glm_stream_mix")


def glm_factor_destroy(h):
    if h:
        _lib.glm_factor_destroy(h)
