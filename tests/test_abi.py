"""The C-ABI library loads, exports every symbol include/glm.h declares, and
its host-side logic (shape validation, workspace sizing) behaves; no device
calls are made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glm.h")
LIB = os.path.join(ROOT, "paper_2510_14471_amd", "libglm_hip.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(glm_[a-z_]+)\s*\(", src)))


def _exported():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    return {ln.split()[-1] for ln in out.splitlines() if " T " in ln}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libglm_hip.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 10
    exported = _exported()
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        getattr(lib, s)


def test_python_binding_names_match_header():
    from paper_2510_14471_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared()


def _shape(G, M, K, n_flat, k=None):
    from paper_2510_14471_amd import _lib
    return _lib.Shape(G, M, K, n_flat, k)


def test_shape_validation_and_workspace_sizes():
    from paper_2510_14471_amd import _lib
    ok = _shape([3, 2], [200, 50], [1, 4], [4, 6, 5, 2, 3])
    assert _lib.glm_validate_shape(ok) == _lib.GLM_OK
    w64 = _lib.glm_workspace_bytes(ok, _lib.GLM_FP64)
    w32 = _lib.glm_workspace_bytes(ok, _lib.GLM_MIXED)
    assert w64 > 8 * (200 * 15 + 50 * 5) and w32 > w64 // 2
    # larger batches need more workspace, monotonically
    big = _shape([3, 2], [400, 50], [1, 4], [4, 6, 5, 2, 3])
    assert _lib.glm_workspace_bytes(big, _lib.GLM_FP64) > w64
    bad = [
        _shape([3], [200], [0], [4, 6, 5]),          # K < 1
        _shape([3], [200], [17], [4, 6, 5]),         # K > 16
        _shape([2], [5], [1], [6, 1]),               # n_i > M
        _shape([1], [5], [1], [5]),                  # n >= G M (no null space)
        _shape([2], [50], [1], [0, 3]),              # n_i < 1
        _shape([1], [50], [1], [3], k=[4]),          # more restrictions than columns
        _shape([], [], [], []),                      # empty batch
        _shape([1], [0], [1], [1]),                  # no observations
        _shape([0], [50], [1], []),                  # no equations
    ]
    for s in bad:
        assert _lib.glm_validate_shape(s) == _lib.GLM_EINVAL
        assert _lib.glm_workspace_bytes(s, _lib.GLM_FP64) == 0
    unsupported = [
        _shape([1], [500], [1], [65]),               # block wider than the QR kernel
        _shape([257], [10], [1], [1] * 257),         # Omega above 64k entries
        _shape([40], [200], [1], [60] * 40),         # n above 2048 columns
        _shape([2], [200], [1], [50, 50], k=[65]),   # more than 64 restrictions
    ]
    for s in unsupported:
        assert _lib.glm_validate_shape(s) == _lib.GLM_EUNSUPPORTED
        assert _lib.glm_workspace_bytes(s, _lib.GLM_FP64) == 0
    # the largest accepted sizes plan a workspace
    edge = _shape([256, 32], [40, 3000], [1, 16], [1] * 256 + [32] * 32, k=[0, 64])
    assert _lib.glm_validate_shape(edge) == _lib.GLM_OK
    assert _lib.glm_workspace_bytes(edge, _lib.GLM_MIXED) > 0


def test_factor_rejects_a_short_workspace_before_any_device_work():
    """The workspace check comes before any HIP call, so it runs without a GPU."""
    import ctypes
    from paper_2510_14471_amd import _lib
    s = _shape([3], [200], [1], [4, 6, 5])
    need = _lib.glm_workspace_bytes(s, _lib.GLM_FP64)
    assert need > 0
    out = ctypes.c_void_p()
    rc = _lib._lib.glm_qr_factor(s.ptr(), _lib.GLM_FP64, ctypes.c_void_p(8), None,
                                 ctypes.c_void_p(8), need - 1, None, ctypes.byref(out))
    assert rc == _lib.GLM_EWORKSPACE and not out.value


def test_strerror_is_total():
    from paper_2510_14471_amd import _lib
    for code in (0, -1, -2, -3, -4, 1, -10, -11, -12, 12345):
        assert isinstance(_lib.glm_strerror(code), str) and _lib.glm_strerror(code)


def test_workspace_for_the_batched_workload_fits_one_gpu():
    import synth
    from paper_2510_14471_amd import BatchLayout, _lib
    sizes = synth.config2_sizes()
    lay = BatchLayout([g for g, m, n in sizes], [m for g, m, n in sizes], [16] * 512,
                      [0] * 512, [n for g, m, n in sizes])
    for prec in (_lib.GLM_FP64, _lib.GLM_MIXED):
        nb = _lib.glm_workspace_bytes(lay.shape(), prec)
        assert 0 < nb < 40e9


def test_reduced_workspace_and_flag_checks():
    """GLM_REDUCED sizes its own workspace (the W copy and rotated vectors plus
    the reduced problem's workspace, smaller than the full problem's), rejects
    an unknown base precision, and checks the workspace before device work."""
    import ctypes
    from paper_2510_14471_amd import _lib
    s = _shape([3, 5], [900, 400], [16, 16], [4, 6, 5, 3, 3, 2, 7, 4])
    for base in (_lib.GLM_FP64, _lib.GLM_MIXED):
        full = _lib.glm_workspace_bytes(s, base)
        red = _lib.glm_workspace_bytes(s, base | _lib.GLM_REDUCED)
        assert 0 < red and 0 < full
    assert _lib.glm_workspace_bytes(s, 2 | _lib.GLM_REDUCED) == 0
    bad = _shape([3], [10], [1], [4, 6, 11])                 # n_i > M
    assert _lib.glm_workspace_bytes(bad, _lib.GLM_FP64 | _lib.GLM_REDUCED) == 0
    need = _lib.glm_workspace_bytes(s, _lib.GLM_MIXED | _lib.GLM_REDUCED)
    out = ctypes.c_void_p()
    rc = _lib._lib.glm_qr_factor(s.ptr(), _lib.GLM_MIXED | _lib.GLM_REDUCED, ctypes.c_void_p(8),
                                 None, ctypes.c_void_p(8), need - 1, None, ctypes.byref(out))
    assert rc == _lib.GLM_EWORKSPACE and not out.value


def test_reduction_takes_the_unreduced_limits():
    """The reduction has no equation limit of its own: 65 and 256 equations
    are planned like the unreduced problem, and the reduced workspace holds
    Q1 (M x min(M, n + 1)) next to the copy of W."""
    from paper_2510_14471_amd import _lib
    for G in (65, 256):
        s = _shape([G], [400], [1], [1] * G)
        full = _lib.glm_workspace_bytes(s, _lib.GLM_FP64)
        red = _lib.glm_workspace_bytes(s, _lib.GLM_FP64 | _lib.GLM_REDUCED)
        assert full > 0 and red > 8 * 400 * (G + G + 1)


@pytest.mark.parametrize("name", sorted(__import__("pass_cases").CASES))
def test_pass_configuration_of_each_parity_case(name):
    """The host-side planner selects, for each batch of the pass-configuration
    parity tests, the configuration that test is meant to reach (so every
    configuration is run on the GPU by some test)."""
    import pass_cases
    from paper_2510_14471_amd import _lib, BatchLayout
    insts = pass_cases.instances(name)
    _, want32, want64, reduced = pass_cases.CASES[name]
    shape = BatchLayout.of(insts).shape()
    precs = [(_lib.GLM_MIXED, True), (_lib.GLM_FP64, False)]
    if reduced:
        precs += [(_lib.GLM_MIXED | _lib.GLM_REDUCED, True),
                  (_lib.GLM_FP64 | _lib.GLM_REDUCED, False)]
    for prec, mixed in precs:
        got = _lib.glm_plan_passes(shape, prec)
        assert pass_cases.matches(got["fp64_passes"], want64), (prec, got)
        if mixed:
            assert pass_cases.matches(got["fp32_passes"], want32), (prec, got)
        else:
            assert got["fp32_passes"]["rowvec"] == -1, got


def test_common_regressor_workspace_validates_the_selection():
    """glm_workspace_bytes_common (host only) accepts strictly increasing
    kept columns below N and rejects anything else with 0."""
    from paper_2510_14471_amd import _lib
    shape = _lib.Shape([2], [50], [1], [3, 2])
    N = [5]
    assert _lib.glm_workspace_bytes_common(shape, _lib.GLM_FP64, N, [0, 2, 4, 1, 3]) > 0
    for bad in ([0, 2, 5, 1, 3],      # column past N
                [0, 2, 2, 1, 3],      # repeated column
                [2, 0, 4, 1, 3],      # not increasing
                [0, 2, 4, -1, 3]):
        assert _lib.glm_workspace_bytes_common(shape, _lib.GLM_FP64, N, bad) == 0, bad
    wide = _lib.Shape([1], [50], [1], [6])
    assert _lib.glm_workspace_bytes_common(wide, _lib.GLM_FP64, [5], list(range(6))) == 0


def test_stream_mix_refuses_bad_arguments_before_any_launch(lib):
    """glm_stream_mix (the streaming-ceiling aid) validates its arguments on
    the host and returns GLM_EINVAL before touching a device: the pointers
    below are never dereferenced."""
    from ctypes import c_int64, c_void_p
    from paper_2510_14471_amd import _lib
    f = lib.glm_stream_mix
    f.argtypes = [c_void_p, c_void_p, ctypes.c_int32, c_void_p, ctypes.c_int32, c_int64,
                  c_void_p, ctypes.c_int32, c_int64, c_void_p]
    f.restype = ctypes.c_int
    aligned, misaligned = 0x10000, 0x10004
    ptrs = lambda *v: (c_void_p * len(v))(*v)            # noqa: E731
    lens = lambda *v: (c_int64 * len(v))(*v)             # noqa: E731
    E = _lib.GLM_EINVAL
    # too many streams of a kind
    assert f(ptrs(*[aligned] * 5), lens(*[64] * 5), 5, None, 0, 0, None, 0, 0, None) == E
    assert f(None, None, 0, ptrs(*[aligned] * 5), 5, 64, None, 0, 0, None) == E
    # misaligned, empty, or ragged read-only stream
    assert f(ptrs(misaligned), lens(64), 1, None, 0, 0, None, 0, 0, None) == E
    assert f(ptrs(aligned), lens(0), 1, None, 0, 0, None, 0, 0, None) == E
    assert f(ptrs(aligned), lens(66), 1, None, 0, 0, None, 0, 0, None) == E
    # read-write streams without a length, or ragged; write-only misaligned
    assert f(None, None, 0, ptrs(aligned), 1, 0, None, 0, 0, None) == E
    assert f(None, None, 0, ptrs(aligned), 1, 30, None, 0, 0, None) == E
    assert f(None, None, 0, None, 0, 0, ptrs(misaligned), 1, 64, None) == E
    # NULL arrays where streams are announced
    assert f(None, None, 1, None, 0, 0, None, 0, 0, None) == E
    assert f(None, None, 0, None, 0, 0, None, 1, 64, None) == E
