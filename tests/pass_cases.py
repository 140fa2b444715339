"""Batches that reach each configuration of the projection passes, with the
configuration each one must select (single-precision inner solves "fp32",
double-precision solves "fp64").  Shared by the host-only check of the
selection (test_abi.py) and the GPU parity tests (test_gpu_pass_configs.py).

Keys of a configuration: rowvec (1 row-vector passes, 0 column-slot passes),
kv (rhs per lane), ks (16 = sixteen-rhs specialisation), omega (-16/-32/-64
matrix-core Omega apply, 32 Omega in registers, 0 Omega in LDS), nim (widest
block rounded up).  For the column-slot passes only rowvec is compared."""
import numpy as np

import synth


def _inst(rng, G, M, n_lo, n_hi, K, shift=0.3):
    n_i = rng.integers(n_lo, n_hi + 1, size=G).tolist()
    Omega = synth.sur._aat_plus(rng, G, shift)
    return synth.sur._instance(rng, M, n_i, Omega, K)


def _build(seed, specs):
    rng = np.random.default_rng(seed)
    return [_inst(rng, *s) for s in specs]


def cfg(rowvec, kv=None, ks=None, omega=None, nim=None):
    return dict(rowvec=rowvec, kv=kv, ks=ks, omega=omega, nim=nim)


# name -> (instance specs (G, M, n_lo, n_hi, K), expected fp32, expected fp64,
#          also run through the model reduction)
CASES = {
    # sixteen rhs and 33..64 equations: Omega on the matrix cores with G
    # padded to 64, one row group per wave
    "mfma_omega_g64": (
        [(33, 300, 3, 8, 16), (50, 420, 3, 8, 16), (64, 520, 3, 8, 16)],
        cfg(1, 4, 16, -64, 8), cfg(0), True),
    # rhs counts divisible by four (not all sixteen): four rhs per lane,
    # Omega column in registers
    "kv4_omega_registers": (
        [(6, 240, 3, 8, 4), (20, 420, 3, 8, 8), (32, 600, 3, 8, 8)],
        cfg(1, 4, 0, 32, 8), cfg(1, 2, 0, 32, 8), True),
    # twelve rhs and blocks of 25..28 columns: four rhs per lane, Omega in LDS
    "kv4_omega_lds_wide_blocks": (
        [(8, 500, 25, 28, 12), (12, 700, 25, 28, 12), (16, 900, 25, 28, 12)],
        cfg(1, 4, 0, 0, 32), cfg(1, 2, 0, 0, 32), False),
    # even rhs counts: two rhs per lane in both precisions
    "kv2": (
        [(5, 200, 3, 8, 2), (12, 380, 3, 8, 6), (20, 520, 3, 8, 6)],
        cfg(1, 2, 0, 32, 8), cfg(1, 2, 0, 32, 8), False),
    # more than 32 equations without sixteen rhs: Omega in LDS, one rhs per lane
    "kv1_omega_lds_g48": (
        [(40, 220, 3, 6, 1), (48, 260, 3, 6, 3)],
        cfg(1, 1, 0, 0, 8), cfg(1, 1, 0, 0, 8), False),
    # 70 equations with sixteen rhs: too many lanes per row for the
    # row-vector passes, so the column-slot passes run with sixteen rhs
    "column_slots_g70_k16": (
        [(70, 180, 3, 5, 16)],
        cfg(0), cfg(0), False),
}


def instances(name, seed=0):
    specs = CASES[name][0]
    return _build(1000 + seed + 17 * list(CASES).index(name), specs)


def matches(got, want):
    if want["rowvec"] == 0:
        return got["rowvec"] == 0
    return all(got[k] == v for k, v in want.items())
