"""Edge cases of the HIP path against the oracle (GPU): the largest supported
block width, equation count and restriction count, systems the iteration
solves at once, and restrictions that fix beta completely."""
import numpy as np
import pytest

import synth
from conftest import rel_err
from oracle import gls
from test_gpu_parity import check_against_oracle, run

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_widest_blocks_with_sixteen_rhs(glmlib, precision):
    """n_i = 64 (the widest block the QR kernel factors) with K = 16."""
    insts = list(synth.small_batch(seed=43, B=2, G_rng=(2, 3), M_rng=(200, 260),
                                   n_rng=(64, 64), K_rng=(16, 16)))
    out = run(glmlib, insts, precision, tol=1e-13)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_most_equations(glmlib, precision):
    """G = 256 equations (Omega of 64k entries, the largest accepted) and a
    G = 100 instance next to a small one: the column-slot passes."""
    big = list(synth.small_batch(seed=47, B=1, G_rng=(256, 256), M_rng=(40, 40),
                                 n_rng=(1, 1), K_rng=(1, 1), shift=2.0))
    mid = list(synth.small_batch(seed=53, B=2, G_rng=(3, 100), M_rng=(60, 120),
                                 n_rng=(1, 3), K_rng=(1, 2), shift=1.0))
    insts = big + mid
    out = run(glmlib, insts, precision, tol=1e-13)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_most_restrictions(glmlib, precision):
    """k = 64 cross-equation restrictions (the largest accepted)."""
    insts = list(synth.small_batch(seed=59, B=2, G_rng=(4, 5), M_rng=(80, 120),
                                   n_rng=(17, 20), K_rng=(1, 2), constraints=64))
    assert all(i.kc == 64 for i in insts)
    out = run(glmlib, insts, precision, tol=1e-13, want_uc=True)
    check_against_oracle(insts, out)
    for b, inst in enumerate(insts):
        assert np.abs(inst.Rc @ out["beta"][b] - inst.r).max() < 1e-9


def test_restrictions_that_fix_beta(glmlib):
    """k = n: R_c is square, so beta = R_c^-1 r whatever y is."""
    inst = synth.small_batch(seed=61, B=1, G_rng=(2, 2), M_rng=(30, 30),
                             n_rng=(2, 3), K_rng=(1, 1))[0]
    rng = np.random.default_rng(1)
    inst.Rc = rng.standard_normal((inst.n, inst.n)) + 3.0 * np.eye(inst.n)
    inst.r = inst.Rc @ inst.beta_true
    out = run(glmlib, [inst], "fp64", tol=1e-13)
    assert rel_err(out["beta"][0], inst.beta_true) < 1e-10
    beta_o, U_o, _ = gls.restricted_gls(inst)
    assert rel_err(out["beta"][0], beta_o) < 1e-10
    assert rel_err(out["u"][0], U_o) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_right_hand_sides(glmlib, precision):
    """y = 0 gives beta = 0 and u = 0 before any iteration; the other rhs of
    the same instance are unaffected."""
    insts = list(synth.small_batch(seed=67, B=2, G_rng=(2, 4), M_rng=(50, 90),
                                   n_rng=(1, 4), K_rng=(3, 3)))
    for inst in insts:
        inst.Y[:, :, 1] = 0.0
    out = run(glmlib, insts, precision, tol=1e-13)
    for b, inst in enumerate(insts):
        assert np.abs(out["beta"][b][:, 1]).max() == 0.0
        assert np.abs(out["u"][b][:, :, 1]).max() == 0.0
        assert out["info"][b][1] == 0
    check_against_oracle(insts, out)


def test_scaled_identity_omega_needs_one_iteration(glmlib):
    """Omega = w I: with D = alpha I (alpha = max w_ii) the preconditioned
    operator is the identity, the iteration ends after one step, and GLS is
    blockwise OLS."""
    insts = list(synth.small_batch(seed=71, B=2, G_rng=(2, 5), M_rng=(40, 80),
                                   n_rng=(1, 4), K_rng=(1, 2)))
    for inst in insts:
        inst.Omega = 2.5 * np.eye(inst.G)
    out = run(glmlib, insts, "fp64", tol=1e-13)
    for b, inst in enumerate(insts):
        for k in range(inst.K):
            assert out["iters"][b][k] == 1, out["iters"][b]
            for i in range(inst.G):
                o, ni = inst.col_off[i], inst.n_i[i]
                ols = np.linalg.lstsq(inst.X(i), inst.Y[:, i, k], rcond=None)[0]
                assert rel_err(out["beta"][b][o:o + ni, k], ols) < 1e-10


def test_ill_conditioned_block_keeps_orthonormal_factors(glmlib):
    """A block with two nearly collinear columns (condition ~1e7): the
    Householder factors still come out orthonormal, reproduce X and count as
    full rank (a Gram-based factorization would lose about eps cond^2)."""
    inst = synth.small_batch(seed=73, B=1, G_rng=(3, 3), M_rng=(400, 400),
                             n_rng=(4, 6), K_rng=(1, 1))[0]
    rng = np.random.default_rng(3)
    o = inst.col_off[1]
    inst.W[:, o + 1] = inst.W[:, o] + 1e-7 * rng.standard_normal(inst.M)
    lay, d = glmlib.pack_instances([inst])
    s = glmlib.SURSolver(lay, "fp64")
    s.factor(d["X"])
    Q, R, rank = s.factors()
    Q = glmlib.unpack(lay, Q, "X")[0]
    R = R.cpu().numpy()
    assert not rank.cpu().numpy().any()
    eps = np.finfo(float).eps
    ro = 0
    for i in range(inst.G):
        ni = inst.n_i[i]
        Qi = Q[:, inst.col_off[i]:inst.col_off[i] + ni]
        Ri = R[ro:ro + ni * ni].reshape(ni, ni)
        ro += ni * ni
        Xi = inst.X(i)
        assert np.abs(Qi.T @ Qi - np.eye(ni)).max() <= 20 * ni * eps * np.sqrt(inst.M)
        assert np.abs(Xi - Qi @ Ri).max() <= 20 * eps * np.abs(Xi).max() * np.sqrt(inst.M)
