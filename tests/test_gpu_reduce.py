"""SUR model reduction on the GPU (GLM_REDUCED): parity with the oracle's
direct GLS of the full model, beta and u, in both precisions; several
Householder panels (n > 32), instances with M <= n (nothing to drop),
restrictions, sixteen rhs (the matrix-core passes of the reduced problem),
and the batched workload at full size.  The reduced route itself is pinned
on the CPU (oracle.reduce against oracle.gls)."""
import numpy as np
import pytest

import synth
from conftest import assert_all_pairs, batch512_with_oracle, rel_err
from oracle import gls
from test_gpu_parity import check_against_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


def run_reduced(glm, insts, precision, tol=1e-13):
    print(f"[case] reduced {precision} B={len(insts)} G={[i.G for i in insts][:6]} "
          f"M={[i.M for i in insts][:6]} n={[i.n for i in insts][:6]} K={insts[0].K} "
          f"k={[i.kc for i in insts][:6]}", flush=True)
    lay, d = glm.pack_instances(insts)
    s = glm.SURSolver(lay, precision, reduce=True)
    s.factor(d["X"], d["Rc"])
    beta, u, _, info, iters = s.solve(d["Omega"], d["y"], d["r"], tol=tol)
    torch.cuda.synchronize()
    out = dict(beta=glm.unpack(lay, beta, "beta"), u=glm.unpack(lay, u, "u"),
               info=glm.unpack(lay, info, "rhs"), iters=glm.unpack(lay, iters, "rhs"),
               stats=s.stats(), solver=s, dev=d)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_ragged_batch(glmlib, precision):
    insts = list(synth.small_batch(seed=161, B=6, G_rng=(1, 6), M_rng=(30, 400),
                                   n_rng=(1, 7), K_rng=(1, 5)))
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_several_panels(glmlib, precision):
    """n from 33 to ~140: two to five Householder panels of 32 columns."""
    insts = list(synth.small_batch(seed=163, B=3, G_rng=(5, 12), M_rng=(300, 900),
                                   n_rng=(6, 12), K_rng=(2, 4)))
    insts += list(synth.small_batch(seed=165, B=1, G_rng=(4, 4), M_rng=(200, 200),
                                    n_rng=(8, 8), K_rng=(3, 3)))        # n = 32 exactly
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)


def test_reduced_when_nothing_is_dropped(glmlib):
    """M <= n + 1: the rotation keeps every observation (and M < n uses only M
    reflectors)."""
    insts = list(synth.small_batch(seed=167, B=1, G_rng=(12, 12), M_rng=(3, 3),
                                   n_rng=(1, 2), K_rng=(3, 3)))
    insts += list(synth.small_batch(seed=169, B=1, G_rng=(4, 4), M_rng=(13, 13),
                                    n_rng=(3, 3), K_rng=(2, 2)))
    out = run_reduced(glmlib, insts, "fp64")
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_with_restrictions(glmlib, precision):
    insts = list(synth.small_batch(seed=171, B=4, G_rng=(2, 5), M_rng=(40, 200),
                                   n_rng=(2, 5), K_rng=(1, 3), constraints=3))
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)
    for b, inst in enumerate(insts):
        if inst.kc:
            assert np.abs(inst.Rc @ out["beta"][b] - inst.r).max() < 1e-10


def test_reduced_sixteen_rhs(glmlib):
    insts = list(synth.small_batch(seed=173, B=3, G_rng=(4, 20), M_rng=(500, 2500),
                                   n_rng=(3, 12), K_rng=(16, 16)))
    out = run_reduced(glmlib, insts, "mixed")
    check_against_oracle(insts, out)


def test_reduced_singular_omega_reports_breakdown(glmlib):
    """Omega^-1 of the dropped rows needs a positive definite Omega: a singular
    one reports GLM_INFO_BREAKDOWN for every rhs of that instance only."""
    good = list(synth.small_batch(seed=175, B=1, G_rng=(3, 3), M_rng=(80, 80),
                                  n_rng=(2, 3), K_rng=(2, 2)))
    bad = list(synth.small_batch(seed=177, B=1, G_rng=(5, 5), M_rng=(120, 120),
                                 n_rng=(2, 3), K_rng=(2, 2), singular=2))
    out = run_reduced(glmlib, good + bad, "fp64")
    assert all(v == -11 for v in out["info"][1]), out["info"][1]
    check_against_oracle(good, {k: v[:1] if isinstance(v, list) else v
                                for k, v in out.items()})


def test_reduced_solver_has_no_backward(glmlib):
    insts = list(synth.small_batch(seed=179, B=1, G_rng=(2, 2), M_rng=(30, 30),
                                   n_rng=(2, 2), K_rng=(1, 1)))
    out = run_reduced(glmlib, insts, "fp64")
    s, d = out["solver"], out["dev"]
    gb = torch.zeros(insts[0].n, dtype=torch.float64, device="cuda")
    u0 = torch.zeros(insts[0].M * insts[0].G, dtype=torch.float64, device="cuda")
    with pytest.raises(glmlib.GLMError):
        s.backward(d["Omega"], gb, u0, gb)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_reduced_batched_workload_full_size(glmlib, precision):
    """The batched workload (512 instances x 16 rhs) through the reduction,
    in the launch configuration the benchmark times: all 8,192 (instance,
    rhs) pairs against the oracle, normwise and element-wise, and
    Sigma u + X beta = y, X_i^T u_i = 0 on every instance."""
    from test_gpu_fullsize import identities
    insts, refs = batch512_with_oracle()
    out = run_reduced(glmlib, insts, precision, tol=1e-12)
    worst = assert_all_pairs(insts, refs, out["beta"], out["u"], out["info"], TOL)
    print(f"[worst] reduced {precision} {worst}", flush=True)
    out["solver"].close()
    worst = (0.0, 0.0)
    for b, inst in enumerate(insts):
        r1, r2 = identities(inst, out["beta"][b], out["u"][b])
        worst = (max(worst[0], r1), max(worst[1], r2))
    assert worst[0] <= TOL and worst[1] <= TOL, worst


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_repeated_intercepts(glmlib, precision):
    """The two widest instances of the batched workload (G = 32, n = 417 and
    419): the intercept repeated in every equation makes W exactly rank
    deficient, and later dependent columns leave subcolumns of ~1e-160 whose
    squares underflow; the QR must take them as zero for Q to stay
    orthogonal."""
    insts = list(synth.config2(subset=[12, 228]))
    out = run_reduced(glmlib, insts, precision, tol=1e-12)
    check_against_oracle(insts, out)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_at_the_equation_limit(glmlib, precision):
    """G = 64, the most equations the reduction takes (Omega^-1 and the
    dropped rows' Z = (Q^T Y) Omega^-1 use 64 x 64 arrays in LDS), with W of
    128 to 192 columns (four to six Householder panels) and rows in several
    apply segments."""
    insts = list(synth.small_batch(seed=181, B=2, G_rng=(64, 64), M_rng=(300, 1500),
                                   n_rng=(2, 3), K_rng=(1, 3)))
    assert all(i.G == 64 for i in insts)
    out = run_reduced(glmlib, insts, precision)
    check_against_oracle(insts, out)
