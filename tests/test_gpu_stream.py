"""The streaming-ceiling kernel (glm_stream_mix), a measurement aid for the
projection passes' roofline: every written element is what its definition
says, across several workgroups, a ragged tail and streams of different
lengths; bad arguments are refused before any launch."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


def _expected(ro, rw_old, n):
    acc = torch.zeros(n, dtype=torch.float64)
    for t in ro:
        m = min(n, t.numel())
        acc[:m] += t[:m].double().cpu()
    return [0.5 * o.double().cpu() + acc for o in rw_old], acc


@pytest.mark.parametrize("lens", [(12, 4100, 9000), (1024 * 16 + 4, 64, 20)])
def test_stream_mix_values(glmlib, lens):
    glm = glmlib
    g = torch.Generator(device="cuda").manual_seed(7)
    n_rw, n_wo = 8196, 5000
    print(f"[case] stream mix ro lengths {lens} rw {n_rw} wo {n_wo}", flush=True)
    ro = [torch.randn(L, device="cuda", generator=g) for L in lens]
    rw = [torch.randn(n_rw, device="cuda", generator=g) for _ in range(2)]
    wo = [torch.full((n_wo,), 3.0, device="cuda")]
    old = [t.clone() for t in rw]
    glm.glm_stream_mix(ro, rw, wo)
    torch.cuda.synchronize()
    exp_rw, acc = _expected(ro, old, n_rw)
    for t, e in zip(rw, exp_rw):
        assert torch.allclose(t.double().cpu(), e, rtol=0, atol=1e-5)
    _, acc_wo = _expected(ro, [], n_wo)
    assert torch.allclose(wo[0].double().cpu(), acc_wo, rtol=0, atol=1e-5)


def test_stream_mix_read_only_and_copy(glmlib):
    glm = glmlib
    x = torch.randn(4 * 70001, device="cuda")
    y = torch.zeros_like(x)
    print("[case] stream mix copy", flush=True)
    glm.glm_stream_mix([x], [], [y])
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    glm.glm_stream_mix([x, y], [], [])   # reads only
    torch.cuda.synchronize()


def test_stream_mix_rejects_bad_arguments(glmlib):
    glm = glmlib
    x = torch.randn(1024, device="cuda")
    with pytest.raises(glm.GLMError):
        glm.glm_stream_mix([x[1:1021]], [], [])          # not 16-byte aligned
    with pytest.raises(glm.GLMError):
        glm.glm_stream_mix([x[:1022]], [], [])           # length not a multiple of 4
    with pytest.raises(glm.GLMError):
        glm.glm_stream_mix([x] * 5, [], [])              # too many streams
    with pytest.raises(glm.GLMError):
        glm.glm_stream_mix([x[:0]], [], [])              # empty read-only stream
