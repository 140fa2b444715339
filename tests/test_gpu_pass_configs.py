"""Every configuration the planner can select for the projection passes,
run on the GPU and compared with the oracle (1e-10 per (instance, rhs),
normwise and element-wise).  Each test asserts, from the solve's own
statistics, that the configuration it targets is the one that ran."""
import numpy as np
import pytest

import pass_cases
from conftest import rel_err
from oracle import gls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module")
def glmlib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2510_14471_amd as glm
    return glm


_ORACLE = {}


def oracle_of(name, insts):
    if name not in _ORACLE:
        _ORACLE[name] = [gls.sur_gls(i) for i in insts]
    return _ORACLE[name]


def check_elementwise(insts, out, ref):
    for b, inst in enumerate(insts):
        beta_o, U_o = ref[b]
        for k in range(inst.K):
            for got, want in ((out["beta"][b][:, k], beta_o[:, k]),
                              (out["u"][b][:, :, k], U_o[:, :, k])):
                assert rel_err(got, want) <= TOL, (b, k, rel_err(got, want))
                scale = np.abs(want).max()
                assert np.abs(got - want).max() <= TOL * scale, (b, k)
            assert out["info"][b][k] in (0, 1), (b, k, out["info"][b][k])


@pytest.mark.parametrize("reduce", [False, True], ids=["full", "reduced"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(pass_cases.CASES))
def test_pass_configuration_parity(glmlib, name, precision, reduce):
    specs, want32, want64, reducible = pass_cases.CASES[name]
    if reduce and not reducible:
        pytest.skip("case not run through the model reduction")
    insts = pass_cases.instances(name)
    print(f"[case] {name} {precision} reduce={reduce} G={[i.G for i in insts]} "
          f"M={[i.M for i in insts]} K={[i.K for i in insts]}", flush=True)
    lay, d = glmlib.pack_instances(insts)
    s = glmlib.SURSolver(lay, precision, reduce=reduce)
    s.factor(d["X"])
    beta, u, _, info, _ = s.solve(d["Omega"], d["y"], tol=1e-13 if precision == "mixed"
                                  else 1e-12)
    torch.cuda.synchronize()
    st = s.stats()
    out = dict(beta=glmlib.unpack(lay, beta, "beta"), u=glmlib.unpack(lay, u, "u"),
               info=glmlib.unpack(lay, info, "rhs"))
    s.close()
    assert pass_cases.matches(st["fp64_passes"], want64), st
    if precision == "mixed":
        assert pass_cases.matches(st["fp32_passes"], want32), st
    check_elementwise(insts, out, oracle_of(name, insts))
