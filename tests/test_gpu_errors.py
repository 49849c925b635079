"""Failure handling on the GPU path: non-finite data end a march or a batched march with HJB_ENONFINITE (no
hang, no fault), and the handle solves correctly afterwards."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import log, to_dev, to_np
from test_gpu_batch import _batch_2d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _interior_node(inst):
    n0, n1 = inst.n[0], inst.n[1]
    return (n1 // 2) * n0 + n0 // 3


@pytest.mark.parametrize("where", ["f0", "g"])
@pytest.mark.parametrize("precond", [2, 3], ids=["vcycle", "amg"])
def test_march_reports_nonfinite_data(slhjb, where, precond):
    inst = workloads.config_c2(33, n_cn=2)
    log(f"non-finite {where}, precond={precond}")
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precond=precond))
    data = {k: getattr(inst, k).copy() for k in ("g", "psi", "f0", "f1")}
    data[where][_interior_node(inst)] = np.nan
    g, psi, f0, f1 = (to_dev(data[k]) for k in ("g", "psi", "f0", "f1"))
    U = torch.empty_like(g)
    with pytest.raises(slhjb.HJBError) as err:
        solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, inst.s, U)
    log(f"  {err.value}")
    assert err.value.code == slhjb.HJB_ENONFINITE
    # the same handle then marches clean data to the oracle's values
    g, psi, f0, f1 = (to_dev(getattr(inst, k)) for k in ("g", "psi", "f0", "f1"))
    solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, inst.s, U)
    ref = oracle.march(inst)
    rel = np.max(np.abs(to_np(U) - ref["U"])) / np.max(np.abs(ref["U"]))
    log(f"  clean march after the failure: rel {rel:.2e}")
    assert rel <= 1e-10
    solver.close()


def test_batch_reports_nonfinite_instance(slhjb):
    insts = _batch_2d()[:3]
    bad = 1
    insts[bad].f0 = insts[bad].f0.copy()
    insts[bad].f0[_interior_node(insts[bad])] = np.nan
    bt = slhjb.Batch(insts, slhjb.Options(precision=1))
    g, psi, f0, f1 = (to_dev(bt.concat(k)) for k in ("g", "psi", "f0", "f1"))
    U = torch.empty_like(g)
    with pytest.raises(slhjb.HJBError) as err:
        bt.solve(g, psi, f0, f1, insts[0].dts, insts[0].thetas, 1.0, U)
    log(f"  {err.value}")
    assert err.value.code == slhjb.HJB_ENONFINITE
    assert f"instance {bad}" in str(err.value)
    bt.close()


@pytest.mark.parametrize("opts,code", [(dict(max_krylov=1), "HJB_ENOCONV_KRYLOV"), (dict(max_pi=1), "HJB_ENOCONV_PI")],
                         ids=["krylov_limit", "pi_limit"])
def test_march_reports_iteration_limits(slhjb, opts, code):
    """A solve that needs more Krylov iterations, or a step that needs more policy iterations, than allowed
    ends with the corresponding status."""
    inst = workloads.config_c2(33, n_cn=2)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(**opts))
    g, psi, f0, f1 = (to_dev(getattr(inst, k)) for k in ("g", "psi", "f0", "f1"))
    U = torch.empty_like(g)
    with pytest.raises(slhjb.HJBError) as err:
        solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, inst.s, U)
    log(f"  {opts}: {err.value}")
    assert err.value.code == getattr(slhjb, code)
    solver.close()


def test_batch_reports_krylov_limit(slhjb):
    insts = _batch_2d()[:3]
    bt = slhjb.Batch(insts, slhjb.Options(precision=1, max_krylov=1))
    g, psi, f0, f1 = (to_dev(bt.concat(k)) for k in ("g", "psi", "f0", "f1"))
    U = torch.empty_like(g)
    with pytest.raises(slhjb.HJBError) as err:
        bt.solve(g, psi, f0, f1, insts[0].dts, insts[0].thetas, 1.0, U)
    log(f"  {err.value}")
    assert err.value.code == slhjb.HJB_ENOCONV_KRYLOV
    bt.close()
