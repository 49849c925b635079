"""BiCGSTAB, the Krylov baseline of Section 3.3, as the outer FP64 method of the linear solves: right-
preconditioned by the same V-cycle (FP64 or FP32) or Jacobi, same stopping rule and certificate as flexible
GMRES.  Its solves, marches and transposed (adjoint) solves meet the oracle to the same bounds."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import log, to_dev, to_np
from test_gpu_adjoint import _check_adjoint
from test_gpu_parity import _march_compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _linsolve_case(seed):
    inst = workloads.config_c2(65)
    pb = oracle.Problem(inst)
    alpha = workloads.random_policy(inst, seed)
    U, _ = workloads.random_fields(inst, seed=seed + 1)
    t_prev, dt, theta = 0.1, 1.0 / 64, 0.5
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    L = pb.assemble(alpha)
    E = oracle.explicit_part(pb, L, alpha, U, f, dt, theta)
    V0 = U.copy()
    V0[pb.bd] = inst.psi[pb.bd]
    Vref, _ = oracle.linear_solve(pb, L, alpha, V0, E, dt, theta, rtol=1e-15)
    return inst, alpha, U, V0, Vref, (t_prev, dt, theta)


@pytest.mark.parametrize("precision,precond", [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2)],
                         ids=["fp64-none", "fp64-jacobi", "fp64-vcycle", "mixed-jacobi", "mixed-vcycle"])
def test_bicgstab_linsolve_matches_oracle(slhjb, precision, precond):
    inst, alpha, U, V0, Vref, (t_prev, dt, theta) = _linsolve_case(7)
    log(f"BiCGSTAB linsolve precision={precision} precond={precond}")
    opts = slhjb.Options(precision=precision, precond=precond, krylov=slhjb.KRYLOV_BICGSTAB, max_krylov=4000)
    solver = slhjb.Solver.from_instance(inst, opts)
    dX = to_dev(V0)
    st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
    X = to_np(dX)
    rel = np.max(np.abs(X - Vref)) / np.max(np.abs(Vref))
    log(f"  krylov={st.krylov_total} res={st.res_inf:.2e} rel={rel:.2e}")
    assert st.krylov_total > 0 and st.krylov_total % 2 == 0
    assert rel <= 1e-11, rel
    assert st.res_inf <= 1e-13 * max(1.0, np.max(np.abs(X)))
    # the boundary values are untouched
    np.testing.assert_array_equal(X[inst.boundary_mask()], V0[inst.boundary_mask()])
    solver.close()


def test_bicgstab_and_fgmres_same_certificate(slhjb):
    """Both methods certify the same discrete solution: their results differ by less than the sum of the two
    residual bounds (M-matrix with row sums >= 1, Section 3.4), and a second BiCGSTAB solve from the first's
    result returns at once, leaving it unchanged bit for bit."""
    inst, alpha, U, V0, Vref, (t_prev, dt, theta) = _linsolve_case(37)
    args = (to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0)
    out = {}
    for kr in (slhjb.KRYLOV_FGMRES, slhjb.KRYLOV_BICGSTAB):
        solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1, krylov=kr))
        dX = to_dev(V0)
        st = solver.linsolve(*args, dX)
        out[kr] = (to_np(dX), st)
        if kr == slhjb.KRYLOV_BICGSTAB:
            X1 = to_np(dX)
            st2 = solver.linsolve(*args, dX)
            assert st2.krylov_total == 0
            np.testing.assert_array_equal(to_np(dX), X1)
        solver.close()
    (Xf, sf), (Xb, sb) = out[0], out[1]
    log(f"  FGMRES {sf.krylov_total} iterations res {sf.res_inf:.2e}; BiCGSTAB {sb.krylov_total} res {sb.res_inf:.2e}")
    assert np.max(np.abs(Xf - Xb)) <= sf.res_inf + sb.res_inf


@pytest.mark.parametrize("precision", [0, 1])
def test_bicgstab_march_c2(slhjb, precision):
    """65^2 Crank-Nicolson march with BiCGSTAB solves: values, every step's policy and fixed point."""
    inst = workloads.config_c2(65, n_cn=8)
    _march_compare(slhjb, inst, slhjb.Options(precision=precision, krylov=slhjb.KRYLOV_BICGSTAB))


def test_bicgstab_march_c1(slhjb):
    _march_compare(slhjb, workloads.config_c1(33), slhjb.Options(krylov=slhjb.KRYLOV_BICGSTAB))


def test_bicgstab_adjoint(slhjb):
    """Transposed solves of the adjoint with BiCGSTAB: gradients meet the dense oracle adjoint."""
    inst = workloads.config_c2(65, n_cn=4)
    for precision in (0, 1):
        _check_adjoint(slhjb, "c2_65 bicgstab", inst, precision, 2, krylov=slhjb.KRYLOV_BICGSTAB)


def test_bicgstab_option_checks(slhjb):
    inst = workloads.config_c2(17)
    with pytest.raises(slhjb.HJBError):
        slhjb.Solver.from_instance(inst, slhjb.Options(krylov=slhjb.KRYLOV_BICGSTAB, restart=2))
    with pytest.raises(slhjb.HJBError):
        slhjb.Solver.from_instance(inst, slhjb.Options(krylov=2))
    solver = slhjb.Solver.from_instance(inst, slhjb.Options())
    solver.set_options(slhjb.Options(krylov=slhjb.KRYLOV_BICGSTAB))
    solver.close()
