"""Full-size checks in the benchmark's launch configuration (2049^2 and the 3D 129^3 workload).

At these sizes the oracle does not solve, but it can (a) run its own search over every node, so the
GPU search is compared bit for bit on the whole grid, and (b) recompute the residual of the discrete
HJB system, max_k (A^k X - F^k)_i = X_i - U_i - dt * min_k G_k(X)_i, of a GPU step.  For these
M-matrices with row sums >= 1 (Section 3.4) the infinity norm of that residual bounds |X - X*|_inf,
where X* is the exact discrete solution (eq. nonlinear_sys), so each GPU step is certified against
it.  The oracle's search started from the GPU policy must also change nothing: the GPU policy is the
tie rule's fixed point at X.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _certify(inst, pb, Uprev, Unext, alpha, t_prev, dt, theta, res_gpu, rel_tol=1e-10):
    """The GPU policy keeps a control within tau of the minimum, so the residual of the discrete HJB system
    exceeds the final linear residual by at most dt*tau; both are recomputed here by the oracle."""
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    tau = pb.tau(Unext, Uprev, f)
    r = pb.improve(Unext, Uprev, theta, f, tau, alpha, want_extra=False)
    I = pb.interior
    R = Unext[I] - Uprev[I] - dt * r["gmin"][I]
    rinf = float(np.max(np.abs(R)))
    xinf = float(np.max(np.abs(Unext)))
    log(f"  residual of the discrete HJB system {rinf:.2e} (linear {res_gpu:.2e}, dt*tau {dt * tau:.2e}), "
        f"oracle search changes {r['changed']}")
    assert r["changed"] == 0
    assert rinf <= res_gpu + dt * tau + 1e-14 * max(1.0, xinf)
    # |X - X*|_inf <= |R|_inf for c = 0 (row sums of Section 3.4): the accuracy target
    assert rinf <= rel_tol * max(1.0, xinf)
    return rinf


def _bench_options(slhjb, precision=1):
    return slhjb.Options(precision=precision)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_h2049_search_bit_exact_full_grid(slhjb, theta):
    inst = workloads.config_h(2049)
    log(f"2049^2 search theta={theta}")
    pb = oracle.Problem(inst)
    X0 = inst.coords()
    t_prev, dt = 0.25, 1.0 / 64
    U = inst.exact(t_prev, X0)
    X = inst.exact(t_prev + dt, X0)
    X[pb.bd] = inst.psi[pb.bd]
    a_in = np.full(inst.N, 8, np.int16)
    a_in[pb.bd] = -1
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    tau = pb.tau(X, U, f)
    ref = pb.improve(X, U, theta, f, tau, a_in, want_extra=False)
    solver = slhjb.Solver.from_instance(inst, _bench_options(slhjb))
    da = torch.empty(inst.N, dtype=torch.int16, device="cuda")
    gmin = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    nch, tau_gpu = solver.policy_sweep(to_dev(X), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0,
                                       to_dev(a_in), da, gmin)
    assert tau_gpu == tau
    np.testing.assert_array_equal(to_np(da), ref["alpha"])
    np.testing.assert_array_equal(to_np(gmin), ref["gmin"])
    assert nch == ref["changed"]
    log(f"  {inst.N} nodes identical, {nch} changed controls")
    solver.close()


def _march_steps(slhjb, inst, n_steps, check_every=1, precision=1):
    pb = oracle.Problem(inst)
    solver = slhjb.Solver.from_instance(inst, _bench_options(slhjb, precision))
    g, psi, f0, f1 = to_dev(inst.g), to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1)
    Ua, Ub, Uc = g.clone(), psi.clone(), g.clone()
    alpha = torch.zeros(inst.N, dtype=torch.int16, device="cuda")
    t = 0.0
    worst = 0.0
    for n in range(n_steps):
        Ub.copy_(psi)
        dt, th = float(inst.dts[n]), float(inst.thetas[n])
        st = solver.step(Ua, Ub, f0, f1, t, dt, th, 1.0, alpha, Uc if n >= 1 else None,
                         float(inst.dts[n - 1]) if n >= 1 else 0.0)
        log(f"  step {n}: theta={th} pi={st.pi_iters} krylov={st.krylov_total} res={st.res_inf:.2e}")
        if n % check_every == 0 or n == n_steps - 1:
            worst = max(worst, _certify(inst, pb, to_np(Ua), to_np(Ub), to_np(alpha), t, dt, th, st.res_inf))
        t += dt
        Ua, Ub, Uc = Ub, Uc, Ua
    solver.close()
    return worst


@pytest.mark.timeout(400)
def test_h2049_march_certified(slhjb):
    """All 65 solves of the benchmark march (two implicit half steps, 63 Crank-Nicolson steps) in the mixed
    configuration; every 8th step (and the last) certified by the oracle."""
    inst = workloads.config_h(2049)
    log("2049^2 march, mixed precision")
    _march_steps(slhjb, inst, len(inst.dts), check_every=8)


@pytest.mark.timeout(400)
def test_c5_129_march_certified(slhjb):
    """3D workload (129^3, 64 directions), all 32 implicit steps in the mixed configuration; every 8th step
    (and the last) certified by the oracle."""
    inst = workloads.config_c5(129)
    log("129^3 march, mixed precision")
    _march_steps(slhjb, inst, len(inst.dts), check_every=8)


def test_c2_257_full_march_certified(slhjb):
    """All 65 solves of the 257^2 Crank-Nicolson drift march, every 8th step certified."""
    inst = workloads.config_c2(257)
    log("257^2 full march")
    _march_steps(slhjb, inst, len(inst.dts), check_every=8, precision=0)
