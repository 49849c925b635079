"""Parity of the HIP path (through the C ABI) with the CPU oracle on identical seeded inputs.

The sweep must match bit for bit (policy indices, minimum values, tie counts, margins and the tie
tolerance).  Operator applications match to rounding; solves and marches match to 1e-10 relative
(the solves stop on an infinity-norm residual certificate of 1e-13).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import log, to_dev, to_np
from policy_parity import check_march_policies

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _toy(n, K, P, seed, drift=True, c=False, h=None, scale=1.0):
    rng = np.random.default_rng(seed)
    dim = len(n)
    N = int(np.prod(n))
    h = h if h is not None else 1.0 / (max(n) - 1)
    sig = rng.normal(size=(K, P, dim)) * scale
    b = rng.normal(size=(K, dim)) * 0.4 if drift else None
    cc = -rng.uniform(0.0, 1.0, size=K) if c else None
    inst = workloads.Instance(name=f"toy{n}", dim=dim, n=tuple(n), lo=(0.0,) * dim, h=h, K=K, P=P, sigma=sig,
                              drift=b, c=cc, f0=rng.normal(size=N), f1=rng.normal(size=N), g=rng.normal(size=N),
                              psi=np.zeros(N), dts=np.array([0.05, 0.05]), thetas=np.array([1.0, 0.5]))
    inst.psi = np.where(inst.boundary_mask(), rng.normal(size=N) * 0.3, 0.0)
    return inst


def _xscaled_toy(n, seed, K=5, P=2):
    """x-scaled coefficients on an off-origin ragged box with a drift of several cells (truncated drift)."""
    inst = _toy(n, K=K, P=P, seed=seed, c=True)
    rng = np.random.default_rng(seed + 100)
    inst.lo = (0.5, 0.25)
    inst.sigma = rng.normal(size=(K, P, 2)) * 0.7
    inst.drift = rng.normal(size=(K, 2)) * 3.0
    inst.coef_model = "xscaled"
    return inst


SWEEP_CASES = [
    ("c1_33", lambda: workloads.config_c1(33)),
    ("c2_65", lambda: workloads.config_c2(65)),
    ("c2_257", lambda: workloads.config_c2(257)),
    ("c5_17", lambda: workloads.config_c5(17)),
    ("ragged_2d", lambda: _toy((37, 29), K=7, P=2, seed=3, c=True)),
    ("ragged_3d", lambda: _toy((11, 9, 13), K=5, P=1, seed=4)),
    ("single_control", lambda: _toy((21, 21), K=1, P=1, seed=5)),
    ("c4_65_xscaled", lambda: workloads.c4_instance(65, 0.15, 0.3, 0.4, 0.03)),
    ("xscaled_ragged", lambda: _xscaled_toy((31, 23), seed=6)),
]


@pytest.mark.parametrize("name,mk", SWEEP_CASES, ids=[c[0] for c in SWEEP_CASES])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_sweep_bit_exact(slhjb, name, mk, theta):
    inst = mk()
    log(f"sweep {name} theta={theta} n={inst.n} K={inst.K}")
    pb = oracle.Problem(inst)
    X, U = workloads.random_fields(inst, seed=11)
    a_in = workloads.random_policy(inst, seed=12)
    t_prev, dt = 0.25, 1.0 / 64
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    tau = pb.tau(X, U, f)
    ref = pb.improve(X, U, theta, f, tau, a_in)
    solver = slhjb.Solver.from_instance(inst)
    dX, dU, df0, df1 = to_dev(X), to_dev(U), to_dev(inst.f0), to_dev(inst.f1)
    da_in = to_dev(a_in)
    da_out = torch.empty_like(da_in)
    gmin = torch.empty_like(dX)
    margin = torch.empty_like(dX)
    ties = torch.empty(inst.N, dtype=torch.int32, device=dX.device)
    nch, tau_gpu = solver.policy_sweep(dX, dU, df0, df1, t_prev, dt, theta, 1.0, da_in, da_out, gmin, margin, ties)
    assert tau_gpu == tau
    np.testing.assert_array_equal(to_np(da_out), ref["alpha"])
    np.testing.assert_array_equal(to_np(gmin), ref["gmin"])
    np.testing.assert_array_equal(to_np(ties), ref["ties"])
    np.testing.assert_array_equal(to_np(margin), ref["margin"])
    assert nch == ref["changed"]
    solver.close()


APPLY_CASES = [
    ("c2_65", lambda: workloads.config_c2(65)),
    ("c5_17", lambda: workloads.config_c5(17)),
    ("ragged_2d_c", lambda: _toy((37, 29), K=7, P=2, seed=3, c=True)),
    ("ragged_3d", lambda: _toy((11, 9, 13), K=5, P=1, seed=4)),
    ("c4_65_xscaled", lambda: workloads.c4_instance(65, 0.15, 0.3, 0.4, 0.03)),
    ("xscaled_ragged", lambda: _xscaled_toy((31, 23), seed=6)),
]


@pytest.mark.parametrize("name,mk", APPLY_CASES, ids=[c[0] for c in APPLY_CASES])
def test_apply_matches_assembled_matrix(slhjb, name, mk):
    inst = mk()
    log(f"apply {name}")
    pb = oracle.Problem(inst)
    rng = np.random.default_rng(5)
    x = rng.normal(size=inst.N)
    alpha = workloads.random_policy(inst, 6)
    dt, theta = 0.03, 0.7
    L = pb.assemble(alpha)
    y_ref = x - theta * dt * (L @ x + pb.c_of(alpha) * x)
    y_ref[pb.bd] = 0.0
    solver = slhjb.Solver.from_instance(inst)
    dy = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    solver.apply(to_dev(alpha), to_dev(x), dy, dt, theta)
    y = to_np(dy)
    np.testing.assert_allclose(y, y_ref, rtol=1e-13, atol=1e-13 * np.max(np.abs(y_ref)))
    solver.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("precond", [1, 2])
def test_linsolve_matches_oracle(slhjb, precision, precond):
    inst = workloads.config_c2(65)
    log(f"linsolve precision={precision} precond={precond}")
    pb = oracle.Problem(inst)
    alpha = workloads.random_policy(inst, 7)
    U, _ = workloads.random_fields(inst, seed=8)
    t_prev, dt, theta = 0.1, 1.0 / 64, 0.5
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    L = pb.assemble(alpha)
    E = oracle.explicit_part(pb, L, alpha, U, f, dt, theta)
    V0 = U.copy()
    V0[pb.bd] = inst.psi[pb.bd]
    Vref, _ = oracle.linear_solve(pb, L, alpha, V0, E, dt, theta, rtol=1e-15)
    opts = slhjb.Options(precision=precision, precond=precond)
    solver = slhjb.Solver.from_instance(inst, opts)
    dX = to_dev(V0)
    st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
    X = to_np(dX)
    log(f"  krylov={st.krylov_total} res={st.res_inf:.2e}")
    rel = np.max(np.abs(X - Vref)) / np.max(np.abs(Vref))
    assert rel <= 1e-11, rel
    assert st.res_inf <= 1e-13 * max(1.0, np.max(np.abs(X)))
    solver.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_linsolve_from_converged_start(slhjb, precision):
    """A solve that starts at the certificate returns at once: the first Arnoldi step queued ahead of the
    residual read is discarded and the iterate is left as it was, bit for bit."""
    inst = workloads.config_c2(65)
    log(f"linsolve from a converged start, precision={precision}")
    alpha = workloads.random_policy(inst, 27)
    U, _ = workloads.random_fields(inst, seed=28)
    V0 = U.copy()
    V0[inst.boundary_mask()] = inst.psi[inst.boundary_mask()]
    args = (to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), 0.1, 1.0 / 64, 0.5, 1.0)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=precision))
    dX = to_dev(V0)
    st1 = solver.linsolve(*args, dX)
    X1 = to_np(dX)
    st2 = solver.linsolve(*args, dX)
    log(f"  first solve {st1.krylov_total} iterations, second {st2.krylov_total}")
    assert st1.krylov_total > 0 and st2.krylov_total == 0
    np.testing.assert_array_equal(to_np(dX), X1)
    solver.close()


@pytest.mark.parametrize("restart", [9, 24])
def test_linsolve_long_arnoldi(slhjb, restart):
    """Jacobi-preconditioned FGMRES(m) runs every Arnoldi step of its cycles: the fused Gram-Schmidt kernels
    for bases of 1 ... 8 vectors and the separate update and sums beyond; the solve still meets the oracle."""
    inst = workloads.config_c2(65)
    log(f"linsolve restart={restart}")
    pb = oracle.Problem(inst)
    alpha = workloads.random_policy(inst, 17)
    U, _ = workloads.random_fields(inst, seed=18)
    t_prev, dt, theta = 0.1, 1.0 / 64, 0.5
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    L = pb.assemble(alpha)
    E = oracle.explicit_part(pb, L, alpha, U, f, dt, theta)
    V0 = U.copy()
    V0[pb.bd] = inst.psi[pb.bd]
    Vref, _ = oracle.linear_solve(pb, L, alpha, V0, E, dt, theta, rtol=1e-15)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=0, precond=1, restart=restart))
    dX = to_dev(V0)
    st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
    X = to_np(dX)
    log(f"  krylov={st.krylov_total} res={st.res_inf:.2e}")
    assert st.krylov_total >= 10  # Arnoldi steps with bases beyond the fused kernels' 8 vectors
    rel = np.max(np.abs(X - Vref)) / np.max(np.abs(Vref))
    assert rel <= 1e-11, rel
    assert st.res_inf <= 1e-13 * max(1.0, np.max(np.abs(X)))
    solver.close()


def _march_compare(slhjb, inst, opts=None, tol=1e-10):
    """Values within tol of the oracle at the end, policies identical at every clear decision of every
    step, and every GPU step the tie rule's fixed point with a certified discrete HJB residual."""
    ref = oracle.march(inst, keep_policies=True, keep_values=True)
    solver = slhjb.Solver.from_instance(inst, opts)
    g, psi, f0, f1 = to_dev(inst.g), to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1)
    U = torch.empty_like(g)
    pol = torch.empty((len(inst.dts), inst.N), dtype=torch.int16, device=g.device)
    vals = torch.empty((len(inst.dts) + 1, inst.N), dtype=torch.float64, device=g.device)
    psi1 = None if inst.psi1 is None else to_dev(inst.psi1)
    st = solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, inst.s, U, pol, vals, psi1=psi1)
    Ug = to_np(U)
    rel = np.max(np.abs(Ug - ref["U"])) / np.max(np.abs(ref["U"]))
    log(f"  {inst.name}: steps={st.steps_done} krylov={st.krylov_total} pi={st.pi_total} rel={rel:.2e}")
    assert st.steps_done == len(inst.dts)
    assert rel <= tol, rel
    vg = to_np(vals)
    steps_rel = np.max(np.abs(vg - ref["values"]), axis=1) / np.maximum(np.max(np.abs(ref["values"]), axis=1), 1e-300)
    assert np.all(steps_rel <= tol), steps_rel
    near = check_march_policies(inst, ref, to_np(pol), vg, s=inst.s, log=log)
    solver.close()
    return rel, near


def test_march_c1(slhjb):
    inst = workloads.config_c1(33)
    _march_compare(slhjb, inst)


@pytest.mark.parametrize("max_levels", [2, 0], ids=["two-level", "deep"])
@pytest.mark.parametrize("precision", [0, 1])
def test_march_c2_small(slhjb, precision, max_levels):
    """65^2 Crank-Nicolson march: the default two-level hierarchy and the full one (65, 33, 17)."""
    inst = workloads.config_c2(65, n_cn=8)
    _march_compare(slhjb, inst, slhjb.Options(precision=precision, max_levels=max_levels))


def test_march_c5_small(slhjb):
    inst = workloads.config_c5(17, n_steps=4)
    _march_compare(slhjb, inst, slhjb.Options(precision=1))


@pytest.mark.timeout(400)
def test_march_c5_33(slhjb):
    """The 3D workload at the oracle's stated size (33^3, 64 Fibonacci-hemisphere directions), its first four
    implicit steps: values, every step's policy and fixed point."""
    inst = workloads.config_c5(33, n_steps=4)
    _march_compare(slhjb, inst, slhjb.Options(precision=1))


def test_march_ragged_no_coarsening(slhjb):
    inst = _toy((30, 27), K=4, P=2, seed=9, c=True)
    _march_compare(slhjb, inst, slhjb.Options(precond=2))


@pytest.mark.parametrize("precision", [0, 1])
def test_march_c4_xscaled(slhjb, precision):
    """Two-asset x-scaled instance at 65^2, all 50 implicit steps."""
    inst = workloads.c4_instance(65, 0.12, 0.29, 0.35, 0.02)
    _march_compare(slhjb, inst, slhjb.Options(precision=precision))


def test_march_xscaled_ragged(slhjb):
    inst = _xscaled_toy((30, 27), seed=9)
    _march_compare(slhjb, inst, slhjb.Options(precision=1))


NEAR_CASES = [("c1_33", lambda: workloads.config_c1(33)), ("c2_65_cn", lambda: workloads.config_c2(65, n_cn=4)),
              ("problem_b_41", lambda: workloads.problem_b(41, dt=0.125))]


@pytest.mark.parametrize("name,mk", NEAR_CASES, ids=[c[0] for c in NEAR_CASES])
def test_step_near_tie_count(slhjb, name, mk):
    """hjb_step reports the near ties of its returned policy: interior nodes whose second-best G_k lies within
    1e3 * tau of the best.  The count equals the oracle's at the GPU's own values (identical searches), and the
    flag is set exactly when it is non-zero.  Problem B's Hamiltonian does not depend on the control in the
    continuum, so nearly every node is a near tie there."""
    inst = mk()
    pb = oracle.Problem(inst)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    g, psi = to_dev(inst.g), to_dev(inst.psi)
    f0, f1 = to_dev(np.ascontiguousarray(inst.f0)), to_dev(np.ascontiguousarray(inst.f1))
    Ua, Ub = g.clone(), psi.clone()
    alpha = torch.zeros(inst.N, dtype=torch.int16, device="cuda")
    t = 0.0
    for n in range(min(3, len(inst.dts))):
        Ub.copy_(psi)
        dt, th = float(inst.dts[n]), float(inst.thetas[n])
        st = solver.step(Ua, Ub, f0, f1, t, dt, th, 1.0, alpha)
        Uprev, X = to_np(Ua), to_np(Ub)
        f = pb.f_at(inst.f0, inst.f1, t + th * dt)
        tau = pb.tau(X, Uprev, f)
        r = pb.improve(X, Uprev, th, f, tau, to_np(alpha), want_extra=True)
        I = pb.interior
        near = int(np.sum(((r["ties"] > 1) | (r["margin"] < 1e3 * tau))[I]))
        log(f"  {name} step {n}: near ties gpu {st.n_near_ties} oracle {near} of {I.size}, flags {st.flags}")
        assert r["changed"] == 0
        assert st.n_near_ties == near
        assert bool(st.flags & slhjb.FLAG_NEAR_TIES) == (near > 0)
        t += dt
        Ua, Ub = Ub, Ua
    solver.close()


@pytest.mark.parametrize("max_levels", [2, 0], ids=["two-level", "deep"])
def test_vcycle_graph_replays_match_eager(slhjb, max_levels):
    """Replayed V-cycle graphs launch the same kernels as the eager path: every replay must give the
    eager result bit for bit, also with eager work and synchronisations between replays."""
    inst = workloads.config_c2(129)
    log("graph replay vs eager")
    alpha = workloads.random_policy(inst, 21)
    U, _ = workloads.random_fields(inst, seed=22)
    V0 = U.copy()
    V0[inst.boundary_mask()] = inst.psi[inst.boundary_mask()]
    args = (to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), 0.1, 1.0 / 64, 0.5, 1.0)
    outs = []
    for use_graphs in (0, 1, 1, 1):
        solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1, use_graphs=use_graphs,
                                                                max_levels=max_levels))
        for rep in range(2):
            dX = to_dev(V0)
            st = solver.linsolve(*args, dX)
            torch.cuda.synchronize()
            outs.append(to_np(dX))
            _ = (dX * 2.0).sum().item()   # unrelated eager work between replays
        solver.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


@pytest.mark.parametrize("period", [1, 5])
def test_kernel_timers_leave_results_unchanged(slhjb, period):
    """A march with every kernel timer enabled (every launch timed, or one V-cycle and one launch per class
    in five) gives the untimed march bit for bit, and the timers record launches of every class."""
    inst = workloads.config_c2(129, n_cn=4)
    log(f"kernel timers, sampling period {period}")
    res, counts = [], None
    for timed in (False, True):
        solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
        if timed:
            for k in slhjb.KERNEL_NAMES:
                solver.profile_enable(k, 20000)
            solver.profile_sample(period)
        g = to_dev(inst.g)
        U = torch.empty_like(g)
        st = solver.solve(g, to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas, inst.s, U)
        res.append((to_np(U), st.krylov_total, st.pi_total))
        if timed:
            counts = {name: solver.profile_read(k) for k, name in slhjb.KERNEL_NAMES.items()}
        solver.close()
    np.testing.assert_array_equal(res[1][0], res[0][0])
    assert res[1][1:] == res[0][1:]
    kry, pi = res[0][1], res[0][2]
    log(f"  krylov {kry}, pi {pi}, timed launches " + ", ".join(f"{k} {v[0]}" for k, v in counts.items()))
    for name, (n, ms, by, fl) in counts.items():
        assert n > 0 and ms > 0.0 and by > 0.0, name
    # every Arnoldi step runs one apply, one multi-dot and two updates (the first fused with the second
    # pass's sums); sampling keeps one launch in `period`
    assert counts["apply"][0] == -(-kry // period)
    assert counts["multidot"][0] == -(-kry // period)
    assert counts["multiaxpy"][0] == -(-2 * kry // period)
    if period == 1:
        assert counts["mg_residual"][0] == kry


def test_new_volatility_scale_recaptures_graphs(slhjb):
    """A march at one volatility scale and then at another on the same handle gives, at the second scale,
    the result of a fresh handle bit for bit: the captured V-cycle graphs (which hold the deep box and
    the operator application by value) are rebuilt with the tables."""
    inst = workloads.config_c2(65, n_cn=4)
    log("graphs across a change of s")
    g = to_dev(inst.g)
    args = (g, to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas)
    reused = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    U = torch.empty_like(g)
    reused.solve(*args, 1.0, U)
    U_re = torch.empty_like(g)
    st_re = reused.solve(*args, 1.6, U_re)
    reused.close()
    fresh = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    U_fr = torch.empty_like(g)
    st_fr = fresh.solve(*args, 1.6, U_fr)
    fresh.close()
    log(f"  krylov {st_re.krylov_total} / {st_fr.krylov_total}")
    np.testing.assert_array_equal(to_np(U_re), to_np(U_fr))
    assert st_re.krylov_total == st_fr.krylov_total


SKIP_CASES = [
    ("c2_129_cn", lambda: workloads.config_c2(129, n_cn=8)),
    ("c2_257_cn", lambda: workloads.config_c2(257, n_cn=4)),
    ("c5_17_3d", lambda: workloads.config_c5(17, n_steps=4)),
    ("ragged_2d_p2", lambda: _toy((37, 29), K=7, P=2, seed=3, c=True)),
    # 12 tiles of 32 x 8: a work list that is not a multiple of the 8 XCD shares
    ("ragged_52x47_p1", lambda: _toy((52, 47), K=3, P=1, seed=11, c=True)),
    ("ragged_3d_p1", lambda: _toy((11, 9, 13), K=5, P=1, seed=4)),
]


@pytest.mark.parametrize("name,mk", SKIP_CASES, ids=[c[0] for c in SKIP_CASES])
def test_certified_skip_matches_full_search(slhjb, name, mk):
    """Searches that keep certified decisions give the controls of full searches: the whole march, every
    policy and every solver count agree bit for bit with certified_skip off."""
    inst = mk()
    log(f"certified skip {name}")
    res = []
    for skip in (0, 1):
        solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1, certified_skip=skip))
        g = to_dev(inst.g)
        U = torch.empty_like(g)
        pol = torch.empty((len(inst.dts), inst.N), dtype=torch.int16, device=g.device)
        st = solver.solve(g, to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas, inst.s, U, pol)
        res.append((to_np(U), to_np(pol), st.krylov_total, st.pi_total))
        solver.close()
    log(f"  krylov {res[0][2]} / {res[1][2]}, pi {res[0][3]} / {res[1][3]}")
    np.testing.assert_array_equal(res[1][1], res[0][1])
    np.testing.assert_array_equal(res[1][0], res[0][0])
    assert res[1][2:] == res[0][2:]


@pytest.mark.parametrize("width", [16, 64, 128])
def test_tile_widths_sweep_and_march(slhjb, width):
    """Every tile shape gives the bit-exact search and a march within the parity bound."""
    for name, mk in (("c2_65", lambda: workloads.config_c2(65)), ("ragged_3d", lambda: _toy((11, 9, 13), K=5, P=1, seed=4)),
                     ("xscaled_ragged", lambda: _xscaled_toy((31, 23), seed=6))):
        inst = mk()
        log(f"tile width {width}: sweep {name}")
        pb = oracle.Problem(inst)
        X, U = workloads.random_fields(inst, seed=11)
        a_in = workloads.random_policy(inst, seed=12)
        t_prev, dt, theta = 0.1, 0.02, 0.5
        f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
        ref = pb.improve(X, U, theta, f, pb.tau(X, U, f), a_in, want_extra=False)
        solver = slhjb.Solver.from_instance(inst)
        solver.set_tile_width(width)
        da = torch.empty(inst.N, dtype=torch.int16, device="cuda")
        solver.policy_sweep(to_dev(X), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0,
                            to_dev(a_in), da)
        np.testing.assert_array_equal(to_np(da), ref["alpha"])
        solver.close()
    inst = workloads.config_c2(65, n_cn=4)
    ref = oracle.march(inst)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    solver.set_tile_width(width)
    g = to_dev(inst.g)
    U = torch.empty_like(g)
    solver.solve(g, to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas, 1.0, U)
    rel = np.max(np.abs(to_np(U) - ref["U"])) / np.max(np.abs(ref["U"]))
    log(f"  march c2_65 rel {rel:.2e}")
    assert rel <= 1e-10
    solver.close()


def test_autotune_and_cache(slhjb, tmp_path):
    inst = workloads.config_c2(129, n_cn=2)
    cache = tmp_path / "tiles.jsonl"
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    w, costs = solver.autotune(str(cache))
    log(f"autotune 129^2: width {w}, costs {costs}")
    assert w in (16, 32, 64, 128) and costs is not None and min(costs, key=costs.get) == w
    w2, costs2 = solver.autotune(str(cache))   # cache hit
    assert w2 == w and costs2 is None
    assert len(cache.read_text().strip().splitlines()) == 1
    # the tuned handle still solves to the parity bound
    ref = oracle.march(inst)
    g = to_dev(inst.g)
    U = torch.empty_like(g)
    solver.solve(g, to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas, 1.0, U)
    rel = np.max(np.abs(to_np(U) - ref["U"])) / np.max(np.abs(ref["U"]))
    assert rel <= 1e-10
    solver.close()
