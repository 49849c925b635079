"""Parity of the discrete adjoint (hjb_adjoint, hjb_apply_transposed) with the oracle.

Policies come from the oracle's own march (or the seeded random generator) and are passed to both
sides.  The transposed operator must satisfy <A^T x, y> = <x, A y> against the GPU's forward apply
and match the oracle's assembled matrix to rounding; the gradients with respect to f0, f1 and g
must match the oracle's sparse direct adjoint to 1e-10 relative, and the gradient with respect to
the diffusion scale s must match a central difference of the oracle's fixed-policy march.

The s-derivative is taken at s = 0.93: at s = 1 on the 33^2 grid the diagonal control directions
move exactly four cells, where the interpolated operator has a kink in s and only one-sided
derivatives exist.
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


def _toy(n, K, P, seed, drift=True, c=False, n_steps=3, thetas=None):
    rng = np.random.default_rng(seed)
    dim = len(n)
    N = int(np.prod(n))
    h = 1.0 / (max(n) - 1)
    sig = rng.normal(size=(K, P, dim))
    b = rng.normal(size=(K, dim)) * 0.4 if drift else None
    cc = -rng.uniform(0.0, 1.0, size=K) if c else None
    dts = np.full(n_steps, 0.05)
    thetas = np.array([1.0] + [0.5] * (n_steps - 1)) if thetas is None else np.asarray(thetas, float)
    inst = workloads.Instance(name=f"toy{n}", dim=dim, n=tuple(n), lo=(0.0,) * dim, h=h, K=K, P=P, sigma=sig,
                              drift=b, c=cc, f0=rng.normal(size=N), f1=rng.normal(size=N), g=rng.normal(size=N),
                              psi=np.zeros(N), dts=dts, thetas=thetas)
    inst.psi = np.where(inst.boundary_mask(), rng.normal(size=N) * 0.3, 0.0)
    return inst


CASES = [
    ("c1_33", lambda: workloads.config_c1(33)),
    ("c2_33_cn", lambda: workloads.config_c2(33, n_cn=8)),
    ("ragged_2d_c", lambda: _toy((37, 29), K=7, P=2, seed=3, c=True)),
    ("ragged_3d", lambda: _toy((11, 9, 13), K=5, P=1, seed=4)),
    ("cn_first_2d", lambda: _toy((23, 19), K=6, P=1, seed=8, c=True, thetas=[0.5, 0.5, 1.0])),
    ("c4_33_xscaled", lambda: workloads.c4_instance(33, 0.15, 0.3, 0.4, 0.03, n_steps=5)),
    ("problem_a_41_field", lambda: workloads.problem_a(41, dt=0.125, theta=1.0)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_apply_transposed(slhjb, name, mk):
    inst = mk()
    log(f"apply_T {name} n={inst.n}")
    pb = oracle.Problem(inst)
    alpha = workloads.random_policy(inst, seed=21)
    rng = np.random.default_rng(22)
    x = rng.normal(size=inst.N)
    y = rng.normal(size=inst.N)
    x[pb.bd] = 0.0
    y[pb.bd] = 0.0
    dt, th = 0.03, 0.5
    solver = slhjb.Solver.from_instance(inst)
    dx, dy, da = to_dev(x), to_dev(y), to_dev(alpha)
    ATx = torch.empty_like(dx)
    Ay = torch.empty_like(dx)
    solver.apply_transposed(da, dx, ATx, dt, th, 1.0)
    solver.apply(da, dy, Ay, dt, th, 1.0)
    ATx, Ay = to_np(ATx), to_np(Ay)
    lhs, rhs = float(ATx @ y), float(x @ Ay)
    log(f"  <A^T x, y> = {lhs:.15e}  <x, A y> = {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(ATx) @ np.abs(y))
    A = oracle._system_matrix(pb, pb.assemble(alpha).tocsr(), alpha, dt, th)
    ref = np.zeros(inst.N)
    ref[pb.interior] = A.T @ x[pb.interior]
    assert np.all(ATx[pb.bd] == 0.0)
    np.testing.assert_allclose(ATx, ref, rtol=0, atol=1e-13 * max(1.0, np.max(np.abs(ref))))
    solver.close()


def _hub(pb, alpha, j, radius):
    """Give every interior row near column j whose stencil (under some control) reaches j such a control, so that
    column j of A collects far more entries than the sliced ELL holds (32 per column); the rest of the column
    comes from the sorted listing."""
    jx, jy = j % pb.n[0], j // pb.n[0]
    hits = 0
    for y in range(max(1, jy - radius), min(pb.n[1] - 1, jy + radius + 1)):
        for x in range(max(1, jx - radius), min(pb.n[0] - 1, jx + radius + 1)):
            i = x + pb.n[0] * y
            for k in range(pb.K):
                cols, vals = pb.row(i, k)
                if np.any((cols == j) & (vals != 0.0)):
                    alpha[i] = k
                    hits += 1
                    break
    return hits


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [513, 2049])
def test_apply_transposed_full_size(slhjb, n):
    """A^T x at the adjoint workload's grid (513^2) and the headline grid (2049^2) against the oracle's assembled
    matrix on every node: the policy is the search's decision at the closed-form solution (piecewise constant, so
    most tiles take the matrix-free reflected gather with one to four controls per window, stencil reach 23 and
    45 cells), with one planted column of a few hundred entries that overflows the ELL width cap."""
    inst = workloads.config_c3(n) if n == 513 else workloads.config_h(n)
    pb = oracle.Problem(inst)
    X0 = inst.coords()
    t_prev, dt, th = 0.25, 1.0 / 64, 0.5
    U = inst.exact(t_prev, X0)
    X = inst.exact(t_prev + dt, X0)
    X[pb.bd] = inst.psi[pb.bd]
    f = pb.f_at(inst.f0, inst.f1, t_prev + th * dt)
    a0 = np.zeros(inst.N, np.int16)
    a0[pb.bd] = -1
    alpha = pb.improve(X, U, th, f, pb.tau(X, U, f), a0, want_extra=False)["alpha"]
    j = (n // 3) + inst.n[0] * (n // 2)
    radius = int(np.ceil(np.max(np.abs(inst.sigma)) / np.sqrt(inst.h))) + 3
    hits = _hub(pb, alpha, j, radius)
    rng = np.random.default_rng(41)
    x = rng.normal(size=inst.N)
    x[pb.bd] = 0.0
    y = rng.normal(size=inst.N)
    y[pb.bd] = 0.0
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    da, dx = to_dev(alpha), to_dev(x)
    ATx = torch.empty_like(dx)
    Ay = torch.empty_like(dx)
    solver.apply_transposed(da, dx, ATx, dt, th, 1.0)
    solver.apply(da, to_dev(y), Ay, dt, th, 1.0)
    ATx, Ay = to_np(ATx), to_np(Ay)
    solver.close()
    A = oracle._system_matrix(pb, pb.assemble(alpha).tocsr(), alpha, dt, th)
    col_len = np.diff(A.tocsc().indptr)
    log(f"apply_T {n}^2: hub column holds {hits} rows; longest column {col_len.max()} entries, "
        f"{int(np.sum(col_len > 32))} columns beyond 32")
    assert col_len.max() > 32
    ref = np.zeros(inst.N)
    ref[pb.interior] = A.T @ x[pb.interior]
    assert np.all(ATx[pb.bd] == 0.0)
    np.testing.assert_allclose(ATx, ref, rtol=0, atol=1e-13 * max(1.0, np.max(np.abs(ref))))
    lhs, rhs = float(ATx @ y), float(x @ Ay)
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(ATx) @ np.abs(y))


S_TEST = 0.93


def _lam_N(inst, UN, seed=31):
    """dJ/dU^N of J = 1/2 |U^N - target|^2 with a seeded target."""
    rng = np.random.default_rng(seed)
    tgt = UN + 0.1 * rng.normal(size=inst.N)
    lam = UN - tgt
    lam[inst.boundary_mask()] = 0.0
    return lam


@pytest.mark.parametrize("precision,precond", [(0, 2), (1, 2), (0, 1)], ids=["fp64-vcycle", "mixed-vcycle", "fp64-jacobi"])
@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_adjoint_matches_oracle(slhjb, name, mk, precision, precond):
    _check_adjoint(slhjb, name, mk(), precision, precond)


def test_adjoint_deep_hierarchy_65(slhjb):
    """The transposed V-cycle over the full hierarchy (65, 33, 17) in both precisions."""
    inst = workloads.config_c2(65, n_cn=4)
    for precision in (0, 1):
        _check_adjoint(slhjb, "c2_65_deep", inst, precision, 2, max_levels=0)


def test_adjoint_uniform_windows_129(slhjb):
    """At 129^2 many tiles lie inside regions of one control, where the mixed mode gathers the transposed
    columns matrix-free (the row stencil reflected); the gradients still match the oracle's."""
    _check_adjoint(slhjb, "c2_129_cn", workloads.config_c2(129, n_cn=4), 1, 2)


@pytest.mark.parametrize("coarse_sweeps_t", [0, 1, 5])
def test_adjoint_coarse_sweeps_option(slhjb, coarse_sweeps_t):
    """The transposed cycles' own coarsest-level sweep count (0: the forward's) changes the work, not the
    gradients: each setting meets the dense oracle adjoint."""
    inst = workloads.config_c2(65, n_cn=4)
    _check_adjoint(slhjb, f"c2_65 coarse_sweeps_t={coarse_sweeps_t}", inst, 1, 2, coarse_sweeps_t=coarse_sweeps_t)


def _check_adjoint(slhjb, name, inst, precision, precond, max_levels=2, coarse_sweeps_t=2, krylov=0):
    log(f"adjoint {name} n={inst.n} steps={len(inst.dts)} precision={precision} precond={precond} krylov={krylov}")
    s = S_TEST
    ref_march = oracle.march(inst, s=s, keep_policies=True)
    pols = ref_march["policies"]
    lam = _lam_N(inst, ref_march["U"])
    ref = oracle.adjoint_dense(inst, pols, lam, s=s)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=precision, precond=precond,
                                                            max_levels=max_levels, coarse_sweeps_t=coarse_sweeps_t,
                                                            krylov=krylov))
    dg = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    df0, df1 = torch.empty_like(dg), torch.empty_like(dg)
    ds, st = solver.adjoint(to_dev(inst.g), to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts,
                            inst.thetas, s, to_dev(pols), to_dev(lam), df0, dg, dJ_df1=df1)
    log(f"  krylov recompute={st.krylov_recompute} adjoint={st.krylov_adjoint} res={st.max_res_adjoint:.2e}")
    for key, got in (("df0", df0), ("df1", df1), ("dg", dg)):
        r = ref[key]
        err = float(np.max(np.abs(to_np(got) - r)))
        log(f"  {key}: max|err| = {err:.2e} (max|ref| {np.max(np.abs(r)):.3e})")
        assert err <= 1e-10 * max(1.0, float(np.max(np.abs(r))))
    ds_ref = oracle.ds_central_difference(inst, pols, lam, s)
    log(f"  ds: {ds:.12e} central difference {ds_ref:.12e}")
    assert abs(ds - ds_ref) <= 1e-6 * max(1.0, abs(ds_ref))
    solver.close()


@pytest.mark.parametrize("store", ["checkpoints", False, True], ids=["checkpoints", "recompute", "stored"])
def test_autograd_march(slhjb, store):
    """HJBMarch: backward of sum(w * U^N) gives the adjoint gradients with lambda_N = w, with the forward
    keeping every ceil(sqrt(n))-th level, no level, or every level."""
    inst = workloads.config_c2(33, n_cn=4)
    log(f"autograd march c2_33, store_values={store}")
    ref_march = oracle.march(inst, keep_policies=True)
    w = _lam_N(inst, ref_march["U"], seed=41)
    ref = oracle.adjoint_dense(inst, ref_march["policies"], w)
    solver = slhjb.Solver.from_instance(inst)
    g = to_dev(inst.g).requires_grad_(True)
    f0 = to_dev(inst.f0).requires_grad_(True)
    f1 = to_dev(inst.f1).requires_grad_(True)
    s = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    U = slhjb.hjb_march(solver, g, to_dev(inst.psi), f0, f1, inst.dts, inst.thetas, s, store_values=store)
    np.testing.assert_allclose(to_np(U.detach()), ref_march["U"], rtol=0, atol=1e-10)
    (U * to_dev(w)).sum().backward()
    for key, t in (("dg", g), ("df0", f0), ("df1", f1)):
        err = float(np.max(np.abs(to_np(t.grad) - ref[key])))
        log(f"  {key}: {err:.2e}")
        assert err <= 1e-10 * max(1.0, float(np.max(np.abs(ref[key]))))
    assert torch.isfinite(s.grad)
    solver.close()


def test_adjoint_rejects_explicit_steps(slhjb):
    inst = workloads.config_c1(17)
    inst.thetas = np.zeros_like(inst.thetas)
    solver = slhjb.Solver.from_instance(inst)
    pols = torch.zeros((len(inst.dts), inst.N), dtype=torch.int16, device="cuda")
    out = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    with pytest.raises(slhjb.HJBError):
        solver.adjoint(to_dev(inst.g), to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas,
                       1.0, pols, out, torch.empty_like(out), torch.empty_like(out))
    solver.close()


def test_adjoint_with_stored_values(slhjb):
    """Passing hjb_solve's stored values gives the same gradients as recomputing them."""
    inst = workloads.config_c2(65, n_cn=6)
    log("adjoint with stored values c2_65")
    solver = slhjb.Solver.from_instance(inst)
    g, psi, f0, f1 = to_dev(inst.g), to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1)
    U = torch.empty_like(g)
    pol = torch.empty((len(inst.dts), inst.N), dtype=torch.int16, device="cuda")
    vals = torch.empty((len(inst.dts) + 1, inst.N), dtype=torch.float64, device="cuda")
    solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, 1.0, U, pol, vals)
    np.testing.assert_array_equal(to_np(vals[-1]), to_np(U))
    np.testing.assert_array_equal(to_np(vals[0]), inst.g)
    lam = torch.from_numpy(_lam_N(inst, to_np(U))).cuda()
    outs = []
    for v in (None, vals):
        dg, df0, df1 = torch.empty_like(g), torch.empty_like(g), torch.empty_like(g)
        ds, st = solver.adjoint(g, psi, f0, f1, inst.dts, inst.thetas, 1.0, pol, lam, df0, dg, dJ_df1=df1, values=v)
        log(f"  values={'stored' if v is not None else 'recomputed'}: recompute its {st.krylov_recompute}, "
            f"adjoint its {st.krylov_adjoint}, ds {ds:.12e}")
        outs.append((to_np(dg), to_np(df0), to_np(df1), ds))
    assert outs[1][0] is not None
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert np.max(np.abs(a - b)) <= 1e-10 * max(1.0, np.max(np.abs(a)))
    assert abs(outs[0][3] - outs[1][3]) <= 1e-9 * max(1.0, abs(outs[0][3]))
    solver.close()


@pytest.mark.parametrize("n_cn", [1, 8, 14])
def test_adjoint_checkpointed_recompute(slhjb, n_cn):
    """Without stored values the adjoint recomputes them from the int16 policies, keeping every
    ceil(sqrt(n_steps))-th value (3, 10 and 16 steps: segments of 2+1, 4+4+2 and 4x4 steps): the
    gradients equal those with the forward's stored values, the recomputation costs about two fixed-policy
    solves per step, and without dJ/ds nothing is recomputed.  With the forward's every k-th level as
    checkpoints (value_stride) only the segments are recomputed, to the same gradients."""
    inst = workloads.config_c2(65, n_cn=n_cn)
    n = len(inst.dts)
    log(f"checkpointed recompute c2_65, {n} steps")
    solver = slhjb.Solver.from_instance(inst)
    g, psi, f0, f1 = to_dev(inst.g), to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1)
    U = torch.empty_like(g)
    pol = torch.empty((n, inst.N), dtype=torch.int16, device="cuda")
    vals = torch.empty((n + 1, inst.N), dtype=torch.float64, device="cuda")
    fst = solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, 1.0, U, pol, vals)
    lam = torch.from_numpy(_lam_N(inst, to_np(U))).cuda()
    res = {}
    for name, v, want in (("stored", vals, True), ("recomputed", None, True), ("no ds", None, False)):
        dg, df0, df1 = torch.empty_like(g), torch.empty_like(g), torch.empty_like(g)
        ds, st = solver.adjoint(g, psi, f0, f1, inst.dts, inst.thetas, 1.0, pol, lam, df0, dg, dJ_df1=df1,
                                values=v, want_ds=want)
        log(f"  {name}: recompute its {st.krylov_recompute}, adjoint its {st.krylov_adjoint}, ds {ds}")
        res[name] = (to_np(dg), to_np(df0), to_np(df1), ds, st)
    # checkpoints from the forward march (every k-th level, value_stride = k): only the segments are recomputed
    k = max(1, int(np.ceil(np.sqrt(n))))
    solver.set_options(slhjb.Options(value_stride=k))
    ck = torch.empty((n // k + 1, inst.N), dtype=torch.float64, device="cuda")
    U2 = torch.empty_like(g)
    solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, 1.0, U2, pol, ck)
    assert torch.equal(U2, U)
    assert torch.equal(ck, vals[::k][: n // k + 1])
    dg, df0, df1 = torch.empty_like(g), torch.empty_like(g), torch.empty_like(g)
    ds, st = solver.adjoint(g, psi, f0, f1, inst.dts, inst.thetas, 1.0, pol, lam, df0, dg, dJ_df1=df1, values=ck)
    log(f"  forward checkpoints (stride {k}): recompute its {st.krylov_recompute}, adjoint its "
        f"{st.krylov_adjoint}, ds {ds}")
    res["checkpoints"] = (to_np(dg), to_np(df0), to_np(df1), ds, st)
    assert res["stored"][4].krylov_recompute == 0 and res["no ds"][4].krylov_recompute == 0
    assert res["recomputed"][4].krylov_recompute > 0
    assert 0 < res["checkpoints"][4].krylov_recompute <= res["recomputed"][4].krylov_recompute
    for name in ("recomputed", "no ds", "checkpoints"):
        for a, b in zip(res[name][:3], res["stored"][:3]):
            assert np.max(np.abs(a - b)) <= 1e-10 * max(1.0, np.max(np.abs(b)))
    for name in ("recomputed", "checkpoints"):
        assert abs(res[name][3] - res["stored"][3]) <= 1e-9 * max(1.0, abs(res["stored"][3]))
    solver.close()
