"""Aggregation-based algebraic multigrid (the introduction and Sections 3.4-3.5: aggregates along the strongest
couplings of the symmetric part, piecewise-constant prolongation, Galerkin coarse matrices, a Krylov-accelerated
cycle) as the preconditioner of the GPU solves.

What is unique is checked against the oracle: the finest matrix equals the oracle's assembled system matrix,
every coarse matrix equals P^T A P of the oracle's matrix chain under the GPU's aggregates, and solves and
marches meet the oracle's solutions.  The aggregates themselves are one valid outcome of the matching rule
(rounding of equal couplings may pick other partners), so they are checked for validity: sizes 1..4, every
aggregate connected through negative couplings of the finer matrix, dominant rows left out."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
import workloads
from gpu_util import log, to_dev, to_np
from test_gpu_parity import _march_compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DOMINANCE = 5.0  # rows with a_ii >= 5 sum_{j != i} |a_ij| join no aggregate


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _ell(cols, vals, n):
    W, R = cols.shape
    rows = np.repeat(np.arange(R)[None, :], W, axis=0).ravel()
    c, v = cols.ravel(), vals.ravel()
    keep = c >= 0
    return sp.csr_matrix((v[keep], (rows[keep], c[keep])), shape=(R, n))


def _prolongation(agg, nc):
    agg = np.asarray(agg)
    rows = np.nonzero(agg >= 0)[0]
    return sp.csr_matrix((np.ones(rows.size), (rows, agg[rows])), shape=(agg.size, nc))


def _setup_case(inst, seed):
    pb = oracle.Problem(inst)
    alpha = workloads.random_policy(inst, seed)
    U, _ = workloads.random_fields(inst, seed=seed + 1)
    return pb, alpha, U


def _check_hierarchy(solver, A0_full, interior):
    """A0_full: the oracle's system matrix over the full grid (identity-free boundary rows empty)."""
    lv0 = solver.amg_level(0)
    nlev = lv0["levels"]
    N = A0_full.shape[0]
    G0 = _ell(to_np(lv0["cols"]), to_np(lv0["vals"]), N)
    d0 = abs(G0 - A0_full).max()
    log(f"  level 0: {N} rows, width {lv0['width']}, max|diff| {d0:.2e}, levels {nlev}")
    assert d0 <= 1e-13 * abs(A0_full).max()
    A, sizes, widths = A0_full, [N], [lv0["width"]]
    for level in range(1, nlev):
        lv = solver.amg_level(level)
        agg = to_np(lv["agg"]).astype(np.int64)
        nc = lv["rows"]
        assert agg.size == A.shape[0]
        assert agg.min() >= -1 and agg.max() == nc - 1
        members = np.bincount(agg[agg >= 0], minlength=nc)
        assert members.min() >= 1 and members.max() <= 4
        # rows outside every aggregate: the finest grid's boundary and dominant rows
        diag = A.diagonal()
        off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(diag)
        out = np.nonzero(agg < 0)[0]
        if level == 1:
            assert np.all(agg[np.setdiff1d(np.arange(N), interior)] == -1)
            out = np.intersect1d(out, interior)
        ratio_out = diag[out] / np.maximum(off[out], 1e-300)
        assert np.all(ratio_out >= DOMINANCE * (1 - 1e-12))
        inside = np.nonzero(agg >= 0)[0]
        assert np.all(diag[inside] < DOMINANCE * off[inside] * (1 + 1e-12))
        # each aggregate is connected through negative couplings of the finer matrix
        neg = A.copy().tocoo()
        m = (neg.data < 0) & (neg.row != neg.col)
        S = sp.csr_matrix((np.ones(int(m.sum())), (neg.row[m], neg.col[m])), shape=A.shape)
        S = S + S.T
        same = agg[S.tocoo().row] == agg[S.tocoo().col]
        Sc = S.tocoo()
        keep = same & (agg[Sc.row] >= 0)
        Sa = sp.csr_matrix((np.ones(int(keep.sum())), (Sc.row[keep], Sc.col[keep])), shape=A.shape)
        ncomp, lab = connected_components(Sa, directed=False)
        comps_per_agg = np.zeros(nc, np.int64)
        first = {}
        for i in inside:
            key = agg[i]
            if key not in first:
                first[key] = lab[i]
            elif first[key] != lab[i]:
                comps_per_agg[key] += 1
        assert comps_per_agg.max() == 0
        P = _prolongation(agg, nc)
        Ac = (P.T @ A @ P).tocsr()
        G = _ell(to_np(lv["cols"]), to_np(lv["vals"]), nc)
        diff = abs(G - Ac).max()
        log(f"  level {level}: {nc} rows (sizes {np.bincount(members)[1:].tolist()}), width {lv['width']}, "
            f"max|diff| {diff:.2e}")
        assert diff <= 1e-13 * abs(Ac).max()
        assert nc <= A.shape[0]
        A = Ac
        sizes.append(nc)
        widths.append(lv["width"])
    # coarsening ends at a level small enough for the dense inverse, or once it stalls (below 5/4 per level) or
    # the rows grow wide
    assert sizes[-1] <= 120 or sizes[-1] * 5 > sizes[-2] * 4 or widths[-1] > 128
    return sizes


def _full_matrix(pb, alpha, dt, theta):
    L = pb.assemble(alpha)
    Ai = oracle._system_matrix(pb, L, alpha, dt, theta).tocsr()
    I = pb.interior
    N = L.shape[0]
    E = sp.csr_matrix((np.ones(I.size), (I, np.arange(I.size))), shape=(N, I.size))
    return (E @ Ai @ E.T).tocsr(), L


@pytest.mark.parametrize("name,mk", [("c2_65", lambda: workloads.config_c2(65, n_cn=2)),
                                     ("c4_xscaled", lambda: workloads.c4_instance(65, 0.12, 0.29, 0.35, 0.02)),
                                     ("c2_129", lambda: workloads.config_c2(129, n_cn=2))],
                         ids=["c2_65", "c4_xscaled", "c2_129"])
def test_amg_hierarchy_matches_oracle_products(slhjb, name, mk):
    inst = mk()
    log(f"aggregation hierarchy {name}")
    pb, alpha, U = _setup_case(inst, 5)
    t_prev, dt, theta = 0.1, float(inst.dts[-1]), 0.5
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=0, precond=slhjb.PRECOND_AMG))
    X = U.copy()
    X[pb.bd] = inst.psi[pb.bd]
    dX = to_dev(X)
    st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
    log(f"  linsolve krylov={st.krylov_total}")
    A0, _ = _full_matrix(pb, alpha, dt, theta)
    sizes = _check_hierarchy(solver, A0, pb.interior)
    log(f"  level sizes {sizes}")
    solver.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kcycle", [-1, 0, 1])
def test_amg_linsolve_matches_oracle(slhjb, precision, kcycle):
    inst = workloads.config_c2(129)
    pb, alpha, U = _setup_case(inst, 7)
    t_prev, dt, theta = 0.1, 1.0 / 128, 0.5
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    L = pb.assemble(alpha)
    E = oracle.explicit_part(pb, L, alpha, U, f, dt, theta)
    V0 = U.copy()
    V0[pb.bd] = inst.psi[pb.bd]
    Vref, _ = oracle.linear_solve(pb, L, alpha, V0, E, dt, theta, rtol=1e-15)
    counts = {}
    for pc in (slhjb.PRECOND_VCYCLE, slhjb.PRECOND_AMG):
        solver = slhjb.Solver.from_instance(
            inst, slhjb.Options(precision=precision, precond=pc, kcycle_levels=kcycle, max_levels=0))
        dX = to_dev(V0)
        st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
        X = to_np(dX)
        rel = np.max(np.abs(X - Vref)) / np.max(np.abs(Vref))
        counts[pc] = st.krylov_total
        log(f"  precond={pc} precision={precision} kcycle_levels={kcycle}: krylov {st.krylov_total}, rel {rel:.2e}")
        assert rel <= 1e-11
        solver.close()


def test_amg_linsolve_bicgstab(slhjb):
    inst = workloads.config_c2(65)
    pb, alpha, U = _setup_case(inst, 9)
    t_prev, dt, theta = 0.0, 1.0 / 64, 1.0
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    L = pb.assemble(alpha)
    E = oracle.explicit_part(pb, L, alpha, U, f, dt, theta)
    V0 = U.copy()
    V0[pb.bd] = inst.psi[pb.bd]
    Vref, _ = oracle.linear_solve(pb, L, alpha, V0, E, dt, theta, rtol=1e-15)
    solver = slhjb.Solver.from_instance(
        inst, slhjb.Options(precond=slhjb.PRECOND_AMG, krylov=slhjb.KRYLOV_BICGSTAB))
    dX = to_dev(V0)
    st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
    rel = np.max(np.abs(to_np(dX) - Vref)) / np.max(np.abs(Vref))
    log(f"  BiCGSTAB + AMG: krylov {st.krylov_total}, rel {rel:.2e}")
    assert rel <= 1e-11
    solver.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_amg_march_c2(slhjb, precision):
    """65^2 Crank-Nicolson march preconditioned by the aggregation cycle: values, policies, fixed points."""
    inst = workloads.config_c2(65, n_cn=6)
    _march_compare(slhjb, inst, slhjb.Options(precision=precision, precond=slhjb.PRECOND_AMG))


def test_amg_march_c1_scaled_cycle(slhjb):
    """C1 (implicit Euler, no drift) with one GCR iteration below the first coarse level."""
    inst = workloads.config_c1(33)
    _march_compare(slhjb, inst, slhjb.Options(precond=slhjb.PRECOND_AMG, kcycle_levels=1))


def test_amg_option_checks(slhjb):
    inst = workloads.config_c2(33, n_cn=1)
    with pytest.raises(slhjb.HJBError):
        slhjb.Solver.from_instance(inst, slhjb.Options(precond=slhjb.PRECOND_AMG, amg_reuse=2))
    with pytest.raises(slhjb.HJBError):
        slhjb.Solver.from_instance(inst, slhjb.Options(precond=slhjb.PRECOND_AMG, kcycle_levels=-2))
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precond=slhjb.PRECOND_AMG))
    with pytest.raises(slhjb.HJBError):
        solver.amg_level(0)  # nothing built yet
    # the transposed solves of the adjoint are not served by the aggregation cycle
    g, psi, f0, f1 = to_dev(inst.g), to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1)
    U = torch.empty_like(g)
    pol = torch.empty((len(inst.dts), inst.N), dtype=torch.int16, device=g.device)
    solver.solve(g, psi, f0, f1, inst.dts, inst.thetas, inst.s, U, pol)
    with pytest.raises(slhjb.HJBError):
        solver.adjoint(g, psi, f0, f1, inst.dts, inst.thetas, inst.s, pol, torch.ones_like(g), torch.empty_like(g),
                       torch.empty_like(g))
    lv = solver.amg_level(0)
    with pytest.raises(slhjb.HJBError):
        solver.amg_level(lv["levels"])
    solver.close()


@pytest.mark.parametrize("name,mk", [("ragged_37x29_p2", lambda: _toy_amg((37, 29), K=7, P=2, seed=3)),
                                     ("ragged_52x47_p1", lambda: _toy_amg((52, 47), K=3, P=1, seed=11)),
                                     ("tiny_9", lambda: workloads.config_c2(9, n_cn=2))],
                         ids=["ragged_37x29_p2", "ragged_52x47_p1", "tiny_9"])
def test_amg_march_ragged_and_tiny(slhjb, name, mk):
    """Ragged boxes with discounting and two diffusion columns, and a grid of 49 unknowns (no coarse level:
    the preconditioner is the smoother alone)."""
    inst = mk()
    log(f"AMG march {name}")
    _march_compare(slhjb, inst, slhjb.Options(precond=slhjb.PRECOND_AMG))


def _toy_amg(n, K, P, seed):
    from test_gpu_parity import _toy
    return _toy(n, K=K, P=P, seed=seed, c=True)


def test_amg_switch_preconditioners(slhjb):
    """One handle: geometric cycle, aggregation, geometric again (set_options), each solve meeting the oracle."""
    inst = workloads.config_c2(65)
    pb, alpha, U = _setup_case(inst, 11)
    t_prev, dt, theta = 0.0, 1.0 / 64, 0.5
    f = pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)
    L = pb.assemble(alpha)
    E = oracle.explicit_part(pb, L, alpha, U, f, dt, theta)
    V0 = U.copy()
    V0[pb.bd] = inst.psi[pb.bd]
    Vref, _ = oracle.linear_solve(pb, L, alpha, V0, E, dt, theta, rtol=1e-15)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    for pc in (slhjb.PRECOND_VCYCLE, slhjb.PRECOND_AMG, slhjb.PRECOND_VCYCLE, slhjb.PRECOND_AMG):
        solver.set_options(slhjb.Options(precision=1, precond=pc))
        dX = to_dev(V0)
        st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
        rel = np.max(np.abs(to_np(dX) - Vref)) / np.max(np.abs(Vref))
        log(f"  precond={pc}: krylov {st.krylov_total}, rel {rel:.2e}")
        assert rel <= 1e-11
    solver.close()


@pytest.mark.parametrize("name,mk", [("c2_65", lambda: workloads.config_c2(65, n_cn=6)),
                                     ("c1_33", lambda: workloads.config_c1(33))], ids=["c2_65", "c1_33"])
def test_amg_march_reused_hierarchy(slhjb, name, mk):
    """amg_reuse: the hierarchy of a step's first policy preconditions the step's later solves (the finest
    level follows the current policy); the marches still meet the oracle."""
    inst = mk()
    log(f"AMG march with the hierarchy kept within each step: {name}")
    _march_compare(slhjb, inst, slhjb.Options(precond=slhjb.PRECOND_AMG, amg_reuse=1))


def _toy3(n, K, P, seed):
    from test_gpu_parity import _toy
    return _toy(n, K=K, P=P, seed=seed, c=True)


@pytest.mark.parametrize("name,mk", [("c5_17", lambda: workloads.config_c5(17, n_steps=2)),
                                     ("ragged_3d", lambda: _toy3((11, 9, 13), K=5, P=1, seed=4))],
                         ids=["c5_17", "ragged_3d"])
def test_amg_hierarchy_3d(slhjb, name, mk):
    """3D grids: eight interpolation corners per stencil point in the finest rows; every level against the
    oracle's matrix chain, and a march against the oracle."""
    inst = mk()
    log(f"aggregation hierarchy 3D {name}")
    pb, alpha, U = _setup_case(inst, 5)
    t_prev, dt, theta = 0.0, float(inst.dts[-1]), float(inst.thetas[-1])
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precond=slhjb.PRECOND_AMG))
    X = U.copy()
    X[pb.bd] = inst.psi[pb.bd]
    dX = to_dev(X)
    st = solver.linsolve(to_dev(alpha), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), t_prev, dt, theta, 1.0, dX)
    log(f"  linsolve krylov={st.krylov_total}")
    A0, _ = _full_matrix(pb, alpha, dt, theta)
    sizes = _check_hierarchy(solver, A0, pb.interior)
    log(f"  level sizes {sizes}")
    solver.close()
    _march_compare(slhjb, inst, slhjb.Options(precond=slhjb.PRECOND_AMG))
