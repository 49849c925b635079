"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test ties a part of the oracle to something other than the oracle itself:
the consistency conditions the truncation weights were derived from
(eqs. AB_drift, AB1, AB2), the properties of multilinear interpolation
(eq. monotone_int_2), the row-sum identity after eq. Lhat, the row and
column sums of Section 3.4, the characterisation of the discrete HJB solution
as the minimum over all policies, the discrete maximum principle, and the
error tables the paper prints for Problems A and B (Section 2.4).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _toy(n=(9, 8), K=5, P=1, seed=0, drift=True, c=False, dim=2, scale=1.0):
    """Small random constant-coefficient instance (sigma, b, c per control)."""
    rng = np.random.default_rng(seed)
    n = tuple(n[:dim])
    h = 1.0 / 8.0
    N = int(np.prod(n))
    sig = rng.normal(size=(K, P, dim)) * scale
    b = rng.normal(size=(K, dim)) * 0.7 if drift else None
    cc = -rng.uniform(0.0, 2.0, size=K) if c else None
    inst = workloads.Instance(name="toy", dim=dim, n=n, lo=(0.0,) * dim, h=h, K=K, P=P, sigma=sig, drift=b, c=cc,
                              f0=rng.normal(size=N), f1=rng.normal(size=N), g=rng.normal(size=N),
                              psi=np.zeros(N), dts=np.array([0.05]), thetas=np.array([1.0]))
    inst.psi = np.where(inst.boundary_mask(), rng.normal(size=N), 0.0)
    return inst


# ---------------------------------------------------------------------------
# Truncation weights: consistency conditions of Prop. pro:scheme2 and Cor. cor:Growth
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_weights_satisfy_consistency_conditions(dim):
    inst = _toy(n=(9, 8, 7), K=6, P=2, seed=1, dim=dim, scale=0.6)
    pb = oracle.Problem(inst)
    n_trunc = 0
    for i in pb.interior:
        for k in range(inst.K):
            w = pb.weights(int(i), k)
            A, B, mp, mm = w["A"], w["B"], w["mu_plus"], w["mu_minus"]
            # eq. AB1: A*mu+ y - B*mu- y = 0 ; eq. AB2: A*mu+^2 + B*mu-^2 = 2 (in units of y_a y_b = dx s^2 sigma_a sigma_b)
            np.testing.assert_allclose(A * mp, B * mm, rtol=1e-14)
            np.testing.assert_allclose(A * mp * mp + B * mm * mm, 2.0, rtol=1e-14)
            # Cor. cor:Growth a): A, B >= 1, and A = B = 1 without overstepping (Section 2.1)
            assert np.all(A >= 1.0 - 1e-15) and np.all(B >= 1.0 - 1e-15)
            untr = (mp == 1.0) & (mm == 1.0)
            assert np.all(A[untr] == 1.0) and np.all(B[untr] == 1.0)
            assert np.all((mp > 0) & (mp <= 1) & (mm > 0) & (mm <= 1))
            n_trunc += int(np.sum(~untr))
            # eq. AB_drift: (A+B) mu_b b = 2 b with A = B = C
            assert abs(2.0 * w["C"] * w["mu_b"] - 2.0) < 1e-14
    assert n_trunc > 0


def test_truncated_point_lies_on_boundary():
    """The truncated point x + mu*y is on the boundary and mu is the largest feasible (Prop. pro:scheme2)."""
    inst = _toy(n=(11, 11), K=1, P=1)
    pb = oracle.Problem(inst)
    rng = np.random.default_rng(3)
    for _ in range(300):
        i = int(rng.choice(pb.interior))
        Y = rng.normal(size=2) * 6.0
        cell, t, mu = pb.landing(i, Y)
        ix = np.array([i % 11, i // 11])
        q = cell + t
        exact_mu = min([1.0] + [((10 - ix[d]) if Y[d] > 0 else ix[d]) / abs(Y[d]) for d in range(2) if Y[d] != 0])
        assert mu == pytest.approx(exact_mu, rel=1e-15)
        np.testing.assert_allclose(q, ix + mu * Y, atol=1e-12)
        assert np.all(q >= 0) and np.all(q <= 10)
        if mu < 1:
            assert np.any(np.isclose(q, 0.0, atol=1e-12) | np.isclose(q, 10.0, atol=1e-12))


# ---------------------------------------------------------------------------
# Interpolation and the operator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_interpolation_weights_nonnegative_and_sum_to_one(dim):
    """eq. monotone_int_2: w >= 0, sum w = 1; row sums of l-hat as after eq. Lhat."""
    inst = _toy(n=(9, 8, 7), K=4, P=1, seed=2, dim=dim)
    pb = oracle.Problem(inst)
    inv2h = 0.5 / inst.h
    for i in pb.interior[::3]:
        for k in range(inst.K):
            cols, vals = pb.row(int(i), k)
            diag_part = vals[-1]
            assert cols[-1] == i
            off = vals[:-1]
            assert np.all(off >= 0.0)
            # the whole row sums to zero (each point's weights sum to one)
            assert abs(np.sum(vals)) < 1e-12 * inv2h
            w = pb.weights(int(i), k)
            total = np.sum(w["A"] + w["B"]) * inv2h + 2.0 * w["C"] * inv2h
            assert np.sum(off) == pytest.approx(total, rel=1e-13)
            # row-sum identity: sum_i l-hat >= M/dx, with equality iff no overstepping
            M = inst.P + 1
            untr = np.all(w["mu_plus"] == 1) and np.all(w["mu_minus"] == 1) and w["mu_b"] == 1
            assert total >= M / inst.h * (1 - 1e-14)
            if untr:
                assert total == pytest.approx(M / inst.h, rel=1e-14)
            else:
                assert total > M / inst.h


@pytest.mark.parametrize("dim", [2, 3])
def test_operator_exact_on_affine_and_bilinear(dim):
    """Consistency conditions + exact multilinear interpolation give closed forms at every interior node,
    truncated or not: L-hat x_a = b_a ; L-hat x_a x_b = s^2 sum_p sig_pa sig_pb + b.D(x_a x_b) + mu_b h b_a b_b."""
    inst = _toy(n=(13, 11, 9), K=4, P=2, seed=5, dim=dim, scale=0.8)
    inst.s = 1.1
    pb = oracle.Problem(inst)
    X = inst.coords()
    I = pb.interior
    for k in range(inst.K):
        alpha = np.full(pb.N, k, np.int16)
        L = pb.assemble(alpha)
        mub = np.array([pb.weights(int(i), k)["mu_b"] for i in I])
        for a in range(dim):
            phi = X[a]
            for val in (pb.lhat(phi, k0=k), L @ phi):
                np.testing.assert_allclose(val[I], inst.drift[k, a], rtol=1e-9, atol=1e-9)
            for b in range(a + 1, dim):
                phi = X[a] * X[b]
                expect = (inst.s ** 2 * np.sum(inst.sigma[k, :, a] * inst.sigma[k, :, b])
                          + inst.drift[k, a] * X[b][I] + inst.drift[k, b] * X[a][I]
                          + mub * inst.h * inst.drift[k, a] * inst.drift[k, b])
                for val in (pb.lhat(phi, k0=k), L @ phi):
                    np.testing.assert_allclose(val[I], expect, rtol=1e-9, atol=1e-9)


def test_xscaled_operator_exact_on_affine_and_bilinear():
    """x-dependent coefficients sigma_k(x) = diag(x) S_k, b_k(x) = diag(x) beta_k: the same closed forms hold
    node by node with the node's own sigma and b (consistency is pointwise)."""
    inst = workloads.c4_instance(17, 0.15, 0.3, 0.4, 0.03)
    inst.drift = inst.drift * 40.0   # drift of several cells, so that its truncation is exercised too
    inst.s = 1.1
    pb = oracle.Problem(inst)
    X = inst.coords()
    I = pb.interior
    for k in range(inst.K):
        alpha = np.full(pb.N, k, np.int16)
        L = pb.assemble(alpha)
        mub = np.array([pb.weights(int(i), k)["mu_b"] for i in I])
        sig = [[X[a][I] * inst.sigma[k, p, a] for a in range(2)] for p in range(inst.P)]
        b = [X[a][I] * inst.drift[k, a] for a in range(2)]
        for a in range(2):
            for val in (pb.lhat(X[a], k0=k), L @ X[a]):
                np.testing.assert_allclose(val[I], b[a], rtol=1e-9, atol=1e-9)
        phi = X[0] * X[1]
        expect = (inst.s ** 2 * sum(sig[p][0] * sig[p][1] for p in range(inst.P))
                  + b[0] * X[1][I] + b[1] * X[0][I] + mub * inst.h * b[0] * b[1])
        for val in (pb.lhat(phi, k0=k), L @ phi):
            np.testing.assert_allclose(val[I], expect, rtol=1e-9, atol=1e-9)
    assert np.any(mub < 1.0)


def test_c4_batch_draws():
    """Batch recipe: sizes from the stated set, parameter ranges, control encoding and payoff data."""
    b = workloads.config_c4(count=16)
    assert len(b) == 16 and {i.n[0] for i in b} <= {65, 129, 257, 513}
    for inst in b:
        m = inst.meta
        assert 0.1 <= m["sig_min"] <= 0.2 and 0.1 <= m["sig_max"] - m["sig_min"] <= 0.2
        assert 0.3 <= m["rho_bar"] <= 0.5 and 0.0 <= m["r"] <= 0.05
        S = inst.sigma
        for k in range(8):
            a = 0.5 * S[k].T @ S[k]          # a = 1/2 sum_p S_p S_p^T (at x = 1)
            s1 = m["sig_max"] if k & 1 else m["sig_min"]
            s2 = m["sig_max"] if k & 2 else m["sig_min"]
            rho = m["rho_bar"] if k & 4 else -m["rho_bar"]
            np.testing.assert_allclose(a, 0.5 * np.array([[s1 * s1, rho * s1 * s2], [rho * s1 * s2, s2 * s2]]),
                                       rtol=1e-14, atol=1e-16)
        X = inst.coords()
        np.testing.assert_array_equal(inst.g, np.maximum(X[0] - X[1], 0.0))


def test_operator_exact_on_squares_for_integer_axis_steps():
    """With axis-aligned integer steps every landing point is a node, so x_a^2 is reproduced:
    L-hat x_a^2 = s^2 sigma_a^2 exactly, also in truncated rows (eq. AB2)."""
    n = (17, 17)
    h = 1.0 / 16
    sig = np.array([[[3.0 * math.sqrt(h), 0.0]], [[0.0, 5.0 * math.sqrt(h)]]])   # 3 and 5 cells
    inst = workloads.Instance(name="axis", dim=2, n=n, lo=(0.0, 0.0), h=h, K=2, P=1, sigma=sig, drift=None,
                              c=None, f0=np.zeros(289), f1=np.zeros(289), g=np.zeros(289), psi=np.zeros(289),
                              dts=np.array([0.1]), thetas=np.array([1.0]))
    pb = oracle.Problem(inst)
    X = inst.coords()
    for k, a in ((0, 0), (1, 1)):
        val = pb.lhat(X[a] ** 2, k0=k)
        np.testing.assert_allclose(val[pb.interior], sig[k, 0, a] ** 2, rtol=1e-12)


def test_evaluator_matches_listing():
    inst = _toy(n=(12, 10), K=5, P=2, seed=7, c=True)
    pb = oracle.Problem(inst)
    rng = np.random.default_rng(0)
    V = rng.normal(size=pb.N)
    alpha = workloads.random_policy(inst, 1)
    L = pb.assemble(alpha)
    np.testing.assert_allclose(pb.lhat(V, alpha), L @ V, rtol=1e-13, atol=1e-12)


# ---------------------------------------------------------------------------
# Matrix properties (Section 1 and Section 3.4)
# ---------------------------------------------------------------------------

def test_system_matrix_is_m_matrix_with_row_sums():
    """A^alpha = I - theta dt (L + c): positive diagonal, non-positive off-diagonal,
    full row sums 1 - theta dt c (Section 3.4, row sums)."""
    inst = _toy(n=(12, 11), K=5, P=1, seed=8, c=True)
    pb = oracle.Problem(inst)
    alpha = workloads.random_policy(inst, 2)
    L = pb.assemble(alpha).tocsr()
    dt, theta = 0.07, 1.0
    A = (-(theta * dt) * L).tolil()
    c = pb.c_of(alpha)
    for i in pb.interior:
        A[i, i] = A[i, i] + 1.0 - theta * dt * c[i]
    A = A.tocsr()
    I = pb.interior
    D = A.diagonal()
    assert np.all(D[I] > 0)
    off = A - __import__("scipy.sparse", fromlist=["diags"]).diags(D)
    assert off[I].max() <= 1e-15
    rs = np.asarray(A[I].sum(axis=1)).ravel()
    np.testing.assert_allclose(rs, 1.0 - theta * dt * c[I], rtol=1e-12)


def test_column_sums_nonnegative_under_bound():
    """Prop. prop-columns: column sums of A are >= 0 for dt <= dx / (max c+ + (3^d - 1)(P+1))."""
    inst = workloads.config_c2(n=33)
    pb = oracle.Problem(inst)
    dt = inst.h / (0.0 + (3 ** 2 - 1) * (inst.P + 1))
    for seed in range(3):
        alpha = workloads.random_policy(inst, seed)
        L = pb.assemble(alpha)
        I = pb.interior
        A = __import__("scipy.sparse", fromlist=["identity"]).identity(I.size) - dt * L[I][:, I]
        cs = np.asarray(A.sum(axis=0)).ravel()
        assert cs.min() >= -1e-12


# ---------------------------------------------------------------------------
# Policy search and policy iteration
# ---------------------------------------------------------------------------

def test_tie_rule_smallest_index_and_hysteresis():
    inst = _toy(n=(8, 8), K=3, P=1, seed=9, drift=False)
    inst.sigma[2] = inst.sigma[0]          # controls 0 and 2 identical -> exact ties
    pb = oracle.Problem(inst)
    rng = np.random.default_rng(1)
    X = rng.normal(size=pb.N)
    f = np.zeros(pb.N)
    tau = pb.tau(X, X, f)
    r = pb.improve(X, X, 1.0, f, tau)
    for i in pb.interior:
        G = pb.node_values(int(i), X, X, 1.0, f)
        assert G[0] == G[2]
        thr = G.min() + tau
        assert r["alpha"][i] == int(np.argmax(G <= thr))
        assert r["alpha"][i] != 2
        assert r["gmin"][i] == G.min()
    keep = np.full(pb.N, 2, np.int16)
    r2 = pb.improve(X, X, 1.0, f, tau, keep)
    for i in pb.interior:
        G = pb.node_values(int(i), X, X, 1.0, f)
        expect = 2 if G[2] <= G.min() + tau else int(np.argmax(G <= G.min() + tau))
        assert r2["alpha"][i] == expect


@pytest.mark.parametrize("theta,cfg", [(1.0, dict(n=(5, 5), K=3, seed=11)), (0.5, dict(n=(5, 5), K=3, seed=12)),
                                       (1.0, dict(n=(6, 6), K=2, seed=13, c=True)),
                                       (0.5, dict(n=(6, 6), K=2, seed=14, c=True)),
                                       (0.3, dict(n=(5, 5), K=3, seed=15, c=True))])
def test_policy_iteration_equals_brute_force(theta, cfg):
    """The discrete solution is the componentwise minimum of (A^alpha)^{-1} F^alpha over all policies
    (M-matrix systems, eq. nonlinear_sys); policy iteration must reach it exactly."""
    inst = _toy(P=1, drift=True, **cfg)
    pb = oracle.Problem(inst)
    dt = 0.3
    alpha0 = np.zeros(pb.N, np.int16)
    alpha0[pb.bd] = -1
    V, alpha, st = oracle.step(pb, inst.g, inst.psi, inst.f0, inst.f1, 0.2, dt, theta, alpha0)
    Vb = oracle.brute_force_step(pb, inst.g, inst.psi, inst.f0, inst.f1, 0.2, dt, theta)
    np.testing.assert_allclose(V, Vb, rtol=1e-11, atol=1e-11)
    assert st.pi_iters >= 1


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.25])
def test_explicit_part_on_constants(theta):
    """Rows of L-hat sum to zero (interpolation reproduces constants and the weights A, B, C enter as
    A v+ + B v- - (A+B) v_i), so for U = 1 on every node the known part of eq. FullScheme is
    1 + (1-theta) dt c + dt f, which fixes the discount term of the explicit part in closed form."""
    inst = _toy(n=(9, 8), K=4, P=1, seed=21, drift=True, c=True)
    pb = oracle.Problem(inst)
    rng = np.random.default_rng(22)
    alpha = rng.integers(0, inst.K, size=pb.N).astype(np.int16)
    alpha[pb.bd] = -1
    dt = 0.07
    f = inst.f0 + 0.3 * inst.f1
    E = oracle.explicit_part(pb, pb.assemble(alpha), alpha, np.ones(pb.N), f, dt, theta)
    I = pb.interior
    expect = 1.0 + (1.0 - theta) * dt * inst.c[alpha[I]] + dt * f[I]
    np.testing.assert_allclose(E[I], expect, rtol=0, atol=1e-13)


def test_policy_iteration_equals_brute_force_xscaled():
    """Same characterisation for the x-scaled two-asset model (8 controls, 4 interior nodes), with a
    random g so that the step is not trivial."""
    inst = workloads.c4_instance(4, 0.15, 0.35, 0.45, 0.04)
    inst.g = np.random.default_rng(21).normal(size=inst.N)
    pb = oracle.Problem(inst)
    alpha0 = np.zeros(pb.N, np.int16)
    alpha0[pb.bd] = -1
    V, alpha, st = oracle.step(pb, inst.g, inst.psi, inst.f0, inst.f1, 0.0, 0.25, 1.0, alpha0)
    Vb = oracle.brute_force_step(pb, inst.g, inst.psi, inst.f0, inst.f1, 0.0, 0.25, 1.0)
    np.testing.assert_allclose(V, Vb, rtol=1e-11, atol=1e-11)


def test_policy_iteration_is_monotone_and_terminates():
    inst = workloads.config_c2(n=33)
    pb = oracle.Problem(inst)
    U = inst.g.copy()
    f = pb.f_at(inst.f0, inst.f1, 1.0 / 128)
    V = U.copy()
    V[pb.bd] = inst.psi[pb.bd]
    alpha = pb.improve(V, U, 1.0, f, pb.tau(V, U, f), None)["alpha"]
    prev = None
    for it in range(30):
        L = pb.assemble(alpha)
        E = oracle.explicit_part(pb, L, alpha, U, f, 1.0 / 128, 1.0)
        V, _ = oracle.linear_solve(pb, L, alpha, V, E, 1.0 / 128, 1.0)
        if prev is not None:
            assert np.all(V <= prev + 1e-12)
        prev = V.copy()
        r = pb.improve(V, U, 1.0, f, pb.tau(V, U, f), alpha)
        if r["changed"] == 0:
            break
        alpha = r["alpha"]
    else:
        pytest.fail("policy iteration did not terminate")


def test_discrete_maximum_principle_and_comparison():
    """theta = 1, f = 0, c = 0: min(U^{n-1}, psi) <= U^n <= max(U^{n-1}, psi); g1 <= g2 => U1 <= U2."""
    inst = workloads.config_c2(n=33)
    inst.f0 = np.zeros(inst.N)
    inst.f1 = np.zeros(inst.N)
    rng = np.random.default_rng(4)
    inst.g = rng.normal(size=inst.N)
    inst.psi = np.where(inst.boundary_mask(), rng.normal(size=inst.N), 0.0)
    inst.dts, inst.thetas = np.full(3, 0.02), np.ones(3)
    out = oracle.march(inst, keep_values=True)
    bd = inst.boundary_mask()
    for a, b in zip(out["values"][:-1], out["values"][1:]):
        lo = min(a.min(), inst.psi[bd].min())
        hi = max(a.max(), inst.psi[bd].max())
        assert b.min() >= lo - 1e-12 and b.max() <= hi + 1e-12
    inst2 = workloads.config_c2(n=33)
    inst2.f0, inst2.f1, inst2.psi, inst2.dts, inst2.thetas = inst.f0, inst.f1, inst.psi, inst.dts, inst.thetas
    inst2.g = inst.g + np.abs(rng.normal(size=inst.N))
    out2 = oracle.march(inst2)
    assert np.all(out2["U"] >= out["U"] - 1e-12)


# ---------------------------------------------------------------------------
# The paper's printed error tables (Section 2.4 and the appendix)
# ---------------------------------------------------------------------------

def _err(inst):
    out = oracle.march(inst)
    return float(np.max(np.abs(out["U"] - inst.exact(inst.T, inst.coords()))))


@pytest.mark.parametrize("Nx", [41, 81, 161])
def test_problem_a_implicit_truncation_table(Nx):
    ref = GOLDEN["implicit_truncation_A"]["dt=T"][str(Nx)]
    assert _err(workloads.problem_a(Nx)) == pytest.approx(ref, rel=5e-3)


@pytest.mark.parametrize("Nx,rel", [(41, 5e-3), (81, 2e-2)])
def test_problem_b_implicit_truncation_table(Nx, rel):
    ref = GOLDEN["implicit_truncation_B"]["dt=T"][str(Nx)]
    assert _err(workloads.problem_b(Nx)) == pytest.approx(ref, rel=rel)


@pytest.mark.parametrize("prob,col,Nx", [("A", "dt=T", 41), ("A", "dt=T", 81), ("A", "dt=dx/4", 41),
                                         ("A", "dt=dx/4", 81), ("A", "dt=dx^2", 41), ("A", "dt=dx^2", 81),
                                         ("B", "dt=T", 41), ("B", "dt=T", 81), ("B", "dt=dx/4", 41),
                                         ("B", "dt=dx/4", 81), ("B", "dt=dx^1.5", 41), ("B", "dt=dx^1.5", 81),
                                         ("B", "dt=dx^2", 41), ("B", "dt=dx^2", 81)])
def test_explicit_truncation_tables(prob, col, Nx):
    ref = GOLDEN[f"explicit_truncation_{prob}"][col][str(Nx)]
    h = 2 * math.pi / (Nx - 1)
    dt = {"dt=T": 0.5, "dt=dx/4": h / 4, "dt=dx^1.5": h ** 1.5, "dt=dx^2": h * h}[col]
    mk = workloads.problem_a if prob == "A" else workloads.problem_b
    assert _err(mk(Nx, dt=dt, theta=0.0)) == pytest.approx(ref, rel=6e-3)


@pytest.mark.slow
def test_explicit_cfl_blowup_with_truncation():
    """Cor. cor:CFL: with truncation the explicit scheme needs dt ~ dx^{3/2}; dt = dx/4 blows up at N_x = 321
    (Table Tab:Linf_matrix_40 prints 1.34e+23) while it is stable at 81."""
    h = 2 * math.pi / 320
    e = _err(workloads.problem_a(321, dt=h / 4, theta=0.0))
    assert e > 1e10


def test_observed_order_one_under_refinement():
    """Manufactured C1 family with the discrete-control source: the error decreases at about first order."""
    errs = []
    for n in (17, 33, 65):
        inst = workloads.config_c1(n=n, source="discrete")
        errs.append(_err(inst))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(0.6 < r < 1.6 for r in rates), (errs, rates)


# ---------------------------------------------------------------------------
# Adjoint oracle (fixed-policy discrete adjoint of the theta-march, eq. FullScheme)
# ---------------------------------------------------------------------------

def _adjoint_toy(seed=7, n=(11, 9), c=True):
    rng = np.random.default_rng(seed)
    dim = len(n)
    N = int(np.prod(n))
    K, P = 4, 2
    inst = workloads.Instance(name="adj_toy", dim=dim, n=tuple(n), lo=(0.0,) * dim, h=1.0 / (max(n) - 1), K=K, P=P,
                              sigma=rng.normal(size=(K, P, dim)), drift=rng.normal(size=(K, dim)) * 0.4,
                              c=(-rng.uniform(0.0, 1.0, size=K) if c else None), f0=rng.normal(size=N),
                              f1=rng.normal(size=N), g=rng.normal(size=N), psi=np.zeros(N),
                              dts=np.array([0.04, 0.05, 0.05]), thetas=np.array([1.0, 0.5, 0.5]))
    inst.psi = np.where(inst.boundary_mask(), rng.normal(size=N) * 0.3, 0.0)
    pols = np.stack([workloads.random_policy(inst, seed + 1 + k) for k in range(len(inst.dts))])
    lam = rng.normal(size=N)
    lam[inst.boundary_mask()] = 0.0
    return inst, pols, lam


def test_fixed_policy_march_reproduces_march():
    inst = workloads.config_c2(17, n_cn=3)
    r = oracle.march(inst, keep_policies=True, keep_values=True)
    vals = oracle.fixed_policy_march(inst, r["policies"])
    for a, b in zip(vals, r["values"]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [(11, 9), (7, 6, 5)])
def test_adjoint_equals_directional_derivatives(n):
    """At fixed policies U^N is affine in (g, f0, f1), so lam . U^N(x + e) - lam . U^N(x) equals the adjoint's
    gradient dotted with e for any e, up to the solves' rounding."""
    inst, pols, lam = _adjoint_toy(n=n)
    ref = oracle.adjoint_dense(inst, pols, lam)
    J0 = float(lam @ oracle.fixed_policy_march(inst, pols)[-1])
    rng = np.random.default_rng(3)
    for field, key in (("g", "dg"), ("f0", "df0"), ("f1", "df1")):
        e = rng.normal(size=inst.N)
        pert = workloads.Instance(**{**inst.__dict__})
        setattr(pert, field, getattr(inst, field) + e)
        J1 = float(lam @ oracle.fixed_policy_march(pert, pols)[-1])
        pred = float(ref[key] @ e)
        assert abs((J1 - J0) - pred) <= 1e-10 * max(1.0, abs(pred)), (field, J1 - J0, pred)
    # boundary entries of the f-gradients vanish (f enters interior rows only); the first step is
    # implicit (theta = 1), whose explicit part is U^0 at the node itself, so dg vanishes there too
    bd = inst.boundary_mask()
    assert np.all(ref["df0"][bd] == 0.0) and np.all(ref["df1"][bd] == 0.0)
    assert inst.thetas[0] == 1.0 and np.all(ref["dg"][bd] == 0.0)


def test_adjoint_boundary_gradient_for_crank_nicolson_start():
    """With theta < 1 in the first step the explicit part reads U^0 on boundary nodes: dg there is the
    directional derivative along boundary perturbations."""
    inst, pols, lam = _adjoint_toy(seed=5)
    inst.thetas = np.array([0.5, 0.5, 1.0])
    ref = oracle.adjoint_dense(inst, pols, lam)
    bd = inst.boundary_mask()
    assert np.any(ref["dg"][bd] != 0.0)
    e = np.where(bd, np.random.default_rng(9).normal(size=inst.N), 0.0)
    J0 = float(lam @ oracle.fixed_policy_march(inst, pols)[-1])
    pert = workloads.Instance(**{**inst.__dict__})
    pert.g = inst.g + e
    J1 = float(lam @ oracle.fixed_policy_march(pert, pols)[-1])
    assert abs((J1 - J0) - float(ref["dg"] @ e)) <= 1e-10 * max(1.0, abs(J1 - J0))


def test_s_central_difference_is_converged():
    inst, pols, lam = _adjoint_toy(seed=11)
    a = oracle.ds_central_difference(inst, pols, lam, 0.93, eps=1e-5)
    b = oracle.ds_central_difference(inst, pols, lam, 0.93, eps=5e-6)
    assert abs(a - b) <= 1e-7 * max(1.0, abs(a))


# ---------------------------------------------------------------------------
# Shifted domain with time-dependent Dirichlet data (Remark rem:two-over, Table Tab:shifted)
# ---------------------------------------------------------------------------

SHIFTED = GOLDEN["explicit_truncation_A_shifted"]


def _shifted_errors(Nx, col):
    h = 2 * math.pi / (Nx - 1)
    dt = {"dt=T": 0.5, "dt=dx/4": h / 4, "dt=dx^1.5": h ** 1.5, "dt=dx^2": h * h}[col]
    inst = workloads.problem_a(Nx, dt=dt, theta=0.0, lo_shift=7 * math.pi / 8)
    out = oracle.march(inst)
    X = inst.coords()
    e = np.abs(out["U"] - inst.exact(inst.T, X))
    lo, hi = 3 * math.pi / 8 - 1e-12, 11 * math.pi / 8 + 1e-12
    m = (X[0] >= lo) & (X[0] <= hi) & (X[1] >= lo) & (X[1] <= hi)
    return float(np.max(e)), float(np.max(e[m]))


@pytest.mark.parametrize("Nx,col", [(41, "dt=T"), (41, "dt=dx/4"), (41, "dt=dx^1.5"), (41, "dt=dx^2"),
                                    (81, "dt=T"), (81, "dt=dx/4"), (81, "dt=dx^1.5"), (81, "dt=dx^2")])
def test_shifted_domain_explicit_table(Nx, col):
    """On the box [-pi/8, 15pi/8]^2 the boundary data (3/2 - t) sin x1 sin x2 move with t and both sides of the
    diffusion stencil overstep near the corner where sigma = (-1, 1): the explicit scheme then needs
    dt ~ dx^2 (Cor. cor:CFL, second condition).  Whole-grid and interior errors of Table Tab:shifted, including
    the blow-ups for dt = dx/4 and dx^(3/2) at N_x = 81."""
    whole, inner = _shifted_errors(Nx, col)
    assert whole == pytest.approx(SHIFTED["whole grid"][col][str(Nx)], rel=6e-3)
    assert inner == pytest.approx(SHIFTED["[3pi/8, 11pi/8]^2"][col][str(Nx)], rel=6e-3)
