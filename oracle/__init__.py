"""CPU FP64 oracle for the implicit semi-Lagrangian HJB scheme (arXiv:1605.04821).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it to check and time the HIP path.  The product path never
imports it, and it imports nothing from the product package.

Layers (each cites the passage it follows):
  * ``sl_oracle.c`` (built to ``liboracle.so``): the truncated Scheme 2 operator
    L-hat (Section 1 Scheme 2, Section 2.1 eq. TruncScheme, Prop. pro:scheme2
    eqs. eqn_APp1/eqn_Ap, eq. Lhat), its sparse row listing, and the row-wise
    policy search of eq. nonlinear_sys.
  * this module: the theta-scheme system of eq. FullScheme (with Dirichlet data
    moved to the right-hand side as in Remark rem:rhs), Howard policy
    iteration (Section 1, the paragraph after eq. nonlinear_sys), the time
    march, explicit stepping (theta = 0) and a brute-force solve over every
    policy for tiny grids.

Readings taken where the paper is silent (repeated in the design doc):
  * the untruncated diagonal weight is M/dx (the truncated row-sum identity
    after eq. Lhat with A = B = 1), not the M/(2 dx) printed before it;
  * the coefficients and the source are evaluated at t_{n-1} + theta*dt_n;
  * policy iteration starts from the previous step's policy, keeps a control
    whose value is within tau of the minimum and otherwise takes the smallest
    index within tau; tau = tau_rel * S with
    S = (2*M/(2h) + max|c|) * max(|X|_inf, |U|_inf) + |f|_inf;
  * the linear solve is run to an infinity-norm residual certificate: for an
    M-matrix with row sums >= 1 - theta*dt*max(c,0) the error is bounded by
    |r|_inf / (1 - theta*dt*max(c,0)) (row sums, Section 3.4).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TAU_REL = 1e-13


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OrcProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("K", ctypes.c_int32), ("P", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double), ("sr", ctypes.c_double),
                ("sigma", ctypes.c_void_p), ("sig_k", ctypes.c_int64), ("sig_i", ctypes.c_int64),
                ("drift", ctypes.c_void_p), ("b_k", ctypes.c_int64), ("b_i", ctypes.c_int64),
                ("c", ctypes.c_void_p), ("c_k", ctypes.c_int64), ("c_i", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_OrcProblem)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_lhat_apply.argtypes = [P, vp, i32, vp, vp]
        L.orc_lhat_apply.restype = None
        L.orc_landing.argtypes = [P, i64, vp, vp, vp, vp]
        L.orc_landing.restype = None
        L.orc_row_capacity.argtypes = [P]
        L.orc_row_capacity.restype = i64
        L.orc_row.argtypes = [P, i64, i32, vp, vp]
        L.orc_row.restype = i64
        L.orc_weights.argtypes = [P, i64, i32, vp, vp, vp, vp, vp, vp]
        L.orc_weights.restype = None
        L.orc_assemble.argtypes = [P, vp, vp, i64, vp, vp]
        L.orc_assemble.restype = None
        L.orc_improve.argtypes = [P, vp, vp, d, vp, i64, i64, d, vp, vp, vp, vp, vp]
        L.orc_improve.restype = i64
        L.orc_node_values.argtypes = [P, i64, vp, vp, d, vp, i64, i64, vp]
        L.orc_node_values.restype = None
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """Grid + coefficients of one instance, marshalled for the C oracle.

    sigma: (K,P,dim) per control, or sigma_node (N,P,dim) shared by all controls;
    drift: (K,dim) or None; c: (K,) or None.  s scales sigma.  With coef_model "xscaled" the
    coefficients at node x are sigma_k(x) = diag(x) S_k and b_k(x) = diag(x) beta_k (S = sigma,
    beta = drift), expanded here into per-node arrays.
    """

    def __init__(self, inst, s: Optional[float] = None):
        self.inst = inst
        self.dim, self.K, self.P = inst.dim, inst.K, inst.P
        self.n = tuple(int(v) for v in inst.n)
        self.N = int(np.prod(self.n))
        self.h = float(inst.h)
        self.s = float(inst.s if s is None else s)
        st = _OrcProblem()
        st.dim, st.K, st.P = self.dim, self.K, self.P
        for d in range(3):
            st.n[d] = self.n[d] if d < self.dim else 1
        st.h = self.h
        st.sr = self.s * (1.0 / math.sqrt(self.h))
        xs = getattr(inst, "coef_model", "const") == "xscaled"
        if xs:
            # sigma_k(x)_{:,p} = x * S_{k,p}, b_k(x) = x * beta_k (elementwise), per node
            X = np.stack(inst.coords(), axis=-1)                                   # (N, dim)
            self._sigma = np.ascontiguousarray(X[None, :, None, :] * _f64(inst.sigma)[:, None, :, :])
            st.sig_k, st.sig_i = self.N * self.P * self.dim, self.P * self.dim
        elif inst.sigma is not None:
            self._sigma = _f64(inst.sigma)
            st.sig_k, st.sig_i = self.P * self.dim, 0
        else:
            self._sigma = _f64(inst.sigma_node)
            st.sig_k, st.sig_i = 0, self.P * self.dim
        st.sigma = self._sigma.ctypes.data
        if xs and inst.drift is not None:
            self._drift = np.ascontiguousarray(X[None, :, :] * _f64(inst.drift)[:, None, :])
            st.b_k, st.b_i = self.N * self.dim, self.dim
        else:
            self._drift = _f64(inst.drift)
            st.b_k, st.b_i = self.dim, 0
        st.drift = None if self._drift is None else self._drift.ctypes.data
        self._c = _f64(inst.c)
        st.c = None if self._c is None else self._c.ctypes.data
        st.c_k, st.c_i = 1, 0
        self.st = st
        self.has_drift = self._drift is not None and bool(np.any(self._drift != 0.0))
        self.M = self.P + (1 if self.has_drift else 0)
        self.cmax = 0.0 if self._c is None else float(np.max(np.abs(self._c)))
        self.cplus = 0.0 if self._c is None else float(max(0.0, np.max(self._c)))
        self.bd = inst.boundary_mask()
        self.interior = np.nonzero(~self.bd)[0].astype(np.int64)
        self.boundary = np.nonzero(self.bd)[0].astype(np.int64)

    @property
    def ref(self):
        return ctypes.byref(self.st)

    # -- operator -----------------------------------------------------------------
    def lhat(self, V, alpha=None, k0: int = 0):
        """(L-hat^{alpha_i} V)_i at interior nodes (eq. TruncScheme), zero on the boundary."""
        V = _f64(V)
        out = np.empty(self.N)
        a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.int16)
        lib().orc_lhat_apply(self.ref, _ptr(a), k0, _ptr(V), _ptr(out))
        return out

    def row(self, i: int, k: int):
        cap = lib().orc_row_capacity(self.ref)
        cols = np.empty(cap, np.int64)
        vals = np.empty(cap)
        e = lib().orc_row(self.ref, i, k, _ptr(cols), _ptr(vals))
        return cols[:e].copy(), vals[:e].copy()

    def weights(self, i: int, k: int):
        A = np.empty(self.P); B = np.empty(self.P); mp = np.empty(self.P); mm = np.empty(self.P)
        C = np.empty(1); mb = np.empty(1)
        lib().orc_weights(self.ref, i, k, _ptr(A), _ptr(B), _ptr(mp), _ptr(mm), _ptr(C), _ptr(mb))
        return dict(A=A, B=B, mu_plus=mp, mu_minus=mm, C=float(C[0]), mu_b=float(mb[0]))

    def landing(self, i: int, Y):
        """Landing cell, fractions and mu of the point x_i + mu*Y (Y in cells), Section 2.1."""
        Yd = np.zeros(3)
        Yd[:self.dim] = Y
        cell = np.zeros(3, np.int64); t = np.zeros(3); mu = np.zeros(1)
        lib().orc_landing(self.ref, i, _ptr(Yd), _ptr(cell), _ptr(t), _ptr(mu))
        return cell[:self.dim].copy(), t[:self.dim].copy(), float(mu[0])

    def assemble(self, alpha) -> sp.csr_matrix:
        """N x N matrix of L-hat^{alpha} (eq. Lhat); rows of boundary nodes are empty."""
        alpha = np.ascontiguousarray(alpha, dtype=np.int16)
        rows = self.interior
        cap = int(lib().orc_row_capacity(self.ref))
        cols = np.empty(rows.size * cap, np.int64)
        vals = np.empty(rows.size * cap)
        lib().orc_assemble(self.ref, _ptr(alpha), _ptr(rows), rows.size, _ptr(cols), _ptr(vals))
        r = np.repeat(rows, cap)
        keep = cols >= 0
        return sp.csr_matrix((vals[keep], (r[keep], cols[keep])), shape=(self.N, self.N))

    def c_of(self, alpha):
        if self._c is None:
            return np.zeros(self.N)
        out = np.zeros(self.N)
        m = alpha >= 0
        out[m] = self._c[alpha[m]]
        return out

    # -- source -------------------------------------------------------------------
    def f_at(self, f0, f1, t):
        """f(t) = f0 + t*f1, shape (N,) or (K,N)."""
        return _f64(f0) + t * _f64(f1)

    @staticmethod
    def f_strides(f, N):
        return (0, 1) if f.ndim == 1 else (N, 1)

    def f_of(self, f, alpha):
        if f.ndim == 1:
            return f
        out = np.zeros(self.N)
        m = alpha >= 0
        out[m] = f[alpha[m], np.nonzero(m)[0]]
        return out

    # -- policy search --------------------------------------------------------------
    def tau(self, X, U, f, tau_rel: float = TAU_REL) -> float:
        """Hysteresis tolerance of the policy search (scale-relative)."""
        vinf = max(float(np.max(np.abs(X))), float(np.max(np.abs(U))))
        if f.ndim == 1:
            finf = float(np.max(np.abs(f[self.interior])))
        else:
            finf = float(np.max(np.abs(f[:, self.interior])))
        inv2h = 0.5 / self.h
        S = (2.0 * self.M * inv2h + self.cmax) * vinf + finf
        return tau_rel * S

    def improve(self, X, U, theta, f, tau, alpha_in=None, want_extra=True):
        """Row-wise minimisation of G_k over the control set (eq. nonlinear_sys), with the tie rule."""
        X = _f64(X); U = _f64(U); f = _f64(f)
        fk, fi = self.f_strides(f, self.N)
        a_in = None if alpha_in is None else np.ascontiguousarray(alpha_in, dtype=np.int16)
        a_out = np.empty(self.N, np.int16)
        gmin = np.empty(self.N); margin = np.empty(self.N) if want_extra else None
        ties = np.empty(self.N, np.int32) if want_extra else None
        changed = lib().orc_improve(self.ref, _ptr(X), _ptr(U), float(theta), _ptr(f), fk, fi, float(tau),
                                    _ptr(a_in), _ptr(a_out), _ptr(gmin), _ptr(margin), _ptr(ties))
        return dict(alpha=a_out, changed=int(changed), gmin=gmin, margin=margin, ties=ties)

    def node_values(self, i, X, U, theta, f):
        X = _f64(X); U = _f64(U); f = _f64(f)
        fk, fi = self.f_strides(f, self.N)
        G = np.empty(self.K)
        lib().orc_node_values(self.ref, i, _ptr(X), _ptr(U), float(theta), _ptr(f), fk, fi, _ptr(G))
        return G


# ---------------------------------------------------------------------------
# theta-scheme system (eq. FullScheme) for a fixed policy
# ---------------------------------------------------------------------------

@dataclass
class StepStats:
    pi_iters: int = 0
    solves: int = 0
    res_inf: float = 0.0
    changed: list = field(default_factory=list)
    near_ties: int = 0


def explicit_part(pb: Problem, L, alpha, U, f_mid, dt, theta):
    """E_i = U_i + (1-theta) dt ((L U)_i + c U_i) + dt f_i at interior nodes (the known part of eq. FullScheme)."""
    c = pb.c_of(alpha)
    f = pb.f_of(f_mid, alpha)
    if theta == 1.0:
        return U + dt * f
    return U + (1.0 - theta) * dt * (L @ U + c * U) + dt * f


def residual(pb: Problem, L, alpha, V, E, dt, theta):
    """r = E - (V - theta dt (L V + c V)) on interior nodes (boundary values of V are the Dirichlet data)."""
    c = pb.c_of(alpha)
    r = E - (V - theta * dt * (L @ V + c * V))
    r[pb.bd] = 0.0
    return r


def _system_matrix(pb: Problem, L, alpha, dt, theta):
    """A^alpha restricted to interior unknowns: I - theta dt (L + c) (eq. FullScheme, Remark rem:rhs)."""
    I = pb.interior
    Lii = L[I][:, I]
    c = pb.c_of(alpha)[I]
    return (sp.identity(I.size, format="csr") - theta * dt * (Lii + sp.diags(c))).tocsc()


def linear_solve(pb: Problem, L, alpha, V, E, dt, theta, rtol=1e-14, max_refine=20, direct_limit=70000,
                 direct_limit_3d=8000):
    """Solve the fixed-policy system to the infinity-norm certificate |r|_inf <= rtol * |V|_inf.

    Direct sparse LU (SuperLU) for up to direct_limit unknowns in 2D (direct_limit_3d in 3D, where the
    fill-in of the wide stencil makes the factorisation slow), else Jacobi-preconditioned GMRES; both
    followed by residual-correction sweeps until the certificate holds.
    """
    I = pb.interior
    A = _system_matrix(pb, L, alpha, dt, theta)
    V = V.copy()
    if I.size <= (direct_limit if pb.dim == 2 else min(direct_limit, direct_limit_3d)):
        lu = spla.splu(A)
        solve = lu.solve
    else:
        dinv = 1.0 / A.diagonal()
        Mop = spla.LinearOperator(A.shape, matvec=lambda x: dinv * x)

        def solve(b):
            x, info = spla.gmres(A, b, rtol=1e-13, atol=0.0, restart=60, maxiter=400, M=Mop)
            return x
    for it in range(max_refine):
        r = residual(pb, L, alpha, V, E, dt, theta)
        rinf = float(np.max(np.abs(r)))
        if rinf <= rtol * max(1.0, float(np.max(np.abs(V)))):
            return V, rinf
        V[I] += solve(r[I])
    r = residual(pb, L, alpha, V, E, dt, theta)
    rinf = float(np.max(np.abs(r)))
    if rinf > 1e3 * rtol * max(1.0, float(np.max(np.abs(V)))):
        raise RuntimeError(f"oracle linear solve did not converge: |r|_inf={rinf:g}")
    return V, rinf


def step(pb: Problem, Uprev, psi, f0, f1, t_prev, dt, theta, alpha_prev, rtol=1e-14, max_pi=50, tau_rel=TAU_REL):
    """One implicit theta-step by Howard policy iteration (eq. nonlinear_sys and the paragraph after it).

    Returns (U_n, alpha, StepStats).  theta = 0 is an explicit step (one search, no solve).
    """
    t_mid = t_prev + theta * dt
    f = pb.f_at(f0, f1, t_mid)
    U = _f64(Uprev)
    st = StepStats()
    if theta == 0.0:
        tau = pb.tau(U, U, f, tau_rel)
        res = pb.improve(U, U, 0.0, f, tau, alpha_prev, want_extra=False)
        V = U + dt * res["gmin"]
        V[pb.bd] = psi[pb.bd]
        return V, res["alpha"], st
    V = U.copy()
    V[pb.bd] = psi[pb.bd]
    tau = pb.tau(V, U, f, tau_rel)
    res = pb.improve(V, U, theta, f, tau, alpha_prev)
    alpha = res["alpha"]
    for it in range(max_pi):
        L = pb.assemble(alpha)
        E = explicit_part(pb, L, alpha, U, f, dt, theta)
        V, rinf = linear_solve(pb, L, alpha, V, E, dt, theta, rtol=rtol)
        st.solves += 1
        st.res_inf = rinf
        tau = pb.tau(V, U, f, tau_rel)
        res = pb.improve(V, U, theta, f, tau, alpha)
        st.pi_iters = it + 1
        st.changed.append(res["changed"])
        if res["changed"] == 0:
            # several policies are correct results where the runner-up is within 1e3 tau of the best
            st.near_ties = int(np.sum(((res["ties"] > 1) | (res["margin"] < 1e3 * tau))[pb.interior]))
            return V, alpha, st
        alpha = res["alpha"]
    raise RuntimeError("policy iteration did not terminate")


def psi_at(inst, t: float):
    """Dirichlet data at time t (eq. 1.3): psi, or psi + t psi1 when the instance gives time-dependent data."""
    psi1 = getattr(inst, "psi1", None)
    return inst.psi if psi1 is None else inst.psi + t * psi1


def march(inst, s: Optional[float] = None, rtol=1e-14, keep_policies=False, keep_values=False, n_steps=None):
    """Time march of the theta-scheme from U^0 = g (eq. 1.2) with U^n = psi(t_n) on the boundary (eq. 1.3)."""
    pb = Problem(inst, s=s)
    U = _f64(inst.g).copy()
    alpha = np.zeros(pb.N, np.int16)
    alpha[pb.bd] = -1
    t = 0.0
    pols, vals, stats = [], [U.copy()], []
    steps = len(inst.dts) if n_steps is None else n_steps
    for n in range(steps):
        dt, th = float(inst.dts[n]), float(inst.thetas[n])
        U, alpha, st = step(pb, U, psi_at(inst, t + dt), inst.f0, inst.f1, t, dt, th, alpha, rtol=rtol)
        t = t + dt
        stats.append(st)
        if keep_policies:
            pols.append(alpha.copy())
        if keep_values:
            vals.append(U.copy())
    out = dict(U=U, alpha=alpha, stats=stats, t=t)
    if keep_policies:
        out["policies"] = np.stack(pols)
    if keep_values:
        out["values"] = np.stack(vals)
    return out


# ---------------------------------------------------------------------------
# Brute force over all policies (tiny grids only)
# ---------------------------------------------------------------------------

def brute_force_step(pb: Problem, Uprev, psi, f0, f1, t_prev, dt, theta):
    """min over every policy alpha of (A^alpha)^{-1} F^alpha, componentwise.

    For M-matrices A^alpha the solution X* of eq. nonlinear_sys satisfies X* <= X^alpha for every
    policy, with equality for an optimal one, so the componentwise minimum is X*.
    """
    I = pb.interior
    n = I.size
    K = pb.K
    if K ** n > 300000:
        raise ValueError("too many policies for brute force")
    t_mid = t_prev + theta * dt
    f = pb.f_at(f0, f1, t_mid)
    U = _f64(Uprev)
    Vb = np.zeros(pb.N)
    Vb[pb.bd] = psi[pb.bd]
    # per control k: dense rows restricted to interior columns and the right-hand side of eq. FullScheme,
    # B U^{n-1} + dt f + the Dirichlet contribution, written out with dense matrices on every node
    Arows = np.empty((K, n, n))
    Frows = np.empty((K, n))
    for k in range(K):
        alpha = np.full(pb.N, k, np.int16)
        alpha[pb.bd] = -1
        Ld = pb.assemble(alpha).toarray()
        c = pb.c_of(alpha)
        B = np.eye(pb.N) + (1.0 - theta) * dt * (Ld + np.diag(c))
        rhs = B @ U + dt * pb.f_of(f, alpha) + theta * dt * (Ld @ Vb)
        Arows[k] = np.eye(n) - theta * dt * (Ld[np.ix_(I, I)] + np.diag(c[I]))
        Frows[k] = rhs[I]
    best = np.full(n, np.inf)
    idx = np.indices((K,) * n).reshape(n, -1).T  # every policy
    chunk = 4096
    for s0 in range(0, idx.shape[0], chunk):
        pol = idx[s0:s0 + chunk]                       # (m, n)
        A = Arows[pol, np.arange(n)[None, :], :]       # (m, n, n)
        F = Frows[pol, np.arange(n)[None, :]]          # (m, n)
        X = np.linalg.solve(A, F[..., None])[..., 0]
        best = np.minimum(best, X.min(axis=0))
    V = Vb.copy()
    V[I] = best
    return V


# ---------------------------------------------------------------------------
# Adjoint at fixed policies (the discrete adjoint of eq. FullScheme, transposed)
# ---------------------------------------------------------------------------

def fixed_policy_march(inst, policies, s: Optional[float] = None, rtol=1e-15):
    """U^0..U^N of the theta-scheme with the given per-step policies (one linear solve per step)."""
    pb = Problem(inst, s=s)
    U = _f64(inst.g).copy()
    out = [U.copy()]
    t = 0.0
    for n in range(len(policies)):
        dt, th = float(inst.dts[n]), float(inst.thetas[n])
        alpha = np.ascontiguousarray(policies[n], dtype=np.int16)
        f = pb.f_at(inst.f0, inst.f1, t + th * dt)
        L = pb.assemble(alpha)
        E = explicit_part(pb, L, alpha, U, f, dt, th)
        V = U.copy()
        V[pb.bd] = psi_at(inst, t + dt)[pb.bd]
        V, _ = linear_solve(pb, L, alpha, V, E, dt, th, rtol=rtol)
        U = V
        out.append(U.copy())
        t = t + dt
    return out


def adjoint_dense(inst, policies, lam_N, s: Optional[float] = None):
    """Gradients of a functional J of U^N with dJ/dU^N = lam_N, at fixed policies.

    Step n solves A_n U^n = B_n U^{n-1} + dt f_n + (Dirichlet terms), A_n = I - theta dt (L + C) on interior
    unknowns, B_n = I + (1-theta) dt (L + C) applied to the full U^{n-1}.  Backwards: A_n^T mu_n = lam_n,
    dJ/df0 += dt mu_n, dJ/df1 += dt t_mid mu_n, lam_{n-1} = B_n^T mu_n; dJ/dg = lam_0 (all nodes).
    """
    pb = Problem(inst, s=s)
    I = pb.interior
    N = pb.N
    lam = _f64(lam_N).copy()
    lam[pb.bd] = 0.0
    df0 = np.zeros(N)
    df1 = np.zeros(N)
    times = np.concatenate([[0.0], np.cumsum(inst.dts)])
    for n in reversed(range(len(policies))):
        dt, th = float(inst.dts[n]), float(inst.thetas[n])
        t_mid = float(times[n]) + th * dt
        alpha = np.ascontiguousarray(policies[n], dtype=np.int16)
        L = pb.assemble(alpha).tocsr()
        c = pb.c_of(alpha)
        A = _system_matrix(pb, L, alpha, dt, th)
        mu = np.zeros(N)
        mu[I] = spla.spsolve(A.T.tocsc(), lam[I])
        df0 += dt * mu
        df1 += dt * t_mid * mu
        lam_new = np.zeros(N)
        lam_new[I] = mu[I] + (1.0 - th) * dt * c[I] * mu[I]
        lam_new += (1.0 - th) * dt * (L[I].T @ mu[I])
        lam = lam_new
    return dict(df0=df0, df1=df1, dg=lam)


def ds_central_difference(inst, policies, lam_N, s: float, eps: float = 1e-5):
    """d/ds of lam_N . U^N(s) at fixed policies by a central difference of the fixed-policy march."""
    up = fixed_policy_march(inst, policies, s=s + eps)[-1]
    dn = fixed_policy_march(inst, policies, s=s - eps)[-1]
    return float(np.dot(lam_N, up - dn) / (2.0 * eps))
