"""Seeded synthetic inputs for the semi-Lagrangian HJB solver and its oracle.

This module only *describes problems*: grids, control sets, coefficient tables
and the data fields f, g, psi of the initial-boundary value problem (1.1)-(1.3)
of Reisinger & Rotaetxe Arto (arXiv:1605.04821, Section 1).  It contains none of
the scheme's arithmetic (no interpolation, truncation, time stepping or
solves), so both the HIP path and the CPU oracle can draw their inputs from it
without sharing any of the method.

Conventions
-----------
* Grids are uniform with spacing h on every axis (Section 2.1 assumes a
  Cartesian mesh with one mesh width); node (i0, i1, i2) sits at
  lo + i*h and the flat index is i0 + n0*(i1 + n1*i2) (x fastest).
  Numpy fields are shaped (n1, n0) in 2D and (n2, n1, n0) in 3D.
* A control k carries P diffusion columns sigma[k, p, :] (a = 1/2 sigma sigma^T,
  eq. (1.1) and the definition of L), a drift b[k, :] and a discount c[k].
* The source is affine in time and the same for every control unless stated:
  f(t, x) = f0(x) + t * f1(x).  Dirichlet data are constant in time unless psi1
  is given: psi(t, x) = psi(x) + t * psi1(x) (the shifted-domain Problem A).  Problem B of Section 2.4 has a
  control-dependent source; it is given as f0[k, :], f1[k, :].
* A time schedule is a list of (dt_n, theta_n).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Instance:
    """One HJB problem on a box: coefficients, data and time schedule."""

    name: str
    dim: int
    n: tuple                     # nodes per axis (n0, n1[, n2])
    lo: tuple                    # lower corner of the box
    h: float                     # mesh width (same on all axes)
    K: int                       # number of controls
    P: int                       # diffusion columns per control
    sigma: Optional[np.ndarray]  # (K, P, dim) constant per control, or None
    drift: Optional[np.ndarray]  # (K, dim) constant per control, or None
    c: Optional[np.ndarray]      # (K,) constant per control, or None
    f0: np.ndarray               # (N,) or (K, N)
    f1: np.ndarray               # (N,) or (K, N)
    g: np.ndarray                # (N,) initial data u(0, x)
    psi: np.ndarray              # (N,) Dirichlet data on the boundary nodes (at t = 0 when psi1 is given)
    dts: np.ndarray              # (n_steps,)
    thetas: np.ndarray           # (n_steps,)
    s: float = 1.0               # volatility scale multiplying sigma
    sigma_node: Optional[np.ndarray] = None   # (N, P, dim): x-dependent, control-independent sigma
    coef_model: str = "const"    # "const": sigma, drift per control; "xscaled": sigma_k(x) = diag(x) S_k,
                                 # b_k(x) = diag(x) beta_k with S = sigma (K, P, dim), beta = drift (K, dim)
    exact: Optional[callable] = None          # closed-form u(t, X) if known, X = coordinate arrays
    psi1: Optional[np.ndarray] = None         # (N,) time-dependent Dirichlet data psi(t) = psi + t * psi1
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def T(self) -> float:
        return float(np.sum(self.dts))

    def coords(self):
        """Coordinate arrays shaped like the fields (x fastest)."""
        axes = [self.lo[d] + np.arange(self.n[d], dtype=np.float64) * self.h for d in range(self.dim)]
        grids = np.meshgrid(*axes[::-1], indexing="ij")  # slowest axis first
        return [g.reshape(-1) for g in grids[::-1]]      # returns x0, x1[, x2] flattened

    def boundary_mask(self) -> np.ndarray:
        idx = np.indices(self.n[::-1]).reshape(self.dim, -1)[::-1]  # idx[d] = i_d
        m = np.zeros(self.N, dtype=bool)
        for d in range(self.dim):
            m |= (idx[d] == 0) | (idx[d] == self.n[d] - 1)
        return m

    def times(self) -> np.ndarray:
        return np.concatenate([[0.0], np.cumsum(self.dts)])


# ---------------------------------------------------------------------------
# Control sets
# ---------------------------------------------------------------------------

def angles_half_circle(K: int) -> np.ndarray:
    """K equispaced angles in [0, pi): theta_k = k*pi/K."""
    return np.arange(K, dtype=np.float64) * (math.pi / K)


def angles_full_circle(K: int) -> np.ndarray:
    """K equispaced angles in [0, 2*pi): phi_k = 2*pi*k/K (control set on the unit circle)."""
    return np.arange(K, dtype=np.float64) * (2.0 * math.pi / K)


def fibonacci_hemisphere(K: int) -> np.ndarray:
    """K unit vectors on the upper hemisphere (golden-angle spiral), shape (K, 3)."""
    k = np.arange(K, dtype=np.float64)
    z = (k + 0.5) / K
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def rannacher_cn(n_cn: int, dt: float, n_startup: int = 2):
    """Crank-Nicolson schedule whose first step is replaced by n_startup implicit steps of dt/n_startup."""
    dts = [dt / n_startup] * n_startup + [dt] * (n_cn - 1)
    thetas = [1.0] * n_startup + [0.5] * (n_cn - 1)
    return np.asarray(dts, dtype=np.float64), np.asarray(thetas, dtype=np.float64)


# ---------------------------------------------------------------------------
# Manufactured 2D problem u = (1+t) sin(pi x) sin(pi y) on the unit square
# ---------------------------------------------------------------------------

def _box(dim, n):
    h = 1.0 / (n - 1)
    return (n,) * dim, (0.0,) * dim, h


def _sinprod_fields(inst_coords, dim):
    s = [np.sin(math.pi * x) for x in inst_coords]
    c = [np.cos(math.pi * x) for x in inst_coords]
    return s, c


def manufactured_2d(n: int, K: int, drift_scale: float, dts, thetas, name: str,
                    source: str = "lambda_min", s: float = 1.0) -> Instance:
    """u=(1+t) sin(pi x) sin(pi y), sigma_k=(cos th_k, sin th_k), th_k = k*pi/K, b_k = drift_scale*(cos th_k, -sin th_k).

    source="lambda_min": f = u_t - 1/2 lambda_min(D^2 u)   (continuous-control closed form)
    source="discrete"  : f = u_t - min_k [1/2 sigma_k^T D^2u sigma_k + b_k . Du]
                         which makes u the exact solution of the PDE with the discrete control set.
    """
    shape, lo, h = _box(2, n)
    th = angles_half_circle(K)
    sigma = np.stack([np.cos(th), np.sin(th)], axis=1)[:, None, :].copy()      # (K,1,2)
    drift = None
    if drift_scale != 0.0:
        drift = drift_scale * np.stack([np.cos(th), -np.sin(th)], axis=1)
    inst = Instance(name=name, dim=2, n=shape, lo=lo, h=h, K=K, P=1, sigma=sigma, drift=drift, c=None,
                    f0=None, f1=None, g=None, psi=None, dts=np.asarray(dts, np.float64),
                    thetas=np.asarray(thetas, np.float64), s=s)
    x, y = inst.coords()
    sx, sy, cx, cy = np.sin(math.pi * x), np.sin(math.pi * y), np.cos(math.pi * x), np.cos(math.pi * y)
    ss = sx * sy
    if source == "lambda_min":
        # D^2u/(1+t) = pi^2 [[-ss, cc],[cc, -ss]],  lambda_min = pi^2 (-ss - |cc|)
        q = 0.5 * math.pi ** 2 * (ss + np.abs(cx * cy))
        inst.f0 = ss + q
        inst.f1 = q.copy()
    elif source == "discrete":
        # Hamiltonian per unit (1+t): 1/2 s^2 sigma^T H0 sigma + b.g0 with H0 = D^2u/(1+t), g0 = Du/(1+t)
        h11 = -math.pi ** 2 * ss
        h12 = math.pi ** 2 * cx * cy
        g1 = math.pi * cx * sy
        g2 = math.pi * sx * cy
        best = np.full(inst.N, np.inf)
        for k in range(K):
            a, b = sigma[k, 0]
            val = 0.5 * s * s * (a * a * h11 + 2 * a * b * h12 + b * b * h11)
            if drift is not None:
                val = val + drift[k, 0] * g1 + drift[k, 1] * g2
            best = np.minimum(best, val)
        inst.f0 = ss - best
        inst.f1 = -best
    else:
        raise ValueError(source)
    inst.g = ss.copy()
    inst.psi = np.zeros(inst.N)
    inst.exact = lambda t, X: (1.0 + t) * np.sin(math.pi * X[0]) * np.sin(math.pi * X[1])
    return inst


def config_c1(n: int = 33, source: str = "lambda_min") -> Instance:
    """2D unit square, 33^2 nodes, T=1, 10 implicit Euler steps, 16 controls th_k=k*pi/16, b=c=0."""
    return manufactured_2d(n, 16, 0.0, [0.1] * 10, [1.0] * 10, name=f"c1_{n}", source=source)


def config_c2(n: int = 257, n_cn: int = 64, source: str = "lambda_min", s: float = 1.0) -> Instance:
    """2D manufactured problem, 32 controls in [0,pi), drift 0.1(cos, -sin), Crank-Nicolson with Rannacher start."""
    dts, thetas = rannacher_cn(n_cn, 1.0 / n_cn)
    return manufactured_2d(n, 32, 0.1, dts, thetas, name=f"c2_{n}", source=source, s=s)


def config_h(n: int = 2049, n_cn: int = 64) -> Instance:
    """Headline workload: the Crank-Nicolson drift problem at 2049^2, 32 controls, dt=1/64 (65 solves)."""
    inst = config_c2(n=n, n_cn=n_cn)
    inst.name = f"h_{n}"
    return inst


def config_c3(n: int = 513, n_cn: int = 64, s: float = 1.0, seed: int = 1605):
    """Adjoint workload: C2 physics at 513^2 plus the target u_tgt = u(1,.) + 1e-3 N(0,1) on interior nodes."""
    inst = config_c2(n=n, n_cn=n_cn, s=s)
    inst.name = f"c3_{n}"
    rng = np.random.default_rng(seed)
    X = inst.coords()
    tgt = inst.exact(inst.T, X)
    interior = ~inst.boundary_mask()
    tgt = tgt + np.where(interior, 1e-3 * rng.standard_normal(inst.N), 0.0)
    inst.meta["u_tgt"] = tgt
    return inst


def config_c5(n: int = 129, K: int = 64, n_steps: int = 32, source: str = "lambda_min") -> Instance:
    """3D unit cube, 64 Fibonacci-hemisphere directions, a = 1/2 v v^T, u=(1+t) prod sin(pi x_i), theta=1."""
    shape, lo, h = _box(3, n)
    v = fibonacci_hemisphere(K)
    inst = Instance(name=f"c5_{n}", dim=3, n=shape, lo=lo, h=h, K=K, P=1, sigma=v[:, None, :].copy(),
                    drift=None, c=None, f0=None, f1=None, g=None, psi=None,
                    dts=np.full(n_steps, 1.0 / n_steps), thetas=np.ones(n_steps))
    X = inst.coords()
    s = [np.sin(math.pi * x) for x in X]
    c = [np.cos(math.pi * x) for x in X]
    prod = s[0] * s[1] * s[2]
    # M = D^2 u / ((1+t) pi^2)
    M = np.empty((inst.N, 3, 3))
    M[:, 0, 0] = M[:, 1, 1] = M[:, 2, 2] = -prod
    M[:, 0, 1] = M[:, 1, 0] = c[0] * c[1] * s[2]
    M[:, 0, 2] = M[:, 2, 0] = c[0] * s[1] * c[2]
    M[:, 1, 2] = M[:, 2, 1] = s[0] * c[1] * c[2]
    if source == "lambda_min":
        lam = np.linalg.eigvalsh(M)[:, 0]
    elif source == "discrete":
        lam = np.min(np.einsum("kd,nde,ke->nk", v, M, v), axis=1)
    else:
        raise ValueError(source)
    q = -0.5 * math.pi ** 2 * lam
    inst.f0 = prod + q
    inst.f1 = q.copy()
    inst.g = prod.copy()
    inst.psi = np.zeros(inst.N)
    inst.exact = lambda t, X: (1.0 + t) * np.sin(math.pi * X[0]) * np.sin(math.pi * X[1]) * np.sin(math.pi * X[2])
    return inst


# ---------------------------------------------------------------------------
# Problems A and B of Section 2.4 (closed-form benchmarks on [-pi, pi]^2, T = 1/2)
# ---------------------------------------------------------------------------

def _problem_box(Nx):
    h = 2.0 * math.pi / (Nx - 1)
    return (Nx, Nx), (-math.pi, -math.pi), h


def _schedule(T, dt, theta):
    n_steps = int(math.ceil(T / dt - 1e-12))
    return np.full(n_steps, T / n_steps), np.full(n_steps, float(theta))


def problem_a(Nx: int, dt: Optional[float] = None, theta: float = 1.0, n_alpha: int = 40,
              lo_shift: float = 0.0) -> Instance:
    """Problem A: u=(3/2-t) sin x1 sin x2, b^alpha = alpha on the unit circle, sigma = sqrt2 (sin(x1+x2), cos(x1+x2)).

    lo_shift moves the box to [-pi+shift, pi+shift]^2 (the shifted-domain experiment uses 7*pi/8).
    """
    T = 0.5
    shape, lo, h = _problem_box(Nx)
    lo = (lo[0] + lo_shift, lo[1] + lo_shift)
    dts, thetas = _schedule(T, T if dt is None else dt, theta)
    phi = angles_full_circle(n_alpha)
    alpha = np.stack([np.cos(phi), np.sin(phi)], axis=1)
    inst = Instance(name=f"problem_a_{Nx}", dim=2, n=shape, lo=lo, h=h, K=n_alpha, P=1, sigma=None,
                    drift=alpha, c=None, f0=None, f1=None, g=None, psi=None, dts=dts, thetas=thetas)
    x1, x2 = inst.coords()
    s1, s2, c1, c2 = np.sin(x1), np.sin(x2), np.cos(x1), np.cos(x2)
    sp, cp = np.sin(x1 + x2), np.cos(x1 + x2)
    inst.sigma_node = (math.sqrt(2.0) * np.stack([sp, cp], axis=1))[:, None, :].copy()
    grad = np.sqrt(c1 * c1 * s2 * s2 + s1 * s1 * c2 * c2)
    br = grad - 2.0 * sp * cp * c1 * c2
    # f = (1/2 - t) s1 s2 + (3/2 - t) br  = [s1 s2/2 + 3 br/2] + t [-s1 s2 - br]
    inst.f0 = 0.5 * s1 * s2 + 1.5 * br
    inst.f1 = -s1 * s2 - br
    inst.g = 1.5 * s1 * s2
    # u on the boundary: (3/2 - t) s1 s2, i.e. psi + t psi1 (zero up to rounding on [-pi,pi]^2; the shifted
    # box of Remark rem:two-over has non-zero, time-dependent boundary data)
    bd = inst.boundary_mask()
    inst.psi = 1.5 * s1 * s2 * bd
    if lo_shift != 0.0:
        inst.psi1 = -(s1 * s2) * bd
    inst.exact = lambda t, X: (1.5 - t) * np.sin(X[0]) * np.sin(X[1])
    return inst


def problem_b(Nx: int, dt: Optional[float] = None, theta: float = 1.0, n_alpha: int = 40) -> Instance:
    """Problem B: u=(2-t) sin x1 sin x2, sigma^alpha = sqrt2 alpha, b=c=0, control-dependent source."""
    T = 0.5
    shape, lo, h = _problem_box(Nx)
    dts, thetas = _schedule(T, T if dt is None else dt, theta)
    phi = angles_full_circle(n_alpha)
    alpha = np.stack([np.cos(phi), np.sin(phi)], axis=1)
    inst = Instance(name=f"problem_b_{Nx}", dim=2, n=shape, lo=lo, h=h, K=n_alpha, P=1,
                    sigma=(math.sqrt(2.0) * alpha)[:, None, :].copy(), drift=None, c=None,
                    f0=None, f1=None, g=None, psi=None, dts=dts, thetas=thetas)
    x1, x2 = inst.coords()
    ss = np.sin(x1) * np.sin(x2)
    cc = np.cos(x1) * np.cos(x2)
    a12 = (alpha[:, 0] * alpha[:, 1])[:, None]
    # f^alpha = (1-t) ss - 2 a1 a2 (2-t) cc = [ss - 4 a1a2 cc] + t [-ss + 2 a1a2 cc]
    inst.f0 = ss[None, :] - 4.0 * a12 * cc[None, :]
    inst.f1 = -ss[None, :] + 2.0 * a12 * cc[None, :]
    inst.g = 2.0 * ss
    inst.psi = np.zeros(inst.N)
    inst.exact = lambda t, X: (2.0 - t) * np.sin(X[0]) * np.sin(X[1])
    return inst


# ---------------------------------------------------------------------------
# Generic random fields for parity tests
# ---------------------------------------------------------------------------

def c4_instance(n: int, sig_min: float, sig_max: float, rho_bar: float, r: float, n_steps: int = 50,
                T: float = 1.0, name: str = "c4") -> Instance:
    """Two-asset model with uncertain volatilities and correlation on [0,4]^2 (x-scaled coefficients).

    Control k: bit 0 picks sigma_1, bit 1 picks sigma_2 in {sig_min, sig_max}, bit 2 picks
    rho in {-rho_bar, +rho_bar}.  a = 1/2 sigma sigma^T with the Cholesky columns S_1 = (s1, rho s2),
    S_2 = (0, sqrt(1 - rho^2) s2) scaled by diag(x); drift diag(x) (r, r); c = -r; f = 0;
    g = psi = max(x_1 - x_2, 0); theta = 1 with dt = T / n_steps.
    """
    shape, lo, h = (n, n), (0.0, 0.0), 4.0 / (n - 1)
    K, P = 8, 2
    S = np.zeros((K, P, 2))
    beta = np.zeros((K, 2))
    for k in range(K):
        s1 = sig_max if (k & 1) else sig_min
        s2 = sig_max if (k & 2) else sig_min
        rho = rho_bar if (k & 4) else -rho_bar
        S[k, 0] = (s1, rho * s2)
        S[k, 1] = (0.0, math.sqrt(1.0 - rho * rho) * s2)
        beta[k] = (r, r)
    inst = Instance(name=f"{name}_{n}", dim=2, n=shape, lo=lo, h=h, K=K, P=P, sigma=S, drift=beta,
                    c=np.full(K, -r), f0=None, f1=None, g=None, psi=None,
                    dts=np.full(n_steps, T / n_steps), thetas=np.ones(n_steps), coef_model="xscaled")
    X = inst.coords()
    payoff = np.maximum(X[0] - X[1], 0.0)
    inst.f0 = np.zeros(inst.N)
    inst.f1 = np.zeros(inst.N)
    inst.g = payoff.copy()
    inst.psi = np.where(inst.boundary_mask(), payoff, 0.0)
    inst.meta.update(sig_min=sig_min, sig_max=sig_max, rho_bar=rho_bar, r=r)
    return inst


def config_c4(count: int = 64, seed: int = 4821, sizes=(65, 129, 257, 513), n_steps: int = 50):
    """Batch of `count` uneven two-asset instances (see c4_instance); per instance the draw order is
    n, sig_min ~ U[.1,.2], sig_max = sig_min + U[.1,.2], rho_bar ~ U[.3,.5], r ~ U[0,.05]."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        smin = float(rng.uniform(0.1, 0.2))
        smax = smin + float(rng.uniform(0.1, 0.2))
        rho = float(rng.uniform(0.3, 0.5))
        r = float(rng.uniform(0.0, 0.05))
        out.append(c4_instance(n, smin, smax, rho, r, n_steps=n_steps, name=f"c4b{b}"))
    return out


def random_fields(inst: Instance, seed: int, scale: float = 1.0):
    """Seeded smooth-plus-noise fields (X, U) with the instance's boundary data, for operator tests."""
    rng = np.random.default_rng(seed)
    X = inst.coords()
    base = np.ones(inst.N)
    for x in X:
        base = base * np.sin(math.pi * (x - inst.lo[0]) / (inst.h * (inst.n[0] - 1)) + 0.3)
    a = scale * (base + 0.05 * rng.standard_normal(inst.N))
    b = scale * (0.7 * base + 0.05 * rng.standard_normal(inst.N))
    bd = inst.boundary_mask()
    a[bd] = inst.psi[bd]
    b[bd] = inst.psi[bd]
    return a, b


def random_policy(inst: Instance, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.integers(0, inst.K, size=inst.N).astype(np.int16)
    a[inst.boundary_mask()] = -1
    return a
