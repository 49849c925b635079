"""CPU FP64 reference for the multigrid study of Section 3 (arXiv:1605.04821).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the tests use it to pin the paper's multigrid
tables and to check the GPU's Galerkin coarse operators; the product path never imports it.

  * ``lisl_laplacian``: the LISL discretisation of the diffusion operator of eq. laplacian on the
    interior nodes of [0,1]^d with 2^l + 1 nodes per axis (eq. def_mAlpha, eq. LSL): per axis the stencil
    2 at the node and -gamma, -(1-gamma) at the nodes m and m+1 cells away on either side; values beyond
    the interior are homogeneous Dirichlet data (zero), so those entries are dropped.
  * ``prolongation``: bilinear interpolation from the interior of the 2^(l-1)+1 grid to the interior of
    the 2^l+1 grid; the Galerkin coarse operator is R A P with R = P^T (Section 3.3).
  * ``complexities``: grid and algebraic complexity (Definitions gridc, algebrac).
  * ``gauss_seidel``, ``mg_cycle``, ``reduction_factor``: lexicographic Gauss-Seidel, V- and W-cycles with
    the Galerkin hierarchy and an exact coarsest solve, and the residual reduction factor
    rho = (r_k / r_0)^(1/k) of Tab:rhoMG (parity unpinned against the printed rates: the right-hand side and
    the order of the post-smoothing sweeps are not stated; with b = 1 and reverse-order post-smoothing the
    rates agree with the printed ones to about 0.03 at l = 6, 7).
  * ``smoothing_factor``: the local Fourier analysis smoothing factor of Gauss-Seidel for the LISL
    Laplacian, eq. smoothingfactorGS (m = 1, gamma = 1 gives the 5-point stencil of Example ex:mu_GS_STD).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def stencil_params(sigma: float, h: float):
    """m and gamma of eq. def_mAlpha for the displacement sigma * sqrt(h) on a grid of spacing h."""
    r = abs(sigma) / math.sqrt(h)
    m = math.floor(r)
    return m, (m + 1) - r


def lisl_laplacian_1d(n: int, sigma: float, h: float) -> sp.csr_matrix:
    """n x n LISL matrix of eq. LSL (interior unknowns, zero values beyond them)."""
    m, g = stencil_params(sigma, h)
    rows, cols, vals = [], [], []
    for i in range(n):
        rows.append(i)
        cols.append(i)
        vals.append(2.0)
        for sgn in (1, -1):
            for off, w in ((m, g), (m + 1, 1.0 - g)):
                j = i + sgn * off
                if 0 <= j < n and w != 0.0:
                    rows.append(i)
                    cols.append(j)
                    vals.append(-w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def lisl_laplacian(l: int, sigma, dim: int = 2) -> sp.csr_matrix:
    """LISL matrix of eq. laplacian with diagonal sigma on the interior of a (2^l + 1)^dim grid of [0,1]^dim:
    the sum over axes of the one-dimensional matrices (Kronecker sums)."""
    n, h = 2 ** l - 1, 2.0 ** -l
    sig = [sigma] * dim if np.isscalar(sigma) else list(sigma)
    I = sp.identity(n, format="csr")
    A = sp.csr_matrix((n ** dim, n ** dim))
    for a in range(dim):
        # axis 0 varies fastest
        parts = [I] * dim
        parts[dim - 1 - a] = lisl_laplacian_1d(n, sig[a], h)
        K = parts[0]
        for p in parts[1:]:
            K = sp.kron(K, p, format="csr")
        A = A + K
    return A.tocsr()


def prolongation_1d(nc: int) -> sp.csr_matrix:
    """Linear interpolation from nc coarse interior nodes to 2 nc + 1 fine interior nodes."""
    nf = 2 * nc + 1
    rows, cols, vals = [], [], []
    for J in range(nc):
        f = 2 * J + 1
        for df, w in ((-1, 0.5), (0, 1.0), (1, 0.5)):
            rows.append(f + df)
            cols.append(J)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def prolongation(nc: int, dim: int = 2) -> sp.csr_matrix:
    """Multilinear (bilinear in 2D) interpolation between the interiors, as a Kronecker product."""
    P1 = prolongation_1d(nc)
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P, format="csr")
    return P


def galerkin_hierarchy(A: sp.csr_matrix, l: int, levels: int, dim: int = 2):
    """[A_1, ..., A_levels] and the prolongations [P_1, ...] with A_{k+1} = P^T A_k P."""
    As, Ps = [A.tocsr()], []
    for k in range(levels - 1):
        P = prolongation(2 ** (l - k - 1) - 1, dim)
        Ac = (P.T @ As[-1] @ P).tocsr()
        Ac.eliminate_zeros()
        As.append(Ac)
        Ps.append(P)
    return As, Ps


def complexities(As):
    """(c_G, c_A) of Definitions gridc and algebrac."""
    n1, z1 = As[0].shape[0], As[0].nnz
    return sum(a.shape[0] for a in As) / n1, sum(a.nnz for a in As) / z1


def gauss_seidel(A: sp.csr_matrix, x: np.ndarray, b: np.ndarray, sweeps: int = 1) -> np.ndarray:
    """Lexicographic (forward) Gauss-Seidel: x <- (D + L)^{-1} (b - U x), sweeps times."""
    DL = sp.tril(A, k=0, format="csr")
    U = sp.triu(A, k=1, format="csr")
    for _ in range(sweeps):
        x = spla.spsolve_triangular(DL, b - U @ x, lower=True)
    return x


def gauss_seidel_backward(A: sp.csr_matrix, x: np.ndarray, b: np.ndarray, sweeps: int = 1) -> np.ndarray:
    """Gauss-Seidel in reverse lexicographic order: x <- (D + U)^{-1} (b - L x)."""
    DU = sp.triu(A, k=0, format="csr")
    L = sp.tril(A, k=-1, format="csr")
    for _ in range(sweeps):
        x = spla.spsolve_triangular(DU, b - L @ x, lower=False)
    return x


def mg_cycle(As, Ps, b, x, nu1=1, nu2=1, gamma=1, k=0):
    """One multigrid cycle on level k (gamma = 1: V-cycle, 2: W-cycle): nu1 lexicographic Gauss-Seidel
    sweeps, the coarse correction with R = P^T (gamma cycles on the next level; one exact solve when it is
    the coarsest), nu2 sweeps in reverse order (the symmetric pairing; the paper names the smoother only)."""
    A = As[k]
    if k == len(As) - 1:
        return spla.spsolve(A.tocsc(), b)
    x = gauss_seidel(A, x, b, nu1)
    rc = Ps[k].T @ (b - A @ x)
    ec = np.zeros(As[k + 1].shape[0])
    for _ in range(gamma if k + 1 < len(As) - 1 else 1):
        ec = mg_cycle(As, Ps, rc, ec, nu1, nu2, gamma, k + 1)
    x = x + Ps[k] @ ec
    return gauss_seidel_backward(A, x, b, nu2)


def reduction_factor(As, Ps, b, nu1=1, nu2=1, gamma=1, tol=1e-6, max_cycles=500):
    """rho = (r_k / r_0)^(1/k) for cycles from x = 0 until |b - A x|_2 / |b|_2 <= tol (Section 3.3)."""
    x = np.zeros_like(b)
    r0 = np.linalg.norm(b)
    for k in range(1, max_cycles + 1):
        x = mg_cycle(As, Ps, b, x, nu1, nu2, gamma)
        rk = np.linalg.norm(b - As[0] @ x)
        if rk <= tol * r0:
            return (rk / r0) ** (1.0 / k), k
    return (rk / r0) ** (1.0 / max_cycles), max_cycles


def smoothing_factor(m, gamma, n: int = 512) -> float:
    """max over high frequencies theta in [-pi,pi)^2 minus [-pi/2,pi/2)^2 of |(g1 + g2) / (4 - conj g1 - conj g2)|,
    g_i = gamma_i e^{i m_i theta_i} + (1 - gamma_i) e^{i (m_i + 1) theta_i} (eq. smoothingfactorGS), on an
    n x n sample of [-pi, pi)^2."""
    th = -math.pi + 2.0 * math.pi * np.arange(n) / n
    T1, T2 = np.meshgrid(th, th, indexing="ij")
    high = ~((np.abs(T1) < math.pi / 2) & (np.abs(T2) < math.pi / 2) | ((T1 == -math.pi / 2) | (T2 == -math.pi / 2))
             & (T1 >= -math.pi / 2) & (T1 < math.pi / 2) & (T2 >= -math.pi / 2) & (T2 < math.pi / 2))
    g = lambda t, ga, mm: ga * np.exp(1j * mm * t) + (1.0 - ga) * np.exp(1j * (mm + 1) * t)
    g1, g2 = g(T1, gamma[0], m[0]), g(T2, gamma[1], m[1])
    S = np.abs((g1 + g2) / (4.0 - np.conj(g1) - np.conj(g2)))
    return float(np.max(S[high]))
