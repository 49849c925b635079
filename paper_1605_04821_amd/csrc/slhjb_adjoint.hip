// Adjoint kernels of libslhjb: the transposed operator of eq. FullScheme at a fixed policy and the
// derivative of the operator with respect to the volatility scale s.
//
// Transposition.  The rows of L-hat^alpha (eq. Lhat: for each stencil point, its truncation weight
// times the corner weights of eq. monotone_int, plus the diagonal) are emitted into fixed slots
// (node i, entry e) and sorted by column with a counting sort that keeps the slot order within a
// column.  The transposed product then gathers, for each column j, the entries of the rows that
// reference j in increasing row order: deterministic, no atomics in the products.
//
// s-derivative.  Diffusion displacements are Y = s*sigma/sqrt(h) (drift points do not depend on s).
// The operator is evaluated with forward-mode dual numbers along the same landing rules as the
// forward kernels, so the derivative includes how truncation (mu, A_p, B_p of Prop. pro:scheme2)
// changes with s; it is the one-sided derivative at the (measure-zero) kinks of floor and min.

#include <algorithm>
#include <climits>

#include "slhjb_internal.h"

namespace slhjb {

__device__ __forceinline__ int remap_block_a(int b, int nb) {
    int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <int DIM>
__device__ __forceinline__ int tile_node_a(const LevelDev &g, int ix[3]) {
    int b = remap_block_a(blockIdx.x, gridDim.x);
    int bx = b % g.ntx, r = b / g.ntx;
    int by = DIM == 3 ? r % g.nty : r;
    int bz = DIM == 3 ? r / g.nty : 0;
    ix[0] = (bx << g.tlog) + (int)(threadIdx.x & ((1u << g.tlog) - 1));
    ix[1] = by * (kBlock >> g.tlog) + (int)(threadIdx.x >> g.tlog);
    ix[2] = bz;
    if (ix[0] >= g.n[0] || ix[1] >= g.n[1]) return -1;
    return ix[0] + ix[1] * (int)g.s1 + (DIM == 3 ? ix[2] * (int)g.s2 : 0);
}

template <int DIM>
__device__ __forceinline__ bool interior_a(const LevelDev &g, const int ix[3]) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ok = ok && ix[d] > 0 && ix[d] < g.n[d] - 1;
    return ok;
}

template <int DIM>
__device__ __forceinline__ bool deep_a(const LevelDev &g, const int ix[3]) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ok = ok && ix[d] >= g.deep_lo[d] && ix[d] <= g.deep_hi[d];
    return ok;
}

// ---- columns of L whose stencil window holds few controls ------------------------------------------

// tset[(1 + kWinMax) T ...] = {n, k_0 < k_1 < ...}: the n <= kWinMax distinct controls of tile T when all its
// nodes are interior and untruncated, else n = -1
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_tile_set(LevelDev g, const int16_t *__restrict__ alpha, int K,
                                                     int32_t *__restrict__ tset) {
    __shared__ int smin;
    int ix[3];
    const int j = tile_node_a<DIM>(g, ix);
    const bool ok = j >= 0 && interior_a<DIM>(g, ix) && deep_a<DIM>(g, ix);
    const int k = ok ? (int)alpha[j] : -1;
    const int all = __syncthreads_and((ok && k >= 0 && k < K) ? 1 : 0);
    int32_t *out = tset + (int64_t)remap_block_a(blockIdx.x, gridDim.x) * (1 + kWinMax);
    if (!all) {
        if (threadIdx.x == 0) out[0] = -1;
        return;
    }
    int n = 0, last = -1;
    for (int it = 0; it <= kWinMax; ++it) {
        if (threadIdx.x == 0) smin = 0x7fffffff;
        __syncthreads();
        if (k > last) atomicMin(&smin, k);
        __syncthreads();
        const int m = smin;
        __syncthreads();
        if (m == 0x7fffffff) break;
        if (it == kWinMax) {
            n = -1;  // more controls than a window may hold
            break;
        }
        if (threadIdx.x == 0) out[1 + n] = m;
        ++n;
        last = m;
    }
    if (threadIdx.x == 0) out[0] = n;
}

void launch_tile_set(int dim, const LevelDev &g, const int16_t *alpha, int K, int32_t *tset, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_tile_set<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, alpha, K, tset);
    else
        hipLaunchKernelGGL(k_tile_set<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, alpha, K, tset);
}

// wset[T] = the union of tset over the tiles within the stencil reach of T (n = -1 when a tile there is
// not all-untruncated, or when the union exceeds kWinMax); a window cut by the grid edge holds boundary
// tiles, so a valid window is never cut
__global__ __launch_bounds__(kBlock) void k_window_set(LevelDev g, const int32_t *__restrict__ tset,
                                                       int32_t *__restrict__ wset, int rx, int ry, int rz) {
    const int T = blockIdx.x * blockDim.x + threadIdx.x;
    const int ntiles = g.ntx * g.nty * g.ntz;
    if (T >= ntiles) return;
    const int bx = T % g.ntx, r = T / g.ntx, by = r % g.nty, bz = r / g.nty;
    int ks[kWinMax];
    int n = 0;
    bool ok = true;
    for (int z = max(bz - rz, 0); ok && z <= min(bz + rz, g.ntz - 1); ++z)
        for (int y = max(by - ry, 0); ok && y <= min(by + ry, g.nty - 1); ++y)
            for (int x = max(bx - rx, 0); ok && x <= min(bx + rx, g.ntx - 1); ++x) {
                const int32_t *t = tset + (int64_t)(x + g.ntx * (y + g.nty * z)) * (1 + kWinMax);
                const int tn = t[0];
                if (tn < 0) {
                    ok = false;
                    break;
                }
                for (int q = 0; ok && q < tn; ++q) {
                    const int k = t[1 + q];
                    bool have = false;
                    for (int m = 0; m < n; ++m) have = have || ks[m] == k;
                    if (have) continue;
                    if (n == kWinMax)
                        ok = false;
                    else
                        ks[n++] = k;
                }
            }
    int32_t *out = wset + (int64_t)T * (1 + kWinMax);
    out[0] = ok ? n : -1;
    for (int m = 0; m < kWinMax; ++m) out[1 + m] = (ok && m < n) ? ks[m] : 0;
}

void launch_window_set(int dim, const LevelDev &g, const int32_t *tset, int32_t *wset, const int R[3],
                       hipStream_t s) {
    const int tw = 1 << g.tlog, th = kBlock >> g.tlog;
    const int rx = (R[0] + tw - 1) / tw, ry = (R[1] + th - 1) / th, rz = dim == 3 ? R[2] : 0;
    const int ntiles = g.ntx * g.nty * g.ntz;
    hipLaunchKernelGGL(k_window_set, dim3((ntiles + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, tset, wset, rx,
                       ry, rz);
}

// (L^T x)_j on a column whose whole stencil window has control k: sum over the points of the row stencil
// of control k, reflected (x at j - off - delta_c with the weight of corner c), minus the diagonal part,
// in the form of the forward operator (TW: weight table record type)
template <int DIM, typename TC, typename TX, typename TW>
__device__ __forceinline__ TC lt_reflect(const LevelDev &g, const StencilDev &st, const TW *__restrict__ tab, int k,
                                         int j, const TX *__restrict__ x, TC xj) {
    const TW *fp = tab + k * st.npt;
    const int s1 = (int)g.s1, s2 = (int)g.s2;
    auto pt = [&](const TW &p) {
        const int o = j - p.off;
        TC v = (TC)p.w[0] * (TC)x[o];
        v = fma((TC)p.w[1], (TC)x[o - 1], v);
        v = fma((TC)p.w[2], (TC)x[o - s1], v);
        v = fma((TC)p.w[3], (TC)x[o - s1 - 1], v);
        if (DIM == 3) {
            v = fma((TC)p.w[4], (TC)x[o - s2], v);
            v = fma((TC)p.w[5], (TC)x[o - s2 - 1], v);
            v = fma((TC)p.w[6], (TC)x[o - s2 - s1], v);
            v = fma((TC)p.w[7], (TC)x[o - s2 - s1 - 1], v);
        }
        return v;
    };
    if (DIM == 2 && st.P == 1) {
        // one diffusion pair (+ drift): all twelve gathers are issued before any sum (the drift's are read
        // from the pair's stencil when there is no drift point, and unused); sums as in the general loop
        const TW &pa = fp[0], &pb = fp[1], &pc = fp[st.has_drift ? 2 : 0];
        const int oa = j - pa.off, ob = j - pb.off, oc = j - pc.off;
        const TX a0 = x[oa], a1 = x[oa - 1], a2 = x[oa - s1], a3 = x[oa - s1 - 1];
        const TX b0 = x[ob], b1 = x[ob - 1], b2 = x[ob - s1], b3 = x[ob - s1 - 1];
        const TX c0 = x[oc], c1 = x[oc - 1], c2 = x[oc - s1], c3 = x[oc - s1 - 1];
        auto ws4 = [](const TW &p, TX v0, TX v1, TX v2, TX v3) {
            TC v = (TC)p.w[0] * (TC)v0;
            v = fma((TC)p.w[1], (TC)v1, v);
            v = fma((TC)p.w[2], (TC)v2, v);
            return fma((TC)p.w[3], (TC)v3, v);
        };
        TC acc = (TC)0;
        acc = acc + ((ws4(pa, a0, a1, a2, a3) + ws4(pb, b0, b1, b2, b3)) - (TC)2 * xj);
        if (st.has_drift) acc = acc + (TC)2 * (ws4(pc, c0, c1, c2, c3) - xj);
        return (TC)st.inv2h * acc;
    }
    TC acc = (TC)0;
    for (int p = 0; p < st.P; ++p) acc = acc + ((pt(fp[2 * p]) + pt(fp[2 * p + 1])) - (TC)2 * xj);
    if (st.has_drift) acc = acc + (TC)2 * (pt(fp[2 * st.P]) - xj);
    return (TC)st.inv2h * acc;
}

// the window set of this block's tile (n = -1: gather from the listing)
struct WSet {
    int n;
    int k[kWinMax];
};
__device__ __forceinline__ WSet window_set(const TransposeView &T) {
    WSet w;
    w.n = -1;
    if (!T.wset) return w;
    const int32_t *p = T.wset + (int64_t)remap_block_a(blockIdx.x, gridDim.x) * (1 + kWinMax);
    w.n = p[0];
#pragma unroll
    for (int m = 0; m < kWinMax; ++m) w.k[m] = p[1 + m];
    return w;
}

// (L^T x)_j on a column whose stencil window holds the controls w.k[0 .. w.n): for each of them, the rows
// that reach j are those of that control among the reflected row-stencil positions j - off - delta_c
template <int DIM, typename TC, typename TX, typename TW>
__device__ __forceinline__ TC lt_reflect_multi(const LevelDev &g, const StencilDev &st, const TW *__restrict__ tab,
                                               const WSet &w, int j, const TX *__restrict__ x,
                                               const int16_t *__restrict__ alpha, TC xj) {
    const int s1 = (int)g.s1, s2 = (int)g.s2;
    TC acc = (TC)0;
    if (DIM == 2 && st.P == 1) {
        // one diffusion pair (+ drift): per control, the corner controls and values of all its points are
        // requested before any sum (twelve of each; a missing drift point reads the pair's stencil, unused)
        const int npt = st.npt;
        for (int m = 0; m < w.n; ++m) {
            const int k = w.k[m];
            const TW *fp = tab + k * npt;
            int o[3];
            int16_t ac[3][4];
            TX xc[3][4];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                o[q] = j - fp[q < npt ? q : 0].off;
                const int ci[4] = {o[q], o[q] - 1, o[q] - s1, o[q] - s1 - 1};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    ac[q][c] = alpha[ci[c]];
                    xc[q][c] = x[ci[c]];
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (q >= npt) break;
                const TW &p = fp[q];
                auto at = [&](int c) { return ac[q][c] == k ? (TC)xc[q][c] : (TC)0; };
                TC v = (TC)p.w[0] * at(0);
                v = fma((TC)p.w[1], at(1), v);
                v = fma((TC)p.w[2], at(2), v);
                v = fma((TC)p.w[3], at(3), v);
                acc = q < 2 ? acc + v : acc + (TC)2 * v;  // drift point weight 2
            }
        }
        const TC b = (TC)(2 + (st.has_drift ? 2 : 0));
        return (TC)st.inv2h * (acc - b * xj);
    }
    for (int m = 0; m < w.n; ++m) {
        const int k = w.k[m];
        const TW *fp = tab + k * st.npt;
        for (int q = 0; q < st.npt; ++q) {
            const TW &p = fp[q];
            const int o = j - p.off;
            auto at = [&](int i) { return alpha[i] == k ? (TC)x[i] : (TC)0; };
            TC v = (TC)p.w[0] * at(o);
            v = fma((TC)p.w[1], at(o - 1), v);
            v = fma((TC)p.w[2], at(o - s1), v);
            v = fma((TC)p.w[3], at(o - s1 - 1), v);
            if (DIM == 3) {
                v = fma((TC)p.w[4], at(o - s2), v);
                v = fma((TC)p.w[5], at(o - s2 - 1), v);
                v = fma((TC)p.w[6], at(o - s2 - s1), v);
                v = fma((TC)p.w[7], at(o - s2 - s1 - 1), v);
            }
            acc = q < 2 * st.P ? acc + v : acc + (TC)2 * v;  // drift point weight 2
        }
    }
    const TC b = (TC)(2 * st.P + (st.has_drift ? 2 : 0));  // the row's own diagonal part
    return (TC)st.inv2h * (acc - b * xj);
}

// ---- dual numbers ---------------------------------------------------------------------------------

struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual dmk(double v, double d) { return Dual{v, d}; }
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}

// landing of x_i + mu*Y with the forward kernels' rules, carrying d/ds (dY = Y/s for diffusion points)
template <int DIM>
__device__ Dual landing_dual(const LevelDev &g, const int ix[3], const double Y[3], const double dY[3], int cell[3],
                             Dual t[3]) {
    Dual m[3];
    Dual mu = dmk(1.0, 0.0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        m[d] = dmk(__builtin_inf(), 0.0);
        if (Y[d] != 0.0) {
            double D = (double)((Y[d] > 0.0) ? (g.n[d] - 1 - ix[d]) : ix[d]);
            double aY = fabs(Y[d]), daY = Y[d] > 0.0 ? dY[d] : -dY[d];
            m[d] = dmk(D / aY, -D * daY / (aY * aY));
            if (m[d].v < mu.v) mu = m[d];
        }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        int c;
        Dual tt;
        if (mu.v == 1.0) {
            double fl = floor(Y[d]);
            c = ix[d] + (int)fl;
            tt = dmk(Y[d] - fl, dY[d]);
        } else if (Y[d] != 0.0 && m[d].v == mu.v) {
            c = (Y[d] > 0.0) ? g.n[d] - 1 : 0;
            tt = dmk(0.0, 0.0);
        } else {
            Dual q = dmk((double)ix[d], 0.0) + mu * dmk(Y[d], dY[d]);
            double top = (double)(g.n[d] - 1);
            if (q.v < 0.0) q = dmk(0.0, 0.0);
            if (q.v > top) q = dmk(top, 0.0);
            double fl = floor(q.v);
            c = (int)fl;
            tt = dmk(q.v - fl, q.d);
        }
        if (c >= g.n[d] - 1) {
            c = g.n[d] - 2;
            tt = dmk(1.0, 0.0);
        }
        cell[d] = c;
        t[d] = tt;
    }
    return mu;
}

template <int DIM>
__device__ Dual interp_dual(const double *__restrict__ V, const LevelDev &g, const int cell[3], const Dual t[3]) {
    Dual v = dmk(0.0, 0.0);
    const int s1 = (int)g.s1, s2 = (int)g.s2;
    int base = cell[0] + cell[1] * s1 + (DIM == 3 ? cell[2] * s2 : 0);
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        Dual w = (c & 1) ? t[0] : dmk(1.0, 0.0) - t[0];
        w = w * (((c >> 1) & 1) ? t[1] : dmk(1.0, 0.0) - t[1]);
        if (DIM == 3) w = w * (((c >> 2) & 1) ? t[2] : dmk(1.0, 0.0) - t[2]);
        int off = (c & 1) + ((c >> 1) & 1) * s1 + (DIM == 3 ? ((c >> 2) & 1) * s2 : 0);
        v = v + w * dmk(V[base + off], 0.0);
    }
    return v;
}

// d/ds (L-hat^k V)_i (only diffusion points depend on s)
template <int DIM>
__device__ double dlhat_ds(const LevelDev &g, const StencilDev &st, int k, int i, const int ix[3],
                           const double *__restrict__ V, double inv_s) {
    const PointTab *pt = st.tab + k * st.npt;
    double Vi = V[i];
    Dual acc = dmk(0.0, 0.0);
    for (int p = 0; p < st.P; ++p) {
        double Ya[3], Yb[3];
        point_Y(st, pt[2 * p], 2 * p, ix, i, DIM, Ya);
        point_Y(st, pt[2 * p + 1], 2 * p + 1, ix, i, DIM, Yb);
        double dYa[3] = {Ya[0] * inv_s, Ya[1] * inv_s, Ya[2] * inv_s};
        double dYb[3] = {Yb[0] * inv_s, Yb[1] * inv_s, Yb[2] * inv_s};
        int cp[3], cm[3];
        Dual tp[3], tm[3];
        Dual mup = landing_dual<DIM>(g, ix, Ya, dYa, cp, tp);
        Dual mum = landing_dual<DIM>(g, ix, Yb, dYb, cm, tm);
        Dual two = dmk(2.0, 0.0);
        Dual A = two / (mup * (mup + mum));
        Dual B = two / (mum * (mum + mup));
        Dual vp = interp_dual<DIM>(V, g, cp, tp);
        Dual vm = interp_dual<DIM>(V, g, cm, tm);
        acc = acc + ((A * vp + B * vm) - (A + B) * dmk(Vi, 0.0));
    }
    return st.inv2h * acc.d;
}

// partial[b] = block b's part of sum_i mu_i (wa * dL V_a + wb * dL V_b)_i over interior nodes
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ds_dot(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                   const double *__restrict__ mu, const double *__restrict__ Va,
                                                   double wa, const double *__restrict__ Vb, double wb, double inv_s,
                                                   double *__restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    int ix[3];
    int i = tile_node_a<DIM>(g, ix);
    double v = 0.0;
    if (i >= 0 && interior_a<DIM>(g, ix)) {
        int k = alpha[i];
        k = ((unsigned)k < (unsigned)st.K) ? k : 0;
        double d = wa * dlhat_ds<DIM>(g, st, k, i, ix, Va, inv_s);
        if (wb != 0.0) d += wb * dlhat_ds<DIM>(g, st, k, i, ix, Vb, inv_s);
        v = mu[i] * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
        partial[remap_block_a(blockIdx.x, gridDim.x)] = t;
    }
}

void launch_ds_dot(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const double *mu,
                   const double *Va, double wa, const double *Vb, double wb, double inv_s, double *partial,
                   hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_ds_dot<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, mu, Va, wa, Vb, wb, inv_s,
                           partial);
    else
        hipLaunchKernelGGL(k_ds_dot<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, mu, Va, wa, Vb, wb, inv_s,
                           partial);
}

// ---- row listing of L-hat^alpha -------------------------------------------------------------------

// landing without derivatives (the forward rules; duplicated here so this file stands alone)
template <int DIM>
__device__ double landing_plain(const LevelDev &g, const int ix[3], const double Y[3], int cell[3], double t[3]) {
    double m[3];
    double mu = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        m[d] = __builtin_inf();
        if (Y[d] != 0.0) {
            int D = (Y[d] > 0.0) ? (g.n[d] - 1 - ix[d]) : ix[d];
            m[d] = (double)D / fabs(Y[d]);
            if (m[d] < mu) mu = m[d];
        }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        int c;
        double tt;
        if (mu == 1.0) {
            double fl = floor(Y[d]);
            c = ix[d] + (int)fl;
            tt = Y[d] - fl;
        } else if (Y[d] != 0.0 && m[d] == mu) {
            c = (Y[d] > 0.0) ? g.n[d] - 1 : 0;
            tt = 0.0;
        } else {
            double q = (double)ix[d] + mu * Y[d];
            double top = (double)(g.n[d] - 1);
            q = q < 0.0 ? 0.0 : (q > top ? top : q);
            double fl = floor(q);
            c = (int)fl;
            tt = q - fl;
        }
        if (c >= g.n[d] - 1) {
            c = g.n[d] - 2;
            tt = 1.0;
        }
        cell[d] = c;
        t[d] = tt;
    }
    return mu;
}

// slots [i*E, (i+1)*E): for each stencil point its 2^d corners (weight * corner weight / 2h), then the
// diagonal -(sum of weights)/2h.  Boundary rows get the sentinel column N.  Weights are stored by slot, the
// columns entry-major (entry e of row i at e * N + i) for the coalesced passes of the column sort.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_emit_rows(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                      int E, int32_t *__restrict__ cols, double *__restrict__ vals) {
    int ix[3];
    int i = tile_node_a<DIM>(g, ix);
    if (i < 0) return;
    int64_t base = (int64_t)i * E;
    if (!interior_a<DIM>(g, ix)) {
        for (int e = 0; e < E; ++e) {
            cols[(int64_t)e * g.N + i] = (int32_t)g.N;
            vals[base + e] = 0.0;
        }
        return;
    }
    int k = alpha[i];
    k = ((unsigned)k < (unsigned)st.K) ? k : 0;
    const PointTab *pt = st.tab + k * st.npt;
    int e = 0;
    double diag = 0.0;
    for (int q = 0; q < st.npt; ++q) {
        double Y[3];
        point_Y(st, pt[q], q, ix, i, DIM, Y);
        int cell[3];
        double t[3];
        double mu = landing_plain<DIM>(g, ix, Y, cell, t);
        double W;
        if (q < 2 * st.P) {
            double Yo[3];
            point_Y(st, pt[q ^ 1], q ^ 1, ix, i, DIM, Yo);
            int co[3];
            double to[3];
            double muo = landing_plain<DIM>(g, ix, Yo, co, to);
            W = 2.0 / (mu * (mu + muo));
        } else {
            W = 2.0 / mu;
        }
        double Ws = W * st.inv2h;
        const int s1 = (int)g.s1, s2 = (int)g.s2;
        int cb = cell[0] + cell[1] * s1 + (DIM == 3 ? cell[2] * s2 : 0);
        for (int c = 0; c < (1 << DIM); ++c) {
            double w = (c & 1) ? t[0] : (1.0 - t[0]);
            w = w * (((c >> 1) & 1) ? t[1] : (1.0 - t[1]));
            if (DIM == 3) w = w * (((c >> 2) & 1) ? t[2] : (1.0 - t[2]));
            int off = (c & 1) + ((c >> 1) & 1) * s1 + (DIM == 3 ? ((c >> 2) & 1) * s2 : 0);
            cols[(int64_t)e * g.N + i] = cb + off;
            vals[base + e] = Ws * w;
            ++e;
        }
        diag -= Ws;
    }
    cols[(int64_t)e * g.N + i] = i;
    vals[base + e] = diag;
    ++e;
    for (; e < E; ++e) {
        cols[(int64_t)e * g.N + i] = (int32_t)g.N;
        vals[base + e] = 0.0;
    }
}

// ---- column-sorted listing: counting sort by column, stable in slot order --------------------------------
// Slot p = i * E + e of the row listing holds entry e of row i.  The listing sorted by column keeps, within a
// column, the slot order (increasing row), so every sum over a column's entries runs in one fixed order.
// The sentinel column N (boundary rows, unused slots) is not listed.

// Threads take the entries entry-major (thread q: entry q / N of row q % N, as the columns are stored), so a
// wavefront's atomics go to the distinct columns of consecutive rows rather than to the columns one row's
// entries share with its neighbours'.
__device__ __forceinline__ int64_t entry_major_slot(int64_t q, int64_t rows, int E) {
    const int64_t e = q / rows;
    return (q - e * rows) * E + e;
}

__global__ __launch_bounds__(kBlock) void k_col_count(const int32_t *__restrict__ cols, int64_t n, int E, int32_t N,
                                                      int32_t *__restrict__ cnt) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const int32_t c = cols[q];
    if (c < N) atomicAdd(&cnt[c], 1);
}

__global__ __launch_bounds__(kBlock) void k_copy_i32(const int32_t *__restrict__ a, int32_t *__restrict__ b,
                                                     int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n) b[p] = a[p];
}

// cursor starts as the column starts; each listed slot takes the next free place of its column
__global__ __launch_bounds__(kBlock) void k_col_scatter(const int32_t *__restrict__ cols, int64_t n, int E, int32_t N,
                                                        int32_t *__restrict__ cursor, int32_t *__restrict__ slot_s) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const int32_t c = cols[q];
    if (c < N) slot_s[atomicAdd(&cursor[c], 1)] = (int32_t)entry_major_slot(q, n / E, E);
}

// The places a column's slots took depend on the order of the atomics: each column's slots are put back in
// increasing order.  Columns of at most kShortCol entries (almost all) are sorted in registers by one thread
// (odd-even transposition network); longer ones (next to the boundary, where truncated landings gather) are
// appended to a list and sorted by one block each.
constexpr int kShortCol = 16, kLongColLds = 8192;

__global__ __launch_bounds__(kBlock) void k_col_order(const int32_t *__restrict__ colptr, int32_t N,
                                                      int32_t *__restrict__ slot_s, int32_t *__restrict__ long_list,
                                                      int32_t *__restrict__ long_count) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= N) return;
    const int32_t a = colptr[j], len = colptr[j + 1] - a;
    if (len <= 1) return;
    if (len > kShortCol) {
        long_list[atomicAdd(long_count, 1)] = (int32_t)j;
        return;
    }
    int32_t v[kShortCol];
#pragma unroll
    for (int q = 0; q < kShortCol; ++q) v[q] = q < len ? slot_s[a + q] : INT32_MAX;
#pragma unroll
    for (int r = 0; r < kShortCol; ++r)
#pragma unroll
        for (int q = r & 1; q + 1 < kShortCol; q += 2)
            if (v[q] > v[q + 1]) {
                const int32_t t = v[q];
                v[q] = v[q + 1];
                v[q + 1] = t;
            }
#pragma unroll
    for (int q = 0; q < kShortCol; ++q)
        if (q < len) slot_s[a + q] = v[q];
}

// one block per listed long column (the grid strides over the list): each entry's place is the number of
// smaller entries of its column (the slots are distinct)
__global__ __launch_bounds__(kBlock) void k_col_order_long(const int32_t *__restrict__ colptr,
                                                           int32_t *__restrict__ slot_s,
                                                           const int32_t *__restrict__ long_list,
                                                           const int32_t *__restrict__ long_count) {
    __shared__ int32_t sh[kLongColLds];
    const int32_t cnt = long_count[0];
    for (int32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const int32_t j = long_list[q];
        const int32_t a = colptr[j], len = colptr[j + 1] - a;
        if (len <= kLongColLds) {
            for (int32_t t = threadIdx.x; t < len; t += blockDim.x) sh[t] = slot_s[a + t];
            __syncthreads();
            for (int32_t t = threadIdx.x; t < len; t += blockDim.x) {
                const int32_t v = sh[t];
                int32_t rank = 0;
                for (int32_t u = 0; u < len; ++u) rank += sh[u] < v ? 1 : 0;
                slot_s[a + rank] = v;
            }
        } else if (threadIdx.x == 0) {
            // beyond the shared-memory copy: insertion sort in place
            for (int32_t p = a + 1; p < a + len; ++p) {
                const int32_t v = slot_s[p];
                int32_t r = p - 1;
                while (r >= a && slot_s[r] > v) {
                    slot_s[r + 1] = slot_s[r];
                    --r;
                }
                slot_s[r + 1] = v;
            }
        }
        __syncthreads();
    }
}

// rows and weights of the listed entries in column order
__global__ __launch_bounds__(kBlock) void k_col_fill(const int32_t *__restrict__ slot_s, const int32_t *__restrict__ total,
                                                     int64_t n, int E, const double *__restrict__ vals,
                                                     double *__restrict__ vals_s, int32_t *__restrict__ rows_s) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n || p >= total[0]) return;
    const int32_t id = slot_s[p];
    vals_s[p] = vals[id];
    rows_s[p] = id / E;
}

// ---- exclusive prefix sums of int32 counts ---------------------------------------------------------------
constexpr int kScanThreads = 1024, kScanItems = 4;
constexpr int kScanChunk = kScanThreads * kScanItems;

// block-wide exclusive scan of one value per thread; returns the block total through *total
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *sh, int32_t *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    __syncthreads();
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            const int32_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[kScanThreads / 64] = run;
    }
    __syncthreads();
    *total = sh[kScanThreads / 64];
    return sh[wid] + x - v;
}

// out[q] = sum of in[0..q) within each chunk of kScanChunk entries; part[b] = total of chunk b
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int32_t *__restrict__ in, int64_t m,
                                                             int32_t *__restrict__ out, int32_t *__restrict__ part) {
    __shared__ int32_t sh[kScanThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems], s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < m ? in[base + q] : 0;
        s += v[q];
    }
    int32_t total;
    int32_t run = block_exclusive_scan(s, sh, &total);
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < m) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// part[0..nb) -> exclusive prefix sums in place (one block, chunk by chunk); *total_out = the sum of all
__global__ __launch_bounds__(kScanThreads) void k_scan_parts(int32_t *__restrict__ part, int nb, int32_t *total_out) {
    __shared__ int32_t sh[kScanThreads / 64 + 1];
    int32_t carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int q = c0 + (int)threadIdx.x;
        const int32_t v = q < nb ? part[q] : 0;
        int32_t total;
        const int32_t ex = block_exclusive_scan(v, sh, &total);
        if (q < nb) part[q] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t *__restrict__ out, int64_t m,
                                                           const int32_t *__restrict__ part) {
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    const int32_t add = part[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < m) out[base + q] += add;
}

// out[q] = in[0] + ... + in[q-1] for q < m, and *total_out (nullable) = the sum of all m; part holds
// scan_parts(m) entries
int64_t scan_parts(int64_t m) { return (m + kScanChunk - 1) / kScanChunk; }
void exclusive_scan(const int32_t *in, int64_t m, int32_t *out, int32_t *part, int32_t *total_out, hipStream_t s) {
    const int nb = (int)std::max<int64_t>(1, scan_parts(m));
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanThreads), 0, s, in, m, out, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanThreads), 0, s, part, nb, total_out);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, s, out, m, (const int32_t *)part);
}

// slice widths: longest column of each wavefront's 64 nodes, capped at kEllCap
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ell_width(LevelDev g, const int32_t *__restrict__ colptr,
                                                      int32_t *__restrict__ width) {
    int ix[3];
    int j = tile_node_a<DIM>(g, ix);
    int cnt = j >= 0 ? colptr[j + 1] - colptr[j] : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt = max(cnt, __shfl_xor(cnt, off, 64));
    if ((threadIdx.x & 63) == 0)
        width[(int64_t)remap_block_a(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6)] = min(cnt, kEllCap);
}

// lane l of a slice copies its column's first `width` entries (zero weight on the node itself past its count)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ell_fill(LevelDev g, const int32_t *__restrict__ colptr,
                                                     const int32_t *__restrict__ rows_s,
                                                     const double *__restrict__ vals_s,
                                                     const int32_t *__restrict__ width, const int32_t *__restrict__ soff,
                                                     int32_t *__restrict__ ell_rows, double *__restrict__ ell_vals,
                                                     float *__restrict__ ell_vals32, int16_t *__restrict__ ell_d16) {
    int ix[3];
    int j = tile_node_a<DIM>(g, ix);
    int64_t sl = (int64_t)remap_block_a(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
    int W = width[sl];
    int64_t base = (int64_t)soff[sl] * 64 + (threadIdx.x & 63);
    int p0 = j >= 0 ? colptr[j] : 0;
    int cnt = j >= 0 ? colptr[j + 1] - p0 : 0;
    int self = j >= 0 ? j : 0;
    const int s1 = (int)g.s1;
    for (int q = 0; q < W; ++q) {
        bool real = q < cnt;
        int row = real ? rows_s[p0 + q] : self;
        double v = real ? vals_s[p0 + q] : 0.0;
        ell_rows[base + (int64_t)q * 64] = row;
        ell_vals[base + (int64_t)q * 64] = v;
        if (ell_vals32) ell_vals32[base + (int64_t)q * 64] = (float)v;
        if (DIM == 2 && ell_d16) {
            int dx = j >= 0 ? row % s1 - ix[0] : 0;
            int dy = j >= 0 ? row / s1 - ix[1] : 0;
            ell_d16[base + (int64_t)q * 64] = (int16_t)((dx & 0xff) | (dy << 8));
        }
    }
}

// Row listing of level g's operator for policy alpha, its column-sorted (CSC) form and the sliced ELL copy.
int build_transpose(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, int E, TransposeBuf &b,
                    hipStream_t s) {
    int64_t n = g.N * (int64_t)E;
    const int nt = tiles_for(g);
    if (dim == 2)
        hipLaunchKernelGGL(k_emit_rows<2>, dim3(nt), dim3(kBlock), 0, s, g, st, alpha, E, b.cols, b.vals);
    else
        hipLaunchKernelGGL(k_emit_rows<3>, dim3(nt), dim3(kBlock), 0, s, g, st, alpha, E, b.cols, b.vals);
    // column starts by counting sort: counts, their prefix sums (colptr[N] = listed entries), scatter, order
    const unsigned gb = (unsigned)((n + kBlock - 1) / kBlock);
    int32_t *part = (int32_t *)b.scratch;
    launch_zero(b.cols_s, (size_t)g.N * 4, s);
    hipLaunchKernelGGL(k_col_count, dim3(gb), dim3(kBlock), 0, s, b.cols, n, E, (int32_t)g.N, b.cols_s);
    exclusive_scan(b.cols_s, g.N, b.colptr, part, b.colptr + g.N, s);
    hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)((g.N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const int32_t *)b.colptr, b.cols_s, g.N);
    hipLaunchKernelGGL(k_col_scatter, dim3(gb), dim3(kBlock), 0, s, b.cols, n, E, (int32_t)g.N, b.cols_s,
                       b.ids_s);
    // the cursor array is free again: it takes the list of long columns, counted behind the partial sums
    int32_t *long_count = part + scan_parts(std::max<int64_t>(g.N, ell_slices(g)));
    launch_zero(long_count, 4, s);
    hipLaunchKernelGGL(k_col_order, dim3((unsigned)((g.N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const int32_t *)b.colptr, (int32_t)g.N, b.ids_s, b.cols_s, long_count);
    hipLaunchKernelGGL(k_col_order_long, dim3(1024), dim3(kBlock), 0, s, (const int32_t *)b.colptr, b.ids_s,
                       (const int32_t *)b.cols_s, (const int32_t *)long_count);
    hipLaunchKernelGGL(k_col_fill, dim3(gb), dim3(kBlock), 0, s, (const int32_t *)b.ids_s,
                       (const int32_t *)(b.colptr + g.N), n, E, (const double *)b.vals, b.vals_s, b.rows_s);
    const int64_t ns = ell_slices(g);
    if (dim == 2)
        hipLaunchKernelGGL(k_ell_width<2>, dim3(nt), dim3(kBlock), 0, s, g, b.colptr, b.ell_w);
    else
        hipLaunchKernelGGL(k_ell_width<3>, dim3(nt), dim3(kBlock), 0, s, g, b.colptr, b.ell_w);
    exclusive_scan(b.ell_w, ns, b.ell_off, part, nullptr, s);
    if (dim == 2)
        hipLaunchKernelGGL(k_ell_fill<2>, dim3(nt), dim3(kBlock), 0, s, g, b.colptr, b.rows_s, b.vals_s, b.ell_w,
                           b.ell_off, b.ell_rows, b.ell_vals, b.ell_vals32, b.ell_d16);
    else
        hipLaunchKernelGGL(k_ell_fill<3>, dim3(nt), dim3(kBlock), 0, s, g, b.colptr, b.rows_s, b.vals_s, b.ell_w,
                           b.ell_off, b.ell_rows, b.ell_vals, b.ell_vals32, b.ell_d16);
    return 0;
}

size_t transpose_scratch_bytes(int64_t n, int N, int nslices) {
    (void)n;
    return (size_t)(scan_parts(std::max<int64_t>(N, nslices)) + 1) * 4;  // partial sums, long-column count
}

// (L^T x)_j over the interior rows that reference column j, in increasing row order: the slice's
// ELL entries, then the column's entries past the cap.
template <typename TX>
__device__ __forceinline__ double lt_gather(int j, const TransposeView &T, const TX *__restrict__ x) {
    const int64_t sl = (int64_t)remap_block_a(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
    const int W = T.ell_w[sl];
    const int32_t *__restrict__ er = T.ell_rows + (int64_t)T.ell_off[sl] * 64 + (threadIdx.x & 63);
    const double *__restrict__ ev = T.ell_vals + (int64_t)T.ell_off[sl] * 64 + (threadIdx.x & 63);
    double acc = 0.0;
    int q = 0;
    for (; q + 8 <= W; q += 8) {
        int r[8];
        double v[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = er[(q + u) * 64];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ev[(q + u) * 64];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = (double)x[r[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u] * xv[u];
    }
    for (; q + 4 <= W; q += 4) {
        const int r0 = er[q * 64], r1 = er[(q + 1) * 64], r2 = er[(q + 2) * 64], r3 = er[(q + 3) * 64];
        const double v0 = ev[q * 64], v1 = ev[(q + 1) * 64], v2 = ev[(q + 2) * 64], v3 = ev[(q + 3) * 64];
        const double x0 = (double)x[r0], x1 = (double)x[r1], x2 = (double)x[r2], x3 = (double)x[r3];
        acc += v0 * x0;
        acc += v1 * x1;
        acc += v2 * x2;
        acc += v3 * x3;
    }
    for (; q < W; ++q) acc += ev[q * 64] * (double)x[er[q * 64]];
    const int p1 = T.colptr[j + 1];
    for (int p = T.colptr[j] + W; p < p1; ++p) acc += T.vals[p] * (double)x[T.rows[p]];
    return acc;
}

// FP32 gather of the preconditioner (same entries and order, float weights and accumulation); the
// loads of four entries are issued before their products are accumulated
template <bool PACKED>
__device__ __forceinline__ float lt_gather32(int j, int s1, const TransposeView &T, const float *__restrict__ x) {
    const int64_t sl = (int64_t)remap_block_a(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
    const int W = T.ell_w[sl];
    const int64_t base = (int64_t)T.ell_off[sl] * 64 + (threadIdx.x & 63);
    const float *__restrict__ ev = T.ell_vals32 + base;
    const int16_t *__restrict__ ed = T.ell_d16 + base;
    const int32_t *__restrict__ er = T.ell_rows + base;
    auto row = [&](int q) -> int {
        if (PACKED) {
            int c = ed[q * 64];
            return j + (int)(int8_t)(c & 0xff) + (c >> 8) * s1;
        }
        return er[q * 64];
    };
    float acc = 0.0f;
    int q = 0;
    for (; q + 8 <= W; q += 8) {
        int r[8];
        float v[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = row(q + u);
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ev[(q + u) * 64];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = x[r[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u] * xv[u];
    }
    for (; q + 4 <= W; q += 4) {
        const int r0 = row(q), r1 = row(q + 1), r2 = row(q + 2), r3 = row(q + 3);
        const float v0 = ev[q * 64], v1 = ev[(q + 1) * 64], v2 = ev[(q + 2) * 64], v3 = ev[(q + 3) * 64];
        const float x0 = x[r0], x1 = x[r1], x2 = x[r2], x3 = x[r3];
        acc += v0 * x0;
        acc += v1 * x1;
        acc += v2 * x2;
        acc += v3 * x3;
    }
    for (; q < W; ++q) acc += ev[q * 64] * x[row(q)];
    const int p1 = T.colptr[j + 1];
    for (int p = T.colptr[j] + W; p < p1; ++p) acc += (float)T.vals[p] * x[T.rows[p]];
    return acc;
}

// mode 0: y = A^T x = x - theta dt (L^T x + c x) on interior nodes, 0 on the boundary
// mode 1: y = B^T x = [interior] (x + (1-theta) dt c x) + (1-theta) dt L^T x on every node
// mode 2: r = b - A^T x on interior nodes (0 on the boundary), partials [sum r^2, max|r|, max|x|]
// mode 3: r = b - A^T x on interior nodes (0 on the boundary), no partials
template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_apply_T(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                    TransposeView T, const double *__restrict__ x,
                                                    const double *__restrict__ b, double w, double *__restrict__ y,
                                                    double *partial) {
    __shared__ double sh[kBlock / 64];
    int ix[3];
    int j = tile_node_a<DIM>(g, ix);
    double rr = 0.0, xx = 0.0;
    if (j >= 0) {
        bool in = interior_a<DIM>(g, ix);
        double cj = 0.0;
        if (in && st.c) {
            int k = alpha[j];
            cj = st.c[((unsigned)k < (unsigned)st.K) ? k : 0];
        }
        double lt = lt_gather<double>(j, T, x);
        double xj = x[j];
        if (MODE == 0) {
            y[j] = in ? xj - w * (lt + cj * xj) : 0.0;
        } else if (MODE == 1) {
            y[j] = (in ? xj + w * cj * xj : 0.0) + w * lt;
        } else {
            double r = in ? b[j] - (xj - w * (lt + cj * xj)) : 0.0;
            y[j] = r;
            rr = r;
            xx = fabs(xj);
        }
    }
    if (MODE == 2) {
        double v2 = rr * rr, vm = fabs(rr), vx = xx;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            v2 += __shfl_down(v2, off, 64);
            vm = fmax(vm, __shfl_down(vm, off, 64));
            vx = fmax(vx, __shfl_down(vx, off, 64));
        }
        __shared__ double sm[kBlock / 64], sx[kBlock / 64];
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            sh[threadIdx.x >> 6] = v2;
            sm[threadIdx.x >> 6] = vm;
            sx[threadIdx.x >> 6] = vx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, m = 0.0, q = 0.0;
            for (int t = 0; t < kBlock / 64; ++t) {
                a += sh[t];
                m = fmax(m, sm[t]);
                q = fmax(q, sx[t]);
            }
            int bb = remap_block_a(blockIdx.x, gridDim.x);
            partial[bb] = a;
            partial[gridDim.x + bb] = m;
            partial[2 * gridDim.x + bb] = q;
        }
    }
}

void launch_apply_T(int dim, int mode, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                    const TransposeView &T, const double *x, const double *b, double w, double *y, double *partial,
                    hipStream_t s) {
#define AT(D, M) hipLaunchKernelGGL((k_apply_T<D, M>), dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, T, x, b, \
                                    w, y, partial)
    if (dim == 2) {
        if (mode == 0) AT(2, 0); else if (mode == 1) AT(2, 1); else if (mode == 2) AT(2, 2); else AT(2, 3);
    } else {
        if (mode == 0) AT(3, 0); else if (mode == 1) AT(3, 1); else if (mode == 2) AT(3, 2); else AT(3, 3);
    }
#undef AT
}

// Damped Jacobi sweep on A^T e = r: y = x + omega (r - A^T x) / d (interior; 0 on the boundary).
// FIRST: x = 0, so y = omega r / d without gathers.
template <int DIM, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_jacobi_T(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                     TransposeView T, const double *__restrict__ x,
                                                     const double *__restrict__ r, const double *__restrict__ d,
                                                     double theta_dt, double omega, double *__restrict__ y) {
    int ix[3];
    int j = tile_node_a<DIM>(g, ix);
    if (j < 0) return;
    if (!interior_a<DIM>(g, ix)) {
        y[j] = 0.0;
        return;
    }
    if (FIRST) {
        y[j] = omega * r[j] / d[j];
        return;
    }
    const double xj = x[j], rj = r[j], dj = d[j];  // requested before the column gathers
    double cj = 0.0;
    if (st.c) {
        int k = alpha[j];
        cj = st.c[((unsigned)k < (unsigned)st.K) ? k : 0];
    }
    double lt = lt_gather<double>(j, T, x);
    double res = rj - (xj - theta_dt * (lt + cj * xj));
    y[j] = xj + omega * res / dj;
}

void launch_jacobi_T(int dim, bool first, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                     const TransposeView &T, const double *x, const double *r, const double *d, double theta_dt,
                     double omega, double *y, hipStream_t s) {
#define JT(D, F) hipLaunchKernelGGL((k_jacobi_T<D, F>), dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, T, x, r, \
                                    d, theta_dt, omega, y)
    if (dim == 2) {
        if (first) JT(2, true); else JT(2, false);
    } else {
        if (first) JT(3, true); else JT(3, false);
    }
#undef JT
}

// y += a * x (interior nodes only) for the f-gradients
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_axpy_interior(LevelDev g, double a, const double *__restrict__ x,
                                                          double *__restrict__ y) {
    int ix[3];
    int i = tile_node_a<DIM>(g, ix);
    if (i < 0 || !interior_a<DIM>(g, ix)) return;
    y[i] += a * x[i];
}

void launch_axpy_interior(int dim, const LevelDev &g, double a, const double *x, double *y, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_axpy_interior<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, a, x, y);
    else
        hipLaunchKernelGGL(k_axpy_interior<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, a, x, y);
}

// y = x on interior nodes, 0 on the boundary
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_mask_interior(LevelDev g, const double *__restrict__ x,
                                                          double *__restrict__ y) {
    int ix[3];
    int i = tile_node_a<DIM>(g, ix);
    if (i < 0) return;
    y[i] = interior_a<DIM>(g, ix) ? x[i] : 0.0;
}

void launch_mask_interior(int dim, const LevelDev &g, const double *x, double *y, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_mask_interior<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, x, y);
    else
        hipLaunchKernelGGL(k_mask_interior<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, x, y);
}


// y = A^T x with an FP32 x (the preconditioned basis vectors of the mixed mode), FP64 weights and output
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_apply_T_f32x(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                         TransposeView T, const float *__restrict__ x, double w,
                                                         double *__restrict__ y) {
    int ix[3];
    int j = tile_node_a<DIM>(g, ix);
    if (j < 0) return;
    if (!interior_a<DIM>(g, ix)) {
        y[j] = 0.0;
        return;
    }
    const WSet ws = window_set(T);
    double xj = (double)x[j];
    double cj = 0.0;
    if (st.c) {
        int k = alpha[j];
        cj = st.c[((unsigned)k < (unsigned)st.K) ? k : 0];
    }
    double lt;
    if (ws.n == 1)
        lt = lt_reflect<DIM, double>(g, st, st.fastD, ws.k[0], j, x, xj);
    else if (ws.n > 1)
        lt = lt_reflect_multi<DIM, double>(g, st, st.fastD, ws, j, x, alpha, xj);
    else
        lt = lt_gather<float>(j, T, x);
    y[j] = xj - w * (lt + cj * xj);
}

void launch_apply_T_f32x(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                         const TransposeView &T, const float *x, double w, double *y, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_apply_T_f32x<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, T, x, w, y);
    else
        hipLaunchKernelGGL(k_apply_T_f32x<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, T, x, w, y);
}

template <int DIM>
__device__ __forceinline__ float coef32(const StencilDev &st, const int16_t *__restrict__ alpha, int j) {
    if (!st.c) return 0.0f;
    int k = alpha[j];
    return (float)st.c[((unsigned)k < (unsigned)st.K) ? k : 0];
}

// FP32 damped Jacobi sweep on A^T e = r (see k_jacobi_T)
template <int DIM, bool FIRST, bool PACKED>
__global__ __launch_bounds__(kBlock) void k_jacobi_T32(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                       TransposeView T, const float *__restrict__ x,
                                                       const float *__restrict__ r, const float *__restrict__ d,
                                                       float theta_dt, float omega, float *__restrict__ y) {
    int ix[3];
    int j = tile_node_a<DIM>(g, ix);
    if (j < 0) return;
    if (!interior_a<DIM>(g, ix)) {
        y[j] = 0.0f;
        return;
    }
    if (FIRST) {
        y[j] = omega * r[j] / d[j];
        return;
    }
    // the node's own operands are requested before the column gathers, so that their latency overlaps
    const float xj = x[j], rj = r[j], dj = d[j];
    const WSet ws = window_set(T);
    float lt, cj;
    if (ws.n == 1) {
        lt = lt_reflect<DIM, float>(g, st, st.fastF, ws.k[0], j, x, xj);
        cj = st.c ? (float)st.c[ws.k[0]] : 0.0f;
    } else {
        lt = ws.n > 1 ? lt_reflect_multi<DIM, float>(g, st, st.fastF, ws, j, x, alpha, xj)
                      : lt_gather32<PACKED>(j, (int)g.s1, T, x);
        cj = coef32<DIM>(st, alpha, j);
    }
    float res = rj - (xj - theta_dt * (lt + cj * xj));
    y[j] = xj + omega * res / dj;
}

void launch_jacobi_T32(int dim, bool first, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                       const TransposeView &T, const float *x, const float *r, const float *d, double theta_dt,
                       double omega, float *y, hipStream_t s) {
    const bool pk = T.ell_d16 != nullptr && dim == 2;
    const float td = (float)theta_dt, om = (float)omega;
#define J32(D, F, P) hipLaunchKernelGGL((k_jacobi_T32<D, F, P>), dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, \
                                        T, x, r, d, td, om, y)
    if (dim == 2) {
        if (first) J32(2, true, false);
        else if (pk) J32(2, false, true);
        else J32(2, false, false);
    } else {
        if (first) J32(3, true, false); else J32(3, false, false);
    }
#undef J32
}

// FP32 residual y = b - A^T x (interior; 0 on the boundary)
template <int DIM, bool PACKED>
__global__ __launch_bounds__(kBlock) void k_resid_T32(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                      TransposeView T, const float *__restrict__ x,
                                                      const float *__restrict__ b, float theta_dt,
                                                      float *__restrict__ y) {
    int ix[3];
    int j = tile_node_a<DIM>(g, ix);
    if (j < 0) return;
    if (!interior_a<DIM>(g, ix)) {
        y[j] = 0.0f;
        return;
    }
    const float xj = x[j], bj = b[j];  // requested before the column gathers
    const WSet ws = window_set(T);
    float lt, cj;
    if (ws.n == 1) {
        lt = lt_reflect<DIM, float>(g, st, st.fastF, ws.k[0], j, x, xj);
        cj = st.c ? (float)st.c[ws.k[0]] : 0.0f;
    } else {
        lt = ws.n > 1 ? lt_reflect_multi<DIM, float>(g, st, st.fastF, ws, j, x, alpha, xj)
                      : lt_gather32<PACKED>(j, (int)g.s1, T, x);
        cj = coef32<DIM>(st, alpha, j);
    }
    y[j] = bj - (xj - theta_dt * (lt + cj * xj));
}

void launch_resid_T32(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const TransposeView &T,
                      const float *x, const float *b, double theta_dt, float *y, hipStream_t s) {
    const bool pk = T.ell_d16 != nullptr && dim == 2;
    const float td = (float)theta_dt;
    if (dim == 2) {
        if (pk)
            hipLaunchKernelGGL((k_resid_T32<2, true>), dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, T, x, b, td, y);
        else
            hipLaunchKernelGGL((k_resid_T32<2, false>), dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, T, x, b, td,
                               y);
    } else {
        hipLaunchKernelGGL((k_resid_T32<3, false>), dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, T, x, b, td, y);
    }
}

}  // namespace slhjb
