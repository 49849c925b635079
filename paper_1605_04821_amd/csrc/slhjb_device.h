// Device functions shared by the node kernels of libslhjb (single-instance and batched launches):
// tile mapping, landing of stencil points with truncation (Prop. pro:scheme2), multilinear
// interpolation (eq. monotone_int), the operator L-hat (eq. TruncScheme), block reductions and the
// search quantity G_k (eq. nonlinear_sys).
#pragma once

#include <type_traits>

#include "slhjb_internal.h"

namespace slhjb {

__device__ __forceinline__ int remap_block(int b, int nb) {
    int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

__device__ __forceinline__ int node_id() { return remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; }

// Node of this thread: blocks cover 2^tlog x (256 / 2^tlog) tiles (x fastest, then y, then z), so that the stencil
// rows gathered by vertically adjacent nodes are shared in cache.  Returns -1 outside the grid.
template <int DIM>
__device__ __forceinline__ int tile_node_at(const LevelDev &g, int b, int ix[3]) {
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
__device__ __forceinline__ int tile_node(const LevelDev &g, int ix[3]) {
    return tile_node_at<DIM>(g, remap_block(blockIdx.x, gridDim.x), ix);
}

// the wave-control table entry of this thread's wavefront (-1 without a table), read through the scalar unit
__device__ __forceinline__ int wave_control(const int16_t *__restrict__ wctl, int tile) {
    return wctl ? (int)wctl[tile * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)] : -1;
}

template <int DIM>
__device__ __forceinline__ void unflatten(const LevelDev &g, int i, int ix[3]) {
    if (DIM == 2) {
        ix[1] = i / g.n[0];
        ix[0] = i - ix[1] * g.n[0];
        ix[2] = 0;
    } else {
        int r = i / g.n[0];
        ix[0] = i - r * g.n[0];
        ix[2] = r / g.n[1];
        ix[1] = r - ix[2] * g.n[1];
    }
}

template <int DIM>
__device__ __forceinline__ bool interior(const LevelDev &g, const int ix[3]) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ok = ok && ix[d] > 0 && ix[d] < g.n[d] - 1;
    return ok;
}

template <int DIM>
__device__ __forceinline__ bool deep_node(const LevelDev &g, const int ix[3]) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ok = ok && ix[d] >= g.deep_lo[d] && ix[d] <= g.deep_hi[d];
    return ok;
}

// ---- landing of a (possibly truncated) stencil point -------------------------------------------

template <int DIM>
__device__ __forceinline__ double landing(const LevelDev &g, const int ix[3], const double Y[3], int cell[3],
                                          double t[3]) {
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
            q = q < 0.0 ? 0.0 : q;
            double top = (double)(g.n[d] - 1);
            q = q > top ? top : q;
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

// The landing rules of landing() in FP32 with approximate reciprocals, for the FP32 multigrid kernels only:
// those kernels precondition the FP64 Krylov solve, so the operator they apply may differ from the FP64 one
// by rounding (near a tie of the rules, by the landing cell chosen).
template <int DIM>
__device__ __forceinline__ float landing_f(const LevelDev &g, const int ix[3], const float Y[3], int cell[3],
                                           float t[3]) {
    float m[3];
    float mu = 1.0f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        m[d] = __builtin_inff();
        if (Y[d] != 0.0f) {
            const int D = (Y[d] > 0.0f) ? (g.n[d] - 1 - ix[d]) : ix[d];
            m[d] = (float)D * __builtin_amdgcn_rcpf(fabsf(Y[d]));
            if (m[d] < mu) mu = m[d];
        }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        int c;
        float tt;
        if (mu == 1.0f) {
            const float fl = floorf(Y[d]);
            c = ix[d] + (int)fl;
            tt = Y[d] - fl;
        } else if (Y[d] != 0.0f && m[d] == mu) {
            c = (Y[d] > 0.0f) ? g.n[d] - 1 : 0;
            tt = 0.0f;
        } else {
            float q = (float)ix[d] + mu * Y[d];
            q = q < 0.0f ? 0.0f : q;
            const float top = (float)(g.n[d] - 1);
            q = q > top ? top : q;
            const float fl = floorf(q);
            c = (int)fl;
            tt = q - fl;
        }
        if (c >= g.n[d] - 1) {
            c = g.n[d] - 2;
            tt = 1.0f;
        }
        if (c < 0) c = 0;
        cell[d] = c;
        t[d] = tt;
    }
    return mu;
}

__device__ __forceinline__ double fmat(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return fmaf(a, b, c); }

// weighted sum over the 2^DIM corners of the cell at `base` (eq. monotone_int); TS storage, TC arithmetic
template <int DIM, typename TS, typename TC>
__device__ __forceinline__ TC interp_w(const TS *__restrict__ V, int base, const LevelDev &g, const TC w[8]) {
    const int s1 = (int)g.s1;
    TC v = w[0] * (TC)V[base];
    v = fmat(w[1], (TC)V[base + 1], v);
    v = fmat(w[2], (TC)V[base + s1], v);
    v = fmat(w[3], (TC)V[base + s1 + 1], v);
    if (DIM == 3) {
        const int s2 = (int)g.s2;
        v = fmat(w[4], (TC)V[base + s2], v);
        v = fmat(w[5], (TC)V[base + s2 + 1], v);
        v = fmat(w[6], (TC)V[base + s2 + s1], v);
        v = fmat(w[7], (TC)V[base + s2 + s1 + 1], v);
    }
    return v;
}

template <typename TC>
struct FastOf;
template <>
struct FastOf<double> {
    using T = FastPtD;
    static __device__ __forceinline__ const FastPtD *get(const StencilDev &s) { return s.fastD; }
};
template <>
struct FastOf<float> {
    using T = FastPtF;
    static __device__ __forceinline__ const FastPtF *get(const StencilDev &s) { return s.fastF; }
};

// untruncated landing: cell i + floor(Y) with the precomputed corner weights
template <int DIM, typename TS, typename TC>
__device__ __forceinline__ TC interp_fast(const TS *__restrict__ V, int i, const typename FastOf<TC>::T &p,
                                          const LevelDev &g) {
    TC w[8];
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) w[c] = (TC)p.w[c];
    return interp_w<DIM, TS, TC>(V, i + p.off, g, w);
}

// the 2^DIM corner values of the cell at `base`, and their weighted sum in interp_w's order with the
// precomputed weights of a table point
template <int DIM, typename TS>
__device__ __forceinline__ void corner_vals(const TS *__restrict__ V, int base, const LevelDev &g, TS c[8]) {
    const int s1 = (int)g.s1;
    c[0] = V[base];
    c[1] = V[base + 1];
    c[2] = V[base + s1];
    c[3] = V[base + s1 + 1];
    if (DIM == 3) {
        const int s2 = (int)g.s2;
        c[4] = V[base + s2];
        c[5] = V[base + s2 + 1];
        c[6] = V[base + s2 + s1];
        c[7] = V[base + s2 + s1 + 1];
    }
}

template <int DIM, typename TS, typename TC>
__device__ __forceinline__ TC corner_wsum(const typename FastOf<TC>::T &p, const TS c[8]) {
    TC v = (TC)p.w[0] * (TC)c[0];
    v = fmat((TC)p.w[1], (TC)c[1], v);
    v = fmat((TC)p.w[2], (TC)c[2], v);
    v = fmat((TC)p.w[3], (TC)c[3], v);
    if (DIM == 3) {
        v = fmat((TC)p.w[4], (TC)c[4], v);
        v = fmat((TC)p.w[5], (TC)c[5], v);
        v = fmat((TC)p.w[6], (TC)c[6], v);
        v = fmat((TC)p.w[7], (TC)c[7], v);
    }
    return v;
}

// general landing: corner weights from the fractions, product over axes in axis order
template <int DIM, typename TS, typename TC, typename TT = double>
__device__ __forceinline__ TC interp_land(const TS *__restrict__ V, const LevelDev &g, const int cell[3],
                                          const TT td[3]) {
    TC t[3], u[3], w[8];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        t[d] = (TC)td[d];
        u[d] = (TC)1 - t[d];
    }
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        TC x = (c & 1) ? t[0] : u[0];
        x = x * (((c >> 1) & 1) ? t[1] : u[1]);
        if (DIM == 3) x = x * (((c >> 2) & 1) ? t[2] : u[2]);
        w[c] = x;
    }
    int base = cell[0] + cell[1] * (int)g.s1 + (DIM == 3 ? cell[2] * (int)g.s2 : 0);
    return interp_w<DIM, TS, TC>(V, base, g, w);
}

// (L-hat^k V)_i for one or two fields sharing the stencil geometry (eq. TruncScheme).
// TS: storage type of the fields, TC: arithmetic type.
template <int DIM, typename TS, typename TC, bool TWO>
__device__ __forceinline__ void lhat_node(const LevelDev &g, const StencilDev &st, int k, int i, const int ix[3],
                                          bool deep, const TS *__restrict__ V, TC Vi, const TS *__restrict__ W, TC Wi,
                                          TC &outV, TC &outW) {
    // policies are validated on entry; the clamp only keeps table reads in bounds
    k = ((unsigned)k < (unsigned)st.K) ? k : 0;
    const PointTab *pt = st.tab + k * st.npt;
    TC accV = (TC)0, accW = (TC)0;
    if (deep && st.pernode) {
        // per-node displacements away from the boundary: no point can leave the box (mu = 1, A = B = C = 1),
        // so the landing is i + floor(Y) with fraction Y - floor(Y), the general rules' untruncated case
        auto land1 = [&](int q, int cell[3], double t[3]) {
            double Y[3];
            point_Y(st, pt[q], q, ix, i, DIM, Y);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                double fl = floor(Y[d]);
                cell[d] = ix[d] + (int)fl;
                t[d] = Y[d] - fl;
            }
        };
        for (int p = 0; p < st.P; ++p) {
            int cp[3], cm[3];
            double tp[3], tm[3];
            land1(2 * p, cp, tp);
            land1(2 * p + 1, cm, tm);
            TC vp = interp_land<DIM, TS, TC>(V, g, cp, tp);
            TC vm = interp_land<DIM, TS, TC>(V, g, cm, tm);
            accV = accV + ((vp + vm) - (TC)2 * Vi);
            if (TWO) {
                TC wp = interp_land<DIM, TS, TC>(W, g, cp, tp);
                TC wm = interp_land<DIM, TS, TC>(W, g, cm, tm);
                accW = accW + ((wp + wm) - (TC)2 * Wi);
            }
        }
        if (st.has_drift) {
            int cb[3];
            double tb[3];
            land1(2 * st.P, cb, tb);
            TC vb = interp_land<DIM, TS, TC>(V, g, cb, tb);
            accV = accV + (TC)2 * (vb - Vi);
            if (TWO) {
                TC wb = interp_land<DIM, TS, TC>(W, g, cb, tb);
                accW = accW + (TC)2 * (wb - Wi);
            }
        }
    } else if (deep && st.P == 1) {
        // one diffusion pair: all corner loads are issued before any is used (the drift point's loads
        // read the node itself when there is no drift, so they need no branch)
        const typename FastOf<TC>::T *fp = FastOf<TC>::get(st) + k * st.npt;
        const auto &a = fp[0];
        const auto &b = fp[1];
        const auto &c = fp[st.has_drift ? 2 : 0];
        const int ba = i + a.off, bb = i + b.off, bc = st.has_drift ? i + c.off : i;
        TS va[8], vb[8], vc[8], wa[TWO ? 8 : 1], wb[TWO ? 8 : 1], wc[TWO ? 8 : 1];
        corner_vals<DIM, TS>(V, ba, g, va);
        corner_vals<DIM, TS>(V, bb, g, vb);
        corner_vals<DIM, TS>(V, bc, g, vc);
        if (TWO) {
            corner_vals<DIM, TS>(W, ba, g, wa);
            corner_vals<DIM, TS>(W, bb, g, wb);
            corner_vals<DIM, TS>(W, bc, g, wc);
        }
        TC vp = corner_wsum<DIM, TS, TC>(a, va);
        TC vm = corner_wsum<DIM, TS, TC>(b, vb);
        accV = accV + ((vp + vm) - (TC)2 * Vi);
        if (TWO) {
            TC wp = corner_wsum<DIM, TS, TC>(a, wa);
            TC wm = corner_wsum<DIM, TS, TC>(b, wb);
            accW = accW + ((wp + wm) - (TC)2 * Wi);
        }
        if (st.has_drift) {
            TC vd = corner_wsum<DIM, TS, TC>(c, vc);
            accV = accV + (TC)2 * (vd - Vi);
            if (TWO) {
                TC wd = corner_wsum<DIM, TS, TC>(c, wc);
                accW = accW + (TC)2 * (wd - Wi);
            }
        }
    } else if (deep) {
        const typename FastOf<TC>::T *fp = FastOf<TC>::get(st) + k * st.npt;  // corner weights precomputed
        for (int p = 0; p < st.P; ++p) {
            const auto &a = fp[2 * p];
            const auto &b = fp[2 * p + 1];
            TC vp = interp_fast<DIM, TS, TC>(V, i, a, g);
            TC vm = interp_fast<DIM, TS, TC>(V, i, b, g);
            accV = accV + ((vp + vm) - (TC)2 * Vi);
            if (TWO) {
                TC wp = interp_fast<DIM, TS, TC>(W, i, a, g);
                TC wm = interp_fast<DIM, TS, TC>(W, i, b, g);
                accW = accW + ((wp + wm) - (TC)2 * Wi);
            }
        }
        if (st.has_drift) {
            const auto &c = fp[2 * st.P];
            TC vb = interp_fast<DIM, TS, TC>(V, i, c, g);
            accV = accV + (TC)2 * (vb - Vi);
            if (TWO) {
                TC wb = interp_fast<DIM, TS, TC>(W, i, c, g);
                accW = accW + (TC)2 * (wb - Wi);
            }
        }
    } else if constexpr (std::is_same<TC, float>::value) {
        // FP32 kernels: the landings in FP32 (landing_f)
        auto yf = [&](int q, float Yf[3]) {
            double Y[3];
            point_Y(st, pt[q], q, ix, i, DIM, Y);
#pragma unroll
            for (int d = 0; d < 3; ++d) Yf[d] = (float)Y[d];
        };
        for (int p = 0; p < st.P; ++p) {
            float Ya[3], Yb[3];
            yf(2 * p, Ya);
            yf(2 * p + 1, Yb);
            int cp[3], cm[3];
            float tp[3], tm[3];
            const float mup = landing_f<DIM>(g, ix, Ya, cp, tp);
            const float mum = landing_f<DIM>(g, ix, Yb, cm, tm);
            const float A = 2.0f * __builtin_amdgcn_rcpf(mup * (mup + mum));
            const float B = 2.0f * __builtin_amdgcn_rcpf(mum * (mum + mup));
            const TC vp = interp_land<DIM, TS, TC, float>(V, g, cp, tp);
            const TC vm = interp_land<DIM, TS, TC, float>(V, g, cm, tm);
            accV = accV + ((A * vp + B * vm) - (A + B) * Vi);
            if (TWO) {
                const TC wp = interp_land<DIM, TS, TC, float>(W, g, cp, tp);
                const TC wm = interp_land<DIM, TS, TC, float>(W, g, cm, tm);
                accW = accW + ((A * wp + B * wm) - (A + B) * Wi);
            }
        }
        if (st.has_drift) {
            float Yc[3];
            yf(2 * st.P, Yc);
            int cb[3];
            float tb[3];
            const float C2 = 2.0f * __builtin_amdgcn_rcpf(landing_f<DIM>(g, ix, Yc, cb, tb));
            const TC vb = interp_land<DIM, TS, TC, float>(V, g, cb, tb);
            accV = accV + C2 * (vb - Vi);
            if (TWO) {
                const TC wb = interp_land<DIM, TS, TC, float>(W, g, cb, tb);
                accW = accW + C2 * (wb - Wi);
            }
        }
    } else {
        for (int p = 0; p < st.P; ++p) {
            double Ya[3], Yb[3];
            point_Y(st, pt[2 * p], 2 * p, ix, i, DIM, Ya);
            point_Y(st, pt[2 * p + 1], 2 * p + 1, ix, i, DIM, Yb);
            int cp[3], cm[3];
            double tp[3], tm[3];
            double mup = landing<DIM>(g, ix, Ya, cp, tp);
            double mum = landing<DIM>(g, ix, Yb, cm, tm);
            double A = 2.0 / (mup * (mup + mum));
            double B = 2.0 / (mum * (mum + mup));
            TC At = (TC)A, Bt = (TC)B, ABt = (TC)(A + B);
            TC vp = interp_land<DIM, TS, TC>(V, g, cp, tp);
            TC vm = interp_land<DIM, TS, TC>(V, g, cm, tm);
            accV = accV + ((At * vp + Bt * vm) - ABt * Vi);
            if (TWO) {
                TC wp = interp_land<DIM, TS, TC>(W, g, cp, tp);
                TC wm = interp_land<DIM, TS, TC>(W, g, cm, tm);
                accW = accW + ((At * wp + Bt * wm) - ABt * Wi);
            }
        }
        if (st.has_drift) {
            double Yc[3];
            point_Y(st, pt[2 * st.P], 2 * st.P, ix, i, DIM, Yc);
            int cb[3];
            double tb[3];
            double mub = landing<DIM>(g, ix, Yc, cb, tb);
            double C = 1.0 / mub;
            TC C2 = (TC)(2.0 * C);
            TC vb = interp_land<DIM, TS, TC>(V, g, cb, tb);
            accV = accV + C2 * (vb - Vi);
            if (TWO) {
                TC wb = interp_land<DIM, TS, TC>(W, g, cb, tb);
                accW = accW + C2 * (wb - Wi);
            }
        }
    }
    outV = (TC)st.inv2h * accV;
    if (TWO) outW = (TC)st.inv2h * accW;
}

template <int DIM, typename TS, typename TC>
__device__ __forceinline__ TC lhat1(const LevelDev &g, const StencilDev &st, int k, int i, const int ix[3], bool deep,
                                    const TS *__restrict__ V, TC Vi) {
    TC a, b;
    // the policy is piecewise constant: when the whole wavefront shares one control (and is untruncated),
    // its stencil tables are read once through the scalar unit instead of per lane
    int k0 = __builtin_amdgcn_readfirstlane(k);
    if (__all(k == k0 && deep)) {
        lhat_node<DIM, TS, TC, false>(g, st, k0, i, ix, true, V, Vi, V, Vi, a, b);
    } else {
        lhat_node<DIM, TS, TC, false>(g, st, k, i, ix, deep, V, Vi, V, Vi, a, b);
    }
    return a;
}

// ---- block reductions ----------------------------------------------------------------------------

template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, Op op, T *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_down(v, off, 64));
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    int nw = (blockDim.x + 63) >> 6;
    T r = sh[0];
    for (int w = 1; w < nw; ++w) r = op(r, sh[w]);
    return r;
}

struct OpSum {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a + b; }
};
// a NaN operand wins, so that a NaN residual or norm is never reported as a finite maximum
struct OpMax {
    __device__ double operator()(double a, double b) const { return (a > b || a != a) ? a : b; }
};

// ---- policy search (Howard's algorithm, eq. nonlinear_sys) ----------------------------------------

// G_k at node i.  QM 0: explicit part evaluated (theta < 1) or absent (theta = 1); QM 1: evaluated and
// stored in Q; QM 2: read from Q.  All three round identically.  Q is tile-major: entry (k, tile, lane)
// at k * qstride + qslot, qslot = tile * kBlock + lane, qstride = tiles * kBlock, so each wavefront
// moves whole aligned cache lines.
template <int DIM, bool CN, int QM>
__device__ __forceinline__ double eval_G(const LevelDev &g, const StencilDev &st, int k, int i, const int ix[3],
                                         bool deep, const double *__restrict__ X, double Xi,
                                         const double *__restrict__ U, double Ui, double theta, double omt, double f,
                                         double *__restrict__ Q, int64_t qslot = 0, int64_t qstride = 0) {
    double ck = st.c ? st.c[k] : 0.0;
    double lx, lu = 0.0;
    double q;
    if (CN && QM == 2) {
        lx = lhat1<DIM, double, double>(g, st, k, i, ix, deep, X, Xi);
        q = Q[(int64_t)k * qstride + qslot];
    } else {
        if (CN)
            lhat_node<DIM, double, double, true>(g, st, k, i, ix, deep, X, Xi, U, Ui, lx, lu);
        else
            lx = lhat1<DIM, double, double>(g, st, k, i, ix, deep, X, Xi);
        q = omt * (lu + ck * Ui);
        if (CN && QM == 1) Q[(int64_t)k * qstride + qslot] = q;
    }
    return theta * (lx + ck * Xi) + q + f;
}

}  // namespace slhjb
