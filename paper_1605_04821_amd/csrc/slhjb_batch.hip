// Batched node kernels of libslhjb: one launch covers the tiles of many independent instances
// (different grids, coefficients and level counts) concatenated in HBM.
//
// Each block looks up its (instance, tile) in a per-level table (the table position is renumbered
// like the single-instance kernels, so each XCD works on a contiguous range of tiles) and runs the
// single-instance arithmetic of slhjb_device.h on that instance's grid, stencil tables and arrays
// (instance arrays start at BInst::off of the level's batch arrays).  Blocks of instances whose flag
// in `active` is 0 exit at once; their outputs and partial sums are left untouched.  Per-block
// partial sums are indexed by table position; the tiles of one instance are contiguous in the table,
// so the segmented reductions below fold them per instance.

#include "slhjb_device.h"

namespace slhjb {

// table position of this block, its instance and whether the instance takes part
struct BCtx {
    int pos, inst;
    bool on;
};
__device__ __forceinline__ BCtx bctx(const BTiles &T) {
    BCtx c;
    c.pos = remap_block(blockIdx.x, gridDim.x);
    c.inst = T.inst[c.pos];
    c.on = !T.active || T.active[c.inst];
    return c;
}

// ---- search --------------------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_norms_b(BTiles T, const double *__restrict__ X,
                                                    const double *__restrict__ U, const double *__restrict__ f0,
                                                    const double *__restrict__ f1, double t_mid, double *partial) {
    __shared__ double sh[kBlock / 64];
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    double vx = 0.0, vf = 0.0;
    if (i >= 0) {
        vx = OpMax()(fabs(X[o + i]), fabs(U[o + i]));
        if (interior<DIM>(I.g, ix)) vf = fabs(f0[o + i] + t_mid * f1[o + i]);
    }
    double a = block_reduce<double>(vx, OpMax(), sh);
    if (threadIdx.x == 0) partial[c.pos] = a;
    double b = block_reduce<double>(vf, OpMax(), sh);
    if (threadIdx.x == 0) partial[T.n + c.pos] = b;
}

// tau[b] = tau_rel * (coefA[b] * max(|X|,|U|) + max|f|) over instance b's tiles [first[b], first[b+1]);
// a NaN wins the maxima (as in the single-instance tolerance), so a non-finite iterate gives a NaN tau
__global__ void k_tau_b(const double *partial, int n, const int32_t *first, const double *coefA, double tau_rel,
                        const uint8_t *active, double *tau) {
    __shared__ double sx[256], sf[256];
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const OpMax mx;
    double ax = 0.0, af = 0.0;
    for (int q = first[b] + threadIdx.x; q < first[b + 1]; q += blockDim.x) {
        ax = mx(ax, partial[q]);
        af = mx(af, partial[n + q]);
    }
    sx[threadIdx.x] = ax;
    sf[threadIdx.x] = af;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sx[threadIdx.x] = mx(sx[threadIdx.x], sx[threadIdx.x + w]);
            sf[threadIdx.x] = mx(sf[threadIdx.x], sf[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) tau[b] = tau_rel * (coefA[b] * sx[0] + sf[0]);
}

template <int DIM, bool CN>
__global__ __launch_bounds__(kBlock) void k_sweep_b(BTiles T, const double *__restrict__ X,
                                                    const double *__restrict__ U, const double *__restrict__ f0,
                                                    const double *__restrict__ f1, double t_mid, double theta,
                                                    const double *__restrict__ tau_b,
                                                    const int16_t *__restrict__ a_in, int16_t *__restrict__ a_out,
                                                    int64_t *changed_partial) {
    __shared__ int64_t sh[kBlock / 64];
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    const LevelDev g = I.g;
    const StencilDev st = I.st;
    const int64_t o = I.off;
    const double tau = tau_b[c.inst];
    const double *Xo = X + o, *Uo = U + o;
    int ix[3];
    int i = tile_node_at<DIM>(g, T.tile[c.pos], ix);
    int64_t changed = 0;
    if (i >= 0) {
        if (!interior<DIM>(g, ix)) {
            a_out[o + i] = -1;
        } else {
            bool deep = deep_node<DIM>(g, ix);
            double Xi = Xo[i], Ui = Uo[i];
            double f = f0[o + i] + t_mid * f1[o + i];
            double omt = 1.0 - theta;
            int cur = a_in[o + i];
            double best = __builtin_inf(), gcur = __builtin_inf();
            int kbest = 0;
            for (int k = 0; k < st.K; ++k) {
                double G = eval_G<DIM, CN, 0>(g, st, k, i, ix, deep, Xo, Xi, Uo, Ui, theta, omt, f, nullptr);
                if (G < best) {
                    best = G;
                    kbest = k;
                }
                if (k == cur) gcur = G;
            }
            double thr = best + tau;
            int pick;
            if (cur >= 0 && cur < st.K && gcur <= thr) {
                pick = cur;
            } else {
                pick = kbest;
                for (int k = 0; k < kbest; ++k) {
                    double G = eval_G<DIM, CN, 0>(g, st, k, i, ix, deep, Xo, Xi, Uo, Ui, theta, omt, f, nullptr);
                    if (G <= thr) {
                        pick = k;
                        break;
                    }
                }
            }
            a_out[o + i] = (int16_t)pick;
            changed = (pick != cur) ? 1 : 0;
        }
    }
    int64_t tot = block_reduce<int64_t>(changed, OpSum(), sh);
    if (threadIdx.x == 0) changed_partial[c.pos] = tot;
}

// ---- FP64 operator -------------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_explicit_b(BTiles T, const int16_t *__restrict__ alpha,
                                                       const double *__restrict__ U, const double *__restrict__ f0,
                                                       const double *__restrict__ f1, double t_mid, double omt_dt,
                                                       double dt, double *__restrict__ E) {
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    const StencilDev st = I.st;
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    if (i < 0) return;
    double e = 0.0;
    if (interior<DIM>(I.g, ix)) {
        double f = f0[o + i] + t_mid * f1[o + i];
        double Ui = U[o + i];
        if (omt_dt != 0.0) {
            int k = alpha[o + i];
            bool deep = deep_node<DIM>(I.g, ix);
            double l = lhat1<DIM, double, double>(I.g, st, k, i, ix, deep, U + o, Ui);
            double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
            e = Ui + omt_dt * (l + ck * Ui) + dt * f;
        } else {
            e = Ui + dt * f;
        }
    }
    E[o + i] = e;
}

// r = E - A V (interior, 0 on the boundary); partials [sum r^2 | max|r| | max|V|] per table position
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual_b(BTiles T, const int16_t *__restrict__ alpha,
                                                       const double *__restrict__ V, const double *__restrict__ E,
                                                       double theta_dt, double *__restrict__ r, double *partial) {
    __shared__ double sh[kBlock / 64];
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    const StencilDev st = I.st;
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    double rr = 0.0, vv = 0.0;
    if (i >= 0) {
        double Vi = V[o + i];
        vv = fabs(Vi);
        if (interior<DIM>(I.g, ix)) {
            int k = alpha[o + i];
            bool deep = deep_node<DIM>(I.g, ix);
            double l = lhat1<DIM, double, double>(I.g, st, k, i, ix, deep, V + o, Vi);
            double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
            rr = E[o + i] - (Vi - theta_dt * (l + ck * Vi));
        }
        r[o + i] = rr;
    }
    double s2 = block_reduce<double>(rr * rr, OpSum(), sh);
    if (threadIdx.x == 0) partial[c.pos] = s2;
    double m = block_reduce<double>(fabs(rr), OpMax(), sh);
    if (threadIdx.x == 0) partial[T.n + c.pos] = m;
    double mv = block_reduce<double>(vv, OpMax(), sh);
    if (threadIdx.x == 0) partial[2 * T.n + c.pos] = mv;
}

template <int DIM, typename TX>
__global__ __launch_bounds__(kBlock) void k_apply_b(BTiles T, const int16_t *__restrict__ alpha,
                                                    const TX *__restrict__ x, double *__restrict__ y,
                                                    double theta_dt) {
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    const StencilDev st = I.st;
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    if (i < 0) return;
    double yy = 0.0;
    if (interior<DIM>(I.g, ix)) {
        int k = alpha[o + i];
        bool deep = deep_node<DIM>(I.g, ix);
        double xi = (double)x[o + i];
        double l = lhat1<DIM, TX, double>(I.g, st, k, i, ix, deep, x + o, xi);
        double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
        yy = xi - theta_dt * (l + ck * xi);
    }
    y[o + i] = yy;
}

// ---- multigrid level kernels --------------------------------------------------------------------

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_diag_b(BTiles Tb, const int16_t *__restrict__ alpha, double theta_dt,
                                                   T *__restrict__ d) {
    BCtx c = bctx(Tb);
    if (!c.on) return;
    const BInst &I = Tb.I[c.inst];
    const LevelDev g = I.g;
    const StencilDev st = I.st;
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(g, Tb.tile[c.pos], ix);
    if (i < 0) return;
    if (!interior<DIM>(g, ix)) {
        d[o + i] = (T)1;
        return;
    }
    int k = alpha[o + i];
    k = ((unsigned)k < (unsigned)st.K) ? k : 0;
    const PointTab *pt = st.tab + k * st.npt;
    double lii = 0.0;
    for (int q = 0; q < st.npt; ++q) {
        double Y[3];
        point_Y(st, pt[q], q, ix, i, DIM, Y);
        int cell[3];
        double t[3];
        double mu = landing<DIM>(g, ix, Y, cell, t);
        double W;
        if (q < 2 * st.P) {
            double Yo[3];
            point_Y(st, pt[q ^ 1], q ^ 1, ix, i, DIM, Yo);
            int co[3];
            double to[3];
            double muo = landing<DIM>(g, ix, Yo, co, to);
            W = 2.0 / (mu * (mu + muo));
        } else {
            W = 2.0 / mu;
        }
        double wself = 1.0;
        for (int dd = 0; dd < DIM; ++dd) {
            if (ix[dd] == cell[dd])
                wself *= (1.0 - t[dd]);
            else if (ix[dd] == cell[dd] + 1)
                wself *= t[dd];
            else
                wself = 0.0;
        }
        lii += W * (wself - 1.0);
    }
    lii *= st.inv2h;
    double ck = st.c ? st.c[k] : 0.0;
    d[o + i] = (T)(1.0 - theta_dt * (lii + ck));
}

template <int DIM, typename T>
__device__ __forceinline__ T apply_level_b(const LevelDev &g, const StencilDev &st, const int16_t *__restrict__ alpha,
                                           const T *__restrict__ e, int i, const int ix[3], T theta_dt) {
    int k = alpha[i];
    bool deep = deep_node<DIM>(g, ix);
    T ei = e[i];
    T l = lhat1<DIM, T, T>(g, st, k, i, ix, deep, e, ei);
    T ck = st.c ? (T)st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : (T)0;
    return ei - theta_dt * (l + ck * ei);
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_b(BTiles Tb, const int16_t *__restrict__ alpha,
                                                     const T *__restrict__ e, const T *__restrict__ r,
                                                     const T *__restrict__ d, T *__restrict__ e_out, T theta_dt,
                                                     T omega, int first) {
    BCtx c = bctx(Tb);
    if (!c.on) return;
    const BInst &I = Tb.I[c.inst];
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(I.g, Tb.tile[c.pos], ix);
    if (i < 0) return;
    T v = (T)0;
    if (interior<DIM>(I.g, ix)) {
        if (first) {
            v = omega * r[o + i] / d[o + i];
        } else {
            T ae = apply_level_b<DIM, T>(I.g, I.st, alpha + o, e + o, i, ix, theta_dt);
            v = e[o + i] + omega * (r[o + i] - ae) / d[o + i];
        }
    }
    e_out[o + i] = v;
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_level_residual_b(BTiles Tb, const int16_t *__restrict__ alpha,
                                                             const T *__restrict__ e, const T *__restrict__ r,
                                                             T *__restrict__ res, T theta_dt) {
    BCtx c = bctx(Tb);
    if (!c.on) return;
    const BInst &I = Tb.I[c.inst];
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(I.g, Tb.tile[c.pos], ix);
    if (i < 0) return;
    T v = (T)0;
    if (interior<DIM>(I.g, ix)) v = r[o + i] - apply_level_b<DIM, T>(I.g, I.st, alpha + o, e + o, i, ix, theta_dt);
    res[o + i] = v;
}

// full weighting into the coarse level (table over coarse tiles; If: the fine level's descriptors)
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_b(BTiles Tc, const BInst *__restrict__ If,
                                                       const T *__restrict__ rf, T *__restrict__ rc) {
    BCtx c = bctx(Tc);
    if (!c.on) return;
    const BInst &C = Tc.I[c.inst];
    const BInst &F = If[c.inst];
    const LevelDev gf = F.g;
    int ix[3];
    int I = tile_node_at<DIM>(C.g, Tc.tile[c.pos], ix);
    if (I < 0) return;
    T v = (T)0;
    if (interior<DIM>(C.g, ix)) {
        const T *r0 = rf + F.off;
        int cc0 = 2 * ix[0] + 2 * ix[1] * (int)gf.s1 + (DIM == 3 ? 2 * ix[2] * (int)gf.s2 : 0);
        const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
        if (DIM == 2) {
            for (int b = -1; b <= 1; ++b) {
                T row = w[0] * r0[cc0 + b * (int)gf.s1 - 1] + w[1] * r0[cc0 + b * (int)gf.s1] +
                        w[2] * r0[cc0 + b * (int)gf.s1 + 1];
                v += w[b + 1] * row;
            }
        } else {
            for (int cz = -1; cz <= 1; ++cz) {
                T pl = (T)0;
                for (int b = -1; b <= 1; ++b) {
                    int q = cc0 + cz * (int)gf.s2 + b * (int)gf.s1;
                    T row = w[0] * r0[q - 1] + w[1] * r0[q] + w[2] * r0[q + 1];
                    pl += w[b + 1] * row;
                }
                v += w[cz + 1] * pl;
            }
        }
    }
    rc[C.off + I] = v;
}

// multilinear prolongation added on fine interior nodes (table over fine tiles; Ic: coarse descriptors)
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add_b(BTiles Tf, const BInst *__restrict__ Ic,
                                                          const T *__restrict__ ec, T *__restrict__ ef) {
    BCtx c = bctx(Tf);
    if (!c.on) return;
    const BInst &F = Tf.I[c.inst];
    const BInst &C = Ic[c.inst];
    int ix[3];
    int i = tile_node_at<DIM>(F.g, Tf.tile[c.pos], ix);
    if (i < 0) return;
    if (!interior<DIM>(F.g, ix)) return;
    int lo[3], hi[3];
    T wl[3], wh[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
            lo[d] = ix[d] >> 1;
            if (ix[d] & 1) {
                hi[d] = lo[d] + 1;
                wl[d] = (T)0.5;
                wh[d] = (T)0.5;
            } else {
                hi[d] = lo[d];
                wl[d] = (T)1;
                wh[d] = (T)0;
            }
        } else {
            lo[d] = hi[d] = 0;
            wl[d] = (T)1;
            wh[d] = (T)0;
        }
    }
    const T *e0 = ec + C.off;
    const int s1 = (int)C.g.s1, s2 = (int)C.g.s2;
    auto at = [&](int a, int b, int cz) { return e0[a + b * s1 + (DIM == 3 ? cz * s2 : 0)]; };
    T a0 = wl[0] * at(lo[0], lo[1], lo[2]) + wh[0] * at(hi[0], lo[1], lo[2]);
    T a1 = wl[0] * at(lo[0], hi[1], lo[2]) + wh[0] * at(hi[0], hi[1], lo[2]);
    T v = wl[1] * a0 + wh[1] * a1;
    if (DIM == 3) {
        T b0 = wl[0] * at(lo[0], lo[1], hi[2]) + wh[0] * at(hi[0], lo[1], hi[2]);
        T b1 = wl[0] * at(lo[0], hi[1], hi[2]) + wh[0] * at(hi[0], hi[1], hi[2]);
        v = wl[2] * v + wh[2] * (wl[1] * b0 + wh[1] * b1);
    }
    ef[F.off + i] += v;
}

// coarsest levels: one workgroup per instance, Jacobi sweeps with the iterate in LDS (N <= maxN)
template <int DIM, typename T>
__global__ __launch_bounds__(1024) void k_coarse_b(const int32_t *__restrict__ list, const BInst *__restrict__ Iv,
                                                   const uint8_t *__restrict__ active,
                                                   const int16_t *__restrict__ alpha, const T *__restrict__ r,
                                                   const T *__restrict__ d, T *__restrict__ e, T theta_dt, T omega,
                                                   int sweeps) {
    extern __shared__ unsigned char smem[];
    const int b = list[blockIdx.x];
    if (active && !active[b]) return;
    const BInst &I = Iv[b];
    const LevelDev g = I.g;
    const int64_t o = I.off;
    T *a = reinterpret_cast<T *>(smem);
    T *bb = a + g.N;
    const int N = (int)g.N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        int ix[3];
        unflatten<DIM>(g, i, ix);
        a[i] = interior<DIM>(g, ix) ? omega * r[o + i] / d[o + i] : (T)0;
    }
    __syncthreads();
    for (int sw = 1; sw < sweeps; ++sw) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            int ix[3];
            unflatten<DIM>(g, i, ix);
            T v = (T)0;
            if (interior<DIM>(g, ix)) {
                T ae = apply_level_b<DIM, T>(g, I.st, alpha + o, a, i, ix, theta_dt);
                v = a[i] + omega * (r[o + i] - ae) / d[o + i];
            }
            bb[i] = v;
        }
        __syncthreads();
        T *tmp = a;
        a = bb;
        bb = tmp;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) e[o + i] = a[i];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_inject_b(BTiles Tc, const BInst *__restrict__ If,
                                                     const int16_t *__restrict__ af, int16_t *__restrict__ ac) {
    BCtx c = bctx(Tc);
    if (!c.on) return;
    const BInst &C = Tc.I[c.inst];
    const BInst &F = If[c.inst];
    int ix[3];
    int I = tile_node_at<DIM>(C.g, Tc.tile[c.pos], ix);
    if (I < 0) return;
    int16_t v = -1;
    if (interior<DIM>(C.g, ix))
        v = af[F.off + 2 * ix[0] + 2 * ix[1] * (int)F.g.s1 + (DIM == 3 ? 2 * ix[2] * (int)F.g.s2 : 0)];
    ac[C.off + I] = v;
}

// ---- whole-grid helpers ----------------------------------------------------------------------------

// mode 0: dst interior = src; mode 1: dst interior = U1 + ratio (U1 - U0) (src = U1, src2 = U0);
// mode 2: dst = src on every node (copy of the instance)
template <int DIM, int MODE, typename TV>
__global__ __launch_bounds__(kBlock) void k_copy_b(BTiles T, const TV *__restrict__ src, const TV *__restrict__ src2,
                                                   double ratio, TV *__restrict__ dst) {
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    const int64_t o = I.off;
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    if (i < 0) return;
    if (MODE == 2) {
        dst[o + i] = src[o + i];
    } else if (interior<DIM>(I.g, ix)) {
        if (MODE == 0)
            dst[o + i] = src[o + i];
        else
            dst[o + i] = (TV)((double)src[o + i] + ratio * ((double)src[o + i] - (double)src2[o + i]));
    }
}

// ---- flexible GMRES vector kernels (per-instance coefficients) ------------------------------------

// partial[v * n + pos] = <w, V_v> over the block's nodes for v < nvec, partial[nvec * n + pos] = |w|^2
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_multidot_b(BTiles T, const double *__restrict__ w,
                                                       const double *__restrict__ V, int64_t ldv, int nvec,
                                                       double *partial) {
    __shared__ double sh[kBlock / 64];
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    const int64_t n = I.off + i;
    double wv = i >= 0 ? w[n] : 0.0;
    for (int v = 0; v < nvec; ++v) {
        double acc = i >= 0 ? wv * V[(int64_t)v * ldv + n] : 0.0;
        double t = block_reduce<double>(acc, OpSum(), sh);
        if (threadIdx.x == 0) partial[(int64_t)v * T.n + c.pos] = t;
    }
    double t = block_reduce<double>(wv * wv, OpSum(), sh);
    if (threadIdx.x == 0) partial[(int64_t)nvec * T.n + c.pos] = t;
}

// w = (w - sum_v coef[b][v] V_v) / sqrt(coef[b][nvec] - sum_v coef[b][v]^2) for instance b
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_multiaxpy_scale_b(BTiles T, double *__restrict__ w,
                                                              const double *__restrict__ V, int64_t ldv, int nvec,
                                                              const double *__restrict__ coef, int ldc) {
    __shared__ double cf[kMaxRestart + 2];
    BCtx c = bctx(T);
    if (!c.on) return;
    const double *cb = coef + (int64_t)c.inst * ldc;
    for (int v = threadIdx.x; v <= nvec; v += blockDim.x) cf[v] = cb[v];
    __syncthreads();
    double h2 = 0.0;
    for (int v = 0; v < nvec; ++v) h2 += cf[v] * cf[v];
    double hn2 = cf[nvec] - h2;
    double inv = hn2 > 0.0 ? 1.0 / sqrt(hn2) : 1.0;
    const BInst &I = T.I[c.inst];
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    if (i < 0) return;
    const int64_t n = I.off + i;
    double x = w[n];
    for (int v = 0; v < nvec; ++v) x -= cf[v] * V[(int64_t)v * ldv + n];
    w[n] = x * inv;
}

// dst = src / sqrt(norm2[b])
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_scale_b(BTiles T, double *__restrict__ dst, const double *__restrict__ src,
                                                    const double *__restrict__ norm2, int ldn) {
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    if (i < 0) return;
    const int64_t n = I.off + i;
    dst[n] = src[n] * (1.0 / sqrt(norm2[(int64_t)c.inst * ldn]));
}

// X += sum_{j < m[b]} y[b][j] Z_j
template <int DIM, typename TZ>
__global__ __launch_bounds__(kBlock) void k_update_b(BTiles T, double *__restrict__ X, const TZ *__restrict__ Z,
                                                     int64_t ldz, const int32_t *__restrict__ m,
                                                     const double *__restrict__ y, int ldy) {
    BCtx c = bctx(T);
    if (!c.on) return;
    const BInst &I = T.I[c.inst];
    int ix[3];
    int i = tile_node_at<DIM>(I.g, T.tile[c.pos], ix);
    if (i < 0) return;
    const int64_t n = I.off + i;
    const int mb = m[c.inst];
    const double *yb = y + (int64_t)c.inst * ldy;
    double x = X[n];
    for (int j = 0; j < mb; ++j) x += yb[j] * (double)Z[(int64_t)j * ldz + n];
    X[n] = x;
}

// out[b * nvec + v] = sum (OP 0) or max (OP 1) of partial[v * n + q] over instance b's positions
template <int OP, typename TV>
__global__ void k_seg_reduce(const TV *__restrict__ partial, int n, const int32_t *__restrict__ first, int nvec,
                             const uint8_t *__restrict__ active, TV *__restrict__ out) {
    __shared__ TV sh[256];
    const int b = blockIdx.x, v = blockIdx.y;
    if (active && !active[b]) return;
    const TV *p = partial + (int64_t)v * n;
    TV acc = (TV)0;
    for (int q = first[b] + threadIdx.x; q < first[b + 1]; q += blockDim.x) acc = OP == 0 ? acc + p[q] : (acc > p[q] ? acc : p[q]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            TV a = sh[threadIdx.x], c = sh[threadIdx.x + w];
            sh[threadIdx.x] = OP == 0 ? a + c : (a > c ? a : c);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)b * nvec + v] = sh[0];
}

// ---- flexible GMRES scalars on the device (one thread per instance) -----------------------------------
// The Hessenberg columns, Givens rotations, residual estimates and the instances' masks of a restart cycle
// are advanced by these kernels, so that a cycle needs no host decision and can be captured as one graph.
// The arithmetic is that of the single-instance host loop (classical Gram-Schmidt twice, the second pass
// skipped where the first kept more than a quarter of |w|^2).

// a cycle starts: g = (|r|_2, 0, ...), no column yet, every solving instance in the cycle
__global__ void k_cycle_init_b(BKrylov K, int B, const uint8_t *__restrict__ solving, const double *__restrict__ r2,
                               uint8_t *__restrict__ cyc) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    cyc[b] = solving[b];
    K.jb[b] = 0;
    if (!solving[b]) return;
    double *g = K.g + (int64_t)b * (K.m + 1);
    g[0] = sqrt(r2[b]);
    for (int i = 1; i <= K.m; ++i) g[i] = 0.0;
}

__global__ void k_mask_copy_b(int B, const uint8_t *__restrict__ src, uint8_t *__restrict__ dst) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) dst[b] = src[b];
}

// after Gram-Schmidt pass `pass` of step j (seg[b][0..j+1]: the pass's products with V_0..V_j and |w|^2):
// the update coefficients, the Hessenberg column, the norm of the new vector, and whether a second pass follows
__global__ void k_arnoldi_pass_b(BKrylov K, int B, int j, int pass, const double *__restrict__ seg,
                                 double *__restrict__ coef, int ldc, const uint8_t *__restrict__ in_pass,
                                 uint8_t *__restrict__ next_pass) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (!in_pass[b]) {
        next_pass[b] = 0;
        return;
    }
    const double *hp = seg + (int64_t)b * (j + 2);
    double *cb = coef + (int64_t)b * ldc;
    for (int i = 0; i <= j + 1; ++i) cb[i] = hp[i];
    const double w2 = hp[j + 1];
    double h2 = 0.0;
    for (int i = 0; i <= j; ++i) h2 += hp[i] * hp[i];
    const double hn2 = w2 - h2;
    const double sc = hn2 > 0.0 ? sqrt(hn2) : 1.0;
    if (!isfinite(w2)) K.bad[b] = 1;
    double *H = K.H + (int64_t)b * (K.m + 1) * K.m;
    if (pass == 0) {
        for (int i = 0; i <= j; ++i) H[(int64_t)i * K.m + j] = hp[i];
        K.hn[b] = sc;
    } else {
        for (int i = 0; i <= j; ++i) H[(int64_t)i * K.m + j] += hp[i] * K.hn[b];
        K.hn[b] = K.hn[b] * sc;
    }
    bool done = hn2 > 0.25 * w2;
    if (!done && (w2 == 0.0 || (pass == 1 && !(hn2 > 0.0)))) {
        K.hn[b] = 0.0;
        done = true;
    }
    next_pass[b] = done ? 0 : 1;
}

// step j closes: subdiagonal entry, earlier rotations applied, the new rotation, the residual estimate; an
// instance leaves the cycle once |g_{j+1}| <= target / 2, at breakdown, or at its iteration limit
__global__ void k_givens_b(BKrylov K, int B, int j, uint8_t *__restrict__ cyc) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || !cyc[b]) return;
    const int m = K.m;
    double *H = K.H + (int64_t)b * (m + 1) * m;
    double *cs = K.cs + (int64_t)b * m, *sn = K.sn + (int64_t)b * m, *g = K.g + (int64_t)b * (m + 1);
    H[(int64_t)(j + 1) * m + j] = K.hn[b];
    K.its[b] += 1;
    for (int i = 0; i < j; ++i) {
        const double a = H[(int64_t)i * m + j], c = H[(int64_t)(i + 1) * m + j];
        H[(int64_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
    }
    const double a = H[(int64_t)j * m + j], c = H[(int64_t)(j + 1) * m + j];
    const double rr = hypot(a, c);
    cs[j] = rr > 0 ? a / rr : 1.0;
    sn[j] = rr > 0 ? c / rr : 0.0;
    H[(int64_t)j * m + j] = rr;
    H[(int64_t)(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    K.jb[b] = j + 1;
    if (fabs(g[j + 1]) <= 0.5 * K.target[b] || K.hn[b] == 0.0 || K.its[b] >= K.maxk) cyc[b] = 0;
}

// y = R^{-1} g over the cycle's columns (the update X += Z y follows); count[b] = the number of columns
__global__ void k_backsolve_b(BKrylov K, int B, const uint8_t *__restrict__ solving, double *__restrict__ y, int ldy,
                              int32_t *__restrict__ count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (!solving[b]) {
        count[b] = 0;
        return;
    }
    const int m = K.m, jj = K.jb[b];
    const double *H = K.H + (int64_t)b * (m + 1) * m, *g = K.g + (int64_t)b * (m + 1);
    double *yb = y + (int64_t)b * ldy;
    for (int i = jj - 1; i >= 0; --i) {
        double acc = g[i];
        for (int q = i + 1; q < jj; ++q) acc -= H[(int64_t)i * m + q] * yb[q];
        yb[i] = acc / H[(int64_t)i * m + i];
    }
    count[b] = jj;
}

// ---- launchers ---------------------------------------------------------------------------------------

#define BGRID(T) dim3((unsigned)(T).n), dim3(kBlock), 0, s

static dim3 bgrid_inst(int B) { return dim3((unsigned)((B + 63) / 64)); }
void launch_cycle_init_b(const BKrylov &K, int B, const uint8_t *solving, const double *r2, uint8_t *cyc,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_init_b, bgrid_inst(B), dim3(64), 0, s, K, B, solving, r2, cyc);
}
void launch_mask_copy_b(int B, const uint8_t *src, uint8_t *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_copy_b, bgrid_inst(B), dim3(64), 0, s, B, src, dst);
}
void launch_arnoldi_pass_b(const BKrylov &K, int B, int j, int pass, const double *seg, double *coef, int ldc,
                           const uint8_t *in_pass, uint8_t *next_pass, hipStream_t s) {
    hipLaunchKernelGGL(k_arnoldi_pass_b, bgrid_inst(B), dim3(64), 0, s, K, B, j, pass, seg, coef, ldc, in_pass,
                       next_pass);
}
void launch_givens_b(const BKrylov &K, int B, int j, uint8_t *cyc, hipStream_t s) {
    hipLaunchKernelGGL(k_givens_b, bgrid_inst(B), dim3(64), 0, s, K, B, j, cyc);
}
void launch_backsolve_b(const BKrylov &K, int B, const uint8_t *solving, double *y, int ldy, int32_t *count,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_backsolve_b, bgrid_inst(B), dim3(64), 0, s, K, B, solving, y, ldy, count);
}

void launch_norms_b(int dim, const BTiles &T, const double *X, const double *U, const double *f0, const double *f1,
                    double t_mid, double *partial, hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_norms_b<2>, BGRID(T), T, X, U, f0, f1, t_mid, partial);
    else hipLaunchKernelGGL(k_norms_b<3>, BGRID(T), T, X, U, f0, f1, t_mid, partial);
}

void launch_tau_b(const double *partial, int n, const int32_t *first, const double *coefA, double tau_rel,
                  const uint8_t *active, double *tau, int B, hipStream_t s) {
    hipLaunchKernelGGL(k_tau_b, dim3(B), dim3(256), 0, s, partial, n, first, coefA, tau_rel, active, tau);
}

void launch_sweep_b(int dim, const BTiles &T, const double *X, const double *U, const double *f0, const double *f1,
                    double t_mid, double theta, const double *tau, const int16_t *a_in, int16_t *a_out,
                    int64_t *changed_partial, hipStream_t s) {
    if (T.n == 0) return;
    const bool cn = theta != 1.0;
#define SWB(D, C) hipLaunchKernelGGL((k_sweep_b<D, C>), BGRID(T), T, X, U, f0, f1, t_mid, theta, tau, a_in, a_out, \
                                     changed_partial)
    if (dim == 2) {
        if (cn) SWB(2, true); else SWB(2, false);
    } else {
        if (cn) SWB(3, true); else SWB(3, false);
    }
#undef SWB
}

void launch_explicit_b(int dim, const BTiles &T, const int16_t *alpha, const double *U, const double *f0,
                       const double *f1, double t_mid, double omt_dt, double dt, double *E, hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_explicit_b<2>, BGRID(T), T, alpha, U, f0, f1, t_mid, omt_dt, dt, E);
    else hipLaunchKernelGGL(k_explicit_b<3>, BGRID(T), T, alpha, U, f0, f1, t_mid, omt_dt, dt, E);
}

void launch_residual_b(int dim, const BTiles &T, const int16_t *alpha, const double *V, const double *E,
                       double theta_dt, double *r, double *partial, hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_residual_b<2>, BGRID(T), T, alpha, V, E, theta_dt, r, partial);
    else hipLaunchKernelGGL(k_residual_b<3>, BGRID(T), T, alpha, V, E, theta_dt, r, partial);
}

void launch_apply_b(int dim, const BTiles &T, const int16_t *alpha, const void *x, bool x_float, double *y,
                    double theta_dt, hipStream_t s) {
    if (T.n == 0) return;
#define APB(D, TX) hipLaunchKernelGGL((k_apply_b<D, TX>), BGRID(T), T, alpha, (const TX *)x, y, theta_dt)
    if (x_float) {
        if (dim == 2) APB(2, float); else APB(3, float);
    } else {
        if (dim == 2) APB(2, double); else APB(3, double);
    }
#undef APB
}

template <typename T>
void launch_diag_b(int dim, const BTiles &Tb, const int16_t *alpha, double theta_dt, T *d, hipStream_t s) {
    if (Tb.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL((k_diag_b<2, T>), BGRID(Tb), Tb, alpha, theta_dt, d);
    else hipLaunchKernelGGL((k_diag_b<3, T>), BGRID(Tb), Tb, alpha, theta_dt, d);
}

template <typename T>
void launch_jacobi_b(int dim, const BTiles &Tb, const int16_t *alpha, const T *e, const T *r, const T *d, T *e_out,
                     double theta_dt, double omega, bool first, hipStream_t s) {
    if (Tb.n == 0) return;
    if (dim == 2)
        hipLaunchKernelGGL((k_jacobi_b<2, T>), BGRID(Tb), Tb, alpha, e, r, d, e_out, (T)theta_dt, (T)omega, (int)first);
    else
        hipLaunchKernelGGL((k_jacobi_b<3, T>), BGRID(Tb), Tb, alpha, e, r, d, e_out, (T)theta_dt, (T)omega, (int)first);
}

template <typename T>
void launch_level_residual_b(int dim, const BTiles &Tb, const int16_t *alpha, const T *e, const T *r, T *res,
                             double theta_dt, hipStream_t s) {
    if (Tb.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL((k_level_residual_b<2, T>), BGRID(Tb), Tb, alpha, e, r, res, (T)theta_dt);
    else hipLaunchKernelGGL((k_level_residual_b<3, T>), BGRID(Tb), Tb, alpha, e, r, res, (T)theta_dt);
}

template <typename T>
void launch_restrict_b(int dim, const BTiles &Tc, const BInst *If, const T *rf, T *rc, hipStream_t s) {
    if (Tc.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL((k_restrict_b<2, T>), BGRID(Tc), Tc, If, rf, rc);
    else hipLaunchKernelGGL((k_restrict_b<3, T>), BGRID(Tc), Tc, If, rf, rc);
}

template <typename T>
void launch_prolong_add_b(int dim, const BTiles &Tf, const BInst *Ic, const T *ec, T *ef, hipStream_t s) {
    if (Tf.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL((k_prolong_add_b<2, T>), BGRID(Tf), Tf, Ic, ec, ef);
    else hipLaunchKernelGGL((k_prolong_add_b<3, T>), BGRID(Tf), Tf, Ic, ec, ef);
}

template <typename T>
void launch_coarse_b(int dim, const int32_t *list, int count, int64_t maxN, const BInst *Iv, const uint8_t *active,
                     const int16_t *alpha, const T *r, const T *d, T *e, double theta_dt, double omega, int sweeps,
                     hipStream_t s) {
    if (count == 0) return;
    size_t shm = 2 * (size_t)maxN * sizeof(T);
    if (dim == 2)
        hipLaunchKernelGGL((k_coarse_b<2, T>), dim3(count), dim3(1024), shm, s, list, Iv, active, alpha, r, d, e,
                           (T)theta_dt, (T)omega, sweeps);
    else
        hipLaunchKernelGGL((k_coarse_b<3, T>), dim3(count), dim3(1024), shm, s, list, Iv, active, alpha, r, d, e,
                           (T)theta_dt, (T)omega, sweeps);
}

void launch_inject_b(int dim, const BTiles &Tc, const BInst *If, const int16_t *af, int16_t *ac, hipStream_t s) {
    if (Tc.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_inject_b<2>, BGRID(Tc), Tc, If, af, ac);
    else hipLaunchKernelGGL(k_inject_b<3>, BGRID(Tc), Tc, If, af, ac);
}

void launch_copy_interior_b(int dim, const BTiles &T, const double *src, double *dst, hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL((k_copy_b<2, 0, double>), BGRID(T), T, src, nullptr, 0.0, dst);
    else hipLaunchKernelGGL((k_copy_b<3, 0, double>), BGRID(T), T, src, nullptr, 0.0, dst);
}

void launch_extrapolate_b(int dim, const BTiles &T, const double *U1, const double *U0, double ratio, double *out,
                          hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL((k_copy_b<2, 1, double>), BGRID(T), T, U1, U0, ratio, out);
    else hipLaunchKernelGGL((k_copy_b<3, 1, double>), BGRID(T), T, U1, U0, ratio, out);
}

void launch_copy_policy_b(int dim, const BTiles &T, const int16_t *src, int16_t *dst, hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL((k_copy_b<2, 2, int16_t>), BGRID(T), T, src, nullptr, 0.0, dst);
    else hipLaunchKernelGGL((k_copy_b<3, 2, int16_t>), BGRID(T), T, src, nullptr, 0.0, dst);
}

void launch_multidot_b(int dim, const BTiles &T, const double *w, const double *V, int64_t ldv, int nvec,
                       double *partial, hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_multidot_b<2>, BGRID(T), T, w, V, ldv, nvec, partial);
    else hipLaunchKernelGGL(k_multidot_b<3>, BGRID(T), T, w, V, ldv, nvec, partial);
}

void launch_multiaxpy_scale_b(int dim, const BTiles &T, double *w, const double *V, int64_t ldv, int nvec,
                              const double *coef, int ldc, hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_multiaxpy_scale_b<2>, BGRID(T), T, w, V, ldv, nvec, coef, ldc);
    else hipLaunchKernelGGL(k_multiaxpy_scale_b<3>, BGRID(T), T, w, V, ldv, nvec, coef, ldc);
}

void launch_scale_b(int dim, const BTiles &T, double *dst, const double *src, const double *norm2, int ldn,
                    hipStream_t s) {
    if (T.n == 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_scale_b<2>, BGRID(T), T, dst, src, norm2, ldn);
    else hipLaunchKernelGGL(k_scale_b<3>, BGRID(T), T, dst, src, norm2, ldn);
}

void launch_update_b(int dim, const BTiles &T, double *X, const void *Z, bool z_float, int64_t ldz, const int32_t *m,
                     const double *y, int ldy, hipStream_t s) {
    if (T.n == 0) return;
#define UPB(D, TZ) hipLaunchKernelGGL((k_update_b<D, TZ>), BGRID(T), T, X, (const TZ *)Z, ldz, m, y, ldy)
    if (z_float) {
        if (dim == 2) UPB(2, float); else UPB(3, float);
    } else {
        if (dim == 2) UPB(2, double); else UPB(3, double);
    }
#undef UPB
}

void launch_seg_sum(const double *partial, int n, const int32_t *first, int nvec, const uint8_t *active, double *out,
                    int B, hipStream_t s) {
    hipLaunchKernelGGL((k_seg_reduce<0, double>), dim3(B, nvec), dim3(256), 0, s, partial, n, first, nvec, active, out);
}
void launch_seg_max(const double *partial, int n, const int32_t *first, int nvec, const uint8_t *active, double *out,
                    int B, hipStream_t s) {
    hipLaunchKernelGGL((k_seg_reduce<1, double>), dim3(B, nvec), dim3(256), 0, s, partial, n, first, nvec, active, out);
}
void launch_seg_sum_i64(const int64_t *partial, int n, const int32_t *first, const uint8_t *active, int64_t *out, int B,
                        hipStream_t s) {
    hipLaunchKernelGGL((k_seg_reduce<0, int64_t>), dim3(B, 1), dim3(256), 0, s, partial, n, first, 1, active, out);
}

#undef BGRID

#define INST_T(T)                                                                                                      \
    template void launch_diag_b<T>(int, const BTiles &, const int16_t *, double, T *, hipStream_t);                    \
    template void launch_jacobi_b<T>(int, const BTiles &, const int16_t *, const T *, const T *, const T *, T *,      \
                                     double, double, bool, hipStream_t);                                              \
    template void launch_level_residual_b<T>(int, const BTiles &, const int16_t *, const T *, const T *, T *, double, \
                                             hipStream_t);                                                            \
    template void launch_restrict_b<T>(int, const BTiles &, const BInst *, const T *, T *, hipStream_t);              \
    template void launch_prolong_add_b<T>(int, const BTiles &, const BInst *, const T *, T *, hipStream_t);           \
    template void launch_coarse_b<T>(int, const int32_t *, int, int64_t, const BInst *, const uint8_t *,              \
                                     const int16_t *, const T *, const T *, T *, double, double, int, hipStream_t);
INST_T(float)
INST_T(double)
#undef INST_T

}  // namespace slhjb
