// HIP kernels of libslhjb for gfx950 (CDNA4).
//
// The operator is the truncated linear-interpolation semi-Lagrangian Scheme 2 of Reisinger &
// Rotaetxe Arto (arXiv:1605.04821): diffusion points x +- sqrt(h) s sigma_p and drift point x + h b
// (Section 1, "Examples of LISL schemes"), multilinear interpolation (eq. monotone_int), and
// truncation at the box boundary with the weights A_p, B_p of eq. eqn_Ap and C = 1/mu of
// eq. eqn_APp1 (Prop. pro:scheme2), summed as in eq. TruncScheme.
//
// Arithmetic of the FP64 operator (identical in every kernel that evaluates it):
//   displacement in cells Y; mu = min(1, min_d D_d/|Y_d|) with D_d the integer distance to the face
//   the point moves towards; if mu == 1 the landing cell is i + floor(Y) with fraction Y - floor(Y);
//   otherwise the limiting coordinate is the face index and the others i + mu*Y (clamped); a landing
//   cell n-1 becomes cell n-2 with fraction 1; interpolation is the weighted corner sum of
//   eq. monotone_int: corner weights are products over axes (in axis order) of t_d or 1 - t_d, the sum
//   is w_0 V_0 then fma(w_c, V_c, sum) in corner order; term_p = (A*v+ + B*v-) - (A+B)*V_i,
//   drift 2C*(v_b - V_i), L = (1/2h)*sum.
// Compiled without floating-point contraction: apart from the explicit fma calls these expressions
// round exactly as written.
//
// Thread mapping: one node per thread, x fastest; blocks are renumbered so that each of the eight
// XCDs (which take hardware blocks round-robin) works on one contiguous slab of rows and keeps the
// stencil halo of its slab in its own L2.

#include "slhjb_device.h"

namespace slhjb {

thread_local LaunchEvents g_launch_events;

int blocks_for(int64_t N) { return (int)((N + kBlock - 1) / kBlock); }


// ---- policy search over untruncated wavefronts ---------------------------------------------------
// When no lane of a wavefront is near the boundary, every stencil point of control k lands at the fixed
// offset of the precomputed table (constant coefficients), so the corner loads of B controls can all be
// issued before any of them is used: one memory round trip per B controls instead of one per point
// group.  The arithmetic is that of eval_G on the deep branch of lhat_node, operation for operation.

template <int DIM>
__device__ __forceinline__ void corner_loads(const double *__restrict__ V, int base, int s1, int s2, double c[8]) {
    c[0] = V[base];
    c[1] = V[base + 1];
    c[2] = V[base + s1];
    c[3] = V[base + s1 + 1];
    if (DIM == 3) {
        c[4] = V[base + s2];
        c[5] = V[base + s2 + 1];
        c[6] = V[base + s2 + s1];
        c[7] = V[base + s2 + s1 + 1];
    }
}

// the weighted corner sum of interp_w, same order
template <int DIM>
__device__ __forceinline__ double corner_sum(const double *w, const double c[8]) {
    double v = w[0] * c[0];
    v = fma(w[1], c[1], v);
    v = fma(w[2], c[2], v);
    v = fma(w[3], c[3], v);
    if (DIM == 3) {
        v = fma(w[4], c[4], v);
        v = fma(w[5], c[5], v);
        v = fma(w[6], c[6], v);
        v = fma(w[7], c[7], v);
    }
    return v;
}

// G_k for k = k0 .. k0+B-1 at a node of an untruncated wavefront (k0 wave-uniform, k0 + B <= K).
// P diffusion pairs and DRIFT are the table layout (npt = 2P + DRIFT).
template <int DIM, bool CN, int QM, int P, bool DRIFT, int B>
__device__ __forceinline__ void eval_G_deep(const LevelDev &g, const StencilDev &st, int k0, int i,
                                            const double *__restrict__ X, double Xi, const double *__restrict__ U,
                                            double Ui, double theta, double omt, double f, double *__restrict__ Q,
                                            int64_t qrow, int64_t qstride, double G[B]) {
    constexpr int NP = 2 * P + (DRIFT ? 1 : 0);
    constexpr int NC = 1 << DIM;
    constexpr bool TWO = CN && QM != 2;
    const int s1 = (int)g.s1, s2 = (int)g.s2;
    const FastPtD *fp = st.fastD + k0 * NP;
    double cx[B][NP][NC];
    double cu[TWO ? B : 1][TWO ? NP : 1][NC];
    double qv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int base = i + fp[b * NP + q].off;
            corner_loads<DIM>(X, base, s1, s2, cx[b][q]);
            if (TWO) corner_loads<DIM>(U, base, s1, s2, cu[TWO ? b : 0][TWO ? q : 0]);
        }
        if (CN && QM == 2) qv[b] = Q[(int64_t)(k0 + b) * qstride + qrow];
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int k = k0 + b;
        double accV = 0.0, accW = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double vp = corner_sum<DIM>(fp[b * NP + 2 * p].w, cx[b][2 * p]);
            double vm = corner_sum<DIM>(fp[b * NP + 2 * p + 1].w, cx[b][2 * p + 1]);
            accV = accV + ((vp + vm) - 2.0 * Xi);
            if (TWO) {
                double wp = corner_sum<DIM>(fp[b * NP + 2 * p].w, cu[TWO ? b : 0][TWO ? 2 * p : 0]);
                double wm = corner_sum<DIM>(fp[b * NP + 2 * p + 1].w, cu[TWO ? b : 0][TWO ? 2 * p + 1 : 0]);
                accW = accW + ((wp + wm) - 2.0 * Ui);
            }
        }
        if (DRIFT) {
            constexpr int QD = DRIFT ? 2 * P : 0;  // the drift point (the guard keeps the index in range)
            double vb = corner_sum<DIM>(fp[b * NP + QD].w, cx[b][QD]);
            accV = accV + 2.0 * (vb - Xi);
            if (TWO) {
                double wb = corner_sum<DIM>(fp[b * NP + QD].w, cu[TWO ? b : 0][TWO ? QD : 0]);
                accW = accW + 2.0 * (wb - Ui);
            }
        }
        const double lx = st.inv2h * accV;
        const double ck = st.c ? st.c[k] : 0.0;
        double q;
        if (CN && QM == 2) {
            q = qv[b];
        } else {
            const double lu = TWO ? st.inv2h * accW : 0.0;
            q = omt * (lu + ck * Ui);
            if (CN && QM == 1) Q[(int64_t)k * qstride + qrow] = q;
        }
        G[b] = theta * (lx + ck * Xi) + q + f;
    }
}

// the whole control loop of the search on an untruncated wavefront: best value, its control and the
// value of the node's current control, as the generic loop finds them
template <int DIM, bool CN, int QM, int P, bool DRIFT>
__device__ __forceinline__ void search_deep(const LevelDev &g, const StencilDev &st, int i, const double *__restrict__ X,
                                            double Xi, const double *__restrict__ U, double Ui, double theta,
                                            double omt, double f, double *__restrict__ Q, int64_t qrow,
                                            int64_t qstride, int cur, double &best, int &kbest, double &gcur,
                                            double &second) {
    constexpr bool TWO = CN && QM != 2;
    constexpr int B = (DIM == 2 && !TWO) ? 2 : 1;
    // second: the least G over the controls other than kbest
    auto take = [&](double G, int k) {
        const double hi = G < best ? best : G;  // the larger of the two competes for second place
        second = hi < second ? hi : second;
        if (G < best) {
            best = G;
            kbest = k;
        }
        if (k == cur) gcur = G;
    };
    int k = 0;
    for (; k + B <= st.K; k += B) {
        double G[B];
        eval_G_deep<DIM, CN, QM, P, DRIFT, B>(g, st, k, i, X, Xi, U, Ui, theta, omt, f, Q, qrow, qstride, G);
#pragma unroll
        for (int b = 0; b < B; ++b) take(G[b], k + b);
    }
    for (; k < st.K; ++k) {
        double G[1];
        eval_G_deep<DIM, CN, QM, P, DRIFT, 1>(g, st, k, i, X, Xi, U, Ui, theta, omt, f, Q, qrow, qstride, G);
        take(G[0], k);
    }
}

// PN: per-node coefficients or per-control sources; otherwise those fields are known to be zero here,
// so the constant-coefficient search compiles without their code (and keeps its register budget).
// NEAR: also count near ties (the runner-up within kNearTie * tau of the best); a separate instantiation
// because keeping the runner-up alive costs the search a wave of occupancy.
template <int DIM, bool CN, bool EXTRA, int QM, bool PN, bool NEAR = false>
__global__ __launch_bounds__(kBlock) void k_sweep(LevelDev g, StencilDev st0, const double *__restrict__ X,
                                                  const double *__restrict__ U, const double *__restrict__ f0,
                                                  const double *__restrict__ f1, double t_mid, double theta,
                                                  const double *__restrict__ tau_p, const int16_t *a_in,
                                                  SweepOut o, double *__restrict__ Q) {
    __shared__ int64_t sh[kBlock / 64];
    StencilDev st = st0;
    if (!PN) {
        st.xs = 0;
        st.field = 0;
        st.pernode = 0;
        st.fk = 0;
    }
    const double tau = tau_p[0];  // written by the tolerance kernel just before
    // the tile of this block: its remapped position, or (with a work list) the list entry of this block's
    // share, each XCD taking an equal contiguous part of the list
    int tile;
    if (o.list) {
        // the grid is a multiple of 8 blocks with at least as many as there are tiles, so every XCD has
        // ceil(tiles / 8) >= c8 blocks
        const int cnt = o.list_count[0], c8 = (cnt + 7) >> 3;
        const int t = (int)(blockIdx.x >> 3), j = (int)(blockIdx.x & 7) * c8 + t;
        if (t >= c8 || j >= cnt) return;
        tile = o.list[j];
    } else {
        tile = remap_block(blockIdx.x, gridDim.x);
    }
    const int64_t qslot = (int64_t)tile * kBlock + threadIdx.x;
    const int64_t qstride = (int64_t)g.ntx * g.nty * g.ntz * kBlock;  // tiles of the grid, list or not
    int ix[3];
    int i = tile_node_at<DIM>(g, tile, ix);
    int64_t changed = 0, near = 0;
    // re-evaluations read the cache this thread has just written
    constexpr int QM2 = QM == 1 ? 2 : QM;
    if (i >= 0) {
        if (!interior<DIM>(g, ix)) {
            o.alpha_out[i] = -1;
            if (o.gmin) o.gmin[i] = 0.0;
            if (EXTRA) {
                if (o.margin) o.margin[i] = __builtin_inf();
                if (o.ties) o.ties[i] = 0;
            }
        } else {
            bool deep = deep_node<DIM>(g, ix);
            const int cur = a_in[i];
            // untruncated wavefront, constant coefficients, one diffusion pair: the pipelined loop
            int fast = 0;
            if (!PN && st.fastD && st.P == 1 && __all(deep)) fast = st.has_drift ? 3 : 2;
            // a wavefront whose decisions the certification pass kept: its controls are already in place
            // (the search then runs in place) and its gap bounds are updated; no store on this path, so
            // the tables of the search below stay scalar reads
            const bool keep = !EXTRA && fast && o.skip == 2 && o.keep[tile * (kBlock / 64) + (threadIdx.x >> 6)];
            if (!keep) {
                double Xi = X[i], Ui = U[i];
                const double f = f0[i] + t_mid * f1[i];
                // the source of control k (one source for all controls unless st.fk != 0)
                auto fk = [&](int k) { return st.fk ? f0[k * st.fk + i] + t_mid * f1[k * st.fk + i] : f; };
                double omt = 1.0 - theta;
                double best = __builtin_inf(), gcur = __builtin_inf(), second = __builtin_inf();
                int kbest = 0;
                if (fast == 3)
                    search_deep<DIM, CN, QM, 1, true>(g, st, i, X, Xi, U, Ui, theta, omt, f, Q, qslot, qstride, cur, best,
                                                      kbest, gcur, second);
                else if (fast == 2)
                    search_deep<DIM, CN, QM, 1, false>(g, st, i, X, Xi, U, Ui, theta, omt, f, Q, qslot, qstride, cur, best,
                                                       kbest, gcur, second);
                else
                    for (int k = 0; k < st.K; ++k) {
                        double G = eval_G<DIM, CN, QM>(g, st, k, i, ix, deep, X, Xi, U, Ui, theta, omt, fk(k), Q, qslot, qstride);
                        if (NEAR) {
                            const double hi = G < best ? best : G;  // second: the least G of the other controls
                            second = hi < second ? hi : second;
                        }
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
                        double G = eval_G<DIM, CN, QM2>(g, st, k, i, ix, deep, X, Xi, U, Ui, theta, omt, fk(k), Q, qslot, qstride);
                        if (G <= thr) {
                            pick = k;
                            break;
                        }
                    }
                }
                o.alpha_out[i] = (int16_t)pick;
                if (!EXTRA && o.skip) o.marg[i] = (fast && pick == kbest) ? second - best : -1.0;
                changed = (pick != cur) ? 1 : 0;
                if (NEAR) near = (second - best < kNearTie * tau) ? 1 : 0;
                if (o.gmin) o.gmin[i] = best;
                if (EXTRA) {
                    double mg = __builtin_inf();
                    int nt = 0;
                    for (int k = 0; k < st.K; ++k) {
                        double G = eval_G<DIM, CN, QM2>(g, st, k, i, ix, deep, X, Xi, U, Ui, theta, omt, fk(k), Q, qslot, qstride);
                        if (G <= thr)
                            ++nt;
                        else if (G - best < mg)
                            mg = G - best;
                    }
                    if (o.margin) o.margin[i] = mg;
                    if (o.ties) o.ties[i] = nt;
                }
            }
        }
    }
    // changed controls in the low 32 bits, near ties in the high ones (either count is below 2^32)
    int64_t tot = block_reduce<int64_t>(changed | (near << 32), OpSum(), sh);
    if (threadIdx.x == 0) o.changed_partial[tile] = tot;
}

template <int DIM>
void launch_sweep_dim(const LevelDev &g, const StencilDev &st, const double *X, const double *U, const double *f0,
                      const double *f1, double t_mid, double theta, const double *tau, const int16_t *a_in,
                      const SweepOut &o, double *Q, int qmode, int nblocks, hipStream_t s) {
    bool cn = theta != 1.0;
    bool extra = o.margin != nullptr || o.ties != nullptr;
    const bool pn = st.pernode || st.fk;
    // with a work list, whole groups of 8 blocks (one per XCD) cover the tiles
    const int grid = o.list ? (tiles_for(g) + 7) / 8 * 8 : tiles_for(g);
    // near ties are counted on request by the lean (no per-node extras) searches
    const bool near = o.count_near && !extra;
#define SW(C, E, QQ)                                                                                                  \
    do {                                                                                                              \
        if (pn && near)                                                                                               \
            SLHJB_LAUNCH((k_sweep<DIM, C, E, QQ, true, !E>), dim3(grid), dim3(kBlock), 0, s, g, st, X, U, f0, f1,     \
                         t_mid, theta, tau, a_in, o, Q);                                                              \
        else if (pn)                                                                                                  \
            SLHJB_LAUNCH((k_sweep<DIM, C, E, QQ, true>), dim3(grid), dim3(kBlock), 0, s, g, st, X, U, f0, f1,         \
                         t_mid, theta, tau, a_in, o, Q);                                                              \
        else if (near)                                                                                                \
            SLHJB_LAUNCH((k_sweep<DIM, C, E, QQ, false, !E>), dim3(grid), dim3(kBlock), 0, s, g, st, X, U, f0, f1,    \
                         t_mid, theta, tau, a_in, o, Q);                                                              \
        else                                                                                                          \
            SLHJB_LAUNCH((k_sweep<DIM, C, E, QQ, false>), dim3(grid), dim3(kBlock), 0, s, g, st, X, U, f0, f1,        \
                         t_mid, theta, tau, a_in, o, Q);                                                              \
    } while (0)
    if (!cn) {
        if (extra) SW(false, true, 0); else SW(false, false, 0);
    } else if (qmode == 1) {
        if (extra) SW(true, true, 1); else SW(true, false, 1);
    } else if (qmode == 2) {
        if (extra) SW(true, true, 2); else SW(true, false, 2);
    } else {
        if (extra) SW(true, true, 0); else SW(true, false, 0);
    }
#undef SW
}

void launch_sweep(int dim, const LevelDev &g, const StencilDev &st, const double *X, const double *U,
                  const double *f0, const double *f1, double t_mid, double theta, const double *tau,
                  const int16_t *a_in, const SweepOut &o, double *Q, int qmode, int nblocks, hipStream_t s) {
    if (dim == 2)
        launch_sweep_dim<2>(g, st, X, U, f0, f1, t_mid, theta, tau, a_in, o, Q, qmode, nblocks, s);
    else
        launch_sweep_dim<3>(g, st, X, U, f0, f1, t_mid, theta, tau, a_in, o, Q, qmode, nblocks, s);
}

// max over all nodes of max(|X|,|U|) and over interior nodes of |f0 + t_mid f1|
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_norms_xuf(LevelDev g, const double *__restrict__ X,
                                                      const double *__restrict__ U, const double *__restrict__ f0,
                                                      const double *__restrict__ f1, double t_mid, int K, int64_t fk,
                                                      double *partial) {
    __shared__ double sh[kBlock / 64];
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    double vx = 0.0, vf = 0.0;
    if (i >= 0) {
        vx = OpMax()(fabs(X[i]), fabs(U[i]));  // a NaN wins
        if (interior<DIM>(g, ix)) {
            if (fk == 0)
                vf = fabs(f0[i] + t_mid * f1[i]);
            else
                for (int k = 0; k < K; ++k) vf = OpMax()(vf, fabs(f0[k * fk + i] + t_mid * f1[k * fk + i]));
        }
    }
    int b = remap_block(blockIdx.x, gridDim.x);
    double a = block_reduce<double>(vx, OpMax(), sh);
    if (threadIdx.x == 0) partial[b] = a;
    double c = block_reduce<double>(vf, OpMax(), sh);
    if (threadIdx.x == 0) partial[gridDim.x + b] = c;
}

void launch_norms_xuf(int dim, const LevelDev &g, const double *X, const double *U, const double *f0, const double *f1,
                      double t_mid, int K, int64_t fk, double *partial, int nblocks, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_norms_xuf<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, X, U, f0, f1, t_mid, K, fk,
                           partial);
    else
        hipLaunchKernelGGL(k_norms_xuf<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, X, U, f0, f1, t_mid, K, fk,
                           partial);
}

// ---- FP64 operator kernels ------------------------------------------------------------------------

template <int DIM, typename TX>
__global__ __launch_bounds__(kBlock) void k_apply(LevelDev g, StencilDev st0, const int16_t *__restrict__ alpha,
                                                  const TX *__restrict__ x, double *__restrict__ y, double theta_dt,
                                                  double *norm2_partial) {
    __shared__ double sh[kBlock / 64];
    const StencilDev &st = st0;
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    double yy = 0.0;
    if (i >= 0) {
        if (interior<DIM>(g, ix)) {
            int k = alpha[i];
            bool deep = deep_node<DIM>(g, ix);
            double xi = (double)x[i];
            double l = lhat1<DIM, TX, double>(g, st, k, i, ix, deep, x, xi);
            double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
            yy = xi - theta_dt * (l + ck * xi);
        }
        y[i] = yy;
    }
    if (norm2_partial) {
        double t = block_reduce<double>(yy * yy, OpSum(), sh);
        if (threadIdx.x == 0) norm2_partial[remap_block(blockIdx.x, gridDim.x)] = t;
    }
}

void launch_apply(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const void *x,
                  bool x_is_float, double *y, double theta_dt, double *norm2_partial, int nblocks, hipStream_t s) {
#define AP(D, TX) SLHJB_LAUNCH((k_apply<D, TX>), dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, \
                               (const TX *)x, y, theta_dt, norm2_partial)
    if (x_is_float) {
        if (dim == 2) AP(2, float); else AP(3, float);
    } else {
        if (dim == 2) AP(2, double); else AP(3, double);
    }
#undef AP
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_explicit(LevelDev g, StencilDev st0, const int16_t *__restrict__ alpha,
                                                     const double *__restrict__ U, const double *__restrict__ f0,
                                                     const double *__restrict__ f1, double t_mid, double omt_dt,
                                                     double dt, double *__restrict__ E) {
    const StencilDev &st = st0;
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    if (i < 0) return;
    double e = 0.0;
    if (interior<DIM>(g, ix)) {
        const int64_t fo = st.fk ? (int64_t)(((unsigned)alpha[i] < (unsigned)st.K) ? alpha[i] : 0) * st.fk : 0;
        double f = f0[fo + i] + t_mid * f1[fo + i];
        double Ui = U[i];
        if (omt_dt != 0.0) {
            int k = alpha[i];
            bool deep = deep_node<DIM>(g, ix);
            double l = lhat1<DIM, double, double>(g, st, k, i, ix, deep, U, Ui);
            double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
            e = Ui + omt_dt * (l + ck * Ui) + dt * f;
        } else {
            e = Ui + dt * f;
        }
    }
    E[i] = e;
}

void launch_explicit(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const double *U,
                     const double *f0, const double *f1, double t_mid, double omt_dt, double dt, double *E, int nblocks,
                     hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_explicit<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, U, f0, f1, t_mid, omt_dt,
                           dt, E);
    else
        hipLaunchKernelGGL(k_explicit<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, U, f0, f1, t_mid, omt_dt,
                           dt, E);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual(LevelDev g, StencilDev st0, const int16_t *__restrict__ alpha,
                                                     const double *__restrict__ V, const double *__restrict__ E,
                                                     double theta_dt, double *__restrict__ r, double *partial) {
    __shared__ double sh[kBlock / 64];
    const StencilDev &st = st0;
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    double rr = 0.0, vv = 0.0;
    if (i >= 0) {
        double Vi = V[i];
        vv = fabs(Vi);
        if (interior<DIM>(g, ix)) {
            int k = alpha[i];
            const double Ei = E[i];  // requested before the stencil gathers
            bool deep = deep_node<DIM>(g, ix);
            double l = lhat1<DIM, double, double>(g, st, k, i, ix, deep, V, Vi);
            double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
            rr = Ei - (Vi - theta_dt * (l + ck * Vi));
        }
        r[i] = rr;
    }
    int b = remap_block(blockIdx.x, gridDim.x);
    double s2 = block_reduce<double>(rr * rr, OpSum(), sh);
    if (threadIdx.x == 0) partial[b] = s2;
    double m = block_reduce<double>(fabs(rr), OpMax(), sh);
    if (threadIdx.x == 0) partial[gridDim.x + b] = m;
    double mv = block_reduce<double>(vv, OpMax(), sh);
    if (threadIdx.x == 0) partial[2 * gridDim.x + b] = mv;
}

void launch_residual(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const double *V,
                     const double *E, double theta_dt, double *r, double *partial, int nblocks, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_residual<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, V, E, theta_dt, r, partial);
    else
        hipLaunchKernelGGL(k_residual<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, V, E, theta_dt, r, partial);
}

// number of interior nodes whose control index is outside [0, K)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_bad_policy(LevelDev g, const int16_t *__restrict__ alpha, int K,
                                                       int64_t *partial) {
    __shared__ int64_t sh[kBlock / 64];
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    int64_t bad = 0;
    if (i >= 0) {
        if (interior<DIM>(g, ix)) {
            int k = alpha[i];
            bad = (k < 0 || k >= K) ? 1 : 0;
        }
    }
    int64_t t = block_reduce<int64_t>(bad, OpSum(), sh);
    if (threadIdx.x == 0) partial[remap_block(blockIdx.x, gridDim.x)] = t;
}

void launch_bad_policy(int dim, const LevelDev &g, const int16_t *alpha, int K, int64_t *partial, int nblocks,
                       hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_bad_policy<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, alpha, K, partial);
    else
        hipLaunchKernelGGL(k_bad_policy<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, alpha, K, partial);
}

// ---- multigrid level kernels ----------------------------------------------------------------------

// Sum over the stencil points of control k of W (w_self - 1) at node ix: the diagonal of L-hat before the
// 1/(2h) scaling (W: the point's weight after truncation, w_self: its interpolation weight on the node).
template <int DIM>
__device__ double diag_lii(const LevelDev &g, const StencilDev &st, int k, const int ix[3], int i) {
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
    return lii;
}

// diagonal of A = I - theta dt (L-hat + c) on one level: d = 1 - theta dt (l_ii + c).  At deep nodes of the
// constant-coefficient model no point is truncated and every displacement is the table's, so l_ii is the
// per-control value diag_lii gives at any deep node (same operations, same rounding): read from the table.
// With wctl (constant coefficients, per-control deep values available): also the wave-control table of this
// level and policy, wctl[tile * 4 + wave] = the control shared by all 64 nodes of the wavefront when every one
// of them is an untruncated interior node, else -1, and dk[k] = the diagonal at untruncated nodes of control k
// (the same operations as d[i] there, so dk[alpha_i] == d[i] bit for bit).  The node kernels then read neither
// the policy nor the diagonal on such wavefronts.
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_diag(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                 double theta_dt, T *__restrict__ d, int16_t *__restrict__ wctl,
                                                 T *__restrict__ dk) {
    const int tile = remap_block(blockIdx.x, gridDim.x);
    int ix[3];
    const int i = tile_node_at<DIM>(g, tile, ix);
    int k = -1;
    bool uni = false;  // an untruncated interior node (its diagonal is the per-control value)
    if (i >= 0) {
        if (!interior<DIM>(g, ix)) {
            d[i] = (T)1;
        } else {
            k = alpha[i];
            k = ((unsigned)k < (unsigned)st.K) ? k : 0;
            uni = st.lii_deep && deep_node<DIM>(g, ix);
            double lii = uni ? st.lii_deep[k] : diag_lii<DIM>(g, st, k, ix, i);
            lii *= st.inv2h;
            double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
            d[i] = (T)(1.0 - theta_dt * (lii + ck));
        }
    }
    if (wctl) {
        // every lane takes part: lanes outside the grid make the wavefront non-uniform
        const int k0 = __shfl(k, 0, 64);
        const bool all = __all(uni && k == k0);
        if ((threadIdx.x & 63) == 0) wctl[tile * (kBlock / 64) + (threadIdx.x >> 6)] = all ? (int16_t)k0 : (int16_t)-1;
        if (blockIdx.x == 0)
            for (int q = threadIdx.x; q < st.K; q += blockDim.x) {
                double lii = st.lii_deep[q];
                lii *= st.inv2h;
                double ck = st.c ? st.c[q] : 0.0;
                dk[q] = (T)(1.0 - theta_dt * (lii + ck));
            }
    }
}

template <int DIM>
__global__ void k_lii_deep(LevelDev g, StencilDev st, int x0, int x1, int x2, double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= st.K) return;
    const int ix[3] = {x0, x1, x2};
    const int i = x0 + x1 * (int)g.s1 + (DIM == 3 ? x2 * (int)g.s2 : 0);
    out[k] = diag_lii<DIM>(g, st, k, ix, i);
}

void launch_lii_deep(int dim, const LevelDev &g, const StencilDev &st, const int ix0[3], double *out, hipStream_t s) {
    const int nb = (st.K + 63) / 64;
    if (dim == 2)
        hipLaunchKernelGGL(k_lii_deep<2>, dim3(nb), dim3(64), 0, s, g, st, ix0[0], ix0[1], ix0[2], out);
    else
        hipLaunchKernelGGL(k_lii_deep<3>, dim3(nb), dim3(64), 0, s, g, st, ix0[0], ix0[1], ix0[2], out);
}

template <typename T>
void launch_diag(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, double theta_dt, T *d,
                 hipStream_t s, int16_t *wctl, T *dk) {
    int nb = tiles_for(g);
    if (!st.lii_deep) wctl = nullptr;
    if (dim == 2)
        hipLaunchKernelGGL((k_diag<2, T>), dim3(nb), dim3(kBlock), 0, s, g, st, alpha, theta_dt, d, wctl, dk);
    else
        hipLaunchKernelGGL((k_diag<3, T>), dim3(nb), dim3(kBlock), 0, s, g, st, alpha, theta_dt, d, wctl, dk);
}

template <int DIM, typename T>
__device__ __forceinline__ T apply_level(const LevelDev &g, const StencilDev &st, const int16_t *__restrict__ alpha,
                                         const T *__restrict__ e, int i, const int ix[3], T theta_dt) {
    int k = alpha[i];
    bool deep = deep_node<DIM>(g, ix);
    T ei = e[i];
    T l = lhat1<DIM, T, T>(g, st, k, i, ix, deep, e, ei);
    T ck = st.c ? (T)st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : (T)0;
    return ei - theta_dt * (l + ck * ei);
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(DIM == 2 ? 8 : 1))) void k_jacobi(LevelDev g, StencilDev st0, const int16_t *__restrict__ alpha,
                                                   const T *__restrict__ e, const T *__restrict__ r,
                                                   const T *__restrict__ d, T *__restrict__ e_out, T theta_dt, T omega,
                                                   int first, const int16_t *__restrict__ wctl,
                                                   const T *__restrict__ dk) {
    const StencilDev &st = st0;
    const int tile = remap_block(blockIdx.x, gridDim.x);
    int ix[3];
    int i = tile_node_at<DIM>(g, tile, ix);
    if (i < 0) return;
    T v = (T)0;
    const int wc = wave_control(wctl, tile);
    if (wc >= 0) {
        // a wavefront of untruncated interior nodes with one control: the control and the diagonal come from
        // the tables (the same values the per-node path reads), the arithmetic is that path's
        const T di = dk[wc];
        if (first) {
            v = omega * r[i] / di;
        } else {
            const T ei = e[i], ri = r[i];
            const double ck = st.c ? st.c[wc] : 0.0;
            T l, unused;
            lhat_node<DIM, T, T, false>(g, st, wc, i, ix, true, e, ei, e, ei, l, unused);
            const T ae = ei - theta_dt * (l + (T)ck * ei);
            v = ei + omega * (ri - ae) / di;
        }
    } else if (interior<DIM>(g, ix)) {
        if (first) {
            v = omega * r[i] / d[i];
        } else {
            // the operands that do not depend on the stencil are requested before its gathers, so that
            // their latency overlaps them (the arithmetic is that of apply_level)
            const int k = alpha[i];
            const T ei = e[i], ri = r[i], di = d[i];
            const double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;  // converted at its use
            const T l = lhat1<DIM, T, T>(g, st, k, i, ix, deep_node<DIM>(g, ix), e, ei);
            const T ae = ei - theta_dt * (l + (T)ck * ei);
            v = ei + omega * (ri - ae) / di;
        }
    }
    e_out[i] = v;
}

template <typename T>
void launch_jacobi(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const T *e, const T *r,
                   const T *d, T *e_out, double theta_dt, double omega, bool first, hipStream_t s,
                   const int16_t *wctl, const T *dk) {
    int nb = tiles_for(g);
    if (dim == 2)
        SLHJB_LAUNCH((k_jacobi<2, T>), dim3(nb), dim3(kBlock), 0, s, g, st, alpha, e, r, d, e_out, (T)theta_dt,
                     (T)omega, (int)first, wctl, dk);
    else
        SLHJB_LAUNCH((k_jacobi<3, T>), dim3(nb), dim3(kBlock), 0, s, g, st, alpha, e, r, d, e_out, (T)theta_dt,
                     (T)omega, (int)first, wctl, dk);
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(DIM == 2 ? 8 : 1))) void k_level_residual(LevelDev g, StencilDev st0, const int16_t *__restrict__ alpha,
                                                           const T *__restrict__ e, const T *__restrict__ r,
                                                           T *__restrict__ res, T theta_dt,
                                                           const int16_t *__restrict__ wctl) {
    const StencilDev &st = st0;
    const int tile = remap_block(blockIdx.x, gridDim.x);
    int ix[3];
    int i = tile_node_at<DIM>(g, tile, ix);
    if (i < 0) return;
    T v = (T)0;
    const int wc = wave_control(wctl, tile);
    if (wc >= 0) {
        const T ei = e[i], ri = r[i];
        const double ck = st.c ? st.c[wc] : 0.0;
        T l, unused;
        lhat_node<DIM, T, T, false>(g, st, wc, i, ix, true, e, ei, e, ei, l, unused);
        v = ri - (ei - theta_dt * (l + (T)ck * ei));
    } else if (interior<DIM>(g, ix)) {
        const int k = alpha[i];
        const T ei = e[i], ri = r[i];
        const double ck = st.c ? st.c[((unsigned)k < (unsigned)st.K) ? k : 0] : 0.0;
        const T l = lhat1<DIM, T, T>(g, st, k, i, ix, deep_node<DIM>(g, ix), e, ei);
        v = ri - (ei - theta_dt * (l + (T)ck * ei));
    }
    res[i] = v;
}

template <typename T>
void launch_level_residual(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const T *e,
                           const T *r, T *res, double theta_dt, hipStream_t s, const int16_t *wctl) {
    int nb = tiles_for(g);
    if (dim == 2)
        SLHJB_LAUNCH((k_level_residual<2, T>), dim3(nb), dim3(kBlock), 0, s, g, st, alpha, e, r, res,
                     (T)theta_dt, wctl);
    else
        SLHJB_LAUNCH((k_level_residual<3, T>), dim3(nb), dim3(kBlock), 0, s, g, st, alpha, e, r, res,
                     (T)theta_dt, wctl);
}

// full weighting: weights 1/4, 1/2, 1/4 per axis around fine node 2I
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelDev gf, LevelDev gc, const T *__restrict__ rf,
                                                     T *__restrict__ rc) {
    int ix[3];
    int I = tile_node<DIM>(gc, ix);
    if (I < 0) return;
    T v = (T)0;
    if (interior<DIM>(gc, ix)) {
        int c = 2 * ix[0] + 2 * ix[1] * (int)gf.s1 + (DIM == 3 ? 2 * ix[2] * (int)gf.s2 : 0);
        const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
        if (DIM == 2) {
            for (int b = -1; b <= 1; ++b) {
                T row = w[0] * rf[c + b * (int)gf.s1 - 1] + w[1] * rf[c + b * (int)gf.s1] + w[2] * rf[c + b * (int)gf.s1 + 1];
                v += w[b + 1] * row;
            }
        } else {
            for (int cc = -1; cc <= 1; ++cc) {
                T pl = (T)0;
                for (int b = -1; b <= 1; ++b) {
                    int o = c + cc * (int)gf.s2 + b * (int)gf.s1;
                    T row = w[0] * rf[o - 1] + w[1] * rf[o] + w[2] * rf[o + 1];
                    pl += w[b + 1] * row;
                }
                v += w[cc + 1] * pl;
            }
        }
    }
    rc[I] = v;
}

template <typename T>
void launch_restrict(int dim, const LevelDev &gf, const LevelDev &gc, const T *rf, T *rc, hipStream_t s) {
    int nb = tiles_for(gc);
    if (dim == 2)
        hipLaunchKernelGGL((k_restrict<2, T>), dim3(nb), dim3(kBlock), 0, s, gf, gc, rf, rc);
    else
        hipLaunchKernelGGL((k_restrict<3, T>), dim3(nb), dim3(kBlock), 0, s, gf, gc, rf, rc);
}

// multilinear prolongation of the coarse correction, added on fine interior nodes
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(LevelDev gf, LevelDev gc, const T *__restrict__ ec,
                                                        T *__restrict__ ef) {
    int ix[3];
    int i = tile_node<DIM>(gf, ix);
    if (i < 0) return;
    if (!interior<DIM>(gf, ix)) return;
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
    const int s1 = (int)gc.s1, s2 = (int)gc.s2;
    T v;
    auto at = [&](int a, int b, int c) { return ec[a + b * s1 + (DIM == 3 ? c * s2 : 0)]; };
    T a0 = wl[0] * at(lo[0], lo[1], lo[2]) + wh[0] * at(hi[0], lo[1], lo[2]);
    T a1 = wl[0] * at(lo[0], hi[1], lo[2]) + wh[0] * at(hi[0], hi[1], lo[2]);
    v = wl[1] * a0 + wh[1] * a1;
    if (DIM == 3) {
        T b0 = wl[0] * at(lo[0], lo[1], hi[2]) + wh[0] * at(hi[0], lo[1], hi[2]);
        T b1 = wl[0] * at(lo[0], hi[1], hi[2]) + wh[0] * at(hi[0], hi[1], hi[2]);
        v = wl[2] * v + wh[2] * (wl[1] * b0 + wh[1] * b1);
    }
    ef[i] += v;
}

template <typename T>
void launch_prolong_add(int dim, const LevelDev &gf, const LevelDev &gc, const T *ec, T *ef, hipStream_t s) {
    int nb = tiles_for(gf);
    if (dim == 2)
        hipLaunchKernelGGL((k_prolong_add<2, T>), dim3(nb), dim3(kBlock), 0, s, gf, gc, ec, ef);
    else
        hipLaunchKernelGGL((k_prolong_add<3, T>), dim3(nb), dim3(kBlock), 0, s, gf, gc, ec, ef);
}

// Coarsest level: Jacobi sweeps by one workgroup with the iterate held in LDS.
template <int DIM, typename T>
__global__ __launch_bounds__(1024) void k_coarse_solve(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                       const T *__restrict__ r, const T *__restrict__ d,
                                                       T *__restrict__ e, T theta_dt, T omega, int sweeps) {
    extern __shared__ unsigned char smem[];
    T *a = reinterpret_cast<T *>(smem);
    T *b = a + g.N;
    const int N = (int)g.N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        int ix[3];
        unflatten<DIM>(g, i, ix);
        a[i] = interior<DIM>(g, ix) ? omega * r[i] / d[i] : (T)0;
    }
    __syncthreads();
    for (int sw = 1; sw < sweeps; ++sw) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            int ix[3];
            unflatten<DIM>(g, i, ix);
            T v = (T)0;
            if (interior<DIM>(g, ix)) {
                T ae = apply_level<DIM, T>(g, st, alpha, a, i, ix, theta_dt);
                v = a[i] + omega * (r[i] - ae) / d[i];
            }
            b[i] = v;
        }
        __syncthreads();
        T *tmp = a;
        a = b;
        b = tmp;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) e[i] = a[i];
}

template <typename T>
void launch_coarse_solve(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const T *r,
                         const T *d, T *e, T *tmp, double theta_dt, double omega, int sweeps, hipStream_t s) {
    (void)tmp;
    size_t shm = 2 * (size_t)g.N * sizeof(T);
    if (dim == 2)
        hipLaunchKernelGGL((k_coarse_solve<2, T>), dim3(1), dim3(1024), shm, s, g, st, alpha, r, d, e, (T)theta_dt,
                           (T)omega, sweeps);
    else
        hipLaunchKernelGGL((k_coarse_solve<3, T>), dim3(1), dim3(1024), shm, s, g, st, alpha, r, d, e, (T)theta_dt,
                           (T)omega, sweeps);
}

// ---- bookkeeping of the certified decision reuse ---------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_delta_tiles(LevelDev g, const double *__restrict__ X,
                                                        double *__restrict__ Xs, double *__restrict__ dtile,
                                                        int record) {
    __shared__ double sh[kBlock / 64];
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    double d = 0.0;
    if (i >= 0) {
        const double x = X[i];
        d = fabs(x - Xs[i]);
        d = (d == d) ? d : __builtin_inf();  // a NaN change is unbounded
        Xs[i] = x;
    }
    if (record) return;
    d = block_reduce<double>(d, OpMax(), sh);
    if (threadIdx.x == 0) dtile[remap_block(blockIdx.x, gridDim.x)] = d;
}

void launch_delta_tiles(int dim, const LevelDev &g, const double *X, double *Xs, double *dtile, bool record,
                        hipStream_t s) {
    int nb = tiles_for(g);
    if (dim == 2)
        hipLaunchKernelGGL(k_delta_tiles<2>, dim3(nb), dim3(kBlock), 0, s, g, X, Xs, dtile, (int)record);
    else
        hipLaunchKernelGGL(k_delta_tiles<3>, dim3(nb), dim3(kBlock), 0, s, g, X, Xs, dtile, (int)record);
}

// tiles are (1 << tlog) x (kBlock >> tlog) x 1 nodes: the stencil window of tile (bx, by, bz) reaches
// ceil(R/width) tiles along x, ceil(R/height) along y and R slabs along z
__global__ __launch_bounds__(kBlock) void k_window_max(LevelDev g, const double *__restrict__ dtile,
                                                       double *__restrict__ dwin, int rx, int ry, int rz) {
    const int T = blockIdx.x * blockDim.x + threadIdx.x;
    const int ntiles = g.ntx * g.nty * g.ntz;
    if (T >= ntiles) return;
    const int bx = T % g.ntx, r = T / g.ntx, by = r % g.nty, bz = r / g.nty;
    const int x0 = max(bx - rx, 0), x1 = min(bx + rx, g.ntx - 1);
    const int y0 = max(by - ry, 0), y1 = min(by + ry, g.nty - 1);
    const int z0 = max(bz - rz, 0), z1 = min(bz + rz, g.ntz - 1);
    double m = 0.0;
    for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const double v = dtile[x + g.ntx * (y + g.nty * z)];
                m = (v > m || v != v) ? v : m;
            }
    dwin[T] = m;
}

void launch_window_max(int dim, const LevelDev &g, const double *dtile, double *dwin, const int R[3], hipStream_t s) {
    const int tw = 1 << g.tlog, th = kBlock >> g.tlog;
    const int rx = (R[0] + tw - 1) / tw, ry = (R[1] + th - 1) / th, rz = dim == 3 ? R[2] : 0;
    const int ntiles = g.ntx * g.nty * g.ntz;
    hipLaunchKernelGGL(k_window_max, dim3((ntiles + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, dtile, dwin, rx, ry,
                       rz);
}

// Certification of the decisions of the next search (constant coefficients, one diffusion pair): a
// wavefront whose interior nodes are all untruncated keeps its controls when every recorded gap, less
// the largest change of G since (lip2 times the window change of X), stays above the rounding slack.
// keep[wave] tells the search; kept nodes get the reduced bound.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_keep_pass(LevelDev g, double *__restrict__ marg,
                                                      const double *__restrict__ dwin, double lip2,
                                                      const double *__restrict__ scale, uint8_t *__restrict__ keep,
                                                      int64_t *__restrict__ kept_partial, uint8_t *__restrict__ need,
                                                      int64_t *__restrict__ changed_partial) {
    __shared__ int64_t sh[kBlock / 64];
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    const int tile = remap_block(blockIdx.x, gridDim.x);
    const bool inter = i >= 0 && interior<DIM>(g, ix);
    const bool deep = inter && deep_node<DIM>(g, ix);
    double lim = 0.0;
    bool ok = false;
    if (deep) {
        lim = marg[i] - lip2 * dwin[tile];
        ok = lim > kSkipSlack * scale[0];
    }
    const uint64_t bi = __ballot(inter), bd = __ballot(deep), bk = __ballot(ok);
    const bool wk = bi != 0 && bd == bi && bk == bi;
    if (wk && inter) marg[i] = lim;
    if ((threadIdx.x & 63) == 0) keep[tile * (kBlock / 64) + (threadIdx.x >> 6)] = wk ? 1 : 0;
    // the search visits the tile unless every wavefront is kept or has no interior node
    const int any = __syncthreads_or((bi != 0 && !wk) ? 1 : 0);
    const int64_t tot = block_reduce<int64_t>((wk && inter) ? 1 : 0, OpSum(), sh);
    if (threadIdx.x == 0) {
        kept_partial[tile] = tot;
        need[tile] = any ? 1 : 0;
        changed_partial[tile] = 0;  // the search rewrites it for the tiles it visits
    }
}

void launch_keep_pass(int dim, const LevelDev &g, double *marg, const double *dwin, double lip2, const double *scale,
                      uint8_t *keep, int64_t *kept_partial, uint8_t *need, int64_t *changed_partial, hipStream_t s) {
    int nb = tiles_for(g);
    if (dim == 2)
        hipLaunchKernelGGL(k_keep_pass<2>, dim3(nb), dim3(kBlock), 0, s, g, marg, dwin, lip2, scale, keep,
                           kept_partial, need, changed_partial);
    else
        hipLaunchKernelGGL(k_keep_pass<3>, dim3(nb), dim3(kBlock), 0, s, g, marg, dwin, lip2, scale, keep,
                           kept_partial, need, changed_partial);
}

// list[0 .. count) = the tiles with need[t] != 0, in increasing order (one workgroup)
__global__ __launch_bounds__(1024) void k_tile_list(const uint8_t *__restrict__ need, int nt, int32_t *__restrict__ list,
                                                    int32_t *__restrict__ count) {
    __shared__ int sh[1024];
    const int per = (nt + (int)blockDim.x - 1) / (int)blockDim.x;
    const int b0 = (int)threadIdx.x * per, b1 = min(b0 + per, nt);
    int c = 0;
    for (int b = b0; b < b1; ++b) c += need[b] ? 1 : 0;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        const int v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int pos = sh[threadIdx.x] - c;
    for (int b = b0; b < b1; ++b)
        if (need[b]) list[pos++] = b;
    if (threadIdx.x == blockDim.x - 1) count[0] = sh[threadIdx.x];
}

void launch_tile_list(const uint8_t *need, int nt, int32_t *list, int32_t *count, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_list, dim3(1), dim3(1024), 0, s, need, nt, list, count);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_inject_policy(LevelDev gf, LevelDev gc, const int16_t *__restrict__ af,
                                                          int16_t *__restrict__ ac) {
    int ix[3];
    int I = tile_node<DIM>(gc, ix);
    if (I < 0) return;
    int16_t v = -1;
    if (interior<DIM>(gc, ix)) v = af[2 * ix[0] + 2 * ix[1] * (int)gf.s1 + (DIM == 3 ? 2 * ix[2] * (int)gf.s2 : 0)];
    ac[I] = v;
}

void launch_inject_policy(int dim, const LevelDev &gf, const LevelDev &gc, const int16_t *af, int16_t *ac,
                          hipStream_t s) {
    int nb = tiles_for(gc);
    if (dim == 2)
        hipLaunchKernelGGL(k_inject_policy<2>, dim3(nb), dim3(kBlock), 0, s, gf, gc, af, ac);
    else
        hipLaunchKernelGGL(k_inject_policy<3>, dim3(nb), dim3(kBlock), 0, s, gf, gc, af, ac);
}

template void launch_diag<float>(int, const LevelDev &, const StencilDev &, const int16_t *, double, float *,
                                 hipStream_t, int16_t *, float *);
template void launch_diag<double>(int, const LevelDev &, const StencilDev &, const int16_t *, double, double *,
                                  hipStream_t, int16_t *, double *);
template void launch_jacobi<float>(int, const LevelDev &, const StencilDev &, const int16_t *, const float *,
                                   const float *, const float *, float *, double, double, bool, hipStream_t,
                                   const int16_t *, const float *);
template void launch_jacobi<double>(int, const LevelDev &, const StencilDev &, const int16_t *, const double *,
                                    const double *, const double *, double *, double, double, bool, hipStream_t,
                                    const int16_t *, const double *);
template void launch_level_residual<float>(int, const LevelDev &, const StencilDev &, const int16_t *, const float *,
                                           const float *, float *, double, hipStream_t, const int16_t *);
template void launch_level_residual<double>(int, const LevelDev &, const StencilDev &, const int16_t *,
                                            const double *, const double *, double *, double, hipStream_t,
                                            const int16_t *);
template void launch_restrict<float>(int, const LevelDev &, const LevelDev &, const float *, float *, hipStream_t);
template void launch_restrict<double>(int, const LevelDev &, const LevelDev &, const double *, double *, hipStream_t);
template void launch_prolong_add<float>(int, const LevelDev &, const LevelDev &, const float *, float *, hipStream_t);
template void launch_prolong_add<double>(int, const LevelDev &, const LevelDev &, const double *, double *,
                                         hipStream_t);
template void launch_coarse_solve<float>(int, const LevelDev &, const StencilDev &, const int16_t *, const float *,
                                         const float *, float *, float *, double, double, int, hipStream_t);
template void launch_coarse_solve<double>(int, const LevelDev &, const StencilDev &, const int16_t *, const double *,
                                          const double *, double *, double *, double, double, int, hipStream_t);

// ---- BLAS-1 for FP64 flexible GMRES ----------------------------------------------------------------

constexpr int kDotItems = 4;  // nodes per thread in the multi-vector kernels

__global__ __launch_bounds__(kBlock) void k_multidot(const double *__restrict__ w, const double *__restrict__ V,
                                                     int64_t ldv, int nvec, int64_t N, double *partial) {
    __shared__ double sh[kBlock / 64];
    int b = remap_block(blockIdx.x, gridDim.x);
    int64_t base = (int64_t)b * kBlock * kDotItems + threadIdx.x;
    double wv[kDotItems];
    double ww = 0.0;
#pragma unroll
    for (int q = 0; q < kDotItems; ++q) {
        int64_t n = base + (int64_t)q * kBlock;
        wv[q] = n < N ? w[n] : 0.0;
        ww += wv[q] * wv[q];
    }
    for (int v = 0; v < nvec; ++v) {
        const double *Vv = V + (int64_t)v * ldv;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kDotItems; ++q) {
            int64_t n = base + (int64_t)q * kBlock;
            if (n < N) acc += wv[q] * Vv[n];
        }
        double t = block_reduce<double>(acc, OpSum(), sh);
        if (threadIdx.x == 0) partial[(int64_t)v * gridDim.x + b] = t;
    }
    double t = block_reduce<double>(ww, OpSum(), sh);
    if (threadIdx.x == 0) partial[(int64_t)nvec * gridDim.x + b] = t;
}

int dot_blocks(int64_t N) { return (int)((N + (int64_t)kBlock * kDotItems - 1) / ((int64_t)kBlock * kDotItems)); }

void launch_multidot(const double *w, const double *V, int64_t ldv, int nvec, int64_t N, double *partial, int nblocks,
                     hipStream_t s) {
    SLHJB_LAUNCH(k_multidot, dim3(nblocks), dim3(kBlock), 0, s, w, V, ldv, nvec, N, partial);
}

__global__ __launch_bounds__(kBlock) void k_multiaxpy_scale(double *__restrict__ w, const double *__restrict__ V,
                                                            int64_t ldv, int nvec, const double *__restrict__ coef,
                                                            int64_t N, float *__restrict__ wf) {
    __shared__ double c[kMaxRestart + 2];
    for (int v = threadIdx.x; v <= nvec; v += blockDim.x) c[v] = coef[v];
    __syncthreads();
    // norm of the orthogonalised vector by Pythagoras (the caller runs a second pass on the result)
    double h2 = 0.0;
    for (int v = 0; v < nvec; ++v) h2 += c[v] * c[v];
    double hn2 = c[nvec] - h2;
    double inv = hn2 > 0.0 ? 1.0 / sqrt(hn2) : 1.0;
    int b = remap_block(blockIdx.x, gridDim.x);
    int64_t base = (int64_t)b * kBlock * kDotItems + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kDotItems; ++q) {
        int64_t n = base + (int64_t)q * kBlock;
        if (n < N) {
            double x = w[n];
            for (int v = 0; v < nvec; ++v) x -= c[v] * V[(int64_t)v * ldv + n];
            x *= inv;
            w[n] = x;
            if (wf) wf[n] = (float)x;  // the single-precision copy the next V-cycle reads
        }
    }
}

void launch_multiaxpy_scale(double *w, const double *V, int64_t ldv, int nvec, const double *coef, int64_t N,
                            int nblocks, hipStream_t s, float *wf) {
    SLHJB_LAUNCH(k_multiaxpy_scale, dim3(nblocks), dim3(kBlock), 0, s, w, V, ldv, nvec, coef, N, wf);
}

// The update of k_multiaxpy_scale followed by the sums of k_multidot on the updated vector, with the NV
// basis vectors held in registers between the two: one sweep over the basis instead of two.  Block
// decomposition, per-thread order and block reduction are those of the two kernels, so the partial sums
// are the same numbers.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_multiaxpy_scale_dot(double *__restrict__ w, const double *__restrict__ V,
                                                                int64_t ldv, const double *__restrict__ coef,
                                                                int64_t N, double *__restrict__ partial) {
    __shared__ double c[NV + 1];
    __shared__ double sh[kBlock / 64];
    for (int v = threadIdx.x; v <= NV; v += blockDim.x) c[v] = coef[v];
    __syncthreads();
    double h2 = 0.0;
    for (int v = 0; v < NV; ++v) h2 += c[v] * c[v];
    const double hn2 = c[NV] - h2;
    const double inv = hn2 > 0.0 ? 1.0 / sqrt(hn2) : 1.0;
    const int b = remap_block(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)b * kBlock * kDotItems + threadIdx.x;
    double vv[NV][kDotItems], x[kDotItems];
#pragma unroll
    for (int q = 0; q < kDotItems; ++q) {
        const int64_t n = base + (int64_t)q * kBlock;
        x[q] = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) vv[v][q] = 0.0;
        if (n < N) {
            double t = w[n];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                vv[v][q] = V[(int64_t)v * ldv + n];
                t -= c[v] * vv[v][q];
            }
            x[q] = t * inv;
            w[n] = x[q];
        }
    }
    double ww = 0.0;
#pragma unroll
    for (int q = 0; q < kDotItems; ++q) ww += x[q] * x[q];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kDotItems; ++q)
            if (base + (int64_t)q * kBlock < N) acc += x[q] * vv[v][q];
        const double t = block_reduce<double>(acc, OpSum(), sh);
        if (threadIdx.x == 0) partial[(int64_t)v * gridDim.x + b] = t;
    }
    const double t = block_reduce<double>(ww, OpSum(), sh);
    if (threadIdx.x == 0) partial[(int64_t)NV * gridDim.x + b] = t;
}

void launch_multiaxpy_scale_dot(double *w, const double *V, int64_t ldv, int nvec, const double *coef, int64_t N,
                                double *partial, int nblocks, hipStream_t s) {
#define MD(NV)                                                                                                  \
    case NV:                                                                                                    \
        SLHJB_LAUNCH(k_multiaxpy_scale_dot<NV>, dim3(nblocks), dim3(kBlock), 0, s, w, V, ldv, coef, N, partial); \
        return
    switch (nvec) {
        MD(1); MD(2); MD(3); MD(4); MD(5); MD(6); MD(7); MD(8);
        default:
            break;
    }
#undef MD
    launch_multiaxpy_scale(w, V, ldv, nvec, coef, N, nblocks, s, nullptr);
    launch_multidot(w, V, ldv, nvec, N, partial, nblocks, s);
}

// Reductions of per-block partials: one workgroup of kRedThreads per vector, four independent
// accumulators per thread so that four loads are in flight at a time (the partial arrays are short and
// latency, not bandwidth, sets the time).
constexpr int kRedThreads = 1024;

template <typename T, typename Op>
__device__ __forceinline__ T reduce_strided(const T *__restrict__ p, int n, Op op, T id) {
    T a0 = id, a1 = id, a2 = id, a3 = id;
    int q = threadIdx.x;
    for (; q + 3 * kRedThreads < n; q += 4 * kRedThreads) {
        const T v0 = p[q], v1 = p[q + kRedThreads], v2 = p[q + 2 * kRedThreads], v3 = p[q + 3 * kRedThreads];
        a0 = op(a0, v0);
        a1 = op(a1, v1);
        a2 = op(a2, v2);
        a3 = op(a3, v3);
    }
    for (; q < n; q += kRedThreads) a0 = op(a0, p[q]);
    return op(op(a0, a1), op(a2, a3));
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_sum(const double *__restrict__ partial, int nblocks,
                                                            double *__restrict__ out) {
    __shared__ double sh[kRedThreads / 64];
    const double t = block_reduce<double>(
        reduce_strided<double>(partial + (int64_t)blockIdx.x * nblocks, nblocks, OpSum(), 0.0), OpSum(), sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// largest entry (the partials are non-negative); a NaN anywhere is the result
__global__ __launch_bounds__(kRedThreads) void k_reduce_max(const double *__restrict__ partial, int nblocks,
                                                            double *__restrict__ out) {
    __shared__ double sh[kRedThreads / 64];
    const double t = block_reduce<double>(
        reduce_strided<double>(partial + (int64_t)blockIdx.x * nblocks, nblocks, OpMax(), 0.0), OpMax(), sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_sum_i64(const int64_t *__restrict__ partial, int nblocks,
                                                                int64_t *__restrict__ out) {
    __shared__ int64_t sh[kRedThreads / 64];
    const int64_t t = block_reduce<int64_t>(reduce_strided<int64_t>(partial, nblocks, OpSum(), (int64_t)0), OpSum(), sh);
    if (threadIdx.x == 0) out[0] = t;
}

void launch_reduce_sum(const double *partial, int nvec, int nblocks, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_sum, dim3(nvec), dim3(kRedThreads), 0, s, partial, nblocks, out);
}
void launch_reduce_max(const double *partial, int nvec, int nblocks, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_max, dim3(nvec), dim3(kRedThreads), 0, s, partial, nblocks, out);
}
void launch_reduce_sum_i64(const int64_t *partial, int nblocks, int64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_sum_i64, dim3(1), dim3(kRedThreads), 0, s, partial, nblocks, out);
}

__global__ __launch_bounds__(kBlock) void k_scale_by_inv_sqrt(double *__restrict__ dst, const double *__restrict__ src,
                                                              const double *__restrict__ norm2, int64_t N,
                                                              float *__restrict__ dstf) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n >= N) return;
    double inv = 1.0 / sqrt(norm2[0]);
    const double x = src[n] * inv;
    dst[n] = x;
    if (dstf) dstf[n] = (float)x;
}

// Hand small device results to the host without a stream event: the 8-byte words of (src0, n0) and
// (src1, n1) are stored to pinned host memory and made visible system-wide, then *flag receives seq with
// a release at system scope, so a host that reads seq from the flag also reads the words.  One wave.
__global__ __launch_bounds__(64) void k_publish(const uint64_t *__restrict__ src0, uint64_t *dst0, int n0,
                                                const uint64_t *__restrict__ src1, uint64_t *dst1, int n1,
                                                unsigned *flag, unsigned seq) {
    for (int q = threadIdx.x; q < n0; q += 64) dst0[q] = src0[q];
    for (int q = threadIdx.x; q < n1; q += 64) dst1[q] = src1[q];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_publish(const void *src0, void *dst0, size_t bytes0, const void *src1, void *dst1, size_t bytes1,
                    unsigned *flag, unsigned seq, hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, (const uint64_t *)src0, (uint64_t *)dst0, (int)(bytes0 / 8),
                       (const uint64_t *)src1, (uint64_t *)dst1, (int)(bytes1 / 8), flag, seq);
}

void launch_scale_by_inv_sqrt(double *dst, const double *src, const double *norm2, int64_t N, hipStream_t s,
                              float *dstf) {
    hipLaunchKernelGGL(k_scale_by_inv_sqrt, dim3(blocks_for(N)), dim3(kBlock), 0, s, dst, src, norm2, N, dstf);
}

__global__ __launch_bounds__(kBlock) void k_to_f32(const double *__restrict__ v, float *__restrict__ out, int64_t N) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n < N) out[n] = (float)v[n];
}
__global__ __launch_bounds__(kBlock) void k_copy_f64(const double *__restrict__ v, double *__restrict__ out, int64_t N) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n < N) out[n] = v[n];
}

void launch_to_precond(const double *v, void *out, bool out_float, int64_t N, hipStream_t s) {
    if (out_float)
        hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(N)), dim3(kBlock), 0, s, v, (float *)out, N);
    else
        hipLaunchKernelGGL(k_copy_f64, dim3(blocks_for(N)), dim3(kBlock), 0, s, v, (double *)out, N);
}

template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_update_solution(double *__restrict__ X, const TZ *__restrict__ Z,
                                                            int64_t ldz, int m, const UpdateCoef y, int64_t N) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n >= N) return;
    double x = X[n];
    for (int j = 0; j < m; ++j) x += y.c[j] * (double)Z[(int64_t)j * ldz + n];
    X[n] = x;
}

void launch_update_solution(double *X, const void *Z, bool z_float, int64_t ldz, int m, const double *y_host, int64_t N,
                            hipStream_t s) {
    UpdateCoef y{};
    for (int j = 0; j < m; ++j) y.c[j] = y_host[j];
    if (z_float)
        hipLaunchKernelGGL(k_update_solution<float>, dim3(blocks_for(N)), dim3(kBlock), 0, s, X, (const float *)Z, ldz,
                           m, y, N);
    else
        hipLaunchKernelGGL(k_update_solution<double>, dim3(blocks_for(N)), dim3(kBlock), 0, s, X, (const double *)Z,
                           ldz, m, y, N);
}

__global__ __launch_bounds__(kBlock) void k_axpy(double *__restrict__ y, double a, const double *__restrict__ x,
                                                 int64_t N) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n < N) y[n] += a * x[n];
}

void launch_axpy(double *y, double a, const double *x, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(N)), dim3(kBlock), 0, s, y, a, x, N);
}

// out = a + t b on every node (time-dependent Dirichlet data psi(t) = psi0 + t psi1)
__global__ __launch_bounds__(kBlock) void k_affine(const double *__restrict__ a, const double *__restrict__ b, double t,
                                                   double *__restrict__ out, int64_t N) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n < N) out[n] = a[n] + t * b[n];
}

void launch_affine(const double *a, const double *b, double t, double *out, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_affine, dim3(blocks_for(N)), dim3(kBlock), 0, s, a, b, t, out, N);
}

// ---- BiCGSTAB vector updates (right preconditioning) ----------------------------------------------
// The recurrence scalars never leave the device.  sc holds the reduced inner products of the current
// iteration: sc[0] = rho = (rhat, r), sc[1] = (rhat, v), sc[3] = (t, s), sc[4] = (t, t) (sc[2], sc[5]
// hold |v|^2 and unused sums).  alpha = rho / (rhat, v), omega = (t, s) / (t, t); a zero denominator gives
// a zero coefficient, which ends the recurrence without a division by zero (the host then restarts it
// from the true residual).  The direction update needs beta = (rho_new / rho_old) (alpha / omega), which
// in these slots is rho_new (t, t) / ((rhat, v) (t, s)): the old rho cancels, so one rho slot suffices.

__device__ __forceinline__ double bicg_alpha(const double *sc) { return sc[1] != 0.0 ? sc[0] / sc[1] : 0.0; }
__device__ __forceinline__ double bicg_omega(const double *sc) { return sc[4] > 0.0 ? sc[3] / sc[4] : 0.0; }

// p = r (first) or p = r + beta (p - omega v); pf (nullable) receives float(p)
__global__ __launch_bounds__(kBlock) void k_bicg_p(double *__restrict__ p, const double *__restrict__ r,
                                                   const double *__restrict__ v, const double *__restrict__ sc,
                                                   bool first, float *__restrict__ pf, int64_t N) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n >= N) return;
    double x;
    if (first) {
        x = r[n];
    } else {
        const double den = sc[1] * sc[3];
        const double beta = den != 0.0 ? sc[0] * sc[4] / den : 0.0;
        x = r[n] + beta * (p[n] - bicg_omega(sc) * v[n]);
    }
    p[n] = x;
    if (pf) pf[n] = (float)x;
}

// s = r - alpha v, in place over r; sf (nullable) receives float(s)
__global__ __launch_bounds__(kBlock) void k_bicg_s(double *__restrict__ r, const double *__restrict__ v,
                                                   const double *__restrict__ sc, float *__restrict__ sf, int64_t N) {
    int64_t n = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n >= N) return;
    const double x = r[n] - bicg_alpha(sc) * v[n];
    r[n] = x;
    if (sf) sf[n] = (float)x;
}

// X += alpha phat + omega shat, r = s - omega t (s in r, in place; shat may be r itself), and the per-block
// partials [sum rhat*r | max |r| | max |X|] over gridDim.x blocks each.
template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_bicg_xr(double *__restrict__ X, double *r, const double *__restrict__ t,
                                                    const TZ *__restrict__ phat, const TZ *shat,
                                                    const double *__restrict__ rhat, const double *__restrict__ sc,
                                                    double *__restrict__ partial, int64_t N) {
    __shared__ double sh[kBlock / 64];
    const int b = remap_block(blockIdx.x, gridDim.x);
    const int64_t n = (int64_t)b * kBlock + threadIdx.x;
    double dot = 0.0, rmax = 0.0, xmax = 0.0;
    if (n < N) {
        const double al = bicg_alpha(sc), om = bicg_omega(sc);
        const double x = X[n] + al * (double)phat[n] + om * (double)shat[n];
        const double rn = r[n] - om * t[n];
        X[n] = x;
        r[n] = rn;
        dot = rhat[n] * rn;
        rmax = fabs(rn);
        xmax = fabs(x);
    }
    double a = block_reduce<double>(dot, OpSum(), sh);
    if (threadIdx.x == 0) partial[b] = a;
    a = block_reduce<double>(rmax, OpMax(), sh);
    if (threadIdx.x == 0) partial[gridDim.x + b] = a;
    a = block_reduce<double>(xmax, OpMax(), sh);
    if (threadIdx.x == 0) partial[2 * gridDim.x + b] = a;
}

void launch_bicg_p(double *p, const double *r, const double *v, const double *sc, bool first, float *pf, int64_t N,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_p, dim3(blocks_for(N)), dim3(kBlock), 0, s, p, r, v, sc, first, pf, N);
}

void launch_bicg_s(double *r, const double *v, const double *sc, float *sf, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_s, dim3(blocks_for(N)), dim3(kBlock), 0, s, r, v, sc, sf, N);
}

void launch_bicg_xr(double *X, double *r, const double *t, const void *phat, const void *shat, bool z_float,
                    const double *rhat, const double *sc, double *partial, int64_t N, hipStream_t s) {
    if (z_float)
        hipLaunchKernelGGL(k_bicg_xr<float>, dim3(blocks_for(N)), dim3(kBlock), 0, s, X, r, t, (const float *)phat,
                           (const float *)shat, rhat, sc, partial, N);
    else
        hipLaunchKernelGGL(k_bicg_xr<double>, dim3(blocks_for(N)), dim3(kBlock), 0, s, X, r, t, (const double *)phat,
                           (const double *)shat, rhat, sc, partial, N);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_copy_interior(LevelDev g, const double *__restrict__ src,
                                                          double *__restrict__ dst) {
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    if (i < 0) return;
    if (interior<DIM>(g, ix)) dst[i] = src[i];
}

void launch_copy_interior(int dim, const LevelDev &g, const double *src, double *dst, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_copy_interior<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, src, dst);
    else
        hipLaunchKernelGGL(k_copy_interior<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, src, dst);
}

// interior of out = U1 + ratio (U1 - U0): the starting point of a step's policy iteration
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_extrapolate(LevelDev g, const double *__restrict__ U1,
                                                        const double *__restrict__ U0, double ratio,
                                                        double *__restrict__ out) {
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    if (i < 0) return;
    if (interior<DIM>(g, ix)) out[i] = U1[i] + ratio * (U1[i] - U0[i]);
}

void launch_extrapolate(int dim, const LevelDev &g, const double *U1, const double *U0, double ratio, double *out,
                        hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_extrapolate<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, U1, U0, ratio, out);
    else
        hipLaunchKernelGGL(k_extrapolate<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, U1, U0, ratio, out);
}

// explicit step: out = U + dt * g on interior nodes (g: the searched minimum of G_k)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_explicit_update(LevelDev g, const double *__restrict__ U,
                                                            const double *__restrict__ gmin, double dt,
                                                            double *__restrict__ out) {
    int ix[3];
    int i = tile_node<DIM>(g, ix);
    if (i < 0) return;
    if (interior<DIM>(g, ix)) out[i] = U[i] + dt * gmin[i];
}

void launch_explicit_update(int dim, const LevelDev &g, const double *U, const double *gmin, double dt, double *out,
                            hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_explicit_update<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, U, gmin, dt, out);
    else
        hipLaunchKernelGGL(k_explicit_update<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, U, gmin, dt, out);
}

// Zero fill by a kernel (stream-ordered, safe inside captured graphs); exact byte count.
__global__ __launch_bounds__(kBlock) void k_zero(unsigned char *__restrict__ p, int64_t bytes) {
    int64_t q = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 4;
    if (q + 4 <= bytes && (((uintptr_t)(p + q)) & 3) == 0) {
        *reinterpret_cast<uint32_t *>(p + q) = 0u;
    } else {
        for (int64_t b = q; b < q + 4 && b < bytes; ++b) p[b] = 0;
    }
}

void launch_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    int64_t words = (int64_t)((bytes + 3) / 4);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (unsigned char *)p, (int64_t)bytes);
}

}  // namespace slhjb
