// Internal definitions shared by the kernels and the host driver of libslhjb.
// Not part of the public C ABI (include/slhjb.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slhjb {

constexpr int kMaxP = 4;                 // diffusion columns per control
constexpr int kMaxPts = 2 * kMaxP + 1;   // stencil points per control (Scheme 2: 2P diffusion + 1 drift)
constexpr int kBlock = 256;              // threads per block of the node-parallel kernels
constexpr int kMaxRestart = 64;
constexpr int kTileLog2 = 5;             // default node tile of one block: 32 x 8 (width 2^kTileLog2)
constexpr int kTileLogMin = 4, kTileLogMax = 7;  // tile widths 16 ... 128 (heights 16 ... 2)
constexpr int kWinMax = 4;  // controls a window may hold for the matrix-free transposed gather

// Start and stop events for the next timed kernel launch.  A host timer scope sets them; the launcher
// of that kernel hands them to hipExtLaunchKernel, which stamps them with the dispatch's own begin and
// end times, so no marker packets sit between the timed kernel and its neighbours.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

inline LaunchEvents take_launch_events() {
    LaunchEvents e = g_launch_events;
    g_launch_events = LaunchEvents{};
    return e;
}

// Launch that consumes the pending timer events, if any (plain launch otherwise).
#define SLHJB_LAUNCH(kernel, grid, block, shmem, stream, ...)                                               \
    do {                                                                                                    \
        const ::slhjb::LaunchEvents ev_ = ::slhjb::take_launch_events();                                    \
        if (ev_.start)                                                                                      \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.start, ev_.stop, 0u, __VA_ARGS__); \
        else                                                                                                \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                            \
    } while (0)

// One stencil point of one control on one grid level.  Y is the displacement in cells of that level
// (diffusion: s*sigma_p/sqrt(h) scaled to the level, drift: b scaled to the level).  The remaining
// fields describe the landing when no truncation happens: cell offset floor(Y) per axis folded into a
// linear offset, fractions t = Y - floor(Y) and u = 1 - t in both precisions.
struct PointTab {
    double Y[3];
    double t[3];
    double u[3];
    float tf[3];
    float uf[3];
    int64_t off;
};

// Untruncated landing used by the node loops: linear offset of the landing cell and the 2^d corner
// weights (corner c: bit d set = upper corner on axis d; weight = product over axes of t_d or 1 - t_d).
// Sizes are multiples of 16 bytes so kernels whose control varies per node can stage them in LDS.
struct FastPtF {
    int32_t off;
    float w[8];
    int32_t pad[3];
};
struct FastPtD {
    int32_t off;
    int32_t pad;
    double w[8];
    int64_t pad2;
};

struct LevelDev {
    int32_t n[3];
    int32_t tlog;                    // tile width 2^tlog nodes along x, height kBlock / 2^tlog along y
    int32_t ntx, nty, ntz;           // tiles covering the grid
    int32_t deep_lo[3], deep_hi[3];  // nodes with deep_lo <= i_d <= deep_hi never truncate
    int64_t N;
    int64_t s1, s2;                  // strides of axes 1 and 2
};

struct StencilDev {
    const PointTab *tab;  // [K][npt]: points 2p (+sigma_p), 2p+1 (-sigma_p), 2P (drift, if any)
    const FastPtF *fastF; // [K][npt]
    const FastPtD *fastD; // [K][npt]
    const double *c;      // [K] or nullptr
    int32_t K, P, npt, has_drift;
    double inv2h;         // 1/(2h) of the finest grid: coarse levels keep the physical displacement
    // x-scaled coefficients (sigma_k(x) = diag(x) S_k, b_k(x) = diag(x) beta_k): the table holds S (signed)
    // and beta; displacements are formed per node, see point_Y
    int32_t xs;
    int32_t field;        // per-node sigma (all controls): diffusion displacements sr * sig_node[i][p]
    int32_t pernode;      // xs || field: displacements vary per node (no precomputed untruncated tables)
    double sr;            // s / sqrt(h) of the finest grid
    double scale;         // 2^-level: displacements in this level's cells
    double lo[3], hl;     // node coordinates on this level: x = lo + i * hl
    const double *sig_node;  // field model: [N_level][P][dim] on this level
    int64_t fk;           // control stride of f0, f1 (0: one source for all controls; N: [K][N])
    // constant coefficients: [K] per-control sum over points of W (w_self - 1) at deep nodes of this level,
    // where it does not depend on the node (nullptr: computed per node)
    const double *lii_deep;
};

// Displacement in cells of stencil point q (table entry p) at node ix (linear index i on its level).
// Constant coefficients: the table's value.  x-scaled: sr * (x * S) for diffusion points and x * beta
// for the drift point, per axis, then the level scale (exact: a power of two).  Per-node sigma: the
// diffusion points from the node's sigma, the drift point from the table.
__device__ __forceinline__ void point_Y(const StencilDev &st, const PointTab &p, int q, const int ix[3], int i,
                                        int dim, double Y[3]) {
    if (st.field && q < 2 * st.P) {
        // per-node sigma: Y = sr * sigma_p(x_i), the minus point its negation
        const double *sg = st.sig_node + ((int64_t)i * st.P + (q >> 1)) * dim;
        for (int d = 0; d < 3; ++d) {
            double v = d < dim ? st.sr * sg[d] : 0.0;
            if (q & 1) v = -v;
            Y[d] = v * st.scale;
        }
        return;
    }
    if (!st.xs) {
        Y[0] = p.Y[0];
        Y[1] = p.Y[1];
        Y[2] = p.Y[2];
        return;
    }
    const bool diffusion = q < 2 * st.P;
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            double x = st.lo[d] + (double)ix[d] * st.hl;
            double v = x * p.Y[d];
            if (diffusion) v = st.sr * v;
            Y[d] = v * st.scale;
        } else {
            Y[d] = 0.0;
        }
    }
}

// ---- kernel launchers (slhjb_kernels.hip) ----------------------------------------------------

// a kept decision needs its gap bound above this multiple of the search scale S (rounding of G is far below)
constexpr double kSkipSlack = 1e-10;
// a decision is a near tie when the second-best G is within kNearTie * tau of the best (several controls
// within tau, or the runner-up closer than this): there several policies are correct results
constexpr double kNearTie = 1e3;

struct SweepOut {
    int16_t *alpha_out;
    double *gmin, *margin;
    int32_t *ties;
    int64_t *changed_partial;  // [nblocks]: changed controls + (near ties << 32)
    // Certified reuse of decisions on untruncated wavefronts (constant coefficients, one diffusion pair).
    // skip 0: off; 1: record, per node, the gap between the second-best and the best G when the node's
    // control is the strict minimiser (-1 otherwise); 2: also keep the control of every wavefront whose
    // recorded gaps, less twice the largest change of any G_k since they were recorded, exceed the
    // rounding slack (such a control is still the strict minimiser, so the search would keep it).
    // Mode 2 runs in place (alpha_out == a_in): kept wavefronts leave their controls as they are.
    int32_t skip;
    double *marg;          // [N] lower bounds of the gaps (modes 1 and 2)
    const uint8_t *keep;   // [tiles * kBlock / 64] wavefronts certified by the keep pass (mode 2)
    // optional work list (mode 2): the search visits only list[0 .. list_count[0]) and leaves the
    // changed counts of the other tiles to the keep pass
    const int32_t *list;
    const int32_t *list_count;
    int32_t count_near;    // also count near ties (high 32 bits of changed_partial)
};

// largest |X - Xs| over each tile (dtile[tile], record == 0), then Xs = X on the tile
void launch_delta_tiles(int dim, const LevelDev &g, const double *X, double *Xs, double *dtile, bool record,
                        hipStream_t s);
// dwin[T] = max of dtile over the tiles within R[a] nodes of tile T along each axis
void launch_window_max(int dim, const LevelDev &g, const double *dtile, double *dwin, const int R[3], hipStream_t s);
// keep[wave] = 1 where every interior node of the wavefront is untruncated and marg - lip2 * dwin stays
// above the rounding slack (scale[0] = S of the search); marg is then reduced by lip2 * dwin there.
// kept_partial[tile]: interior nodes kept in the tile.
// need[tile] = 1 where some wavefront with interior nodes is not kept; changed_partial[tile] = 0.
void launch_keep_pass(int dim, const LevelDev &g, double *marg, const double *dwin, double lip2, const double *scale,
                      uint8_t *keep, int64_t *kept_partial, uint8_t *need, int64_t *changed_partial, hipStream_t s);
// list[0 .. *count) = tiles t < nt with need[t] != 0, increasing
void launch_tile_list(const uint8_t *need, int nt, int32_t *list, int32_t *count, hipStream_t s);

// qmode: 0 evaluate the explicit part (theta < 1) or skip it (theta = 1); 1 evaluate it and store
// (1-theta)((L^k U)_i + c_k U_i) in Q (K * blocks * kBlock doubles, tile-major); 2 read it from Q.
void launch_sweep(int dim, const LevelDev &g, const StencilDev &st, const double *X, const double *U,
                  const double *f0, const double *f1, double t_mid, double theta, const double *tau,
                  const int16_t *a_in, const SweepOut &o, double *Q, int qmode, int nblocks, hipStream_t s);

void launch_norms_xuf(int dim, const LevelDev &g, const double *X, const double *U, const double *f0, const double *f1,
                      double t_mid, int K, int64_t fk, double *partial, int nblocks, hipStream_t s);
void launch_explicit_update(int dim, const LevelDev &g, const double *U, const double *gmin, double dt, double *out,
                            hipStream_t s);

// Wave-control table (wctl, nullable): per wavefront of the tile mapping, the control shared by all its 64 nodes
// when all are untruncated interior nodes, else -1; written by launch_diag for the level's current policy.  With
// it the multigrid smoother and residual read neither the policy nor the diagonal on such wavefronts.

// y = x - theta dt (L x + c x) on interior nodes, 0 on the boundary (x may be float or double)
void launch_apply(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const void *x,
                  bool x_is_float, double *y, double theta_dt, double *norm2_partial, int nblocks, hipStream_t s);

// E = U + (1-theta) dt (L U + c U) + dt (f0 + t_mid f1)
void launch_explicit(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const double *U,
                     const double *f0, const double *f1, double t_mid, double omt_dt, double dt, double *E,
                     int nblocks, hipStream_t s);

// r = E - (V - theta dt (L V + c V)); partials: [3][nblocks] = sum r^2, max|r|, max|V| (interior)
void launch_residual(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const double *V,
                     const double *E, double theta_dt, double *r, double *partial, int nblocks, hipStream_t s);

// multigrid level kernels, T = float or double
// d = diagonal of A on the level; with wctl (ignored without per-control deep values) also the wave-control
// table and dk[k], the diagonal at untruncated nodes of control k
template <typename T>
void launch_diag(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, double theta_dt, T *d,
                 hipStream_t s, int16_t *wctl = nullptr, T *dk = nullptr);
// per-control table of StencilDev::lii_deep, evaluated at the deep node ix0 of the level (K entries)
void launch_lii_deep(int dim, const LevelDev &g, const StencilDev &st, const int ix0[3], double *out, hipStream_t s);
template <typename T>
void launch_jacobi(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const T *e, const T *r,
                   const T *d, T *e_out, double theta_dt, double omega, bool first, hipStream_t s,
                   const int16_t *wctl = nullptr, const T *dk = nullptr);
template <typename T>
void launch_level_residual(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const T *e,
                           const T *r, T *res, double theta_dt, hipStream_t s, const int16_t *wctl = nullptr);
template <typename T>
void launch_restrict(int dim, const LevelDev &gf, const LevelDev &gc, const T *rf, T *rc, hipStream_t s);
template <typename T>
void launch_prolong_add(int dim, const LevelDev &gf, const LevelDev &gc, const T *ec, T *ef, hipStream_t s);
template <typename T>
void launch_coarse_solve(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const T *r,
                         const T *d, T *e, T *tmp, double theta_dt, double omega, int sweeps, hipStream_t s);
void launch_bad_policy(int dim, const LevelDev &g, const int16_t *alpha, int K, int64_t *partial, int nblocks,
                       hipStream_t s);
void launch_inject_policy(int dim, const LevelDev &gf, const LevelDev &gc, const int16_t *af, int16_t *ac,
                          hipStream_t s);

// BLAS-1 (FP64 Krylov)
// partial[v][b] = block b's part of <w, V_v> for v < nvec, and partial[nvec][b] = part of <w, w>
void launch_multidot(const double *w, const double *V, int64_t ldv, int nvec, int64_t N, double *partial,
                     int nblocks, hipStream_t s);
// w = (w - sum_v coef[v] V_v) / sqrt(coef[nvec] - sum_v coef[v]^2)  (divisor 1 if that is not positive)
// w <- (w - sum_v coef[v] V_v) / sqrt(coef[nvec] - sum_v coef[v]^2); wf (nullable) receives float(w)
void launch_multiaxpy_scale(double *w, const double *V, int64_t ldv, int nvec, const double *coef, int64_t N,
                            int nblocks, hipStream_t s, float *wf = nullptr);
// the same update followed by the per-block partial sums of launch_multidot on the updated w
void launch_multiaxpy_scale_dot(double *w, const double *V, int64_t ldv, int nvec, const double *coef, int64_t N,
                                double *partial, int nblocks, hipStream_t s);
void launch_reduce_sum(const double *partial, int nvec, int nblocks, double *out, hipStream_t s);
void launch_reduce_max(const double *partial, int nvec, int nblocks, double *out, hipStream_t s);
void launch_reduce_sum_i64(const int64_t *partial, int nblocks, int64_t *out, hipStream_t s);
// copy bytes0 (bytes1) from device src0 (src1) to pinned host dst0 (dst1), multiples of 8 bytes, then
// store seq to the pinned host word *flag with a system-scope release
void launch_publish(const void *src0, void *dst0, size_t bytes0, const void *src1, void *dst1, size_t bytes1,
                    unsigned *flag, unsigned seq, hipStream_t s);
void launch_scale_by_inv_sqrt(double *dst, const double *src, const double *norm2, int64_t N, hipStream_t s,
                              float *dstf = nullptr);
void launch_to_precond(const double *v, void *out, bool out_float, int64_t N, hipStream_t s);
// X += sum_{j<m} y_host[j] Z_j; the m <= kMaxRestart coefficients travel as a kernel argument
struct UpdateCoef {
    double c[kMaxRestart];
};
void launch_update_solution(double *X, const void *Z, bool z_float, int64_t ldz, int m, const double *y_host, int64_t N,
                            hipStream_t s);
void launch_axpy(double *y, double a, const double *x, int64_t N, hipStream_t s);
// BiCGSTAB updates; sc = device slots [rho, (rhat,v), |v|^2, (t,s), (t,t)] (alpha and omega derived there)
void launch_bicg_p(double *p, const double *r, const double *v, const double *sc, bool first, float *pf, int64_t N,
                   hipStream_t s);
void launch_bicg_s(double *r, const double *v, const double *sc, float *sf, int64_t N, hipStream_t s);
// partial: [sum rhat*r | max|r| | max|X|], blocks_for(N) entries each
void launch_bicg_xr(double *X, double *r, const double *t, const void *phat, const void *shat, bool z_float,
                    const double *rhat, const double *sc, double *partial, int64_t N, hipStream_t s);
void launch_affine(const double *a, const double *b, double t, double *out, int64_t N, hipStream_t s);
void launch_copy_interior(int dim, const LevelDev &g, const double *src, double *dst, hipStream_t s);
void launch_zero(void *p, size_t bytes, hipStream_t s);
void launch_extrapolate(int dim, const LevelDev &g, const double *U1, const double *U0, double ratio, double *out,
                        hipStream_t s);

int blocks_for(int64_t N);

// Galerkin coarse operators (slhjb_galerkin.hip), 2D: ELL slot-major (entry s of row i at s * N + i, column -1
// unused).  emit: rows of A = I - theta dt (L-hat + c) at the interior nodes of the finest level (E = npt * 4 + 1
// slots); rap: R A P onto the next level (Wc slots; *overflow = the widest row when wider than Wc); diag: the
// diagonal (1 on boundary rows) and optional FP32 weights; jacobi / residual: the smoother and residual.
void launch_gal_emit(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, double theta_dt, int E,
                     int32_t *col, double *val, hipStream_t s);
int gal_sort_size(int Wf);
int launch_gal_rap(const LevelDev &gf, const LevelDev &gc, int Wf, const int32_t *fcol, const double *fval, int Wc,
                   int32_t *ccol, double *cval, int32_t *overflow, hipStream_t s);
void launch_gal_diag(int64_t N, int W, const int32_t *col, const double *val, float *val32, float *d32, double *d64,
                     hipStream_t s);
template <typename T>
void launch_gal_jacobi(int64_t N, int W, const int32_t *col, const T *val, const T *d, const T *e, const T *r, T *out,
                       double omega, bool first, hipStream_t s);
template <typename T>
void launch_gal_residual(int64_t N, int W, const int32_t *col, const T *val, const T *e, const T *r, T *res,
                         hipStream_t s);

// Aggregation AMG (slhjb_amg.hip): ELL slot-major levels with compact rows.  merge: emitted finest rows ->
// one entry per column; colcount / scatter / sym: the symmetric part S of the couplings (column counts and
// their largest, transposed segments, S rows of width Ws); init / match_round / leader / assign: one pairing
// pass (state in mate, candidates in cand, leader flags, aggregate ids from their prefix sums, members two per
// aggregate); compose / members4: two
// passes as one map with four members per aggregate; product: P^T M P for piecewise-constant P (-1: the row
// sum exceeds the sort capacity); diag; restrict / prolong; spmv; dot2: (a,b), (a,c) into out[0..1] (part holds
// 2 * amg_dot_parts(n) doubles); gcr: the GCR updates of the cycle; coarse: Jacobi sweeps in one workgroup.
constexpr int kAmgCoarseMax = 2048;  // coarsest level solved by Jacobi sweeps in one workgroup, at most
constexpr int kAmgDenseMax = 120;    // coarsest level solved through its dense inverse (LDS-resident), at most
void launch_amg_merge(int64_t n, int nx, int ny, int nz, int E, const int32_t *icol, const double *ival,
                      int32_t *ocol, double *oval, hipStream_t s);
void launch_amg_init(int64_t n, int W, const int32_t *col, const double *val, double dd, int32_t *mate,
                     hipStream_t s);
void launch_amg_colcount(int64_t n, int W, const int32_t *col, int32_t *cnt, int32_t *mx, hipStream_t s);
void launch_amg_scatter(int64_t n, int W, const int32_t *col, const double *val, const int32_t *off, int32_t *fill,
                        int32_t *trow, double *tval, hipStream_t s);
int launch_amg_sym(int64_t n, int W, int maxcol, const int32_t *col, const double *val, const int32_t *off,
                   const int32_t *cnt, const int32_t *trow, const double *tval, int Ws, int32_t *scol, double *sval,
                   hipStream_t s);
void launch_amg_match_round(int64_t n, int Ws, const int32_t *scol, const double *sval, double beta, int32_t *mate,
                            int32_t *cand, hipStream_t s);
void launch_amg_leader(int64_t n, const int32_t *mate, int32_t *flag, hipStream_t s);
void launch_amg_assign(int64_t n, const int32_t *mate, const int32_t *id, int32_t *agg, int32_t *mem2, hipStream_t s);
void launch_amg_compose(int64_t n, const int32_t *agg1, const int32_t *agg2, int32_t *agg, hipStream_t s);
void launch_amg_members4(int64_t nc, const int32_t *mem2b, const int32_t *mem2a, int32_t *mem4, hipStream_t s);
int launch_amg_product(int64_t nf, int W, const int32_t *fcol, const double *fval, const int32_t *agg,
                       const int32_t *mem, int maxm, int64_t nc, int Wc, int32_t *ccol, double *cval, int32_t *widest,
                       hipStream_t s);
void launch_amg_diag(int64_t n, int W, const int32_t *col, const double *val, double *d, hipStream_t s);
void launch_amg_restrict(int64_t nc, const int32_t *mem4, const double *rf, double *rc, hipStream_t s);
void launch_amg_prolong(int64_t nf, const int32_t *agg, const double *ec, double *ef, hipStream_t s);
void launch_amg_spmv(int64_t n, int W, const int32_t *col, const double *val, const double *x, double *y,
                     hipStream_t s);
int amg_dot_parts(int64_t n);
void launch_amg_dot2(int64_t n, const double *a, const double *b, const double *c, double *part, double *out,
                     hipStream_t s);
void launch_amg_gcr(int64_t n, int mode, const double *sc, double *x, double *v, double *w, const double *v1,
                    const double *w1, const double *r, double *r_out, hipStream_t s);
void launch_amg_coarse(int n, int W, const int32_t *col, const double *val, const double *d, const double *r,
                       int sweeps, double *x, hipStream_t s);
void launch_amg_dense_inverse(int n, int W, const int32_t *col, const double *val, double *inv, hipStream_t s);
// wide levels: row-major copy (entry s of row i at i * W + s) and one wavefront per row; mode 0: y = A x,
// 1: y = r - A x, 2: damped Jacobi y = x + omega (r - A x) / d (first: y = omega r / d)
void launch_amg_rowmajor(int64_t n, int W, const int32_t *col, const double *val, int32_t *rcol, double *rval,
                         hipStream_t s);
void launch_amg_wave_op(int64_t n, int W, const int32_t *rcol, const double *rval, const double *d, const double *x,
                        const double *r, double *y, int mode, double omega, bool first, hipStream_t s);
constexpr int kAmgWaveWidth = 32;       // levels with wider rows and at most kAmgWaveRows rows use the row-major
constexpr int64_t kAmgWaveRows = 262144;  // copy and the wavefront kernels
void launch_amg_dense_solve(int n, const double *inv, const double *r, double *x, hipStream_t s);
// exclusive prefix sums of int32 counts (slhjb_adjoint.hip): out[q] = in[0] + ... + in[q-1], *total_out
// (nullable, device) = the sum; part holds scan_parts(m) + 1 entries
int64_t scan_parts(int64_t m);
void exclusive_scan(const int32_t *in, int64_t m, int32_t *out, int32_t *part, int32_t *total_out, hipStream_t s);

// adjoint (slhjb_adjoint.hip)
// Row listing of one level's operator (slots [i*E, (i+1)*E)) and its column-sorted form.
// The sorted entries are also laid out as sliced ELL: slice = one wavefront of the node kernels' launch
// (remapped block * 4 + wave), width = the slice's longest column capped at kEllCap, entry q of lane l
// at (off[slice] + q) * 64 + l; entries past the cap stay in the CSC arrays.
constexpr int kEllCap = 32;
// The FP32 copy (preconditioner) holds the weights as float and, in 2D when every stencil point stays
// within 127 cells, the row as int8 offsets (dx | dy << 8) from the column node.
struct TransposeBuf {
    int32_t *cols, *cols_s, *ids_s, *colptr, *rows_s;  // cols_s: counts / scatter cursor, ids_s: slots
    double *vals, *vals_s;
    int32_t *ell_w, *ell_off, *ell_rows;
    double *ell_vals;
    float *ell_vals32;   // nullable: no FP32 copy
    int16_t *ell_d16;    // nullable: rows not packed
    void *scratch;
    size_t scratch_bytes;
};
struct TransposeView {
    const int32_t *colptr, *rows;
    const double *vals;
    const int32_t *ell_w, *ell_off, *ell_rows;
    const double *ell_vals;
    const float *ell_vals32;
    const int16_t *ell_d16;
    // optional, per tile, 5 entries: {n, k_0..k_3}, the n <= 4 controls found within the stencil reach of
    // the tile when every node there is untruncated (constant coefficients), else n = -1.  There column j
    // of L is gathered from the row stencils reflected (entries w_c at j - off - delta_c, of the rows whose
    // control is the stencil's), without the listing.
    const int32_t *wset;
};
// tset[5 T ..] = {n, controls} of tile T when all its nodes are interior and untruncated and it holds at
// most 4 controls, else n = -1
void launch_tile_set(int dim, const LevelDev &g, const int16_t *alpha, int K, int32_t *tset, hipStream_t s);
// wset[5 T ..] = union of tset over the tiles within R[a] nodes of T along each axis (n = -1 if invalid)
void launch_window_set(int dim, const LevelDev &g, const int32_t *tset, int32_t *wset, const int R[3],
                       hipStream_t s);
int build_transpose(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, int E, TransposeBuf &b,
                    hipStream_t s);
size_t transpose_scratch_bytes(int64_t n, int N, int nslices);
inline int64_t ell_slices(const LevelDev &g);
void launch_apply_T(int dim, int mode, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                    const TransposeView &T, const double *x, const double *b, double w, double *y, double *partial,
                    hipStream_t s);
void launch_apply_T_f32x(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                         const TransposeView &T, const float *x, double w, double *y, hipStream_t s);
void launch_jacobi_T32(int dim, bool first, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                       const TransposeView &T, const float *x, const float *r, const float *d, double theta_dt,
                       double omega, float *y, hipStream_t s);
void launch_resid_T32(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const TransposeView &T,
                      const float *x, const float *b, double theta_dt, float *y, hipStream_t s);
void launch_jacobi_T(int dim, bool first, const LevelDev &g, const StencilDev &st, const int16_t *alpha,
                     const TransposeView &T, const double *x, const double *r, const double *d, double theta_dt,
                     double omega, double *y, hipStream_t s);
void launch_ds_dot(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, const double *mu,
                   const double *Va, double wa, const double *Vb, double wb, double inv_s, double *partial,
                   hipStream_t s);
void launch_axpy_interior(int dim, const LevelDev &g, double a, const double *x, double *y, hipStream_t s);
void launch_mask_interior(int dim, const LevelDev &g, const double *x, double *y, hipStream_t s);
inline int tiles_for(const LevelDev &g) { return g.ntx * g.nty * g.ntz; }

// ---- batched launches (slhjb_batch.hip) ------------------------------------------------------------

// one instance on one level of a batch: grid, stencil, and where its arrays start in the level's
// concatenated batch arrays
struct BInst {
    LevelDev g;
    StencilDev st;
    int64_t off;
};
// tiles of one batched launch: entry p = (instance inst[p], tile tile[p]); an instance's entries are
// contiguous; blocks of instances with active[b] == 0 exit at once (active may be null)
struct BTiles {
    const int32_t *inst, *tile;
    const BInst *I;
    const uint8_t *active;
    int32_t n;
};
void launch_norms_b(int dim, const BTiles &T, const double *X, const double *U, const double *f0, const double *f1,
                    double t_mid, double *partial, hipStream_t s);
void launch_tau_b(const double *partial, int n, const int32_t *first, const double *coefA, double tau_rel,
                  const uint8_t *active, double *tau, int B, hipStream_t s);
void launch_sweep_b(int dim, const BTiles &T, const double *X, const double *U, const double *f0, const double *f1,
                    double t_mid, double theta, const double *tau, const int16_t *a_in, int16_t *a_out,
                    int64_t *changed_partial, hipStream_t s);
void launch_explicit_b(int dim, const BTiles &T, const int16_t *alpha, const double *U, const double *f0,
                       const double *f1, double t_mid, double omt_dt, double dt, double *E, hipStream_t s);
void launch_residual_b(int dim, const BTiles &T, const int16_t *alpha, const double *V, const double *E,
                       double theta_dt, double *r, double *partial, hipStream_t s);
void launch_apply_b(int dim, const BTiles &T, const int16_t *alpha, const void *x, bool x_float, double *y,
                    double theta_dt, hipStream_t s);
template <typename T>
void launch_diag_b(int dim, const BTiles &Tb, const int16_t *alpha, double theta_dt, T *d, hipStream_t s);
template <typename T>
void launch_jacobi_b(int dim, const BTiles &Tb, const int16_t *alpha, const T *e, const T *r, const T *d, T *e_out,
                     double theta_dt, double omega, bool first, hipStream_t s);
template <typename T>
void launch_level_residual_b(int dim, const BTiles &Tb, const int16_t *alpha, const T *e, const T *r, T *res,
                             double theta_dt, hipStream_t s);
template <typename T>
void launch_restrict_b(int dim, const BTiles &Tc, const BInst *If, const T *rf, T *rc, hipStream_t s);
template <typename T>
void launch_prolong_add_b(int dim, const BTiles &Tf, const BInst *Ic, const T *ec, T *ef, hipStream_t s);
template <typename T>
void launch_coarse_b(int dim, const int32_t *list, int count, int64_t maxN, const BInst *Iv, const uint8_t *active,
                     const int16_t *alpha, const T *r, const T *d, T *e, double theta_dt, double omega, int sweeps,
                     hipStream_t s);
void launch_inject_b(int dim, const BTiles &Tc, const BInst *If, const int16_t *af, int16_t *ac, hipStream_t s);
void launch_copy_interior_b(int dim, const BTiles &T, const double *src, double *dst, hipStream_t s);
void launch_extrapolate_b(int dim, const BTiles &T, const double *U1, const double *U0, double ratio, double *out,
                          hipStream_t s);
void launch_copy_policy_b(int dim, const BTiles &T, const int16_t *src, int16_t *dst, hipStream_t s);
void launch_multidot_b(int dim, const BTiles &T, const double *w, const double *V, int64_t ldv, int nvec,
                       double *partial, hipStream_t s);
void launch_multiaxpy_scale_b(int dim, const BTiles &T, double *w, const double *V, int64_t ldv, int nvec,
                              const double *coef, int ldc, hipStream_t s);
void launch_scale_b(int dim, const BTiles &T, double *dst, const double *src, const double *norm2, int ldn,
                    hipStream_t s);
void launch_update_b(int dim, const BTiles &T, double *X, const void *Z, bool z_float, int64_t ldz, const int32_t *m,
                     const double *y, int ldy, hipStream_t s);
// device-side FGMRES scalars of a batch: per instance the Hessenberg matrix ((m+1) x m, row-major), Givens
// cosines and sines (m), residual estimates g (m+1), the new vector's norm, the target, iteration counts,
// the columns of the current cycle and a non-finite flag
struct BKrylov {
    double *H, *cs, *sn, *g, *hn, *target;
    int32_t *its, *jb, *bad;
    int m, maxk;
};
void launch_cycle_init_b(const BKrylov &K, int B, const uint8_t *solving, const double *r2, uint8_t *cyc,
                         hipStream_t s);
void launch_mask_copy_b(int B, const uint8_t *src, uint8_t *dst, hipStream_t s);
void launch_arnoldi_pass_b(const BKrylov &K, int B, int j, int pass, const double *seg, double *coef, int ldc,
                           const uint8_t *in_pass, uint8_t *next_pass, hipStream_t s);
void launch_givens_b(const BKrylov &K, int B, int j, uint8_t *cyc, hipStream_t s);
void launch_backsolve_b(const BKrylov &K, int B, const uint8_t *solving, double *y, int ldy, int32_t *count,
                        hipStream_t s);
void launch_seg_sum(const double *partial, int n, const int32_t *first, int nvec, const uint8_t *active, double *out,
                    int B, hipStream_t s);
void launch_seg_max(const double *partial, int n, const int32_t *first, int nvec, const uint8_t *active, double *out,
                    int B, hipStream_t s);
void launch_seg_sum_i64(const int64_t *partial, int n, const int32_t *first, const uint8_t *active, int64_t *out, int B,
                        hipStream_t s);

inline int64_t ell_slices(const LevelDev &g) { return (int64_t)tiles_for(g) * (kBlock / 64); }
inline void set_tiles(LevelDev &g, int dim) {
    const int tx = 1 << g.tlog, ty = kBlock >> g.tlog;
    g.ntx = (g.n[0] + tx - 1) / tx;
    g.nty = (g.n[1] + ty - 1) / ty;
    g.ntz = dim == 3 ? g.n[2] : 1;
}

}  // namespace slhjb
