// Galerkin coarse operators of the multigrid hierarchy (Section 3.3: the coarse system matrix built by the
// Galerkin principle, A_c = R A P, with bilinear prolongation P and full-weighting restriction R), as an
// alternative to rediscretising the operator on each level.  2D grids.
//
// Level operators are held in a sliced ELL layout, slot-major: entry s of row i at s * N + i (column, value),
// column -1 for an unused slot.  The finest level's rows are emitted from the stencil (the general landing
// rules of eq. TruncScheme, as the node kernels evaluate them) as rows of A = I - theta dt (L-hat + c) on the
// interior unknowns; a coarse row I is assembled by one wavefront from the 9 fine rows its restriction
// weighs, each entry spread over the (up to) 4 coarse nodes that interpolate its column.  The wavefront sorts
// its contributions by (coarse column, contribution index) in LDS and sums each column's run in that order,
// so the coarse operator does not depend on scheduling.

#include "slhjb_device.h"

namespace slhjb {

constexpr int kGalMaxSort = 4096;  // contributions of one coarse row held in LDS, at most

// rows of the finest level's A at interior nodes: slot e < E of row i; boundary rows empty.  E = npt 2^DIM + 1:
// the 2^DIM interpolation corners of each stencil point, then the diagonal
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_gal_emit(LevelDev g, StencilDev st, const int16_t *__restrict__ alpha,
                                                     double theta_dt, int E, int32_t *__restrict__ col,
                                                     double *__restrict__ val) {
    int ix[3];
    const int i = tile_node<DIM>(g, ix);
    if (i < 0) return;
    const int64_t N = g.N;
    if (!interior<DIM>(g, ix)) {
        for (int e = 0; e < E; ++e) col[e * N + i] = -1;
        return;
    }
    int k = alpha[i];
    k = ((unsigned)k < (unsigned)st.K) ? k : 0;
    const PointTab *pt = st.tab + k * st.npt;
    const int s1 = (int)g.s1, s2 = (int)g.s2;
    int e = 0;
    double self = 0.0;
    auto emit_point = [&](int q, double factor) {
        double Y[3];
        point_Y(st, pt[q], q, ix, i, DIM, Y);
        int cell[3];
        double t[3];
        landing<DIM>(g, ix, Y, cell, t);
        const int cb = cell[0] + cell[1] * s1 + (DIM == 3 ? cell[2] * s2 : 0);
        for (int c = 0; c < (1 << DIM); ++c) {
            double w = (c & 1) ? t[0] : (1.0 - t[0]);
            w = w * ((c & 2) ? t[1] : (1.0 - t[1]));
            if (DIM == 3) w = w * ((c & 4) ? t[2] : (1.0 - t[2]));
            const int j = cb + (c & 1) + ((c & 2) ? s1 : 0) + ((DIM == 3 && (c & 4)) ? s2 : 0);
            const double a = -theta_dt * st.inv2h * factor * w;
            col[e * N + i] = (j == i) ? -1 : j;  // the node's own corner weight joins the diagonal
            val[e * N + i] = a;
            if (j == i) self += a;
            ++e;
        }
    };
    double sumf = 0.0;
    for (int p = 0; p < st.P; ++p) {
        double Ya[3], Yb[3];
        point_Y(st, pt[2 * p], 2 * p, ix, i, DIM, Ya);
        point_Y(st, pt[2 * p + 1], 2 * p + 1, ix, i, DIM, Yb);
        int cc[3];
        double tt[3];
        const double mup = landing<DIM>(g, ix, Ya, cc, tt);
        const double mum = landing<DIM>(g, ix, Yb, cc, tt);
        const double A = 2.0 / (mup * (mup + mum)), B = 2.0 / (mum * (mum + mup));
        emit_point(2 * p, A);
        emit_point(2 * p + 1, B);
        sumf += A + B;
    }
    if (st.has_drift) {
        double Yc[3];
        point_Y(st, pt[2 * st.P], 2 * st.P, ix, i, DIM, Yc);
        int cc[3];
        double tt[3];
        const double C2 = 2.0 / landing<DIM>(g, ix, Yc, cc, tt);
        emit_point(2 * st.P, C2);
        sumf += C2;
    }
    const double ck = st.c ? st.c[k] : 0.0;
    col[e * N + i] = i;
    val[e * N + i] = 1.0 - theta_dt * (ck - st.inv2h * sumf) + self;
    ++e;
    for (; e < E; ++e) col[e * N + i] = -1;
}

// coarse row I of R A P (R: full weighting, P: bilinear; both act on interior nodes only); *widest receives
// the largest number of distinct columns of a row (rows wider than Wc keep their first Wc)
template <int NSORT>
__global__ __launch_bounds__(64) void k_gal_rap(LevelDev gf, LevelDev gc, int Wf, const int32_t *__restrict__ fcol,
                                                const double *__restrict__ fval, int Wc, int32_t *__restrict__ ccol,
                                                double *__restrict__ cval, int32_t *__restrict__ widest) {
    constexpr int nsort = NSORT;
    __shared__ uint64_t key[NSORT];
    __shared__ double sval[NSORT];
    const int64_t I = blockIdx.x;
    const int lane = threadIdx.x;
    const int nc0 = gc.n[0], nf0 = gf.n[0];
    const int X = (int)(I % nc0), Y = (int)(I / nc0);
    const bool inside = X > 0 && X < nc0 - 1 && Y > 0 && Y < gc.n[1] - 1;
    if (!inside) {
        for (int s = lane; s < Wc; s += 64) ccol[s * gc.N + I] = -1;
        return;
    }
    const int total = 9 * Wf * 4;  // (fine row, slot, coarse corner)
    for (int c = lane; c < nsort; c += 64) {
        uint64_t kk = ~0ull;
        double v = 0.0;
        if (c < total) {
            const int q = c & 3, s = (c >> 2) % Wf, r = (c >> 2) / Wf;
            const int dx = r % 3 - 1, dy = r / 3 - 1;
            const int fx = 2 * X + dx, fy = 2 * Y + dy;
            const double rw = (dx ? 0.25 : 0.5) * (dy ? 0.25 : 0.5);  // full weighting, as the restriction
            const int64_t f = (int64_t)fx + (int64_t)fy * nf0;
            const bool fin = fx > 0 && fx < nf0 - 1 && fy > 0 && fy < gf.n[1] - 1;
            const int j = fin ? fcol[(int64_t)s * gf.N + f] : -1;
            if (j >= 0) {
                const int jx = j % nf0, jy = j / nf0;
                const bool jin = jx > 0 && jx < nf0 - 1 && jy > 0 && jy < gf.n[1] - 1;
                // coarse corner q: x from bit 0, y from bit 1 (an even fine coordinate has one coarse node)
                const int Jx = (jx >> 1) + ((q & 1) ? (jx & 1) : 0), Jy = (jy >> 1) + ((q & 2) ? (jy & 1) : 0);
                const bool dup = ((q & 1) && !(jx & 1)) || ((q & 2) && !(jy & 1));
                const double px = (jx & 1) ? 0.5 : 1.0, py = (jy & 1) ? 0.5 : 1.0;
                const bool cin = Jx > 0 && Jx < nc0 - 1 && Jy > 0 && Jy < gc.n[1] - 1;
                if (jin && !dup && cin) {
                    kk = ((uint64_t)(Jx + Jy * nc0) << 20) | (uint64_t)c;
                    v = rw * fval[(int64_t)s * gf.N + f] * px * py;
                }
            }
        }
        key[c] = kk;
        sval[c] = v;
    }
    __syncthreads();
    // bitonic sort of nsort (a power of two) entries by key
    for (int size = 2; size <= nsort; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < nsort / 2; t += 64) {
                const int a = 2 * t - (t & (stride - 1)), b = a + stride;
                const bool up = (a & size) == 0;
                const uint64_t ka = key[a], kb = key[b];
                if ((ka > kb) == up) {
                    key[a] = kb;
                    key[b] = ka;
                    const double va = sval[a];
                    sval[a] = sval[b];
                    sval[b] = va;
                }
            }
            __syncthreads();
        }
    }
    // runs of equal columns: the lane at a run's first entry sums the run in order (contribution order) and
    // writes it at the run's rank among the runs, found by counting run heads chunk by chunk
    int out = 0;  // runs before the current chunk (wave-uniform)
    for (int base = 0; base < nsort; base += 64) {
        const int p = base + lane;
        const uint64_t kp = key[p];
        const bool valid = kp != ~0ull;
        const bool head = valid && (p == 0 || (key[p - 1] >> 20) != (kp >> 20));
        const uint64_t heads = __ballot(head);
        if (head) {
            const int rank = out + __popcll(heads & ((1ull << lane) - 1ull));
            const uint64_t J = kp >> 20;
            double acc = 0.0;
            for (int q = p; q < nsort && key[q] != ~0ull && (key[q] >> 20) == J; ++q) acc += sval[q];
            if (rank < Wc) {
                ccol[(int64_t)rank * gc.N + I] = (int32_t)J;
                cval[(int64_t)rank * gc.N + I] = acc;
            }
        }
        out += __popcll(heads);
        if (!__any(valid)) break;
    }
    // the widest row so far only grows: a row no wider than the value read skips the atomic (a stale read
    // costs one atomic more), so that most of the coarse rows do not queue on the one address
    if (lane == 0 && out > __atomic_load_n(widest, __ATOMIC_RELAXED)) atomicMax(widest, out);
    for (int s = out + lane; s < Wc; s += 64) ccol[(int64_t)s * gc.N + I] = -1;
}

// Jacobi divisor of an ELL level, the row's absolute sum sum_j |a_ij| (l1 Jacobi; boundary rows: 1), and,
// optionally, its FP32 weights.  Galerkin products of the wide-stencil operator need not be diagonally
// dominant, and plain damped Jacobi on them can diverge; the absolute row sum bounds the row's spectrum.
__global__ __launch_bounds__(kBlock) void k_gal_diag(int64_t N, int W, const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, float *__restrict__ val32,
                                                     float *__restrict__ d32, double *__restrict__ d64) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    double dg = 0.0;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * N + i];
        if (j >= 0) dg += fabs(val[s * N + i]);
        if (val32) val32[s * N + i] = j >= 0 ? (float)val[s * N + i] : 0.0f;
    }
    if (!(dg > 0.0)) dg = 1.0;
    if (d32) d32[i] = (float)dg;
    if (d64) d64[i] = dg;
}

// damped Jacobi on an ELL level: out = e + omega (r - A e) / d, or omega r / d (first sweep, e = 0)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gal_jacobi(int64_t N, int W, const int32_t *__restrict__ col,
                                                       const T *__restrict__ val, const T *__restrict__ d,
                                                       const T *__restrict__ e, const T *__restrict__ r,
                                                       T *__restrict__ out, T omega, int first) {
    const int64_t i = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= N) return;
    if (first) {
        out[i] = omega * r[i] / d[i];
        return;
    }
    T ae = (T)0;
    for (int s = 0; s < W; ++s) {  // a row's entries fill its first slots
        const int j = col[s * N + i];
        if (j < 0) break;
        ae += val[s * N + i] * e[j];
    }
    out[i] = e[i] + omega * (r[i] - ae) / d[i];
}

// res = r - A e on an ELL level
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gal_residual(int64_t N, int W, const int32_t *__restrict__ col,
                                                         const T *__restrict__ val, const T *__restrict__ e,
                                                         const T *__restrict__ r, T *__restrict__ res) {
    const int64_t i = (int64_t)remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= N) return;
    T ae = (T)0;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * N + i];
        if (j < 0) break;
        ae += val[s * N + i] * e[j];
    }
    res[i] = r[i] - ae;
}

void launch_gal_emit(int dim, const LevelDev &g, const StencilDev &st, const int16_t *alpha, double theta_dt, int E,
                     int32_t *col, double *val, hipStream_t s) {
    if (dim == 3)
        hipLaunchKernelGGL(k_gal_emit<3>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, theta_dt, E, col, val);
    else
        hipLaunchKernelGGL(k_gal_emit<2>, dim3(tiles_for(g)), dim3(kBlock), 0, s, g, st, alpha, theta_dt, E, col, val);
}

int gal_sort_size(int Wf) {
    int n = 64;
    while (n < 36 * Wf) n <<= 1;
    return n;
}

int launch_gal_rap(const LevelDev &gf, const LevelDev &gc, int Wf, const int32_t *fcol, const double *fval, int Wc,
                   int32_t *ccol, double *cval, int32_t *widest, hipStream_t s) {
    const int nsort = gal_sort_size(Wf);
    const dim3 grid((unsigned)gc.N), block(64);
#define RAP(NS) hipLaunchKernelGGL(k_gal_rap<NS>, grid, block, 0, s, gf, gc, Wf, fcol, fval, Wc, ccol, cval, widest)
    if (nsort <= 512) RAP(512);
    else if (nsort <= 1024) RAP(1024);
    else if (nsort <= 2048) RAP(2048);
    else if (nsort <= kGalMaxSort) RAP(kGalMaxSort);
    else return -1;
#undef RAP
    return 0;
}

void launch_gal_diag(int64_t N, int W, const int32_t *col, const double *val, float *val32, float *d32, double *d64,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_gal_diag, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, W, col, val, val32, d32, d64);
}

template <typename T>
void launch_gal_jacobi(int64_t N, int W, const int32_t *col, const T *val, const T *d, const T *e, const T *r, T *out,
                       double omega, bool first, hipStream_t s) {
    SLHJB_LAUNCH((k_gal_jacobi<T>), dim3(blocks_for(N)), dim3(kBlock), 0, s, N, W, col, val, d, e, r, out, (T)omega,
                 (int)first);
}

template <typename T>
void launch_gal_residual(int64_t N, int W, const int32_t *col, const T *val, const T *e, const T *r, T *res,
                         hipStream_t s) {
    SLHJB_LAUNCH((k_gal_residual<T>), dim3(blocks_for(N)), dim3(kBlock), 0, s, N, W, col, val, e, r, res);
}

template void launch_gal_jacobi<float>(int64_t, int, const int32_t *, const float *, const float *, const float *,
                                       const float *, float *, double, bool, hipStream_t);
template void launch_gal_jacobi<double>(int64_t, int, const int32_t *, const double *, const double *, const double *,
                                        const double *, double *, double, bool, hipStream_t);
template void launch_gal_residual<float>(int64_t, int, const int32_t *, const float *, const float *, const float *,
                                         float *, hipStream_t);
template void launch_gal_residual<double>(int64_t, int, const int32_t *, const double *, const double *,
                                          const double *, double *, hipStream_t);

}  // namespace slhjb
