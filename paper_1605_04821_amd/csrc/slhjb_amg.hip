// Aggregation-based algebraic multigrid (the introduction and Sections 3.4-3.5: aggregates formed along the
// strongest couplings, piecewise-constant transfer operators, Galerkin coarse matrices and a Krylov-accelerated
// cycle).  Kernels of the setup (finest rows merged, strength and handshake matching, aggregate numbering and
// member lists, coarse products, diagonals) and of the cycle (restriction by aggregate sums, prolongation by
// injection, ELL products, inner products and GCR updates whose coefficients stay on the device, the coarsest
// solve in one workgroup).
//
// Matrices are sliced ELL, slot-major: entry s of row i at s * n + i, column -1 unused, a row's entries in its
// first slots (the finest level's emitted rows, which have holes, are merged first).  An aggregate map agg[i]
// gives the coarse index of fine node i, or -1 for a node in no aggregate (an empty row of the finest grid's
// boundary, or a row dominant enough that the smoother alone resolves it).

#include "slhjb_device.h"

namespace slhjb {

constexpr int kAmgSortMax = 1024;  // contributions of one coarse row sorted in LDS, at most
constexpr int kAmgMergeMax = 8 * kMaxPts + 1;  // slots of an emitted finest row (3D: 8 corners per point)
constexpr int kAmgCoarseThreads = 1024;

// ---- setup -----------------------------------------------------------------------------------------------

// Emitted rows (E slots with holes, duplicate columns where landings share interpolation corners) merged into
// one entry per column, in order of first occurrence, duplicates summed in slot order; columns of boundary
// nodes (nx x ny x nz grid, nz = 1 in 2D) are dropped, their values being Dirichlet data of the right-hand
// side, so that the rows are those of the system on the interior unknowns.  One wavefront per row.
__global__ __launch_bounds__(256) void k_amg_merge(int64_t n, int nx, int ny, int nz, int E,
                                                   const int32_t *__restrict__ icol, const double *__restrict__ ival,
                                                   int32_t *__restrict__ ocol, double *__restrict__ oval) {
    __shared__ int32_t sc[4][kAmgMergeMax];
    __shared__ double sv[4][kAmgMergeMax];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    const bool row = i < n;
    for (int c = lane; c < E; c += 64) {
        int j = row ? icol[(int64_t)c * n + i] : -1;
        if (j >= 0) {
            const int jx = j % nx, jr = j / nx, jy = jr % ny, jz = jr / ny;
            if (jx == 0 || jx == nx - 1 || jy == 0 || jy == ny - 1 || (nz > 1 && (jz == 0 || jz == nz - 1))) j = -1;
        }
        sc[w][c] = j;
        sv[w][c] = row ? ival[(int64_t)c * n + i] : 0.0;
    }
    __syncthreads();
    if (!row) return;
    int out = 0;
    for (int base = 0; base < E; base += 64) {
        const int p = base + lane;
        const int j = p < E ? sc[w][p] : -1;
        bool head = j >= 0;
        for (int q = 0; q < p && head; ++q) head = sc[w][q] != j;
        const uint64_t heads = __ballot(head);
        if (head) {
            double acc = 0.0;
            for (int q = p; q < E; ++q)
                if (sc[w][q] == j) acc += sv[w][q];
            const int rank = out + __popcll(heads & ((1ull << lane) - 1ull));
            ocol[(int64_t)rank * n + i] = j;
            oval[(int64_t)rank * n + i] = acc;
        }
        out += __popcll(heads);
    }
    for (int s = out + lane; s < E; s += 64) ocol[(int64_t)s * n + i] = -1;
}

// matching state: -2 takes no part, -1 unmatched, >= 0 matched partner.  Rows without entries take no part;
// with dd > 0, neither do rows with a_ii >= dd * sum_{j != i} |a_ij|
__global__ __launch_bounds__(kBlock) void k_amg_init(int64_t n, int W, const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, double dd,
                                                     int32_t *__restrict__ mate) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double diag = 0.0, off = 0.0;
    int cnt = 0;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * n + i];
        if (j < 0) break;
        ++cnt;
        if (j == i) diag += val[s * n + i];
        else off += fabs(val[s * n + i]);
    }
    mate[i] = (cnt == 0 || (dd > 0.0 && diag >= dd * off)) ? -2 : -1;
}

// Symmetric part of the off-diagonal couplings, S = -(M + M^T)/2 (Sections 3.4-3.5: the aggregation theory
// for these nonsymmetric M-matrices rests on the symmetric part), in three steps: count the entries of each
// column and atomically scatter them (row, value) into column segments (transposed rows, in any order); then
// row i of S lists, for every j != i coupled to i in either direction, w_ij = -(m_ij + m_ji)/2 when positive.
// The same two numbers are added at both ends, so w_ij = w_ji exactly, and the segment order does not matter.
__global__ __launch_bounds__(kBlock) void k_amg_colcount(int64_t n, int W, const int32_t *__restrict__ col,
                                                         int32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * n + i];
        if (j < 0) break;
        if (j != i) atomicAdd(&cnt[j], 1);
    }
}
__global__ __launch_bounds__(kBlock) void k_amg_colmax(int64_t n, const int32_t *__restrict__ cnt,
                                                       int32_t *__restrict__ mx) {
    __shared__ int32_t sm[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    sm[threadIdx.x] = i < n ? cnt[i] : 0;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && sm[0] > __atomic_load_n(mx, __ATOMIC_RELAXED)) atomicMax(mx, sm[0]);
}
__global__ __launch_bounds__(kBlock) void k_amg_scatter(int64_t n, int W, const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const int32_t *__restrict__ off, int32_t *__restrict__ fill,
                                                        int32_t *__restrict__ trow, double *__restrict__ tval) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * n + i];
        if (j < 0) break;
        if (j == i) continue;
        const int p = off[j] + atomicAdd(&fill[j], 1);
        trow[p] = (int)i;
        tval[p] = val[s * n + i];
    }
}
__global__ __launch_bounds__(kBlock) void k_amg_sym(int64_t n, int W, const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ cnt, const int32_t *__restrict__ trow,
                                                    const double *__restrict__ tval, int Ws, int32_t *__restrict__ scol,
                                                    double *__restrict__ sval) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int t0 = off[i], t1 = off[i] + cnt[i];
    int k = 0;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * n + i];
        if (j < 0) break;
        if (j == i) continue;
        // the last entry of column i's segment from row j (searched from the end, so the search stops there)
        double b = 0.0;
        for (int p = t1 - 1; p >= t0; --p)
            if (trow[p] == j) {
                b = tval[p];
                break;
            }
        const double w = -0.5 * (val[s * n + i] + b);
        if (w > 0.0) {
            scol[(int64_t)k * n + i] = j;
            sval[(int64_t)k * n + i] = w;
            ++k;
        }
    }
    for (int p = t0; p < t1; ++p) {
        const int j = trow[p];
        bool in_row = false;
        for (int s = 0; s < W; ++s) {
            const int c = col[s * n + i];
            if (c < 0) break;
            if (c == j) {
                in_row = true;
                break;
            }
        }
        if (in_row) continue;
        const double w = -0.5 * (tval[p] + 0.0);
        if (w > 0.0) {
            scol[(int64_t)k * n + i] = j;
            sval[(int64_t)k * n + i] = w;
            ++k;
        }
    }
    for (; k < Ws; ++k) scol[(int64_t)k * n + i] = -1;
}

// the same rows of S for wide levels: one wavefront per row (four rows per workgroup), the row and chunks of
// its column segment staged in LDS, so that the lookups run at LDS speed and in parallel over the row's entries
constexpr int kSymRow = 512, kSymChunk = 256;
__global__ __launch_bounds__(256) void k_amg_sym_wave(int64_t n, int W, const int32_t *__restrict__ col,
                                                      const double *__restrict__ val, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ cnt, const int32_t *__restrict__ trow,
                                                      const double *__restrict__ tval, int Ws,
                                                      int32_t *__restrict__ scol, double *__restrict__ sval) {
    __shared__ int32_t rc[4][kSymRow], tc[4][kSymChunk];
    __shared__ double rv[4][kSymRow], rb[4][kSymRow], tv[4][kSymChunk];
    __shared__ int tns[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    const bool row = i < n;
    for (int s = lane; s < W; s += 64) {
        const int c = row ? col[s * n + i] : -1;
        rc[w][s] = c;
        rv[w][s] = c >= 0 ? val[s * n + i] : 0.0;
        rb[w][s] = 0.0;
    }
    const int t0 = row ? off[i] : 0, tn = row ? cnt[i] : 0;
    if (lane == 0) tns[w] = tn;
    __syncthreads();
    const int tmax = max(max(tns[0], tns[1]), max(tns[2], tns[3]));
    int k = 0;  // entries written (wave-uniform)
    auto emit = [&](bool e, int j, double wv) {
        const uint64_t m = __ballot(e);
        if (e) {
            const int slot = k + __popcll(m & ((1ull << lane) - 1ull));
            scol[(int64_t)slot * n + i] = j;
            sval[(int64_t)slot * n + i] = wv;
        }
        k += __popcll(m);
    };
    for (int base = 0; base < tmax; base += kSymChunk) {  // the same trip count in every wave of the block
        const int m = max(0, min(kSymChunk, tn - base));
        for (int q = lane; q < m; q += 64) {
            tc[w][q] = trow[t0 + base + q];
            tv[w][q] = tval[t0 + base + q];
        }
        __syncthreads();
        for (int s = lane; s < W; s += 64) {
            const int c = rc[w][s];
            if (c < 0 || c == (int)i) continue;
            for (int q = 0; q < m; ++q)
                if (tc[w][q] == c) rb[w][s] = tv[w][q];
        }
        for (int q0 = 0; q0 < m; q0 += 64) {
            const int q = q0 + lane;
            bool e = false;
            int j = -1;
            double wv = 0.0;
            if (q < m) {
                j = tc[w][q];
                bool in_row = false;
                for (int s = 0; s < W; ++s) {
                    const int c = rc[w][s];
                    if (c < 0) break;
                    in_row = in_row || c == j;
                }
                wv = -0.5 * (tv[w][q] + 0.0);
                e = !in_row && wv > 0.0;
            }
            emit(e, j, wv);
        }
        __syncthreads();
    }
    if (!row) return;
    for (int s0 = 0; s0 < W; s0 += 64) {
        const int s = s0 + lane;
        bool e = false;
        int j = -1;
        double wv = 0.0;
        if (s < W) {
            j = rc[w][s];
            if (j >= 0 && j != (int)i) {
                wv = -0.5 * (rv[w][s] + rb[w][s]);
                e = wv > 0.0;
            }
        }
        emit(e, j, wv);
    }
    for (int s = k + lane; s < Ws; s += 64) scol[(int64_t)s * n + i] = -1;
}

// the order in which both ends of an edge rank it among equally strong ones: a hash of the unordered pair,
// then the pair itself (a total order, so the strongest edge of a neighbourhood is each end's choice)
__device__ __forceinline__ uint64_t edge_rank(int i, int j) {
    const uint32_t a = (uint32_t)min(i, j), b = (uint32_t)max(i, j);
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return ((uint64_t)h << 32) | (uint64_t)(a ^ (b << 16) ^ (b >> 16));
}

// strongest admissible partner of each unmatched node on S: an unmatched j with w_ij >= beta * max_k w_ik,
// the largest w_ij, equal ones ordered by edge_rank (then by j); -1 if there is none
__global__ __launch_bounds__(kBlock) void k_amg_strong(int64_t n, int Ws, const int32_t *__restrict__ scol,
                                                       const double *__restrict__ sval, double beta,
                                                       const int32_t *__restrict__ mate, int32_t *__restrict__ cand) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (mate[i] != -1) {
        cand[i] = -1;
        return;
    }
    double mx = 0.0;
    for (int s = 0; s < Ws; ++s) {
        const int j = scol[s * n + i];
        if (j < 0) break;
        mx = fmax(mx, sval[s * n + i]);
    }
    int best = -1;
    double bs = 0.0;
    uint64_t br = 0;
    for (int s = 0; s < Ws; ++s) {
        const int j = scol[s * n + i];
        if (j < 0) break;
        if (mate[j] != -1) continue;
        const double a = sval[s * n + i];
        if (a < beta * mx) continue;
        const uint64_t r = edge_rank((int)i, j);
        if (best < 0 || a > bs || (a == bs && (r > br || (r == br && j < best)))) {
            bs = a;
            br = r;
            best = j;
        }
    }
    cand[i] = best;
}

// the same choice for wide rows of S: one wavefront per row (four per workgroup), the maximum and the best
// entry reduced across lanes
__device__ __forceinline__ bool better(double a, uint64_t r, int j, double b, uint64_t rb, int jb) {
    if (jb < 0) return j >= 0;
    if (j < 0) return false;
    return a > b || (a == b && (r > rb || (r == rb && j < jb)));
}
__global__ __launch_bounds__(256) void k_amg_strong_wave(int64_t n, int Ws, const int32_t *__restrict__ scol,
                                                         const double *__restrict__ sval, double beta,
                                                         const int32_t *__restrict__ mate, int32_t *__restrict__ cand) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    if (mate[i] != -1) {
        if (lane == 0) cand[i] = -1;
        return;
    }
    double mx = 0.0;
    for (int s = lane; s < Ws; s += 64) {
        const int j = scol[s * n + i];
        if (j < 0) break;
        mx = fmax(mx, sval[s * n + i]);
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    int best = -1;
    double bs = 0.0;
    uint64_t br = 0;
    for (int s = lane; s < Ws; s += 64) {
        const int j = scol[s * n + i];
        if (j < 0) break;
        if (mate[j] != -1) continue;
        const double a = sval[s * n + i];
        if (a < beta * mx) continue;
        const uint64_t r = edge_rank((int)i, j);
        if (better(a, r, j, bs, br, best)) {
            bs = a;
            br = r;
            best = j;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double a = __shfl_xor(bs, o, 64);
        const uint64_t r = __shfl_xor(br, o, 64);
        const int j = __shfl_xor(best, o, 64);
        if (better(a, r, j, bs, br, best)) {
            bs = a;
            br = r;
            best = j;
        }
    }
    if (lane == 0) cand[i] = best;
}

// handshake: i and j pair when each is the other's candidate
__global__ __launch_bounds__(kBlock) void k_amg_handshake(int64_t n, const int32_t *__restrict__ cand,
                                                          int32_t *__restrict__ mate) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || mate[i] != -1) return;
    const int j = cand[i];
    if (j >= 0 && cand[j] == (int)i) mate[i] = j;
}

// one aggregate per singleton and per pair (led by its smaller node): flag 1 at the leaders
__global__ __launch_bounds__(kBlock) void k_amg_leader(int64_t n, const int32_t *__restrict__ mate,
                                                       int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int m = mate[i];
    flag[i] = (m == -1 || (m >= 0 && (int)i < m)) ? 1 : 0;
}

// aggregate of every node (id: exclusive prefix sums of the leader flags) and each aggregate's members
// (leader, then partner or -1)
__global__ __launch_bounds__(kBlock) void k_amg_assign(int64_t n, const int32_t *__restrict__ mate,
                                                       const int32_t *__restrict__ id, int32_t *__restrict__ agg,
                                                       int32_t *__restrict__ mem2) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int m = mate[i];
    if (m == -2) {
        agg[i] = -1;
        return;
    }
    const bool lead = m == -1 || (int)i < m;
    const int a = lead ? id[i] : id[m];
    agg[i] = a;
    if (lead) {
        mem2[2 * (int64_t)a] = (int)i;
        mem2[2 * (int64_t)a + 1] = m >= 0 ? m : -1;
    }
}

// two pairings composed: agg[i] = agg2[agg1[i]], and the (up to) four members of each final aggregate
__global__ __launch_bounds__(kBlock) void k_amg_compose(int64_t n, const int32_t *__restrict__ agg1,
                                                        const int32_t *__restrict__ agg2, int32_t *__restrict__ agg) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int a = agg1[i];
    agg[i] = a >= 0 ? agg2[a] : -1;
}
__global__ __launch_bounds__(kBlock) void k_amg_members4(int64_t nc, const int32_t *__restrict__ mem2b,
                                                         const int32_t *__restrict__ mem2a, int32_t *__restrict__ mem4) {
    const int64_t A = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (A >= nc) return;
    for (int p = 0; p < 2; ++p) {
        const int b = mem2b[2 * A + p];
        mem4[4 * A + 2 * p] = b >= 0 ? mem2a[2 * (int64_t)b] : -1;
        mem4[4 * A + 2 * p + 1] = b >= 0 ? mem2a[2 * (int64_t)b + 1] : -1;
    }
}

// coarse row A of P^T M P for piecewise-constant P: the entries of A's members (mem[maxm * A ..]), columns
// mapped to their aggregates, sorted by (coarse column, contribution index) in LDS and each column's run
// summed in that order, so the result does not depend on scheduling.  *widest receives the largest row.
// One wavefront per coarse row, R rows per workgroup (millions of one-wave workgroups are dispatch-bound).
template <int NSORT, int R>
__global__ __launch_bounds__(64 * R) void k_amg_product(int64_t nf, int W, const int32_t *__restrict__ fcol,
                                                        const double *__restrict__ fval,
                                                        const int32_t *__restrict__ agg, const int32_t *__restrict__ mem,
                                                        int maxm, int64_t nc, int Wc, int32_t *__restrict__ ccol,
                                                        double *__restrict__ cval, int32_t *__restrict__ widest) {
    __shared__ uint64_t keys[R][NSORT];
    __shared__ double svals[R][NSORT];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t A = (int64_t)blockIdx.x * R + wv;  // one wavefront per coarse row
    const bool rowok = A < nc;
    uint64_t *key = keys[wv];
    double *sval = svals[wv];
    const int total = maxm * W;
    for (int c = lane; c < NSORT; c += 64) {
        uint64_t kk = ~0ull;
        double v = 0.0;
        if (rowok && c < total) {
            const int m = mem[(int64_t)maxm * A + c / W];
            const int s = c % W;
            if (m >= 0) {
                const int j = fcol[(int64_t)s * nf + m];
                const int J = j >= 0 ? agg[j] : -1;
                if (J >= 0) {
                    kk = ((uint64_t)J << 20) | (uint64_t)c;
                    v = fval[(int64_t)s * nf + m];
                }
            }
        }
        key[c] = kk;
        sval[c] = v;
    }
    __syncthreads();
    for (int size = 2; size <= NSORT; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < NSORT / 2; t += 64) {
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
    if (!rowok) return;
    int out = 0;  // columns before the current chunk (wave-uniform)
    for (int base = 0; base < NSORT; base += 64) {
        const int p = base + lane;
        const uint64_t kp = key[p];
        const bool valid = kp != ~0ull;
        const bool head = valid && (p == 0 || (key[p - 1] >> 20) != (kp >> 20));
        const uint64_t heads = __ballot(head);
        if (head) {
            const int rank = out + __popcll(heads & ((1ull << lane) - 1ull));
            const uint64_t J = kp >> 20;
            double acc = 0.0;
            for (int q = p; q < NSORT && key[q] != ~0ull && (key[q] >> 20) == J; ++q) acc += sval[q];
            if (rank < Wc) {
                ccol[(int64_t)rank * nc + A] = (int32_t)J;
                cval[(int64_t)rank * nc + A] = acc;
            }
        }
        out += __popcll(heads);
        if (!__any(valid)) break;
    }
    // the widest row so far only grows: a row no wider than the value read skips the atomic (a stale read
    // costs one atomic more), so that most of the coarse rows do not queue on the one address
    if (lane == 0 && out > __atomic_load_n(widest, __ATOMIC_RELAXED)) atomicMax(widest, out);
    for (int s = out + lane; s < Wc; s += 64) ccol[(int64_t)s * nc + A] = -1;
}

// diagonal of an ELL level (1 where a row has none: rows outside every aggregate never reach a coarse level)
__global__ __launch_bounds__(kBlock) void k_amg_diag(int64_t n, int W, const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, double *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double dg = 0.0;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * n + i];
        if (j < 0) break;
        if (j == i) dg += val[s * n + i];
    }
    d[i] = dg > 0.0 ? dg : 1.0;
}

// ---- cycle -----------------------------------------------------------------------------------------------

// r_c[A] = sum of r over A's members, in member order (the transpose of the piecewise-constant prolongation)
__global__ __launch_bounds__(kBlock) void k_amg_restrict(int64_t nc, const int32_t *__restrict__ mem4,
                                                         const double *__restrict__ rf, double *__restrict__ rc) {
    const int64_t A = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (A >= nc) return;
    double s = 0.0;
    for (int q = 0; q < 4; ++q) {
        const int m = mem4[4 * A + q];
        if (m >= 0) s += rf[m];
    }
    rc[A] = s;
}

// e_f[i] += e_c[agg[i]]
__global__ __launch_bounds__(kBlock) void k_amg_prolong(int64_t nf, const int32_t *__restrict__ agg,
                                                        const double *__restrict__ ec, double *__restrict__ ef) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nf) return;
    const int a = agg[i];
    if (a >= 0) ef[i] += ec[a];
}

// y = A x on an ELL level
__global__ __launch_bounds__(kBlock) void k_amg_spmv(int64_t n, int W, const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, const double *__restrict__ x,
                                                     double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    for (int s = 0; s < W; ++s) {
        const int j = col[s * n + i];
        if (j < 0) break;
        a += val[s * n + i] * x[j];
    }
    y[i] = a;
}

// (a, b) and (a, c) over n entries: per-block sums of a grid-strided range in a fixed tree order; with one block
// the sums go to out[0..1], else to part[2 * block ..] for k_amg_dot2_final
__global__ __launch_bounds__(1024) void k_amg_dot2(int64_t n, const double *__restrict__ a,
                                                   const double *__restrict__ b, const double *__restrict__ c,
                                                   double *__restrict__ part, double *__restrict__ out) {
    __shared__ double s0[1024], s1[1024];
    double x = 0.0, y = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 1024) {
        const double ai = a[i];
        x += ai * b[i];
        y += ai * c[i];
    }
    s0[threadIdx.x] = x;
    s1[threadIdx.x] = y;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *dst = gridDim.x == 1 ? out : part + 2 * (int64_t)blockIdx.x;
        dst[0] = s0[0];
        dst[1] = s1[0];
    }
}
__global__ __launch_bounds__(1024) void k_amg_dot2_final(int nb, const double *__restrict__ part,
                                                         double *__restrict__ out) {
    __shared__ double s0[1024], s1[1024];
    double x = 0.0, y = 0.0;
    for (int q = threadIdx.x; q < nb; q += 1024) {
        x += part[2 * q];
        y += part[2 * q + 1];
    }
    s0[threadIdx.x] = x;
    s1[threadIdx.x] = y;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
    }
}

// GCR updates with the coefficient c = sc[0] / sc[1] read on the device (0 when sc[1] = 0):
//   mode 0: x = c v, r_out = r - c w                  (sc: (w, r), (w, w))
//   mode 1: v -= c v1, w -= c w1                       (sc: (w1, w), (w1, w1))
//   mode 2: x += c v                                   (sc: (w, r), (w, w))
__global__ __launch_bounds__(kBlock) void k_amg_gcr(int64_t n, int mode, const double *__restrict__ sc,
                                                    double *__restrict__ x, double *__restrict__ v,
                                                    double *__restrict__ w, const double *__restrict__ v1,
                                                    const double *__restrict__ w1, const double *__restrict__ r,
                                                    double *__restrict__ r_out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double c = sc[1] != 0.0 ? sc[0] / sc[1] : 0.0;
    if (mode == 0) {
        x[i] = c * v[i];
        r_out[i] = r[i] - c * w[i];
    } else if (mode == 1) {
        v[i] -= c * v1[i];
        w[i] -= c * w1[i];
    } else {
        x[i] += c * v[i];
    }
}

// coarsest level (n <= kAmgCoarseMax): `sweeps` Jacobi sweeps x <- x + (r - A x) / d from x = 0, the iterate
// in LDS, one workgroup
__global__ __launch_bounds__(kAmgCoarseThreads) void k_amg_coarse(int n, int W, const int32_t *__restrict__ col,
                                                                  const double *__restrict__ val,
                                                                  const double *__restrict__ d,
                                                                  const double *__restrict__ r, int sweeps,
                                                                  double *__restrict__ x) {
    __shared__ double xa[kAmgCoarseMax], xb[kAmgCoarseMax];
    double *cur = xa, *nxt = xb;
    for (int i = threadIdx.x; i < n; i += kAmgCoarseThreads) cur[i] = r[i] / d[i];
    __syncthreads();
    for (int q = 1; q < sweeps; ++q) {
        for (int i = threadIdx.x; i < n; i += kAmgCoarseThreads) {
            double a = 0.0;
            for (int s = 0; s < W; ++s) {
                const int j = col[s * n + i];
                if (j < 0) break;
                a += val[s * n + i] * cur[j];
            }
            nxt[i] = cur[i] + (r[i] - a) / d[i];
        }
        __syncthreads();
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int i = threadIdx.x; i < n; i += kAmgCoarseThreads) x[i] = cur[i];
}

// coarsest level with n <= kAmgDenseMax rows: the dense inverse of its matrix by Gauss-Jordan elimination in
// place in LDS, without pivoting (the aggregated matrices are M-matrices with non-negative row sums and a
// positive diagonal: diagonally dominant, so every pivot stays positive); one workgroup
__global__ __launch_bounds__(kAmgCoarseThreads) void k_amg_dense_inverse(int n, int W, const int32_t *__restrict__ col,
                                                                         const double *__restrict__ val,
                                                                         double *__restrict__ inv) {
    __shared__ double a[kAmgDenseMax * kAmgDenseMax];
    __shared__ double prow[kAmgDenseMax], pcol[kAmgDenseMax];
    for (int q = threadIdx.x; q < n * n; q += kAmgCoarseThreads) a[q] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kAmgCoarseThreads)
        for (int s = 0; s < W; ++s) {
            const int j = col[s * n + i];
            if (j < 0) break;
            a[i * n + j] += val[s * n + i];
        }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double p = 1.0 / a[k * n + k];
        // the pivot row scaled, the pivot column saved before the sweep overwrites it
        for (int j = threadIdx.x; j < n; j += kAmgCoarseThreads) {
            prow[j] = (j == k ? 1.0 : a[k * n + j]) * p;
            pcol[j] = a[j * n + k];
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n * n; q += kAmgCoarseThreads) {
            const int i = q / n, j = q % n;
            if (i == k) a[q] = prow[j];
            else a[q] = (j == k ? 0.0 : a[q]) - pcol[i] * prow[j];
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < n * n; q += kAmgCoarseThreads) inv[q] = a[q];
}

// x = inv r on the coarsest level: one row per wavefront lane group, rows in order
__global__ __launch_bounds__(kAmgCoarseThreads) void k_amg_dense_solve(int n, const double *__restrict__ inv,
                                                                       const double *__restrict__ r,
                                                                       double *__restrict__ x) {
    __shared__ double rs[kAmgDenseMax];
    for (int j = threadIdx.x; j < n; j += kAmgCoarseThreads) rs[j] = r[j];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kAmgCoarseThreads) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += inv[i * n + j] * rs[j];
        x[i] = acc;
    }
}

// ---- wide levels: row-major copies and one wavefront per row ----------------------------------------------
// Coarse aggregation levels have rows of tens to hundreds of entries over few rows: one thread per row leaves
// most of the GPU idle and walks each row serially.  Such levels keep a row-major copy (entry s of row i at
// i * W + s) and the cycle's kernels give each row one wavefront: lanes take the row's entries in strides of
// 64 (coalesced) and the partial sums are combined by a fixed butterfly, so the result does not depend on
// scheduling.

__global__ __launch_bounds__(kBlock) void k_amg_rowmajor(int64_t n, int W, const int32_t *__restrict__ col,
                                                         const double *__restrict__ val, int32_t *__restrict__ rcol,
                                                         double *__restrict__ rval) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;  // entry of the row-major copy
    if (q >= n * W) return;
    const int64_t i = q / W;
    const int s = (int)(q % W);
    const int j = col[(int64_t)s * n + i];
    rcol[q] = j;
    rval[q] = j >= 0 ? val[(int64_t)s * n + i] : 0.0;
}

__device__ __forceinline__ double wave_row_dot(int64_t i, int W, const int32_t *__restrict__ rcol,
                                               const double *__restrict__ rval, const double *__restrict__ x,
                                               int lane) {
    double a = 0.0;
    const int64_t base = i * W;
    for (int s = lane; s < W; s += 64) {
        const int j = rcol[base + s];
        if (j >= 0) a += rval[base + s] * x[j];
    }
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
}

// mode 0: y = A x; mode 1: y = r - A x; mode 2: Jacobi y = x + omega (r - A x) / d (first: y = omega r / d)
__global__ __launch_bounds__(256) void k_amg_wave_op(int64_t n, int W, const int32_t *__restrict__ rcol,
                                                     const double *__restrict__ rval, const double *__restrict__ d,
                                                     const double *__restrict__ x, const double *__restrict__ r,
                                                     double *__restrict__ y, int mode, double omega, int first) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    if (mode == 2 && first) {
        if (lane == 0) y[i] = omega * r[i] / d[i];
        return;
    }
    const double a = wave_row_dot(i, W, rcol, rval, x, lane);
    if (lane != 0) return;
    if (mode == 0) y[i] = a;
    else if (mode == 1) y[i] = r[i] - a;
    else y[i] = x[i] + omega * (r[i] - a) / d[i];
}

// ---- launchers -------------------------------------------------------------------------------------------

static unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }

void launch_amg_merge(int64_t n, int nx, int ny, int nz, int E, const int32_t *icol, const double *ival,
                      int32_t *ocol, double *oval, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_merge, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, nx, ny, nz, E, icol, ival,
                       ocol, oval);
}
void launch_amg_init(int64_t n, int W, const int32_t *col, const double *val, double dd, int32_t *mate,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_amg_init, dim3(grid_for(n)), dim3(kBlock), 0, s, n, W, col, val, dd, mate);
}
void launch_amg_colcount(int64_t n, int W, const int32_t *col, int32_t *cnt, int32_t *mx, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_colcount, dim3(grid_for(n)), dim3(kBlock), 0, s, n, W, col, cnt);
    hipLaunchKernelGGL(k_amg_colmax, dim3(grid_for(n)), dim3(kBlock), 0, s, n, (const int32_t *)cnt, mx);
}
void launch_amg_scatter(int64_t n, int W, const int32_t *col, const double *val, const int32_t *off, int32_t *fill,
                        int32_t *trow, double *tval, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_scatter, dim3(grid_for(n)), dim3(kBlock), 0, s, n, W, col, val, off, fill, trow, tval);
}
int launch_amg_sym(int64_t n, int W, int maxcol, const int32_t *col, const double *val, const int32_t *off,
                   const int32_t *cnt, const int32_t *trow, const double *tval, int Ws, int32_t *scol, double *sval,
                   hipStream_t s) {
    // one thread per row where rows are narrow, or many and of moderate width (it then fills the GPU; the long
    // columns of a few rows cost only their own threads), one wavefront per row on wide levels
    if ((W <= 32 && maxcol <= 32) || (n > kAmgWaveRows && W <= 48)) {
        hipLaunchKernelGGL(k_amg_sym, dim3(grid_for(n)), dim3(kBlock), 0, s, n, W, col, val, off, cnt, trow, tval, Ws,
                           scol, sval);
        return 0;
    }
    if (W > kSymRow) return -1;
    hipLaunchKernelGGL(k_amg_sym_wave, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, W, col, val, off, cnt, trow,
                       tval, Ws, scol, sval);
    return 0;
}
void launch_amg_match_round(int64_t n, int Ws, const int32_t *scol, const double *sval, double beta, int32_t *mate,
                            int32_t *cand, hipStream_t s) {
    if (Ws > 64 && n <= kAmgWaveRows)
        hipLaunchKernelGGL(k_amg_strong_wave, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, Ws, scol, sval, beta,
                           (const int32_t *)mate, cand);
    else
        hipLaunchKernelGGL(k_amg_strong, dim3(grid_for(n)), dim3(kBlock), 0, s, n, Ws, scol, sval, beta,
                           (const int32_t *)mate, cand);
    hipLaunchKernelGGL(k_amg_handshake, dim3(grid_for(n)), dim3(kBlock), 0, s, n, (const int32_t *)cand, mate);
}
void launch_amg_leader(int64_t n, const int32_t *mate, int32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_leader, dim3(grid_for(n)), dim3(kBlock), 0, s, n, mate, flag);
}
void launch_amg_assign(int64_t n, const int32_t *mate, const int32_t *id, int32_t *agg, int32_t *mem2, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_assign, dim3(grid_for(n)), dim3(kBlock), 0, s, n, mate, id, agg, mem2);
}
void launch_amg_compose(int64_t n, const int32_t *agg1, const int32_t *agg2, int32_t *agg, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_compose, dim3(grid_for(n)), dim3(kBlock), 0, s, n, agg1, agg2, agg);
}
void launch_amg_members4(int64_t nc, const int32_t *mem2b, const int32_t *mem2a, int32_t *mem4, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_members4, dim3(grid_for(nc)), dim3(kBlock), 0, s, nc, mem2b, mem2a, mem4);
}
int launch_amg_product(int64_t nf, int W, const int32_t *fcol, const double *fval, const int32_t *agg,
                       const int32_t *mem, int maxm, int64_t nc, int Wc, int32_t *ccol, double *cval, int32_t *widest,
                       hipStream_t s) {
    if (nc <= 0) return 0;
    const int total = maxm * W;
#define PR(NS, R)                                                                                                  \
    hipLaunchKernelGGL((k_amg_product<NS, R>), dim3((unsigned)((nc + R - 1) / R)), dim3(64 * R), 0, s, nf, W, fcol, \
                       fval, agg, mem, maxm, nc, Wc, ccol, cval, widest)
    if (total <= 128) PR(128, 4);
    else if (total <= 256) PR(256, 4);
    else if (total <= 512) PR(512, 4);
    else if (total <= kAmgSortMax) PR(kAmgSortMax, 2);
    else return -1;
#undef PR
    return 0;
}
void launch_amg_diag(int64_t n, int W, const int32_t *col, const double *val, double *d, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_diag, dim3(grid_for(n)), dim3(kBlock), 0, s, n, W, col, val, d);
}
void launch_amg_restrict(int64_t nc, const int32_t *mem4, const double *rf, double *rc, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_restrict, dim3(grid_for(nc)), dim3(kBlock), 0, s, nc, mem4, rf, rc);
}
void launch_amg_prolong(int64_t nf, const int32_t *agg, const double *ec, double *ef, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_prolong, dim3(grid_for(nf)), dim3(kBlock), 0, s, nf, agg, ec, ef);
}
void launch_amg_spmv(int64_t n, int W, const int32_t *col, const double *val, const double *x, double *y,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_amg_spmv, dim3(grid_for(n)), dim3(kBlock), 0, s, n, W, col, val, x, y);
}
int amg_dot_parts(int64_t n) { return n <= 32768 ? 1 : (int)std::min<int64_t>(1024, (n + 8191) / 8192); }
void launch_amg_dot2(int64_t n, const double *a, const double *b, const double *c, double *part, double *out,
                     hipStream_t s) {
    const int nb = amg_dot_parts(n);
    hipLaunchKernelGGL(k_amg_dot2, dim3(nb), dim3(1024), 0, s, n, a, b, c, part, out);
    if (nb > 1) hipLaunchKernelGGL(k_amg_dot2_final, dim3(1), dim3(1024), 0, s, nb, (const double *)part, out);
}
void launch_amg_gcr(int64_t n, int mode, const double *sc, double *x, double *v, double *w, const double *v1,
                    const double *w1, const double *r, double *r_out, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_gcr, dim3(grid_for(n)), dim3(kBlock), 0, s, n, mode, sc, x, v, w, v1, w1, r, r_out);
}
void launch_amg_coarse(int n, int W, const int32_t *col, const double *val, const double *d, const double *r,
                       int sweeps, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_coarse, dim3(1), dim3(kAmgCoarseThreads), 0, s, n, W, col, val, d, r, sweeps, x);
}
void launch_amg_rowmajor(int64_t n, int W, const int32_t *col, const double *val, int32_t *rcol, double *rval,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_amg_rowmajor, dim3(grid_for(n * W)), dim3(kBlock), 0, s, n, W, col, val, rcol, rval);
}
void launch_amg_wave_op(int64_t n, int W, const int32_t *rcol, const double *rval, const double *d, const double *x,
                        const double *r, double *y, int mode, double omega, bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_wave_op, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, W, rcol, rval, d, x, r, y,
                       mode, omega, (int)first);
}
void launch_amg_dense_inverse(int n, int W, const int32_t *col, const double *val, double *inv, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_dense_inverse, dim3(1), dim3(kAmgCoarseThreads), 0, s, n, W, col, val, inv);
}
void launch_amg_dense_solve(int n, const double *inv, const double *r, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_amg_dense_solve, dim3(1), dim3(kAmgCoarseThreads), 0, s, n, inv, r, x);
}

}  // namespace slhjb
