// Host driver of libslhjb: handle and workspace, per-level stencil tables, policy iteration,
// flexible GMRES with a geometric multigrid V-cycle preconditioner, time march, and the C ABI
// declared in include/slhjb.h.
//
// Method: Reisinger & Rotaetxe Arto (arXiv:1605.04821).  Each theta-step (eq. FullScheme) is a
// row-wise nonlinear system (eq. nonlinear_sys) solved by Howard policy iteration; each policy's
// linear system is an M-matrix with row sums >= 1 - theta dt max(c,0) (Section 3.4), so the
// infinity-norm residual bounds the error and serves as the stopping certificate.
// The V-cycle rediscretises the operator on each coarse level with the same physical stencil
// displacements (the 1/(2h) scaling of the finest grid is kept), injects the fine policy, smooths
// with damped Jacobi (the paper's Gauss-Seidel is sequential) and transfers with full weighting and
// multilinear prolongation.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/slhjb.h"
#include "slhjb_internal.h"

using namespace slhjb;

namespace slhjb {
int dot_blocks(int64_t N);
}

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// Slots of the small device/host scalar arrays (dvals, hpin): [0, 16) solver scalars, [16, 23) the
// BiCGSTAB recurrence, 200 the adjoint gradient term, 230 the widest Galerkin row, and the two
// Gram-Schmidt passes of one Arnoldi step from kGsSlot0 and kGsSlot1 (m + 2 each).
constexpr int kGsSlot0 = 256, kGsSlot1 = kGsSlot0 + kMaxRestart + 2;
constexpr int kGalSlot = 230;  // the widest Galerkin row
constexpr int kSmallSlots = 512;
static_assert(kGsSlot1 + kMaxRestart + 2 <= kSmallSlots, "small-slot layout");

#define HIPCHK(call)                                                                         \
    do {                                                                                     \
        hipError_t _e = (call);                                                              \
        if (_e != hipSuccess) return fail(HJB_EDEVICE, "%s: %s", #call, hipGetErrorString(_e)); \
    } while (0)

struct Level {
    LevelDev g{};
    PointTab *tab = nullptr;  // device [K][npt]
    FastPtF *fastF = nullptr; // device [K][npt]
    FastPtD *fastD = nullptr; // device [K][npt]
    int16_t *alpha = nullptr; // level policy (level 0: not owned)
    void *r = nullptr, *e = nullptr, *t = nullptr, *d = nullptr;  // precision of the V-cycle
    void *r64 = nullptr, *e64 = nullptr, *t64 = nullptr, *d64 = nullptr;  // FP64 copies (plain path)
    void *r32 = nullptr, *e32 = nullptr, *t32 = nullptr, *d32 = nullptr;
    double *sig_node = nullptr;  // per-node sigma model: [N][P][dim] on this level (injected from level 0)
    int reach[3] = {0, 0, 0};    // largest stencil corner offset in nodes along each axis (any control)
    double *lii = nullptr;       // device [K]: StencilDev::lii_deep of this level
    bool lii_ok = false;         // lii holds the current tables' values (constant coefficients, deep nodes exist)
    // wave-control table of the current policy (tiles x 4 wavefronts) and the per-control deep diagonal in
    // both precisions, written with the diagonal; valid (wctl_ok) after prepare_mg when lii_ok
    int16_t *wctl = nullptr;
    float *dk32 = nullptr;
    double *dk64 = nullptr;
    bool wctl_ok = false;
    // Galerkin coarse operator (levels >= 1 with HJB_COARSE_GALERKIN): sliced ELL, kGalWidth slots
    int32_t *gcol = nullptr;
    double *gval = nullptr;
    float *gval32 = nullptr;
    int gw = 0;  // widest row of the current operator (slots past it are unused)
};

constexpr int kGalWidth = 128;  // slots of a Galerkin coarse row

// device buffer that grows on demand (aggregation hierarchy: level sizes are known only once built)
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    template <typename T> T *as() const { return (T *)p; }
};

// one level of the aggregation hierarchy: its matrix (ELL, n rows, W widest row, slot stride n), its diagonal,
// the map from the finer level's nodes and the aggregates' members (4 per row, -1 unused), the cycle's vectors
struct AmgLevel {
    int64_t n = 0;
    int W = 0;
    bool wide = false;  // rows wider than kAmgWaveWidth: the cycle reads the row-major copy (rcol, rval)
    DevBuf col, val, d, agg, mem4, inv, rcol, rval;
    DevBuf x, r, t, v1, w1, v2, w2, r1;
};

}  // namespace

struct hjb_handle {
    hjb_desc desc{};
    int device = 0;        // the GPU current at setup (its copy of the allocation-free scratch)
    std::vector<double> sigma, drift, c;
    bool has_drift = false;
    int npt = 0, M = 0;
    double cmax = 0.0, cplus = 0.0;
    hipStream_t stream = nullptr;
    int dim = 2;
    int64_t N = 0;
    int nb = 0, nbd = 0;
    int nb_cap = 0;      // largest level-0 tile count over the tile shapes the handle may take
    // Galerkin coarse operators: the finest level's rows (npt * 4 + 1 slots) and a device overflow word
    int32_t *g0col = nullptr;
    double *g0val = nullptr;
    int32_t *goverflow = nullptr;
    // aggregation AMG (HJB_PRECOND_AMG), rebuilt for every policy: amg[0] is the finest matrix (merged rows)
    std::vector<AmgLevel> amg;
    DevBuf amg_rawc, amg_rawv, amg_mate, amg_cand, amg_flag, amg_id, amg_part, amg_aggA, amg_aggB, amg_mem2a, amg_mem2b,
        amg_icol, amg_ival, amg_words, amg_dpart, amg_sc, amg_trow, amg_tval, amg_scol, amg_sval;
    int amg_levels = 0;  // levels of the current hierarchy (0: none built)
    bool amg_fresh = true;     // the next hierarchy is built anew (a time step or a single solve starts)
    double amg_theta_dt = -1;  // theta*dt of the current hierarchy
    // certified reuse of search decisions within a step: gap bounds [N], X at the previous search [N],
    // per-tile largest change of X and its stencil-window maximum [nb_cap], window radius in nodes per axis
    double *marg = nullptr, *Xs = nullptr, *dtile = nullptr, *dwin = nullptr;
    uint8_t *keep = nullptr;  // [nb_cap * kBlock / 64] wavefronts whose decisions the next search keeps
    int64_t *kpartial = nullptr;  // [nb_cap] kept interior nodes per tile
    uint8_t *need = nullptr;      // [nb_cap] tiles the next search visits
    int32_t *tlist = nullptr;     // [nb_cap + 1] their list and (last entry) its length
    int64_t kept_last = 0;        // interior nodes whose decisions the last search kept
    int reach[3] = {0, 0, 0};
    int tlog = kTileLog2;
    std::vector<Level> lev;
    double s_tab = -1.0;
    double *c_dev = nullptr;
    // fine-level buffers
    double *E = nullptr, *R = nullptr, *Vb = nullptr, *Zb = nullptr;
    double *Ua = nullptr, *Ub = nullptr, *Uc = nullptr;
    int16_t *a0 = nullptr, *a1 = nullptr, *acarry = nullptr;
    double *Q = nullptr;        // [K][blocks][kBlock] explicit part of G for the searches of one step (or null)
    double *partial = nullptr;  // >= max(3*nb, (m+2)*nbd)
    double *dvals = nullptr;    // device scalars / small vectors [512]
    int64_t *ipartial = nullptr, *ival = nullptr;
    double *hpin = nullptr;     // pinned host mirror of small results [512]
    int64_t *hpin_i = nullptr;
    unsigned *hflag = nullptr;  // pinned host word the publish kernel releases sequence numbers into
    unsigned pub_seq = 0;
    std::vector<void *> allocs;
    bool trace = false;  // SLHJB_TRACE=1: policy-iteration progress on stderr
    // captured V-cycles, keyed by the buffers and scalars baked into their kernel arguments
    struct VGraph {
        const void *a0, *v, *z;
        double theta_dt;
        int nu1, nu2;
        bool rhs_ready;  // the graph starts from the single-precision right-hand side already in place
        const void *aa;  // policy of the operator application appended to the cycle (nullptr: none)
        const double *w; // its output
        hipGraphExec_t exec;
    };
    std::vector<VGraph> vgraphs;
    // sweep counts of the V-cycles of the current solve: nu1/nu2, or nu_tight for solves to the certificate
    int nu_pre = 3, nu_post = 3;
    hipStream_t capture_stream = nullptr;
    struct Timer {
        int cap = 0, used = 0;
        std::vector<hipEvent_t> ev;  // 2*cap events
        std::vector<double> bytes, flops;
        int64_t calls = 0;  // launches seen since enabled (sampling of the non-V-cycle classes)
    } timers[HJB_KERNEL_COUNT];
    int sample_period = 1;   // time one unit in sample_period (hjb_profile_sample)
    int64_t vc_count = 0;    // V-cycles since the V-cycle timers were enabled
    bool vc_timed = false;   // the V-cycle being launched is a sampled one
    bool apply_with_vcycle = false;  // the operator application being launched follows a V-cycle
};

namespace {

// time the one kernel launched in this scope (class `id`) when its timer is enabled: the launch stamps
// the slot's events with the dispatch's begin and end
struct TimedLaunch {
    hjb_handle *hd;
    int id;
    int slot = -1;
    TimedLaunch(hjb_handle *h, int i, double bytes, double flops = 0.0) : hd(h), id(i) {
        if (id < 0) return;
        auto &T = hd->timers[id];
        if (T.used >= T.cap) return;
        // the policy search is timed at every launch: its launches are few and long, and two kinds (the first
        // search of a step and the later ones) alternate, which a fixed sampling stride would alias
        const bool in_vcycle = id == HJB_KERNEL_SMOOTH || id == HJB_KERNEL_MG_RESID ||
                               (id == HJB_KERNEL_APPLY && hd->apply_with_vcycle);
        const bool take = id == HJB_KERNEL_SWEEP || (in_vcycle ? hd->vc_timed : (T.calls++ % hd->sample_period == 0));
        if (take) {
            slot = T.used++;
            T.bytes[slot] = bytes;
            T.flops[slot] = flops;
            g_launch_events = LaunchEvents{T.ev[2 * slot], T.ev[2 * slot + 1]};
        }
    }
    ~TimedLaunch() {
        if (slot >= 0 && g_launch_events.start) {  // the scope launched no kernel: drop the slot
            g_launch_events = LaunchEvents{};
            --hd->timers[id].used;
        }
    }
};

void fill_tables(hjb_handle *hd, double s, std::vector<PointTab> &host, int level) {
    const hjb_desc &d = hd->desc;
    const int dim = d.dim, K = d.K, P = d.P, npt = hd->npt;
    const double sr = s * (1.0 / sqrt(d.h));
    const double scale = ldexp(1.0, -level);
    const Level &L = hd->lev[level];
    host.assign((size_t)K * npt, PointTab{});
    for (int k = 0; k < K; ++k) {
        for (int q = 0; q < npt; ++q) {
            PointTab &p = host[(size_t)k * npt + q];
            for (int a = 0; a < 3; ++a) p.Y[a] = 0.0;
            const bool xs = d.coef_model == HJB_COEF_XSCALED;  // table holds S and beta (see point_Y)
            if (q < 2 * P) {
                int pp = q / 2;  // points 2p and 2p+1 are x + y_p and x - y_p
                for (int a = 0; a < dim; ++a) {
                    if (d.coef_model == HJB_COEF_FIELD) break;  // per node: see point_Y
                    double Y = xs ? d.sigma[((size_t)k * P + pp) * dim + a] : sr * d.sigma[((size_t)k * P + pp) * dim + a];
                    if (q & 1) Y = -Y;
                    p.Y[a] = xs ? Y : Y * scale;
                }
            } else {
                for (int a = 0; a < dim; ++a) p.Y[a] = xs ? hd->drift[(size_t)k * dim + a] : hd->drift[(size_t)k * dim + a] * scale;
            }
            int64_t off = 0;
            for (int a = 0; a < 3; ++a) {
                double fl = floor(p.Y[a]);
                p.t[a] = p.Y[a] - fl;
                p.u[a] = 1.0 - p.t[a];
                p.tf[a] = (float)p.t[a];
                p.uf[a] = (float)p.u[a];
                int64_t stride = a == 0 ? 1 : (a == 1 ? L.g.s1 : L.g.s2);
                if (a < dim) off += (int64_t)fl * stride;
            }
            p.off = off;
        }
    }
}

StencilDev stencil(const hjb_handle *hd, int level);
void drop_graphs(hjb_handle *hd);
int tiles_cap(const LevelDev &g0, int dim);

int build_tables(hjb_handle *hd, double s) {
    if (hd->s_tab == s) return HJB_OK;
    if (!(s > 0.0) || !isfinite(s)) return fail(HJB_EINVAL, "volatility scale s must be positive and finite");
    std::vector<PointTab> host;
    for (size_t l = 0; l < hd->lev.size(); ++l) {
        Level &L = hd->lev[l];
        fill_tables(hd, s, host, (int)l);
        // deep box: no point of any control can leave the box or be clamped from these nodes
        double E[3] = {0, 0, 0};
        if (hd->desc.coef_model == HJB_COEF_XSCALED) {
            // largest displacement anywhere on the grid: |sr * x * S| (diffusion), |x * beta| (drift)
            const double sr = s * (1.0 / sqrt(hd->desc.h)), scale = ldexp(1.0, -(int)l);
            for (int a = 0; a < hd->dim; ++a) {
                const double xm = std::max(fabs(hd->desc.lo[a]),
                                           fabs(hd->desc.lo[a] + (hd->desc.n[a] - 1) * hd->desc.h));
                for (int k = 0; k < hd->desc.K; ++k)
                    for (int q = 0; q < hd->npt; ++q) {
                        const double y = fabs(host[(size_t)k * hd->npt + q].Y[a]) * xm * (q < 2 * hd->desc.P ? sr : 1.0);
                        E[a] = std::max(E[a], y * scale);
                    }
                E[a] = E[a] * (1.0 + 1e-12) + 1e-12;  // the kernels round sr*(x*S) in another order
            }
        } else if (hd->desc.coef_model == HJB_COEF_FIELD) {
            // largest per-node diffusion displacement, and the drift points of the table
            const double sr = s * (1.0 / sqrt(hd->desc.h)), scale = ldexp(1.0, -(int)l);
            const int pd = hd->desc.P * hd->dim;
            for (size_t q = 0; q < hd->sigma.size(); ++q) {
                const int a = (int)(q % pd) % hd->dim;
                E[a] = std::max(E[a], sr * fabs(hd->sigma[q]) * scale);
            }
            for (int k = 0; k < hd->desc.K; ++k)
                for (int q = 2 * hd->desc.P; q < hd->npt; ++q)
                    for (int a = 0; a < hd->dim; ++a) E[a] = std::max(E[a], fabs(host[(size_t)k * hd->npt + q].Y[a]));
            for (int a = 0; a < hd->dim; ++a) E[a] = E[a] * (1.0 + 1e-12) + 1e-12;
        } else {
            for (const PointTab &p : host)
                for (int a = 0; a < 3; ++a) E[a] = std::max(E[a], fabs(p.Y[a]));
        }
        for (int a = 0; a < 3; ++a) L.reach[a] = a < hd->dim ? (int)ceil(E[a]) + 1 : 0;
        if (l == 0)
            for (int a = 0; a < 3; ++a) hd->reach[a] = L.reach[a];
        for (int a = 0; a < 3; ++a) {
            if (a < hd->dim) {
                int lo = (int)ceil(E[a]);
                int hi = L.g.n[a] - 2 - (int)floor(E[a]);
                L.g.deep_lo[a] = std::max(1, lo);
                L.g.deep_hi[a] = std::min(L.g.n[a] - 2, hi);
            } else {
                L.g.deep_lo[a] = 0;
                L.g.deep_hi[a] = 0;
            }
        }
        HIPCHK(hipMemcpyAsync(L.tab, host.data(), host.size() * sizeof(PointTab), hipMemcpyHostToDevice, hd->stream));
        // corner weights of the untruncated landing: product over axes (axis order) of t or 1 - t
        std::vector<FastPtF> hf(host.size());
        std::vector<FastPtD> hdd(host.size());
        for (size_t q = 0; q < host.size(); ++q) {
            memset(&hf[q], 0, sizeof(FastPtF));
            memset(&hdd[q], 0, sizeof(FastPtD));
            hf[q].off = hdd[q].off = (int32_t)host[q].off;
            const double *t = host[q].t;
            for (int c = 0; c < (1 << hd->dim); ++c) {
                double w = (c & 1) ? t[0] : (1.0 - t[0]);
                w = w * (((c >> 1) & 1) ? t[1] : (1.0 - t[1]));
                if (hd->dim == 3) w = w * (((c >> 2) & 1) ? t[2] : (1.0 - t[2]));
                hdd[q].w[c] = w;
                hf[q].w[c] = (float)w;
            }
        }
        HIPCHK(hipMemcpyAsync(L.fastF, hf.data(), hf.size() * sizeof(FastPtF), hipMemcpyHostToDevice, hd->stream));
        HIPCHK(hipMemcpyAsync(L.fastD, hdd.data(), hdd.size() * sizeof(FastPtD), hipMemcpyHostToDevice, hd->stream));
        // per-control diagonal sums at deep nodes (constant coefficients), from the tables just uploaded
        L.lii_ok = false;
        bool has_deep = hd->desc.coef_model == HJB_COEF_CONST;
        for (int a = 0; a < hd->dim; ++a) has_deep = has_deep && L.g.deep_lo[a] <= L.g.deep_hi[a];
        if (has_deep) {
            StencilDev st = stencil(hd, (int)l);  // lii_deep is not read by the table kernel
            launch_lii_deep(hd->dim, L.g, st, L.g.deep_lo, L.lii, hd->stream);
            HIPCHK(hipGetLastError());
            L.lii_ok = true;
        }
        HIPCHK(hipStreamSynchronize(hd->stream));  // host vectors go out of scope
    }
    HIPCHK(hipStreamSynchronize(hd->stream));
    hd->s_tab = s;
    // captured graphs hold level descriptors and stencil scalars by value (the deep box, s / sqrt(h))
    drop_graphs(hd);
    return HJB_OK;
}

StencilDev stencil(const hjb_handle *hd, int level) {
    StencilDev st;
    st.tab = hd->lev[level].tab;
    st.fastF = hd->lev[level].fastF;
    st.fastD = hd->lev[level].fastD;
    st.c = hd->c.empty() ? nullptr : hd->c_dev;
    st.K = hd->desc.K;
    st.P = hd->desc.P;
    st.npt = hd->npt;
    st.has_drift = hd->has_drift ? 1 : 0;
    st.inv2h = 0.5 / hd->desc.h;
    st.xs = hd->desc.coef_model == HJB_COEF_XSCALED ? 1 : 0;
    st.field = hd->desc.coef_model == HJB_COEF_FIELD ? 1 : 0;
    st.pernode = st.xs || st.field;
    st.sig_node = hd->lev[level].sig_node;
    st.fk = (level == 0 && hd->desc.f_per_control) ? hd->N : 0;
    st.sr = hd->s_tab * (1.0 / sqrt(hd->desc.h));
    st.scale = ldexp(1.0, -level);
    for (int a = 0; a < 3; ++a) st.lo[a] = hd->desc.lo[a];
    st.hl = ldexp(hd->desc.h, level);
    st.lii_deep = (!st.pernode && hd->lev[level].lii_ok) ? hd->lev[level].lii : nullptr;
    return st;
}

int dalloc(hjb_handle *hd, void **p, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(HJB_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    }
    hd->allocs.push_back(*p);
    return HJB_OK;
}

#define TRY(x)                 \
    do {                       \
        int _rc = (x);         \
        if (_rc != HJB_OK) return _rc; \
    } while (0)

bool mixed(const hjb_handle *hd) { return hd->desc.precision == HJB_PREC_MIXED; }

void select_precision(hjb_handle *hd) {
    bool f = mixed(hd);
    for (Level &L : hd->lev) {
        L.r = f ? L.r32 : L.r64;
        L.e = f ? L.e32 : L.e64;
        L.t = f ? L.t32 : L.t64;
        L.d = f ? L.d32 : L.d64;
    }
}

int check_options(const hjb_desc *d) {
    if (d->precision != HJB_PREC_FP64 && d->precision != HJB_PREC_MIXED) return fail(HJB_EINVAL, "precision");
    if (d->precond < HJB_PRECOND_NONE || d->precond > HJB_PRECOND_AMG) return fail(HJB_EINVAL, "precond");
    if (d->kcycle_levels < -1) return fail(HJB_EINVAL, "kcycle_levels must be >= -1");
    if (d->value_stride < 1) return fail(HJB_EINVAL, "value_stride must be >= 1");
    if (d->amg_reuse != 0 && d->amg_reuse != 1) return fail(HJB_EINVAL, "amg_reuse must be 0 or 1");
    if (d->restart < 1 || d->restart > kMaxRestart) return fail(HJB_EINVAL, "restart must be in 1..%d", kMaxRestart);
    if (d->max_krylov < 1) return fail(HJB_EINVAL, "max_krylov must be >= 1");
    if (d->max_pi < 1) return fail(HJB_EINVAL, "max_pi must be >= 1");
    if (d->nu1 < 1 || d->nu2 < 0 || d->nu1 > 16 || d->nu2 > 16) return fail(HJB_EINVAL, "nu1 in 1..16, nu2 in 0..16");
    if (d->coarse_sweeps < 1 || d->coarse_sweeps > 1000) return fail(HJB_EINVAL, "coarse_sweeps in 1..1000");
    if (!(d->omega > 0.0 && d->omega < 2.0)) return fail(HJB_EINVAL, "omega must be in (0,2)");
    if (!(d->rtol_inf > 0.0) || !(d->tau_rel >= 0.0)) return fail(HJB_EINVAL, "rtol_inf > 0 and tau_rel >= 0 required");
    if (!(d->pi_eta >= 0.0 && d->pi_eta < 1.0)) return fail(HJB_EINVAL, "pi_eta must be in [0,1)");
    if (d->max_levels < 0) return fail(HJB_EINVAL, "max_levels must be >= 0");
    if (d->nu_tight < 0 || d->nu_tight > 16) return fail(HJB_EINVAL, "nu_tight in 0..16");
    if (d->coarse_sweeps_t < 0 || d->coarse_sweeps_t > 1000) return fail(HJB_EINVAL, "coarse_sweeps_t in 0..1000");
    if (d->krylov != HJB_KRYLOV_FGMRES && d->krylov != HJB_KRYLOV_BICGSTAB) return fail(HJB_EINVAL, "krylov");
    if (d->coarse_op != HJB_COARSE_REDISCRETIZED && d->coarse_op != HJB_COARSE_GALERKIN)
        return fail(HJB_EINVAL, "coarse_op");
    if (d->coarse_op == HJB_COARSE_GALERKIN && d->dim != 2)
        return fail(HJB_EUNSUPPORTED, "Galerkin coarse operators are provided for 2D grids");
    if (d->krylov == HJB_KRYLOV_BICGSTAB && d->restart < 3)
        return fail(HJB_EINVAL, "BiCGSTAB keeps four vectors in the Krylov basis storage: restart must be >= 3");
    return HJB_OK;
}

// ---- multigrid ---------------------------------------------------------------------------------

constexpr int64_t kCoarseMaxNodes = 2048;  // LDS-resident coarsest level (two FP64 buffers = 32 KiB)

// Galerkin coarse operators for the policy: the finest level's rows, then A_{l+1} = R A_l P level by level,
// each level's diagonal (for the smoother) and FP32 weights; the widest row is checked against the ELL width.
int publish_wait(hjb_handle *hd, const void *dev0, void *host0, size_t bytes0, const void *dev1, void *host1,
                 size_t bytes1);

int build_galerkin(hjb_handle *hd, const int16_t *alpha, double theta_dt) {
    hipStream_t s = hd->stream;
    const int E0 = hd->npt * 4 + 1;
    int32_t *wide = (int32_t *)(hd->hpin + kGalSlot);  // pinned host word
    launch_gal_emit(2, hd->lev[0].g, stencil(hd, 0), alpha, theta_dt, E0, hd->g0col, hd->g0val, s);
    int Wf = E0;
    for (size_t l = 1; l < hd->lev.size(); ++l) {
        Level &F = hd->lev[l - 1], &C = hd->lev[l];
        const int32_t *fc = l == 1 ? hd->g0col : F.gcol;
        const double *fv = l == 1 ? hd->g0val : F.gval;
        launch_zero(hd->goverflow, 4, s);
        if (launch_gal_rap(F.g, C.g, Wf, fc, fv, kGalWidth, C.gcol, C.gval, hd->goverflow, s) != 0)
            return fail(HJB_EUNSUPPORTED, "Galerkin product: rows of level %d have %d entries", (int)l - 1, Wf);
        launch_gal_diag(C.g.N, kGalWidth, C.gcol, C.gval, C.gval32, mixed(hd) ? (float *)C.d : nullptr,
                        mixed(hd) ? nullptr : (double *)C.d, s);
        TRY(publish_wait(hd, hd->goverflow, wide, 8, nullptr, nullptr, 0));
        if (wide[0] > kGalWidth)
            return fail(HJB_EUNSUPPORTED, "Galerkin coarse row with %d entries (the ELL width is %d)", wide[0],
                        kGalWidth);
        Wf = std::max(1, wide[0]);
        C.gw = Wf;
    }
    return HJB_OK;
}

int prepare_amg(hjb_handle *hd, const int16_t *alpha, double theta_dt);

int prepare_mg(hjb_handle *hd, const int16_t *alpha, double theta_dt) {
    if (hd->desc.precond == HJB_PRECOND_AMG) return prepare_amg(hd, alpha, theta_dt);
    hipStream_t s = hd->stream;
    hd->lev[0].alpha = const_cast<int16_t *>(alpha);
    for (size_t l = 1; l < hd->lev.size(); ++l)
        launch_inject_policy(hd->dim, hd->lev[l - 1].g, hd->lev[l].g, hd->lev[l - 1].alpha, hd->lev[l].alpha, s);
    for (size_t l = 0; l < hd->lev.size(); ++l) {
        Level &L = hd->lev[l];
        const StencilDev st = stencil(hd, (int)l);
        L.wctl_ok = L.wctl && st.lii_deep;
        if (mixed(hd))
            launch_diag<float>(hd->dim, L.g, st, L.alpha, theta_dt, (float *)L.d, s, L.wctl_ok ? L.wctl : nullptr,
                               L.dk32);
        else
            launch_diag<double>(hd->dim, L.g, st, L.alpha, theta_dt, (double *)L.d, s, L.wctl_ok ? L.wctl : nullptr,
                                L.dk64);
    }
    if (hd->desc.coarse_op == HJB_COARSE_GALERKIN && hd->lev.size() > 1) TRY(build_galerkin(hd, alpha, theta_dt));
    HIPCHK(hipGetLastError());
    return HJB_OK;
}

template <typename T>
void smooth_level(hjb_handle *hd, int l, T *&e, T *&t, const T *r, int sweeps, bool first, double theta_dt) {
    Level &L = hd->lev[l];
    StencilDev st = stencil(hd, l);
    if (l >= 1 && L.gcol) {
        const T *gv;
        if constexpr (std::is_same<T, float>::value) gv = L.gval32; else gv = L.gval;
        for (int q = 0; q < sweeps; ++q) {
            launch_gal_jacobi<T>(L.g.N, L.gw, L.gcol, gv, (const T *)L.d, e, r, t, hd->desc.omega,
                                 first && q == 0, hd->stream);
            std::swap(e, t);
        }
        return;
    }
    for (int q = 0; q < sweeps; ++q) {
        bool gathers = !(first && q == 0);
        // algorithmic bytes: e, r, alpha in, e out (the diagonal is a derived quantity, not counted)
        TimedLaunch tl(hd, (l == 0 && gathers) ? HJB_KERNEL_SMOOTH : -1, (double)L.g.N * (3.0 * sizeof(T) + 2.0));
        const T *dk = nullptr;
        if constexpr (std::is_same<T, float>::value) dk = L.dk32; else dk = L.dk64;
        launch_jacobi<T>(hd->dim, L.g, st, L.alpha, e, r, (const T *)L.d, t, theta_dt, hd->desc.omega,
                         first && q == 0, hd->stream, L.wctl_ok ? L.wctl : nullptr, dk);
        std::swap(e, t);
    }
}

// z = V-cycle(v): approximate solve of A z = v; r0 is the level-0 right-hand side (precision T),
// z the level-0 output buffer (precision T).
template <typename T>
void vcycle(hjb_handle *hd, const T *r0, T *z, double theta_dt) {
    const int Lc = (int)hd->lev.size() - 1;
    const hjb_desc &d = hd->desc;
    hipStream_t s = hd->stream;
    std::vector<T *> e(Lc + 1), t(Lc + 1);
    std::vector<const T *> r(Lc + 1);
    for (int l = 0; l <= Lc; ++l) {
        e[l] = (T *)hd->lev[l].e;
        t[l] = (T *)hd->lev[l].t;
        r[l] = (const T *)hd->lev[l].r;
    }
    r[0] = r0;
    // every smoothing sweep writes the other buffer of the pair; start so that level 0 ends in z
    int flips0 = hd->nu_pre + hd->nu_post;
    if (Lc == 0) flips0 = d.coarse_sweeps;
    if (flips0 % 2 == 0) {
        e[0] = z;
    } else {
        e[0] = (T *)hd->lev[0].t;
        t[0] = z;
    }
    if (Lc == 0) {
        smooth_level<T>(hd, 0, e[0], t[0], r[0], d.coarse_sweeps, true, theta_dt);
        return;
    }
    for (int l = 0; l < Lc; ++l) {
        Level &L = hd->lev[l];
        smooth_level<T>(hd, l, e[l], t[l], r[l], hd->nu_pre, true, theta_dt);
        {
            TimedLaunch tl(hd, l == 0 ? HJB_KERNEL_MG_RESID : -1, (double)L.g.N * (3.0 * sizeof(T) + 2.0));
            if (l >= 1 && L.gcol) {
                const T *gv;
                if constexpr (std::is_same<T, float>::value) gv = L.gval32; else gv = L.gval;
                launch_gal_residual<T>(L.g.N, L.gw, L.gcol, gv, e[l], r[l], t[l], s);
            } else {
                launch_level_residual<T>(hd->dim, L.g, stencil(hd, l), L.alpha, e[l], r[l], t[l], theta_dt, s,
                                         L.wctl_ok ? L.wctl : nullptr);
            }
        }
        launch_restrict<T>(hd->dim, L.g, hd->lev[l + 1].g, t[l], (T *)hd->lev[l + 1].r, s);
    }
    {
        Level &C = hd->lev[Lc];
        if (C.g.N <= kCoarseMaxNodes && !C.gcol) {
            launch_coarse_solve<T>(hd->dim, C.g, stencil(hd, Lc), C.alpha, r[Lc], (const T *)C.d, e[Lc], t[Lc],
                                   theta_dt, d.omega, d.coarse_sweeps, s);
        } else {
            smooth_level<T>(hd, Lc, e[Lc], t[Lc], r[Lc], d.coarse_sweeps, true, theta_dt);
        }
    }
    for (int l = Lc - 1; l >= 0; --l) {
        Level &L = hd->lev[l];
        launch_prolong_add<T>(hd->dim, L.g, hd->lev[l + 1].g, e[l + 1], e[l], s);
        smooth_level<T>(hd, l, e[l], t[l], r[l], hd->nu_post, false, theta_dt);
    }
}

// ---- aggregation AMG -------------------------------------------------------------------------------
//
// The hierarchy is rebuilt for every policy: the finest rows of A = I - theta dt (L-hat + c) emitted from the
// stencil and merged, then level by level two pairing passes (double pairwise aggregation: aggregates of up to
// four nodes) and the Galerkin product with the piecewise-constant prolongation, until a level has at most
// kAmgDenseMax rows, whose dense inverse is formed (or until the coarsening stalls, below 5/4 per level, or the
// rows grow wider than kAmgMaxWidth: then the last level is solved by Jacobi sweeps).  The cycle smooths with damped Jacobi (matrix-free on the
// finest level), restricts by aggregate sums and solves each coarse residual equation by GCR iterations
// preconditioned by the cycle one level down (two on the first kcycle_levels coarse levels, one below), with
// the GCR coefficients kept on the device.

constexpr double kAmgBeta = 0.25;      // strong coupling: -a_ij >= kAmgBeta * (the row's largest -a_ik)
constexpr double kAmgDominance = 5.0;  // rows with a_ii >= kAmgDominance * sum_{j != i} |a_ij| join no aggregate
constexpr int kAmgRounds = 6;          // handshake rounds per pairing pass
constexpr int kAmgMaxWidth = 256;      // coarsening stops at a level with rows wider than this (the products
                                       // sort two rows of a pair, at most 1024 entries, in LDS)
constexpr int kAmgMaxLevels = 24;
constexpr int kAmgSlot = 232;          // pinned host words of the hierarchy build
constexpr int kAmgScSlots = 8;         // device GCR scalars per level

int grow(hjb_handle *hd, DevBuf &b, size_t bytes) {
    if (bytes <= b.cap) return HJB_OK;
    if (b.p) {
        HIPCHK(hipStreamSynchronize(hd->stream));
        HIPCHK(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    const size_t want = std::max<size_t>(256, bytes + bytes / 8);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(HJB_ENOMEM, "aggregation hierarchy: %zu bytes: %s", want, hipGetErrorString(e));
    }
    b.cap = want;
    return HJB_OK;
}

void release(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// One pairing pass over the n rows of (col, val): the symmetric part S of the couplings is formed, then
// kAmgRounds handshake rounds pair each unmatched node with its strongest unmatched neighbour on S when the
// choice is mutual; agg (n entries) maps each row to its pair or singleton (-1: none, the row being empty or
// dominant by dd), mem2 (2 per aggregate) lists the members.  *nc receives the number of aggregates and, when
// wide is given, *wide the widest row of the last product (device word 0, read with the same synchronisation).
int amg_pair(hjb_handle *hd, int64_t n, int W, const int32_t *col, const double *val, double dd, int32_t *agg,
             int32_t *mem2, int64_t *nc, int *wide) {
    hipStream_t s = hd->stream;
    int32_t *mate = hd->amg_mate.as<int32_t>(), *cand = hd->amg_cand.as<int32_t>();
    int32_t *flag = hd->amg_flag.as<int32_t>(), *id = hd->amg_id.as<int32_t>(), *part = hd->amg_part.as<int32_t>();
    // device words: [0] the widest row of the last product, [1] the longest column, [2] the number of aggregates
    // (read 16 bytes at a time)
    int32_t *words = hd->amg_words.as<int32_t>();
    int32_t *h = (int32_t *)(hd->hpin + kAmgSlot);
    // S = -(M + M^T)/2 off the diagonal: column counts (in flag), segment offsets (in id), fill counters (in cand)
    TRY(grow(hd, hd->amg_trow, (size_t)n * W * 4));
    TRY(grow(hd, hd->amg_tval, (size_t)n * W * 8));
    launch_zero(flag, (size_t)n * 4, s);
    launch_zero(cand, (size_t)n * 4, s);
    launch_zero(words + 1, 4, s);
    launch_amg_colcount(n, W, col, flag, words + 1, s);
    exclusive_scan(flag, n, id, part, words + 3, s);
    launch_amg_scatter(n, W, col, val, id, cand, hd->amg_trow.as<int32_t>(), hd->amg_tval.as<double>(), s);
    TRY(publish_wait(hd, words, h, 16, nullptr, nullptr, 0));
    if (wide) *wide = h[0];
    const int Ws = std::max(1, W + h[1]);
    TRY(grow(hd, hd->amg_scol, (size_t)n * Ws * 4));
    TRY(grow(hd, hd->amg_sval, (size_t)n * Ws * 8));
    int32_t *scol = hd->amg_scol.as<int32_t>();
    double *sval = hd->amg_sval.as<double>();
    if (launch_amg_sym(n, W, h[1], col, val, id, flag, hd->amg_trow.as<int32_t>(), hd->amg_tval.as<double>(), Ws, scol,
                       sval, s) != 0)
        return fail(HJB_EUNSUPPORTED, "aggregation: rows of %d entries", W);
    // matching
    launch_amg_init(n, W, col, val, dd, mate, s);
    for (int q = 0; q < kAmgRounds; ++q) launch_amg_match_round(n, Ws, scol, sval, kAmgBeta, mate, cand, s);
    launch_amg_leader(n, mate, flag, s);
    exclusive_scan(flag, n, id, part, words + 2, s);
    launch_amg_assign(n, mate, id, agg, mem2, s);
    TRY(publish_wait(hd, words, h, 16, nullptr, nullptr, 0));
    *nc = h[2];
    return HJB_OK;
}

int amg_vectors(hjb_handle *hd, AmgLevel &L) {
    const size_t b = (size_t)std::max<int64_t>(1, L.n) * 8;
    for (DevBuf *v : {&L.x, &L.r, &L.t, &L.v1, &L.w1, &L.v2, &L.w2, &L.r1}) TRY(grow(hd, *v, b));
    return HJB_OK;
}

int build_amg(hjb_handle *hd, const int16_t *alpha, double theta_dt) {
    hipStream_t s = hd->stream;
    const int64_t N = hd->N;
    const int E0 = (hd->npt << hd->dim) + 1;
    hd->amg_levels = 0;
    TRY(grow(hd, hd->amg_rawc, (size_t)N * E0 * 4));
    TRY(grow(hd, hd->amg_rawv, (size_t)N * E0 * 8));
    for (DevBuf *b : {&hd->amg_mate, &hd->amg_cand, &hd->amg_flag, &hd->amg_id, &hd->amg_aggA, &hd->amg_aggB})
        TRY(grow(hd, *b, (size_t)N * 4));
    TRY(grow(hd, hd->amg_mem2a, (size_t)N * 8));
    TRY(grow(hd, hd->amg_mem2b, (size_t)N * 8));
    TRY(grow(hd, hd->amg_part, (size_t)(scan_parts(N) + 2) * 4));
    TRY(grow(hd, hd->amg_words, 16));
    TRY(grow(hd, hd->amg_dpart, (size_t)2 * 1024 * 8));
    TRY(grow(hd, hd->amg_sc, (size_t)kAmgMaxLevels * kAmgScSlots * 8));
    if (hd->amg.empty()) hd->amg.resize(1);
    {
        AmgLevel &F0 = hd->amg[0];
        F0.n = N;
        F0.W = E0;
        TRY(grow(hd, F0.col, (size_t)N * E0 * 4));
        TRY(grow(hd, F0.val, (size_t)N * E0 * 8));
        launch_gal_emit(hd->dim, hd->lev[0].g, stencil(hd, 0), alpha, theta_dt, E0, hd->amg_rawc.as<int32_t>(),
                        hd->amg_rawv.as<double>(), s);
        launch_amg_merge(N, hd->lev[0].g.n[0], hd->lev[0].g.n[1], hd->lev[0].g.n[2], E0, hd->amg_rawc.as<int32_t>(),
                         hd->amg_rawv.as<double>(), F0.col.as<int32_t>(), F0.val.as<double>(), s);
    }
    int32_t *widest = hd->amg_words.as<int32_t>();
    int32_t *aggA = hd->amg_aggA.as<int32_t>(), *aggB = hd->amg_aggB.as<int32_t>();
    int32_t *mem2a = hd->amg_mem2a.as<int32_t>(), *mem2b = hd->amg_mem2b.as<int32_t>();
    int levels = 1;
    bool w_pending = false;  // the last level's W is an upper bound; its widest row is in *widest
    for (;;) {
        if ((int)hd->amg.size() < levels + 1) hd->amg.resize(levels + 1);
        AmgLevel &F = hd->amg[levels - 1], &C = hd->amg[levels];
        if (F.n <= kAmgDenseMax || levels >= kAmgMaxLevels) break;
        // first pass on the level's matrix (which also reads the level's widest row)
        int64_t nA = 0;
        int wf = 0;
        TRY(amg_pair(hd, F.n, F.W, F.col.as<int32_t>(), F.val.as<double>(), kAmgDominance, aggA, mem2a, &nA, &wf));
        if (w_pending) F.W = std::max(1, wf);
        w_pending = false;
        if (nA == 0) break;  // every row is dominant: the smoother resolves the level
        if (F.W > kAmgMaxWidth) break;  // rows this wide: the level is the coarsest
        const int wi_cap = 2 * F.W;
        TRY(grow(hd, hd->amg_icol, (size_t)nA * wi_cap * 4));
        TRY(grow(hd, hd->amg_ival, (size_t)nA * wi_cap * 8));
        int32_t *icol = hd->amg_icol.as<int32_t>();
        double *ival = hd->amg_ival.as<double>();
        launch_zero(widest, 4, s);
        launch_amg_product(F.n, F.W, F.col.as<int32_t>(), F.val.as<double>(), aggA, mem2a, 2, nA, wi_cap, icol, ival,
                           widest, s);
        // second pass on the pairs' matrix
        int64_t nB = 0;
        int wi = 0;
        TRY(amg_pair(hd, nA, wi_cap, icol, ival, 0.0, aggB, mem2b, &nB, &wi));
        wi = std::max(1, wi);
        if (wi > kAmgMaxWidth) break;  // the pairs' rows are already this wide: the level is the coarsest
        C.n = nB;
        const int wc_cap = 2 * wi;
        TRY(grow(hd, C.agg, (size_t)F.n * 4));
        TRY(grow(hd, C.mem4, (size_t)nB * 16));
        TRY(grow(hd, C.col, (size_t)nB * wc_cap * 4));
        TRY(grow(hd, C.val, (size_t)nB * wc_cap * 8));
        TRY(grow(hd, C.d, (size_t)nB * 8));
        TRY(amg_vectors(hd, C));
        launch_amg_compose(F.n, aggA, aggB, C.agg.as<int32_t>(), s);
        launch_amg_members4(nB, mem2b, mem2a, C.mem4.as<int32_t>(), s);
        launch_zero(widest, 4, s);
        launch_amg_product(nA, wi, icol, ival, aggB, mem2b, 2, nB, wc_cap, C.col.as<int32_t>(), C.val.as<double>(),
                           widest, s);
        C.W = wc_cap;
        w_pending = true;
        launch_amg_diag(nB, C.W, C.col.as<int32_t>(), C.val.as<double>(), C.d.as<double>(), s);
        const bool stalled = 5 * nB > 4 * F.n;
        ++levels;
        if (stalled) break;
    }
    AmgLevel &Lc = hd->amg[levels - 1];
    if (w_pending) {
        int32_t *h = (int32_t *)(hd->hpin + kAmgSlot);
        TRY(publish_wait(hd, widest, h, 8, nullptr, nullptr, 0));
        Lc.W = std::max(1, h[0]);
    }
    if (levels > 1 && Lc.n <= kAmgDenseMax) {
        TRY(grow(hd, Lc.inv, (size_t)Lc.n * Lc.n * 8));
        launch_amg_dense_inverse((int)Lc.n, Lc.W, Lc.col.as<int32_t>(), Lc.val.as<double>(), Lc.inv.as<double>(), s);
    }
    for (int l = 1; l < levels; ++l) {
        AmgLevel &A = hd->amg[l];
        // a wavefront per row pays where rows are wide and few; with many rows one thread per row already fills
        // the GPU and reads the slot-major layout coalesced
        A.wide = A.W > kAmgWaveWidth && A.n <= kAmgWaveRows;
        if (!A.wide) continue;
        TRY(grow(hd, A.rcol, (size_t)A.n * A.W * 4));
        TRY(grow(hd, A.rval, (size_t)A.n * A.W * 8));
        launch_amg_rowmajor(A.n, A.W, A.col.as<int32_t>(), A.val.as<double>(), A.rcol.as<int32_t>(),
                            A.rval.as<double>(), s);
    }
    hd->amg_levels = levels;
    return HJB_OK;
}

int prepare_amg(hjb_handle *hd, const int16_t *alpha, double theta_dt) {
    Level &L = hd->lev[0];
    L.alpha = const_cast<int16_t *>(alpha);
    const StencilDev st = stencil(hd, 0);
    L.wctl_ok = L.wctl && st.lii_deep;
    launch_diag<double>(hd->dim, L.g, st, alpha, theta_dt, (double *)L.d64, hd->stream,
                        L.wctl_ok ? L.wctl : nullptr, L.dk64);
    // with amg_reuse, later policies of a time step keep the step's coarse levels (the finest level, smoothed
    // and reduced matrix-free with the current policy, is always current)
    const bool keep = hd->desc.amg_reuse && !hd->amg_fresh && hd->amg_levels > 0 && hd->amg_theta_dt == theta_dt;
    if (!keep) TRY(build_amg(hd, alpha, theta_dt));
    hd->amg_fresh = false;
    hd->amg_theta_dt = theta_dt;
    HIPCHK(hipGetLastError());
    return HJB_OK;
}

// damped Jacobi sweeps on level l (the finest level matrix-free), alternating between e and t
void amg_smooth(hjb_handle *hd, int l, double *&e, double *&t, const double *r, int sweeps, bool first,
                double theta_dt) {
    hipStream_t s = hd->stream;
    if (l == 0) {
        Level &L = hd->lev[0];
        for (int q = 0; q < sweeps; ++q) {
            TimedLaunch tl(hd, (q > 0 || !first) ? HJB_KERNEL_SMOOTH : -1, (double)L.g.N * (3.0 * 8 + 2.0));
            launch_jacobi<double>(hd->dim, L.g, stencil(hd, 0), L.alpha, e, r, (const double *)L.d64, t, theta_dt,
                                  hd->desc.omega, first && q == 0, s, L.wctl_ok ? L.wctl : nullptr, L.dk64);
            std::swap(e, t);
        }
        return;
    }
    AmgLevel &A = hd->amg[l];
    for (int q = 0; q < sweeps; ++q) {
        if (A.wide)
            launch_amg_wave_op(A.n, A.W, A.rcol.as<int32_t>(), A.rval.as<double>(), A.d.as<double>(), e, r, t, 2,
                               hd->desc.omega, first && q == 0, s);
        else
            launch_gal_jacobi<double>(A.n, A.W, A.col.as<int32_t>(), A.val.as<double>(), A.d.as<double>(), e, r, t,
                                      hd->desc.omega, first && q == 0, s);
        std::swap(e, t);
    }
}

void amg_solve(hjb_handle *hd, int l, const double *r, double *x, double theta_dt);

// out = one cycle on level l for the right-hand side r from a zero initial guess: pre-smoothing, the
// residual restricted by aggregate sums, the coarse residual equation solved by amg_solve, its solution
// added to the aggregates' nodes, post-smoothing
void amg_cycle(hjb_handle *hd, int l, const double *r, double *out, double theta_dt) {
    hipStream_t s = hd->stream;
    double *tmp = l == 0 ? (double *)hd->lev[0].t64 : hd->amg[l].t.as<double>();
    double *e = out, *t = tmp;
    if ((hd->nu_pre + hd->nu_post) % 2) std::swap(e, t);
    amg_smooth(hd, l, e, t, r, hd->nu_pre, true, theta_dt);
    if (l == 0) {
        Level &L = hd->lev[0];
        TimedLaunch tl(hd, HJB_KERNEL_MG_RESID, (double)L.g.N * (3.0 * 8 + 2.0));
        launch_level_residual<double>(hd->dim, L.g, stencil(hd, 0), L.alpha, e, r, t, theta_dt, s,
                                      L.wctl_ok ? L.wctl : nullptr);
    } else {
        AmgLevel &A = hd->amg[l];
        if (A.wide)
            launch_amg_wave_op(A.n, A.W, A.rcol.as<int32_t>(), A.rval.as<double>(), nullptr, e, r, t, 1, 0.0, false,
                               s);
        else
            launch_gal_residual<double>(A.n, A.W, A.col.as<int32_t>(), A.val.as<double>(), e, r, t, s);
    }
    AmgLevel &C = hd->amg[l + 1];
    launch_amg_restrict(C.n, C.mem4.as<int32_t>(), t, C.r.as<double>(), s);
    amg_solve(hd, l + 1, C.r.as<double>(), C.x.as<double>(), theta_dt);
    launch_amg_prolong(hd->amg[l].n, C.agg.as<int32_t>(), C.x.as<double>(), e, s);
    amg_smooth(hd, l, e, t, r, hd->nu_post, false, theta_dt);
}

// x ~ A_l^{-1} r on level l >= 1: the coarsest level through its dense inverse (or Jacobi sweeps when the
// coarsening stopped early), other levels by GCR iterations preconditioned by amg_cycle(l): x = a1 v1 with
// v1 = cycle(r), a1 minimising |r - a1 A v1|; then (two-iteration levels) v2 = cycle(r - a1 A v1)
// orthogonalised against A v1 and x += a2 v2 minimising the residual again
void amg_solve(hjb_handle *hd, int l, const double *r, double *x, double theta_dt) {
    hipStream_t s = hd->stream;
    AmgLevel &A = hd->amg[l];
    const int32_t *col = A.col.as<int32_t>();
    const double *val = A.val.as<double>();
    if (l == hd->amg_levels - 1) {
        if (A.n <= kAmgDenseMax) {
            launch_amg_dense_solve((int)A.n, A.inv.as<double>(), r, x, s);
        } else if (A.wide) {
            double *e = x, *t = A.t.as<double>();
            if (hd->desc.coarse_sweeps % 2) std::swap(e, t);
            for (int q = 0; q < hd->desc.coarse_sweeps; ++q) {
                launch_amg_wave_op(A.n, A.W, A.rcol.as<int32_t>(), A.rval.as<double>(), A.d.as<double>(), e, r, t, 2,
                                   1.0, q == 0, s);
                std::swap(e, t);
            }
        } else if (A.n <= kAmgCoarseMax) {
            launch_amg_coarse((int)A.n, A.W, col, val, A.d.as<double>(), r, hd->desc.coarse_sweeps, x, s);
        } else {
            double *e = x, *t = A.t.as<double>();
            if (hd->desc.coarse_sweeps % 2) std::swap(e, t);
            for (int q = 0; q < hd->desc.coarse_sweeps; ++q) {
                launch_gal_jacobi<double>(A.n, A.W, col, val, A.d.as<double>(), e, r, t, 1.0, q == 0, s);
                std::swap(e, t);
            }
        }
        return;
    }
    double *sc = hd->amg_sc.as<double>() + (size_t)l * kAmgScSlots;
    double *part = hd->amg_dpart.as<double>();
    double *v1 = A.v1.as<double>(), *w1 = A.w1.as<double>(), *v2 = A.v2.as<double>(), *w2 = A.w2.as<double>();
    double *r1 = A.r1.as<double>();
    auto spmv = [&](const double *x, double *y) {
        if (A.wide)
            launch_amg_wave_op(A.n, A.W, A.rcol.as<int32_t>(), A.rval.as<double>(), nullptr, x, nullptr, y, 0, 0.0,
                               false, s);
        else
            launch_amg_spmv(A.n, A.W, col, val, x, y, s);
    };
    amg_cycle(hd, l, r, v1, theta_dt);
    spmv(v1, w1);
    launch_amg_dot2(A.n, w1, r, w1, part, sc, s);
    launch_amg_gcr(A.n, 0, sc, x, v1, w1, nullptr, nullptr, r, r1, s);
    if (hd->desc.kcycle_levels >= 0 && l > hd->desc.kcycle_levels) return;
    amg_cycle(hd, l, r1, v2, theta_dt);
    spmv(v2, w2);
    launch_amg_dot2(A.n, w1, w2, w1, part, sc + 2, s);
    launch_amg_gcr(A.n, 1, sc + 2, nullptr, v2, w2, v1, w1, nullptr, nullptr, s);
    launch_amg_dot2(A.n, w2, r1, w2, part, sc + 4, s);
    launch_amg_gcr(A.n, 2, sc + 4, x, v2, nullptr, nullptr, nullptr, nullptr, nullptr, s);
}

// z = M^{-1} v for the aggregation preconditioner (FP64)
void amg_precondition(hjb_handle *hd, const double *v, double *z, double theta_dt) {
    if (hd->amg_levels > 1) {
        amg_cycle(hd, 0, v, z, theta_dt);
        return;
    }
    double *e = z, *t = (double *)hd->lev[0].t64;
    const int sw = hd->nu_pre + hd->nu_post;
    if (sw % 2) std::swap(e, t);
    amg_smooth(hd, 0, e, t, v, sw, true, theta_dt);
}

__global__ void k_jacobi_precond64(const double *v, const double *dg, double *z, int64_t N) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) z[n] = v[n] / dg[n];
}
__global__ void k_jacobi_precond32(const double *v, const float *dg, float *z, int64_t N) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) z[n] = (float)v[n] / dg[n];
}

// z_j = M^{-1} v_j (mixed precision: rhs_ready = the level-0 right-hand side already holds float(v_j))
void precondition_eager(hjb_handle *hd, const double *v, void *z, double theta_dt, bool rhs_ready) {
    const int64_t N = hd->N;
    hipStream_t s = hd->stream;
    Level &L0 = hd->lev[0];
    if (hd->desc.precond == HJB_PRECOND_AMG) {
        amg_precondition(hd, v, (double *)z, theta_dt);
        return;
    }
    if (hd->desc.precond == HJB_PRECOND_JACOBI) {
        int nb = blocks_for(N);
        if (mixed(hd))
            hipLaunchKernelGGL(k_jacobi_precond32, dim3(nb), dim3(kBlock), 0, s, v, (const float *)L0.d, (float *)z, N);
        else
            hipLaunchKernelGGL(k_jacobi_precond64, dim3(nb), dim3(kBlock), 0, s, v, (const double *)L0.d, (double *)z,
                               N);
        return;
    }
    if (mixed(hd)) {
        if (!rhs_ready) launch_to_precond(v, L0.r, true, N, s);
        vcycle<float>(hd, (const float *)L0.r, (float *)z, theta_dt);
    } else {
        vcycle<double>(hd, v, (double *)z, theta_dt);
    }
}

void drop_graphs(hjb_handle *hd) {
    for (auto &g : hd->vgraphs) (void)hipGraphExecDestroy(g.exec);
    hd->vgraphs.clear();
}

using ApplyFn = std::function<void(const void *, bool, double *)>;

// z = M^{-1} v, then, when apply is given, w = A z (policy apply_alpha).  The launch sequence depends only
// on buffer addresses and theta*dt, so it is captured once per (level-0 policy buffer, v, z, theta*dt,
// sweep counts, operator application) and replayed; policy, diagonal and table contents are refreshed in
// place before each replay.  A cycle sampled by the smoother, residual or apply timers runs eagerly
// (events cannot be accumulated from inside a replayed graph), its application timed with it.
int precondition(hjb_handle *hd, const double *v, void *z, double theta_dt, bool rhs_ready,
                 const ApplyFn *apply = nullptr, const void *apply_alpha = nullptr, double *w = nullptr,
                 bool zf = false) {
    const bool timers = hd->timers[HJB_KERNEL_SMOOTH].cap > 0 || hd->timers[HJB_KERNEL_MG_RESID].cap > 0 ||
                        (apply && hd->timers[HJB_KERNEL_APPLY].cap > 0);
    const bool sampled = timers && hd->vc_count++ % hd->sample_period == 0;
    auto eager = [&](bool timed) {
        hd->vc_timed = timed;
        precondition_eager(hd, v, z, theta_dt, rhs_ready);
        if (apply) {
            hd->apply_with_vcycle = true;
            (*apply)(z, zf, w);
            hd->apply_with_vcycle = false;
        }
        hd->vc_timed = false;
    };
    if (!hd->desc.use_graphs || hd->desc.precond != HJB_PRECOND_VCYCLE || sampled) {
        eager(sampled);
        return HJB_OK;
    }
    const void *a0 = hd->lev[0].alpha;
    const void *aa = apply ? apply_alpha : nullptr;
    const double *wk = apply ? w : nullptr;
    for (auto &g : hd->vgraphs)
        if (g.a0 == a0 && g.v == v && g.z == z && g.theta_dt == theta_dt && g.nu1 == hd->nu_pre &&
            g.nu2 == hd->nu_post && g.rhs_ready == rhs_ready && g.aa == aa && g.w == wk) {
            HIPCHK(hipGraphLaunch(g.exec, hd->stream));
            return HJB_OK;
        }
    if (hd->vgraphs.size() >= 256) drop_graphs(hd);
    if (!hd->capture_stream) HIPCHK(hipStreamCreateWithFlags(&hd->capture_stream, hipStreamNonBlocking));
    hipStream_t saved = hd->stream;
    hd->stream = hd->capture_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(hd->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        eager(false);
        e = hipStreamEndCapture(hd->capture_stream, &graph);
    }
    hd->stream = saved;
    if (e != hipSuccess) return fail(HJB_EDEVICE, "V-cycle capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HJB_EDEVICE, "V-cycle instantiate: %s", hipGetErrorString(e));
    hd->vgraphs.push_back({a0, v, z, theta_dt, hd->nu_pre, hd->nu_post, rhs_ready, aa, wk, exec});
    HIPCHK(hipGraphLaunch(exec, hd->stream));
    return HJB_OK;
}

// ---- flexible GMRES(m) on A^alpha x = b, with x = X on interior nodes ----------------------------

// Read small device results: a one-wave kernel copies them to pinned host memory and then releases a
// new sequence number in the pinned flag word, which the host polls (no stream event, no copy engine).
// The stream is queried every few thousand polls so that a device error ends the wait.
int publish(hjb_handle *hd, unsigned *seq, const void *dev0, void *host0, size_t bytes0,
            const void *dev1 = nullptr, void *host1 = nullptr, size_t bytes1 = 0) {
    *seq = ++hd->pub_seq;
    launch_publish(dev0, host0, bytes0, dev1, host1, bytes1, hd->hflag, *seq, hd->stream);
    HIPCHK(hipGetLastError());
    return HJB_OK;
}

int wait_published(hjb_handle *hd, unsigned seq) {
    int after_idle = 0;
    for (uint64_t it = 1;; ++it) {
        if (__atomic_load_n(hd->hflag, __ATOMIC_ACQUIRE) == seq) return HJB_OK;
        if ((it & 4095) == 0) {
            hipError_t e = hipStreamQuery(hd->stream);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return fail(HJB_EDEVICE, "hipStreamQuery: %s", hipGetErrorString(e));
            // the stream has drained; the flag store may still be on its way to host memory
            if (++after_idle > 1000) return fail(HJB_EDEVICE, "stream drained without publishing its results");
        }
    }
}

int publish_wait(hjb_handle *hd, const void *dev0, void *host0, size_t bytes0, const void *dev1 = nullptr,
                 void *host1 = nullptr, size_t bytes1 = 0) {
    unsigned seq = 0;
    TRY(publish(hd, &seq, dev0, host0, bytes0, dev1, host1, bytes1));
    return wait_published(hd, seq);
}

int sync_small(hjb_handle *hd, const void *dev, void *host, size_t bytes) {
    return publish_wait(hd, dev, host, bytes);
}

// The operator of one linear solve: residual() writes r = b - A X into hd->R with the partials
// [sum r^2 | max|r| | max|X|] (hd->nb each) in hd->partial; apply(z, z_is_float, w) writes w = A z;
// precond(v, z, ready) writes z = M^{-1} v (empty: no preconditioner, z = v).  When rhs32 is set, the
// preconditioner starts from float(v) in rhs32: the solver writes that copy while forming v and passes
// ready = true, else the preconditioner converts v itself.
struct KrylovOp {
    std::function<void()> residual;
    std::function<void(const void *, bool, double *)> apply;
    std::function<int(const double *, void *, bool)> precond;
    // optional: precond(v, z, ready) followed by apply(z, zf, w) as one unit (one captured graph)
    std::function<int(const double *, void *, double *, bool)> precond_apply;
    bool zf = false;
    float *rhs32 = nullptr;
};

// Flexible GMRES(m).  Stops when |r|_inf <= rtol_inf*max(1,|X|_inf), or, when eta > 0, once
// |r|_inf <= eta * (initial |r|_inf).
int fgmres_core(hjb_handle *hd, const KrylovOp &op, double *X, double eta, int *its_out, double *res_out,
                bool *tight_out) {
    const hjb_desc &d = hd->desc;
    const int64_t N = hd->N;
    const int m = d.restart;
    hipStream_t s = hd->stream;
    const bool none = !op.precond;
    const bool zf = !none && op.zf;
    float *const rhs32 = none ? nullptr : op.rhs32;
    // z = M^{-1} v (z = v without a preconditioner), then w = A z
    auto precond_then_apply = [&](const double *v, void *z, double *w) -> int {
        if (none) {
            op.apply(v, false, w);
            return HJB_OK;
        }
        if (op.precond_apply) return op.precond_apply(v, z, w, rhs32 != nullptr);
        TRY(op.precond(v, z, rhs32 != nullptr));
        op.apply(z, zf, w);
        return HJB_OK;
    };
    const size_t zsz = zf ? sizeof(float) : sizeof(double);
    double *V = hd->Vb;
    double *dv = hd->dvals;
    double *hp = hd->hpin;
    int its = 0;
    double loose = 0.0;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gvec(m + 1), y(m);
    for (int cycle = 0;; ++cycle) {
        op.residual();
        launch_reduce_sum(hd->partial, 1, hd->nb, dv + 0, s);
        launch_reduce_max(hd->partial + hd->nb, 2, hd->nb, dv + 1, s);
        unsigned seq = 0;
        TRY(publish(hd, &seq, dv, hp, 3 * sizeof(double)));
        // a solve rarely starts converged: its first basis vector and preconditioner application are
        // queued before the host reads the residual norms (and discarded if it has converged)
        const bool ahead = cycle == 0 && !none;
        if (ahead) {
            launch_scale_by_inv_sqrt(V, hd->R, dv + 0, N, s, rhs32);
            TRY(precond_then_apply(V, hd->Zb, V + N));
        }
        TRY(wait_published(hd, seq));
        double beta = sqrt(hp[0]), rinf = hp[1], xinf = hp[2];
        *res_out = rinf;
        *its_out = its;
        if (!isfinite(beta) || !isfinite(xinf)) return fail(HJB_ENONFINITE, "non-finite residual in linear solve");
        double target = d.rtol_inf * std::max(1.0, xinf);
        if (cycle == 0 && eta > 0.0) loose = eta * rinf;
        *tight_out = rinf <= target;
        if (rinf <= std::max(target, loose)) return HJB_OK;
        target = std::max(target, loose);
        if (its >= d.max_krylov)
            return fail(HJB_ENOCONV_KRYLOV, "FGMRES: |r|_inf = %.3e > %.3e after %d iterations", rinf, target, its);
        // v0 = r / beta
        if (!ahead) launch_scale_by_inv_sqrt(V, hd->R, dv + 0, N, s, rhs32);
        std::fill(gvec.begin(), gvec.end(), 0.0);
        gvec[0] = beta;
        int j = 0;
        for (; j < m && its < d.max_krylov; ++j) {
            double *vj = V + (int64_t)j * N;
            double *w = V + (int64_t)(j + 1) * N;
            void *zj = none ? (void *)vj : (void *)((char *)hd->Zb + (int64_t)j * N * zsz);
            if (!(ahead && j == 0)) TRY(precond_then_apply(vj, zj, w));
            // classical Gram-Schmidt run twice (CGS2): the sums <w,V_i> and |w|^2, the update and
            // normalisation (norm by Pythagoras) fused with the second pass's sums, then the second update,
            // which also writes the single-precision copy of v_{j+1} for the next preconditioner call.  A
            // strong preconditioner makes w nearly parallel to v_j, so the second pass is needed almost
            // every time; both passes are queued before the host reads their coefficients.
            {
                TimedLaunch tl(hd, HJB_KERNEL_DOT, (double)N * 8.0 * (j + 2));
                launch_multidot(w, V, N, j + 1, N, hd->partial, hd->nbd, s);
            }
            launch_reduce_sum(hd->partial, j + 2, hd->nbd, dv + kGsSlot0, s);
            {
                TimedLaunch tl(hd, HJB_KERNEL_AXPY, (double)N * 8.0 * (j + 3));
                launch_multiaxpy_scale_dot(w, V, N, j + 1, dv + kGsSlot0, N, hd->partial, hd->nbd, s);
            }
            launch_reduce_sum(hd->partial, j + 2, hd->nbd, dv + kGsSlot1, s);
            {
                TimedLaunch tl(hd, HJB_KERNEL_AXPY, (double)N * (8.0 * (j + 3) + (rhs32 ? 4.0 : 0.0)));
                launch_multiaxpy_scale(w, V, N, j + 1, dv + kGsSlot1, N, hd->nbd, s, rhs32);
            }
            TRY(publish_wait(hd, dv + kGsSlot0, hp + kGsSlot0, (size_t)(kGsSlot1 - kGsSlot0 + j + 2) * sizeof(double)));
            double hn = 0.0;
            bool dependent = false;
            for (int pass = 0; pass < 2; ++pass) {
                const double *c = hp + (pass == 0 ? kGsSlot0 : kGsSlot1);
                double w2 = c[j + 1], h2 = 0.0;
                for (int i = 0; i <= j; ++i) h2 += c[i] * c[i];
                double hn2 = w2 - h2;
                double sc = hn2 > 0.0 ? sqrt(hn2) : 1.0;  // the factor the kernel divided by
                if (!isfinite(w2)) return fail(HJB_ENONFINITE, "non-finite Arnoldi vector");
                if (pass == 0) {
                    for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = c[i];
                    hn = sc;
                    if (w2 == 0.0) dependent = true;
                } else {
                    for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] += c[i] * hn;
                    hn = hn * sc;
                    if (!(hn2 > 0.0)) dependent = true;
                }
            }
            if (dependent) hn = 0.0;  // w lies in the span of the basis: the Krylov space holds the solution
            H[(size_t)(j + 1) * m + j] = hn;
            ++its;
            // apply previous rotations to column j, then a new one
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            double r = hypot(a, b);
            cs[j] = r > 0 ? a / r : 1.0;
            sn[j] = r > 0 ? b / r : 0.0;
            H[(size_t)j * m + j] = r;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gvec[j + 1] = -sn[j] * gvec[j];
            gvec[j] = cs[j] * gvec[j];
            if (fabs(gvec[j + 1]) <= 0.5 * target || hn == 0.0) {
                ++j;
                break;
            }
        }
        // y = H^{-1} g (upper triangular j x j), x += Z y
        for (int i = j - 1; i >= 0; --i) {
            double acc = gvec[i];
            for (int q = i + 1; q < j; ++q) acc -= H[(size_t)i * m + q] * y[q];
            y[i] = acc / H[(size_t)i * m + i];
        }
        const void *Z = none ? (const void *)V : (const void *)hd->Zb;
        launch_update_solution(X, Z, zf, N, j, y.data(), N, s);
        HIPCHK(hipGetLastError());
    }
}

// BiCGSTAB with right preconditioning (the paper's Krylov baseline of Section 3.3), same stopping rule
// and certificate as fgmres_core: the recurrence runs until its updated residual meets half the target,
// then the true residual b - A X is recomputed and certifies the result, or restarts the recurrence
// (fresh shadow vector rhat = r) when rounding has made the two drift apart.  A zero denominator
// (breakdown) also restarts it.  Each iteration applies the preconditioned operator twice and counts as
// two Krylov iterations.  Vectors: rhat, p, v, t in the first four slices of Vb, s in R over r, phat and
// shat in the first two slices of Zb; the recurrence scalars stay in device slots (one host read per
// iteration, for the residual norm).
constexpr int kBicgSlot = 16;  // [rho, (rhat,v), |v|^2, (t,s), (t,t), max|r|, max|X|]

int bicgstab_core(hjb_handle *hd, const KrylovOp &op, double *X, double eta, int *its_out, double *res_out,
                  bool *tight_out) {
    const hjb_desc &d = hd->desc;
    const int64_t N = hd->N;
    hipStream_t s = hd->stream;
    const bool none = !op.precond;
    const bool zf = !none && op.zf;
    float *const rhs32 = none ? nullptr : op.rhs32;
    const size_t zsz = zf ? sizeof(float) : sizeof(double);
    double *const r = hd->R;
    double *const rhat = hd->Vb, *const p = hd->Vb + N, *const v = hd->Vb + 2 * N, *const t = hd->Vb + 3 * N;
    void *const phat = none ? (void *)p : hd->Zb;
    void *const shat = none ? (void *)r : (void *)((char *)hd->Zb + N * zsz);
    double *const sc = hd->dvals + kBicgSlot;
    double *const hs = hd->hpin + kBicgSlot;
    double *dv = hd->dvals;
    double *hp = hd->hpin;
    auto precond_then_apply = [&](const double *in, void *z, double *w) -> int {
        if (none) {
            op.apply(in, false, w);
            return HJB_OK;
        }
        if (op.precond_apply) return op.precond_apply(in, z, w, rhs32 != nullptr);
        TRY(op.precond(in, z, rhs32 != nullptr));
        op.apply(z, zf, w);
        return HJB_OK;
    };
    const int nbx = blocks_for(N);
    int its = 0;
    double loose = 0.0;
    for (int cycle = 0;; ++cycle) {
        op.residual();
        launch_reduce_sum(hd->partial, 1, hd->nb, dv + 0, s);
        launch_reduce_max(hd->partial + hd->nb, 2, hd->nb, dv + 1, s);
        TRY(publish_wait(hd, dv, hp, 3 * sizeof(double)));
        const double rr = hp[0], rinf = hp[1], xinf = hp[2];
        *res_out = rinf;
        *its_out = its;
        if (!isfinite(rr) || !isfinite(xinf)) return fail(HJB_ENONFINITE, "non-finite residual in linear solve");
        double target = d.rtol_inf * std::max(1.0, xinf);
        if (cycle == 0 && eta > 0.0) loose = eta * rinf;
        *tight_out = rinf <= target;
        if (rinf <= std::max(target, loose)) return HJB_OK;
        if (its >= d.max_krylov)
            return fail(HJB_ENOCONV_KRYLOV, "BiCGSTAB: |r|_inf = %.3e > %.3e after %d iterations", rinf,
                        std::max(target, loose), its);
        // rhat = r and rho = (rhat, r) = |r|^2
        launch_to_precond(r, rhat, false, N, s);
        launch_reduce_sum(hd->partial, 1, hd->nb, sc + 0, s);  // the residual's partial sums of r^2
        for (bool first = true; its < d.max_krylov; first = false) {
            launch_bicg_p(p, r, v, sc, first, rhs32, N, s);
            TRY(precond_then_apply(p, phat, v));
            launch_multidot(v, rhat, N, 1, N, hd->partial, hd->nbd, s);
            launch_reduce_sum(hd->partial, 2, hd->nbd, sc + 1, s);
            launch_bicg_s(r, v, sc, rhs32, N, s);
            TRY(precond_then_apply(r, shat, t));
            launch_multidot(t, r, N, 1, N, hd->partial, hd->nbd, s);
            launch_reduce_sum(hd->partial, 2, hd->nbd, sc + 3, s);
            // the update's partials come from blocks_for(N) flat blocks, not the node kernels' tiles
            launch_bicg_xr(X, r, t, phat, shat, zf, rhat, sc, hd->partial, N, s);
            launch_reduce_sum(hd->partial, 1, nbx, sc + 0, s);
            launch_reduce_max(hd->partial + nbx, 2, nbx, sc + 5, s);
            TRY(publish_wait(hd, sc, hs, 7 * sizeof(double)));
            its += 2;
            if (!isfinite(hs[5]) || !isfinite(hs[6]))
                return fail(HJB_ENONFINITE, "non-finite BiCGSTAB iterate");
            const double goal = std::max(d.rtol_inf * std::max(1.0, hs[6]), loose);
            if (hs[5] <= 0.5 * goal) break;
            if (hs[0] == 0.0 || hs[1] == 0.0 || !(hs[4] > 0.0) || hs[3] == 0.0) break;  // breakdown: restart
        }
        HIPCHK(hipGetLastError());
    }
}

// The Krylov method the descriptor selects (flexible GMRES or BiCGSTAB).
int krylov_core(hjb_handle *hd, const KrylovOp &op, double *X, double eta, int *its_out, double *res_out,
                bool *tight_out) {
    if (hd->desc.krylov == HJB_KRYLOV_BICGSTAB) return bicgstab_core(hd, op, X, eta, its_out, res_out, tight_out);
    return fgmres_core(hd, op, X, eta, its_out, res_out, tight_out);
}

int fgmres(hjb_handle *hd, const int16_t *alpha, const double *E, double *X, double theta_dt, double eta,
           int *its_out, double *res_out, bool *tight_out) {
    const int dim = hd->dim;
    const Level &L0 = hd->lev[0];
    const StencilDev st = stencil(hd, 0);
    hipStream_t s = hd->stream;
    KrylovOp op;
    op.residual = [=]() {
        launch_residual(dim, L0.g, st, alpha, X, E, theta_dt, hd->R, hd->partial, hd->nb, s);
    };
    // the application reads the handle's stream when it runs: it may be captured into a V-cycle's graph
    op.apply = [=](const void *z, bool zf, double *w) {
        TimedLaunch tl(hd, HJB_KERNEL_APPLY, (double)hd->N * ((zf ? 4.0 : 8.0) + 2.0 + 8.0));
        launch_apply(dim, L0.g, st, alpha, z, zf, w, theta_dt, nullptr, hd->nb, hd->stream);
    };
    if (hd->desc.precond != HJB_PRECOND_NONE)
        op.precond = [=](const double *v, void *z, bool ready) { return precondition(hd, v, z, theta_dt, ready); };
    if (hd->desc.precond == HJB_PRECOND_VCYCLE) {
        const ApplyFn ap = op.apply;
        const bool zf = mixed(hd);
        op.precond_apply = [=](const double *v, void *z, double *w, bool ready) {
            return precondition(hd, v, z, theta_dt, ready, &ap, alpha, w, zf);
        };
    }
    op.zf = mixed(hd) && hd->desc.precond != HJB_PRECOND_AMG;  // the aggregation cycle runs in FP64
    if (op.zf && hd->desc.precond == HJB_PRECOND_VCYCLE) op.rhs32 = (float *)L0.r;
    return krylov_core(hd, op, X, eta, its_out, res_out, tight_out);
}

// ---- policy search ------------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_tau(const double *partial, int nb, double coefA, double tau_rel,
                                              double *out) {
    // out[0] = tau and out[1] = S from max(|X|,|U|) (partial[0..nb)) and max|f| (partial[nb..2nb)); two
    // loads of each array in flight per thread; a NaN wins the maximum
    __shared__ double sx[1024], sf[1024];
    auto mx = [](double a, double b) { return (a > b || a != a) ? a : b; };
    const int t = threadIdx.x, nt = blockDim.x;
    double ax0 = 0.0, ax1 = 0.0, af0 = 0.0, af1 = 0.0;
    int q = t;
    for (; q + nt < nb; q += 2 * nt) {
        const double a0 = partial[q], a1 = partial[q + nt], f0 = partial[nb + q], f1 = partial[nb + q + nt];
        ax0 = mx(ax0, a0);
        ax1 = mx(ax1, a1);
        af0 = mx(af0, f0);
        af1 = mx(af1, f1);
    }
    for (; q < nb; q += nt) {
        ax0 = mx(ax0, partial[q]);
        af0 = mx(af0, partial[nb + q]);
    }
    sx[t] = mx(ax0, ax1);
    sf[t] = mx(af0, af1);
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (t < w) {
            sx[t] = mx(sx[t], sx[t + w]);
            sf[t] = mx(sf[t], sf[t + w]);
        }
        __syncthreads();
    }
    if (t == 0) {
        double S = coefA * sx[0] + sf[0];
        out[0] = tau_rel * S;
        out[1] = S;
    }
}

__global__ void k_sweep_tau_arg(const double *tau_dev, double *tau_copy) {
    if (threadIdx.x == 0) tau_copy[0] = tau_dev[0];
}

// Device buffers of one search: block partials of the tolerance's maxima [2 nb], tau and S [2], per-tile
// counts [nb] and their sums [2].  By default the handle's own; the allocation-free entry point passes
// slices of its static scratch.
struct SweepScratch {
    double *partial;
    double *tauS;
    int64_t *ipartial;
    int64_t *ival;
};

int sweep(hjb_handle *hd, const double *X, const double *U, const double *f0, const double *f1, double t_prev,
          double dt, double theta, const int16_t *a_in, int16_t *a_out, double *gmin, double *margin, int32_t *ties,
          int64_t *n_changed, double *tau_used, int qmode = 0, int skip = 0, int64_t *n_near = nullptr,
          const SweepScratch *sc = nullptr) {
    hipStream_t s = hd->stream;
    const Level &L0 = hd->lev[0];
    double t_mid = t_prev + theta * dt;
    const SweepScratch own{hd->partial, hd->dvals + 4, hd->ipartial, hd->ival};
    const SweepScratch &B = sc ? *sc : own;
    // decisions are reused only where the search keeps no per-node extras and the tables are fixed; the
    // reusing search runs in place (and keeps its bookkeeping in handle buffers: never with outside scratch)
    if (sc || !hd->marg || !hd->desc.certified_skip || gmin || margin || ties ||
        hd->desc.coef_model != HJB_COEF_CONST || hd->desc.f_per_control || hd->desc.P != 1)
        skip = 0;
    if (sc) qmode = 0;
    if (skip == 2 && a_in != a_out) skip = 1;
    launch_norms_xuf(hd->dim, L0.g, X, U, f0, f1, t_mid, hd->desc.K, stencil(hd, 0).fk, B.partial, hd->nb, s);
    double inv2h = 0.5 / hd->desc.h;
    double coefA = 2.0 * hd->M * inv2h + hd->cmax;
    hipLaunchKernelGGL(k_tau, dim3(1), dim3(1024), 0, s, B.partial, hd->nb, coefA, hd->desc.tau_rel, B.tauS);
    if (skip == 1) {
        launch_delta_tiles(hd->dim, L0.g, X, hd->Xs, hd->dtile, true, s);
    } else if (skip == 2) {
        // |change of G_k| <= theta (4 M / (2h) + max|c|) max|change of X| over the node's stencil (untruncated
        // nodes: unit interpolation weights); the gap shrinks by at most twice that
        const double lip2 = 2.0 * theta * (4.0 * hd->M * inv2h + hd->cmax);
        launch_delta_tiles(hd->dim, L0.g, X, hd->Xs, hd->dtile, false, s);
        launch_window_max(hd->dim, L0.g, hd->dtile, hd->dwin, hd->reach, s);
        launch_keep_pass(hd->dim, L0.g, hd->marg, hd->dwin, lip2, hd->dvals + 5, hd->keep, hd->kpartial, hd->need,
                         hd->ipartial, s);
        launch_tile_list(hd->need, hd->nb, hd->tlist, hd->tlist + hd->nb_cap, s);
    }
    SweepOut o{a_out, gmin, margin, ties, B.ipartial, skip, hd->marg, hd->keep,
               skip == 2 ? hd->tlist : nullptr, skip == 2 ? hd->tlist + hd->nb_cap : nullptr, n_near ? 1 : 0};
    if (!hd->Q) qmode = 0;
    // algorithmic FP64 work of the untruncated stencil per control and field: each point is a 2^d-corner
    // weighted sum (2^(d+1) - 1 flops), each diffusion pair adds 4, the drift 3, the 1/(2h) scaling 1
    const int P = hd->desc.P, dpts = 2 * P + (hd->has_drift ? 1 : 0);
    const double per_field = dpts * ((2 << hd->dim) - 1) + 4.0 * P + (hd->has_drift ? 3.0 : 0.0) + 1.0;
    const bool cn = theta != 1.0;
    const double per_ctl = per_field + 5.0 + ((cn && qmode != 2) ? per_field + 3.0 : 0.0);
    double n_int = 1.0;
    for (int a = 0; a < hd->dim; ++a) n_int *= (double)(hd->desc.n[a] - 2);
    const double bytes_all = (double)hd->N * (4 * 8.0 + 2.0 + 2.0) + (qmode == 2 ? n_int * 8.0 * hd->desc.K : 0.0);
    const double flops_all = n_int * (hd->desc.K * per_ctl + 2.0);
    int slot = -1;
    {
        TimedLaunch tl(hd, HJB_KERNEL_SWEEP, bytes_all, flops_all);
        slot = tl.slot;
        launch_sweep(hd->dim, L0.g, stencil(hd, 0), X, U, f0, f1, t_mid, theta, B.tauS, a_in, o, hd->Q, qmode,
                     hd->nb, s);
    }
    HIPCHK(hipGetLastError());
    hd->kept_last = 0;
    if (n_changed || tau_used || n_near || skip == 2) {
        launch_reduce_sum_i64(B.ipartial, hd->nb, B.ival, s);
        if (skip == 2) launch_reduce_sum_i64(hd->kpartial, hd->nb, B.ival + 1, s);
        TRY(publish_wait(hd, B.ival, hd->hpin_i, 2 * sizeof(int64_t), B.tauS, hd->hpin + 4, sizeof(double)));
        // the search's partials hold the changed controls in their low 32 bits and the near ties above
        if (n_changed) *n_changed = hd->hpin_i[0] & 0xffffffffll;
        if (n_near) *n_near = (int64_t)((uint64_t)hd->hpin_i[0] >> 32);
        if (tau_used) *tau_used = hd->hpin[4];
        if (skip == 2) {
            hd->kept_last = hd->hpin_i[1];
            // the timed launch did the work of the evaluated nodes only (kept ones read their control)
            if (slot >= 0) {
                const double ev = std::max(0.0, n_int - (double)hd->kept_last) / n_int;
                hd->timers[HJB_KERNEL_SWEEP].flops[slot] = flops_all * ev;
                hd->timers[HJB_KERNEL_SWEEP].bytes[slot] = bytes_all * ev + 2.0 * (double)hd->kept_last;
            }
        }
    }
    return HJB_OK;
}

bool finite_param(double x) { return isfinite(x); }

// caller-supplied policies must name a control on every interior node
int check_policy(hjb_handle *hd, const int16_t *alpha) {
    launch_bad_policy(hd->dim, hd->lev[0].g, alpha, hd->desc.K, hd->ipartial, hd->nb, hd->stream);
    launch_reduce_sum_i64(hd->ipartial, hd->nb, hd->ival, hd->stream);
    HIPCHK(hipMemcpyAsync(hd->hpin_i, hd->ival, sizeof(int64_t), hipMemcpyDeviceToHost, hd->stream));
    HIPCHK(hipStreamSynchronize(hd->stream));
    if (hd->hpin_i[0] != 0)
        return fail(HJB_EINVAL, "policy has %lld interior entries outside [0, K)", (long long)hd->hpin_i[0]);
    return HJB_OK;
}

int check_time(double dt, double theta) {
    if (!(dt > 0.0) || !isfinite(dt)) return fail(HJB_EINVAL, "dt must be positive and finite");
    if (!(theta >= 0.0 && theta <= 1.0)) return fail(HJB_EINVAL, "theta must be in [0,1]");
    return HJB_OK;
}

// V-cycle sweep counts for the next solve: solves to the certificate take nu_tight (when set)
void set_sweeps(hjb_handle *hd, bool tight) {
    const bool t = tight && hd->desc.nu_tight > 0;
    hd->nu_pre = t ? hd->desc.nu_tight : hd->desc.nu1;
    hd->nu_post = t ? hd->desc.nu_tight : hd->desc.nu2;
}

int linsolve_impl(hjb_handle *hd, const int16_t *alpha, const double *U, const double *f0, const double *f1,
                  double t_prev, double dt, double theta, double *X, double eta, int *its, double *res, bool *tight) {
    hipStream_t s = hd->stream;
    double t_mid = t_prev + theta * dt;
    launch_explicit(hd->dim, hd->lev[0].g, stencil(hd, 0), alpha, U, f0, f1, t_mid, (1.0 - theta) * dt, dt, hd->E,
                    hd->nb, s);
    TRY(prepare_mg(hd, alpha, theta * dt));
    set_sweeps(hd, eta <= 0.0);
    return fgmres(hd, alpha, hd->E, X, theta * dt, eta, its, res, tight);
}

int step_impl(hjb_handle *hd, const double *Uprev, double *Unext, const double *f0, const double *f1, double t_prev,
              double dt, double theta, int16_t *alpha_io, const double *Uprev2, double dt_prev, hjb_step_stats *st) {
    hipStream_t s = hd->stream;
    const int64_t N = hd->N;
    hjb_step_stats loc{};
    hd->amg_fresh = true;
    if (theta == 0.0) {
        // explicit scheme: U^n = U^{n-1} + dt min_k G_k(U^{n-1}) on interior nodes, one search and no solve
        // (G_k at theta = 0 equals the theta = 1 quantity evaluated at X = U, with f at t_{n-1})
        TRY(sweep(hd, Uprev, Uprev, f0, f1, t_prev, 0.0, 1.0, alpha_io, hd->a0, hd->E, nullptr, nullptr, nullptr,
                  nullptr, 0));
        launch_explicit_update(hd->dim, hd->lev[0].g, Uprev, hd->E, dt, Unext, s);
        HIPCHK(hipMemcpyAsync(alpha_io, hd->a0, (size_t)N * sizeof(int16_t), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipGetLastError());
        // positivity of the explicit scheme (eq. CFL_trunc): (1 - theta) dt (M/h + |c|) <= 1 for interior weights
        if (dt * (hd->M / hd->desc.h + hd->cmax) > 1.0) loc.flags |= HJB_FLAG_POSITIVITY;
        if (st) *st = loc;
        return HJB_OK;
    }
    if (Uprev2)
        launch_extrapolate(hd->dim, hd->lev[0].g, Uprev, Uprev2, dt / dt_prev, Unext, s);
    else
        launch_copy_interior(hd->dim, hd->lev[0].g, Uprev, Unext, s);
    int16_t *acur = hd->a0;
    int64_t changed = 0;
    // the explicit part of every G_k is fixed within the step: the first search stores it (when the
    // handle could afford the K*N cache) and the later searches read it
    TRY(sweep(hd, Unext, Uprev, f0, f1, t_prev, dt, theta, alpha_io, acur, nullptr, nullptr, nullptr, &changed,
              nullptr, 1, 1));
    loc.n_changed_first = changed;
    double cert_den = 1.0 - theta * dt * hd->cplus;
    if (theta < 1.0) {
        // eq. CFL_trunc can only be guaranteed for theta < 1 when (1-theta) dt M/h <= 1 (interior weights)
        double lhs = (1.0 - theta) * dt * (hd->M / hd->desc.h + hd->cmax);
        if (lhs > 1.0) loc.flags |= HJB_FLAG_POSITIVITY;
    }
    int rc = HJB_OK;
    // Policy iteration.  While the policy may still change a solve only reduces the residual by pi_eta;
    // a step ends after a solve to rtol_inf whose search changes no control.
    bool want_tight = hd->desc.pi_eta <= 0.0;
    for (int it = 0; it < hd->desc.max_pi; ++it) {
        int its = 0;
        double res = 0.0;
        bool tight = false;
        rc = linsolve_impl(hd, acur, Uprev, f0, f1, t_prev, dt, theta, Unext, want_tight ? 0.0 : hd->desc.pi_eta,
                           &its, &res, &tight);
        loc.pi_iters = it + 1;
        loc.krylov_total += its;
        loc.krylov_max = std::max(loc.krylov_max, its);
        loc.res_inf = res;
        loc.cert_bound = cert_den > 0 ? res / cert_den : INFINITY;
        if (rc != HJB_OK) break;
        // the search updates the policy in place (it reads only each node's own control)
        // near ties are counted by the searches that may end the step: those after a solve to the certificate
        int64_t near = 0;
        TRY(sweep(hd, Unext, Uprev, f0, f1, t_prev, dt, theta, acur, acur, nullptr, nullptr, nullptr, &changed,
                  nullptr, 2, 2, tight ? &near : nullptr));
        if (tight) loc.n_near_ties = near;
        if (hd->trace)
            fprintf(stderr, "[slhjb] pi %d: krylov %d res %.3e tight %d changed %lld kept %lld\n", it, its, res,
                    (int)tight, (long long)changed, (long long)hd->kept_last);
        if (changed == 0) {
            if (tight) break;
            want_tight = true;  // same policy, finish the solve
        } else {
            want_tight = hd->desc.pi_eta <= 0.0;
        }
        if (it + 1 == hd->desc.max_pi) rc = fail(HJB_ENOCONV_PI, "policy iteration not converged after %d", it + 1);
    }
    // the decisions of the last search are those of the returned policy
    if (loc.n_near_ties > 0) loc.flags |= HJB_FLAG_NEAR_TIES;
    if (acur != alpha_io) {
        hipError_t e = hipMemcpyAsync(alpha_io, acur, (size_t)N * sizeof(int16_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) rc = fail(HJB_EDEVICE, "copy policy: %s", hipGetErrorString(e));
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess && rc == HJB_OK) rc = fail(HJB_EDEVICE, "%s", hipGetErrorString(e));
    if (st) *st = loc;
    return rc;
}

}  // namespace

// =====================================================================================================
// C ABI
// =====================================================================================================

extern "C" {

void hjb_desc_default(hjb_desc *d) {
    if (!d) return;
    memset(d, 0, sizeof *d);
    d->dim = 2;
    d->scheme = 2;
    d->coef_model = HJB_COEF_CONST;
    d->precision = HJB_PREC_FP64;
    d->precond = HJB_PRECOND_VCYCLE;
    d->restart = 10;
    d->max_krylov = 600;
    d->max_pi = 50;
    d->nu1 = 3;
    d->nu2 = 3;
    d->coarse_sweeps = 4;
    d->min_coarse = 17;
    d->omega = 0.9;
    d->rtol_inf = 1e-13;
    d->tau_rel = 1e-13;
    d->pi_eta = 0.35;
    d->use_graphs = 1;
    d->certified_skip = 1;
    d->max_levels = 2;
    d->nu_tight = 4;
    d->coarse_sweeps_t = 2;
    d->krylov = HJB_KRYLOV_FGMRES;
    d->coarse_op = HJB_COARSE_REDISCRETIZED;
    d->kcycle_levels = -1;
    d->value_stride = 1;
    d->amg_reuse = 0;
    d->stream = nullptr;
}

const char *hjb_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// tables_only: level geometry and stencil tables, no work vectors (instances of a batch)
// ---- allocation-free search ----------------------------------------------------------------------
// The scratch of hjb_policy_sweep_noalloc (see SweepScratch), one copy per GPU for the life of the process.
// In host code `scratch` names a host-side stand-in; the device address of each GPU's copy is looked up once
// per device (at the first setup on it) and only that address is used.
constexpr size_t kNoAllocScratchBytes = (size_t)1 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// slices of the scratch for a search over nb tiles: [partial 2nb | tau, S | ipartial nb | ival 2], each
// 256-byte aligned; the bytes needed (may exceed the scratch: checked by the caller)
size_t noalloc_layout(char *base, int nb, SweepScratch *sc) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_partial = off;
    off += up((size_t)2 * nb * 8);
    const size_t o_tau = off;
    off += up(2 * 8);
    const size_t o_ip = off;
    off += up((size_t)nb * 8);
    const size_t o_iv = off;
    off += up(2 * 8);
    if (sc && base) {
        sc->partial = (double *)(base + o_partial);
        sc->tauS = (double *)(base + o_tau);
        sc->ipartial = (int64_t *)(base + o_ip);
        sc->ival = (int64_t *)(base + o_iv);
    }
    return off;
}

// device address of the current GPU's scratch (looked up once per device)
int scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HJB_EDEVICE, "device id %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return HJB_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(HJB_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    return HJB_OK;
}

int setup_impl(const hjb_desc *desc, hjb_handle **out, bool tables_only) {
    g_err.clear();
    if (!desc || !out) return fail(HJB_EINVAL, "null argument");
    *out = nullptr;
    const hjb_desc &d = *desc;
    if (d.dim != 2 && d.dim != 3) return fail(HJB_EINVAL, "dim must be 2 or 3");
    int64_t N = 1;
    for (int a = 0; a < d.dim; ++a) {
        if (d.n[a] < 3) return fail(HJB_EINVAL, "n[%d] must be >= 3", a);
        N *= d.n[a];
    }
    if (N >= (int64_t)1 << 31) return fail(HJB_EINVAL, "grid too large (N must be < 2^31)");
    if (!(d.h > 0.0) || !isfinite(d.h)) return fail(HJB_EINVAL, "h must be positive");
    if (d.K < 1 || d.K > 32767) return fail(HJB_EINVAL, "K must be in 1..32767");
    if (d.P < 1 || d.P > kMaxP) return fail(HJB_EINVAL, "P must be in 1..%d", kMaxP);
    if (d.scheme != 2) return fail(HJB_EUNSUPPORTED, "only Scheme 2 is provided (consistent truncation)");
    if (d.coef_model != HJB_COEF_CONST && d.coef_model != HJB_COEF_XSCALED && d.coef_model != HJB_COEF_FIELD)
        return fail(HJB_EUNSUPPORTED, "coefficient model %d is not provided", d.coef_model);
    if (!d.sigma) return fail(HJB_EINVAL, "sigma is required");
    TRY(check_options(&d));
    const int64_t nsig = (d.coef_model == HJB_COEF_FIELD ? N : (int64_t)d.K) * d.P * d.dim;
    for (int64_t q = 0; q < nsig; ++q)
        if (!isfinite(d.sigma[q])) return fail(HJB_EINVAL, "non-finite sigma");
    if (d.drift)
        for (int64_t q = 0; q < (int64_t)d.K * d.dim; ++q)
            if (!isfinite(d.drift[q])) return fail(HJB_EINVAL, "non-finite drift");
    if (d.c)
        for (int q = 0; q < d.K; ++q)
            if (!isfinite(d.c[q])) return fail(HJB_EINVAL, "non-finite c");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(HJB_EDEVICE, "no HIP device available");

    hjb_handle *hd = new hjb_handle();
    hd->desc = d;
    {
        const char *tr = getenv("SLHJB_TRACE");
        hd->trace = tr && tr[0] == '1';
    }
    hd->dim = d.dim;
    hd->N = N;
    hd->stream = (hipStream_t)d.stream;
    hd->sigma.assign(d.sigma, d.sigma + (size_t)nsig);
    hd->drift.assign((size_t)d.K * d.dim, 0.0);
    if (d.drift) {
        hd->drift.assign(d.drift, d.drift + (size_t)d.K * d.dim);
        for (double b : hd->drift) hd->has_drift |= (b != 0.0);
    }
    if (d.c) {
        hd->c.assign(d.c, d.c + d.K);
        for (double cc : hd->c) {
            hd->cmax = std::max(hd->cmax, fabs(cc));
            hd->cplus = std::max(hd->cplus, cc);
        }
    }
    hd->desc.sigma = hd->sigma.data();
    hd->desc.drift = hd->drift.data();
    hd->desc.c = hd->c.empty() ? nullptr : hd->c.data();
    hd->npt = 2 * d.P + (hd->has_drift ? 1 : 0);
    hd->M = d.P + (hd->has_drift ? 1 : 0);
    hd->nbd = dot_blocks(N);

    auto cleanup_fail = [&](int rc) {
        hjb_destroy(hd);
        return rc;
    };
#define STRY(x)                                 \
    do {                                        \
        int _rc = (x);                          \
        if (_rc != HJB_OK) return cleanup_fail(_rc); \
    } while (0)

    // levels: halve while every axis has an even number of cells and the grid is above the coarse size
    {
        int n[3] = {d.n[0], d.dim > 1 ? d.n[1] : 1, d.dim > 2 ? d.n[2] : 1};
        for (;;) {
            Level L;
            for (int a = 0; a < 3; ++a) L.g.n[a] = a < d.dim ? n[a] : 1;
            L.g.N = (int64_t)L.g.n[0] * L.g.n[1] * L.g.n[2];
            L.g.s1 = L.g.n[0];
            L.g.s2 = (int64_t)L.g.n[0] * L.g.n[1];
            L.g.tlog = kTileLog2;
            set_tiles(L.g, d.dim);
            hd->lev.push_back(L);
            bool can = true, small = true;
            for (int a = 0; a < d.dim; ++a) {
                can = can && ((n[a] - 1) % 2 == 0) && ((n[a] - 1) / 2 + 1 >= 3);
                small = small && n[a] <= std::max(3, d.min_coarse);
            }
            if (!can || (small && L.g.N <= kCoarseMaxNodes)) break;
            if (d.max_levels > 0 && (int)hd->lev.size() >= d.max_levels) break;
            for (int a = 0; a < d.dim; ++a) n[a] = (n[a] - 1) / 2 + 1;
        }
    }
    for (size_t l = 0; l < hd->lev.size(); ++l) {
        Level &L = hd->lev[l];
        size_t n = (size_t)L.g.N;
        STRY(dalloc(hd, (void **)&L.tab, (size_t)d.K * hd->npt * sizeof(PointTab)));
        STRY(dalloc(hd, (void **)&L.fastF, (size_t)d.K * hd->npt * sizeof(FastPtF)));
        STRY(dalloc(hd, (void **)&L.fastD, (size_t)d.K * hd->npt * sizeof(FastPtD)));
        STRY(dalloc(hd, (void **)&L.lii, (size_t)d.K * sizeof(double)));
        STRY(dalloc(hd, (void **)&L.wctl, (size_t)tiles_cap(L.g, d.dim) * (kBlock / 64) * sizeof(int16_t)));
        STRY(dalloc(hd, (void **)&L.dk32, (size_t)d.K * sizeof(float)));
        STRY(dalloc(hd, (void **)&L.dk64, (size_t)d.K * sizeof(double)));
        if (d.coarse_op == HJB_COARSE_GALERKIN && l >= 1 && !tables_only) {
            STRY(dalloc(hd, (void **)&L.gcol, n * kGalWidth * 4));
            STRY(dalloc(hd, (void **)&L.gval, n * kGalWidth * 8));
            STRY(dalloc(hd, (void **)&L.gval32, n * kGalWidth * 4));
        }
        if (d.coarse_op == HJB_COARSE_GALERKIN && l == 0 && !tables_only) {
            const size_t E0 = (size_t)hd->npt * 4 + 1;
            STRY(dalloc(hd, (void **)&hd->g0col, n * E0 * 4));
            STRY(dalloc(hd, (void **)&hd->g0val, n * E0 * 8));
            STRY(dalloc(hd, (void **)&hd->goverflow, 8));
        }
        if (d.coef_model == HJB_COEF_FIELD) {
            // per-node sigma on this level: the finest level's value at the coinciding node
            const int pd = d.P * d.dim, stp = 1 << l;
            std::vector<double> sl(n * pd);
            for (size_t I = 0; I < n; ++I) {
                const int64_t ix = (int64_t)(I % L.g.n[0]), r = (int64_t)(I / L.g.n[0]);
                const int64_t iy = r % L.g.n[1], iz = r / L.g.n[1];
                const int64_t i0 = ix * stp + iy * stp * d.n[0] + (d.dim > 2 ? iz * stp * (int64_t)d.n[0] * d.n[1] : 0);
                for (int q = 0; q < pd; ++q) sl[I * pd + q] = hd->sigma[(size_t)i0 * pd + q];
            }
            STRY(dalloc(hd, (void **)&L.sig_node, n * pd * 8));
            hipError_t e = hipMemcpy(L.sig_node, sl.data(), n * pd * 8, hipMemcpyHostToDevice);
            if (e != hipSuccess) return cleanup_fail(fail(HJB_EDEVICE, "%s", hipGetErrorString(e)));
        }
        if (tables_only) continue;
        if (l > 0) STRY(dalloc(hd, (void **)&L.alpha, n * sizeof(int16_t)));
        STRY(dalloc(hd, &L.r64, n * 8));
        STRY(dalloc(hd, &L.e64, n * 8));
        STRY(dalloc(hd, &L.t64, n * 8));
        STRY(dalloc(hd, &L.d64, n * 8));
        STRY(dalloc(hd, &L.r32, n * 4));
        STRY(dalloc(hd, &L.e32, n * 4));
        STRY(dalloc(hd, &L.t32, n * 4));
        STRY(dalloc(hd, &L.d32, n * 4));
    }
    hd->nb = tiles_for(hd->lev[0].g);  // blocks of the node kernels on the finest grid (partial sums)
    for (int tl = kTileLogMin; tl <= kTileLogMax; ++tl) {
        LevelDev g = hd->lev[0].g;
        g.tlog = tl;
        set_tiles(g, d.dim);
        hd->nb_cap = std::max(hd->nb_cap, tiles_for(g));
    }
    select_precision(hd);
    set_sweeps(hd, false);
    if (!tables_only) {
    STRY(dalloc(hd, (void **)&hd->E, N * 8));
    STRY(dalloc(hd, (void **)&hd->R, N * 8));
    STRY(dalloc(hd, (void **)&hd->Vb, (size_t)(d.restart + 1) * N * 8));
    STRY(dalloc(hd, (void **)&hd->Zb, (size_t)d.restart * N * 8));
    STRY(dalloc(hd, (void **)&hd->Ua, N * 8));
    STRY(dalloc(hd, (void **)&hd->Ub, N * 8));
    STRY(dalloc(hd, (void **)&hd->Uc, N * 8));
    STRY(dalloc(hd, (void **)&hd->marg, N * 8));
    STRY(dalloc(hd, (void **)&hd->Xs, N * 8));
    STRY(dalloc(hd, (void **)&hd->dtile, (size_t)hd->nb_cap * 8));
    STRY(dalloc(hd, (void **)&hd->dwin, (size_t)hd->nb_cap * 8));
    STRY(dalloc(hd, (void **)&hd->keep, (size_t)hd->nb_cap * (kBlock / 64)));
    STRY(dalloc(hd, (void **)&hd->kpartial, (size_t)hd->nb_cap * 8));
    STRY(dalloc(hd, (void **)&hd->need, (size_t)hd->nb_cap));
    STRY(dalloc(hd, (void **)&hd->tlist, ((size_t)hd->nb_cap + 1) * 4));
    STRY(dalloc(hd, (void **)&hd->a0, N * 2));
    STRY(dalloc(hd, (void **)&hd->a1, N * 2));
    STRY(dalloc(hd, (void **)&hd->acarry, N * 2));
    {
        // cache of the explicit part of the search values (K doubles per node) when it is affordable
        size_t qbytes = (size_t)d.K * (size_t)hd->nb_cap * kBlock * 8;  // tile-major, one slot per thread
        size_t freeb = 0, totalb = 0;
        if (hipMemGetInfo(&freeb, &totalb) == hipSuccess && qbytes <= freeb / 4 && qbytes <= ((size_t)16 << 30)) {
            void *p = nullptr;
            if (hipMalloc(&p, qbytes) == hipSuccess) {
                hd->Q = (double *)p;
                hd->allocs.push_back(p);
            } else {
                (void)hipGetLastError();
            }
        }
    }
    }
    size_t np = tables_only ? 16 : std::max<size_t>(3 * (size_t)hd->nb_cap, (size_t)(kMaxRestart + 2) * hd->nbd);
    STRY(dalloc(hd, (void **)&hd->partial, np * 8));
    STRY(dalloc(hd, (void **)&hd->dvals, kSmallSlots * 8));
    STRY(dalloc(hd, (void **)&hd->ipartial, (size_t)hd->nb_cap * 8));
    STRY(dalloc(hd, (void **)&hd->ival, 64));
    if (!hd->c.empty()) {
        STRY(dalloc(hd, (void **)&hd->c_dev, (size_t)d.K * 8));
        hipError_t e = hipMemcpy(hd->c_dev, hd->c.data(), (size_t)d.K * 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) return cleanup_fail(fail(HJB_EDEVICE, "%s", hipGetErrorString(e)));
    }
    {
        // fine-grained (coherent) host memory: kernels store small results and the publish flag into it
        hipError_t e = hipHostMalloc((void **)&hd->hpin, kSmallSlots * sizeof(double), hipHostMallocCoherent);
        if (e != hipSuccess) return cleanup_fail(fail(HJB_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e)));
        e = hipHostMalloc((void **)&hd->hpin_i, 8 * sizeof(int64_t), hipHostMallocCoherent);
        if (e != hipSuccess) return cleanup_fail(fail(HJB_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e)));
        e = hipHostMalloc((void **)&hd->hflag, 64, hipHostMallocCoherent);
        if (e != hipSuccess) return cleanup_fail(fail(HJB_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e)));
        *hd->hflag = 0u;
    }
    STRY(build_tables(hd, 1.0));
    {
        // this GPU's copy of the allocation-free scratch
        hipError_t e = hipGetDevice(&hd->device);
        if (e != hipSuccess) return cleanup_fail(fail(HJB_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
        STRY(scratch_init(hd->device));
    }
#undef STRY
    *out = hd;
    return HJB_OK;
}

}  // namespace

extern "C" {

int hjb_setup(const hjb_desc *desc, hjb_handle **out) { return setup_impl(desc, out, false); }

int hjb_set_stream(hjb_handle *hd, void *stream) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    hd->stream = (hipStream_t)stream;
    return HJB_OK;
}

int hjb_set_options(hjb_handle *hd, const hjb_desc *desc) {
    if (!hd || !desc) return fail(HJB_EINVAL, "null argument");
    TRY(check_options(desc));
    if (desc->restart > hd->desc.restart)
        return fail(HJB_EINVAL, "restart cannot grow beyond the value given at setup (%d)", hd->desc.restart);
    hjb_desc &d = hd->desc;
    d.precision = desc->precision;
    d.precond = desc->precond;
    d.restart = desc->restart;
    d.max_krylov = desc->max_krylov;
    d.max_pi = desc->max_pi;
    d.nu1 = desc->nu1;
    d.nu2 = desc->nu2;
    d.coarse_sweeps = desc->coarse_sweeps;
    d.omega = desc->omega;
    d.rtol_inf = desc->rtol_inf;
    d.tau_rel = desc->tau_rel;
    d.pi_eta = desc->pi_eta;
    d.use_graphs = desc->use_graphs;
    d.certified_skip = desc->certified_skip;
    d.nu_tight = desc->nu_tight;
    d.coarse_sweeps_t = desc->coarse_sweeps_t;
    d.krylov = desc->krylov;
    d.kcycle_levels = desc->kcycle_levels;
    d.value_stride = desc->value_stride;
    d.amg_reuse = desc->amg_reuse;
    if (desc->coarse_op != d.coarse_op) return fail(HJB_EINVAL, "coarse_op is fixed at setup");
    select_precision(hd);
    set_sweeps(hd, false);
    drop_graphs(hd);
    return HJB_OK;
}

int hjb_policy_sweep(hjb_handle *hd, const double *X, const double *U, const double *f0, const double *f1,
                     double t_prev, double dt, double theta, double s, const int16_t *alpha_in, int16_t *alpha_out,
                     double *gmin, double *margin, int32_t *ties, int64_t *n_changed, double *tau_used) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!X || !U || !f0 || !f1 || !alpha_in || !alpha_out) return fail(HJB_EINVAL, "null array argument");
    if (!finite_param(t_prev)) return fail(HJB_EINVAL, "t_prev must be finite");
    TRY(check_time(dt, theta));
    TRY(build_tables(hd, s));
    int64_t ch = 0;
    TRY(sweep(hd, X, U, f0, f1, t_prev, dt, theta, alpha_in, alpha_out, gmin, margin, ties, n_changed ? &ch : nullptr,
              tau_used));
    if (n_changed) *n_changed = ch;
    return HJB_OK;
}

int hjb_policy_sweep_noalloc(hjb_handle *hd, const double *X, const double *U, const double *f0, const double *f1,
                             double t_prev, double dt, double theta, double s, const int16_t *alpha_in,
                             int16_t *alpha_out, double *gmin, double *margin, int32_t *ties, int64_t *n_changed,
                             double *tau_used) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!X || !U || !f0 || !f1 || !alpha_in || !alpha_out) return fail(HJB_EINVAL, "null array argument");
    if (!finite_param(t_prev)) return fail(HJB_EINVAL, "t_prev must be finite");
    TRY(check_time(dt, theta));
    // building tables for another s allocates host memory: the tables must already be those of s
    if (s != hd->s_tab)
        return fail(HJB_EINVAL, "allocation-free search: the handle's stencil tables are built for s = %.17g, not %.17g "
                                "(one call of another entry point with this s builds them)", hd->s_tab, s);
    const size_t need = noalloc_layout(nullptr, hd->nb, nullptr);
    if (need > kNoAllocScratchBytes)
        return fail(HJB_EINVAL, "allocation-free search: %d tiles need %zu bytes of scratch, the limit is %zu "
                                "(about %zu tiles)", hd->nb, need, kNoAllocScratchBytes,
                    (kNoAllocScratchBytes - 1024) / 24);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = (hd->device >= 0 && hd->device < kMaxDevices) ? g_scratch_ptr[hd->device] : nullptr;
    }
    if (!base) return fail(HJB_EDEVICE, "allocation-free scratch not set up on device %d", hd->device);
    SweepScratch sc{};
    noalloc_layout((char *)base, hd->nb, &sc);
    int64_t ch = 0;
    TRY(sweep(hd, X, U, f0, f1, t_prev, dt, theta, alpha_in, alpha_out, gmin, margin, ties, n_changed ? &ch : nullptr,
              tau_used, 0, 0, nullptr, &sc));
    if (n_changed) *n_changed = ch;
    return HJB_OK;
}

int hjb_apply(hjb_handle *hd, const int16_t *alpha, const double *x, double *y, double dt, double theta, double s) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!alpha || !x || !y) return fail(HJB_EINVAL, "null array argument");
    if (x == y) return fail(HJB_EINVAL, "x and y must be distinct");
    TRY(check_time(dt, theta));
    TRY(build_tables(hd, s));
    TRY(check_policy(hd, alpha));
    launch_apply(hd->dim, hd->lev[0].g, stencil(hd, 0), alpha, x, false, y, theta * dt, nullptr, hd->nb, hd->stream);
    HIPCHK(hipGetLastError());
    return HJB_OK;
}

int hjb_linsolve(hjb_handle *hd, const int16_t *alpha, const double *U, const double *f0, const double *f1,
                 double t_prev, double dt, double theta, double s, double *X, hjb_step_stats *st) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!alpha || !U || !f0 || !f1 || !X) return fail(HJB_EINVAL, "null array argument");
    TRY(check_time(dt, theta));
    if (theta == 0.0) return fail(HJB_EINVAL, "theta = 0 has no linear system");
    TRY(build_tables(hd, s));
    TRY(check_policy(hd, alpha));
    int its = 0;
    double res = 0.0;
    bool tight = false;
    hd->amg_fresh = true;
    int rc = linsolve_impl(hd, alpha, U, f0, f1, t_prev, dt, theta, X, 0.0, &its, &res, &tight);
    if (st) {
        memset(st, 0, sizeof *st);
        st->pi_iters = 0;
        st->krylov_total = its;
        st->krylov_max = its;
        st->res_inf = res;
        double den = 1.0 - theta * dt * hd->cplus;
        st->cert_bound = den > 0 ? res / den : INFINITY;
    }
    hipError_t e = hipStreamSynchronize(hd->stream);
    if (e != hipSuccess && rc == HJB_OK) rc = fail(HJB_EDEVICE, "%s", hipGetErrorString(e));
    return rc;
}

int hjb_step(hjb_handle *hd, const double *Uprev, double *Unext, const double *f0, const double *f1, double t_prev,
             double dt, double theta, double s, int16_t *alpha_io, const double *Uprev2, double dt_prev,
             hjb_step_stats *st) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!Uprev || !Unext || !f0 || !f1 || !alpha_io) return fail(HJB_EINVAL, "null array argument");
    if (Uprev == Unext || Uprev2 == Unext) return fail(HJB_EINVAL, "Unext must differ from Uprev and Uprev2");
    if (Uprev2 && !(dt_prev > 0.0 && isfinite(dt_prev))) return fail(HJB_EINVAL, "dt_prev must be positive");
    TRY(check_time(dt, theta));
    TRY(build_tables(hd, s));
    return step_impl(hd, Uprev, Unext, f0, f1, t_prev, dt, theta, alpha_io, Uprev2, dt_prev, st);
}

int hjb_solve(hjb_handle *hd, const double *g, const double *psi, const double *psi1, const double *f0,
              const double *f1, int32_t n_steps, const double *dts, const double *thetas, double s, double *U_final,
              int16_t *policies, double *values, hjb_solve_stats *st) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!g || !psi || !f0 || !f1 || !dts || !thetas || !U_final) return fail(HJB_EINVAL, "null argument");
    if (n_steps < 0) return fail(HJB_EINVAL, "n_steps must be >= 0");
    for (int n = 0; n < n_steps; ++n) TRY(check_time(dts[n], thetas[n]));
    TRY(build_tables(hd, s));
    const int64_t N = hd->N;
    hipStream_t str = hd->stream;
    hjb_solve_stats loc{};
    HIPCHK(hipMemcpyAsync(hd->Ua, g, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
    HIPCHK(hipMemcpyAsync(hd->Uc, g, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
    int16_t *acarry = hd->acarry;
    launch_zero(acarry, (size_t)N * 2, str);
    double *Ucur = hd->Ua, *Unx = hd->Ub, *Uold = hd->Uc;
    double t = 0.0;
    int rc = HJB_OK;
    if (values) HIPCHK(hipMemcpyAsync(values, g, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
    for (int n = 0; n < n_steps; ++n) {
        // boundary entries of U^n: psi(t_n) (the interior is overwritten by the step)
        if (psi1)
            launch_affine(psi, psi1, t + dts[n], Unx, N, str);
        else
            HIPCHK(hipMemcpyAsync(Unx, psi, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
        hjb_step_stats sst{};
        rc = step_impl(hd, Ucur, Unx, f0, f1, t, dts[n], thetas[n], acarry, n >= 1 ? Uold : nullptr,
                       n >= 1 ? dts[n - 1] : 0.0, &sst);
        loc.krylov_total += sst.krylov_total;
        loc.pi_total += sst.pi_iters;
        loc.flags |= sst.flags;
        loc.near_ties_total += sst.n_near_ties;
        loc.max_cert_bound = std::max(loc.max_cert_bound, sst.cert_bound);
        if (rc != HJB_OK) break;
        if (policies) HIPCHK(hipMemcpyAsync(policies + (int64_t)n * N, acarry, (size_t)N * 2, hipMemcpyDeviceToDevice, str));
        if (values && (n + 1) % hd->desc.value_stride == 0)
            HIPCHK(hipMemcpyAsync(values + (int64_t)((n + 1) / hd->desc.value_stride) * N, Unx, (size_t)N * 8,
                                  hipMemcpyDeviceToDevice, str));
        std::swap(Uold, Ucur);  // Uold <- U^{n-1}
        std::swap(Ucur, Unx);   // Ucur <- U^n
        t = t + dts[n];
        loc.steps_done = n + 1;
    }
    HIPCHK(hipMemcpyAsync(U_final, Ucur, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
    HIPCHK(hipStreamSynchronize(str));
    if (st) *st = loc;
    return rc;
}

int hjb_profile_enable(hjb_handle *hd, int32_t kernel, int32_t max_launches) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (kernel < 0 || kernel >= HJB_KERNEL_COUNT) return fail(HJB_EINVAL, "unknown kernel id %d", kernel);
    if (max_launches < 0 || max_launches > 100000) return fail(HJB_EINVAL, "max_launches in 0..100000");
    auto &T = hd->timers[kernel];
    HIPCHK(hipStreamSynchronize(hd->stream));
    while ((int)T.ev.size() < 2 * max_launches) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        T.ev.push_back(e);
    }
    T.bytes.assign((size_t)max_launches, 0.0);
    T.flops.assign((size_t)max_launches, 0.0);
    T.cap = max_launches;
    T.used = 0;
    T.calls = 0;
    if (kernel == HJB_KERNEL_SMOOTH || kernel == HJB_KERNEL_MG_RESID) hd->vc_count = 0;
    return HJB_OK;
}

int hjb_profile_sample(hjb_handle *hd, int32_t period) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (period < 1 || period > 1000000) return fail(HJB_EINVAL, "sampling period in 1..1000000");
    hd->sample_period = period;
    return HJB_OK;
}

int hjb_profile_read(hjb_handle *hd, int32_t kernel, int64_t *launches, double *total_ms, double *total_bytes,
                     double *total_flops) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (kernel < 0 || kernel >= HJB_KERNEL_COUNT) return fail(HJB_EINVAL, "unknown kernel id %d", kernel);
    auto &T = hd->timers[kernel];
    HIPCHK(hipStreamSynchronize(hd->stream));
    double ms = 0.0, by = 0.0, fl = 0.0;
    for (int q = 0; q < T.used; ++q) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, T.ev[2 * q], T.ev[2 * q + 1]));
        ms += t;
        by += T.bytes[q];
        fl += T.flops[q];
    }
    if (launches) *launches = T.used;
    if (total_ms) *total_ms = ms;
    if (total_bytes) *total_bytes = by;
    if (total_flops) *total_flops = fl;
    return HJB_OK;
}

}  // extern "C"

// ---- tile shape and its tuner ---------------------------------------------------------------------

namespace {

// every level takes width 2^tlog, but not wider than the level's own next power of two
void apply_tiles(hjb_handle *hd, int tlog) {
    for (Level &L : hd->lev) {
        int w = kTileLogMin;
        while (w < tlog && (1 << w) < L.g.n[0]) ++w;
        L.g.tlog = w;
        set_tiles(L.g, hd->dim);
    }
    hd->nb = tiles_for(hd->lev[0].g);
    hd->tlog = tlog;
    drop_graphs(hd);
}

std::string tune_key(const hjb_handle *hd) {
    const hjb_desc &d = hd->desc;
    double reach = 0.0, xmax = 1.0;
    if (d.coef_model == HJB_COEF_XSCALED) {
        xmax = 0.0;
        for (int a = 0; a < d.dim; ++a)
            xmax = std::max(xmax, std::max(fabs(d.lo[a]), fabs(d.lo[a] + (d.n[a] - 1) * d.h)));
    }
    const double sr = hd->s_tab * (1.0 / sqrt(d.h));
    for (double v : hd->sigma) reach = std::max(reach, fabs(sr * v) * xmax);
    for (double v : hd->drift) reach = std::max(reach, fabs(v) * xmax);
    char buf[256];
    snprintf(buf, sizeof buf, "dim=%d n=%dx%dx%d K=%d P=%d npt=%d coef=%d prec=%d reach=%.1f", d.dim, d.n[0],
             d.dim > 1 ? d.n[1] : 1, d.dim > 2 ? d.n[2] : 1, d.K, d.P, hd->npt, d.coef_model, d.precision,
             std::round(reach * 2.0) / 2.0);
    return buf;
}

// tile width recorded for `key` in a JSON-lines cache, or 0
int cache_lookup(const char *path, const std::string &key) {
    FILE *f = fopen(path, "r");
    if (!f) return 0;
    char line[4096];
    int found = 0;
    const std::string pat = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, pat.c_str())) continue;
        const char *w = strstr(line, "\"tile_width\": ");
        if (w) found = atoi(w + 14);
    }
    fclose(f);
    return found;
}

}  // namespace

extern "C" {

int hjb_set_tile_width(hjb_handle *hd, int32_t width) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    int tl = -1;
    for (int c = kTileLogMin; c <= kTileLogMax; ++c)
        if (width == (1 << c)) tl = c;
    if (tl < 0) return fail(HJB_EINVAL, "tile width must be 16, 32, 64 or 128");
    HIPCHK(hipStreamSynchronize(hd->stream));
    apply_tiles(hd, tl);
    return HJB_OK;
}

int hjb_autotune(hjb_handle *hd, const char *cache_path, int32_t *tile_width_out, double *cost_ms_out) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    const std::string key = tune_key(hd);
    if (cache_path) {
        int w = cache_lookup(cache_path, key);
        if (w) {
            TRY(hjb_set_tile_width(hd, w));
            if (tile_width_out) *tile_width_out = w;
            return HJB_OK;
        }
    }
    const int64_t N = hd->N;
    const int dim = hd->dim;
    hipStream_t s = hd->stream;
    HIPCHK(hipStreamSynchronize(s));
    // synthetic data: zero fields, a policy of 8-node patches cycling through the controls
    std::vector<int16_t> pol((size_t)N);
    const hjb_desc &d = hd->desc;
    for (int64_t i = 0; i < N; ++i) {
        int ix = (int)(i % d.n[0]), r = (int)(i / d.n[0]);
        int iy = dim > 1 ? r % d.n[1] : 0, iz = dim > 2 ? r / d.n[1] : 0;
        bool bd = ix == 0 || ix == d.n[0] - 1 || iy == 0 || iy == d.n[1] - 1 ||
                  (dim == 3 && (iz == 0 || iz == d.n[2] - 1));
        pol[(size_t)i] = bd ? -1 : (int16_t)((ix / 8 + 3 * (iy / 8) + 5 * (iz / 8)) % d.K);
    }
    HIPCHK(hipMemcpy(hd->a0, pol.data(), (size_t)N * 2, hipMemcpyHostToDevice));
    launch_zero(hd->Ua, (size_t)N * 8, s);
    launch_zero(hd->Uc, (size_t)N * 8, s);
    launch_zero(hd->E, (size_t)N * 8, s);
    launch_zero(hd->R, (size_t)N * 8, s);
    launch_zero(hd->Vb, (size_t)N * 8, s);
    launch_zero(hd->Zb, (size_t)N * 8, s);
    const double dt = 1.0 / 64, theta_dt = dt;
    const bool zf = mixed(hd) && hd->desc.precond != HJB_PRECOND_NONE && hd->desc.precond != HJB_PRECOND_AMG;
    hipEvent_t ev[4];
    for (hipEvent_t &e : ev) HIPCHK(hipEventCreate(&e));
    double best = INFINITY;
    int best_tl = hd->tlog;
    std::vector<std::pair<int, double>> costs;
    int rc = HJB_OK;
    for (int tl = kTileLogMin; tl <= kTileLogMax && rc == HJB_OK; ++tl) {
        apply_tiles(hd, tl);
        TRY(prepare_mg(hd, hd->a0, theta_dt));
        // weights: searches and Krylov iterations (one apply and one V-cycle each) per time step of the
        // Crank-Nicolson benchmark march
        const int ns = 2, na = 5;
        for (int rep = 0; rep < 2; ++rep) {  // the first pass warms caches and code
            HIPCHK(hipEventRecord(ev[0], s));
            for (int q = 0; q < ns; ++q)
                TRY(sweep(hd, hd->Ua, hd->Uc, hd->E, hd->R, 0.0, dt, 1.0, hd->a0, hd->a1, nullptr, nullptr, nullptr,
                          nullptr, nullptr, 0));
            HIPCHK(hipEventRecord(ev[1], s));
            for (int q = 0; q < na; ++q)
                launch_apply(dim, hd->lev[0].g, stencil(hd, 0), hd->a0, hd->Zb, zf, hd->Vb + N, theta_dt, nullptr,
                             hd->nb, s);
            HIPCHK(hipEventRecord(ev[2], s));
            if (hd->desc.precond != HJB_PRECOND_NONE)
                for (int q = 0; q < na; ++q) precondition_eager(hd, hd->Vb, hd->Zb, theta_dt, false);
            HIPCHK(hipEventRecord(ev[3], s));
        }
        HIPCHK(hipEventSynchronize(ev[3]));
        float t_sw = 0, t_ap = 0, t_vc = 0;
        HIPCHK(hipEventElapsedTime(&t_sw, ev[0], ev[1]));
        HIPCHK(hipEventElapsedTime(&t_ap, ev[1], ev[2]));
        HIPCHK(hipEventElapsedTime(&t_vc, ev[2], ev[3]));
        double cost = 9.5 * t_sw / ns + 45.0 * (t_ap + t_vc) / na;
        costs.push_back({1 << tl, cost});
        if (cost < best) {
            best = cost;
            best_tl = tl;
        }
    }
    for (hipEvent_t &e : ev) (void)hipEventDestroy(e);
    apply_tiles(hd, best_tl);
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"key\": \"%s\", \"tile_width\": %d, \"cost_ms\": {", key.c_str(), 1 << best_tl);
            for (size_t q = 0; q < costs.size(); ++q)
                fprintf(f, "%s\"%d\": %.4f", q ? ", " : "", costs[q].first, costs[q].second);
            fprintf(f, "}}\n");
            fclose(f);
        }
    }
    if (tile_width_out) *tile_width_out = 1 << best_tl;
    if (cost_ms_out)
        for (size_t q = 0; q < costs.size(); ++q) cost_ms_out[q] = costs[q].second;
    return HJB_OK;
}

}  // extern "C"

// ---- adjoint ------------------------------------------------------------------------------------

namespace {

// the largest tile count of a level over the tile shapes the handle may take
int tiles_cap(const LevelDev &g0, int dim) {
    int cap = 0;
    for (int tl = kTileLogMin; tl <= kTileLogMax; ++tl) {
        LevelDev g = g0;
        g.tlog = tl;
        set_tiles(g, dim);
        cap = std::max(cap, tiles_for(g));
    }
    return cap;
}

struct TransposeWork {
    int E = 0;
    TransposeBuf b{};
    int32_t *tset = nullptr, *wset = nullptr;  // [5 tiles] window control sets (constant coefficients)
    bool wf = false;                           // wset holds the current policy's windows
    std::vector<void *> mem;
    TransposeWork() = default;
    TransposeWork(const TransposeWork &) = delete;
    TransposeWork &operator=(const TransposeWork &) = delete;
    ~TransposeWork() {
        for (void *p : mem) (void)hipFree(p);
    }
    TransposeView view() const {
        return TransposeView{b.colptr, b.rows_s,   b.vals_s,     b.ell_w,   b.ell_off,
                             b.ell_rows, b.ell_vals, b.ell_vals32, b.ell_d16, wf ? wset : nullptr};
    }
    int alloc(hjb_handle *hd, int level, bool f32, bool pack) {
        const LevelDev &g = hd->lev[level].g;
        const int64_t nodes = g.N;
        E = hd->npt * (1 << hd->dim) + 1;
        int64_t n = nodes * (int64_t)E;
        const int64_t ns = ell_slices(g);
        const int64_t ne = ns * 64 * kEllCap;  // ELL entries at most
        if (n >= ((int64_t)1 << 31) || ne >= ((int64_t)1 << 31))
            return fail(HJB_EUNSUPPORTED, "transposed operator too large (%lld entries)", (long long)n);
        b.scratch_bytes = transpose_scratch_bytes(n, (int)nodes, (int)ns);
        struct R {
            void **p;
            size_t bytes;
        } req[] = {{(void **)&b.cols, (size_t)n * 4},
                   {(void **)&b.cols_s, (size_t)nodes * 4}, {(void **)&b.ids_s, (size_t)n * 4},
                   {(void **)&b.rows_s, (size_t)n * 4}, {(void **)&b.vals, (size_t)n * 8},
                   {(void **)&b.vals_s, (size_t)n * 8}, {(void **)&b.colptr, (size_t)(nodes + 1) * 4},
                   {(void **)&b.ell_w, (size_t)ns * 4}, {(void **)&b.ell_off, (size_t)ns * 4},
                   {(void **)&b.ell_rows, (size_t)ne * 4}, {(void **)&b.ell_vals, (size_t)ne * 8},
                   {&b.scratch, b.scratch_bytes + 256}, {(void **)&tset, (size_t)tiles_cap(g, hd->dim) * 4 * (1 + kWinMax)},
                   {(void **)&wset, (size_t)tiles_cap(g, hd->dim) * 4 * (1 + kWinMax)}};
        for (auto &r : req) {
            if (hipMalloc(r.p, r.bytes) != hipSuccess) {
                (void)hipGetLastError();
                return fail(HJB_ENOMEM, "adjoint workspace (%zu bytes)", r.bytes);
            }
            mem.push_back(*r.p);
        }
        b.ell_vals32 = nullptr;
        b.ell_d16 = nullptr;
        if (f32) {
            if (hipMalloc((void **)&b.ell_vals32, (size_t)ne * 4) != hipSuccess) {
                (void)hipGetLastError();
                return fail(HJB_ENOMEM, "adjoint workspace (FP32 weights)");
            }
            mem.push_back(b.ell_vals32);
        }
        if (pack) {
            if (hipMalloc((void **)&b.ell_d16, (size_t)ne * 2) != hipSuccess) {
                (void)hipGetLastError();
                return fail(HJB_ENOMEM, "adjoint workspace (packed rows)");
            }
            mem.push_back(b.ell_d16);
        }
        return HJB_OK;
    }
    int build(hjb_handle *hd, int level, const int16_t *alpha) {
        const LevelDev &g = hd->lev[level].g;
        if (build_transpose(hd->dim, g, stencil(hd, level), alpha, E, b, hd->stream) != 0)
            return fail(HJB_EDEVICE, "column sort of the transposed operator failed");
        HIPCHK(hipGetLastError());
        if (hd->trace) {  // padding of the sliced ELL copy
            const int64_t ns = ell_slices(g);
            int32_t last[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(&last[0], b.ell_off + ns - 1, 4, hipMemcpyDeviceToHost, hd->stream));
            HIPCHK(hipMemcpyAsync(&last[1], b.ell_w + ns - 1, 4, hipMemcpyDeviceToHost, hd->stream));
            int32_t nnz = 0;
            HIPCHK(hipMemcpyAsync(&nnz, b.colptr + g.N, 4, hipMemcpyDeviceToHost, hd->stream));
            HIPCHK(hipStreamSynchronize(hd->stream));
            fprintf(stderr, "[slhjb] level %d transposed operator: %d entries, ELL slots %lld (%.2f per entry)\n", level,
                    nnz, (long long)(last[0] + last[1]) * 64, (double)(last[0] + last[1]) * 64.0 / std::max(1, nnz));
        }
        return HJB_OK;
    }
};

// Transposed operators of every multigrid level for one policy (coarse policies injected as in the
// forward V-cycle), with FP64 Jacobi diagonals (diag(A^T) = diag(A)).
struct TransposeHierarchy {
    std::vector<std::unique_ptr<TransposeWork>> lev;
    bool f32 = false;
    // all_levels: V-cycle preconditioner; f32: FP32 copies for the mixed mode; pack: 2D int8 row offsets
    int alloc(hjb_handle *hd, bool all_levels, bool f32_, bool pack) {
        f32 = f32_;
        size_t nl = all_levels ? hd->lev.size() : 1;
        for (size_t l = 0; l < nl; ++l) {
            lev.emplace_back(new TransposeWork());
            TRY(lev.back()->alloc(hd, (int)l, f32, pack));
        }
        return HJB_OK;
    }
    int build(hjb_handle *hd, const int16_t *alpha, double theta_dt) {
        hipStream_t s = hd->stream;
        // the level policies change: the forward kernels' per-policy tables no longer apply
        for (Level &L : hd->lev) L.wctl_ok = false;
        hd->lev[0].alpha = const_cast<int16_t *>(alpha);
        for (size_t l = 1; l < lev.size(); ++l)
            launch_inject_policy(hd->dim, hd->lev[l - 1].g, hd->lev[l].g, hd->lev[l - 1].alpha, hd->lev[l].alpha, s);
        for (size_t l = 0; l < lev.size(); ++l) {
            Level &L = hd->lev[l];
            launch_diag<double>(hd->dim, L.g, stencil(hd, (int)l), L.alpha, theta_dt, (double *)L.d64, s);
            if (f32) launch_diag<float>(hd->dim, L.g, stencil(hd, (int)l), L.alpha, theta_dt, (float *)L.d32, s);
            TRY(lev[l]->build(hd, (int)l, L.alpha));
            // columns whose stencil window holds few untruncated controls are gathered matrix-free
            lev[l]->wf = hd->desc.coef_model == HJB_COEF_CONST && !hd->desc.f_per_control;
            if (lev[l]->wf) {
                launch_tile_set(hd->dim, L.g, L.alpha, hd->desc.K, lev[l]->tset, s);
                launch_window_set(hd->dim, L.g, lev[l]->tset, lev[l]->wset, L.reach, s);
            }
        }
        return HJB_OK;
    }
};

template <typename T>
void smooth_T(hjb_handle *hd, const TransposeHierarchy &H, int l, T *&e, T *&t, const T *r, int sweeps, bool first,
              double theta_dt) {
    Level &L = hd->lev[l];
    for (int q = 0; q < sweeps; ++q) {
        if constexpr (std::is_same<T, float>::value)
            launch_jacobi_T32(hd->dim, first && q == 0, L.g, stencil(hd, l), L.alpha, H.lev[l]->view(), e, r,
                              (const float *)L.d32, theta_dt, hd->desc.omega, t, hd->stream);
        else
            launch_jacobi_T(hd->dim, first && q == 0, L.g, stencil(hd, l), L.alpha, H.lev[l]->view(), e, r,
                            (const double *)L.d64, theta_dt, hd->desc.omega, t, hd->stream);
        std::swap(e, t);
    }
}

// z = V-cycle for A^T z = v: the forward cycle's transfers and sweep counts, with damped Jacobi on the
// transposed level operators and sweeps on the coarsest level.  T = float in the mixed mode.
template <typename T>
void vcycle_T(hjb_handle *hd, const TransposeHierarchy &H, const T *r0, T *z, double theta_dt) {
    constexpr bool F = std::is_same<T, float>::value;
    const int Lc = (int)H.lev.size() - 1;
    const hjb_desc &d = hd->desc;
    hipStream_t s = hd->stream;
    std::vector<T *> e(Lc + 1), t(Lc + 1);
    std::vector<const T *> r(Lc + 1);
    for (int l = 0; l <= Lc; ++l) {
        e[l] = (T *)(F ? hd->lev[l].e32 : hd->lev[l].e64);
        t[l] = (T *)(F ? hd->lev[l].t32 : hd->lev[l].t64);
        r[l] = (const T *)(F ? hd->lev[l].r32 : hd->lev[l].r64);
    }
    r[0] = r0;
    int flips0 = Lc == 0 ? d.coarse_sweeps : hd->nu_pre + hd->nu_post;
    if (flips0 % 2 == 0) {
        e[0] = z;
    } else {
        e[0] = (T *)(F ? hd->lev[0].t32 : hd->lev[0].t64);
        t[0] = z;
    }
    if (Lc == 0) {
        smooth_T<T>(hd, H, 0, e[0], t[0], r[0], d.coarse_sweeps, true, theta_dt);
        return;
    }
    for (int l = 0; l < Lc; ++l) {
        Level &L = hd->lev[l];
        smooth_T<T>(hd, H, l, e[l], t[l], r[l], hd->nu_pre, true, theta_dt);
        if constexpr (F)
            launch_resid_T32(hd->dim, L.g, stencil(hd, l), L.alpha, H.lev[l]->view(), e[l], r[l], theta_dt, t[l], s);
        else
            launch_apply_T(hd->dim, 3, L.g, stencil(hd, l), L.alpha, H.lev[l]->view(), e[l], r[l], theta_dt, t[l],
                           nullptr, s);
        launch_restrict<T>(hd->dim, L.g, hd->lev[l + 1].g, t[l], (T *)(F ? hd->lev[l + 1].r32 : hd->lev[l + 1].r64), s);
    }
    // the transposed cycle's coarsest level takes its own sweep count: more sweeps there did not lower
    // the adjoint's Krylov count on the benchmark workloads
    smooth_T<T>(hd, H, Lc, e[Lc], t[Lc], r[Lc], d.coarse_sweeps_t > 0 ? d.coarse_sweeps_t : d.coarse_sweeps, true,
                theta_dt);
    for (int l = Lc - 1; l >= 0; --l) {
        launch_prolong_add<T>(hd->dim, hd->lev[l].g, hd->lev[l + 1].g, e[l + 1], e[l], s);
        smooth_T<T>(hd, H, l, e[l], t[l], r[l], hd->nu_post, false, theta_dt);
    }
}

// Solve A_alpha^T mu = b (interior) with FGMRES preconditioned by the transposed V-cycle (or Jacobi,
// following the handle's preconditioner option), starting from the given mu.
int solve_transposed(hjb_handle *hd, TransposeHierarchy &H, const int16_t *alpha, const double *b, double *mu,
                     double theta_dt, int *its, double *res) {
    const int dim = hd->dim;
    const Level &L0 = hd->lev[0];
    const StencilDev st = stencil(hd, 0);
    hipStream_t s = hd->stream;
    const TransposeView T0 = H.lev[0]->view();
    KrylovOp op;
    op.residual = [=]() {
        launch_apply_T(dim, 2, L0.g, st, alpha, T0, mu, b, theta_dt, hd->R, hd->partial, s);
    };
    op.apply = [=](const void *z, bool zf, double *w) {
        if (zf)
            launch_apply_T_f32x(dim, L0.g, st, alpha, T0, (const float *)z, theta_dt, w, s);
        else
            launch_apply_T(dim, 0, L0.g, st, alpha, T0, (const double *)z, nullptr, theta_dt, w, nullptr, s);
    };
    op.zf = false;
    if (hd->desc.precond == HJB_PRECOND_VCYCLE && H.f32) {
        op.precond = [=, &H](const double *v, void *z, bool ready) {
            if (!ready) launch_to_precond(v, L0.r32, true, hd->N, s);
            vcycle_T<float>(hd, H, (const float *)L0.r32, (float *)z, theta_dt);
            return HJB_OK;
        };
        op.zf = true;
        op.rhs32 = (float *)L0.r32;
    } else if (hd->desc.precond == HJB_PRECOND_VCYCLE) {
        op.precond = [=, &H](const double *v, void *z, bool) {
            vcycle_T<double>(hd, H, v, (double *)z, theta_dt);
            return HJB_OK;
        };
    } else if (hd->desc.precond == HJB_PRECOND_JACOBI) {
        op.precond = [=](const double *v, void *z, bool) {
            hipLaunchKernelGGL(k_jacobi_precond64, dim3(blocks_for(hd->N)), dim3(kBlock), 0, s, v,
                               (const double *)L0.d64, (double *)z, hd->N);
            return HJB_OK;
        };
    }
    bool tight = false;
    set_sweeps(hd, true);
    return krylov_core(hd, op, mu, 0.0, its, res, &tight);
}

}  // namespace

extern "C" {

int hjb_apply_transposed(hjb_handle *hd, const int16_t *alpha, const double *x, double *y, double dt, double theta,
                         double s) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!alpha || !x || !y) return fail(HJB_EINVAL, "null array argument");
    if (x == y) return fail(HJB_EINVAL, "x and y must be distinct");
    TRY(check_time(dt, theta));
    TRY(build_tables(hd, s));
    TRY(check_policy(hd, alpha));
    TransposeWork T;
    TRY(T.alloc(hd, 0, false, false));
    TRY(T.build(hd, 0, alpha));
    // the same column gathers as the adjoint's transposed solves: matrix-free where the stencil window of a
    // tile holds few untruncated controls (constant coefficients), the sorted listing elsewhere
    T.wf = hd->desc.coef_model == HJB_COEF_CONST && !hd->desc.f_per_control;
    if (T.wf) {
        launch_tile_set(hd->dim, hd->lev[0].g, alpha, hd->desc.K, T.tset, hd->stream);
        launch_window_set(hd->dim, hd->lev[0].g, T.tset, T.wset, hd->lev[0].reach, hd->stream);
    }
    launch_apply_T(hd->dim, 0, hd->lev[0].g, stencil(hd, 0), alpha, T.view(), x, nullptr, theta * dt, y, nullptr,
                   hd->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(hd->stream));
    return HJB_OK;
}

int hjb_adjoint(hjb_handle *hd, const double *g, const double *psi, const double *f0, const double *f1, int32_t n_steps,
                const double *dts, const double *thetas, double s, const int16_t *policies, const double *values,
                const double *dJ_dUN, double *dJ_df0, double *dJ_df1, double *dJ_dg, double *dJ_ds,
                hjb_adjoint_stats *stats) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (!g || !psi || !f0 || !f1 || !dts || !thetas || !policies || !dJ_dUN || !dJ_df0 || !dJ_dg)
        return fail(HJB_EINVAL, "null argument");
    if (n_steps < 1) return fail(HJB_EINVAL, "n_steps must be >= 1");
    for (int n = 0; n < n_steps; ++n) {
        TRY(check_time(dts[n], thetas[n]));
        if (thetas[n] == 0.0) return fail(HJB_EUNSUPPORTED, "explicit steps (theta = 0) are not provided");
    }
    if (hd->desc.f_per_control) return fail(HJB_EUNSUPPORTED, "the adjoint takes one source for all controls");
    if (hd->desc.precond == HJB_PRECOND_AMG)
        return fail(HJB_EUNSUPPORTED, "the aggregation preconditioner serves forward solves only");
    TRY(build_tables(hd, s));
    const int64_t N = hd->N;
    const int dim = hd->dim;
    const LevelDev &g0 = hd->lev[0].g;
    hipStream_t str = hd->stream;
    for (int n = 0; n < n_steps; ++n) TRY(check_policy(hd, policies + (int64_t)n * N));
    hjb_adjoint_stats loc{};
    double *lam = nullptr, *mu = nullptr;
    struct Free {
        std::vector<void *> p;
        ~Free() {
            for (void *q : p) (void)hipFree(q);
        }
    } fr;
    auto get = [&](double **p, size_t bytes) -> int {
        if (hipMalloc((void **)p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HJB_ENOMEM, "adjoint storage (%zu bytes)", bytes);
        }
        fr.p.push_back(*p);
        return HJB_OK;
    };
    TRY(get(&lam, (size_t)N * 8));
    TRY(get(&mu, (size_t)N * 8));
    std::vector<double> tprev(n_steps);
    {
        double t = 0.0;
        for (int n = 0; n < n_steps; ++n) {
            tprev[n] = t;
            t = t + dts[n];
        }
    }
    // Values U^n enter only the s-derivative.  Given `values`, they are read from there.  Otherwise (with
    // dJ_ds) they are recomputed from g and the int16 policies by fixed-policy solves: a forward pass keeps
    // every seg-th value (seg = ceil(sqrt(n_steps))), and the backward sweep recomputes one segment of at most
    // seg + 1 values from its checkpoint before stepping through it: 2 n_steps solves and about
    // 2 sqrt(n_steps) + 1 FP64 arrays instead of n_steps + 1.  With values holding every k-th level
    // (value_stride = k > 1) those are the checkpoints and only the backward recomputation remains.
    const bool need_values = dJ_ds != nullptr;
    const int stride = hd->desc.value_stride;
    const bool all_values = values && stride == 1;
    const int seg = (all_values || !need_values) ? n_steps
                    : values ? stride : std::max(1, (int)ceil(sqrt((double)n_steps)));
    double *ck = nullptr, *sb = nullptr;  // checkpoints U^{k seg}, segment buffer U^{n0} .. U^{n0 + seg}
    int seg_n0 = -1;                      // first step of the segment in sb
    // U^n by a fixed-policy solve from U^{n-1}, started from the linear extrapolation of U^{n-2}, U^{n-1}
    auto recompute = [&](int n, const double *Up, const double *Upp, double *Un) -> int {
        HIPCHK(hipMemcpyAsync(Un, psi, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
        if (Upp)
            launch_extrapolate(dim, g0, Up, Upp, dts[n] / dts[n - 1], Un, str);
        else
            launch_copy_interior(dim, g0, Up, Un, str);
        int its = 0;
        double res = 0.0;
        bool tight = false;
        int rc = linsolve_impl(hd, policies + (int64_t)n * N, Up, f0, f1, tprev[n], dts[n], thetas[n], Un, 0.0, &its,
                               &res, &tight);
        loc.krylov_recompute += its;
        return rc;
    };
    if (!values && need_values) {
        const int ncp = (n_steps + seg - 1) / seg;
        TRY(get(&ck, (size_t)ncp * N * 8));
        TRY(get(&sb, (size_t)(seg + 1) * N * 8));
        HIPCHK(hipMemcpyAsync(ck, g, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
        const double *Up = g, *Upp = nullptr;  // three buffers of sb rotate (seg >= 2 here)
        for (int n = 0; n + 1 < (ncp - 1) * seg + 1; ++n) {
            double *Un = sb + (int64_t)(n % 3) * N;
            TRY(recompute(n, Up, Upp, Un));
            if ((n + 1) % seg == 0)
                HIPCHK(hipMemcpyAsync(ck + (int64_t)((n + 1) / seg) * N, Un, (size_t)N * 8, hipMemcpyDeviceToDevice,
                                      str));
            Upp = Up;
            Up = Un;
        }
    }
    if (values && !all_values && need_values) {
        ck = const_cast<double *>(values);  // read only
        TRY(get(&sb, (size_t)(std::min(seg, n_steps) + 1) * N * 8));
    }
    // U^m for a step n of the backward sweep (m = n or n + 1)
    auto U_at = [&](int n, int m, const double **out) -> int {
        if (all_values) {
            *out = values + (int64_t)m * N;
            return HJB_OK;
        }
        const int n0 = (n / seg) * seg;
        if (n0 != seg_n0) {
            const int n1 = std::min(n0 + seg, n_steps);
            HIPCHK(hipMemcpyAsync(sb, ck + (int64_t)(n0 / seg) * N, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
            for (int q = n0; q < n1; ++q)
                TRY(recompute(q, sb + (int64_t)(q - n0) * N, q > n0 ? sb + (int64_t)(q - n0 - 1) * N : nullptr,
                              sb + (int64_t)(q - n0 + 1) * N));
            seg_n0 = n0;
        }
        *out = sb + (int64_t)(m - n0) * N;
        return HJB_OK;
    };
    TransposeHierarchy TH;
    {
        // int8 row offsets need every stencil point within 127 cells (2D)
        double reach = 0.0, xmax = 1.0;
        const double sr = s / sqrt(hd->desc.h);
        if (hd->desc.coef_model == HJB_COEF_XSCALED) {
            xmax = 0.0;
            for (int a = 0; a < dim; ++a)
                xmax = std::max(xmax, std::max(fabs(hd->desc.lo[a]),
                                               fabs(hd->desc.lo[a] + (hd->desc.n[a] - 1) * hd->desc.h)));
        }
        for (double v : hd->sigma) reach = std::max(reach, fabs(sr * v) * xmax);
        for (double v : hd->drift) reach = std::max(reach, fabs(v) * xmax);
        const bool vc = hd->desc.precond == HJB_PRECOND_VCYCLE;
        const bool f32 = vc && mixed(hd);
        TRY(TH.alloc(hd, vc, f32, f32 && dim == 2 && reach + 2.0 <= 127.0));
    }
    launch_mask_interior(dim, g0, dJ_dUN, lam, str);
    launch_zero(mu, (size_t)N * 8, str);  // mu_{n+1} is the initial guess of mu_n
    launch_zero(dJ_df0, (size_t)N * 8, str);
    if (dJ_df1) launch_zero(dJ_df1, (size_t)N * 8, str);
    double ds = 0.0;
    const double inv_s = 1.0 / s;
    for (int n = n_steps - 1; n >= 0; --n) {
        const int16_t *alpha = policies + (int64_t)n * N;
        const double dt = dts[n], th = thetas[n];
        const double t_mid = tprev[n] + th * dt;
        TRY(TH.build(hd, alpha, th * dt));
        int its = 0;
        double res = 0.0;
        int rc = solve_transposed(hd, TH, alpha, lam, mu, th * dt, &its, &res);
        loc.krylov_adjoint += its;
        loc.max_res_adjoint = std::max(loc.max_res_adjoint, res);
        if (rc != HJB_OK) return rc;
        launch_axpy_interior(dim, g0, dt, mu, dJ_df0, str);
        if (dJ_df1) launch_axpy_interior(dim, g0, dt * t_mid, mu, dJ_df1, str);
        if (dJ_ds) {
            const double *Un = nullptr, *Up = nullptr;
            TRY(U_at(n, n + 1, &Un));
            TRY(U_at(n, n, &Up));
            launch_ds_dot(dim, g0, stencil(hd, 0), alpha, mu, Un, th, Up, 1.0 - th, inv_s, hd->partial, str);
            launch_reduce_sum(hd->partial, 1, hd->nb, hd->dvals + 200, str);
            TRY(sync_small(hd, hd->dvals + 200, hd->hpin + 200, sizeof(double)));
            ds += dt * hd->hpin[200];
        }
        // lambda_{n-1} = B_n^T mu_n on every node
        launch_apply_T(dim, 1, g0, stencil(hd, 0), alpha, TH.lev[0]->view(), mu, nullptr, (1.0 - th) * dt,
                       n > 0 ? lam : dJ_dg, nullptr, str);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(str));
    if (dJ_ds) *dJ_ds = ds;
    if (stats) *stats = loc;
    return HJB_OK;
}

int hjb_coarse_operator(hjb_handle *hd, int32_t level, int32_t *width, int64_t *nodes, int32_t *cols, double *vals) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (level < 1 || level >= (int)hd->lev.size() || !hd->lev[level].gcol)
        return fail(HJB_EINVAL, "level %d has no Galerkin operator", (int)level);
    const Level &L = hd->lev[level];
    if (width) *width = kGalWidth;
    if (nodes) *nodes = L.g.N;
    const size_t n = (size_t)L.g.N * kGalWidth;
    if (cols) HIPCHK(hipMemcpyAsync(cols, L.gcol, n * 4, hipMemcpyDeviceToDevice, hd->stream));
    if (vals) HIPCHK(hipMemcpyAsync(vals, L.gval, n * 8, hipMemcpyDeviceToDevice, hd->stream));
    HIPCHK(hipStreamSynchronize(hd->stream));
    return HJB_OK;
}

int hjb_amg_level(hjb_handle *hd, int32_t level, int32_t *levels, int64_t *rows, int32_t *width, int32_t *agg,
                  int32_t *cols, double *vals) {
    if (!hd) return fail(HJB_EINVAL, "null handle");
    if (levels) *levels = hd->amg_levels;
    if (hd->amg_levels == 0) return fail(HJB_EINVAL, "no aggregation hierarchy has been built");
    if (level < 0 || level >= hd->amg_levels) return fail(HJB_EINVAL, "level %d of %d", (int)level, hd->amg_levels);
    const AmgLevel &L = hd->amg[level];
    if (rows) *rows = L.n;
    if (width) *width = L.W;
    if (agg && level >= 1)
        HIPCHK(hipMemcpyAsync(agg, L.agg.p, (size_t)hd->amg[level - 1].n * 4, hipMemcpyDeviceToDevice, hd->stream));
    // a row's entries fill its first W slots: slots W.. of the buffer are not part of the level
    if (cols) HIPCHK(hipMemcpyAsync(cols, L.col.p, (size_t)L.n * L.W * 4, hipMemcpyDeviceToDevice, hd->stream));
    if (vals) HIPCHK(hipMemcpyAsync(vals, L.val.p, (size_t)L.n * L.W * 8, hipMemcpyDeviceToDevice, hd->stream));
    HIPCHK(hipStreamSynchronize(hd->stream));
    return HJB_OK;
}

void hjb_destroy(hjb_handle *hd) {
    if (!hd) return;
    drop_graphs(hd);
    if (hd->capture_stream) (void)hipStreamDestroy(hd->capture_stream);
    for (auto &T : hd->timers)
        for (hipEvent_t e : T.ev) (void)hipEventDestroy(e);
    if (hd->stream) (void)hipStreamSynchronize(hd->stream);
    else (void)hipDeviceSynchronize();
    for (void *p : hd->allocs) (void)hipFree(p);
    for (AmgLevel &L : hd->amg)
        for (DevBuf *b : {&L.col, &L.val, &L.d, &L.agg, &L.mem4, &L.inv, &L.rcol, &L.rval, &L.x, &L.r, &L.t, &L.v1,
                          &L.w1, &L.v2, &L.w2, &L.r1})
            release(*b);
    for (DevBuf *b : {&hd->amg_rawc, &hd->amg_rawv, &hd->amg_mate, &hd->amg_cand, &hd->amg_flag, &hd->amg_id,
                      &hd->amg_part, &hd->amg_aggA, &hd->amg_aggB, &hd->amg_mem2a, &hd->amg_mem2b, &hd->amg_icol,
                      &hd->amg_ival, &hd->amg_words, &hd->amg_dpart, &hd->amg_sc, &hd->amg_trow, &hd->amg_tval,
                      &hd->amg_scol, &hd->amg_sval})
        release(*b);
    if (hd->hpin) (void)hipHostFree(hd->hpin);
    if (hd->hpin_i) (void)hipHostFree(hd->hpin_i);
    if (hd->hflag) (void)hipHostFree(hd->hflag);
    delete hd;
}

}  // extern "C"

// =====================================================================================================
// Batches of independent instances
// =====================================================================================================
//
// Instances keep their own grids, coefficient tables and multigrid depths (set up as tables-only
// handles); their arrays are concatenated per level.  Every launch covers all instances that take
// part (per-level tile tables, per-instance flags), and the per-instance scalars of policy iteration
// and FGMRES (Hessenberg matrices, rotations, convergence) are advanced in lockstep on the host.

namespace {

struct TileTab {
    int32_t n = 0;
    int32_t *inst = nullptr, *tile = nullptr, *first_dev = nullptr;
    std::vector<int32_t> first;  // [B+1] entry range of each instance
};

struct BLevel {
    std::vector<int64_t> off;      // [B] start of each instance's array, -1 without this level
    int64_t total = 0;
    BInst *I = nullptr;            // device [B]
    std::vector<BInst> Ih;
    TileTab all;                   // instances that have this level
    TileTab fine;                  // instances with a coarser level below this one
    TileTab csm;                   // coarsest here but too large for the one-workgroup solve
    std::vector<int32_t> lds;      // coarsest here, solved by one workgroup in LDS
    int32_t *lds_dev = nullptr;
    int64_t lds_maxN = 0;
    int16_t *alpha = nullptr;      // injected policy (levels >= 1)
    void *r64 = nullptr, *e64 = nullptr, *t64 = nullptr, *d64 = nullptr;
    void *r32 = nullptr, *e32 = nullptr, *t32 = nullptr, *d32 = nullptr;
};

}  // namespace

struct hjb_batch {
    int B = 0, dim = 2;
    hjb_desc opt{};                 // solver options (from the first descriptor)
    std::vector<hjb_handle *> sub;  // per instance: level geometry and stencil tables
    std::vector<int> nlev;
    hipStream_t stream = nullptr;
    std::vector<BLevel> lev;
    int64_t N = 0;                  // level-0 nodes of all instances
    double *E = nullptr, *R = nullptr, *Vb = nullptr, *Zb = nullptr, *Ua = nullptr, *Ub = nullptr, *Uc = nullptr;
    int16_t *a0 = nullptr, *a1 = nullptr, *acarry = nullptr;
    double *partial = nullptr;
    int64_t *ipartial = nullptr;
    double *dseg = nullptr, *dtau = nullptr, *dcoefA = nullptr, *dcoef = nullptr, *dy = nullptr;
    int64_t *dchg = nullptr;
    int32_t *dm = nullptr;
    uint8_t *dmask[4] = {nullptr, nullptr, nullptr, nullptr};  // step, solve, Arnoldi cycle, second pass / changed
    double *hseg = nullptr, *hcoef = nullptr, *hy = nullptr;
    int64_t *hchg = nullptr;
    int32_t *hm = nullptr;
    uint8_t *hmask[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<void *> allocs, pinned;
    struct VGraph {
        const void *a0, *v, *z;
        double theta_dt;
        hipGraphExec_t exec;
    };
    std::vector<VGraph> vgraphs;    // captured batched V-cycles (masks are read from fixed buffers)
    hipStream_t capture_stream = nullptr;
    // FGMRES scalars on the device (BKrylov) and the pinned host copies read once per restart cycle
    double *dH = nullptr, *dcs = nullptr, *dsn = nullptr, *dg = nullptr, *dhn = nullptr, *dtarget = nullptr;
    int32_t *dits = nullptr, *djb = nullptr, *dbad = nullptr;
    uint8_t *dnext = nullptr;       // instances that take a second Gram-Schmidt pass
    double *htarget = nullptr;
    int32_t *hits = nullptr;        // [its | bad], 2 B entries
    struct CGraph {
        const void *a0;
        int j;
        double theta_dt;
        hipGraphExec_t exec;
    };
    std::vector<CGraph> cgraphs;    // captured Arnoldi steps
    int64_t maxn_cap = 0;           // tile entries of one level the partial-sum buffers hold
};

namespace {

constexpr int kLdc = kMaxRestart + 2;  // per-instance stride of the coefficient arrays

int balloc(hjb_batch *bh, void **p, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HJB_ENOMEM, "batch workspace (%zu bytes)", bytes);
    }
    bh->allocs.push_back(*p);
    return HJB_OK;
}

int bpin(hjb_batch *bh, void **p, size_t bytes) {
    if (hipHostMalloc(p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HJB_ENOMEM, "pinned batch buffer (%zu bytes)", bytes);
    }
    bh->pinned.push_back(*p);
    return HJB_OK;
}

// tile table over the instances selected by `take`, in instance order
int build_tiletab(hjb_batch *bh, int l, const std::function<bool(int)> &take, TileTab &T) {
    std::vector<int32_t> inst, tile;
    T.first.assign(bh->B + 1, 0);
    for (int b = 0; b < bh->B; ++b) {
        T.first[b] = (int32_t)inst.size();
        if (l < bh->nlev[b] && take(b)) {
            const int nt = tiles_for(bh->sub[b]->lev[l].g);
            for (int t = 0; t < nt; ++t) {
                inst.push_back(b);
                tile.push_back(t);
            }
        }
    }
    T.first[bh->B] = (int32_t)inst.size();
    T.n = (int32_t)inst.size();
    TRY(balloc(bh, (void **)&T.inst, std::max<size_t>(1, inst.size()) * 4));
    TRY(balloc(bh, (void **)&T.tile, std::max<size_t>(1, tile.size()) * 4));
    TRY(balloc(bh, (void **)&T.first_dev, (size_t)(bh->B + 1) * 4));
    if (!inst.empty()) {
        HIPCHK(hipMemcpy(T.inst, inst.data(), inst.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(T.tile, tile.data(), tile.size() * 4, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(T.first_dev, T.first.data(), (size_t)(bh->B + 1) * 4, hipMemcpyHostToDevice));
    return HJB_OK;
}

BTiles btiles(const TileTab &T, const BInst *I, const uint8_t *mask) { return BTiles{T.inst, T.tile, I, mask, T.n}; }

int bwait(hjb_batch *bh) {
    HIPCHK(hipStreamSynchronize(bh->stream));
    return HJB_OK;
}

int bupload_mask(hjb_batch *bh, int k) {
    HIPCHK(hipMemcpyAsync(bh->dmask[k], bh->hmask[k], (size_t)bh->B, hipMemcpyHostToDevice, bh->stream));
    return HJB_OK;
}

// per-instance descriptors of every level for the current tables (deep boxes and s)
int brefresh(hjb_batch *bh) {
    for (size_t l = 0; l < bh->lev.size(); ++l) {
        BLevel &L = bh->lev[l];
        for (int b = 0; b < bh->B; ++b) {
            if ((int)l < bh->nlev[b]) {
                L.Ih[b].g = bh->sub[b]->lev[l].g;
                L.Ih[b].st = stencil(bh->sub[b], (int)l);
                L.Ih[b].off = L.off[b];
            }
        }
        HIPCHK(hipMemcpyAsync(L.I, L.Ih.data(), (size_t)bh->B * sizeof(BInst), hipMemcpyHostToDevice, bh->stream));
    }
    return bwait(bh);
}

void bdrop_graphs(hjb_batch *bh) {
    for (auto &g : bh->vgraphs) (void)hipGraphExecDestroy(g.exec);
    bh->vgraphs.clear();
    for (auto &g : bh->cgraphs) (void)hipGraphExecDestroy(g.exec);
    bh->cgraphs.clear();
}

// tile tables of every level for the instances' current tile shapes (after a change of tile widths): the
// launch lists, the partial-sum buffers when they must grow, the per-instance descriptors; captured graphs
// hold the old lists and are dropped
int brebuild_tiles(hjb_batch *bh) {
    int64_t maxn = 0;
    for (size_t l = 0; l < bh->lev.size(); ++l) {
        BLevel &L = bh->lev[l];
        const int li = (int)l;
        TRY(build_tiletab(bh, li, [&](int) { return true; }, L.all));
        TRY(build_tiletab(bh, li, [&](int b) { return li + 1 < bh->nlev[b]; }, L.fine));
        TRY(build_tiletab(bh, li, [&](int b) {
            return li == bh->nlev[b] - 1 && bh->sub[b]->lev[li].g.N > kCoarseMaxNodes; }, L.csm));
        maxn = std::max<int64_t>(maxn, L.all.n);
    }
    if (maxn > bh->maxn_cap) {
        TRY(balloc(bh, (void **)&bh->partial, (size_t)kLdc * maxn * 8));
        TRY(balloc(bh, (void **)&bh->ipartial, (size_t)maxn * 8));
        bh->maxn_cap = maxn;
    }
    bdrop_graphs(bh);
    return brefresh(bh);
}

// ---- batched multigrid ---------------------------------------------------------------------------

template <typename T>
void bprepare_mg(hjb_batch *bh, const int16_t *alpha0, double theta_dt, const uint8_t *mask) {
    constexpr bool F = std::is_same<T, float>::value;
    hipStream_t s = bh->stream;
    for (size_t l = 1; l < bh->lev.size(); ++l) {
        const int16_t *af = l == 1 ? alpha0 : bh->lev[l - 1].alpha;
        launch_inject_b(bh->dim, btiles(bh->lev[l].all, bh->lev[l].I, mask), bh->lev[l - 1].I, af, bh->lev[l].alpha,
                        s);
    }
    for (size_t l = 0; l < bh->lev.size(); ++l) {
        BLevel &L = bh->lev[l];
        const int16_t *al = l == 0 ? alpha0 : L.alpha;
        launch_diag_b<T>(bh->dim, btiles(L.all, L.I, mask), al, theta_dt, (T *)(F ? L.d32 : L.d64), s);
    }
}

// even number of Jacobi sweeps on the listed instances, ending in e
template <typename T>
void bsweeps_even(hjb_batch *bh, int l, const TileTab &TT, const int16_t *al, T *e, T *t, const T *r, const T *d,
                  double theta_dt, const uint8_t *mask) {
    if (TT.n == 0) return;
    const int sweeps = bh->opt.coarse_sweeps + (bh->opt.coarse_sweeps & 1);
    BTiles bt = btiles(TT, bh->lev[l].I, mask);
    for (int q = 0; q < sweeps; ++q) {
        if (q % 2 == 0)
            launch_jacobi_b<T>(bh->dim, bt, al, e, r, d, t, theta_dt, bh->opt.omega, q == 0, bh->stream);
        else
            launch_jacobi_b<T>(bh->dim, bt, al, t, r, d, e, theta_dt, bh->opt.omega, false, bh->stream);
    }
}

// z = V-cycle(r0) for every instance with mask[b] = 1 (nu1 + nu2 even: each level ends in its e buffer)
template <typename T>
void bvcycle(hjb_batch *bh, const T *r0, T *z, double theta_dt, const int16_t *alpha0, const uint8_t *mask) {
    constexpr bool F = std::is_same<T, float>::value;
    const hjb_desc &d = bh->opt;
    hipStream_t s = bh->stream;
    const int Lm = (int)bh->lev.size();
    std::vector<T *> e(Lm), t(Lm), dd(Lm);
    std::vector<const T *> r(Lm);
    std::vector<const int16_t *> al(Lm);
    for (int l = 0; l < Lm; ++l) {
        BLevel &L = bh->lev[l];
        e[l] = (T *)(F ? L.e32 : L.e64);
        t[l] = (T *)(F ? L.t32 : L.t64);
        r[l] = (const T *)(F ? L.r32 : L.r64);
        dd[l] = (T *)(F ? L.d32 : L.d64);
        al[l] = l == 0 ? alpha0 : L.alpha;
    }
    r[0] = r0;
    e[0] = z;
    auto coarse = [&](int l) {
        BLevel &L = bh->lev[l];
        launch_coarse_b<T>(bh->dim, L.lds_dev, (int)L.lds.size(), L.lds_maxN, L.I, mask, al[l], r[l], dd[l], e[l],
                           theta_dt, d.omega, d.coarse_sweeps, s);
        bsweeps_even<T>(bh, l, L.csm, al[l], e[l], t[l], r[l], dd[l], theta_dt, mask);
    };
    coarse(0);
    for (int l = 0; l + 1 < Lm; ++l) {
        BLevel &L = bh->lev[l];
        BTiles ft = btiles(L.fine, L.I, mask);
        for (int q = 0; q < d.nu1; ++q) {
            launch_jacobi_b<T>(bh->dim, ft, al[l], e[l], r[l], dd[l], t[l], theta_dt, d.omega, q == 0, s);
            std::swap(e[l], t[l]);
        }
        launch_level_residual_b<T>(bh->dim, ft, al[l], e[l], r[l], t[l], theta_dt, s);
        launch_restrict_b<T>(bh->dim, btiles(bh->lev[l + 1].all, bh->lev[l + 1].I, mask), L.I, t[l],
                             (T *)(F ? bh->lev[l + 1].r32 : bh->lev[l + 1].r64), s);
        coarse(l + 1);
    }
    for (int l = Lm - 2; l >= 0; --l) {
        BLevel &L = bh->lev[l];
        BTiles ft = btiles(L.fine, L.I, mask);
        launch_prolong_add_b<T>(bh->dim, ft, bh->lev[l + 1].I, e[l + 1], e[l], s);
        for (int q = 0; q < d.nu2; ++q) {
            launch_jacobi_b<T>(bh->dim, ft, al[l], e[l], r[l], dd[l], t[l], theta_dt, d.omega, false, s);
            std::swap(e[l], t[l]);
        }
    }
}

void bprecondition_eager(hjb_batch *bh, const double *v, void *z, double theta_dt, const int16_t *alpha,
                         const uint8_t *mask) {
    if (bh->opt.precision == HJB_PREC_MIXED) {
        launch_to_precond(v, bh->lev[0].r32, true, bh->N, bh->stream);
        bvcycle<float>(bh, (const float *)bh->lev[0].r32, (float *)z, theta_dt, alpha, mask);
    } else {
        bvcycle<double>(bh, v, (double *)z, theta_dt, alpha, mask);
    }
}

// z = V-cycle(v) for the instances flagged in mask, replayed from a graph captured once per
// (policy buffer, v, z, theta*dt); the flags, diagonals and policies are read from fixed buffers
int bprecondition(hjb_batch *bh, const double *v, void *z, double theta_dt, const int16_t *alpha, const uint8_t *mask) {
    if (!bh->opt.use_graphs) {
        bprecondition_eager(bh, v, z, theta_dt, alpha, mask);
        return HJB_OK;
    }
    for (auto &g : bh->vgraphs)
        if (g.a0 == alpha && g.v == v && g.z == z && g.theta_dt == theta_dt) {
            HIPCHK(hipGraphLaunch(g.exec, bh->stream));
            return HJB_OK;
        }
    if (bh->vgraphs.size() >= 256) {
        for (auto &g : bh->vgraphs) (void)hipGraphExecDestroy(g.exec);
        bh->vgraphs.clear();
    }
    if (!bh->capture_stream) HIPCHK(hipStreamCreateWithFlags(&bh->capture_stream, hipStreamNonBlocking));
    hipStream_t saved = bh->stream;
    bh->stream = bh->capture_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(bh->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        bprecondition_eager(bh, v, z, theta_dt, alpha, mask);
        e = hipStreamEndCapture(bh->capture_stream, &graph);
    }
    bh->stream = saved;
    if (e != hipSuccess) return fail(HJB_EDEVICE, "batched V-cycle capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HJB_EDEVICE, "batched V-cycle instantiate: %s", hipGetErrorString(e));
    bh->vgraphs.push_back({alpha, v, z, theta_dt, exec});
    HIPCHK(hipGraphLaunch(exec, bh->stream));
    return HJB_OK;
}

// ---- batched FGMRES ------------------------------------------------------------------------------

struct BSolveOut {
    std::vector<int> its;
    std::vector<double> res;
    std::vector<uint8_t> tight;
};

// Solve A_b X_b = E_b for every instance with on[b]; eta[b] as in fgmres_core.
// Arnoldi step j of every instance in the cycle mask (dmask[2]): preconditioner, operator, two Gram-Schmidt
// passes and the Givens rotation, each advancing the device-side scalars and masks (an instance that
// converges leaves the mask), so that no host decision is needed inside the step and its launch sequence
// depends only on buffer addresses, theta*dt and j.
void bstep_eager(hjb_batch *bh, const int16_t *alpha, double theta_dt, int j) {
    const hjb_desc &d = bh->opt;
    const int B = bh->B, dim = bh->dim;
    const int64_t N = bh->N;
    hipStream_t s = bh->stream;
    const bool none = d.precond == HJB_PRECOND_NONE;
    const bool zf = d.precision == HJB_PREC_MIXED && !none && d.precond == HJB_PRECOND_VCYCLE;
    const size_t zsz = zf ? 4 : 8;
    BLevel &L0 = bh->lev[0];
    const TileTab &A0 = L0.all;
    uint8_t *mC = bh->dmask[2], *mP = bh->dmask[3];
    const BKrylov K{bh->dH, bh->dcs, bh->dsn, bh->dg, bh->dhn, bh->dtarget, bh->dits, bh->djb, bh->dbad, d.restart,
                    d.max_krylov};
    double *vj = bh->Vb + (int64_t)j * N;
    double *w = bh->Vb + (int64_t)(j + 1) * N;
    void *zj = none ? (void *)vj : (void *)((char *)bh->Zb + (int64_t)j * N * zsz);
    if (!none) bprecondition_eager(bh, vj, zj, theta_dt, alpha, mC);
    launch_apply_b(dim, btiles(A0, L0.I, mC), alpha, zj, zf, w, theta_dt, s);
    launch_mask_copy_b(B, mC, mP, s);
    for (int pass = 0; pass < 2; ++pass) {
        launch_multidot_b(dim, btiles(A0, L0.I, mP), w, bh->Vb, N, j + 1, bh->partial, s);
        launch_seg_sum(bh->partial, A0.n, A0.first_dev, j + 2, mP, bh->dseg, B, s);
        launch_arnoldi_pass_b(K, B, j, pass, bh->dseg, bh->dcoef, kLdc, mP, bh->dnext, s);
        launch_multiaxpy_scale_b(dim, btiles(A0, L0.I, mP), w, bh->Vb, N, j + 1, bh->dcoef, kLdc, s);
        if (pass == 0) launch_mask_copy_b(B, bh->dnext, mP, s);
    }
    launch_givens_b(K, B, j, mC, s);
}

// the step, replayed from a captured graph per (policy buffer, theta*dt, j) unless graphs are off
int bstep_arnoldi(hjb_batch *bh, const int16_t *alpha, double theta_dt, int j) {
    if (!bh->opt.use_graphs) {
        bstep_eager(bh, alpha, theta_dt, j);
        HIPCHK(hipGetLastError());
        return HJB_OK;
    }
    for (auto &g : bh->cgraphs)
        if (g.a0 == alpha && g.j == j && g.theta_dt == theta_dt) {
            HIPCHK(hipGraphLaunch(g.exec, bh->stream));
            return HJB_OK;
        }
    if (bh->cgraphs.size() >= 256) {
        for (auto &g : bh->cgraphs) (void)hipGraphExecDestroy(g.exec);
        bh->cgraphs.clear();
    }
    if (!bh->capture_stream) HIPCHK(hipStreamCreateWithFlags(&bh->capture_stream, hipStreamNonBlocking));
    hipStream_t saved = bh->stream;
    bh->stream = bh->capture_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(bh->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        bstep_eager(bh, alpha, theta_dt, j);
        e = hipStreamEndCapture(bh->capture_stream, &graph);
    }
    bh->stream = saved;
    if (e != hipSuccess) return fail(HJB_EDEVICE, "batched Arnoldi step capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HJB_EDEVICE, "batched Arnoldi step instantiate: %s", hipGetErrorString(e));
    bh->cgraphs.push_back({alpha, j, theta_dt, exec});
    HIPCHK(hipGraphLaunch(exec, bh->stream));
    return HJB_OK;
}

// Flexible GMRES(m) of every instance with on[b], each to its own certificate: the host reads the residual
// norms, iteration counts and non-finite flags once per restart cycle and decides which instances continue,
// and the cycle mask once per Arnoldi step; the Gram-Schmidt and Givens scalars stay on the device.
int bfgmres(hjb_batch *bh, const int16_t *alpha, double *X, double theta_dt, const std::vector<uint8_t> &on,
            const std::vector<double> &eta, BSolveOut &out) {
    const hjb_desc &d = bh->opt;
    const int B = bh->B, dim = bh->dim;
    hipStream_t s = bh->stream;
    BLevel &L0 = bh->lev[0];
    const TileTab &A0 = L0.all;
    const int n0 = A0.n;
    out.its.assign(B, 0);
    out.res.assign(B, 0.0);
    out.tight.assign(B, 0);
    std::vector<double> loose(B, 0.0);
    std::vector<uint8_t> act = on;  // still solving
    uint8_t *mS = bh->dmask[1];
    uint8_t *hS = bh->hmask[1];
    const bool none = d.precond == HJB_PRECOND_NONE;
    const bool zf = d.precision == HJB_PREC_MIXED && !none && d.precond == HJB_PRECOND_VCYCLE;
    launch_zero(bh->dits, (size_t)B * 2 * 4, s);  // iteration counts and non-finite flags
    for (int cycle = 0;; ++cycle) {
        for (int b = 0; b < B; ++b) hS[b] = act[b];
        TRY(bupload_mask(bh, 1));
        launch_residual_b(dim, btiles(A0, L0.I, mS), alpha, X, bh->E, theta_dt, bh->R, bh->partial, s);
        launch_seg_sum(bh->partial, n0, A0.first_dev, 1, mS, bh->dseg, B, s);
        launch_seg_max(bh->partial + n0, n0, A0.first_dev, 2, mS, bh->dseg + B, B, s);
        HIPCHK(hipMemcpyAsync(bh->hseg, bh->dseg, (size_t)3 * B * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(bh->hits, bh->dits, (size_t)2 * B * 4, hipMemcpyDeviceToHost, s));
        TRY(bwait(bh));
        bool any = false;
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            if (bh->hits[B + b]) return fail(HJB_ENONFINITE, "non-finite Arnoldi vector (instance %d)", b);
            out.its[b] = bh->hits[b];
            double b2 = bh->hseg[b], rinf = bh->hseg[B + 2 * b], xinf = bh->hseg[B + 2 * b + 1];
            out.res[b] = rinf;
            if (!isfinite(b2) || !isfinite(xinf)) return fail(HJB_ENONFINITE, "non-finite residual (instance %d)", b);
            double target = d.rtol_inf * std::max(1.0, xinf);
            if (cycle == 0 && eta[b] > 0.0) loose[b] = eta[b] * rinf;
            out.tight[b] = rinf <= target;
            if (rinf <= std::max(target, loose[b])) {
                act[b] = 0;
                continue;
            }
            target = std::max(target, loose[b]);
            if (out.its[b] >= d.max_krylov)
                return fail(HJB_ENOCONV_KRYLOV, "FGMRES (instance %d): |r|_inf = %.3e > %.3e after %d iterations", b,
                            rinf, target, out.its[b]);
            bh->htarget[b] = target;
            any = true;
        }
        if (!any) return HJB_OK;
        for (int b = 0; b < B; ++b) hS[b] = act[b];
        TRY(bupload_mask(bh, 1));
        HIPCHK(hipMemcpyAsync(bh->dtarget, bh->htarget, (size_t)B * 8, hipMemcpyHostToDevice, s));
        // the cycle: v_0 = r / |r|_2, Arnoldi steps while any instance is still in the cycle (one host read of
        // the cycle mask per step), then y = R^{-1} g and X += Z y
        const BKrylov K{bh->dH, bh->dcs, bh->dsn, bh->dg, bh->dhn, bh->dtarget, bh->dits, bh->djb, bh->dbad,
                        d.restart, d.max_krylov};
        uint8_t *mC = bh->dmask[2], *hC = bh->hmask[2];
        launch_cycle_init_b(K, B, mS, bh->dseg, mC, s);  // dseg[b]: sum r^2 of the residual just reduced
        launch_scale_b(dim, btiles(A0, L0.I, mC), bh->Vb, bh->R, bh->dseg, 1, s);
        for (int j = 0; j < d.restart; ++j) {
            TRY(bstep_arnoldi(bh, alpha, theta_dt, j));
            HIPCHK(hipMemcpyAsync(hC, mC, (size_t)B, hipMemcpyDeviceToHost, s));
            TRY(bwait(bh));
            bool inc = false;
            for (int b = 0; b < B; ++b) inc |= hC[b] != 0;
            if (!inc) break;
        }
        launch_backsolve_b(K, B, mS, bh->dy, kMaxRestart, bh->dm, s);
        launch_update_b(dim, btiles(A0, L0.I, mS), X, none ? (const void *)bh->Vb : (const void *)bh->Zb, zf,
                        bh->N, bh->dm, bh->dy, kMaxRestart, s);
        HIPCHK(hipGetLastError());
    }
}

// search of every instance with on[b]: a_out from a_in at X (U: previous level); changed counts in hchg
int bsweep(hjb_batch *bh, const double *X, const double *U, const double *f0, const double *f1, double t_prev,
           double dt, double theta, const int16_t *a_in, int16_t *a_out, const std::vector<uint8_t> &on) {
    hipStream_t s = bh->stream;
    BLevel &L0 = bh->lev[0];
    for (int b = 0; b < bh->B; ++b) bh->hmask[0][b] = on[b];
    TRY(bupload_mask(bh, 0));
    const double t_mid = t_prev + theta * dt;
    BTiles bt = btiles(L0.all, L0.I, bh->dmask[0]);
    launch_norms_b(bh->dim, bt, X, U, f0, f1, t_mid, bh->partial, s);
    launch_tau_b(bh->partial, L0.all.n, L0.all.first_dev, bh->dcoefA, bh->opt.tau_rel, bh->dmask[0], bh->dtau, bh->B, s);
    launch_sweep_b(bh->dim, bt, X, U, f0, f1, t_mid, theta, bh->dtau, a_in, a_out, bh->ipartial, s);
    launch_seg_sum_i64(bh->ipartial, L0.all.n, L0.all.first_dev, bh->dmask[0], bh->dchg, bh->B, s);
    HIPCHK(hipMemcpyAsync(bh->hchg, bh->dchg, (size_t)bh->B * 8, hipMemcpyDeviceToHost, s));
    return bwait(bh);
}

int blinsolve(hjb_batch *bh, const int16_t *alpha, const double *U, const double *f0, const double *f1, double t_prev,
              double dt, double theta, double *X, const std::vector<uint8_t> &on, const std::vector<double> &eta,
              BSolveOut &out) {
    hipStream_t s = bh->stream;
    BLevel &L0 = bh->lev[0];
    for (int b = 0; b < bh->B; ++b) bh->hmask[0][b] = on[b];
    TRY(bupload_mask(bh, 0));
    const double theta_dt = theta * dt;
    if (bh->opt.precond == HJB_PRECOND_VCYCLE) {
        if (bh->opt.precision == HJB_PREC_MIXED)
            bprepare_mg<float>(bh, alpha, theta_dt, bh->dmask[0]);
        else
            bprepare_mg<double>(bh, alpha, theta_dt, bh->dmask[0]);
    }
    launch_explicit_b(bh->dim, btiles(L0.all, L0.I, bh->dmask[0]), alpha, U, f0, f1, t_prev + theta * dt,
                      (1.0 - theta) * dt, dt, bh->E, s);
    return bfgmres(bh, alpha, X, theta_dt, on, eta, out);
}

// one time step of every instance: policy iteration in lockstep (instances stop independently)
int bstep(hjb_batch *bh, const double *Uprev, double *Unext, const double *f0, const double *f1, double t_prev,
          double dt, double theta, const double *Uprev2, double dt_prev, std::vector<hjb_step_stats> &st) {
    const int B = bh->B;
    const hjb_desc &d = bh->opt;
    hipStream_t s = bh->stream;
    BLevel &L0 = bh->lev[0];
    st.assign(B, hjb_step_stats{});
    std::vector<uint8_t> on(B, 1);
    BTiles all0 = btiles(L0.all, L0.I, nullptr);
    if (Uprev2)
        launch_extrapolate_b(bh->dim, all0, Uprev, Uprev2, dt / dt_prev, Unext, s);
    else
        launch_copy_interior_b(bh->dim, all0, Uprev, Unext, s);
    TRY(bsweep(bh, Unext, Uprev, f0, f1, t_prev, dt, theta, bh->acarry, bh->a0, on));
    for (int b = 0; b < B; ++b) st[b].n_changed_first = bh->hchg[b];
    std::vector<uint8_t> want_tight(B, d.pi_eta <= 0.0 ? 1 : 0);
    std::vector<double> eta(B, 0.0);
    BSolveOut so;
    for (int it = 0; it < d.max_pi; ++it) {
        for (int b = 0; b < B; ++b) eta[b] = want_tight[b] ? 0.0 : d.pi_eta;
        TRY(blinsolve(bh, bh->a0, Uprev, f0, f1, t_prev, dt, theta, Unext, on, eta, so));
        for (int b = 0; b < B; ++b) {
            if (!on[b]) continue;
            st[b].pi_iters = it + 1;
            st[b].krylov_total += so.its[b];
            st[b].krylov_max = std::max(st[b].krylov_max, so.its[b]);
            st[b].res_inf = so.res[b];
            double den = 1.0 - theta * dt * bh->sub[b]->cplus;
            st[b].cert_bound = den > 0 ? so.res[b] / den : INFINITY;
        }
        TRY(bsweep(bh, Unext, Uprev, f0, f1, t_prev, dt, theta, bh->a0, bh->a1, on));
        bool any_left = false, any_changed = false;
        for (int b = 0; b < B; ++b) {
            bh->hmask[3][b] = 0;
            if (!on[b]) continue;
            if (bh->hchg[b] == 0) {
                if (so.tight[b])
                    on[b] = 0;
                else
                    want_tight[b] = 1;
            } else {
                bh->hmask[3][b] = 1;
                any_changed = true;
                want_tight[b] = d.pi_eta <= 0.0 ? 1 : 0;
            }
            any_left |= on[b] != 0;
        }
        if (any_changed) {
            TRY(bupload_mask(bh, 3));
            launch_copy_policy_b(bh->dim, btiles(L0.all, L0.I, bh->dmask[3]), bh->a1, bh->a0, s);
        }
        if (!any_left) break;
        if (it + 1 == d.max_pi) return fail(HJB_ENOCONV_PI, "policy iteration not converged after %d", it + 1);
    }
    HIPCHK(hipMemcpyAsync(bh->acarry, bh->a0, (size_t)bh->N * 2, hipMemcpyDeviceToDevice, s));
    return bwait(bh);
}

}  // namespace

extern "C" {

int hjb_setup_batch(const hjb_desc *descs, int32_t count, hjb_batch **out) {
    g_err.clear();
    if (!descs || !out) return fail(HJB_EINVAL, "null argument");
    *out = nullptr;
    if (count < 1) return fail(HJB_EINVAL, "count must be >= 1");
    const hjb_desc &d0 = descs[0];
    TRY(check_options(&d0));
    if ((d0.nu1 + d0.nu2) % 2 != 0) return fail(HJB_EUNSUPPORTED, "batched V-cycles take an even nu1 + nu2");
    if (d0.precond == HJB_PRECOND_JACOBI || d0.precond == HJB_PRECOND_AMG)
        return fail(HJB_EUNSUPPORTED, "batched solves take the V-cycle or no preconditioner");
    if (d0.krylov != HJB_KRYLOV_FGMRES) return fail(HJB_EUNSUPPORTED, "batched solves use flexible GMRES");
    for (int b = 0; b < count; ++b) {
        if (descs[b].dim != d0.dim) return fail(HJB_EINVAL, "all instances of a batch have the same dimension");
        if (descs[b].f_per_control) return fail(HJB_EUNSUPPORTED, "batched instances take one source for all controls");
    }
    hjb_batch *bh = new hjb_batch();
    auto bail = [&](int rc) {
        hjb_destroy_batch(bh);
        return rc;
    };
#define BTRY(x)                            \
    do {                                   \
        int _rc = (x);                     \
        if (_rc != HJB_OK) return bail(_rc); \
    } while (0)
    bh->B = count;
    bh->dim = d0.dim;
    bh->opt = d0;
    bh->stream = (hipStream_t)d0.stream;
    for (int b = 0; b < count; ++b) {
        hjb_desc db = descs[b];
        // solver options are the batch's
        db.precision = d0.precision;
        db.precond = d0.precond;
        db.restart = d0.restart;
        db.max_krylov = d0.max_krylov;
        db.max_pi = d0.max_pi;
        db.nu1 = d0.nu1;
        db.nu2 = d0.nu2;
        db.coarse_sweeps = d0.coarse_sweeps;
        db.min_coarse = d0.min_coarse;
        db.max_levels = d0.max_levels;
        db.omega = d0.omega;
        db.rtol_inf = d0.rtol_inf;
        db.tau_rel = d0.tau_rel;
        db.pi_eta = d0.pi_eta;
        db.use_graphs = 0;
        db.stream = d0.stream;
        hjb_handle *h = nullptr;
        int rc = setup_impl(&db, &h, true);
        if (rc != HJB_OK) {
            std::string msg = g_err;
            bail(rc);
            return fail(rc, "instance %d: %s", b, msg.c_str());
        }
        bh->sub.push_back(h);
        bh->nlev.push_back((int)h->lev.size());
    }
    const int Lm = *std::max_element(bh->nlev.begin(), bh->nlev.end());
    bh->lev.resize(Lm);
    const bool mixed_p = d0.precision == HJB_PREC_MIXED;
    int64_t maxn = 0;
    for (int l = 0; l < Lm; ++l) {
        BLevel &L = bh->lev[l];
        L.off.assign(count, -1);
        L.Ih.assign(count, BInst{});
        for (int b = 0; b < count; ++b) {
            if (l >= bh->nlev[b]) continue;
            L.off[b] = L.total;
            L.total += bh->sub[b]->lev[l].g.N;
            const bool coarsest = l == bh->nlev[b] - 1;
            if (coarsest && bh->sub[b]->lev[l].g.N <= kCoarseMaxNodes) {
                L.lds.push_back(b);
                L.lds_maxN = std::max(L.lds_maxN, bh->sub[b]->lev[l].g.N);
            }
        }
        BTRY(balloc(bh, (void **)&L.I, (size_t)count * sizeof(BInst)));
        BTRY(build_tiletab(bh, l, [&](int) { return true; }, L.all));
        BTRY(build_tiletab(bh, l, [&](int b) { return l + 1 < bh->nlev[b]; }, L.fine));
        BTRY(build_tiletab(bh, l, [&](int b) {
            return l == bh->nlev[b] - 1 && bh->sub[b]->lev[l].g.N > kCoarseMaxNodes; }, L.csm));
        BTRY(balloc(bh, (void **)&L.lds_dev, std::max<size_t>(1, L.lds.size()) * 4));
        if (!L.lds.empty())
            HIPCHK(hipMemcpy(L.lds_dev, L.lds.data(), L.lds.size() * 4, hipMemcpyHostToDevice));
        const size_t n = (size_t)L.total;
        if (l > 0) BTRY(balloc(bh, (void **)&L.alpha, n * 2));
        if (!mixed_p || l == 0) {
            BTRY(balloc(bh, &L.r64, n * 8));
            BTRY(balloc(bh, &L.e64, n * 8));
            BTRY(balloc(bh, &L.t64, n * 8));
            BTRY(balloc(bh, &L.d64, n * 8));
        }
        if (mixed_p) {
            BTRY(balloc(bh, &L.r32, n * 4));
            BTRY(balloc(bh, &L.e32, n * 4));
            BTRY(balloc(bh, &L.t32, n * 4));
            BTRY(balloc(bh, &L.d32, n * 4));
        }
        maxn = std::max<int64_t>(maxn, L.all.n);
    }
    bh->N = bh->lev[0].total;
    const size_t N = (size_t)bh->N;
    const int m = d0.restart;
    BTRY(balloc(bh, (void **)&bh->E, N * 8));
    BTRY(balloc(bh, (void **)&bh->R, N * 8));
    BTRY(balloc(bh, (void **)&bh->Vb, (size_t)(m + 1) * N * 8));
    BTRY(balloc(bh, (void **)&bh->Zb, (size_t)m * N * 8));
    BTRY(balloc(bh, (void **)&bh->Ua, N * 8));
    BTRY(balloc(bh, (void **)&bh->Ub, N * 8));
    BTRY(balloc(bh, (void **)&bh->Uc, N * 8));
    BTRY(balloc(bh, (void **)&bh->a0, N * 2));
    BTRY(balloc(bh, (void **)&bh->a1, N * 2));
    BTRY(balloc(bh, (void **)&bh->acarry, N * 2));
    BTRY(balloc(bh, (void **)&bh->partial, (size_t)kLdc * maxn * 8));
    BTRY(balloc(bh, (void **)&bh->ipartial, (size_t)maxn * 8));
    bh->maxn_cap = maxn;
    BTRY(balloc(bh, (void **)&bh->dseg, (size_t)count * kLdc * 8));
    BTRY(balloc(bh, (void **)&bh->dtau, (size_t)count * 8));
    BTRY(balloc(bh, (void **)&bh->dcoefA, (size_t)count * 8));
    BTRY(balloc(bh, (void **)&bh->dcoef, (size_t)count * kLdc * 8));
    BTRY(balloc(bh, (void **)&bh->dy, (size_t)count * kMaxRestart * 8));
    BTRY(balloc(bh, (void **)&bh->dchg, (size_t)count * 8));
    BTRY(balloc(bh, (void **)&bh->dm, (size_t)count * 4));
    for (int k = 0; k < 4; ++k) {
        BTRY(balloc(bh, (void **)&bh->dmask[k], (size_t)count));
        BTRY(bpin(bh, (void **)&bh->hmask[k], (size_t)count));
    }
    BTRY(bpin(bh, (void **)&bh->hseg, (size_t)count * kLdc * 8));
    BTRY(bpin(bh, (void **)&bh->hcoef, (size_t)count * kLdc * 8));
    BTRY(bpin(bh, (void **)&bh->hy, (size_t)count * kMaxRestart * 8));
    BTRY(bpin(bh, (void **)&bh->hchg, (size_t)count * 8));
    BTRY(bpin(bh, (void **)&bh->hm, (size_t)count * 4));
    {
        const size_t mr = (size_t)d0.restart;
        BTRY(balloc(bh, (void **)&bh->dH, (size_t)count * (mr + 1) * mr * 8));
        BTRY(balloc(bh, (void **)&bh->dcs, (size_t)count * mr * 8));
        BTRY(balloc(bh, (void **)&bh->dsn, (size_t)count * mr * 8));
        BTRY(balloc(bh, (void **)&bh->dg, (size_t)count * (mr + 1) * 8));
        BTRY(balloc(bh, (void **)&bh->dhn, (size_t)count * 8));
        BTRY(balloc(bh, (void **)&bh->dtarget, (size_t)count * 8));
        BTRY(balloc(bh, (void **)&bh->dits, (size_t)count * 3 * 4));  // its | bad | columns
        bh->dbad = bh->dits + count;
        bh->djb = bh->dits + 2 * count;
        BTRY(balloc(bh, (void **)&bh->dnext, (size_t)count));
        BTRY(bpin(bh, (void **)&bh->htarget, (size_t)count * 8));
        BTRY(bpin(bh, (void **)&bh->hits, (size_t)count * 2 * 4));
    }
    memset(bh->hcoef, 0, (size_t)count * kLdc * 8);
    memset(bh->hy, 0, (size_t)count * kMaxRestart * 8);
    {
        std::vector<double> cA(count);
        for (int b = 0; b < count; ++b) {
            const hjb_handle *h = bh->sub[b];
            cA[b] = 2.0 * h->M * (0.5 / h->desc.h) + h->cmax;
        }
        HIPCHK(hipMemcpy(bh->dcoefA, cA.data(), (size_t)count * 8, hipMemcpyHostToDevice));
    }
#undef BTRY
    *out = bh;
    return HJB_OK;
}

int hjb_batch_layout(const hjb_batch *bh, int64_t *offsets, int64_t *total) {
    if (!bh) return fail(HJB_EINVAL, "null batch");
    if (offsets)
        for (int b = 0; b < bh->B; ++b) offsets[b] = bh->lev[0].off[b];
    if (total) *total = bh->N;
    return HJB_OK;
}

int hjb_batch_set_stream(hjb_batch *bh, void *stream) {
    if (!bh) return fail(HJB_EINVAL, "null batch");
    bh->stream = (hipStream_t)stream;
    for (hjb_handle *h : bh->sub) h->stream = bh->stream;
    return HJB_OK;
}

int hjb_batch_set_tile_widths(hjb_batch *bh, const int32_t *widths) {
    if (!bh || !widths) return fail(HJB_EINVAL, "null argument");
    std::vector<int> tl(bh->B, -1);
    for (int b = 0; b < bh->B; ++b) {
        for (int c = kTileLogMin; c <= kTileLogMax; ++c)
            if (widths[b] == (1 << c)) tl[b] = c;
        if (tl[b] < 0) return fail(HJB_EINVAL, "instance %d: tile width must be 16, 32, 64 or 128", b);
    }
    HIPCHK(hipStreamSynchronize(bh->stream));
    for (int b = 0; b < bh->B; ++b) apply_tiles(bh->sub[b], tl[b]);
    return brebuild_tiles(bh);
}

int hjb_batch_autotune(hjb_batch *bh, const char *cache_path, int32_t *widths_out) {
    if (!bh) return fail(HJB_EINVAL, "null batch");
    // one tuning run per distinct key (grid, controls, coefficient model, precision, stencil reach), on a
    // full handle set up from a representative instance
    std::map<std::string, int> width_of;
    std::vector<int32_t> widths(bh->B, 1 << kTileLog2);
    for (int b = 0; b < bh->B; ++b) {
        const std::string key = tune_key(bh->sub[b]);
        auto it = width_of.find(key);
        if (it == width_of.end()) {
            hjb_desc db = bh->sub[b]->desc;
            db.stream = bh->stream;
            hjb_handle *h = nullptr;
            TRY(setup_impl(&db, &h, false));
            int32_t w = 0;
            const int rc = hjb_autotune(h, cache_path, &w, nullptr);
            hjb_destroy(h);
            TRY(rc);
            it = width_of.emplace(key, w).first;
        }
        widths[b] = it->second;
    }
    if (widths_out)
        for (int b = 0; b < bh->B; ++b) widths_out[b] = widths[b];
    return hjb_batch_set_tile_widths(bh, widths.data());
}

int hjb_solve_batch(hjb_batch *bh, const double *g, const double *psi, const double *f0, const double *f1,
                    int32_t n_steps, const double *dts, const double *thetas, double s, double *U_final,
                    int16_t *policies, hjb_solve_stats *st) {
    if (!bh) return fail(HJB_EINVAL, "null batch");
    if (!g || !psi || !f0 || !f1 || !dts || !thetas || !U_final) return fail(HJB_EINVAL, "null argument");
    if (n_steps < 0) return fail(HJB_EINVAL, "n_steps must be >= 0");
    for (int n = 0; n < n_steps; ++n) {
        TRY(check_time(dts[n], thetas[n]));
        if (thetas[n] == 0.0) return fail(HJB_EUNSUPPORTED, "explicit steps (theta = 0) are not provided");
    }
    const int B = bh->B;
    const int64_t N = bh->N;
    hipStream_t str = bh->stream;
    for (hjb_handle *h : bh->sub) {
        h->stream = str;
        TRY(build_tables(h, s));
    }
    TRY(brefresh(bh));
    std::vector<hjb_solve_stats> loc(B, hjb_solve_stats{});
    HIPCHK(hipMemcpyAsync(bh->Ua, g, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
    HIPCHK(hipMemcpyAsync(bh->Uc, g, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
    launch_zero(bh->acarry, (size_t)N * 2, str);
    double *Ucur = bh->Ua, *Unx = bh->Ub, *Uold = bh->Uc;
    double t = 0.0;
    int rc = HJB_OK;
    std::vector<hjb_step_stats> sst;
    for (int n = 0; n < n_steps; ++n) {
        HIPCHK(hipMemcpyAsync(Unx, psi, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
        rc = bstep(bh, Ucur, Unx, f0, f1, t, dts[n], thetas[n], n >= 1 ? Uold : nullptr, n >= 1 ? dts[n - 1] : 0.0,
                   sst);
        if (rc != HJB_OK) break;
        for (int b = 0; b < B; ++b) {
            loc[b].krylov_total += sst[b].krylov_total;
            loc[b].pi_total += sst[b].pi_iters;
            loc[b].flags |= sst[b].flags;
            loc[b].max_cert_bound = std::max(loc[b].max_cert_bound, sst[b].cert_bound);
            loc[b].steps_done = n + 1;
        }
        if (policies)
            HIPCHK(hipMemcpyAsync(policies + (int64_t)n * N, bh->acarry, (size_t)N * 2, hipMemcpyDeviceToDevice, str));
        std::swap(Uold, Ucur);
        std::swap(Ucur, Unx);
        t = t + dts[n];
    }
    HIPCHK(hipMemcpyAsync(U_final, Ucur, (size_t)N * 8, hipMemcpyDeviceToDevice, str));
    HIPCHK(hipStreamSynchronize(str));
    if (st)
        for (int b = 0; b < B; ++b) st[b] = loc[b];
    return rc;
}

void hjb_destroy_batch(hjb_batch *bh) {
    if (!bh) return;
    if (bh->stream) (void)hipStreamSynchronize(bh->stream);
    else (void)hipDeviceSynchronize();
    for (auto &g : bh->vgraphs) (void)hipGraphExecDestroy(g.exec);
    for (auto &g : bh->cgraphs) (void)hipGraphExecDestroy(g.exec);
    if (bh->capture_stream) (void)hipStreamDestroy(bh->capture_stream);
    for (hjb_handle *h : bh->sub) hjb_destroy(h);
    for (void *p : bh->allocs) (void)hipFree(p);
    for (void *p : bh->pinned) (void)hipHostFree(p);
    delete bh;
}

}  // extern "C"
