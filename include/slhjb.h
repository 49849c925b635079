/*
 * slhjb — implicit semi-Lagrangian solver for Hamilton-Jacobi-Bellman equations on MI355X.
 *
 * The method is that of Reisinger & Rotaetxe Arto, "Boundary Treatment and
 * Multigrid Preconditioning for Semi-Lagrangian Schemes Applied to
 * Hamilton-Jacobi-Bellman Equations" (arXiv:1605.04821):
 *   u_t - inf_alpha { L^alpha u + c^alpha u + f } = 0 on (0,T] x Omega,  u(0) = g,  u = psi on the boundary
 *   (eqs. 1.1-1.3), L^alpha u = tr[a^alpha D^2 u] + b^alpha . Du with a^alpha = 1/2 sigma^alpha sigma^alpha,T.
 * Space: the linear-interpolation semi-Lagrangian Scheme 2 (Section 1) with diffusion points
 * x +- sqrt(h) s sigma_p and drift point x + h b, truncated at the box boundary (Section 2.1,
 * eq. TruncScheme with the weights of Prop. pro:scheme2).  Time: the theta-scheme of eq. FullScheme.
 * Each step solves the row-wise nonlinear system of eq. nonlinear_sys by Howard policy iteration;
 * each fixed-policy linear system is solved by flexible GMRES preconditioned with a geometric
 * multigrid V-cycle (Section 3 studies multigrid preconditioning for this class of matrices).
 *
 * Memory and threading conventions (all entry points):
 *   - Every array argument is a DEVICE pointer (e.g. a torch tensor's data_ptr), contiguous, in the
 *     dtype stated, unless marked "host".  Full-grid arrays hold all nodes including the boundary,
 *     x fastest: node (i0,i1,i2) is element i0 + n0*(i1 + n1*i2).
 *   - Coefficient tables in hjb_desc are HOST memory and are copied during hjb_setup.
 *   - The library never frees or keeps caller memory; the handle owns its workspace.
 *   - Work is enqueued on the stream given in hjb_desc (NULL = the default stream).  Calls that return
 *     statistics synchronise that stream before returning.
 *   - Return values are status codes (HJB_OK or a negative HJB_E*); no exception crosses the ABI.
 *     hjb_last_error() gives a message for the calling thread's last failure.
 *   - Arguments are validated on the host before any device work; an invalid argument leaves all
 *     outputs untouched.  Without a usable GPU, hjb_setup fails with HJB_EDEVICE.
 *   - A handle must not be used by two threads at once.
 */
#ifndef SLHJB_H
#define SLHJB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hjb_handle hjb_handle;

enum {
    HJB_OK = 0,
    HJB_EINVAL = -1,          /* invalid argument (shape, pointer, parameter range) */
    HJB_EDEVICE = -2,         /* no usable GPU, or a HIP runtime error */
    HJB_ENOMEM = -3,          /* device allocation failed */
    HJB_ENOCONV_KRYLOV = -4,  /* linear solve missed its tolerance within max_krylov iterations */
    HJB_ENOCONV_PI = -5,      /* policy iteration still changing after max_pi iterations */
    HJB_ENONFINITE = -6,      /* non-finite value met in a residual or norm */
    HJB_EUNSUPPORTED = -7     /* valid request this build does not implement */
};

enum {
    HJB_COEF_CONST = 0,     /* sigma, b, c constant per control */
    HJB_COEF_XSCALED = 1,   /* sigma_k(x) = diag(x) S_k, b_k(x) = diag(x) beta_k (x the node's coordinates,
                               eq. 1.1 with x-dependent coefficients): sigma holds S, drift holds beta;
                               c constant per control */
    HJB_COEF_FIELD = 2      /* sigma(x) per node, the same for every control: sigma[(i*P + p)*dim + d]
                               (host, N*P*dim, full grid, x fastest); drift, c constant per control */
};
enum { HJB_PREC_FP64 = 0, HJB_PREC_MIXED = 1 }; /* V-cycle in FP64, or in FP32 under FP64 FGMRES */
/* preconditioner of the linear solves: none, Jacobi, the geometric V-cycle, or aggregation-based algebraic
   multigrid with a Krylov-accelerated cycle (the introduction, Sections 3.4-3.5; HJB_PRECOND_AMG: FP64,
   forward solves only) */
enum { HJB_PRECOND_NONE = 0, HJB_PRECOND_JACOBI = 1, HJB_PRECOND_VCYCLE = 2, HJB_PRECOND_AMG = 3 };
enum { HJB_KRYLOV_FGMRES = 0, HJB_KRYLOV_BICGSTAB = 1 };  /* outer FP64 Krylov method of the linear solves */
/* coarse operators of the V-cycle: rediscretised on each level, or Galerkin products R A P (Section 3.3) */
enum { HJB_COARSE_REDISCRETIZED = 0, HJB_COARSE_GALERKIN = 1 };
/* Flags of hjb_step_stats / hjb_solve_stats (bitwise or). */
enum {
    HJB_FLAG_POSITIVITY = 1,  /* positivity of the weights (eq. CFL_trunc) may fail: theta < 1 and
                                 (1 - theta) dt (M/h + max|c|) > 1 */
    HJB_FLAG_NEAR_TIES = 2    /* the returned policy has near ties: nodes where the second-best G_k is within
                                 1e3 * tau of the best, so that several policies are correct results */
};

typedef struct {
    /* Grid (eqs. 1.1-1.3 on a box, Section 2.1): n[d] nodes per axis, uniform spacing h, corner lo. */
    int32_t dim;            /* 2 or 3 */
    int32_t n[3];           /* >= 3 per used axis */
    double lo[3];
    double h;
    /* Controls (Section 1, definition of L): K controls, P diffusion columns each.
       sigma[(k*P + p)*dim + d] (host, K*P*dim), drift[k*dim + d] (host, K*dim, may be NULL = no drift),
       c[k] (host, K, may be NULL = 0); coef_model: HJB_COEF_* (how sigma and drift depend on x).
       Only Scheme 2 (scheme = 2) is provided: its truncation is the consistent one (Prop. pro:scheme2). */
    int32_t K, P, coef_model, scheme;
    const double *sigma, *drift, *c;
    /* Solver controls. */
    int32_t precision;      /* HJB_PREC_FP64 | HJB_PREC_MIXED */
    int32_t precond;        /* HJB_PRECOND_* */
    int32_t restart;        /* FGMRES restart length m, 1..64 (BiCGSTAB: >= 3, its four vectors use that storage) */
    int32_t max_krylov;     /* total Krylov iterations per linear solve (a BiCGSTAB iteration counts two) */
    int32_t max_pi;         /* policy iterations per time step */
    int32_t nu1, nu2;       /* V-cycle pre/post Jacobi sweeps */
    int32_t coarse_sweeps;  /* Jacobi sweeps on the coarsest level */
    int32_t min_coarse;     /* stop coarsening at the first level with <= min_coarse nodes per axis that also
                               fits the one-workgroup coarsest solve (<= 2048 nodes) */
    double omega;           /* Jacobi damping */
    double rtol_inf;        /* linear solve stops when |F - A X|_inf <= rtol_inf * max(1,|X|_inf) */
    double tau_rel;         /* policy tie tolerance relative to the scale S of the search */
    double pi_eta;          /* policy iterations whose policy may still change solve only until the
                               residual has dropped by this factor (0: every solve to rtol_inf); the
                               last solve of a step always meets rtol_inf and is confirmed by a search */
    int32_t use_graphs;     /* 1: replay captured HIP graphs of the V-cycle (identical kernels), 0: launch eagerly */
    int32_t f_per_control;  /* 0: f0, f1 are full-grid arrays shared by all controls; 1: [K][N], the source
                               of each control (the search and the right-hand side take the node's control's) */
    int32_t certified_skip; /* 1: within a time step, a search keeps the control of every untruncated wavefront
                               whose recorded gap between its best and second-best G still exceeds twice the
                               largest change of G allowed by the change of X since (constant coefficients,
                               P = 1): the same controls as a full search, at a fraction of its cost.  0: every
                               search evaluates every control */
    int32_t max_levels;     /* at most this many multigrid levels (0: no limit); setup only */
    int32_t nu_tight;       /* pre- and post-sweeps of the V-cycles of solves that must reach the certificate
                               (the last solve of a step, hjb_linsolve, every transposed solve); 0: nu1, nu2 */
    int32_t coarse_sweeps_t; /* damped Jacobi sweeps on the coarsest level of the transposed V-cycles of the
                               adjoint (0: coarse_sweeps; a single-level hierarchy always takes coarse_sweeps);
                               0..1000 */
    int32_t krylov;         /* HJB_KRYLOV_FGMRES (default) or HJB_KRYLOV_BICGSTAB (Section 3.3's Krylov baseline,
                               right-preconditioned by the same V-cycle or Jacobi, same stopping rule and
                               certificate, restarted from the true residual) for every linear solve of the
                               handle, transposed solves included; batches take FGMRES only */
    int32_t coarse_op;      /* HJB_COARSE_REDISCRETIZED (default) or HJB_COARSE_GALERKIN: coarse levels of the forward
                               V-cycle are A_{l+1} = R A_l P (full weighting R, bilinear P, Section 3.3), rebuilt
                               for every policy and held as sliced ELL rows of at most 128 entries (wider rows
                               fail with HJB_EUNSUPPORTED); damped Jacobi on them.  2D only; the adjoint's
                               transposed cycles and batches keep rediscretised levels */
    int32_t kcycle_levels;  /* HJB_PRECOND_AMG: coarse levels 1..kcycle_levels solve their residual equation by two
                               GCR iterations preconditioned by the cycle below (the K-cycle), deeper levels by one
                               (a V-cycle whose coarse correction is scaled by its minimal-residual factor);
                               -1 (default): every level */
    int32_t value_stride;   /* k >= 1: the `values` of hjb_solve and hjb_adjoint hold every k-th level only, U^0,
                               U^k, U^2k, ... (n_steps / k + 1 arrays); hjb_adjoint recomputes the levels between
                               them one segment at a time (default 1: every level) */
    int32_t amg_reuse;      /* HJB_PRECOND_AMG: 0 (default) rebuilds the aggregation hierarchy for every policy;
                               1 builds it at the first solve of each time step and keeps its coarse levels for
                               the step's later policies (the finest level always follows the current policy;
                               the outer Krylov method still meets the certificate) */
    void *stream;           /* hipStream_t */
} hjb_desc;

typedef struct {
    int32_t pi_iters;       /* policy iterations (linear solves) in the step */
    int32_t krylov_total;   /* Krylov iterations summed over the step's solves: applications of the
                               preconditioned operator (one per FGMRES iteration, two per BiCGSTAB iteration) */
    int32_t krylov_max;     /* largest Krylov count of one solve */
    int32_t flags;          /* HJB_FLAG_* */
    double res_inf;         /* final |F - A X|_inf of the last solve */
    double cert_bound;      /* bound on |X - X*|_inf of the last solve: res_inf / (1 - theta dt max(c,0)) */
    int64_t n_changed_first;/* controls changed by the first search of the step */
    int64_t n_near_ties;    /* interior nodes whose decision in the step's last search is a near tie
                               (HJB_FLAG_NEAR_TIES): the second-best G_k lies within 1e3 * tau of the best.
                               Nodes kept by certified reuse are not evaluated and count as clear decisions
                               (their certified gap exceeds 1e-10 S, which is 1e3 * tau at the default
                               tau_rel). 0 for explicit steps. */
} hjb_step_stats;

typedef struct {
    int32_t steps_done;
    int32_t flags;          /* HJB_FLAG_* of every step, or-ed */
    int64_t krylov_total;
    int64_t pi_total;
    double max_cert_bound;
    int64_t near_ties_total; /* n_near_ties summed over the steps */
} hjb_solve_stats;

/* Fill *d with defaults (2D, FP64, V-cycle(3,3) and (4,4) for solves to the certificate, m = 10, rtol 1e-13,
   tau_rel 1e-13, pi_eta 0.35, ...). Grid and controls
   still have to be set by the caller. */
void hjb_desc_default(hjb_desc *d);

/* Validate the problem description (eqs. 1.1-1.3 on a box), build per-control stencil tables for every
   multigrid level and allocate the workspace.  On success *out owns device memory until hjb_destroy. */
int hjb_setup(const hjb_desc *desc, hjb_handle **out);

/* Replace the stream used by later calls (hipStream_t; NULL = default stream). */
int hjb_set_stream(hjb_handle *hd, void *stream);

/* Change solver controls after setup (precision, precond, restart, max_krylov, max_pi, nu1, nu2,
   coarse_sweeps, omega, rtol_inf, tau_rel, pi_eta, use_graphs, certified_skip, nu_tight, coarse_sweeps_t,
   krylov, kcycle_levels, value_stride, amg_reuse are taken from
   *desc; grid and controls
   are those of the setup).  restart may not exceed its value at setup. */
int hjb_set_options(hjb_handle *hd, const hjb_desc *desc);

/*
 * Policy improvement (Howard's algorithm on eq. nonlinear_sys; the theta-scheme of eq. FullScheme):
 * for each interior node i and control k,
 *   G_k = theta*((L^k X)_i + c_k X_i) + (1-theta)*((L^k U)_i + c_k U_i) + f_i,   f = f0 + t_mid*f1,
 *   t_mid = t_prev + theta*dt.  The residual of row i is X_i - U_i - dt*G_k, so the search minimises G_k.
 * Tie rule: g* = min_k G_k, tau = tau_rel*S with S = (2*M*(0.5/h) + max|c|)*max(|X|inf,|U|inf) + |f|inf
 * (M = P + 1 with drift, else P); alpha_in[i] is kept if G_{alpha_in} <= g* + tau, otherwise the smallest
 * k with G_k <= g* + tau is taken.
 *   X, U: full-grid FP64 (boundary entries are the Dirichlet values used by truncated points);
 *   f0, f1: full-grid FP64; alpha_in: full-grid int16 (boundary entries ignored; may equal alpha_out);
 *   alpha_out: full-grid int16, boundary entries set to -1;
 *   gmin (nullable): g* per node (0 on the boundary); margin (nullable): min{G_k - g* : G_k > g*+tau};
 *   ties (nullable, int32): #{k : G_k <= g* + tau};  n_changed (host, nullable): changed interior nodes;
 *   tau_used (host, nullable): the tau applied.  Synchronises the stream when n_changed or tau_used is given.
 */
int hjb_policy_sweep(hjb_handle *hd, const double *X, const double *U, const double *f0, const double *f1,
                     double t_prev, double dt, double theta, double s,
                     const int16_t *alpha_in, int16_t *alpha_out, double *gmin, double *margin, int32_t *ties,
                     int64_t *n_changed, double *tau_used);

/* hjb_policy_sweep for callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same arguments, kernels and results, bit for bit, but the search's
 * own scratch (block partials of the tolerance, tau, the per-tile change counts and their sums) lives in a static
 * 1 MiB device array that the library holds on each GPU until the process ends, instead of the handle's buffers.
 * No hipMalloc, hipFree or other allocating routine is called.
 *   - The handle comes from hjb_setup (which allocates, once); its stencil tables must already be those of s
 *     (s = 1 after setup, else the s of the handle's latest call of another entry point): HJB_EINVAL otherwise.
 *   - Grids needing more than the 1 MiB (about 43,000 tiles of 256 nodes, e.g. 3300 x 3300 in 2D) give HJB_EINVAL.
 *   - Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU (other streams, other
 *     threads, other handles) race and must be serialised by the caller.  Every value the search reads from the
 *     array is written earlier in the same call, so what a previous call left there does not matter.
 *   - Without n_changed and tau_used nothing is read back and the call only enqueues work on the stream.
 */
int hjb_policy_sweep_noalloc(hjb_handle *hd, const double *X, const double *U, const double *f0, const double *f1,
                             double t_prev, double dt, double theta, double s, const int16_t *alpha_in,
                             int16_t *alpha_out, double *gmin, double *margin, int32_t *ties, int64_t *n_changed,
                             double *tau_used);

/* y = A^alpha x for the fixed-policy matrix of eq. FullScheme restricted to interior nodes,
   (A x)_i = x_i - theta*dt*((L^{alpha_i} x)_i + c x_i), reading boundary entries of x as given
   (pass zeros there for the matrix itself).  y is written on interior nodes and zeroed on the boundary.
   x, y: full-grid FP64 (distinct); alpha: full-grid int16. */
int hjb_apply(hjb_handle *hd, const int16_t *alpha, const double *x, double *y, double dt, double theta, double s);

/* Solve the fixed-policy system of eq. FullScheme (Dirichlet data moved to the right-hand side as in
   Remark rem:rhs): X_i - theta*dt*((L X)_i + c X_i) = U_i + (1-theta)*dt*((L U)_i + c U_i) + dt*f_i.
   X (full-grid FP64): in = initial guess on interior nodes and the Dirichlet data on the boundary;
   out = solution on interior nodes (boundary untouched).  U: previous time level (full grid). */
int hjb_linsolve(hjb_handle *hd, const int16_t *alpha, const double *U, const double *f0, const double *f1,
                 double t_prev, double dt, double theta, double s, double *X, hjb_step_stats *st);

/* One theta-step by policy iteration (eq. nonlinear_sys): searches start from alpha_io (the previous
   step's policy) and alternate with linear solves until no control changes.
   Uprev: full-grid FP64 U^{n-1}; Unext: full-grid FP64 whose boundary entries hold psi on entry
   (never written) and whose interior receives U^n; alpha_io: full-grid int16, in/out.
   Uprev2 (nullable): U^{n-2}; when given, policy iteration starts from the linear extrapolation
   U^{n-1} + (dt/dt_prev)(U^{n-1} - U^{n-2}) instead of U^{n-1}.  The starting point only changes how many
   iterations are needed: the result meets the same residual certificate and policy condition.
   theta = 0 is the explicit scheme: one search at U^{n-1} (f at t_{n-1}) and U^n = U^{n-1} + dt min_k G_k
   on interior nodes, queued on the stream without a wait; stats flag bit 0 when dt (M/h + max|c|) > 1
   (positivity of the untruncated weights may fail). */
int hjb_step(hjb_handle *hd, const double *Uprev, double *Unext, const double *f0, const double *f1,
             double t_prev, double dt, double theta, double s, int16_t *alpha_io, const double *Uprev2,
             double dt_prev, hjb_step_stats *st);

/* March U^0 = g (eq. 1.2), U^n = psi(t_n) on the boundary (eq. 1.3) through n_steps theta-steps with
   dts[n], thetas[n] (host arrays), t_n = t_{n-1} + dts[n-1]; from the third step on, each step starts from the
   extrapolation of the two previous levels (see hjb_step).  Dirichlet data: psi (full-grid FP64, only boundary
   entries are read) and psi1 (nullable, full-grid FP64): psi(t) = psi + t * psi1, constant when psi1 is NULL.
   theta = 0 steps are explicit (see hjb_step).  U_final: full-grid FP64 output.  policies (nullable): int16
   [n_steps][N], the converged policy of each step (the checkpoints an adjoint sweep reuses).
   values (nullable): FP64 [n_steps / value_stride + 1][N], U^0 = g and every value_stride-th U^n, for
   hjb_adjoint to use instead of recomputing them. */
int hjb_solve(hjb_handle *hd, const double *g, const double *psi, const double *psi1, const double *f0,
              const double *f1, int32_t n_steps, const double *dts, const double *thetas, double s,
              double *U_final, int16_t *policies, double *values, hjb_solve_stats *st);

typedef struct {
    int64_t krylov_recompute;  /* Krylov iterations of the recomputation of the values (0 with values given) */
    int64_t krylov_adjoint;    /* Krylov iterations of the transposed solves */
    double max_res_adjoint;    /* largest final |lambda - A^T mu|_inf of the transposed solves */
} hjb_adjoint_stats;

/*
 * Discrete adjoint of hjb_solve at the policies it returned (gradients of a functional J of U^N).
 * Each step solves A_n U^n = B_n U^{n-1} + dt_n f(t_mid) + Dirichlet terms (eq. FullScheme with
 * A_n = I - theta dt (L^{alpha_n} + C) on interior nodes and B_n = I + (1-theta) dt (L^{alpha_n} + C) on the
 * full previous level).  The values U^n enter only dJ/ds: they are taken from `values` (hjb_solve's output)
 * or, when it is NULL and dJ_ds is requested, recomputed from g and the int16 policies by fixed-policy solves,
 * keeping only every ceil(sqrt(n_steps))-th value and recomputing one segment at a time in the backward
 * sweep (2 n_steps solves, about 2 sqrt(n_steps) + 1 FP64 arrays); with values holding every k-th level
 * (value_stride = k > 1, as hjb_solve stored them) only the segments are recomputed (n_steps solves, k + 1
 * arrays); without dJ_ds nothing is recomputed.
 * Then backwards: A_n^T mu_n = lambda_n, dJ/df0 += dt mu_n, dJ/df1 += dt t_mid mu_n,
 * dJ/ds += dt mu_n^T (theta d_s L U^n + (1-theta) d_s L U^{n-1}), lambda_{n-1} = B_n^T mu_n, dJ/dg = lambda_0.
 * Policies are held fixed, so the gradient is exact away from policy switches (where J is differentiable).
 *   g, psi, f0, f1: full-grid FP64 as for hjb_solve; policies: int16 [n_steps][N] from hjb_solve;
 *   values (nullable): FP64 [n_steps / value_stride + 1][N] from hjb_solve with the same value_stride;
 *   dts, thetas: host [n_steps]; dJ_dUN: full-grid FP64 (boundary entries ignored);
 *   dJ_df0, dJ_dg: full-grid FP64 outputs (dJ_df0 zero on the boundary); dJ_df1: nullable;
 *   dJ_ds: host scalar (nullable).  Transposed solves use FGMRES on an explicitly transposed operator
 *   (rows listed and stably sorted by column, no atomics), preconditioned by a V-cycle on the transposed
 *   level operators (or Jacobi, following the handle's preconditioner option), each starting from the
 *   previous step's multiplier.  Workspace is allocated per call.
 */
int hjb_adjoint(hjb_handle *hd, const double *g, const double *psi, const double *f0, const double *f1,
                int32_t n_steps, const double *dts, const double *thetas, double s, const int16_t *policies,
                const double *values, const double *dJ_dUN, double *dJ_df0, double *dJ_df1, double *dJ_dg, double *dJ_ds,
                hjb_adjoint_stats *st);

/* y = (A^alpha)^T x for the matrix of hjb_apply (interior rows and columns; y zero on the boundary).
   x, y: full-grid FP64 (distinct). */
int hjb_apply_transposed(hjb_handle *hd, const int16_t *alpha, const double *x, double *y, double dt, double theta,
                         double s);

/* The Galerkin coarse operator of multigrid level `level` (>= 1; HJB_COARSE_GALERKIN) for the policy of the
 * handle's last solve: sliced ELL rows over the level's full grid, entry s of node i at s * nodes + i
 * (column index on the level, -1 for an unused slot; boundary rows empty), copied to the caller's device
 * buffers cols / vals (width * nodes entries each; either may be NULL).  width and nodes (nullable) receive
 * the ELL width and the level's node count.  HJB_EINVAL for a level without a Galerkin operator. */
int hjb_coarse_operator(hjb_handle *hd, int32_t level, int32_t *width, int64_t *nodes, int32_t *cols, double *vals);

/* One level of the aggregation hierarchy (HJB_PRECOND_AMG, Sections 3.4-3.5) of the handle's last hierarchy
 * build (the last solve's policy, or with amg_reuse the policy of its time step's first solve).  Level 0 is the finest system matrix A = I - theta dt (L-hat + c) of the interior unknowns,
 * indexed by full-grid node (boundary rows empty, boundary columns left to the right-hand side); level l >= 1 holds A_l = P_l^T A_{l-1} P_l, where P_l is piecewise constant: fine node i of
 * level l-1 maps to aggregate agg[i] of level l (-1: in no aggregate).  Rows are sliced ELL, entry s of row i
 * at s * rows + i (column -1 unused, a row's entries in its first slots).  levels, rows and width (nullable)
 * receive the hierarchy's depth, the level's row count and ELL width; agg (level >= 1: rows of level l-1
 * entries), cols and vals (width * rows entries) are the caller's device buffers, each nullable.
 * HJB_EINVAL when no hierarchy is built or level is out of range. */
int hjb_amg_level(hjb_handle *hd, int32_t level, int32_t *levels, int64_t *rows, int32_t *width, int32_t *agg,
                  int32_t *cols, double *vals);

/* ---- batches of independent instances (uneven grids, coefficients and multigrid depths) ----------

   One handle drives many instances together: every kernel launch covers the tiles of all instances
   that take part, and policy iteration and FGMRES advance in lockstep, each instance stopping on its
   own certificate.  Instances may differ in n, lo, h, K, P, coef_model and coefficient tables; dim and
   the solver options (taken from descs[0]; nu1 + nu2 even, V-cycle or no preconditioner) are shared.
   Full-grid arrays of the batch are the instances' arrays concatenated, instance b starting at node
   offsets[b] of hjb_batch_layout. */
typedef struct hjb_batch hjb_batch;
int hjb_setup_batch(const hjb_desc *descs, int32_t count, hjb_batch **out);
/* offsets (host, count entries, nullable) and total nodes (host, nullable) of the concatenated layout */
int hjb_batch_layout(const hjb_batch *bh, int64_t *offsets, int64_t *total);
int hjb_batch_set_stream(hjb_batch *bh, void *stream);

/* Tile shape of each instance: widths[b] (16, 32, 64 or 128 nodes along x; each level takes at most its own
   next power of two) for instance b (host, count entries).  The batch's launch lists are rebuilt; results
   agree with any other widths to the solver's certificate (partial sums follow the tiles).  HJB_EINVAL for
   another width. */
int hjb_batch_set_tile_widths(hjb_batch *bh, const int32_t *widths);

/* The autotuner over a batch: for each distinct (grid, controls, coefficient model, precision, stencil reach)
   among the instances, hjb_autotune on a full handle of one such instance (its cache file cache_path,
   nullable, shared with hjb_autotune), then hjb_batch_set_tile_widths with the chosen widths; widths_out
   (host, count entries, nullable) receives them. */
int hjb_batch_autotune(hjb_batch *bh, const char *cache_path, int32_t *widths_out);
/* hjb_solve for every instance with one shared schedule and s; arrays in the concatenated layout
   (device, FP64; policies int16 [n_steps][total], nullable); st: host [count] (nullable; near ties are not
   counted in batches: near_ties_total is 0).
   The first instance that fails (e.g. HJB_ENOCONV_KRYLOV) stops the whole batch; the message names it. */
int hjb_solve_batch(hjb_batch *bh, const double *g, const double *psi, const double *f0, const double *f1,
                    int32_t n_steps, const double *dts, const double *thetas, double s, double *U_final,
                    int16_t *policies, hjb_solve_stats *st);
void hjb_destroy_batch(hjb_batch *bh);

/* Node tile of the kernels' blocks (256 threads): width 16, 32 (default), 64 or 128 nodes along x.
   Results do not depend on it apart from the order of the reductions inside the Krylov solver. */
int hjb_set_tile_width(hjb_handle *hd, int32_t width);
/* Chooses the tile width for this handle's grid and coefficients by timing the search, the operator
   apply and the V-cycle on synthetic data for each width (weighted as 9.5 searches and 45 Krylov
   iterations per time step), and keeps it in the handle.  cache_path (nullable): a JSON-lines file of
   earlier choices keyed by dim, n, K, P, stencil points, coefficient model, precision and stencil reach
   at the handle's current s; a hit skips the timing, a miss appends the new choice.
   tile_width_out, cost_ms_out (host, nullable; cost_ms_out: 4 entries for widths 16..128, filled only
   when timed).  Overwrites the handle's work buffers; synchronises the stream. */
int hjb_autotune(hjb_handle *hd, const char *cache_path, int32_t *tile_width_out, double *cost_ms_out);

/* Kernel timers.  Any caller that wants the duration of one class of kernel launches during real work
   (e.g. a benchmark's roofline) enables a timer; launches of that class then carry HIP events on the
   handle's stream, stamped with the dispatch's own begin and end (hipExtLaunchKernel), at most
   max_launches of them (enable again to reset).
   hjb_profile_read synchronises the stream and reports the recorded launches, their summed duration in
   milliseconds, their summed algorithmic bytes (each input element read once, each output written
   once; halo re-reads of gathered stencil points are not counted) and, for the policy search, their
   summed algorithmic FP64 operations on interior nodes (untruncated stencil arithmetic; 0 otherwise).
   The smoother and multigrid-residual timers, and with the V-cycle preconditioner the operator-application
   timer (the application is captured with the cycle it follows), record the launches of sampled V-cycles,
   which run without their captured graph; see hjb_profile_sample. */
enum {
    HJB_KERNEL_APPLY = 0,     /* y = A^alpha z in FGMRES (FP64 out; z FP64 or FP32) */
    HJB_KERNEL_SMOOTH = 1,    /* damped Jacobi sweep with stencil gathers on the finest level */
    HJB_KERNEL_MG_RESID = 2,  /* multigrid residual on the finest level */
    HJB_KERNEL_DOT = 3,       /* fused multi-vector dot products of the Arnoldi step */
    HJB_KERNEL_AXPY = 4,      /* fused multi-vector update of the Arnoldi step */
    HJB_KERNEL_SWEEP = 5,     /* policy search (all controls per node) */
    HJB_KERNEL_COUNT = 6
};
int hjb_profile_enable(hjb_handle *hd, int32_t kernel, int32_t max_launches);
int hjb_profile_read(hjb_handle *hd, int32_t kernel, int64_t *launches, double *total_ms, double *total_bytes,
                     double *total_flops);

/* Timer sampling: with period p >= 1, one V-cycle in p is sampled (launched eagerly, its finest-level
   smoother and residual launches and the operator application after it timed) while the others replay
   their captured graph untimed, and one launch in p of the multi-dot and update classes is timed; the
   policy search is timed at every launch.  p = 1 (the default) times every launch and runs
   every V-cycle eagerly while a smoother or residual timer is enabled.  Results do not depend on p.
   Returns HJB_EINVAL for p outside 1..1000000. */
int hjb_profile_sample(hjb_handle *hd, int32_t period);

/* Free the handle and its device workspace (NULL is ignored). */
void hjb_destroy(hjb_handle *hd);

/* Message for the calling thread's last failed call ("" if none). */
const char *hjb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLHJB_H */
