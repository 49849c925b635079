/*
 * CPU FP64 oracle for the truncated semi-Lagrangian (LISL, Scheme 2) operator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code with the
 * HIP path: it is written directly from Reisinger & Rotaetxe Arto,
 * "Boundary Treatment and Multigrid Preconditioning for Semi-Lagrangian
 * Schemes Applied to HJB Equations" (arXiv:1605.04821).
 *
 * What it computes
 *   - Scheme 2 stencil (Section 1, "Examples of LISL schemes"): diffusion
 *     points x +- sqrt(dx) sigma_p, drift point x + dx b, M = P + 1.
 *   - Multilinear interpolation with non-negative weights (eq. monotone_int,
 *     monotone_int_2).
 *   - Stencil truncation on a box (Section 2.1, eq. TruncScheme): the point is
 *     pulled back to the boundary by the largest mu in (0,1] (Prop. pro:scheme2)
 *     and weighted by A_p = 2/(mu+^2 + mu+ mu-), B_p = 2/(mu-^2 + mu- mu+)
 *     (eq. eqn_Ap) and A_{P+1} = B_{P+1} = 1/mu (eq. eqn_APp1).
 *   - The operator in l-hat form (eq. Lhat) both as a direct evaluation and as
 *     an explicit sparse row listing, for assembling A^alpha (eq. FullScheme).
 *   - The policy-improvement step of Howard's algorithm: the row-wise search
 *     over the finite control set for the system (eq. nonlinear_sys).
 *
 * Arithmetic conventions (the reading taken where the paper is silent):
 *   - Displacements are measured in cells: Y = s*sigma/sqrt(h) for diffusion,
 *     Y = b for the drift (dx*b/dx).
 *   - mu = min(1, min_d D_d/|Y_d|) with D_d the integer distance to the face the
 *     point moves towards.  If mu == 1 the landing coordinate i_d + Y_d is split
 *     exactly into cell i_d + floor(Y_d) and fraction Y_d - floor(Y_d).  If
 *     mu < 1 the limiting coordinate is set to the face index exactly and the
 *     others are i_d + mu*Y_d, clamped to [0, n_d-1].
 *   - A landing cell n_d-1 is replaced by cell n_d-2 with fraction 1.
 *   - Interpolation is the weighted sum of eq. monotone_int over the 2^d cell
 *     corners c = 0..2^d-1 (bit d of c set: upper corner along axis d): the
 *     weight is the product over axes, in axis order, of t_d (upper) or 1-t_d
 *     (lower), and the sum is w_0*V_0 followed by fma(w_c, V_c, sum) in corner
 *     order.
 *   - Apart from those explicit fma() calls every expression is evaluated left
 *     to right as written (compiled with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dim;
    int32_t K, P;
    int64_t n[3];
    double h;
    double sr;                 /* s / sqrt(h): cells per unit of sigma */
    const double *sigma;       /* element (k,i,p,d) at sigma[k*sig_k + i*sig_i + p*dim + d] */
    int64_t sig_k, sig_i;
    const double *drift;       /* element (k,i,d) at drift[k*b_k + i*b_i + d]; NULL: no drift */
    int64_t b_k, b_i;
    const double *c;           /* element (k,i) at c[k*c_k + i*c_i]; NULL: c = 0 */
    int64_t c_k, c_i;
} orc_problem;

typedef struct {
    int64_t cell[3];
    double t[3];
    double mu;
} orc_land;

static void unflatten(const orc_problem *pb, int64_t i, int64_t ix[3]) {
    ix[0] = i % pb->n[0];
    int64_t r = i / pb->n[0];
    ix[1] = pb->dim > 1 ? r % pb->n[1] : 0;
    ix[2] = pb->dim > 2 ? r / pb->n[1] : 0;
}

static int is_interior(const orc_problem *pb, const int64_t ix[3]) {
    for (int d = 0; d < pb->dim; ++d)
        if (ix[d] <= 0 || ix[d] >= pb->n[d] - 1) return 0;
    return 1;
}

/* Where the (possibly truncated) point x_i + mu*Y lands, Section 2.1 and Prop. pro:scheme2. */
static void landing(const orc_problem *pb, const int64_t ix[3], const double Y[3], orc_land *L) {
    double m[3];
    double mu = 1.0;
    for (int d = 0; d < pb->dim; ++d) {
        m[d] = INFINITY;
        if (Y[d] != 0.0) {
            int64_t D = (Y[d] > 0.0) ? (pb->n[d] - 1 - ix[d]) : ix[d];
            m[d] = (double)D / fabs(Y[d]);
            if (m[d] < mu) mu = m[d];
        }
    }
    L->mu = mu;
    for (int d = 0; d < pb->dim; ++d) {
        int64_t cell;
        double t;
        if (mu == 1.0) {
            double fl = floor(Y[d]);
            cell = ix[d] + (int64_t)fl;
            t = Y[d] - fl;
        } else if (Y[d] != 0.0 && m[d] == mu) {
            cell = (Y[d] > 0.0) ? pb->n[d] - 1 : 0;
            t = 0.0;
        } else {
            double q = (double)ix[d] + mu * Y[d];
            if (q < 0.0) q = 0.0;
            if (q > (double)(pb->n[d] - 1)) q = (double)(pb->n[d] - 1);
            double fl = floor(q);
            cell = (int64_t)fl;
            t = q - fl;
        }
        if (cell >= pb->n[d] - 1) { cell = pb->n[d] - 2; t = 1.0; }
        L->cell[d] = cell;
        L->t[d] = t;
    }
}

/* Weight of corner c (bit d set: upper corner on axis d) of a landing, eq. monotone_int_2. */
static double corner_weight(const orc_problem *pb, const orc_land *L, int c) {
    double w = ((c & 1) ? L->t[0] : (1.0 - L->t[0]));
    for (int d = 1; d < pb->dim; ++d) w = w * (((c >> d) & 1) ? L->t[d] : (1.0 - L->t[d]));
    return w;
}

static int64_t corner_index(const orc_problem *pb, const orc_land *L, int c) {
    int64_t s1 = pb->n[0], s2 = pb->n[0] * pb->n[1];
    int64_t idx = L->cell[0] + (c & 1);
    if (pb->dim > 1) idx += (L->cell[1] + ((c >> 1) & 1)) * s1;
    if (pb->dim > 2) idx += (L->cell[2] + ((c >> 2) & 1)) * s2;
    return idx;
}

/* Multilinear interpolant (eq. monotone_int): sum over the cell corners of weight times value. */
static double interp(const orc_problem *pb, const orc_land *L, const double *V) {
    int nc = 1 << pb->dim;
    double v = corner_weight(pb, L, 0) * V[corner_index(pb, L, 0)];
    for (int c = 1; c < nc; ++c) v = fma(corner_weight(pb, L, c), V[corner_index(pb, L, c)], v);
    return v;
}

static void diffusion_Y(const orc_problem *pb, int k, int64_t i, int p, double Y[3]) {
    const double *sg = pb->sigma + k * pb->sig_k + i * pb->sig_i + (int64_t)p * pb->dim;
    for (int d = 0; d < 3; ++d) Y[d] = d < pb->dim ? pb->sr * sg[d] : 0.0;
}

static int drift_Y(const orc_problem *pb, int k, int64_t i, double Y[3]) {
    if (!pb->drift) return 0;
    const double *b = pb->drift + k * pb->b_k + i * pb->b_i;
    int nz = 0;
    for (int d = 0; d < 3; ++d) {
        Y[d] = d < pb->dim ? b[d] : 0.0;
        if (Y[d] != 0.0) nz = 1;
    }
    return nz;
}

static double coef_c(const orc_problem *pb, int k, int64_t i) {
    return pb->c ? pb->c[k * pb->c_k + i * pb->c_i] : 0.0;
}

/* (L-hat^k V)_i, eq. TruncScheme with Scheme 2 and weights eqn_Ap / eqn_APp1. */
static double lhat_eval(const orc_problem *pb, int64_t i, const int64_t ix[3], int k, const double *V) {
    double inv2h = 0.5 / pb->h;
    double Vi = V[i];
    double acc = 0.0;
    for (int p = 0; p < pb->P; ++p) {
        double Yp[3], Ym[3];
        diffusion_Y(pb, k, i, p, Yp);
        for (int d = 0; d < 3; ++d) Ym[d] = -Yp[d];
        orc_land Lp, Lm;
        landing(pb, ix, Yp, &Lp);
        landing(pb, ix, Ym, &Lm);
        double A = 2.0 / (Lp.mu * (Lp.mu + Lm.mu));
        double B = 2.0 / (Lm.mu * (Lm.mu + Lp.mu));
        double vp = interp(pb, &Lp, V);
        double vm = interp(pb, &Lm, V);
        double term = (A * vp + B * vm) - (A + B) * Vi;
        acc = acc + term;
    }
    double Yb[3];
    if (drift_Y(pb, k, i, Yb)) {
        orc_land Lb;
        landing(pb, ix, Yb, &Lb);
        double C = 1.0 / Lb.mu;
        double vb = interp(pb, &Lb, V);
        acc = acc + (2.0 * C) * (vb - Vi);
    }
    return inv2h * acc;
}

/* ---------------------------------------------------------------------------
 * Exported entry points
 * ------------------------------------------------------------------------- */

/* (L-hat^{alpha_i} V)_i for every interior node (boundary entries set to 0). alpha == NULL: control k0 everywhere. */
void orc_lhat_apply(const orc_problem *pb, const int16_t *alpha, int32_t k0, const double *V, double *out) {
    int64_t N = pb->n[0] * (pb->dim > 1 ? pb->n[1] : 1) * (pb->dim > 2 ? pb->n[2] : 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int64_t ix[3];
        unflatten(pb, i, ix);
        if (!is_interior(pb, ix)) { out[i] = 0.0; continue; }
        int k = alpha ? alpha[i] : k0;
        out[i] = lhat_eval(pb, i, ix, k, V);
    }
}

/* Landing data for one point (exposed for tests of the truncation rule). */
void orc_landing(const orc_problem *pb, int64_t i, const double *Y, int64_t *cell, double *t, double *mu) {
    int64_t ix[3];
    double Yl[3] = {0, 0, 0};
    for (int d = 0; d < pb->dim; ++d) Yl[d] = Y[d];
    unflatten(pb, i, ix);
    orc_land L;
    landing(pb, ix, Yl, &L);
    for (int d = 0; d < pb->dim; ++d) { cell[d] = L.cell[d]; t[d] = L.t[d]; }
    *mu = L.mu;
}

static int64_t emit_point(const orc_problem *pb, const orc_land *L, double weight, int64_t *cols, double *vals) {
    int nc = 1 << pb->dim;
    for (int c = 0; c < nc; ++c) {
        cols[c] = corner_index(pb, L, c);
        vals[c] = weight * corner_weight(pb, L, c);
    }
    return nc;
}

/* Maximum number of entries orc_row can emit. */
int64_t orc_row_capacity(const orc_problem *pb) {
    return (int64_t)(2 * pb->P + 1) * (1 << pb->dim) + 1;
}

/* Row i of L-hat^k as (col, val) pairs with duplicates (eq. Lhat): sum_j val_j * V[col_j] = (L-hat^k V)_i. */
int64_t orc_row(const orc_problem *pb, int64_t i, int32_t k, int64_t *cols, double *vals) {
    int64_t ix[3];
    unflatten(pb, i, ix);
    double inv2h = 0.5 / pb->h;
    int64_t e = 0;
    double diag = 0.0;
    for (int p = 0; p < pb->P; ++p) {
        double Yp[3], Ym[3];
        diffusion_Y(pb, k, i, p, Yp);
        for (int d = 0; d < 3; ++d) Ym[d] = -Yp[d];
        orc_land Lp, Lm;
        landing(pb, ix, Yp, &Lp);
        landing(pb, ix, Ym, &Lm);
        double A = 2.0 / (Lp.mu * (Lp.mu + Lm.mu));
        double B = 2.0 / (Lm.mu * (Lm.mu + Lp.mu));
        e += emit_point(pb, &Lp, A * inv2h, cols + e, vals + e);
        e += emit_point(pb, &Lm, B * inv2h, cols + e, vals + e);
        diag -= (A + B) * inv2h;
    }
    double Yb[3];
    if (drift_Y(pb, k, i, Yb)) {
        orc_land Lb;
        landing(pb, ix, Yb, &Lb);
        double C = 1.0 / Lb.mu;
        e += emit_point(pb, &Lb, 2.0 * C * inv2h, cols + e, vals + e);
        diag -= 2.0 * C * inv2h;
    }
    cols[e] = i;
    vals[e] = diag;
    return e + 1;
}

/* Truncation weights of node i, control k: A[p], B[p], mu+[p], mu-[p] for p < P and C, mu_b for the drift. */
void orc_weights(const orc_problem *pb, int64_t i, int32_t k, double *A, double *B, double *mup, double *mum,
                 double *C, double *mub) {
    int64_t ix[3];
    unflatten(pb, i, ix);
    for (int p = 0; p < pb->P; ++p) {
        double Yp[3], Ym[3];
        diffusion_Y(pb, k, i, p, Yp);
        for (int d = 0; d < 3; ++d) Ym[d] = -Yp[d];
        orc_land Lp, Lm;
        landing(pb, ix, Yp, &Lp);
        landing(pb, ix, Ym, &Lm);
        A[p] = 2.0 / (Lp.mu * (Lp.mu + Lm.mu));
        B[p] = 2.0 / (Lm.mu * (Lm.mu + Lp.mu));
        mup[p] = Lp.mu;
        mum[p] = Lm.mu;
    }
    double Yb[3];
    *C = 1.0;
    *mub = 1.0;
    if (drift_Y(pb, k, i, Yb)) {
        orc_land Lb;
        landing(pb, ix, Yb, &Lb);
        *C = 1.0 / Lb.mu;
        *mub = Lb.mu;
    }
}

/* COO listing of L-hat^{alpha} over all interior rows.  Buffers sized N_int * orc_row_capacity.
   Row r of the output uses slots [r*cap, (r+1)*cap); unused slots get col = -1. */
void orc_assemble(const orc_problem *pb, const int16_t *alpha, const int64_t *rows, int64_t n_rows,
                  int64_t *cols, double *vals) {
    int64_t cap = orc_row_capacity(pb);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = rows[r];
        int64_t e = orc_row(pb, i, alpha[i], cols + r * cap, vals + r * cap);
        for (int64_t q = e; q < cap; ++q) { cols[r * cap + q] = -1; vals[r * cap + q] = 0.0; }
    }
}

/*
 * Policy improvement (Howard's algorithm applied to eq. nonlinear_sys).
 *
 * For every interior node and control k:
 *   G_k = theta*((Lhat^k X)_i + c_k X_i) + (1-theta)*((Lhat^k U)_i + c_k U_i) + f_{k,i}
 * The residual of row i of the discrete system is X_i - U_i - dt*G_k, so the
 * maximising control of eq. nonlinear_sys is the minimiser of G_k.
 * Tie rule: g* = min_k G_k; keep alpha_in if G_{alpha_in} <= g* + tau, otherwise
 * take the smallest k with G_k <= g* + tau.
 * Outputs (all optional except alpha_out): gmin = g*, margin = min{G_k - g* : G_k > g* + tau}
 * (INFINITY if none), ties = #{k : G_k <= g* + tau}.  Returns the number of changed controls.
 * f is given per (k, i) through strides (f_k = 0 for a control-independent source).
 */
int64_t orc_improve(const orc_problem *pb, const double *X, const double *U, double theta,
                    const double *f, int64_t f_k, int64_t f_i, double tau,
                    const int16_t *alpha_in, int16_t *alpha_out, double *gmin, double *margin, int32_t *ties) {
    int64_t N = pb->n[0] * (pb->dim > 1 ? pb->n[1] : 1) * (pb->dim > 2 ? pb->n[2] : 1);
    int64_t changed = 0;
    double omt = 1.0 - theta;
    int K = pb->K;
#pragma omp parallel
    {
        double *G = (double *)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(dynamic, 256) reduction(+ : changed)
        for (int64_t i = 0; i < N; ++i) {
            int64_t ix[3];
            unflatten(pb, i, ix);
            if (!is_interior(pb, ix)) {
                alpha_out[i] = -1;
                if (gmin) gmin[i] = 0.0;
                if (margin) margin[i] = INFINITY;
                if (ties) ties[i] = 0;
                continue;
            }
            double best = INFINITY;
            for (int k = 0; k < K; ++k) {
                double ck = coef_c(pb, k, i);
                double lx = lhat_eval(pb, i, ix, k, X);
                double lu = (omt != 0.0) ? lhat_eval(pb, i, ix, k, U) : 0.0;
                double g = theta * (lx + ck * X[i]) + omt * (lu + ck * U[i]) + f[k * f_k + i * f_i];
                G[k] = g;
                if (g < best) best = g;
            }
            double thr = best + tau;
            int cur = alpha_in ? alpha_in[i] : -1;
            int pick;
            if (cur >= 0 && cur < K && G[cur] <= thr) {
                pick = cur;
            } else {
                pick = 0;
                while (!(G[pick] <= thr)) ++pick;
            }
            alpha_out[i] = (int16_t)pick;
            if (pick != cur) changed += 1;
            if (gmin) gmin[i] = best;
            if (margin || ties) {
                double mg = INFINITY;
                int nt = 0;
                for (int k = 0; k < K; ++k) {
                    if (G[k] <= thr) nt++;
                    else if (G[k] - best < mg) mg = G[k] - best;
                }
                if (margin) margin[i] = mg;
                if (ties) ties[i] = nt;
            }
        }
        free(G);
    }
    return changed;
}

/* All K values G_k at one node (tests; brute-force checks of the search). */
void orc_node_values(const orc_problem *pb, int64_t i, const double *X, const double *U, double theta,
                     const double *f, int64_t f_k, int64_t f_i, double *G) {
    int64_t ix[3];
    unflatten(pb, i, ix);
    double omt = 1.0 - theta;
    for (int k = 0; k < pb->K; ++k) {
        double ck = coef_c(pb, k, i);
        double lx = lhat_eval(pb, i, ix, k, X);
        double lu = (omt != 0.0) ? lhat_eval(pb, i, ix, k, U) : 0.0;
        G[k] = theta * (lx + ck * X[i]) + omt * (lu + ck * U[i]) + f[k * f_k + i * f_i];
    }
}
