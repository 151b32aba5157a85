/*
 * abacus_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 reference for the near-field force of the
 * Abacus method (Garrison et al. 2021, "The Abacus Cosmological N-body Code").
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library; the product path never does.  It shares no code, header,
 * table or constant with the HIP implementation.
 *
 * What it computes (each function cites the passage it follows):
 *   oracle_bin     cell assignment, cell-relative offsets and a stable counting
 *                  sort by cell (Sec. 2.2 grid of K^3 cells; Sec. 3.5.1
 *                  positions stored as offsets from cell centres).
 *   oracle_forces  the near-field acceleration of selected sinks: a direct sum
 *                  over every particle in the (2R+1)^3 cells around the sink's
 *                  cell (Sec. 3.4.1), open boundary conditions on the periodic
 *                  image that lies in the neighbouring cell (Sec. 3.4.2), with
 *                  the spline-softened force of Eq. 3 and eps_s = 2.16 eps_p
 *                  (Sec. 3.2).
 *   oracle_force_abs  per sink, the sum of the absolute summands of that
 *                  acceleration and their number: the scale that bounds the
 *                  rounding of any summation order.
 *   oracle_vjp     the vector-Jacobian product of those accelerations with a
 *                  cotangent, binning frozen (derived from Eq. 3).
 *   oracle_fd      a central finite difference of the same loss (binning
 *                  frozen), used to pin oracle_vjp.
 *   oracle_density the apodized top-hat density estimate over the same near
 *                  field (Sec. 3.4.4).
 *   oracle_kick_drift  one leapfrog kick and drift (Sec. 3.1) with the per-cell
 *                  rms velocity and maximum acceleration of the time-step
 *                  criterion, Eq. 1; oracle_timestep evaluates Eq. 1.
 *   oracle_multipoles  the cell multipoles of Eq. 4 in the complete basis of
 *                  order p (Sec. 3.3.2), and their lossless reduction to
 *                  (p+1)^2 values per cell using the harmonic (trace-free)
 *                  property of the derivatives of 1/r.
 *
 * The force law is a parameter of oracle_forces, oracle_vjp and oracle_fd:
 * ORACLE_LAW_SPLINE is Eq. 3 with eps_s = 2.16 eps_p; ORACLE_LAW_PLUMMER is
 * Eq. 2, F = d / (r^2 + eps_p^2)^(3/2), with eps_p as given.
 *
 * Readings of the paper taken here (Eq. 3 gives F(r) with no sign, G or mass):
 *   - attractive force, d = x_j - x_i, G*m = 1 for every particle;
 *   - a particle never acts on itself; coincident particles (r = 0) give 0;
 *   - near-field membership is by periodic cell offset in [-R, R]^3 (Chebyshev
 *     distance in cells), K >= 2R+1 required;
 *   - positions with |x*K/L| >= 2^30 or non-finite are rejected.
 *
 * Build: cc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so every
 * product and sum below is one IEEE operation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_EPOS (-5)

/* The spline softening length is 2.16 times the Plummer-equivalent length
 * (Sec. 3.2, same minimum pairwise orbital time). */
static const double SPLINE_OVER_PLUMMER = 2.16;

#define ORACLE_LAW_SPLINE 0
#define ORACLE_LAW_PLUMMER 1

/* ------------------------------------------------------------------------- */
/* Cell assignment (Sec. 2.2, Sec. 3.5.1).                                     */
/* t = x * (K/L) in cell units; the unwrapped cell is floor(t); its periodic   */
/* index is that floor mod K; the offset from the cell centre is               */
/* t - (floor(t) + 1/2), rounded once to FP32.                                 */
/* ------------------------------------------------------------------------- */
static int cell_coord(float x, double cells_per_len, int64_t K, int64_t *unwrapped,
                      int64_t *wrapped, float *offset)
{
    double t = (double)x * cells_per_len;
    if (!isfinite(t) || fabs(t) >= 1073741824.0) return ORACLE_EPOS;
    double fl = floor(t);
    int64_t cu = (int64_t)fl;
    int64_t c = cu % K;
    if (c < 0) c += K;
    *unwrapped = cu;
    *wrapped = c;
    *offset = (float)(t - (fl + 0.5));
    return ORACLE_OK;
}

static int check_box(double L, int32_t K, int32_t R, double eps_p)
{
    if (!(L > 0.0) || !isfinite(L)) return ORACLE_EINVAL;
    if (R < 0 || K < 2 * R + 1) return ORACLE_EINVAL;
    if (!(eps_p > 0.0) || !isfinite(eps_p)) return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* Per-particle unwrapped and wrapped cell coordinates plus the linear cell id
 * (x slowest, z fastest: slabs along x, pencils along z). */
typedef struct {
    int64_t n, K;
    int64_t *cu;     /* n x 3 unwrapped cell coordinates */
    int32_t *cell;   /* n linear cell ids */
    int32_t *start;  /* K^3 + 1 offsets into order[] */
    int32_t *order;  /* n particle indices sorted by cell, stable */
} grid_t;

static void grid_free(grid_t *g)
{
    free(g->cu); free(g->cell); free(g->start); free(g->order);
    memset(g, 0, sizeof(*g));
}

static int grid_build(grid_t *g, int64_t n, const float *pos, double L, int64_t K,
                      float *rel /* optional n x 4 */)
{
    memset(g, 0, sizeof(*g));
    g->n = n; g->K = K;
    int64_t ncell = K * K * K;
    g->cu = (int64_t *)malloc(sizeof(int64_t) * (size_t)(3 * (n > 0 ? n : 1)));
    g->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    g->start = (int32_t *)calloc((size_t)(ncell + 1), sizeof(int32_t));
    g->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!g->cu || !g->cell || !g->start || !g->order) { grid_free(g); return ORACLE_ENOMEM; }
    double s = (double)K / L;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            float off;
            int rc = cell_coord(pos[3 * i + a], s, K, &g->cu[3 * i + a], &c[a], &off);
            if (rc) { grid_free(g); return rc; }
            if (rel) rel[4 * i + a] = off;
        }
        if (rel) rel[4 * i + 3] = 0.0f;
        g->cell[i] = (int32_t)((c[0] * K + c[1]) * K + c[2]);
    }
    /* counting sort: counts, exclusive prefix sum, placement in index order */
    for (int64_t i = 0; i < n; ++i) g->start[g->cell[i] + 1] += 1;
    for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
    if (!fill) { grid_free(g); return ORACLE_ENOMEM; }
    memcpy(fill, g->start, sizeof(int32_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; ++i) g->order[fill[g->cell[i]]++] = (int32_t)i;
    free(fill);
    return ORACLE_OK;
}

/*
 * oracle_bin: cell ids, cell offsets (K^3+1), the sorted order (slot -> original
 * index, ascending original index inside a cell) and the FP32 cell-relative
 * coordinates in sorted order (n x 4, 4th component 0).
 */
int oracle_bin(int64_t n, const float *pos, double L, int32_t K, int32_t *cell_out,
               int32_t *offsets_out, int32_t *perm_out, float *rel_out)
{
    if (n < 0 || (n > 0 && !pos) || !(L > 0.0) || !isfinite(L) || K < 1) return ORACLE_EINVAL;
    float *rel = (float *)malloc(sizeof(float) * (size_t)(4 * (n > 0 ? n : 1)));
    if (!rel) return ORACLE_ENOMEM;
    grid_t g;
    int rc = grid_build(&g, n, pos, L, K, rel);
    if (rc) { free(rel); return rc; }
    int64_t ncell = (int64_t)K * K * K;
    if (cell_out) memcpy(cell_out, g.cell, sizeof(int32_t) * (size_t)n);
    if (offsets_out) memcpy(offsets_out, g.start, sizeof(int32_t) * (size_t)(ncell + 1));
    if (perm_out) memcpy(perm_out, g.order, sizeof(int32_t) * (size_t)n);
    if (rel_out)
        for (int64_t s = 0; s < n; ++s)
            memcpy(&rel_out[4 * s], &rel[4 * (int64_t)g.order[s]], 4 * sizeof(float));
    free(rel);
    grid_free(&g);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Eq. 3, spline softening.  F(d) = f(r) d with                               */
/*   f = (10 - 15u + 6u^2) / eps^3   for u = r/eps < 1,                       */
/*   f = 1 / r^3                     otherwise.                               */
/* f_over_r_deriv is h = f'(r)/r, used by the Jacobian H = f I + h d d^T:      */
/*   h = (12u - 15) / (eps^4 r)      for u < 1,                               */
/*   h = -3 / r^5                    otherwise.                               */
/* ------------------------------------------------------------------------- */
static double spline_f(double r, double eps)
{
    double u = r / eps;
    if (u < 1.0) return (10.0 - 15.0 * u + 6.0 * u * u) / (eps * eps * eps);
    return 1.0 / (r * r * r);
}

static double spline_h(double r, double eps)
{
    double u = r / eps;
    if (u < 1.0) return (12.0 * u - 15.0) / (eps * eps * eps * eps * r);
    return -3.0 / (r * r * r * r * r);
}

/* Eq. 2, Plummer softening: F(d) = f(r) d with f = (r^2 + eps^2)^(-3/2), and
 * h = f'(r)/r = -3 (r^2 + eps^2)^(-5/2). */
static double plummer_f(double r, double eps)
{
    double s = r * r + eps * eps;
    return 1.0 / (s * sqrt(s));
}

static double plummer_h(double r, double eps)
{
    double s = r * r + eps * eps;
    return -3.0 / (s * s * sqrt(s));
}

/* The softening law selected by `law`, with its own softening length: the
 * spline's eps_s = 2.16 eps_p, or eps_p itself for Plummer. */
typedef struct { int law; double eps; } law_t;

static int make_law(int32_t law, double eps_p, law_t *out)
{
    if (law == ORACLE_LAW_SPLINE) { out->law = law; out->eps = SPLINE_OVER_PLUMMER * eps_p; return ORACLE_OK; }
    if (law == ORACLE_LAW_PLUMMER) { out->law = law; out->eps = eps_p; return ORACLE_OK; }
    return ORACLE_EINVAL;
}

static double law_f(const law_t *l, double r)
{
    return l->law == ORACLE_LAW_PLUMMER ? plummer_f(r, l->eps) : spline_f(r, l->eps);
}

static double law_h(const law_t *l, double r)
{
    return l->law == ORACLE_LAW_PLUMMER ? plummer_h(r, l->eps) : spline_h(r, l->eps);
}

/*
 * The image of source j seen from sink i: for each axis the integer shift m
 * that brings the unwrapped cell difference into [-R, R]; returns 0 if j is not
 * in the near field of i (some axis has no such shift).  The displacement is
 * d = (x_j + m L) - x_i in FP64.
 */
static int nf_displacement(const grid_t *g, const float *pos, double L, int64_t R,
                           int64_t i, int64_t j, double d[3])
{
    int64_t K = g->K;
    for (int a = 0; a < 3; ++a) {
        int64_t dc = g->cu[3 * j + a] - g->cu[3 * i + a];
        /* residue of dc in [-R, R] modulo K; unique because K >= 2R+1 */
        int64_t r = dc % K;
        if (r < 0) r += K;
        if (r > R) r -= K;
        if (r < -R || r > R) return 0;
        int64_t m = (r - dc) / K; /* exact: r - dc is a multiple of K */
        d[a] = ((double)pos[3 * j + a] + (double)m * L) - (double)pos[3 * i + a];
    }
    return 1;
}

/* Visit every near-field source j of sink i: the (2R+1)^3 cells around i's cell
 * (periodic in the cell index), every particle in them except i itself. */
typedef void (*pair_fn)(void *ctx, int64_t i, int64_t j, const double d[3]);

static int64_t visit_near_field(const grid_t *g, const float *pos, double L, int64_t R,
                                int64_t i, pair_fn fn, void *ctx)
{
    int64_t K = g->K, npairs = 0;
    int64_t ci[3];
    for (int a = 0; a < 3; ++a) {
        ci[a] = g->cu[3 * i + a] % K;
        if (ci[a] < 0) ci[a] += K;
    }
    for (int64_t ox = -R; ox <= R; ++ox)
        for (int64_t oy = -R; oy <= R; ++oy)
            for (int64_t oz = -R; oz <= R; ++oz) {
                int64_t cx = ((ci[0] + ox) % K + K) % K;
                int64_t cy = ((ci[1] + oy) % K + K) % K;
                int64_t cz = ((ci[2] + oz) % K + K) % K;
                int64_t c = (cx * K + cy) * K + cz;
                for (int32_t s = g->start[c]; s < g->start[c + 1]; ++s) {
                    int64_t j = g->order[s];
                    if (j == i) continue;
                    double d[3];
                    if (!nf_displacement(g, pos, L, R, i, j, d)) continue; /* never for K >= 2R+1 */
                    fn(ctx, i, j, d);
                    ++npairs;
                }
            }
    return npairs;
}

typedef struct { law_t law; double a[3]; } force_ctx;

static void force_pair(void *vctx, int64_t i, int64_t j, const double d[3])
{
    (void)i; (void)j;
    force_ctx *ctx = (force_ctx *)vctx;
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r == 0.0) return; /* coincident: F(0) = f(0) * 0 = 0 */
    double f = law_f(&ctx->law, r);
    for (int a = 0; a < 3; ++a) ctx->a[a] += f * d[a];
}

/*
 * oracle_forces: near-field acceleration (box units, G*m = 1, attractive) of the
 * sinks listed in sinks[0..nsink) (all particles if sinks == NULL, nsink == n).
 * acc is nsink x 3 FP64.  *npairs (optional) receives the number of ordered
 * (sink, source) pairs summed.
 */
int oracle_forces(int64_t n, const float *pos, double L, int32_t K, int32_t R, double eps_p,
                  int32_t law, int64_t nsink, const int64_t *sinks, double *acc, int64_t *npairs)
{
    int rc = check_box(L, K, R, eps_p);
    if (rc) return rc;
    force_ctx ctx;
    if ((rc = make_law(law, eps_p, &ctx.law))) return rc;
    if (n < 0 || nsink < 0 || (n > 0 && !pos) || (nsink > 0 && !acc)) return ORACLE_EINVAL;
    grid_t g;
    rc = grid_build(&g, n, pos, L, K, NULL);
    if (rc) return rc;
    int64_t total = 0;
    for (int64_t k = 0; k < nsink; ++k) {
        int64_t i = sinks ? sinks[k] : k;
        if (i < 0 || i >= n) { grid_free(&g); return ORACLE_EINVAL; }
        ctx.a[0] = ctx.a[1] = ctx.a[2] = 0.0;
        total += visit_near_field(&g, pos, L, R, i, force_pair, &ctx);
        for (int a = 0; a < 3; ++a) acc[3 * k + a] = ctx.a[a];
    }
    if (npairs) *npairs = total;
    grid_free(&g);
    return ORACLE_OK;
}

typedef struct { law_t law; double s[3]; } abs_ctx;

static void abs_pair(void *vctx, int64_t i, int64_t j, const double d[3])
{
    (void)i; (void)j;
    abs_ctx *ctx = (abs_ctx *)vctx;
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r == 0.0) return;
    double f = law_f(&ctx->law, r);
    for (int a = 0; a < 3; ++a) ctx->s[a] += fabs(f * d[a]);
}

/*
 * oracle_force_abs: for the listed sinks (all if NULL), the sum over the near
 * field of the absolute value of every summand of oracle_forces, per component,
 *   abs_out[k][a] = sum_{j in NF(i)} |f(r_ij) d_ij,a|   (box units),
 * and count_out[k] = the number of sources j summed (Sec. 3.4.1, Eq. 3).  Any
 * summation order of the same terms in a floating-point format with unit
 * roundoff u errs by at most about (count - 1) u abs_out (Higham's bound for
 * recursive summation), so this is the scale the FP32 sums are checked against.
 */
int oracle_force_abs(int64_t n, const float *pos, double L, int32_t K, int32_t R, double eps_p,
                     int32_t law, int64_t nsink, const int64_t *sinks, double *abs_out,
                     int64_t *count_out)
{
    int rc = check_box(L, K, R, eps_p);
    if (rc) return rc;
    abs_ctx ctx;
    if ((rc = make_law(law, eps_p, &ctx.law))) return rc;
    if (n < 0 || nsink < 0 || (n > 0 && !pos) || (nsink > 0 && (!abs_out || !count_out)))
        return ORACLE_EINVAL;
    grid_t g;
    rc = grid_build(&g, n, pos, L, K, NULL);
    if (rc) return rc;
    for (int64_t k = 0; k < nsink; ++k) {
        int64_t i = sinks ? sinks[k] : k;
        if (i < 0 || i >= n) { grid_free(&g); return ORACLE_EINVAL; }
        ctx.s[0] = ctx.s[1] = ctx.s[2] = 0.0;
        count_out[k] = visit_near_field(&g, pos, L, R, i, abs_pair, &ctx);
        for (int a = 0; a < 3; ++a) abs_out[3 * k + a] = ctx.s[a];
    }
    grid_free(&g);
    return ORACLE_OK;
}

typedef struct { law_t law; const float *w; double g[3]; } vjp_ctx;

static void vjp_pair(void *vctx, int64_t k, int64_t j, const double d[3])
{
    vjp_ctx *ctx = (vjp_ctx *)vctx;
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = (double)ctx->w[3 * j + a] - (double)ctx->w[3 * k + a];
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r == 0.0) {
        /* limit r -> 0: H = f(0) I, the d d^T term vanishes */
        double f0 = law_f(&ctx->law, 0.0);
        for (int a = 0; a < 3; ++a) ctx->g[a] += f0 * v[a];
        return;
    }
    double f = law_f(&ctx->law, r);
    double h = law_h(&ctx->law, r);
    double dv = d[0] * v[0] + d[1] * v[1] + d[2] * v[2];
    for (int a = 0; a < 3; ++a) ctx->g[a] += f * v[a] + h * dv * d[a];
}

/*
 * oracle_vjp: g_k = dL/dx_k for L = sum_i w_i . a_i with the binning frozen,
 *   g_k = sum_{j in NF(k)} H(d_kj) (w_j - w_k),   H = f I + h d d^T,
 * for the particles listed in sinks (all if NULL).  g is nsink x 3 FP64 in box
 * units (a is box units, so g has units of a / length).
 */
int oracle_vjp(int64_t n, const float *pos, const float *w, double L, int32_t K, int32_t R,
               double eps_p, int32_t law, int64_t nsink, const int64_t *sinks, double *g_out)
{
    int rc = check_box(L, K, R, eps_p);
    if (rc) return rc;
    vjp_ctx ctx;
    if ((rc = make_law(law, eps_p, &ctx.law))) return rc;
    if (n < 0 || nsink < 0 || (n > 0 && (!pos || !w)) || (nsink > 0 && !g_out)) return ORACLE_EINVAL;
    grid_t g;
    rc = grid_build(&g, n, pos, L, K, NULL);
    if (rc) return rc;
    ctx.w = w;
    for (int64_t q = 0; q < nsink; ++q) {
        int64_t k = sinks ? sinks[q] : q;
        if (k < 0 || k >= n) { grid_free(&g); return ORACLE_EINVAL; }
        ctx.g[0] = ctx.g[1] = ctx.g[2] = 0.0;
        visit_near_field(&g, pos, L, R, k, vjp_pair, &ctx);
        for (int a = 0; a < 3; ++a) g_out[3 * q + a] = ctx.g[a];
    }
    grid_free(&g);
    return ORACLE_OK;
}

typedef struct { law_t law; const float *w; int axis; double h; double sum; } fd_ctx;

static void fd_pair(void *vctx, int64_t k, int64_t j, const double d[3])
{
    fd_ctx *ctx = (fd_ctx *)vctx;
    double dm[3] = {d[0], d[1], d[2]}, dp[3] = {d[0], d[1], d[2]};
    dm[ctx->axis] -= ctx->h;
    dp[ctx->axis] += ctx->h;
    double rm = sqrt(dm[0] * dm[0] + dm[1] * dm[1] + dm[2] * dm[2]);
    double rp = sqrt(dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2]);
    double fm = rm == 0.0 ? 0.0 : law_f(&ctx->law, rm);
    double fp = rp == 0.0 ? 0.0 : law_f(&ctx->law, rp);
    for (int a = 0; a < 3; ++a) {
        double wk_minus_wj = (double)ctx->w[3 * k + a] - (double)ctx->w[3 * j + a];
        ctx->sum += wk_minus_wj * (fm * dm[a] - fp * dp[a]);
    }
}

/*
 * oracle_fd: central difference of L = sum_i w_i . a_i with respect to x_{k,axis}
 * at step h, binning and images frozen:
 *   D(h) = sum_{j in NF(k)} (w_k - w_j) . [F(d_kj - h e) - F(d_kj + h e)] / (2h),
 * which is exactly (L(x + h e_k) - L(x - h e_k)) / (2h) because F is odd and the
 * near-field relation is symmetric.
 */
int oracle_fd(int64_t n, const float *pos, const float *w, double L, int32_t K, int32_t R,
              double eps_p, int32_t law, int64_t k, int32_t axis, double h, double *out)
{
    int rc = check_box(L, K, R, eps_p);
    if (rc) return rc;
    fd_ctx ctx;
    if ((rc = make_law(law, eps_p, &ctx.law))) return rc;
    if (n <= 0 || !pos || !w || !out || k < 0 || k >= n || axis < 0 || axis > 2 || !(h > 0.0))
        return ORACLE_EINVAL;
    grid_t g;
    rc = grid_build(&g, n, pos, L, K, NULL);
    if (rc) return rc;
    ctx.w = w; ctx.axis = axis; ctx.h = h; ctx.sum = 0.0;
    visit_near_field(&g, pos, L, R, k, fd_pair, &ctx);
    *out = ctx.sum / (2.0 * h);
    grid_free(&g);
    return ORACLE_OK;
}

typedef struct { double b2; double sum; } density_ctx;

static void density_pair(void *vctx, int64_t i, int64_t j, const double d[3])
{
    (void)i; (void)j;
    density_ctx *ctx = (density_ctx *)vctx;
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 < ctx->b2) ctx->sum += 1.0 - r2 / ctx->b2;
}

/*
 * oracle_density: the apodized top-hat density estimate of Sec. 3.4.4 for the
 * listed sinks (all if NULL): rho_i = sum over j with r_ij < b of (1 - r_ij^2/b^2),
 * j running over the sink itself (r = 0, weight 1) and its near-field
 * neighbours.  Readings: the self term is included (the paper's GPU sum runs
 * over every particle of the sink's own cell, the sink included) and the
 * weight is normalised by b^2 so that an isolated particle has rho = 1.
 * Requires 0 < b <= R L/K, so that every particle within b is in the near field.
 */
int oracle_density(int64_t n, const float *pos, double L, int32_t K, int32_t R, double b,
                   int64_t nsink, const int64_t *sinks, double *rho)
{
    if (!(L > 0.0) || !isfinite(L) || R < 0 || K < 2 * R + 1) return ORACLE_EINVAL;
    if (!(b > 0.0) || !(b <= (double)R * L / (double)K)) return ORACLE_EINVAL;
    if (n < 0 || nsink < 0 || (n > 0 && !pos) || (nsink > 0 && !rho)) return ORACLE_EINVAL;
    grid_t g;
    int rc = grid_build(&g, n, pos, L, K, NULL);
    if (rc) return rc;
    density_ctx ctx;
    ctx.b2 = b * b;
    for (int64_t k = 0; k < nsink; ++k) {
        int64_t i = sinks ? sinks[k] : k;
        if (i < 0 || i >= n) { grid_free(&g); return ORACLE_EINVAL; }
        ctx.sum = 1.0; /* the sink itself */
        visit_near_field(&g, pos, L, R, i, density_pair, &ctx);
        rho[k] = ctx.sum;
    }
    grid_free(&g);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Cell multipoles, Eq. 4.                                                     */
/* ------------------------------------------------------------------------- */

/* Number of complete-basis terms (a, b, c), a + b + c <= p: (p+3)(p+2)(p+1)/6. */
int64_t oracle_multipole_terms(int32_t p, int32_t reduced)
{
    if (p < 0) return 0;
    if (reduced) return (int64_t)(p + 1) * (p + 1);
    return (int64_t)(p + 3) * (p + 2) * (p + 1) / 6;
}

/* Position of (a, b, c) in the complete basis, enumerated with a outermost and
 * c innermost (a = 0..p, b = 0..p-a, c = 0..p-a-b). */
static int64_t complete_index(int p, int a, int b, int c)
{
    int64_t k = 0;
    for (int aa = 0; aa <= p; ++aa)
        for (int bb = 0; bb <= p - aa; ++bb)
            for (int cc = 0; cc <= p - aa - bb; ++cc) {
                if (aa == a && bb == b && cc == c) return k;
                ++k;
            }
    return -1;
}

/* x^e for an integer e >= 0 by e successive multiplications (x^0 = 1). */
static double int_power(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r = r * x;
    return r;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

static double binomial(int n, int k)
{
    return factorial(n) / (factorial(k) * factorial(n - k));
}

/*
 * oracle_multipoles: for every cell of the K^3 grid, the complete multipoles of
 * Eq. 4, M^{a,b,c} = sum_q x_q^a y_q^b z_q^c over the particles q of the cell,
 * with (x_q, y_q, z_q) the particle's displacement from the cell centre in box
 * units: its stored FP32 cell-relative offset (as oracle_bin makes it) times
 * the cell width w = L/K.  Each summand is formed in FP64 straight from the
 * definition: the three integer powers x^a, y^b, z^c are computed separately
 * (int_power) and multiplied, then added to the term's sum.
 *
 * reduced != 0 instead returns (p+1)^2 values per cell: for c0 in {0, 1} and
 * a + b + c0 <= p (same enumeration order, c restricted to {0, 1}),
 *   R^{a,b,c0} = sum_{m>=0} sum_{i=0..m} (-1)^m C(m,i)
 *                 a! b! c0! / ((a-2i)! (b-2m+2i)! (c0+2m)!) M^{a-2i, b-2m+2i, c0+2m}
 * over the terms whose indices are non-negative.  This follows from the
 * expansion phi(r) = sum_q 1/|r - x_q| = sum (-1)^n M^{abc}/(a!b!c!) D_{abc}(r),
 * D_{abc} = d^a/dx^a d^b/dy^b d^c/dz^c (1/r): because 1/r is harmonic,
 * D_{a,b,c+2} = -D_{a+2,b,c} - D_{a,b+2,c}, so every D with c >= 2 is a
 * combination of those with c <= 1, and the reduced values give the same
 * phi(r) = sum_{c0<=1} (-1)^n R^{a,b,c0}/(a!b!c0!) D_{a,b,c0}(r).
 *
 * out is K^3 x terms FP64, cell-major, cell id (x K + y) K + z.
 */
int oracle_multipoles(int64_t n, const float *pos, double L, int32_t K, int32_t p,
                      int32_t reduced, double *out)
{
    if (n < 0 || (n > 0 && !pos) || !(L > 0.0) || !isfinite(L) || K < 1 || p < 0 || p > 16 || !out)
        return ORACLE_EINVAL;
    const int64_t ncell = (int64_t)K * K * K;
    const int64_t cml = oracle_multipole_terms(p, 0);
    double *M = (double *)calloc((size_t)(ncell * cml), sizeof(double));
    float *rel = (float *)malloc(sizeof(float) * (size_t)(4 * (n > 0 ? n : 1)));
    if (!M || !rel) { free(M); free(rel); return ORACLE_ENOMEM; }
    grid_t g;
    int rc = grid_build(&g, n, pos, L, K, rel);
    if (rc) { free(M); free(rel); return rc; }
    /* the (a, b, c) of every complete-basis term, in output order */
    int *ta = (int *)malloc(sizeof(int) * (size_t)cml);
    int *tb = (int *)malloc(sizeof(int) * (size_t)cml);
    int *tc = (int *)malloc(sizeof(int) * (size_t)cml);
    if (!ta || !tb || !tc) {
        free(ta); free(tb); free(tc); free(M); free(rel); grid_free(&g);
        return ORACLE_ENOMEM;
    }
    for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p - a; ++b)
            for (int cc = 0; cc <= p - a - b; ++cc) {
                const int64_t k = complete_index(p, a, b, cc);
                ta[k] = a;
                tb[k] = b;
                tc[k] = cc;
            }
    const double w = L / (double)K;
    for (int64_t c = 0; c < ncell; ++c) {
        double *Mc = M + c * cml;
        for (int32_t s = g.start[c]; s < g.start[c + 1]; ++s) {
            const int64_t q = g.order[s];
            const double X = (double)rel[4 * q + 0] * w;
            const double Y = (double)rel[4 * q + 1] * w;
            const double Z = (double)rel[4 * q + 2] * w;
            for (int64_t k = 0; k < cml; ++k)
                Mc[k] += int_power(X, ta[k]) * int_power(Y, tb[k]) * int_power(Z, tc[k]);
        }
    }
    free(ta);
    free(tb);
    free(tc);
    if (!reduced) {
        memcpy(out, M, sizeof(double) * (size_t)(ncell * cml));
    } else {
        const int64_t rml = oracle_multipole_terms(p, 1);
        for (int64_t c = 0; c < ncell; ++c) {
            const double *Mc = M + c * cml;
            double *Rc = out + c * rml;
            int64_t k = 0;
            for (int a = 0; a <= p; ++a)
                for (int b = 0; b <= p - a; ++b)
                    for (int c0 = 0; c0 <= 1 && c0 <= p - a - b; ++c0) {
                        double sum = 0.0;
                        for (int m = 0; 2 * m <= a + b; ++m)
                            for (int i = 0; i <= m; ++i) {
                                const int sa = a - 2 * i, sb = b - 2 * (m - i), sc = c0 + 2 * m;
                                if (sa < 0 || sb < 0) continue;
                                const double coef = (m % 2 ? -1.0 : 1.0) * binomial(m, i) *
                                                    factorial(a) * factorial(b) * factorial(c0) /
                                                    (factorial(sa) * factorial(sb) * factorial(sc));
                                sum += coef * Mc[complete_index(p, sa, sb, sc)];
                            }
                        Rc[k++] = sum;
                    }
        }
    }
    free(M);
    free(rel);
    grid_free(&g);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Kick, drift and the time-step statistics (Sec. 3.1, Eq. 1).                 */
/* ------------------------------------------------------------------------- */

/* Periodic wrap of an FP64 coordinate into [0, L), rounded to FP32; a value
 * that rounds up to L becomes 0. */
static float wrap_coord(double t, double L)
{
    double q = floor(t / L);
    double r = t - q * L;
    if (r < 0.0) r += L;
    if (r >= L) r -= L;
    float f = (float)r;
    if (f >= (float)L) f = 0.0f;
    return f;
}

/*
 * oracle_kick_drift: for every particle (FP32 state, each update formed in FP64
 * and rounded once to FP32, no fused multiply-add):
 *   kick   v' = v + kick * a       (the velocity moves a full step, from the
 *                                   half step before to the half step after)
 *   drift  x' = wrap(x + drift * v')
 * and, per cell of the grid that x (before the drift) falls in,
 *   cell_stats[2c]   = v_rms = sqrt(sum |v'|^2 / n_c)  (mean not subtracted)
 *   cell_stats[2c+1] = a_max = max |a|                 (0 for an empty cell)
 * plus box_stats = {min over cells with n_c > 0 and a_max > 0 of v_rms/a_max
 * (+inf if none), global v_rms = sqrt(sum |v'|^2 / N), global a_max, N}.
 * |a| = sqrt(ax^2 + ay^2 + az^2) in FP64.  pos_out/vel_out may equal pos/vel.
 */
int oracle_kick_drift(int64_t n, const float *pos, const float *vel, const float *acc, double L,
                      int32_t K, double kick, double drift, float *pos_out, float *vel_out,
                      double *cell_stats, double *box_stats)
{
    if (n < 0 || (n > 0 && (!pos || !vel || !acc || !pos_out || !vel_out)) || !(L > 0.0) ||
        !isfinite(L) || K < 1 || !isfinite(kick) || !isfinite(drift))
        return ORACLE_EINVAL;
    grid_t g;
    int rc = grid_build(&g, n, pos, L, K, NULL);
    if (rc) return rc;
    const int64_t ncell = (int64_t)K * K * K;
    double *sumsq = (double *)calloc((size_t)ncell, sizeof(double));
    double *amax = (double *)calloc((size_t)ncell, sizeof(double));
    if (!sumsq || !amax) { free(sumsq); free(amax); grid_free(&g); return ORACLE_ENOMEM; }
    double total_sq = 0.0, global_amax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        float vn[3];
        double v2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            vn[a] = (float)((double)vel[3 * i + a] + kick * (double)acc[3 * i + a]);
            v2 += (double)vn[a] * (double)vn[a];
        }
        const double ax = acc[3 * i], ay = acc[3 * i + 1], az = acc[3 * i + 2];
        const double am = sqrt(ax * ax + ay * ay + az * az);
        const int32_t c = g.cell[i];
        sumsq[c] += v2;
        if (am > amax[c]) amax[c] = am;
        total_sq += v2;
        if (am > global_amax) global_amax = am;
        for (int a = 0; a < 3; ++a) {
            pos_out[3 * i + a] = wrap_coord((double)pos[3 * i + a] + drift * (double)vn[a], L);
            vel_out[3 * i + a] = vn[a];
        }
    }
    double min_ratio = INFINITY;
    for (int64_t c = 0; c < ncell; ++c) {
        const int32_t nc = g.start[c + 1] - g.start[c];
        const double vr = nc > 0 ? sqrt(sumsq[c] / (double)nc) : 0.0;
        if (cell_stats) {
            cell_stats[2 * c] = vr;
            cell_stats[2 * c + 1] = amax[c];
        }
        if (nc > 0 && amax[c] > 0.0 && vr / amax[c] < min_ratio) min_ratio = vr / amax[c];
    }
    if (box_stats) {
        box_stats[0] = min_ratio;
        box_stats[1] = n > 0 ? sqrt(total_sq / (double)n) : 0.0;
        box_stats[2] = global_amax;
        box_stats[3] = (double)n;
    }
    free(sumsq);
    free(amax);
    grid_free(&g);
    return ORACLE_OK;
}

/* Eq. 1: the global step in scale factor,
 *   da = min(eta_H a, eta_acc a H max(min_c [v_rms/a_max]_c, v_rms,global / a_max,global)),
 * from box_stats as oracle_kick_drift returns them (a ratio with a_max = 0 is
 * +inf and leaves the other terms to decide). */
double oracle_timestep(const double *box_stats, double a, double H, double eta_acc, double eta_H)
{
    const double global = box_stats[2] > 0.0 ? box_stats[1] / box_stats[2] : INFINITY;
    const double ratio = box_stats[0] > global ? box_stats[0] : global;
    const double acc_step = eta_acc * a * H * ratio;
    const double hubble_step = eta_H * a;
    return acc_step < hubble_step ? acc_step : hubble_step;
}

/* The softening conversion constant, exported so tests can check it. */
double oracle_spline_over_plummer(void) { return SPLINE_OVER_PLUMMER; }

/* Eq. 3 for one separation, exported for the closed-form tests. */
double oracle_pair_f(double r, double eps_s) { return spline_f(r, eps_s); }
double oracle_pair_h(double r, double eps_s) { return spline_h(r, eps_s); }
/* Eq. 2 for one separation. */
double oracle_plummer_f(double r, double eps_p) { return plummer_f(r, eps_p); }
double oracle_plummer_h(double r, double eps_p) { return plummer_h(r, eps_p); }
