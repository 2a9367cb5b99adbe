/*
 * FP64 CPU oracle for sparse-matrix parallel-beam CT reconstruction.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library.  It shares no
 * code with the GPU library: every routine below is written out from the
 * paper and from the plain definitions of the operations it composes.
 *
 * What it computes (Barnard & Archibald, "Accelerating optimization-based
 * computed tomography via sparse matrix approximations"):
 *   - the parallel-beam Radon transform R (Section 1, the data term of
 *     eq:objmin) as an exact ray/pixel intersection-length matrix (Siddon,
 *     Med. Phys. 12(2) 1985), the angle row selector M, and R^T;
 *   - plain CSR products y = (MR)x and x = (MR)^T y;
 *   - the forward-difference gradient K with Neumann boundary and K^T;
 *   - the normal operator A = alpha R^T M^T M R + lambda K^T K + sigma I that
 *     appears in eq:KKT (sigma = 0), eq:SB_solve (sigma = 0) and
 *     eq:PD_resolve (alpha <- tau*alpha, lambda = 0, sigma = 1), Section 2;
 *   - textbook conjugate gradients on A (Section 2: the systems have no
 *     closed form and are solved iteratively);
 *   - anisotropic-TV split Bregman (Goldstein-Osher; set-up of Section 4);
 *   - losses and their gradients, including a reverse sweep through a fixed
 *     number of unrolled CG iterations.
 *
 * Geometry reading (the paper does not fix it): unit pixels on [-N/2, N/2]^2,
 * pixel (iy, ix) = [ix - N/2, ix - N/2 + 1) x [iy - N/2, iy - N/2 + 1), flat
 * index iy*N + ix; angles theta_k = pi*k/n_a with cos/sin reduced so that
 * 0, pi/4, pi/2 are exact and cos(pi - theta) = -cos(theta) exactly; bins
 * s_b = b - (n_b - 1)/2; ray (k, b) is the line {p : p . w = s_b},
 * w = (cos, sin), parametrised p(t) = s_b w + t w_perp, w_perp = (-sin, cos).
 * A ray lying exactly on a pixel edge (only possible at theta = 0 or pi/2)
 * gives half of each length to each of the two pixels sharing the edge;
 * segment lengths <= 1e-12 are dropped.
 *
 * Floating point: plain double, sequential sums in index order.  Build
 * without -ffast-math and without FMA contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SLIVER 1e-12

/* ------------------------------------------------------------------ */
/* Geometry                                                             */
/* ------------------------------------------------------------------ */

/* cos/sin of pi*k/na, reduced to [0, pi/4] so that symmetric angles get
 * values that are exact mirror images of each other. */
void ora_trig(int k, int na, double *c_out, double *s_out)
{
    double c, s;
    int kk = k;
    int flip = 0;                 /* theta > pi/2: cos changes sign */
    if (2 * kk > na) { kk = na - kk; flip = 1; }
    if (kk == 0) { c = 1.0; s = 0.0; }
    else if (2 * kk == na) { c = 0.0; s = 1.0; }
    else if (4 * kk == na) { c = sqrt(0.5); s = sqrt(0.5); }
    else if (4 * kk > na) {
        /* theta' in (pi/4, pi/2): use the complement pi/2 - theta' */
        double phi = M_PI * (double)(na - 2 * kk) / (2.0 * (double)na);
        c = sin(phi); s = cos(phi);
    } else {
        double th = M_PI * (double)kk / (double)na;
        c = cos(th); s = sin(th);
    }
    if (flip) c = -c;
    *c_out = c; *s_out = s;
}

typedef struct { int32_t j; double v; } ora_ent;

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

static int cmp_ent(const void *a, const void *b)
{
    int32_t x = ((const ora_ent *)a)->j, y = ((const ora_ent *)b)->j;
    return (x > y) - (x < y);
}

/* Entries of ray (k, b), sorted by pixel, duplicates summed.  tbuf must hold
 * 2n+2 doubles and ebuf 2n+2 entries (the axis-aligned edge case needs 2n). */
static int ray_entries(int n, int na, int nb, int k, int b, double *tbuf, ora_ent *ebuf)
{
    double c, s;
    ora_trig(k, na, &c, &s);
    const double sb = (double)b - 0.5 * (double)(nb - 1);
    const double h = 0.5 * (double)n;
    int m = 0;

    if (s == 0.0 || c == 0.0) {
        /* Axis-aligned ray: theta = 0 gives the vertical line x = sb,
         * theta = pi/2 the horizontal line y = sb.  pos is the line's
         * coordinate measured in pixel units from the image's low edge. */
        const int vertical = (s == 0.0);
        const double pos = (vertical ? sb * c : sb * s) + h;
        if (pos == floor(pos)) {
            /* on the edge between pixel lines e-1 and e: split 50/50 */
            const long e = (long)pos;
            if (e < 0 || e > n) return 0;
            if (vertical) {
                for (int iy = 0; iy < n; ++iy) {
                    if (e - 1 >= 0) { ebuf[m].j = iy * n + (int)(e - 1); ebuf[m].v = 0.5; ++m; }
                    if (e < n) { ebuf[m].j = iy * n + (int)e; ebuf[m].v = 0.5; ++m; }
                }
            } else {
                if (e - 1 >= 0)
                    for (int ix = 0; ix < n; ++ix) { ebuf[m].j = (int)(e - 1) * n + ix; ebuf[m].v = 0.5; ++m; }
                if (e < n)
                    for (int ix = 0; ix < n; ++ix) { ebuf[m].j = (int)e * n + ix; ebuf[m].v = 0.5; ++m; }
            }
            return m;
        }
        if (!(pos > 0.0 && pos < (double)n)) return 0;
        const int q = (int)floor(pos);
        for (int r = 0; r < n; ++r) {
            ebuf[m].j = vertical ? r * n + q : q * n + r;
            ebuf[m].v = 1.0;
            ++m;
        }
        return m;
    }

    /* General ray: x(t) = sb*c - t*s, y(t) = sb*s + t*c. */
    const double sc = sb * c, ss = sb * s;
    const double tx0 = (sc - (-h)) / s, tx1 = (sc - h) / s;
    const double ty0 = ((-h) - ss) / c, ty1 = (h - ss) / c;
    const double tin = fmax(fmin(tx0, tx1), fmin(ty0, ty1));
    const double tout = fmin(fmax(tx0, tx1), fmax(ty0, ty1));
    if (!(tout - tin > SLIVER)) return 0;

    int nt = 0;
    tbuf[nt++] = tin;
    for (int q = 1; q < n; ++q) {                 /* interior vertical lines */
        const double X = (double)q - h;
        const double t = (sc - X) / s;
        if (t > tin && t < tout) tbuf[nt++] = t;
    }
    for (int q = 1; q < n; ++q) {                 /* interior horizontal lines */
        const double Y = (double)q - h;
        const double t = (Y - ss) / c;
        if (t > tin && t < tout) tbuf[nt++] = t;
    }
    tbuf[nt++] = tout;
    qsort(tbuf, (size_t)nt, sizeof(double), cmp_double);

    for (int i = 0; i + 1 < nt; ++i) {
        const double ta = tbuf[i], tb = tbuf[i + 1];
        const double len = tb - ta;
        if (!(len > SLIVER)) continue;
        const double tm = 0.5 * (ta + tb);
        const double px = sc - tm * s, py = ss + tm * c;
        int ix = (int)floor(px + h), iy = (int)floor(py + h);
        if (ix < 0) ix = 0;
        if (ix > n - 1) ix = n - 1;
        if (iy < 0) iy = 0;
        if (iy > n - 1) iy = n - 1;
        ebuf[m].j = iy * n + ix;
        ebuf[m].v = len;
        ++m;
    }
    qsort(ebuf, (size_t)m, sizeof(ora_ent), cmp_ent);
    int w = 0;
    for (int i = 0; i < m; ++i) {
        if (w > 0 && ebuf[w - 1].j == ebuf[i].j) ebuf[w - 1].v += ebuf[i].v;
        else ebuf[w++] = ebuf[i];
    }
    return w;
}

/* One ray's entries into caller arrays of capacity 2n+2; returns the count. */
int ora_ray(int n, int na, int nb, int k, int b, int32_t *cols, double *vals)
{
    double *tbuf = (double *)malloc(sizeof(double) * (size_t)(2 * n + 4));
    ora_ent *ebuf = (ora_ent *)malloc(sizeof(ora_ent) * (size_t)(2 * n + 4));
    int m = ray_entries(n, na, nb, k, b, tbuf, ebuf);
    for (int i = 0; i < m; ++i) { cols[i] = ebuf[i].j; vals[i] = ebuf[i].v; }
    free(tbuf);
    free(ebuf);
    return m;
}

/* CSR of R over the listed angles (rows = angle-list order x bins).
 * Pass col == NULL to only fill row_ptr (counts + prefix). */
void ora_build(int n, int na, int nb, int n_list, const int32_t *angles,
               int64_t *row_ptr, int32_t *col, double *val)
{
    const int64_t rows = (int64_t)n_list * nb;
    if (col == NULL) {
        row_ptr[0] = 0;
        int64_t *cnt = row_ptr + 1;
#pragma omp parallel
        {
            double *tbuf = (double *)malloc(sizeof(double) * (size_t)(2 * n + 4));
            ora_ent *ebuf = (ora_ent *)malloc(sizeof(ora_ent) * (size_t)(2 * n + 4));
#pragma omp for schedule(dynamic, 16)
            for (int64_t r = 0; r < rows; ++r)
                cnt[r] = ray_entries(n, na, nb, angles[r / nb], (int)(r % nb), tbuf, ebuf);
            free(tbuf);
            free(ebuf);
        }
        for (int64_t r = 0; r < rows; ++r) row_ptr[r + 1] += row_ptr[r];
        return;
    }
#pragma omp parallel
    {
        double *tbuf = (double *)malloc(sizeof(double) * (size_t)(2 * n + 4));
        ora_ent *ebuf = (ora_ent *)malloc(sizeof(ora_ent) * (size_t)(2 * n + 4));
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < rows; ++r) {
            int m = ray_entries(n, na, nb, angles[r / nb], (int)(r % nb), tbuf, ebuf);
            int64_t o = row_ptr[r];
            for (int i = 0; i < m; ++i) { col[o + i] = ebuf[i].j; val[o + i] = ebuf[i].v; }
        }
        free(tbuf);
        free(ebuf);
    }
}

/* Counting-sort transpose: rows of the result are columns of the input, each
 * holding its entries in ascending input-row order. */
void ora_transpose(int64_t rows, int64_t cols, const int64_t *rp, const int32_t *ci,
                   const double *v, int64_t *trp, int32_t *tci, double *tv)
{
    memset(trp, 0, sizeof(int64_t) * (size_t)(cols + 1));
    for (int64_t e = 0; e < rp[rows]; ++e) trp[ci[e] + 1]++;
    for (int64_t j = 0; j < cols; ++j) trp[j + 1] += trp[j];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cols > 0 ? cols : 1));
    memcpy(fill, trp, sizeof(int64_t) * (size_t)cols);
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t o = fill[ci[e]]++;
            tci[o] = (int32_t)i;
            tv[o] = v[e];
        }
    free(fill);
}

/* ------------------------------------------------------------------ */
/* Linear algebra                                                       */
/* ------------------------------------------------------------------ */

/* y = A x for a CSR matrix, each row summed in stored order. */
void ora_spmv(int64_t rows, const int64_t *rp, const int32_t *ci, const double *v,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i) {
        double acc = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * x[ci[e]];
        y[i] = acc;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* K u = (D_x u, D_y u), forward differences, zero last difference. */
void ora_grad(int n, const double *u, double *gx, double *gy)
{
#pragma omp parallel for schedule(static)
    for (int iy = 0; iy < n; ++iy)
        for (int ix = 0; ix < n; ++ix) {
            const int64_t j = (int64_t)iy * n + ix;
            gx[j] = (ix < n - 1) ? u[j + 1] - u[j] : 0.0;
            gy[j] = (iy < n - 1) ? u[j + n] - u[j] : 0.0;
        }
}

/* K^T (vx, vy): the exact transpose of ora_grad. */
void ora_gradT(int n, const double *vx, const double *vy, double *out)
{
#pragma omp parallel for schedule(static)
    for (int iy = 0; iy < n; ++iy)
        for (int ix = 0; ix < n; ++ix) {
            const int64_t j = (int64_t)iy * n + ix;
            double a = 0.0;
            if (ix >= 1) a += vx[j - 1];
            if (ix <= n - 2) a -= vx[j];
            if (iy >= 1) a += vy[j - n];
            if (iy <= n - 2) a -= vy[j];
            out[j] = a;
        }
}

/* The measured-ray operator: MR and (MR)^T as two CSR matrices. */
typedef struct {
    int32_t n;
    int64_t rows;                  /* measured rays */
    const int64_t *rp; const int32_t *ci; const double *v;     /* MR      */
    const int64_t *trp; const int32_t *tci; const double *tv;  /* (MR)^T  */
    int32_t sur_r;                 /* >= 0: R^T M^T M R is replaced by the surrogate T */
    const double *sur_w;           /* T's weights, (2 sur_r + 1)^2, row-major in (dy, dx) */
} ora_op;

/* Surrogate operator of Section 3.2 (eq:def_sparse_surr): T is the sum over
 * all pixels q of the point-spread function P = R^T M^T M R e_c of the centre
 * pixel c, moved to q and cut to the disc of radius r around q; entries that
 * fall outside the image are dropped (the suppression of the opposite edge).
 * So (T x)_p = sum over |d| <= r with p - d inside the image of
 * w(d) x_{p - d}, w(d) = P_{c + d}.  Weights outside the disc are zero. */
void ora_stencil(int n, int r, const double *w, const double *x, double *out)
{
    const int k = 2 * r + 1;
    for (int py = 0; py < n; ++py)
        for (int px = 0; px < n; ++px) {
            double acc = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    const int qy = py - dy, qx = px - dx;
                    if (qy < 0 || qy >= n || qx < 0 || qx >= n) continue;
                    acc += w[(dy + r) * k + (dx + r)] * x[(int64_t)qy * n + qx];
                }
            out[(int64_t)py * n + px] = acc;
        }
}

/* The weights w(d) = P_{c + d} for |d| <= r (Euclidean), c = (n/2, n/2),
 * P = R^T M^T M R e_c; symmetrized as (w(d) + w(-d)) / 2 so that T is
 * symmetric (the surrogate system is solved by CG).  w has (2r+1)^2 entries;
 * returns -1 if the disc does not fit in the image. */
int ora_surrogate_weights(const ora_op *op, int r, double *w)
{
    const int n = op->n, k = 2 * r + 1, cy = n / 2, cx = n / 2;
    if (r < 0 || cy - r < 0 || cy + r >= n || cx - r < 0 || cx + r >= n) return -1;
    const int64_t nn = (int64_t)n * n;
    double *e = (double *)calloc((size_t)nn, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * (size_t)op->rows);
    double *P = (double *)malloc(sizeof(double) * (size_t)nn);
    e[(int64_t)cy * n + cx] = 1.0;
    ora_spmv(op->rows, op->rp, op->ci, op->v, e, y);
    ora_spmv(nn, op->trp, op->tci, op->tv, y, P);
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            double v = 0.0;
            if (dy * dy + dx * dx <= r * r)
                v = 0.5 * (P[(int64_t)(cy + dy) * n + (cx + dx)] + P[(int64_t)(cy - dy) * n + (cx - dx)]);
            w[(dy + r) * k + (dx + r)] = v;
        }
    free(e); free(y); free(P);
    return 0;
}

/* scratch: rows + 4*n*n doubles */
static void normal_apply(const ora_op *op, double alpha, double lambda, double sigma,
                         const double *x, double *out, double *scratch)
{
    const int64_t nn = (int64_t)op->n * op->n;
    double *y = scratch, *t = scratch + op->rows;
    double *gx = t + nn, *gy = gx + nn, *ktk = gy + nn;
    if (op->sur_r >= 0) {
        ora_stencil(op->n, op->sur_r, op->sur_w, x, t);
    } else {
        ora_spmv(op->rows, op->rp, op->ci, op->v, x, y);
        ora_spmv(nn, op->trp, op->tci, op->tv, y, t);
    }
    ora_grad(op->n, x, gx, gy);
    ora_gradT(op->n, gx, gy, ktk);
    for (int64_t j = 0; j < nn; ++j) out[j] = alpha * t[j] + lambda * ktk[j] + sigma * x[j];
}

void ora_normal(const ora_op *op, double alpha, double lambda, double sigma,
                const double *x, double *out)
{
    const int64_t nn = (int64_t)op->n * op->n;
    double *scratch = (double *)malloc(sizeof(double) * (size_t)(op->rows + 4 * nn));
    normal_apply(op, alpha, lambda, sigma, x, out, scratch);
    free(scratch);
}

/* Conjugate gradients on A(alpha, lambda, sigma) from x (in/out) with the
 * given starting residual r (in/out).  rho_hist gets rho_0..rho_n_iter (the
 * squared residual norm after each iteration; entries after a stop repeat
 * the last value).  Returns the number of iterations that changed x; sets
 * *breakdown to the iteration index + 1 at which <p, Ap> <= 0 or non-finite
 * (0 if none).  rtol > 0 stops once sqrt(rho) <= rtol*sqrt(rho_0). */
int ora_cg(const ora_op *op, double alpha, double lambda, double sigma,
           double *x, double *r, int n_iter, double rtol, double *rho_hist, int *breakdown)
{
    const int64_t nn = (int64_t)op->n * op->n;
    double *p = (double *)malloc(sizeof(double) * (size_t)nn);
    double *q = (double *)malloc(sizeof(double) * (size_t)nn);
    double *scratch = (double *)malloc(sizeof(double) * (size_t)(op->rows + 4 * nn));
    memcpy(p, r, sizeof(double) * (size_t)nn);
    double rho = dot(nn, r, r);
    const double rho0 = rho;
    int done = 0;
    *breakdown = 0;
    if (rho_hist) rho_hist[0] = rho;
    for (int it = 0; it < n_iter; ++it) {
        int stop = (rho == 0.0) || (rtol > 0.0 && sqrt(rho) <= rtol * sqrt(rho0));
        if (!stop) {
            normal_apply(op, alpha, lambda, sigma, p, q, scratch);
            const double gamma = dot(nn, p, q);
            if (!(gamma > 0.0) || !isfinite(gamma)) { *breakdown = it + 1; stop = 1; }
            else {
                const double a = rho / gamma;
                for (int64_t j = 0; j < nn; ++j) { x[j] += a * p[j]; r[j] -= a * q[j]; }
                const double rho_new = dot(nn, r, r);
                const double beta = rho_new / rho;
                for (int64_t j = 0; j < nn; ++j) p[j] = r[j] + beta * p[j];
                rho = rho_new;
                ++done;
            }
        }
        if (rho_hist) rho_hist[it + 1] = rho;
        if (stop) {
            for (int j = it + 2; j <= n_iter; ++j) if (rho_hist) rho_hist[j] = rho;
            break;
        }
    }
    free(p); free(q); free(scratch);
    return done;
}

static double shrink(double z, double g)
{
    const double a = fabs(z) - g;
    if (a <= 0.0) return 0.0;
    return z > 0.0 ? a : -a;
}

/* Anisotropic-TV split Bregman (Goldstein-Osher), one CG solve of n_cg steps
 * per outer iteration on (alpha R^T M^T M R + lambda K^T K) u = alpha R^T M^T f
 * + lambda K^T (d - b), warm-started from the previous u with the residual
 * carried across outer iterations.
 *   f: measured sinogram (rows entries); u: in/out (in is the start when
 *   warm != 0, else zeroed);  state (optional, 5*n*n): d_x, d_y, b_x, b_y, r
 *   in/out when resume != 0.
 *   upd_b[k] = ||b^{k+1} - b^k||_1, upd_u[k] = ||u^{k+1} - u^k||_1.
 *   Stops after the first outer iteration whose upd_b < tol * upd_b[0]
 *   (tol > 0).  Returns the number of outer iterations run. */
int ora_sb(const ora_op *op, double alpha, double lambda, int n_outer, int n_cg, double tol,
           const double *f, double *u, int warm, double *state, int resume,
           double *upd_b, double *upd_u)
{
    const int n = op->n;
    const int64_t nn = (int64_t)n * n;
    double *own = NULL;
    if (!state) { own = (double *)calloc((size_t)(5 * nn), sizeof(double)); state = own; }
    double *dx = state, *dy = state + nn, *bx = state + 2 * nn, *by = state + 3 * nn;
    double *r = state + 4 * nn;
    double *gx = (double *)malloc(sizeof(double) * (size_t)nn);
    double *gy = (double *)malloc(sizeof(double) * (size_t)nn);
    double *wx = (double *)malloc(sizeof(double) * (size_t)nn);
    double *wy = (double *)malloc(sizeof(double) * (size_t)nn);
    double *kt = (double *)malloc(sizeof(double) * (size_t)nn);
    double *uprev = (double *)malloc(sizeof(double) * (size_t)nn);
    double *rho_hist = (double *)malloc(sizeof(double) * (size_t)(n_cg + 1));

    if (!resume) {
        memset(state, 0, sizeof(double) * (size_t)(4 * nn));
        if (!warm) memset(u, 0, sizeof(double) * (size_t)nn);
        /* r = alpha (MR)^T f - A u   (d = b = 0) */
        ora_spmv(nn, op->trp, op->tci, op->tv, f, r);
        for (int64_t j = 0; j < nn; ++j) r[j] *= alpha;
        if (warm) {
            ora_normal(op, alpha, lambda, 0.0, u, kt);
            for (int64_t j = 0; j < nn; ++j) r[j] -= kt[j];
        }
    }
    int k;
    for (k = 0; k < n_outer; ++k) {
        memcpy(uprev, u, sizeof(double) * (size_t)nn);
        for (int64_t j = 0; j < nn; ++j) { wx[j] = dx[j] - bx[j]; wy[j] = dy[j] - by[j]; }
        int bd = 0;
        ora_cg(op, alpha, lambda, 0.0, u, r, n_cg, 0.0, rho_hist, &bd);
        ora_grad(n, u, gx, gy);
        double ub = 0.0, uu = 0.0;
        for (int64_t j = 0; j < nn; ++j) {
            const double ndx = shrink(gx[j] + bx[j], 1.0 / lambda);
            const double ndy = shrink(gy[j] + by[j], 1.0 / lambda);
            const double nbx = bx[j] + gx[j] - ndx;
            const double nby = by[j] + gy[j] - ndy;
            ub += fabs(nbx - bx[j]) + fabs(nby - by[j]);
            uu += fabs(u[j] - uprev[j]);
            dx[j] = ndx; dy[j] = ndy; bx[j] = nbx; by[j] = nby;
            /* change of w = d - b, for the right-hand side of the next solve */
            wx[j] = (ndx - nbx) - wx[j];
            wy[j] = (ndy - nby) - wy[j];
        }
        /* carry: the next right-hand side grows by lambda K^T (w^{k+1} - w^k) */
        ora_gradT(n, wx, wy, kt);
        for (int64_t j = 0; j < nn; ++j) r[j] += lambda * kt[j];
        if (upd_b) upd_b[k] = ub;
        if (upd_u) upd_u[k] = uu;
        if (tol > 0.0 && upd_b && k > 0 && ub < tol * upd_b[0]) { ++k; break; }
    }
    free(gx); free(gy); free(wx); free(wy); free(kt); free(uprev); free(rho_hist);
    free(own);
    return k;
}

/* Chambolle-Pock primal-dual method (the method whose primal step is
 * eq:PD_resolve, Section 2) for min_u ||K u||_1 + alpha/2 ||M R u - f||^2
 * with anisotropic TV:
 *   y <- clip(y + sigma K ubar, -1, 1)               (prox of the dual of ||.||_1)
 *   u_new solves (I + tau alpha R^T M^T M R) u_new = u - tau K^T y + tau alpha R^T M^T f
 *         approximately: n_cg CG steps from u_new = u with the true residual
 *   ubar <- 2 u_new - u                              (extrapolation, theta = 1)
 * u (in/out: the start if warm, else set to 0), y and ubar start as 0 and u.
 * Returns the number of outer iterations. */
int ora_pd(const ora_op *op, double alpha, double tau, double sigma, int n_outer, int n_cg,
           const double *f, double *u, int warm)
{
    const int n = op->n;
    const int64_t nn = (int64_t)n * n;
    double *yx = (double *)calloc((size_t)nn, sizeof(double));
    double *yy = (double *)calloc((size_t)nn, sizeof(double));
    double *ub = (double *)malloc(sizeof(double) * (size_t)nn);
    double *uo = (double *)malloc(sizeof(double) * (size_t)nn);
    double *g = (double *)malloc(sizeof(double) * (size_t)nn);
    double *gx = (double *)malloc(sizeof(double) * (size_t)nn);
    double *gy = (double *)malloc(sizeof(double) * (size_t)nn);
    double *kt = (double *)malloc(sizeof(double) * (size_t)nn);
    double *r = (double *)malloc(sizeof(double) * (size_t)nn);
    double *au = (double *)malloc(sizeof(double) * (size_t)nn);
    double *scratch = (double *)malloc(sizeof(double) * (size_t)(op->rows + 4 * nn));
    if (!warm) memset(u, 0, sizeof(double) * (size_t)nn);
    memcpy(ub, u, sizeof(double) * (size_t)nn);
    ora_spmv(nn, op->trp, op->tci, op->tv, f, g);              /* (MR)^T f */
    for (int64_t j = 0; j < nn; ++j) g[j] *= tau * alpha;
    int k;
    for (k = 0; k < n_outer; ++k) {
        ora_grad(n, ub, gx, gy);
        for (int64_t j = 0; j < nn; ++j) {
            const double vx = yx[j] + sigma * gx[j], vy = yy[j] + sigma * gy[j];
            yx[j] = vx > 1.0 ? 1.0 : (vx < -1.0 ? -1.0 : vx);
            yy[j] = vy > 1.0 ? 1.0 : (vy < -1.0 ? -1.0 : vy);
        }
        ora_gradT(n, yx, yy, kt);
        memcpy(uo, u, sizeof(double) * (size_t)nn);
        /* r = (u - tau K^T y + g) - (I + tau alpha R^T M^T M R) u */
        normal_apply(op, tau * alpha, 0.0, 1.0, u, au, scratch);
        for (int64_t j = 0; j < nn; ++j) r[j] = (u[j] - tau * kt[j] + g[j]) - au[j];
        int bd = 0;
        ora_cg(op, tau * alpha, 0.0, 1.0, u, r, n_cg, 0.0, NULL, &bd);
        for (int64_t j = 0; j < nn; ++j) ub[j] = 2.0 * u[j] - uo[j];
    }
    free(yx); free(yy); free(ub); free(uo); free(g); free(gx); free(gy); free(kt); free(r);
    free(au); free(scratch);
    return k;
}

/* L1 = 0.5 ||MR mu - f||^2 ; g_mu = (MR)^T (MR mu - f) ; g_f = f - MR mu. */
double ora_loss1(const ora_op *op, const double *mu, const double *f, double *g_mu, double *g_f)
{
    double *y = (double *)malloc(sizeof(double) * (size_t)op->rows);
    ora_spmv(op->rows, op->rp, op->ci, op->v, mu, y);
    double L = 0.0;
    for (int64_t i = 0; i < op->rows; ++i) { y[i] -= f[i]; L += 0.5 * y[i] * y[i]; }
    const int64_t nn = (int64_t)op->n * op->n;
    if (g_mu) ora_spmv(nn, op->trp, op->tci, op->tv, y, g_mu);
    if (g_f) for (int64_t i = 0; i < op->rows; ++i) g_f[i] = -y[i];
    free(y);
    return L;
}

/* L2: rhs = mu + ta (MR)^T f;  u_n from n_iter unrolled CG steps on
 * (I + ta R^T M^T M R) u = rhs with u_0 = 0, r_0 = rhs (a step with rho == 0
 * is skipped);  L2 = 0.5 ||MR u_n - f||^2.  Gradients by a reverse sweep over
 * all stored iterates.  u_out (optional) receives u_n. */
double ora_loss2(const ora_op *op, double ta, int n_iter, const double *mu, const double *f,
                 double *g_mu, double *g_f, double *u_out)
{
    const int64_t nn = (int64_t)op->n * op->n, rows = op->rows;
    const int L = n_iter;
    double *P = (double *)calloc((size_t)((L + 1) * nn), sizeof(double));   /* p_i */
    double *Rr = (double *)calloc((size_t)((L + 1) * nn), sizeof(double));  /* r_i */
    double *Q = (double *)calloc((size_t)(L * nn + 1), sizeof(double));     /* q_i */
    double *rho = (double *)calloc((size_t)(L + 1), sizeof(double));
    double *gam = (double *)calloc((size_t)(L + 1), sizeof(double));
    double *aa = (double *)calloc((size_t)(L + 1), sizeof(double));
    double *bb = (double *)calloc((size_t)(L + 1), sizeof(double));
    int *active = (int *)calloc((size_t)(L + 1), sizeof(int));
    double *u = (double *)calloc((size_t)nn, sizeof(double));
    double *scratch = (double *)malloc(sizeof(double) * (size_t)(rows + 4 * nn));
    double *y = (double *)malloc(sizeof(double) * (size_t)rows);

    /* forward */
    ora_spmv(nn, op->trp, op->tci, op->tv, f, Rr);                 /* (MR)^T f */
    for (int64_t j = 0; j < nn; ++j) Rr[j] = mu[j] + ta * Rr[j];    /* r_0 = rhs */
    memcpy(P, Rr, sizeof(double) * (size_t)nn);
    rho[0] = dot(nn, Rr, Rr);
    for (int i = 0; i < L; ++i) {
        double *p = P + i * nn, *r = Rr + i * nn, *q = Q + i * nn;
        double *pn = P + (i + 1) * nn, *rn = Rr + (i + 1) * nn;
        if (rho[i] == 0.0) {           /* converged: this and later steps do nothing */
            memcpy(pn, p, sizeof(double) * (size_t)nn);
            memcpy(rn, r, sizeof(double) * (size_t)nn);
            rho[i + 1] = rho[i];
            continue;
        }
        active[i] = 1;
        normal_apply(op, ta, 0.0, 1.0, p, q, scratch);
        gam[i] = dot(nn, p, q);
        aa[i] = rho[i] / gam[i];
        for (int64_t j = 0; j < nn; ++j) { u[j] += aa[i] * p[j]; rn[j] = r[j] - aa[i] * q[j]; }
        rho[i + 1] = dot(nn, rn, rn);
        bb[i] = rho[i + 1] / rho[i];
        for (int64_t j = 0; j < nn; ++j) pn[j] = rn[j] + bb[i] * p[j];
    }
    if (u_out) memcpy(u_out, u, sizeof(double) * (size_t)nn);
    ora_spmv(rows, op->rp, op->ci, op->v, u, y);
    double loss = 0.0;
    for (int64_t i = 0; i < rows; ++i) { y[i] -= f[i]; loss += 0.5 * y[i] * y[i]; }

    /* reverse sweep */
    double *ub = (double *)calloc((size_t)nn, sizeof(double));
    double *rb = (double *)calloc((size_t)nn, sizeof(double));
    double *pb = (double *)calloc((size_t)nn, sizeof(double));
    double *qb = (double *)calloc((size_t)nn, sizeof(double));
    double *aq = (double *)calloc((size_t)nn, sizeof(double));
    double *rhob = (double *)calloc((size_t)(L + 1), sizeof(double));
    ora_spmv(nn, op->trp, op->tci, op->tv, y, ub);                  /* dL/du_n */
    if (g_f) for (int64_t i = 0; i < rows; ++i) g_f[i] = -y[i];
    for (int i = L - 1; i >= 0; --i) {
        if (!active[i]) { rhob[i] += rhob[i + 1]; continue; }   /* copies pass through */
        double *p = P + i * nn, *q = Q + i * nn, *rn = Rr + (i + 1) * nn;
        /* p_{i+1} = r_{i+1} + b_i p_i */
        const double bbar = dot(nn, pb, p);
        for (int64_t j = 0; j < nn; ++j) { rb[j] += pb[j]; pb[j] *= bb[i]; }
        /* b_i = rho_{i+1} / rho_i */
        rhob[i + 1] += bbar / rho[i];
        rhob[i] -= bbar * rho[i + 1] / (rho[i] * rho[i]);
        /* rho_{i+1} = <r_{i+1}, r_{i+1}> */
        for (int64_t j = 0; j < nn; ++j) rb[j] += 2.0 * rhob[i + 1] * rn[j];
        /* r_{i+1} = r_i - a_i q_i ; u_{i+1} = u_i + a_i p_i */
        const double abar = dot(nn, ub, p) - dot(nn, rb, q);
        for (int64_t j = 0; j < nn; ++j) { qb[j] = -aa[i] * rb[j]; pb[j] += aa[i] * ub[j]; }
        /* a_i = rho_i / gamma_i */
        rhob[i] += abar / gam[i];
        const double gbar = -abar * rho[i] / (gam[i] * gam[i]);
        /* gamma_i = <p_i, q_i> */
        for (int64_t j = 0; j < nn; ++j) { pb[j] += gbar * q[j]; qb[j] += gbar * p[j]; }
        /* q_i = A p_i, A symmetric */
        normal_apply(op, ta, 0.0, 1.0, qb, aq, scratch);
        for (int64_t j = 0; j < nn; ++j) pb[j] += aq[j];
    }
    /* p_0 = r_0, rho_0 = <r_0, r_0>, r_0 = rhs */
    for (int64_t j = 0; j < nn; ++j) rb[j] += pb[j] + 2.0 * rhob[0] * Rr[j];
    if (g_mu) memcpy(g_mu, rb, sizeof(double) * (size_t)nn);
    if (g_f) {
        ora_spmv(rows, op->rp, op->ci, op->v, rb, y);
        for (int64_t i = 0; i < rows; ++i) g_f[i] += ta * y[i];
    }
    free(P); free(Rr); free(Q); free(rho); free(gam); free(aa); free(bb); free(active);
    free(u); free(scratch); free(y); free(ub); free(rb); free(pb); free(qb); free(aq); free(rhob);
    return loss;
}

/* Threads of the OpenMP loops (timing only; the results do not depend on
 * it: every parallel loop writes disjoint rows and the sums are sequential).
 * Returns the count in effect. */
int ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
