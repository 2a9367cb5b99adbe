/* Runs every entry point of the C oracle once on small geometries, built
 * with -fsanitize=address,undefined by tests/test_oracle_sanitize.py: any
 * out-of-bounds access, use after free, leak or undefined behaviour in the
 * oracle aborts the run.  The geometries cover odd and even sizes, rays on
 * pixel edges (angle 0 and pi/2), bins missing the image, subsampled
 * angles, and a NaN in the data (the CG breakdown path). */
#include "../../oracle/oracle.c"

#include <stdio.h>

static double lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

static int run(int n, int na, int nb, int every)
{
    int32_t angles[512];
    int n_list = 0;
    for (int k = 0; k < na; k += every) angles[n_list++] = k;
    const int64_t rows = (int64_t)n_list * nb, nn = (int64_t)n * n;
    int64_t *rp = calloc((size_t)rows + 1, sizeof(int64_t));
    ora_build(n, na, nb, n_list, angles, rp, NULL, NULL);
    const int64_t nnz = rp[rows];
    int32_t *ci = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    double *v = malloc(sizeof(double) * (size_t)(nnz + 1));
    ora_build(n, na, nb, n_list, angles, rp, ci, v);
    int64_t *trp = malloc(sizeof(int64_t) * (size_t)(nn + 1));
    int32_t *tci = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    double *tv = malloc(sizeof(double) * (size_t)(nnz + 1));
    ora_transpose(rows, nn, rp, ci, v, trp, tci, tv);
    ora_op op = {n, rows, rp, ci, v, trp, tci, tv, -1, NULL};

    uint64_t s = 12345u + (uint64_t)n;
    double *x = malloc(sizeof(double) * (size_t)nn), *out = malloc(sizeof(double) * (size_t)nn);
    double *f = malloc(sizeof(double) * (size_t)rows), *g = malloc(sizeof(double) * (size_t)nn);
    double *gf = malloc(sizeof(double) * (size_t)rows), *u = malloc(sizeof(double) * (size_t)nn);
    double *r = malloc(sizeof(double) * (size_t)nn), *hist = malloc(sizeof(double) * 16);
    double *state = calloc((size_t)(5 * nn), sizeof(double));
    double ub[8], uu[8];
    for (int64_t j = 0; j < nn; ++j) x[j] = lcg(&s);
    for (int64_t i = 0; i < rows; ++i) f[i] = lcg(&s);
    ora_normal(&op, 1.5, 0.5, 0.25, x, out);
    int bd = 0;
    memcpy(r, x, sizeof(double) * (size_t)nn);
    memset(u, 0, sizeof(double) * (size_t)nn);
    ora_cg(&op, 1.0, 1.0, 0.0, u, r, 12, 0.0, hist, &bd);
    ora_sb(&op, 1.0, 1.0, 4, 3, 0.0, f, u, 0, state, 0, ub, uu);
    ora_sb(&op, 1.0, 1.0, 4, 3, 0.0, f, u, 0, state, 1, ub, uu);   /* resume */
    ora_sb(&op, 1.0, 1.0, 6, 3, 0.5, f, u, 1, NULL, 0, ub, uu);     /* warm, tolerance stop */
    ora_pd(&op, 1.0, 0.3, 0.3, 3, 3, f, u, 0);
    ora_loss1(&op, x, f, g, gf);
    ora_loss2(&op, 0.1, 5, x, f, g, gf, u);
    /* CG breakdown: a NaN in the data of the central ray of the first angle
     * reaches <p, Ap> in every inner solve, so u never moves from 0 */
    f[nb / 2] = NAN;
    ora_sb(&op, 1.0, 1.0, 2, 3, 0.0, f, u, 0, NULL, 0, ub, uu);
    int bad = 0;
    for (int64_t j = 0; j < nn; ++j) bad |= u[j] != 0.0;
    if (bad) fprintf(stderr, "NaN data: u moved from 0\n");
    if (n >= 9) {
        double w[49];
        if (ora_surrogate_weights(&op, 3, w) == 0) {
            ora_stencil(n, 3, w, x, out);
            ora_op sur = op;
            sur.sur_r = 3;
            sur.sur_w = w;
            memset(u, 0, sizeof(double) * (size_t)nn);
            f[nb / 2] = 0.0;
            ora_sb(&sur, 1.0, 1.0, 3, 3, 0.0, f, u, 0, NULL, 0, ub, uu);
        }
    }
    int32_t cols[4 * 64 + 8];
    double vals[4 * 64 + 8];
    for (int b = 0; b < nb; ++b) ora_ray(n, na, nb, angles[n_list - 1], b, cols, vals);
    double c, sn;
    ora_trig(na / 2, na, &c, &sn);
    free(rp); free(ci); free(v); free(trp); free(tci); free(tv);
    free(x); free(out); free(f); free(g); free(gf); free(u); free(r); free(hist); free(state);
    return bad;
}

int main(void)
{
    const int cases[][4] = {{8, 8, 13, 1}, {7, 6, 11, 1}, {16, 12, 25, 2}, {33, 10, 47, 3},
                            {9, 4, 5, 1}, {12, 18, 17, 1}, {1, 4, 3, 1}, {2, 1, 3, 1}};
    for (size_t i = 0; i < sizeof cases / sizeof cases[0]; ++i) {
        if (run(cases[i][0], cases[i][1], cases[i][2], cases[i][3])) return 1;
        printf("case n=%d angles=%d bins=%d ok\n", cases[i][0], cases[i][1], cases[i][2]);
    }
    return 0;
}
