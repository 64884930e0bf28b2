/*
 * Driver for a host build of the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (TEST INFRASTRUCTURE ONLY, like the oracle).
 *
 *   sanitize_check <pulses.bin>
 *
 * pulses.bin: int64 count, then per pulse int64 nt, float64 dt, float64
 * r_max, nt float64 samples.  Every entry point of fftt_oracle.c is called
 * on a tiny ring geometry with one band per pulse, in quadrature and table
 * mode, with and without a region-of-interest mask, plus the degenerate
 * cases (no rows, no active voxel, a single voxel).  Prints a checksum of
 * every result; exits non-zero on a failed call or a non-finite value.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_BANDS 8

typedef struct {
    double c0;
    const double *tx;
    int64_t n_tx;
    const int32_t *pairs;
    int64_t n_pairs;
    double origin[3];
    double spacing[3];
    int64_t dims[3];
    const uint8_t *mask;
    int32_t n_bands;
    int32_t use_table;
    int64_t nw;
    const double *qa;
    const double *qb;
    int64_t n_tab;
    const double *tab;
    double r_max[ORC_MAX_BANDS];
} orc_geom;

int orc_quad_coeffs(const double *f, int64_t nt, double dt, double c0, double w_max,
                    int64_t nw, double *a, double *b);
void orc_spectrum(const double *f, int64_t nt, double dt, const double *w, int64_t nw,
                  double *S);
void orc_h(const double *a, const double *b, int64_t nw, const double *R, int64_t n,
           double *out);
void orc_table(const double *a, const double *b, int64_t nw, double r_max, int64_t n,
               double *tab);
void orc_rows(const orc_geom *g, const int64_t *rows, int64_t nr, const double *x, double *y);
void orc_cols(const orc_geom *g, const int64_t *cols, int64_t nc, const double *y, double *x);
void orc_apply_J(const orc_geom *g, const double *x, double *y);
void orc_apply_JT(const orc_geom *g, const double *y, double *x);
void orc_block(const orc_geom *g, int band, const int64_t *rows, int64_t nr,
               const int64_t *cols, int64_t nc, double *out);
int64_t orc_count_pv(const orc_geom *g);
void orc_kernel_points(const double *xs, const double *xr, double c0, const double *a,
                       const double *b, int64_t nw, double r_max, const double *pts, int64_t n,
                       double *out);

static double checksum = 0.0;
static int bad = 0;

static void fold(const char *what, const double *v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(v[i])) {
            fprintf(stderr, "%s: non-finite value at %lld\n", what, (long long)i);
            bad = 1;
            return;
        }
        checksum += fabs(v[i]) * (double)((i % 7) + 1);
    }
}

static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(3);
    }
    return p;
}

#define NW 128
#define NTAB 257

static void run_geometry(orc_geom *g, int64_t N, int64_t M)
{
    const int B = g->n_bands;
    double *x = xmalloc(sizeof(double) * (size_t)N);
    double *y = xmalloc(sizeof(double) * (size_t)(B * M));
    /* room for the three sampled rows / columns as well */
    double *xo = xmalloc(sizeof(double) * (size_t)(N > 3 ? N : 3));
    double *yo = xmalloc(sizeof(double) * (size_t)(B * (M > 3 ? M : 3)));
    for (int64_t j = 0; j < N; ++j) x[j] = sin(0.37 * (double)j);
    for (int64_t i = 0; i < B * M; ++i) y[i] = 1e-7 * cos(0.11 * (double)i);
    orc_apply_J(g, x, yo);
    fold("apply_J", yo, B * M);
    orc_apply_JT(g, y, xo);
    fold("apply_JT", xo, N);
    int64_t rows[3] = {0, M / 2, M - 1};
    int64_t cols[3] = {0, N / 2, N - 1};
    orc_rows(g, rows, M > 0 ? 3 : 0, x, yo);
    fold("rows", yo, M > 0 ? 3 * B : 0);
    orc_cols(g, cols, N > 0 ? 3 : 0, y, xo);
    fold("cols", xo, N > 0 ? 3 : 0);
    orc_rows(g, rows, 0, x, yo);   /* no rows */
    if (M > 0 && N > 0) {
        double *blk = xmalloc(sizeof(double) * 9);
        for (int b = 0; b < B; ++b) {
            orc_block(g, b, rows, 3, cols, 3, blk);
            fold("block", blk, 9);
        }
        free(blk);
    }
    const int64_t pv = orc_count_pv(g);
    checksum += (double)pv;
    free(x);
    free(y);
    free(xo);
    free(yo);
}

int main(int argc, char **argv)
{
    if (argc != 2) {
        fprintf(stderr, "usage: %s pulses.bin\n", argv[0]);
        return 2;
    }
    FILE *fp = fopen(argv[1], "rb");
    if (!fp) {
        perror(argv[1]);
        return 2;
    }
    int64_t np = 0;
    if (fread(&np, sizeof np, 1, fp) != 1 || np < 1 || np > ORC_MAX_BANDS) {
        fprintf(stderr, "bad pulse count\n");
        return 2;
    }
    const double c0 = 1500.0;
    double *qa = xmalloc(sizeof(double) * (size_t)(np * NW));
    double *qb = xmalloc(sizeof(double) * (size_t)(np * NW));
    double *tab = xmalloc(sizeof(double) * (size_t)(np * NTAB));
    double r_max[ORC_MAX_BANDS];
    for (int64_t p = 0; p < np; ++p) {
        int64_t nt = 0;
        double dt = 0.0, rm = 0.0;
        if (fread(&nt, sizeof nt, 1, fp) != 1 || fread(&dt, sizeof dt, 1, fp) != 1 ||
            fread(&rm, sizeof rm, 1, fp) != 1 || nt < 1 || nt > (1 << 22)) {
            fprintf(stderr, "bad pulse header\n");
            return 2;
        }
        double *f = xmalloc(sizeof(double) * (size_t)nt);
        if (fread(f, sizeof(double), (size_t)nt, fp) != (size_t)nt) {
            fprintf(stderr, "short pulse\n");
            return 2;
        }
        r_max[p] = rm;
        const double w_max = 2.0 * M_PI * 4.0 / (64.0 * dt);   /* a quarter of Nyquist */
        if (orc_quad_coeffs(f, nt, dt, c0, w_max, NW, qa + p * NW, qb + p * NW) != 0) {
            fprintf(stderr, "orc_quad_coeffs failed\n");
            bad = 1;
        }
        /* invalid arguments are refused without touching the outputs */
        if (orc_quad_coeffs(f, nt, dt, c0, w_max, 1, qa, qb) == 0 ||
            orc_quad_coeffs(f, nt, -dt, c0, w_max, NW, qa, qb) == 0)
            bad = 1;
        fold("quad", qa + p * NW, NW);
        double w[5] = {0.0, 1e5, 1e6, 6e6, 2e7}, S[5];
        orc_spectrum(f, nt, dt, w, 5, S);
        fold("spectrum", S, 5);
        double R[4] = {0.0, 0.3 * rm, rm, 2.0 * rm}, h[4];
        orc_h(qa + p * NW, qb + p * NW, NW, R, 4, h);
        fold("h", h, 4);
        orc_table(qa + p * NW, qb + p * NW, NW, rm, NTAB, tab + p * NTAB);
        fold("table", tab + p * NTAB, NTAB);
        double xs[3] = {0.02, 0.0, 0.0}, xr[3] = {-0.02, 0.001, 0.0};
        double pts[9] = {0.0, 0.0, 0.0, 0.0, 0.001, 0.0005, 0.019, 0.0, 0.0};
        double kv[3];
        orc_kernel_points(xs, xr, c0, qa + p * NW, qb + p * NW, NW, rm, pts, 3, kv);
        fold("kernel_points", kv, 3);
        free(f);
    }
    fclose(fp);

    /* a ring of 6 transducers, radius 3 cm; all ordered pairs */
    double tx[6 * 3];
    for (int k = 0; k < 6; ++k) {
        tx[3 * k] = 0.03 * cos(2.0 * M_PI * k / 6.0);
        tx[3 * k + 1] = 0.03 * sin(2.0 * M_PI * k / 6.0);
        tx[3 * k + 2] = 0.0;
    }
    int32_t pairs[30 * 2];
    int64_t M = 0;
    for (int s = 0; s < 6; ++s)
        for (int r = 0; r < 6; ++r)
            if (s != r) {
                pairs[2 * M] = s;
                pairs[2 * M + 1] = r;
                ++M;
            }
    orc_geom g;
    memset(&g, 0, sizeof g);
    g.c0 = c0;
    g.tx = tx;
    g.n_tx = 6;
    g.pairs = pairs;
    g.n_pairs = M;
    g.dims[0] = 7;
    g.dims[1] = 6;
    g.dims[2] = 3;
    for (int k = 0; k < 3; ++k) {
        g.spacing[k] = 1.5e-3;
        g.origin[k] = -0.5 * (double)(g.dims[k] - 1) * 1.5e-3;
    }
    const int64_t N = g.dims[0] * g.dims[1] * g.dims[2];
    uint8_t *mask = xmalloc((size_t)N);
    for (int64_t j = 0; j < N; ++j) mask[j] = (uint8_t)((j % 5) != 0);
    g.n_bands = (int32_t)np;
    for (int64_t p = 0; p < np; ++p) g.r_max[p] = r_max[p];
    g.nw = NW;
    g.qa = qa;
    g.qb = qb;
    g.n_tab = NTAB;
    g.tab = tab;
    for (int mode = 0; mode < 2; ++mode) {
        g.use_table = mode;
        g.mask = NULL;
        run_geometry(&g, N, M);
        g.mask = mask;
        run_geometry(&g, N, M);
    }
    /* no active voxel */
    memset(mask, 0, (size_t)N);
    g.mask = mask;
    run_geometry(&g, N, M);
    /* a single voxel, one pair */
    g.mask = NULL;
    g.dims[0] = g.dims[1] = g.dims[2] = 1;
    g.n_pairs = 1;
    run_geometry(&g, 1, 1);
    free(mask);
    free(qa);
    free(qb);
    free(tab);
    printf("checksum %.17g\n", checksum);
    return bad;
}
