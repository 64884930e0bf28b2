/*
 * Plain FP64 CPU oracle for the linearised cross-correlation traveltime
 * Jacobian of finite-frequency ultrasound tomography
 * (Korta Martiartu, Boehm, Fichtner, arXiv:1908.03302).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP path and is deliberately slow and literal: every sensitivity value
 * is obtained by direct frequency quadrature, every product by a compensated
 * (Kahan) sum over the dense index range.
 *
 * What it computes (paper Sec. II):
 *   S(w)  = |F(w)|^2, F = Fourier transform of the calibration pulse f(t)
 *           (here the discrete-time transform of the given samples).
 *   h(R)  = int_0^inf w^3 S(w) sin(w R / c0) dw / int_0^inf w^2 S(w) dw
 *           -- the frequency-domain kernel of Sec. II-C (eq. Kernel_freq),
 *           upper limit read as infinity, written as a function of the
 *           detour R = R_xs + R_xr - R_sr alone.
 *   A(x)  = -R_sr / (2 pi c0^3 R_xs R_xr)  (eq. Linearized_sensitivity_A)
 *   K0(x) = A(x) h(R), zero for R >= R_max (truncation of Sec. II-C).
 *   J_ij  = K0(x_j; pair i) * dV : midpoint rule at voxel centres for the
 *           volume integral dT = int K dc dx (eq. forward_ffttt, forward_compact).
 *   J x   and J^T y           : eq. forward_compact and its transpose, the
 *                               matrix-vector products of Sec. II-D.
 *
 * The integrals are trapezoid sums on uniform nodes w_m = m dw,
 * m = 0..nw-1, chosen by the caller; the coefficients a_m, b_m below are the
 * "coefficients and arguments of the trigonometric functions" of Sec. II-C:
 *   h(R) = sum_m a_m sin(b_m R).
 * A second mode evaluates a tabulated h_k = h(k R_max/(n-1)) by linear
 * interpolation, which isolates the interpolation error of a tabulated
 * kernel from everything else.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_BANDS 8

typedef struct {
    double c0;
    const double *tx;        /* [n_tx][3] */
    int64_t n_tx;
    const int32_t *pairs;    /* [n_pairs][2] = (source, receiver) */
    int64_t n_pairs;
    double origin[3];
    double spacing[3];
    int64_t dims[3];
    const uint8_t *mask;     /* [N] or NULL: every voxel active */
    int32_t n_bands;
    int32_t use_table;       /* 0: quadrature, 1: table */
    int64_t nw;              /* quadrature nodes per band */
    const double *qa;        /* [n_bands][nw] */
    const double *qb;        /* [n_bands][nw] */
    int64_t n_tab;           /* table entries per band */
    const double *tab;       /* [n_bands][n_tab] */
    double r_max[ORC_MAX_BANDS];
} orc_geom;

/* ---------------------------------------------------------------- spectra */

/* a_m = q_m w_m^3 S(w_m) / sum_k q_k w_k^2 S(w_k), b_m = w_m / c0 with
 * trapezoid weights q_m on w_m = m * w_max/(nw-1).  S is |DTFT|^2 of the
 * pulse samples f_n at times n*dt (a time shift does not change |F|). */
int orc_quad_coeffs(const double *f, int64_t nt, double dt, double c0,
                    double w_max, int64_t nw, double *a, double *b)
{
    if (nw < 2 || nt < 1 || dt <= 0 || c0 <= 0 || w_max <= 0) return -1;
    const double dw = w_max / (double)(nw - 1);
    double den = 0.0;
    for (int64_t m = 0; m < nw; ++m) {
        const double w = dw * (double)m;
        double re = 0.0, im = 0.0;
        for (int64_t n = 0; n < nt; ++n) {
            const double ph = w * dt * (double)n;
            re += f[n] * cos(ph);
            im -= f[n] * sin(ph);
        }
        re *= dt;
        im *= dt;
        const double S = re * re + im * im;
        const double q = (m == 0 || m == nw - 1) ? 0.5 * dw : dw;
        a[m] = q * w * w * w * S;
        den += q * w * w * S;
        b[m] = w / c0;
    }
    if (!(den > 0.0)) return -2;
    for (int64_t m = 0; m < nw; ++m) a[m] /= den;
    return 0;
}

/* Spectrum samples S(w) at arbitrary frequencies (for tests). */
void orc_spectrum(const double *f, int64_t nt, double dt, const double *w,
                  int64_t nw, double *S)
{
    for (int64_t m = 0; m < nw; ++m) {
        double re = 0.0, im = 0.0;
        for (int64_t n = 0; n < nt; ++n) {
            const double ph = w[m] * dt * (double)n;
            re += f[n] * cos(ph);
            im -= f[n] * sin(ph);
        }
        re *= dt;
        im *= dt;
        S[m] = re * re + im * im;
    }
}

static double h_quad(const double *a, const double *b, int64_t nw, double R)
{
    double s = 0.0;
    for (int64_t m = 0; m < nw; ++m) s += a[m] * sin(b[m] * R);
    return s;
}

/* h at arbitrary R, no truncation. */
void orc_h(const double *a, const double *b, int64_t nw, const double *R,
           int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = h_quad(a, b, nw, R[i]);
}

/* Table h_k = h(k r_max/(n-1)), k = 0..n-1, from the quadrature. */
void orc_table(const double *a, const double *b, int64_t nw, double r_max,
               int64_t n, double *tab)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k)
        tab[k] = h_quad(a, b, nw, r_max * (double)k / (double)(n - 1));
}

/* ------------------------------------------------------------- geometry */

static void voxel_centre(const orc_geom *g, int64_t j, double x[3])
{
    const int64_t nx = g->dims[0], ny = g->dims[1];
    const int64_t i0 = j % nx, i1 = (j / nx) % ny, i2 = j / (nx * ny);
    x[0] = g->origin[0] + (double)i0 * g->spacing[0];
    x[1] = g->origin[1] + (double)i1 * g->spacing[1];
    x[2] = g->origin[2] + (double)i2 * g->spacing[2];
}

static double dist3(const double *p, const double *q)
{
    const double d0 = p[0] - q[0], d1 = p[1] - q[1], d2 = p[2] - q[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

static double h_band(const orc_geom *g, int band, double R)
{
    if (R >= g->r_max[band]) return 0.0;
    if (!g->use_table)
        return h_quad(g->qa + band * g->nw, g->qb + band * g->nw, g->nw, R);
    /* linear interpolation on the uniform grid R_k = k r_max/(n-1) */
    const double *t = g->tab + band * g->n_tab;
    const double u = R * (double)(g->n_tab - 1) / g->r_max[band];
    int64_t k = (int64_t)floor(u);
    if (k < 0) k = 0;
    if (k > g->n_tab - 2) k = g->n_tab - 2;
    const double fr = u - (double)k;
    return t[k] + fr * (t[k + 1] - t[k]);
}

static double voxel_volume(const orc_geom *g)
{
    return g->spacing[0] * g->spacing[1] * g->spacing[2];
}

static double r_max_all(const orc_geom *g)
{
    double r = 0.0;
    for (int b = 0; b < g->n_bands; ++b) if (g->r_max[b] > r) r = g->r_max[b];
    return r;
}

/* J_ij for every band at once; returns 0 when the detour is beyond every
 * band's truncation radius. */
static int entry_all(const orc_geom *g, int64_t i, const double x[3],
                     double *out)
{
    const double *xs = g->tx + 3 * (int64_t)g->pairs[2 * i];
    const double *xr = g->tx + 3 * (int64_t)g->pairs[2 * i + 1];
    const double Rs = dist3(x, xs), Rr = dist3(x, xr), L = dist3(xs, xr);
    const double R = Rs + Rr - L;
    if (R >= r_max_all(g)) return 0;
    const double c0 = g->c0;
    const double A = -L / (2.0 * M_PI * c0 * c0 * c0 * Rs * Rr);
    const double dV = voxel_volume(g);
    for (int b = 0; b < g->n_bands; ++b) out[b] = A * h_band(g, b, R) * dV;
    return 1;
}

static int active(const orc_geom *g, int64_t j)
{
    return g->mask == NULL || g->mask[j] != 0;
}

static int64_t n_voxels(const orc_geom *g)
{
    return g->dims[0] * g->dims[1] * g->dims[2];
}

/* Kahan-compensated accumulator */
typedef struct { double s, c; } kahan;
static inline void kadd(kahan *k, double v)
{
    const double y = v - k->c;
    const double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* y[b][r] = sum_j J^b_{rows[r], j} x_j  over active voxels */
void orc_rows(const orc_geom *g, const int64_t *rows, int64_t nr,
              const double *x, double *y)
{
    const int64_t N = n_voxels(g);
    const int B = g->n_bands;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nr; ++r) {
        kahan acc[ORC_MAX_BANDS];
        memset(acc, 0, sizeof(acc));
        double e[ORC_MAX_BANDS], xc[3];
        for (int64_t j = 0; j < N; ++j) {
            if (!active(g, j)) continue;
            voxel_centre(g, j, xc);
            if (!entry_all(g, rows[r], xc, e)) continue;
            for (int b = 0; b < B; ++b) kadd(&acc[b], e[b] * x[j]);
        }
        for (int b = 0; b < B; ++b) y[(int64_t)b * nr + r] = acc[b].s;
    }
}

/* x[c] = sum_b sum_i J^b_{i, cols[c]} y[b][i] */
void orc_cols(const orc_geom *g, const int64_t *cols, int64_t nc,
              const double *y, double *x)
{
    const int64_t M = g->n_pairs;
    const int B = g->n_bands;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t j = cols[c];
        if (!active(g, j)) { x[c] = 0.0; continue; }
        kahan acc = {0.0, 0.0};
        double e[ORC_MAX_BANDS], xc[3];
        voxel_centre(g, j, xc);
        for (int64_t i = 0; i < M; ++i) {
            if (!entry_all(g, i, xc, e)) continue;
            for (int b = 0; b < B; ++b) kadd(&acc, e[b] * y[(int64_t)b * M + i]);
        }
        x[c] = acc.s;
    }
}

void orc_apply_J(const orc_geom *g, const double *x, double *y)
{
    const int64_t M = g->n_pairs;
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    for (int64_t i = 0; i < M; ++i) rows[i] = i;
    orc_rows(g, rows, M, x, y);
    free(rows);
}

void orc_apply_JT(const orc_geom *g, const double *y, double *x)
{
    const int64_t N = n_voxels(g);
    int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    for (int64_t j = 0; j < N; ++j) cols[j] = j;
    orc_cols(g, cols, N, y, x);
    free(cols);
}

/* Dense sub-block J^band[rows][cols] (row-major, nr x nc). */
void orc_block(const orc_geom *g, int band, const int64_t *rows, int64_t nr,
               const int64_t *cols, int64_t nc, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nr; ++r) {
        double e[ORC_MAX_BANDS], xc[3];
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t j = cols[c];
            double v = 0.0;
            if (active(g, j)) {
                voxel_centre(g, j, xc);
                if (entry_all(g, rows[r], xc, e)) v = e[band];
            }
            out[r * nc + c] = v;
        }
    }
}

/* Number of (pair, active voxel) combinations with detour below the largest
 * truncation radius: the unit of work of one operator application. */
int64_t orc_count_pv(const orc_geom *g)
{
    const int64_t N = n_voxels(g), M = g->n_pairs;
    const double rm = r_max_all(g);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int64_t i = 0; i < M; ++i) {
        const double *xs = g->tx + 3 * (int64_t)g->pairs[2 * i];
        const double *xr = g->tx + 3 * (int64_t)g->pairs[2 * i + 1];
        const double L = dist3(xs, xr);
        double xc[3];
        for (int64_t j = 0; j < N; ++j) {
            if (!active(g, j)) continue;
            voxel_centre(g, j, xc);
            if (dist3(xc, xs) + dist3(xc, xr) - L < rm) ++total;
        }
    }
    return total;
}

/* Kernel values K0 (no voxel volume) at arbitrary points for one source /
 * receiver position pair: used by the geometric pins. */
void orc_kernel_points(const double *xs, const double *xr, double c0,
                       const double *a, const double *b, int64_t nw,
                       double r_max, const double *pts, int64_t n, double *out)
{
    const double L = dist3(xs, xr);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        const double *x = pts + 3 * p;
        const double Rs = dist3(x, xs), Rr = dist3(x, xr);
        const double R = Rs + Rr - L;
        double v = 0.0;
        if (R < r_max) {
            const double A = -L / (2.0 * M_PI * c0 * c0 * c0 * Rs * Rr);
            v = A * h_quad(a, b, nw, R);
        }
        out[p] = v;
    }
}
