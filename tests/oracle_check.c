/* CPU check of the FP64 oracle's C loops (oracle/oracle.c), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_host_sanitized.py.  Runs every exported routine on small cone,
 * 3-D parallel, fan and 2-D parallel geometries, including one-voxel
 * volumes, rays along a grid axis and steep rays, and checks:
 *   the dot-product identity <A x, y> = <x, A^T y>;
 *   per-ray tap counts within the documented capacity 4 max(n) + 4;
 *   box-restricted adjoints and selected rays / voxels against the full
 *   operators.
 * Prints "oracle_check OK" and exits 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_forward(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                   int64_t n_views, const double *P, int64_t nv, int64_t nu, const double *vol, double *sino,
                   int nthreads);
int oracle_forward_rays(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                        const double *P, const double *vol, int64_t n_rays, const int64_t *view, const int64_t *row,
                        const int64_t *col, double *out, int nthreads);
int oracle_adjoint(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                   int64_t n_views, const double *P, int64_t nv, int64_t nu, const double *sino, const int64_t box[6],
                   double *out, int nthreads);
int oracle_backproject(int dims, const int64_t n[3], const double s[3], const double o[3], int64_t n_views,
                       const double *P, int64_t nv, int64_t nu, const double *sino, double *vol, int nthreads);
int oracle_backproject_voxels(int dims, const int64_t n[3], const double s[3], const double o[3], int64_t n_views,
                              const double *P, int64_t nv, int64_t nu, const double *sino, int64_t n_vox,
                              const int64_t *vi, const int64_t *vj, const int64_t *vk, double *out, int nthreads);
int64_t oracle_ray_taps(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                        const double *P, int64_t r, int64_t c, int64_t *idx, double *w);

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

static uint64_t rng_state = 88172645463325252ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * 0x1p-53;
}

static void inv3(const double m[9], double r[9])
{
    double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                 m[2] * (m[3] * m[7] - m[4] * m[6]);
    r[0] = (m[4] * m[8] - m[5] * m[7]) / det;
    r[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    r[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    r[3] = (m[5] * m[6] - m[3] * m[8]) / det;
    r[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    r[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    r[6] = (m[3] * m[7] - m[4] * m[6]) / det;
    r[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    r[8] = (m[0] * m[4] - m[1] * m[3]) / det;
}

/* cone view at angle b with a small tilt; rows x cols detector at pitch d */
static void cone_view(double b, double tilt, int64_t rows, int64_t cols, double d, double *P)
{
    double S[3] = {60 * cos(b), 60 * sin(b), 3 * tilt};
    double C[3] = {-40 * cos(b), -40 * sin(b), 0};
    double eu[3] = {-d * sin(b), d * cos(b), d * tilt}, ev[3] = {0, d * tilt, d};
    double M[9], Mi[9];
    for (int i = 0; i < 3; ++i) {
        double d00 = C[i] - 0.5 * (cols - 1) * eu[i] - 0.5 * (rows - 1) * ev[i];
        M[3 * i] = eu[i];
        M[3 * i + 1] = ev[i];
        M[3 * i + 2] = d00 - S[i];
    }
    inv3(M, Mi);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) P[4 * r + c] = Mi[3 * r + c];
        P[4 * r + 3] = -(Mi[3 * r] * S[0] + Mi[3 * r + 1] * S[1] + Mi[3 * r + 2] * S[2]);
    }
}

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void run_case(int dims, int parallel, const int64_t n[3], const double s[3], int64_t nviews, const double *P,
                     int64_t nv, int64_t nu)
{
    const double o[3] = {-0.5 * (n[0] - 1) * s[0], -0.5 * (n[1] - 1) * s[1], dims == 2 ? 0.0 : -0.5 * (n[2] - 1) * s[2]};
    const int64_t nvox = n[0] * n[1] * n[2], npix = nviews * nv * nu;
    double *x = malloc(sizeof(double) * nvox), *y = malloc(sizeof(double) * (npix ? npix : 1));
    double *Ax = malloc(sizeof(double) * (npix ? npix : 1)), *ATy = malloc(sizeof(double) * nvox);
    double *bp = malloc(sizeof(double) * nvox);
    for (int64_t i = 0; i < nvox; ++i) x[i] = urand() - 0.3;
    for (int64_t i = 0; i < npix; ++i) y[i] = urand() - 0.3;
    const int64_t full[6] = {0, n[0], 0, n[1], 0, n[2]};
    CHECK(oracle_forward(dims, parallel, n, s, o, nviews, P, nv, nu, x, Ax, 1) == 0);
    CHECK(oracle_adjoint(dims, parallel, n, s, o, nviews, P, nv, nu, y, full, ATy, 1) == 0);
    const double l = dot(Ax, y, npix), r = dot(x, ATy, nvox);
    CHECK(fabs(l - r) <= 1e-12 * (fabs(l) + fabs(r) + 1e-300) + 1e-300 || (npix == 0 && r == 0.0));
    if (!parallel) CHECK(oracle_backproject(dims, n, s, o, nviews, P, nv, nu, y, bp, 1) == 0);
    /* a box of the adjoint equals that part of the full adjoint */
    int64_t box[6];
    for (int a = 0; a < 3; ++a) {
        box[2 * a] = n[a] / 3;
        box[2 * a + 1] = n[a] - n[a] / 4;
    }
    const int64_t bx = box[1] - box[0], by = box[3] - box[2], bz = box[5] - box[4];
    const int64_t nbox = bx * by * bz;
    double *part = malloc(sizeof(double) * (nbox > 0 ? nbox : 1));
    CHECK(oracle_adjoint(dims, parallel, n, s, o, nviews, P, nv, nu, y, box, part, 1) == 0);
    for (int64_t k = 0; k < bz; ++k)
        for (int64_t j = 0; j < by; ++j)
            for (int64_t i = 0; i < bx; ++i) {
                const double f = ATy[((k + box[4]) * n[1] + j + box[2]) * n[0] + i + box[0]];
                CHECK(fabs(part[(k * by + j) * bx + i] - f) <= 1e-12 * (fabs(f) + 1.0));
            }
    /* selected rays and voxels; tap counts within capacity */
    const int64_t cap = 4 * (n[0] > n[1] ? (n[0] > n[2] ? n[0] : n[2]) : (n[1] > n[2] ? n[1] : n[2])) + 4;
    int64_t *idx = malloc(sizeof(int64_t) * cap);
    double *w = malloc(sizeof(double) * cap);
    const int64_t psz = dims == 2 ? 6 : 12;
    for (int t = 0; t < 25 && npix > 0; ++t) {
        int64_t view = (int64_t)(urand() * nviews), row = (int64_t)(urand() * nv), col = (int64_t)(urand() * nu);
        double one;
        CHECK(oracle_forward_rays(dims, parallel, n, s, o, P, x, 1, &view, &row, &col, &one, 1) == 0);
        CHECK(fabs(one - Ax[(view * nv + row) * nu + col]) <= 1e-12 * (fabs(one) + 1.0));
        const int64_t cnt = oracle_ray_taps(dims, parallel, n, s, o, P + view * psz, row, col, idx, w);
        CHECK(cnt >= 0 && cnt <= cap);
        for (int64_t q = 0; q < cnt; ++q) CHECK(idx[q] >= 0 && idx[q] < nvox);
    }
    if (!parallel) {
        for (int t = 0; t < 25; ++t) {
            int64_t i = (int64_t)(urand() * n[0]), j = (int64_t)(urand() * n[1]), k = (int64_t)(urand() * n[2]);
            double one;
            CHECK(oracle_backproject_voxels(dims, n, s, o, nviews, P, nv, nu, y, 1, &i, &j, &k, &one, 1) == 0);
            CHECK(fabs(one - bp[(k * n[1] + j) * n[0] + i]) <= 1e-12 * (fabs(one) + 1.0));
        }
    }
    free(x), free(y), free(Ax), free(ATy), free(bp), free(part), free(idx), free(w);
}

int main(void)
{
    /* 3-D cone: ragged volume, tilted views, and a one-voxel volume */
    {
        const int64_t n[3] = {9, 7, 5};
        const double s[3] = {1.0, 0.8, 1.2};
        double P[12 * 6];
        for (int k = 0; k < 6; ++k) cone_view(0.7 * k + 0.1, k % 2 ? 0.2 : 0.0, 6, 11, 1.3, P + 12 * k);
        cone_view(0.0, 0.0, 6, 11, 1.3, P);          /* rays in the x-z plane at the centre column */
        cone_view(0.7853981633974483, 0.0, 6, 11, 1.3, P + 12); /* near-diagonal rays */
        run_case(3, 0, n, s, 6, P, 6, 11);
        const int64_t one[3] = {1, 1, 1};
        run_case(3, 0, one, s, 6, P, 6, 11);
        run_case(3, 0, n, s, 0, P, 6, 11);
    }
    /* 3-D parallel: rays along (cos t, sin t, 0.3) */
    {
        const int64_t n[3] = {6, 8, 5};
        const double s[3] = {1.0, 1.0, 1.0};
        double P[12 * 4];
        for (int k = 0; k < 4; ++k) {
            const double t = 0.5 * k, d[3] = {cos(t), sin(t), k == 3 ? 0.0 : 0.3};
            const double eu[3] = {-sin(t), cos(t), 0}, ev[3] = {0, -0.3 * sin(t), 1};
            double M[9] = {eu[0], ev[0], d[0], eu[1], ev[1], d[1], eu[2], ev[2], d[2]}, Mi[9];
            inv3(M, Mi);
            double *p = P + 12 * k;
            for (int r = 0; r < 2; ++r) {
                for (int j = 0; j < 3; ++j) p[4 * r + j] = Mi[3 * r + j];
                p[4 * r + 3] = r == 0 ? 4.5 : 3.0;
            }
            p[8] = p[9] = p[10] = 0.0;
            p[11] = 1.0;
        }
        run_case(3, 1, n, s, 4, P, 7, 10);
    }
    /* 2-D fan and 2-D parallel, including a view along a grid axis */
    {
        const int64_t n[3] = {11, 8, 1};
        const double s[3] = {0.9, 1.1, 1.0};
        double P[6 * 5], Q[6 * 5];
        for (int k = 0; k < 5; ++k) {
            const double b = k == 0 ? 0.0 : 1.3 * k, c = cos(b), sn = sin(b);
            /* fan: M = [eu | d0 - S], P = M^-1 [I | -S] */
            const double S[2] = {50 * c, 50 * sn}, eu[2] = {-1.1 * sn, 1.1 * c};
            const double d0[2] = {-30 * c - 8 * eu[0], -30 * sn - 8 * eu[1]};
            const double m00 = eu[0], m01 = d0[0] - S[0], m10 = eu[1], m11 = d0[1] - S[1];
            const double det = m00 * m11 - m01 * m10;
            const double i00 = m11 / det, i01 = -m01 / det, i10 = -m10 / det, i11 = m00 / det;
            double *p = P + 6 * k;
            p[0] = i00, p[1] = i01, p[2] = -(i00 * S[0] + i01 * S[1]);
            p[3] = i10, p[4] = i11, p[5] = -(i10 * S[0] + i11 * S[1]);
            /* parallel: u = (-sin, cos) . X / 1.1 + 8, rays along (cos, sin) */
            double *q = Q + 6 * k;
            q[0] = -sn / 1.1, q[1] = c / 1.1, q[2] = 8.0, q[3] = 0.0, q[4] = 0.0, q[5] = 1.0;
        }
        run_case(2, 0, n, s, 5, P, 1, 17);
        run_case(2, 1, n, s, 5, Q, 1, 17);
    }
    printf("oracle_check OK\n");
    return 0;
}
