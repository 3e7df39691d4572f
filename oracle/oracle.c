/*
 * oracle.c -- FP64 CPU reference for the CT projector operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * library.
 *
 * What it computes (PYRO-NN update, Sec. 2.1 "Modular Layer Design" and
 * Sec. 2.2 "CT Reconstruction in Neural Networks"):
 *
 *   forward A      ray-driven: one ray per detector pixel is cast through the
 *                  volume and the absorption values along it are summed
 *                  (Sec. 2.1).  The sampling is Joseph's plane-crossing rule:
 *                  the ray is cut by every volume plane perpendicular to its
 *                  dominant index-space axis, the volume is (bi)linearly
 *                  interpolated at each crossing with zero padding outside
 *                  the grid, and the sum is scaled by the path length per
 *                  plane.
 *   adjoint  A^T   the exact transpose of A (Sec. 2.2 names the pair
 *                  A, A^T): every interpolation tap of every ray is
 *                  scattered back with the same weight.
 *   back-project   voxel-driven: each voxel centre is projected onto the
 *                  detector with the view's projection matrix, the detector
 *                  value there is (bi)linearly interpolated with zero
 *                  padding, weighted by (W0/W)^2 and summed over views
 *                  (Sec. 2.1; the distance weight is the FDK weight, with
 *                  W0 the W coordinate of the world origin).
 *   splat          the transpose of back-project, its analytic gradient
 *                  (Sec. 2: gradients for all operators): each voxel's
 *                  weighted value is spread over the interpolation taps of
 *                  its projection.
 *
 * Conventions (all readings of the paper, which fixes none of them):
 *   volume     array [nz][ny][nx], voxel (i,j,k) centre at
 *              (ox + i*sx, oy + j*sy, oz + k*sz) in mm;
 *   detector   array [n_views][nv][nu]; pixel (column c, row r) has image
 *              coordinates (u, v) = (c, r);
 *   matrices   3-D: P is 3x4 row-major, (U,V,W) = P (x,y,z,1), u = U/W,
 *              v = V/W.  Cone beam uses a general P; parallel beam has last
 *              row (0,0,0,w).  2-D: P is 2x3, (U,W) = P (x,y,1), u = U/W;
 *              parallel beam has last row (0,0,w);
 *   rays       perspective: source S = -M^-1 p4 and direction
 *              D = M^-1 (u,v,1), M = P[:, :3], p4 = P[:, 3].  Parallel:
 *              D spans the null space of the first two rows' linear part,
 *              and the ray passes through the least-norm solution of
 *              P[0:2] (X,1) = (u,v).  2-D analogously;
 *   Joseph     index-space line xi(t) = xi0 + t*delta with xi0 = (X0-o)/s
 *              and delta = D/s; dominant axis a = argmax |delta_a|, exact
 *              ties resolved to the lowest axis (x, then y, then z); for
 *              every plane m = 0..n_a-1 the crossing is
 *              xi0 + ((m - xi0_a)/delta_a) delta; the ray sum is multiplied
 *              by ds = s_a |D| / |D_a|, the mm of ray per plane.  The whole
 *              line is integrated (no clipping to a source-detector segment).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n[3];   /* nx, ny, nz */
    double s[3];    /* sx, sy, sz */
    double o[3];    /* world position of voxel (0,0,0) centre, (x, y, z) */
} grid_t;

typedef struct {
    double x0[3];   /* a point on the ray, world mm (x, y, z)  */
    double d[3];    /* ray direction, world (any scale) */
} ray_t;

/* ---------------------------------------------------------------- rays -- */

static int inverse3(const double m[9], double inv[9])
{
    double det = m[0] * (m[4] * m[8] - m[5] * m[7])
               - m[1] * (m[3] * m[8] - m[5] * m[6])
               + m[2] * (m[3] * m[7] - m[4] * m[6]);
    if (det == 0.0 || !isfinite(det)) return -1;
    inv[0] = (m[4] * m[8] - m[5] * m[7]) / det;
    inv[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    inv[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    inv[3] = (m[5] * m[6] - m[3] * m[8]) / det;
    inv[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    inv[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    inv[6] = (m[3] * m[7] - m[4] * m[6]) / det;
    inv[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    inv[8] = (m[0] * m[4] - m[1] * m[3]) / det;
    return 0;
}

/* The ray through pixel (u, v) for a 3x4 matrix P (row-major). */
static void ray_3d(int parallel, const double P[12], double u, double v, ray_t *ray)
{
    if (!parallel) {
        double M[9] = {P[0], P[1], P[2], P[4], P[5], P[6], P[8], P[9], P[10]};
        double Mi[9];
        if (inverse3(M, Mi) != 0)
            for (int i = 0; i < 9; ++i) Mi[i] = NAN;
        for (int i = 0; i < 3; ++i) {
            ray->x0[i] = -(Mi[3 * i] * P[3] + Mi[3 * i + 1] * P[7] + Mi[3 * i + 2] * P[11]);
            ray->d[i] = Mi[3 * i] * u + Mi[3 * i + 1] * v + Mi[3 * i + 2];
        }
    } else {
        /* rows divided by the constant last-row entry w */
        double w = P[11];
        double a[3] = {P[0] / w, P[1] / w, P[2] / w}, b[3] = {P[4] / w, P[5] / w, P[6] / w};
        double ru = u - P[3] / w, rv = v - P[7] / w;
        /* direction: null space of [a; b] */
        ray->d[0] = a[1] * b[2] - a[2] * b[1];
        ray->d[1] = a[2] * b[0] - a[0] * b[2];
        ray->d[2] = a[0] * b[1] - a[1] * b[0];
        /* least-norm X with a.X = ru, b.X = rv: X = [a b] G^-1 (ru, rv) */
        double g00 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
        double g01 = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
        double g11 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        double det = g00 * g11 - g01 * g01;
        double ca = (g11 * ru - g01 * rv) / det, cb = (g00 * rv - g01 * ru) / det;
        for (int i = 0; i < 3; ++i) ray->x0[i] = ca * a[i] + cb * b[i];
    }
}

/* The ray through detector coordinate u for a 2x3 matrix P (row-major). */
static void ray_2d(int parallel, const double P[6], double u, ray_t *ray)
{
    if (!parallel) {
        double det = P[0] * P[4] - P[1] * P[3];
        double i00 = P[4] / det, i01 = -P[1] / det, i10 = -P[3] / det, i11 = P[0] / det;
        ray->x0[0] = -(i00 * P[2] + i01 * P[5]);
        ray->x0[1] = -(i10 * P[2] + i11 * P[5]);
        ray->d[0] = i00 * u + i01;
        ray->d[1] = i10 * u + i11;
    } else {
        double w = P[5];
        double a = P[0] / w, b = P[1] / w, c = P[2] / w;
        ray->d[0] = -b;
        ray->d[1] = a;
        double t = (u - c) / (a * a + b * b);
        ray->x0[0] = a * t;
        ray->x0[1] = b * t;
    }
    ray->x0[2] = 0.0;
    ray->d[2] = 0.0;
}

/* ------------------------------------------------------ Joseph sampling -- */

/* Enumerate the interpolation taps of one ray.  Writes linear voxel indices
 * (k*ny + j)*nx + i to idx[] and weight * ds to w[]; returns the tap count.
 * dims = 2 uses linear interpolation in the single in-plane axis (nz == 1),
 * dims = 3 bilinear interpolation in the two in-plane axes.  Taps outside
 * the grid are dropped (zero padding).  Capacity needed: 4 * max(n). */
/* Upper-tap weight of a crossing at fraction wf of a voxel: wf itself, or,
 * with wbits = B > 0 (the sampler variant's reduced-precision weights), wf
 * rounded to the nearest multiple of 2^-B, ties upward.  t = wf 2^B, its
 * floor q and t - q are exact, so the rounding decision is exact. */
static double tap_weight(double wf, int wbits)
{
    if (wbits <= 0) return wf;
    double sc = ldexp(1.0, wbits);
    double t = wf * sc, q = floor(t);
    if (t - q >= 0.5) q += 1.0;
    return q / sc;
}

static int64_t ray_taps_planes(const grid_t *g, int dims, const ray_t *ray, const int64_t *plane_box,
                               int wbits, int64_t *idx, double *w)
{
    double xi0[3], de[3];
    for (int i = 0; i < 3; ++i) {
        xi0[i] = (ray->x0[i] - g->o[i]) / g->s[i];
        de[i] = ray->d[i] / g->s[i];
    }
    int a = 0;
    if (dims == 2) {
        a = fabs(de[0]) >= fabs(de[1]) ? 0 : 1;
    } else {
        if (fabs(de[0]) >= fabs(de[1]) && fabs(de[0]) >= fabs(de[2])) a = 0;
        else if (fabs(de[1]) >= fabs(de[2])) a = 1;
        else a = 2;
    }
    double dnorm = sqrt(ray->d[0] * ray->d[0] + ray->d[1] * ray->d[1] + ray->d[2] * ray->d[2]);
    double ds = g->s[a] * dnorm / fabs(ray->d[a]);
    /* the in-plane axes (dims == 2: only the other of x/y) */
    int b = (a == 0) ? 1 : 0;
    int c = (a == 2) ? 1 : 2;
    int64_t cnt = 0;
    /* plane_box (i0,i1,j0,j1,k0,k1), if given, limits the planes visited to
       those of the box along the dominant axis: a tap of plane m lies in
       plane m, so other planes cannot reach the box */
    int64_t m_lo = 0, m_hi = g->n[a];
    if (plane_box) {
        if (plane_box[2 * a] > m_lo) m_lo = plane_box[2 * a];
        if (plane_box[2 * a + 1] < m_hi) m_hi = plane_box[2 * a + 1];
    }
    for (int64_t m = m_lo; m < m_hi; ++m) {
        double t = ((double)m - xi0[a]) / de[a];
        double pb = xi0[b] + t * de[b];
        double fb = floor(pb), wb = tap_weight(pb - fb, wbits);
        int64_t ib = (int64_t)fb;
        if (dims == 2) {
            for (int tb = 0; tb < 2; ++tb) {
                int64_t jb = ib + tb;
                if (jb < 0 || jb >= g->n[b]) continue;
                int64_t ijk[3];
                ijk[a] = m; ijk[b] = jb; ijk[2] = 0;
                idx[cnt] = ijk[1] * g->n[0] + ijk[0];
                w[cnt] = (tb ? wb : 1.0 - wb) * ds;
                ++cnt;
            }
        } else {
            double pc = xi0[c] + t * de[c];
            double fc = floor(pc), wc = tap_weight(pc - fc, wbits);
            int64_t ic = (int64_t)fc;
            for (int tc = 0; tc < 2; ++tc) {
                int64_t jc = ic + tc;
                if (jc < 0 || jc >= g->n[c]) continue;
                for (int tb = 0; tb < 2; ++tb) {
                    int64_t jb = ib + tb;
                    if (jb < 0 || jb >= g->n[b]) continue;
                    int64_t ijk[3];
                    ijk[a] = m; ijk[b] = jb; ijk[c] = jc;
                    idx[cnt] = (ijk[2] * g->n[1] + ijk[1]) * g->n[0] + ijk[0];
                    w[cnt] = (tb ? wb : 1.0 - wb) * (tc ? wc : 1.0 - wc) * ds;
                    ++cnt;
                }
            }
        }
    }
    return cnt;
}

static int64_t ray_taps(const grid_t *g, int dims, const ray_t *ray, int64_t *idx, double *w)
{
    return ray_taps_planes(g, dims, ray, NULL, 0, idx, w);
}

static void make_grid(grid_t *g, const int64_t n[3], const double s[3], const double o[3])
{
    for (int i = 0; i < 3; ++i) { g->n[i] = n[i]; g->s[i] = s[i]; g->o[i] = o[i]; }
}

static int64_t max_n(const grid_t *g)
{
    int64_t m = g->n[0];
    if (g->n[1] > m) m = g->n[1];
    if (g->n[2] > m) m = g->n[2];
    return m;
}

static void pixel_ray(const grid_t *g, int dims, int parallel, const double *P, int64_t r, int64_t c, ray_t *ray)
{
    (void)g;
    if (dims == 2) ray_2d(parallel, P, (double)c, ray);
    else ray_3d(parallel, P, (double)c, (double)r, ray);
}

/* ------------------------------------------------------------- exports -- */

/* Forward projection A.  n = (nx, ny, nz), s, o in (x, y, z) order.
 * P: n_views matrices (2x3 when dims == 2, else 3x4).  sino: [n_views][nv][nu]
 * (nv == 1 when dims == 2).  wbits > 0: the sampler variant, whose in-plane
 * interpolation weights are rounded to multiples of 2^-wbits (tap_weight);
 * oracle_forward is wbits = 0, the operator A itself. */
int oracle_forward_q(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                     int64_t n_views, const double *P, int64_t nv, int64_t nu,
                     const double *vol, double *sino, int nthreads, int wbits)
{
    grid_t g;
    make_grid(&g, n, s, o);
    int64_t cap = 4 * max_n(&g) + 4;
    int64_t psz = dims == 2 ? 6 : 12;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *w = (double *)malloc(sizeof(double) * cap);
        if (!idx || !w) err = 1;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < n_views; ++k) {
            if (!idx || !w) continue;
            for (int64_t r = 0; r < nv; ++r)
                for (int64_t c = 0; c < nu; ++c) {
                    ray_t ray;
                    pixel_ray(&g, dims, parallel, P + k * psz, r, c, &ray);
                    int64_t cnt = ray_taps_planes(&g, dims, &ray, NULL, wbits, idx, w);
                    double acc = 0.0;
                    for (int64_t t = 0; t < cnt; ++t) acc += w[t] * vol[idx[t]];
                    sino[(k * nv + r) * nu + c] = acc;
                }
        }
        free(idx);
        free(w);
    }
    return err;
}

int oracle_forward(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                   int64_t n_views, const double *P, int64_t nv, int64_t nu,
                   const double *vol, double *sino, int nthreads)
{
    return oracle_forward_q(dims, parallel, n, s, o, n_views, P, nv, nu, vol, sino, nthreads, 0);
}

/* Forward projection of selected rays only: out[t] = (A vol)[view[t], row[t], col[t]]
 * (wbits as oracle_forward_q). */
int oracle_forward_rays_q(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                          const double *P, const double *vol, int64_t n_rays, const int64_t *view,
                          const int64_t *row, const int64_t *col, double *out, int nthreads, int wbits)
{
    grid_t g;
    make_grid(&g, n, s, o);
    int64_t cap = 4 * max_n(&g) + 4;
    int64_t psz = dims == 2 ? 6 : 12;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *w = (double *)malloc(sizeof(double) * cap);
        if (!idx || !w) err = 1;
#pragma omp for schedule(static)
        for (int64_t t = 0; t < n_rays; ++t) {
            if (!idx || !w) continue;
            ray_t ray;
            pixel_ray(&g, dims, parallel, P + view[t] * psz, row[t], col[t], &ray);
            int64_t cnt = ray_taps_planes(&g, dims, &ray, NULL, wbits, idx, w);
            double acc = 0.0;
            for (int64_t q = 0; q < cnt; ++q) acc += w[q] * vol[idx[q]];
            out[t] = acc;
        }
        free(idx);
        free(w);
    }
    return err;
}

int oracle_forward_rays(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                        const double *P, const double *vol, int64_t n_rays, const int64_t *view,
                        const int64_t *row, const int64_t *col, double *out, int nthreads)
{
    return oracle_forward_rays_q(dims, parallel, n, s, o, P, vol, n_rays, view, row, col, out, nthreads, 0);
}

/* Adjoint A^T restricted to a box of voxels.  box = (i0, i1, j0, j1, k0, k1),
 * half-open; the output holds the box only, [k1-k0][j1-j0][i1-i0].  Pass the
 * full extents for the whole volume.  Each thread scatters the views it owns
 * into a private accumulator; the accumulators are summed in thread order. */
int oracle_adjoint(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                   int64_t n_views, const double *P, int64_t nv, int64_t nu,
                   const double *sino, const int64_t box[6], double *out, int nthreads)
{
    grid_t g;
    make_grid(&g, n, s, o);
    int64_t cap = 4 * max_n(&g) + 4;
    int64_t psz = dims == 2 ? 6 : 12;
    int64_t bx = box[1] - box[0], by = box[3] - box[2], bz = box[5] - box[4];
    int64_t nout = bx * by * bz;
    int nthr = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    nthr = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nthr * (size_t)nout, sizeof(double));
    if (!priv) return 1;
    int err = 0;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = priv + (size_t)tid * (size_t)nout;
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *w = (double *)malloc(sizeof(double) * cap);
        if (!idx || !w) err = 1;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < n_views; ++k) {
            if (!idx || !w) continue;
            for (int64_t r = 0; r < nv; ++r)
                for (int64_t c = 0; c < nu; ++c) {
                    double q = sino[(k * nv + r) * nu + c];
                    ray_t ray;
                    pixel_ray(&g, dims, parallel, P + k * psz, r, c, &ray);
                    int64_t cnt = ray_taps_planes(&g, dims, &ray, box, 0, idx, w);
                    for (int64_t t = 0; t < cnt; ++t) {
                        int64_t e = idx[t];
                        int64_t i = e % g.n[0], j = (e / g.n[0]) % g.n[1], kk = e / (g.n[0] * g.n[1]);
                        if (i < box[0] || i >= box[1] || j < box[2] || j >= box[3] || kk < box[4] || kk >= box[5])
                            continue;
                        acc[((kk - box[4]) * by + (j - box[2])) * bx + (i - box[0])] += w[t] * q;
                    }
                }
        }
        free(idx);
        free(w);
    }
    for (int64_t e = 0; e < nout; ++e) {
        double sum = 0.0;
        for (int t = 0; t < nthr; ++t) sum += priv[(size_t)t * (size_t)nout + e];
        out[e] = sum;
    }
    free(priv);
    return err;
}

/* Zero-padded linear (dims 2) / bilinear (dims 3) detector sample. */
static double detector_sample(const double *img, int64_t nv, int64_t nu, double u, double v, int dims, int wbits)
{
    double fu = floor(u), wu = tap_weight(u - fu, wbits);
    int64_t iu = (int64_t)fu;
    if (dims == 2) {
        double val = 0.0;
        if (iu >= 0 && iu < nu) val += (1.0 - wu) * img[iu];
        if (iu + 1 >= 0 && iu + 1 < nu) val += wu * img[iu + 1];
        return val;
    }
    double fv = floor(v), wv = tap_weight(v - fv, wbits);
    int64_t iv = (int64_t)fv;
    double val = 0.0;
    for (int tv = 0; tv < 2; ++tv) {
        int64_t r = iv + tv;
        if (r < 0 || r >= nv) continue;
        for (int tu = 0; tu < 2; ++tu) {
            int64_t c = iu + tu;
            if (c < 0 || c >= nu) continue;
            val += (tv ? wv : 1.0 - wv) * (tu ? wu : 1.0 - wu) * img[r * nu + c];
        }
    }
    return val;
}

/* Back-projection value at voxel (i, j, k): sum over views of
 * (W0/W)^2 * interp(sino_view, U/W, V/W).  wbits > 0: the sampler variant,
 * detector weights rounded to multiples of 2^-wbits (tap_weight). */
static double bp_voxel(const grid_t *g, int dims, int64_t n_views, const double *P, int64_t nv, int64_t nu,
                       const double *sino, int64_t i, int64_t j, int64_t k, int wbits)
{
    double x = g->o[0] + (double)i * g->s[0];
    double y = g->o[1] + (double)j * g->s[1];
    double z = g->o[2] + (double)k * g->s[2];
    double acc = 0.0;
    for (int64_t view = 0; view < n_views; ++view) {
        const double *img = sino + view * nv * nu;
        if (dims == 2) {
            const double *p = P + view * 6;
            double U = p[0] * x + p[1] * y + p[2];
            double W = p[3] * x + p[4] * y + p[5];
            double W0 = p[5];
            double wt = (W0 / W) * (W0 / W);
            acc += wt * detector_sample(img, 1, nu, U / W, 0.0, 2, wbits);
        } else {
            const double *p = P + view * 12;
            double U = p[0] * x + p[1] * y + p[2] * z + p[3];
            double V = p[4] * x + p[5] * y + p[6] * z + p[7];
            double W = p[8] * x + p[9] * y + p[10] * z + p[11];
            double W0 = p[11];
            double wt = (W0 / W) * (W0 / W);
            acc += wt * detector_sample(img, nv, nu, U / W, V / W, 3, wbits);
        }
    }
    return acc;
}

/* Voxel-driven back-projection of the whole volume (wbits as bp_voxel;
 * oracle_backproject is wbits = 0). */
int oracle_backproject_q(int dims, const int64_t n[3], const double s[3], const double o[3],
                         int64_t n_views, const double *P, int64_t nv, int64_t nu,
                         const double *sino, double *vol, int nthreads, int wbits)
{
    grid_t g;
    make_grid(&g, n, s, o);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static) collapse(2)
    for (int64_t k = 0; k < g.n[2]; ++k)
        for (int64_t j = 0; j < g.n[1]; ++j)
            for (int64_t i = 0; i < g.n[0]; ++i)
                vol[(k * g.n[1] + j) * g.n[0] + i] = bp_voxel(&g, dims, n_views, P, nv, nu, sino, i, j, k, wbits);
    return 0;
}

int oracle_backproject(int dims, const int64_t n[3], const double s[3], const double o[3],
                       int64_t n_views, const double *P, int64_t nv, int64_t nu,
                       const double *sino, double *vol, int nthreads)
{
    return oracle_backproject_q(dims, n, s, o, n_views, P, nv, nu, sino, vol, nthreads, 0);
}

/* Back-projection at selected voxels only (wbits as bp_voxel). */
int oracle_backproject_voxels_q(int dims, const int64_t n[3], const double s[3], const double o[3],
                                int64_t n_views, const double *P, int64_t nv, int64_t nu,
                                const double *sino, int64_t n_vox, const int64_t *vi, const int64_t *vj,
                                const int64_t *vk, double *out, int nthreads, int wbits)
{
    grid_t g;
    make_grid(&g, n, s, o);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n_vox; ++t)
        out[t] = bp_voxel(&g, dims, n_views, P, nv, nu, sino, vi[t], vj[t], vk[t], wbits);
    return 0;
}

int oracle_backproject_voxels(int dims, const int64_t n[3], const double s[3], const double o[3],
                              int64_t n_views, const double *P, int64_t nv, int64_t nu,
                              const double *sino, int64_t n_vox, const int64_t *vi, const int64_t *vj,
                              const int64_t *vk, double *out, int nthreads)
{
    return oracle_backproject_voxels_q(dims, n, s, o, n_views, P, nv, nu, sino, n_vox, vi, vj, vk, out,
                                       nthreads, 0);
}

/* Transpose of the voxel-driven back-projection (the splat projector):
 * every voxel centre is projected onto each view's detector and its value,
 * times the distance weight (W0/W)^2, is spread over the (bi)linear
 * interpolation taps of its projection (zero padding: taps off the detector
 * are dropped), so that <backproject(q), x> = <q, splat(x)>.  sino:
 * [n_views][nv][nu], overwritten.  Parallel over views. */
int oracle_splat(int dims, const int64_t n[3], const double s[3], const double o[3], int64_t n_views,
                 const double *P, int64_t nv, int64_t nu, const double *vol, double *sino, int nthreads)
{
    grid_t g;
    make_grid(&g, n, s, o);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
    for (int64_t view = 0; view < n_views; ++view) {
        double *img = sino + view * nv * nu;
        for (int64_t e = 0; e < nv * nu; ++e) img[e] = 0.0;
        for (int64_t k = 0; k < g.n[2]; ++k)
            for (int64_t j = 0; j < g.n[1]; ++j)
                for (int64_t i = 0; i < g.n[0]; ++i) {
                    const double val = vol[(k * g.n[1] + j) * g.n[0] + i];
                    const double x = g.o[0] + (double)i * g.s[0];
                    const double y = g.o[1] + (double)j * g.s[1];
                    const double z = g.o[2] + (double)k * g.s[2];
                    double u, v = 0.0, W, W0;
                    if (dims == 2) {
                        const double *p = P + view * 6;
                        W = p[3] * x + p[4] * y + p[5];
                        u = (p[0] * x + p[1] * y + p[2]) / W;
                        W0 = p[5];
                    } else {
                        const double *p = P + view * 12;
                        W = p[8] * x + p[9] * y + p[10] * z + p[11];
                        u = (p[0] * x + p[1] * y + p[2] * z + p[3]) / W;
                        v = (p[4] * x + p[5] * y + p[6] * z + p[7]) / W;
                        W0 = p[11];
                    }
                    const double wt = (W0 / W) * (W0 / W) * val;
                    const double fu = floor(u), wu = u - fu;
                    const double fv = floor(v), wv = v - fv;
                    const int64_t iu = (int64_t)fu, iv = (int64_t)fv;
                    for (int tv = 0; tv < (dims == 2 ? 1 : 2); ++tv) {
                        const int64_t r = iv + tv;
                        if (r < 0 || r >= nv) continue;
                        const double fvw = dims == 2 ? 1.0 : (tv ? wv : 1.0 - wv);
                        for (int tu = 0; tu < 2; ++tu) {
                            const int64_t c = iu + tu;
                            if (c < 0 || c >= nu) continue;
                            img[r * nu + c] += wt * fvw * (tu ? wu : 1.0 - wu);
                        }
                    }
                }
    }
    return 0;
}

/* The taps of one ray, for brute-force matrix checks: returns the count and
 * fills idx/w (capacity 4*max(n)+4). */
int64_t oracle_ray_taps(int dims, int parallel, const int64_t n[3], const double s[3], const double o[3],
                        const double *P, int64_t r, int64_t c, int64_t *idx, double *w)
{
    grid_t g;
    make_grid(&g, n, s, o);
    ray_t ray;
    pixel_ray(&g, dims, parallel, P, r, c, &ray);
    return ray_taps(&g, dims, &ray, idx, w);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
