// Host-side parts of the CT projector library that need no device: error
// text, argument and geometry validation, the FP64 per-view tables, and the
// projection-matrix composition entry points of include/pyronn_mi.h
// (pn_check_geometry, pn_*_matrices, pn_last_error).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <limits>

#include "pn_internal.hpp"

namespace {

thread_local std::string t_err;

}  // namespace

namespace pn {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

void clear_error() { t_err.clear(); }

int64_t esize(int32_t dt) { return dt == PN_F32 ? 4 : 2; }

bool dtype_ok(int32_t dt) { return dt == PN_F32 || dt == PN_BF16 || dt == PN_F16; }

// --------------------------------------------------------- small algebra --

bool inv3(const double m[9], double r[9])
{
    double c0 = m[4] * m[8] - m[5] * m[7];
    double c1 = m[5] * m[6] - m[3] * m[8];
    double c2 = m[3] * m[7] - m[4] * m[6];
    double det = m[0] * c0 + m[1] * c1 + m[2] * c2;
    double n0 = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    double n1 = std::sqrt(m[3] * m[3] + m[4] * m[4] + m[5] * m[5]);
    double n2 = std::sqrt(m[6] * m[6] + m[7] * m[7] + m[8] * m[8]);
    if (!std::isfinite(det) || std::fabs(det) <= 1e-12 * n0 * n1 * n2) return false;
    double id = 1.0 / det;
    r[0] = c0 * id;
    r[1] = (m[2] * m[7] - m[1] * m[8]) * id;
    r[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    r[3] = c1 * id;
    r[4] = (m[0] * m[8] - m[2] * m[6]) * id;
    r[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    r[6] = c2 * id;
    r[7] = (m[1] * m[6] - m[0] * m[7]) * id;
    r[8] = (m[0] * m[4] - m[1] * m[3]) * id;
    return true;
}

// --------------------------------------------------------- geometry -------

int normalise_geometry(const pn_geometry *pg, Geo &g)
{
    if (!pg) return fail(PN_EINVAL, "geometry pointer is NULL");
    if (pg->ndim != 2 && pg->ndim != 3) return fail(PN_EINVAL, "ndim must be 2 or 3 (got %d)", pg->ndim);
    if (pg->ndim == 2 && pg->beam != PN_PARALLEL && pg->beam != PN_FAN)
        return fail(PN_EINVAL, "2-D geometry needs beam PN_PARALLEL or PN_FAN (got %d)", pg->beam);
    if (pg->ndim == 3 && pg->beam != PN_PARALLEL && pg->beam != PN_CONE)
        return fail(PN_EINVAL, "3-D geometry needs beam PN_PARALLEL or PN_CONE (got %d)", pg->beam);
    const int64_t lim = 65535;
    for (int a = 0; a < 3; ++a)
        if (pg->vol_shape[a] < 1 || pg->vol_shape[a] > lim)
            return fail(PN_EINVAL, "vol_shape[%d] = %lld outside [1, %lld]", a, (long long)pg->vol_shape[a],
                        (long long)lim);
    for (int a = 0; a < 2; ++a)
        if (pg->det_shape[a] < 1 || pg->det_shape[a] > lim)
            return fail(PN_EINVAL, "det_shape[%d] = %lld outside [1, %lld]", a, (long long)pg->det_shape[a],
                        (long long)lim);
    if (pg->ndim == 2 && pg->vol_shape[0] != 1) return fail(PN_EINVAL, "2-D geometry needs vol_shape[0] == 1");
    if (pg->ndim == 2 && pg->det_shape[0] != 1) return fail(PN_EINVAL, "2-D geometry needs det_shape[0] == 1");
    const int64_t item = pg->vol_shape[0] * pg->vol_shape[1] * pg->vol_shape[2];
    if (item > INT32_MAX) return fail(PN_EINVAL, "volume has more than 2^31-1 voxels");
    if (pg->n_views < 0 || pg->n_views > 1000000) return fail(PN_EINVAL, "n_views = %lld out of range",
                                                              (long long)pg->n_views);
    if (pg->n_views * pg->det_shape[0] * pg->det_shape[1] > INT32_MAX)
        return fail(PN_EINVAL, "sinogram has more than 2^31-1 pixels");
    for (int a = (pg->ndim == 2 ? 1 : 0); a < 3; ++a)
        if (!std::isfinite(pg->vol_spacing[a]) || !(pg->vol_spacing[a] > 0))
            return fail(PN_EINVAL, "vol_spacing[%d] must be finite and > 0", a);
    for (int a = 0; a < 3; ++a)
        if (std::isinf(pg->vol_origin[a])) return fail(PN_EINVAL, "vol_origin[%d] is infinite", a);
    if (pg->n_views > 0 && !pg->proj) return fail(PN_EINVAL, "proj is NULL");

    g.ndim = pg->ndim;
    g.beam = pg->beam;
    g.parallel = pg->beam == PN_PARALLEL;
    g.n[0] = (int32_t)pg->vol_shape[2];
    g.n[1] = (int32_t)pg->vol_shape[1];
    g.n[2] = (int32_t)pg->vol_shape[0];
    g.s[0] = pg->vol_spacing[2];
    g.s[1] = pg->vol_spacing[1];
    g.s[2] = pg->ndim == 2 ? 1.0 : pg->vol_spacing[0];
    for (int a = 0; a < 3; ++a) {
        double org = pg->vol_origin[2 - a];
        g.o[a] = std::isnan(org) ? -0.5 * (g.n[a] - 1) * g.s[a] : org;
    }
    if (pg->ndim == 2) g.o[2] = 0.0;
    g.nv = (int32_t)pg->det_shape[0];
    g.nu = (int32_t)pg->det_shape[1];
    g.n_views = (int32_t)pg->n_views;
    const int psz = pg->ndim == 2 ? 6 : 12;
    g.raw.assign(pg->proj, pg->proj + (size_t)psz * g.n_views);
    double sc[16] = {g.s[0], g.s[1], g.s[2], g.o[0], g.o[1], g.o[2]};
    std::memcpy(g.raw_scalars, sc, sizeof sc);
    g.P.resize((size_t)12 * g.n_views);
    for (int k = 0; k < g.n_views; ++k) {
        const double *q = pg->proj + (size_t)psz * k;
        double *P = &g.P[(size_t)12 * k];
        for (int e = 0; e < psz; ++e)
            if (!std::isfinite(q[e])) return fail(PN_EGEOM, "view %d: non-finite matrix entry", k);
        if (pg->ndim == 2) {
            // (U, W) = P2 (x, y, 1) embedded as rows (U, V = z, W)
            double e3[12] = {q[0], q[1], 0.0, q[2], 0.0, 0.0, 1.0, 0.0, q[3], q[4], 0.0, q[5]};
            std::memcpy(P, e3, sizeof e3);
        } else {
            std::memcpy(P, q, sizeof(double) * 12);
        }
        double scale = 0;
        for (int e = 0; e < 12; ++e) scale = std::max(scale, std::fabs(P[e]));
        if (!(scale > 0)) return fail(PN_EGEOM, "view %d: zero matrix", k);
        if (g.parallel) {
            if (std::fabs(P[8]) > 1e-12 * scale || std::fabs(P[9]) > 1e-12 * scale || std::fabs(P[10]) > 1e-12 * scale ||
                P[11] == 0.0)
                return fail(PN_EGEOM, "view %d: a parallel-beam matrix needs last row (0, 0, 0, w), w != 0", k);
            P[8] = P[9] = P[10] = 0.0;
            if (P[11] < 0)
                for (int e = 0; e < 12; ++e) P[e] = -P[e];
            double a[3] = {P[0], P[1], P[2]}, b[3] = {P[4], P[5], P[6]};
            double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
            double na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            double nb = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
            if (!(std::sqrt(cx * cx + cy * cy + cz * cz) > 1e-12 * na * nb))
                return fail(PN_EGEOM, "view %d: parallel-beam matrix rows are dependent", k);
        } else {
            double M[9] = {P[0], P[1], P[2], P[4], P[5], P[6], P[8], P[9], P[10]}, Mi[9];
            if (!inv3(M, Mi)) return fail(PN_EGEOM, "view %d: singular 3x3 block", k);
            // sign: W > 0 at the volume centre
            double c[3];
            for (int a = 0; a < 3; ++a) c[a] = g.o[a] + 0.5 * (g.n[a] - 1) * g.s[a];
            double Wc = P[8] * c[0] + P[9] * c[1] + P[10] * c[2] + P[11];
            if (Wc < 0)
                for (int e = 0; e < 12; ++e) P[e] = -P[e];
            // the whole volume, dilated by one voxel, must be in front of the source
            for (int corner = 0; corner < 8; ++corner) {
                double X[3];
                for (int a = 0; a < 3; ++a) {
                    double idx = (corner >> a & 1) ? (double)g.n[a] : -1.0;
                    X[a] = g.o[a] + idx * g.s[a];
                }
                if (pg->ndim == 2) X[2] = 0.0;
                double W = P[8] * X[0] + P[9] * X[1] + P[10] * X[2] + P[11];
                if (!(W > 1e-12 * scale))
                    return fail(PN_EGEOM, "view %d: the volume (dilated by one voxel) is not entirely in front of the source", k);
            }
        }
    }
    return PN_OK;
}

// Sutherland-Hodgman: keep the part of a convex polygon with a*u + b*v + c >= 0.
void clip_poly(std::vector<double> &poly, double a, double b, double c)
{
    std::vector<double> out;
    const size_t n = poly.size() / 2;
    for (size_t i = 0; i < n; ++i) {
        double u0 = poly[2 * i], v0 = poly[2 * i + 1];
        double u1 = poly[2 * ((i + 1) % n)], v1 = poly[2 * ((i + 1) % n) + 1];
        double f0 = a * u0 + b * v0 + c, f1 = a * u1 + b * v1 + c;
        if (f0 >= 0) { out.push_back(u0); out.push_back(v0); }
        if ((f0 >= 0) != (f1 >= 0)) {
            double t = f0 / (f0 - f1);
            out.push_back(u0 + t * (u1 - u0));
            out.push_back(v0 + t * (v1 - v0));
        }
    }
    poly.swap(out);
}

// Which dominant axes can occur among the view's rays (conservative: near
// ties count for both axes).  delta(u, v) = A (u, v, 1) is linear in (u, v),
// so the pixels (centres in [0, nu-1] x [0, nv-1]) where axis a dominates
// with sign sg form the detector rectangle clipped by four half-planes
// sg delta_a +- delta_b >= 0.  box[a] receives the bounding box of those
// pixels, widened by one pixel and clamped to the detector, as two words
// (first column | first row << 16, last column | last row << 16); the
// adjoint takes its candidate rays of pass a from inside it.
int32_t axis_mask(const double A[9], int32_t nu, int32_t nv, uint32_t box[3][2])
{
    const double U = nu - 1, V = nv - 1;
    double dmax = 0;
    for (int cu = 0; cu < 2; ++cu)
        for (int cv = 0; cv < 2; ++cv)
            for (int i = 0; i < 3; ++i)
                dmax = std::max(dmax, std::fabs(A[3 * i] * cu * U + A[3 * i + 1] * cv * V + A[3 * i + 2]));
    const double tau = 1e-9 * dmax;
    int32_t mask = 0;
    for (int a = 0; a < 3; ++a) {
        double u0 = HUGE_VAL, u1 = -HUGE_VAL, v0 = HUGE_VAL, v1 = -HUGE_VAL;
        for (int sg = -1; sg <= 1; sg += 2) {
            std::vector<double> poly = {0, 0, U, 0, U, V, 0, V};
            for (int b = 0; b < 3 && !poly.empty(); ++b) {
                if (b == a) continue;
                for (int pm = -1; pm <= 1 && !poly.empty(); pm += 2) {
                    // sg*delta_a + pm*delta_b >= -tau
                    clip_poly(poly, sg * A[3 * a] + pm * A[3 * b], sg * A[3 * a + 1] + pm * A[3 * b + 1],
                              sg * A[3 * a + 2] + pm * A[3 * b + 2] + tau);
                }
            }
            if (!poly.empty()) mask |= 1 << a;
            for (size_t i = 0; i + 1 < poly.size(); i += 2) {
                u0 = std::min(u0, poly[i]);
                u1 = std::max(u1, poly[i]);
                v0 = std::min(v0, poly[i + 1]);
                v1 = std::max(v1, poly[i + 1]);
            }
        }
        if (mask & (1 << a)) {
            const uint32_t c0 = (uint32_t)std::min(std::max(std::floor(u0) - 1.0, 0.0), U);
            const uint32_t c1 = (uint32_t)std::min(std::max(std::ceil(u1) + 1.0, 0.0), U);
            const uint32_t r0 = (uint32_t)std::min(std::max(std::floor(v0) - 1.0, 0.0), V);
            const uint32_t r1 = (uint32_t)std::min(std::max(std::ceil(v1) + 1.0, 0.0), V);
            box[a][0] = c0 | r0 << 16;
            box[a][1] = c1 | r1 << 16;
        } else {
            box[a][0] = 1u;  // empty: first column after the last
            box[a][1] = 0u;
        }
    }
    return mask;
}

// Upper bound on the number of rays of one view whose sample in some plane
// lies within one voxel, in both in-plane axes, of a given voxel (the rays
// that can add to that voxel in the adjoint).  Such a sample lies in a 2 x 2
// square of the plane around the voxel; the ray's pixel is the projection
// of the sample, so it lies in the projection of the square, which fits in
// a detector box of 2 Du x 2 Dv pixels, Du bounding |du/df| + |du/ds| over
// the dilated volume (mean value theorem).  With u = U/W,
// du/dx_c = (Pi_0c - u Pi_2c) / W, and over the box W >= Wmin > 0 and
// |u| <= max |u| at the corners (u is linear-fractional).  The box holds at
// most (floor(2 Du) + 1) (floor(2 Dv) + 1) pixel centres.  The sum over all
// three axes covers every pass.
double cell_ray_bound(const double *Pi, const Geo &g)
{
    double wmin = std::numeric_limits<double>::infinity(), umax = 0.0, vmax = 0.0;
    for (int c = 0; c < 8; ++c) {
        const double x = (c & 1) ? g.n[0] : -1.0, y = (c & 2) ? g.n[1] : -1.0, z = (c & 4) ? g.n[2] : -1.0;
        const double U = Pi[0] * x + Pi[1] * y + Pi[2] * z + Pi[3];
        const double V = Pi[4] * x + Pi[5] * y + Pi[6] * z + Pi[7];
        const double W = Pi[8] * x + Pi[9] * y + Pi[10] * z + Pi[11];
        wmin = std::min(wmin, W);
        umax = std::max(umax, std::fabs(U / W));
        vmax = std::max(vmax, std::fabs(V / W));
    }
    double du = 0.0, dv = 0.0;
    for (int c = 0; c < 3; ++c) {
        du += (std::fabs(Pi[c]) + umax * std::fabs(Pi[8 + c])) / wmin;
        dv += (std::fabs(Pi[4 + c]) + vmax * std::fabs(Pi[8 + c])) / wmin;
    }
    const double cu = std::min(std::ceil(2.0 * du * (1.0 + 1e-9)) + 1.0, (double)g.nu);
    const double cv = std::min(std::ceil(2.0 * dv * (1.0 + 1e-9)) + 1.0, (double)g.nv);
    return std::max(cu * cv, 1.0);
}

void build_host_tables(const Geo &g, HostTables &pl)
{
    pl.tab.resize(g.n_views);
    pl.tabf.resize(g.n_views);
    for (int a = 0; a < 3; ++a) pl.pass_views[a].clear();
    pl.axes_union = 0;
    double umin = HUGE_VAL, umax = -HUGE_VAL, vmin = HUGE_VAL, vmax = -HUGE_VAL;
    pl.vwin.assign((size_t)4 * g.n_views, 0);
    pl.axbox.assign((size_t)6 * g.n_views, 0u);
    for (int k = 0; k < g.n_views; ++k) {
        const double *P = &g.P[(size_t)12 * k];
        ViewTab &t = pl.tab[k];
        // index-space matrix: Pi = P [diag(s) o; 0 1]
        for (int r = 0; r < 3; ++r) {
            for (int a = 0; a < 3; ++a) t.Pi[4 * r + a] = P[4 * r + a] * g.s[a];
            t.Pi[4 * r + 3] = P[4 * r + 3] + P[4 * r] * g.o[0] + P[4 * r + 1] * g.o[1] + P[4 * r + 2] * g.o[2];
        }
        std::memset(t.A, 0, sizeof t.A);
        std::memset(t.B, 0, sizeof t.B);
        if (!g.parallel) {
            double M[9] = {t.Pi[0], t.Pi[1], t.Pi[2], t.Pi[4], t.Pi[5], t.Pi[6], t.Pi[8], t.Pi[9], t.Pi[10]};
            inv3(M, t.A);  // validated non-singular (scaling by s keeps it so)
            for (int i = 0; i < 3; ++i)
                t.B[3 * i + 2] = -(t.A[3 * i] * t.Pi[3] + t.A[3 * i + 1] * t.Pi[7] + t.A[3 * i + 2] * t.Pi[11]);
        } else {
            const double w = t.Pi[11];
            double a[3] = {t.Pi[0] / w, t.Pi[1] / w, t.Pi[2] / w};
            double b[3] = {t.Pi[4] / w, t.Pi[5] / w, t.Pi[6] / w};
            double cu = t.Pi[3] / w, cv = t.Pi[7] / w;
            t.A[2] = a[1] * b[2] - a[2] * b[1];
            t.A[5] = a[2] * b[0] - a[0] * b[2];
            t.A[8] = a[0] * b[1] - a[1] * b[0];
            double g00 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
            double g01 = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
            double g11 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
            double det = g00 * g11 - g01 * g01;
            double h00 = g11 / det, h01 = -g01 / det, h11 = g00 / det;
            for (int i = 0; i < 3; ++i) {
                double ku = a[i] * h00 + b[i] * h01;  // coefficient of (u - cu)
                double kv = a[i] * h01 + b[i] * h11;  // coefficient of (v - cv)
                t.B[3 * i] = ku;
                t.B[3 * i + 1] = kv;
                t.B[3 * i + 2] = -(ku * cu + kv * cv);
            }
        }
        ViewTabF &tf = pl.tabf[k];
        for (int e = 0; e < 12; ++e) tf.Pi[e] = (float)t.Pi[e];
        tf.W0 = (float)P[11];
        tf.axes = axis_mask(t.A, g.nu, g.nv, reinterpret_cast<uint32_t(*)[2]>(&pl.axbox[(size_t)6 * k]));
        tf.kcell = (float)cell_ray_bound(t.Pi, g);
        tf.pad = 0;
        pl.kmax = std::max(pl.kmax, tf.kcell);
        pl.axes_union |= tf.axes;
        // the dilated volume [-1, n] projects into the convex hull of its
        // corners' projections (W > 0 there): rays outside it sum to zero
        double vu0 = HUGE_VAL, vu1 = -HUGE_VAL, vv0 = HUGE_VAL, vv1 = -HUGE_VAL;
        for (int c = 0; c < 8; ++c) {
            const double x = (c & 1) ? g.n[0] : -1.0, y = (c & 2) ? g.n[1] : -1.0, z = (c & 4) ? g.n[2] : -1.0;
            const double U = t.Pi[0] * x + t.Pi[1] * y + t.Pi[2] * z + t.Pi[3];
            const double V = t.Pi[4] * x + t.Pi[5] * y + t.Pi[6] * z + t.Pi[7];
            const double W = t.Pi[8] * x + t.Pi[9] * y + t.Pi[10] * z + t.Pi[11];
            vu0 = std::min(vu0, U / W);
            vu1 = std::max(vu1, U / W);
            vv0 = std::min(vv0, V / W);
            vv1 = std::max(vv1, V / W);
        }
        umin = std::min(umin, vu0);
        umax = std::max(umax, vu1);
        vmin = std::min(vmin, vv0);
        vmax = std::max(vmax, vv1);
        // one pixel of margin for the rounding of the bounds
        const bool fin = std::isfinite(vu0) && std::isfinite(vu1) && std::isfinite(vv0) && std::isfinite(vv1);
        pl.vwin[4 * k] = fin ? (int32_t)std::max(-1.0, std::min((double)g.nu, std::floor(vu0) - 1.0)) : 0;
        pl.vwin[4 * k + 1] = fin ? (int32_t)std::max(-1.0, std::min((double)g.nu, std::ceil(vu1) + 1.0)) : g.nu;
        pl.vwin[4 * k + 2] = fin ? (int32_t)std::max(-1.0, std::min((double)g.nv, std::floor(vv0) - 1.0)) : 0;
        pl.vwin[4 * k + 3] = fin ? (int32_t)std::max(-1.0, std::min((double)g.nv, std::ceil(vv1) + 1.0)) : g.nv;
        for (int a = 0; a < 3; ++a)
            if (tf.axes >> a & 1) pl.pass_views[a].push_back(k);
    }
    // one pixel of margin for the rounding of the bounds
    if (g.n_views > 0 && std::isfinite(umin) && std::isfinite(umax) && std::isfinite(vmin) && std::isfinite(vmax)) {
        pl.win_c0 = (int32_t)std::max(0.0, std::min((double)g.nu, std::floor(umin) - 1.0));
        pl.win_c1 = (int32_t)std::min((double)g.nu - 1.0, std::max(-1.0, std::ceil(umax) + 1.0));
        pl.win_r0 = (int32_t)std::max(0.0, std::min((double)g.nv, std::floor(vmin) - 1.0));
        pl.win_r1 = (int32_t)std::min((double)g.nv - 1.0, std::max(-1.0, std::ceil(vmax) + 1.0));
    } else {
        pl.win_c0 = 0;
        pl.win_c1 = g.nu - 1;
        pl.win_r0 = 0;
        pl.win_r1 = g.nv - 1;
    }
}

int check_ptr(const void *p, int32_t dt, const char *name)
{
    if (!p) return fail(PN_EINVAL, "%s is NULL", name);
    if ((uintptr_t)p % (uintptr_t)esize(dt)) return fail(PN_EINVAL, "%s is not %lld-byte aligned", name,
                                                         (long long)esize(dt));
    return PN_OK;
}

int common_checks(int64_t batch, int32_t in_dt, int32_t out_dt)
{
    if (!dtype_ok(in_dt)) return fail(PN_EDTYPE, "unknown input dtype %d", in_dt);
    if (!dtype_ok(out_dt)) return fail(PN_EDTYPE, "unknown output dtype %d", out_dt);
    if (batch < 0 || batch > 65535) return fail(PN_EINVAL, "batch = %lld out of range", (long long)batch);
    return PN_OK;
}

// Pointer checks; a buffer with no elements may be NULL (as torch passes it).
int buffer_checks(const void *in, bool in_empty, const void *out, bool out_empty, int32_t in_dt, int32_t out_dt)
{
    int rc;
    if (!in_empty && (rc = check_ptr(in, in_dt, "input"))) return rc;
    if (!out_empty && (rc = check_ptr(out, out_dt, "output"))) return rc;
    if (!in_empty && in == out) return fail(PN_EINVAL, "input and output alias");
    return PN_OK;
}

// Argument checks that need no device: dtypes, batch, then (after the
// geometry) the pointers.  Runs before anything is allocated or enqueued.
int preflight(const pn_geometry *pg, int64_t batch, const void *in, const void *out, int32_t in_dt, int32_t out_dt,
              bool sino_is_input, Geo &g)
{
    int rc = common_checks(batch, in_dt, out_dt);
    if (rc) return rc;
    if (batch == 0) return PN_OK;
    if ((rc = normalise_geometry(pg, g))) return rc;
    const bool sino_empty = g.n_views == 0;
    return sino_is_input ? buffer_checks(in, sino_empty, out, false, in_dt, out_dt)
                         : buffer_checks(in, false, out, sino_empty, in_dt, out_dt);
}

}  // namespace pn

namespace {

using namespace pn;

// ------------------------------------------------ matrix composition -----

int cone_one(const double *S, const double *C, const double *eu, const double *ev, int64_t rows, int64_t cols,
             double *P)
{
    double d00[3], M[9], Mi[9];
    for (int i = 0; i < 3; ++i) d00[i] = C[i] - 0.5 * (cols - 1) * eu[i] - 0.5 * (rows - 1) * ev[i];
    for (int i = 0; i < 3; ++i) {
        M[3 * i] = eu[i];
        M[3 * i + 1] = ev[i];
        M[3 * i + 2] = d00[i] - S[i];
    }
    if (!inv3(M, Mi)) return -1;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) P[4 * r + c] = Mi[3 * r + c];
        P[4 * r + 3] = -(Mi[3 * r] * S[0] + Mi[3 * r + 1] * S[1] + Mi[3 * r + 2] * S[2]);
    }
    return 0;
}

}  // namespace

extern "C" {

int pn_check_geometry(const pn_geometry *pg)
{
    clear_error();
    Geo g;
    return normalise_geometry(pg, g);
}

int pn_cone_matrices(int64_t n_views, const double *S, const double *C, const double *eu, const double *ev,
                     int64_t rows, int64_t cols, double *P_out)
{
    clear_error();
    if (n_views < 0 || rows < 1 || cols < 1) return fail(PN_EINVAL, "bad sizes");
    if (n_views > 0 && (!S || !C || !eu || !ev || !P_out)) return fail(PN_EINVAL, "NULL vector");
    for (int64_t k = 0; k < n_views; ++k)
        if (cone_one(S + 3 * k, C + 3 * k, eu + 3 * k, ev + 3 * k, rows, cols, P_out + 12 * k))
            return fail(PN_EGEOM, "view %lld: degenerate source/detector vectors", (long long)k);
    return PN_OK;
}

int pn_fan_matrices(int64_t n_views, const double *S, const double *C, const double *eu, int64_t cols,
                    double *P_out)
{
    clear_error();
    if (n_views < 0 || cols < 1) return fail(PN_EINVAL, "bad sizes");
    if (n_views > 0 && (!S || !C || !eu || !P_out)) return fail(PN_EINVAL, "NULL vector");
    for (int64_t k = 0; k < n_views; ++k) {
        const double *s = S + 2 * k, *c = C + 2 * k, *e = eu + 2 * k;
        double d0[2] = {c[0] - 0.5 * (cols - 1) * e[0], c[1] - 0.5 * (cols - 1) * e[1]};
        // M = [eu | d0 - S], P = M^-1 [I | -S]
        double m00 = e[0], m01 = d0[0] - s[0], m10 = e[1], m11 = d0[1] - s[1];
        double det = m00 * m11 - m01 * m10;
        double sc = std::sqrt(m00 * m00 + m10 * m10) * std::sqrt(m01 * m01 + m11 * m11);
        if (!std::isfinite(det) || std::fabs(det) <= 1e-12 * sc)
            return fail(PN_EGEOM, "view %lld: degenerate source/detector vectors", (long long)k);
        double i00 = m11 / det, i01 = -m01 / det, i10 = -m10 / det, i11 = m00 / det;
        double *P = P_out + 6 * k;
        P[0] = i00;
        P[1] = i01;
        P[2] = -(i00 * s[0] + i01 * s[1]);
        P[3] = i10;
        P[4] = i11;
        P[5] = -(i10 * s[0] + i11 * s[1]);
    }
    return PN_OK;
}

int pn_parallel2d_matrices(int64_t n_views, const double *dir, const double *C, const double *eu, int64_t cols,
                           double *P_out)
{
    clear_error();
    if (n_views < 0 || cols < 1) return fail(PN_EINVAL, "bad sizes");
    if (n_views > 0 && (!dir || !C || !eu || !P_out)) return fail(PN_EINVAL, "NULL vector");
    for (int64_t k = 0; k < n_views; ++k) {
        const double *d = dir + 2 * k, *c = C + 2 * k, *e = eu + 2 * k;
        // [eu | dir]^-1 (X - C) = (u - (cols-1)/2, t)
        double det = e[0] * d[1] - d[0] * e[1];
        double sc = std::sqrt(e[0] * e[0] + e[1] * e[1]) * std::sqrt(d[0] * d[0] + d[1] * d[1]);
        if (!std::isfinite(det) || std::fabs(det) <= 1e-12 * sc)
            return fail(PN_EGEOM, "view %lld: detector axis parallel to the rays", (long long)k);
        double r0 = d[1] / det, r1 = -d[0] / det;
        double *P = P_out + 6 * k;
        P[0] = r0;
        P[1] = r1;
        P[2] = -(r0 * c[0] + r1 * c[1]) + 0.5 * (cols - 1);
        P[3] = 0.0;
        P[4] = 0.0;
        P[5] = 1.0;
    }
    return PN_OK;
}

int pn_parallel3d_matrices(int64_t n_views, const double *dir, const double *C, const double *eu, const double *ev,
                           int64_t rows, int64_t cols, double *P_out)
{
    clear_error();
    if (n_views < 0 || rows < 1 || cols < 1) return fail(PN_EINVAL, "bad sizes");
    if (n_views > 0 && (!dir || !C || !eu || !ev || !P_out)) return fail(PN_EINVAL, "NULL vector");
    for (int64_t k = 0; k < n_views; ++k) {
        const double *d = dir + 3 * k, *c = C + 3 * k, *e = eu + 3 * k, *f = ev + 3 * k;
        double M[9] = {e[0], f[0], d[0], e[1], f[1], d[1], e[2], f[2], d[2]}, Mi[9];
        if (!inv3(M, Mi)) return fail(PN_EGEOM, "view %lld: degenerate direction/detector vectors", (long long)k);
        double *P = P_out + 12 * k;
        const double off[2] = {0.5 * (cols - 1), 0.5 * (rows - 1)};
        for (int r = 0; r < 2; ++r) {
            for (int j = 0; j < 3; ++j) P[4 * r + j] = Mi[3 * r + j];
            P[4 * r + 3] = -(Mi[3 * r] * c[0] + Mi[3 * r + 1] * c[1] + Mi[3 * r + 2] * c[2]) + off[r];
        }
        P[8] = P[9] = P[10] = 0.0;
        P[11] = 1.0;
    }
    return PN_OK;
}

const char *pn_last_error(void) { return t_err.c_str(); }

}  // extern "C"
