// Host side of the CT projector library: argument and geometry validation,
// FP64 per-view tables, the plan cache, work buffers, and the extern "C"
// entry points declared in include/pyronn_mi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pyronn_mi.h"
#include "pn_common.hpp"

namespace pn {
hipError_t launch_relayout(int32_t dtype, const void *in, void *out, const int32_t n[3], int axis, int32_t batch,
                           int64_t item, int32_t row, int64_t plane, hipStream_t st);
hipError_t launch_forward(const FwdParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st);
hipError_t launch_adjoint(const AdjParams &p, int32_t in_dt, int shape, hipStream_t st);
hipError_t launch_backproject(const BpParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st);
hipError_t launch_maxabs(int32_t in_dt, const void *src, int64_t n, uint32_t *out, hipStream_t st);
hipError_t launch_cbox(const AdjParams &ap, const uint32_t *axbox, int32_t L, int32_t TS, int32_t TF, uint32_t *out,
                       hipStream_t st);
hipError_t launch_fill_zero(void *dst, int64_t bytes, hipStream_t st);
hipError_t launch_filter(const FiltParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st);
int32_t filter_max_cols();
hipError_t launch_noise(const NoiseParams &p, int32_t dt, hipStream_t st);
hipError_t launch_ring(const RingParams &p, int32_t dt, hipStream_t st);
hipError_t launch_jitter(const JitterParams &p, int32_t dt, hipStream_t st);
hipError_t launch_blur(const BlurParams &p, int32_t dt, hipStream_t st);
hipError_t launch_convert(const float *src, void *dst, int32_t out_dt, int64_t n, hipStream_t st);
int adjoint_shape_count();
void adjoint_shape(int id, int32_t &L, int32_t &TS, int32_t &TF);
void forward_tile_shape(bool two_d, int32_t &tu, int32_t &tv, int32_t &views);
int64_t forward_blocks(const FwdParams &p);
int64_t adjoint_blocks(const AdjParams &p);
int64_t backproject_blocks(const BpParams &p);
hipError_t launch_forward_batch(const Batch<FwdParams> &w, bool two_d, int32_t in_dt, int32_t out_dt, hipStream_t st);
hipError_t launch_adjoint_batch(const Batch<AdjParams> &w, int axis, int32_t in_dt, int shape, hipStream_t st);
hipError_t launch_backproject_batch(const Batch<BpParams> &w, bool two_d, int32_t in_dt, int32_t out_dt,
                                    hipStream_t st);
}  // namespace pn

namespace {

using namespace pn;

// ---------------------------------------------------------------- errors --

thread_local std::string t_err;

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

int fail_hip(hipError_t e, const char *what)
{
    return fail(PN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t esize(int32_t dt) { return dt == PN_F32 ? 4 : 2; }

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}
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

// Normalised geometry: 2-D problems embedded as 3-D with nz = 1, every
// matrix 3x4, sign chosen so that W > 0 over the volume.
struct Geo {
    int32_t ndim = 3, beam = PN_CONE;
    bool parallel = false;
    int32_t n[3] = {0, 0, 0};  // nx, ny, nz
    double s[3] = {1, 1, 1};   // sx, sy, sz
    double o[3] = {0, 0, 0};   // ox, oy, oz
    int32_t nv = 0, nu = 0;
    int32_t n_views = 0;
    std::vector<double> P;     // n_views x 12 (world matrices)
    std::vector<double> raw;   // caller's matrices, for exact cache matching
    double raw_scalars[16] = {};

    bool same(const Geo &g) const
    {
        return ndim == g.ndim && beam == g.beam && nv == g.nv && nu == g.nu && n_views == g.n_views &&
               std::memcmp(n, g.n, sizeof n) == 0 && std::memcmp(raw_scalars, g.raw_scalars, sizeof raw_scalars) == 0 &&
               raw == g.raw;
    }
};

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

// ------------------------------------------------------------- plans ------

struct Plan {
    Geo g;
    int device = 0;
    std::vector<ViewTab> tab;
    std::vector<ViewTabF> tabf;
    int32_t axes_union = 0;
    std::vector<int32_t> pass_views[3];
    ViewTab *d_tab = nullptr;
    ViewTabF *d_tabf = nullptr;
    int32_t *d_views[3] = {nullptr, nullptr, nullptr};
    // forward work copies, one allocation per dominant axis
    void *d_lay[3] = {nullptr, nullptr, nullptr};
    size_t lay_cap[3] = {0, 0, 0};
    int32_t lay_dtype[3] = {-1, -1, -1};
    int64_t lay_item[3] = {0, 0, 0}, lay_plane[3] = {0, 0, 0};
    int32_t lay_row[3] = {0, 0, 0};
    // FP32 accumulation buffer of the adjoint for 16-bit outputs
    float *d_acc = nullptr;
    size_t acc_cap = 0;
    // max |sinogram| of the current adjoint call (fixed-point scale)
    uint32_t *d_maxabs = nullptr;
    // largest per-view bound on the rays that sample one voxel's neighbourhood
    float kmax = 1.0f;
    // 3-D adjoint block shape chosen by the autotuner (0: not tuned)
    int adj_shape = 0;
    // adjoint candidate pixel boxes per pass axis, for block shape cbox_shape
    uint32_t *d_cbox[3] = {nullptr, nullptr, nullptr};
    int cbox_shape[3] = {-1, -1, -1};
    // detector window that holds every ray meeting the dilated volume in
    // some view (inclusive pixel bounds; c0 > c1: no ray meets it)
    int32_t win_c0 = 0, win_c1 = -1, win_r0 = 0, win_r1 = -1;
    // the same per view (c0, c1, r0, r1), host and device
    std::vector<int32_t> vwin;
    int32_t *d_vwin = nullptr;
    // per view and axis: detector box of the pixels whose ray may have that
    // dominant axis (axis_mask)
    std::vector<uint32_t> axbox;
    uint32_t *d_axbox = nullptr;

    ~Plan()
    {
        dev_free(d_tab);
        dev_free(d_tabf);
        for (int a = 0; a < 3; ++a) {
            dev_free(d_views[a]);
            dev_free(d_lay[a]);
        }
        dev_free(d_acc);
        dev_free(d_maxabs);
        for (int a = 0; a < 3; ++a) dev_free(d_cbox[a]);
        dev_free(d_vwin);
        dev_free(d_axbox);
    }
};

std::mutex g_mu;
std::list<std::unique_ptr<Plan>> g_plans;  // most recently used first
const size_t kMaxPlans = 32;

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

void build_tables(Plan &pl)
{
    const Geo &g = pl.g;
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

template <typename T>
int upload(T **dst, const std::vector<T> &src)
{
    if (src.empty()) return PN_OK;
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * src.size());
    if (e != hipSuccess) return fail(PN_ENOMEM, "hipMalloc(%zu): %s", sizeof(T) * src.size(), hipGetErrorString(e));
    e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
    return PN_OK;
}

// Looks up or builds the plan of a geometry.  Caller holds g_mu.
int get_plan(const pn_geometry *pg, Plan **out)
{
    Geo g;
    int rc = normalise_geometry(pg, g);
    if (rc) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
        if ((*it)->device == dev && (*it)->g.same(g)) {
            if (it != g_plans.begin()) g_plans.splice(g_plans.begin(), g_plans, it);
            *out = g_plans.front().get();
            return PN_OK;
        }
    }
    auto pl = std::make_unique<Plan>();
    pl->g = std::move(g);
    pl->device = dev;
    build_tables(*pl);
    if ((rc = upload(&pl->d_tab, pl->tab))) return rc;
    if ((rc = upload(&pl->d_tabf, pl->tabf))) return rc;
    for (int a = 0; a < 3; ++a)
        if ((rc = upload(&pl->d_views[a], pl->pass_views[a]))) return rc;
    if ((rc = upload(&pl->d_maxabs, std::vector<uint32_t>(1, 0u)))) return rc;
    if ((rc = upload(&pl->d_vwin, pl->vwin))) return rc;
    if ((rc = upload(&pl->d_axbox, pl->axbox))) return rc;
    g_plans.push_front(std::move(pl));
    while (g_plans.size() > kMaxPlans) g_plans.pop_back();
    *out = g_plans.front().get();
    return PN_OK;
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

int ensure_work_copy(Plan &pl, int a, int32_t dt, int64_t batch, hipStream_t st)
{
    const Geo &g = pl.g;
    const int f = a == 0 ? 1 : 0, sl = a == 2 ? 1 : 2;
    const int32_t row = work_row(g.n[f]);
    const int64_t plane = (int64_t)row * (g.n[sl] + PADR_LO + PADR_HI);
    const int64_t item = plane * g.n[a];
    const size_t need = (size_t)(item * batch * esize(dt));
    bool zero = pl.lay_dtype[a] != dt;
    if (need > pl.lay_cap[a]) {
        dev_free(pl.d_lay[a]);
        pl.d_lay[a] = nullptr;
        pl.lay_cap[a] = 0;
        hipError_t e = hipMalloc(&pl.d_lay[a], need);
        if (e != hipSuccess) {
            pl.d_lay[a] = nullptr;
            return fail(PN_ENOMEM, "work copy hipMalloc(%zu): %s", need, hipGetErrorString(e));
        }
        pl.lay_cap[a] = need;
        zero = true;
    }
    if (zero) {
        // padding must read as zero; the interior is rewritten on every call
        hipError_t e = launch_fill_zero(pl.d_lay[a], (int64_t)pl.lay_cap[a], st);
        if (e != hipSuccess) return fail_hip(e, "fill");
        pl.lay_dtype[a] = dt;
    }
    pl.lay_item[a] = item;
    pl.lay_plane[a] = plane;
    pl.lay_row[a] = row;
    return PN_OK;
}

// 3-D adjoint block shape: PN_ADJ_SHAPE=<id> selects one of the compiled
// shapes (1..count-1) for tuning; the default is shape 1 (16 x 16 x 16).
int adjoint_shape_3d()
{
    static int shape = [] {
        const char *e = std::getenv("PN_ADJ_SHAPE");
        int v = e ? std::atoi(e) : 1;
        return (v >= 1 && v < adjoint_shape_count()) ? v : 1;
    }();
    return shape;
}

// ------------------------------------------------------------ autotuner --
//
// With PN_AUTOTUNE=1 the first 3-D adjoint of a plan (outside graph
// capture) times every compiled block shape on the caller's stream and keeps
// the fastest for the plan.  PN_TUNE_CACHE=<file> keeps the choices across
// processes, one line per geometry: "nz ny nx rows cols views beam shape".
// Different shapes round the fixed-point sums at different points, so with
// tuning on, the last bits of the adjoint can differ between processes
// whose choices differ; without it the shape is fixed (PN_ADJ_SHAPE or 16^3).

bool autotune_on()
{
    static const bool on = [] {
        const char *e = std::getenv("PN_AUTOTUNE");
        return e && std::atoi(e) != 0;
    }();
    return on;
}

std::string tune_key(const Geo &g)
{
    char buf[160];
    std::snprintf(buf, sizeof buf, "%d %d %d %d %d %d %d", g.n[2], g.n[1], g.n[0], g.nv, g.nu, g.n_views,
                  g.parallel ? 0 : 1);
    return buf;
}

int tune_cache_lookup(const Geo &g)
{
    const char *path = std::getenv("PN_TUNE_CACHE");
    if (!path) return 0;
    FILE *f = std::fopen(path, "r");
    if (!f) return 0;
    const std::string key = tune_key(g);
    char line[256];
    int found = 0;
    while (std::fgets(line, sizeof line, f)) {
        const std::string l(line);
        if (l.compare(0, key.size(), key) == 0 && l.size() > key.size() && l[key.size()] == ' ') {
            const int v = std::atoi(l.c_str() + key.size() + 1);
            if (v >= 1 && v < adjoint_shape_count()) found = v;
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(const Geo &g, int shape)
{
    const char *path = std::getenv("PN_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", tune_key(g).c_str(), shape);
    std::fclose(f);
}

// The 3-D adjoint block shape of a plan: tuned, cached, or the fixed one.
int plan_adjoint_shape(Plan *pl)
{
    if (pl->adj_shape == 0 && autotune_on()) pl->adj_shape = tune_cache_lookup(pl->g);
    return pl->adj_shape ? pl->adj_shape : adjoint_shape_3d();
}

// ---------------------------------------------------- prepared problems --
//
// Every call is validated and prepared problem by problem (plan, work
// copies, pre-passes, kernel parameters); the main kernels of a single call
// are then launched directly, and those of a batched call in work lists of
// up to kMaxBatch problems per launch.  A prepared problem owns its plan's
// work buffers until its launch, so a work list never holds two problems of
// one plan.  Callers hold g_mu.

struct FwdJob {
    FwdParams p;
    bool two_d;
    Plan *plan;
};

int forward_prepare(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dt,
                    int32_t out_dt, hipStream_t st, Plan *pl, FwdJob &job, bool &none)
{
    const Geo &g = pl->g;
    none = g.n_views == 0;
    if (none) return PN_OK;
    FwdParams p{};
    p.tab = pl->d_tab;
    p.n_views = g.n_views;
    p.nu = g.nu;
    p.nv = g.nv;
    p.batch = (int32_t)batch;
    int rc;
    for (int a = 0; a < 3; ++a) {
        p.n[a] = g.n[a];
        p.s[a] = g.s[a];
        p.lay[a] = nullptr;
        if (pl->axes_union >> a & 1) {
            if ((rc = ensure_work_copy(*pl, a, in_dt, batch, st))) return rc;
            hipError_t e = launch_relayout(in_dt, vol, pl->d_lay[a], g.n, a, (int32_t)batch, pl->lay_item[a],
                                           pl->lay_row[a], pl->lay_plane[a], st);
            if (e != hipSuccess) return fail_hip(e, "relayout launch");
            p.lay[a] = pl->d_lay[a];
            p.lay_item[a] = pl->lay_item[a];
            p.lay_plane[a] = pl->lay_plane[a];
            p.lay_row[a] = pl->lay_row[a];
        }
    }
    p.vol = vol;
    p.sino = sino;
    forward_tile_shape(g.ndim == 2, p.tile_u, p.tile_v, p.view_group);
    // only the tiles of the detector window that can see the volume are
    // launched; the rest of the sinogram is zero
    const bool full = pl->win_c0 == 0 && pl->win_r0 == 0 && pl->win_c1 == g.nu - 1 && pl->win_r1 == g.nv - 1;
    if (!full) {
        hipError_t e = launch_fill_zero(sino, (int64_t)g.n_views * g.nv * g.nu * batch * esize(out_dt), st);
        if (e != hipSuccess) return fail_hip(e, "fill");
    }
    const bool empty = pl->win_c0 > pl->win_c1 || pl->win_r0 > pl->win_r1;
    p.c_lo = empty ? 0 : pl->win_c0;
    p.r_lo = empty ? 0 : pl->win_r0;
    p.tiles_u = empty ? 0 : (pl->win_c1 - pl->win_c0 + p.tile_u) / p.tile_u;
    p.tiles_v = empty ? 0 : (pl->win_r1 - pl->win_r0 + p.tile_v) / p.tile_v;
    p.vwin = pl->d_vwin;
    p.point_source = g.parallel ? 0 : 1;
    if (forward_blocks(p) > INT32_MAX) return fail(PN_EINVAL, "problem too large for one launch");
    none = forward_blocks(p) == 0;
    (void)pg;
    job.p = p;
    job.two_d = g.ndim == 2;
    job.plan = pl;
    return PN_OK;
}

struct AdjJob {
    AdjParams pass[3];  // per dominant axis; pass[a].n_pass_views == 0: none
    bool two_d;
    int shape;
    Plan *plan;
    float *acc;         // FP32 accumulation target
    void *out;          // caller's output, converted from acc when not FP32
    int32_t out_dt;
    int64_t total;
};

int adjoint_prepare(int64_t batch, const void *sino, void *vol, int32_t in_dt, int32_t out_dt, hipStream_t st,
                    Plan *pl, AdjJob &job, bool &none, int force_shape = 0)
{
    const Geo &g = pl->g;
    const int64_t item = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t total = item * batch;
    int npass = 0;
    for (int a = 0; a < 3; ++a) npass += pl->pass_views[a].empty() ? 0 : 1;
    none = npass == 0;
    if (none) {
        hipError_t e = launch_fill_zero(vol, total * esize(out_dt), st);
        return e == hipSuccess ? PN_OK : fail_hip(e, "fill");
    }
    float *target = nullptr;
    if (out_dt == PN_F32) {
        target = static_cast<float *>(vol);
    } else {
        const size_t need = (size_t)total * 4;
        if (need > pl->acc_cap) {
            dev_free(pl->d_acc);
            pl->d_acc = nullptr;
            pl->acc_cap = 0;
            hipError_t e = hipMalloc((void **)&pl->d_acc, need);
            if (e != hipSuccess) {
                pl->d_acc = nullptr;
                return fail(PN_ENOMEM, "adjoint accumulator hipMalloc(%zu): %s", need, hipGetErrorString(e));
            }
            pl->acc_cap = need;
        }
        target = pl->d_acc;
    }
    const bool two_d = g.ndim == 2;
    const int shape = two_d ? 0 : (force_shape ? force_shape : plan_adjoint_shape(pl));
    int32_t L, TS, TF;
    adjoint_shape(shape, L, TS, TF);
    {
        hipError_t e = launch_maxabs(in_dt, sino, (int64_t)g.n_views * g.nv * g.nu * batch, pl->d_maxabs, st);
        if (e != hipSuccess) return fail_hip(e, "maxabs launch");
    }
    // |s (.) delta| / |delta_a| <= |s| because delta_a is the largest component
    const float ds_bound = (float)(std::sqrt(g.s[0] * g.s[0] + g.s[1] * g.s[1] + g.s[2] * g.s[2]) * 1.0001);
    int done = 0;
    for (int a = 0; a < 3; ++a) {
        AdjParams &p = job.pass[a];
        p = AdjParams{};
        if (pl->pass_views[a].empty()) continue;
        const int f = a == 0 ? 1 : 0, sl = a == 2 ? 1 : 2;
        p.tab = pl->d_tab;
        p.tabf = pl->d_tabf;
        p.maxabs = pl->d_maxabs;
        p.ds_bound = ds_bound;
        // a flush period holds >= 256 units of max|q ds| (and one view's
        // worth at least); the rounding error of a contribution is
        // <= kunits max|q ds| / 2^30
        p.kunits = std::max(256.0f, pl->kmax);
        p.point_source = g.parallel ? 0 : 1;
        p.views = pl->d_views[a];
        p.n_pass_views = (int32_t)pl->pass_views[a].size();
        p.axis = a;
        p.nu = g.nu;
        p.nv = g.nv;
        p.n_views = g.n_views;
        p.batch = (int32_t)batch;
        for (int i = 0; i < 3; ++i) {
            p.n[i] = g.n[i];
            p.s[i] = g.s[i];
        }
        p.sino = sino;
        p.out = target;
        p.accumulate = done > 0;
        p.blocks_a = (g.n[a] + L - 1) / L;
        p.blocks_s = (g.n[sl] + TS - 1) / TS;
        p.blocks_f = (g.n[f] + TF - 1) / TF;
        if (adjoint_blocks(p) > INT32_MAX) return fail(PN_EINVAL, "problem too large for one launch");
        // candidate boxes depend on the geometry and the block shape only:
        // built once per plan and shape (a kernel on the caller's stream)
        if (pl->cbox_shape[a] != shape) {
            dev_free(pl->d_cbox[a]);
            pl->d_cbox[a] = nullptr;
            pl->cbox_shape[a] = -1;
            const size_t need = (size_t)p.blocks_a * p.blocks_s * p.blocks_f * p.n_pass_views * 8;
            hipError_t e = hipMalloc((void **)&pl->d_cbox[a], need);
            if (e != hipSuccess) {
                pl->d_cbox[a] = nullptr;
                return fail(PN_ENOMEM, "candidate box hipMalloc(%zu): %s", need, hipGetErrorString(e));
            }
            if ((e = launch_cbox(p, pl->d_axbox, L, TS, TF, pl->d_cbox[a], st)) != hipSuccess) return fail_hip(e, "cbox launch");
            pl->cbox_shape[a] = shape;
        }
        p.cbox = pl->d_cbox[a];
        ++done;
    }
    job.two_d = two_d;
    job.shape = shape;
    job.plan = pl;
    job.acc = target;
    job.out = vol;
    job.out_dt = out_dt;
    job.total = total;
    return PN_OK;
}

int adjoint_finish(const AdjJob &job, hipStream_t st)
{
    if (job.out_dt == PN_F32) return PN_OK;
    hipError_t e = launch_convert(job.acc, job.out, job.out_dt, job.total, st);
    return e == hipSuccess ? PN_OK : fail_hip(e, "convert launch");
}

struct BpJob {
    BpParams p;
    bool two_d;
    Plan *plan;
};

void backproject_prepare(int64_t batch, const void *sino, void *vol, Plan *pl, BpJob &job)
{
    const Geo &g = pl->g;
    BpParams p{};
    p.tabf = pl->d_tabf;
    p.n_views = g.n_views;
    p.nu = g.nu;
    p.nv = g.nv;
    p.batch = (int32_t)batch;
    for (int a = 0; a < 3; ++a) p.n[a] = g.n[a];
    p.sino = sino;
    p.vol = vol;
    job.p = p;
    job.two_d = g.n[2] == 1;
    job.plan = pl;
}

// ------------------------------------------------------------ single calls

int forward_impl(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dt, int32_t out_dt,
                 hipStream_t st)
{
    Geo pre;
    int rc = preflight(pg, batch, vol, sino, in_dt, out_dt, false, pre);
    if (rc || batch == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, &pl))) return rc;
    FwdJob job;
    bool none;
    if ((rc = forward_prepare(pg, batch, vol, sino, in_dt, out_dt, st, pl, job, none)) || none) return rc;
    hipError_t e = launch_forward(job.p, in_dt, out_dt, st);
    if (e != hipSuccess) return fail_hip(e, "forward launch");
    return PN_OK;
}

int adjoint_impl(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dt, int32_t out_dt,
                 hipStream_t st)
{
    Geo pre;
    int rc = preflight(pg, batch, sino, vol, in_dt, out_dt, true, pre);
    if (rc || batch == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, &pl))) return rc;
    AdjJob job;
    bool none;
    auto run = [&](int force) -> int {
        int r = adjoint_prepare(batch, sino, vol, in_dt, out_dt, st, pl, job, none, force);
        if (r || none) return r;
        for (int a = 0; a < 3; ++a) {
            if (job.pass[a].n_pass_views == 0) continue;
            hipError_t e = launch_adjoint(job.pass[a], in_dt, job.shape, st);
            if (e != hipSuccess) return fail_hip(e, "adjoint launch");
        }
        return PN_OK;
    };
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (autotune_on() && pl->g.ndim == 3 && plan_adjoint_shape(pl) && pl->adj_shape == 0 &&
        hipStreamIsCapturing(st, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) {
        // time every shape (each run overwrites the output), keep the fastest
        const int ns = adjoint_shape_count();
        std::vector<hipEvent_t> ev(2 * ns, nullptr);
        int best = 0;
        float best_ms = 0.0f;
        for (int k = 1; k < ns && rc == PN_OK; ++k) {
            if (hipEventCreate(&ev[2 * k]) != hipSuccess || hipEventCreate(&ev[2 * k + 1]) != hipSuccess) {
                rc = fail(PN_EHIP, "autotune: hipEventCreate failed");
                break;
            }
            if (hipEventRecord(ev[2 * k], st) != hipSuccess) {
                rc = fail(PN_EHIP, "autotune: hipEventRecord failed");
                break;
            }
            if ((rc = run(k))) break;
            if (hipEventRecord(ev[2 * k + 1], st) != hipSuccess) {
                rc = fail(PN_EHIP, "autotune: hipEventRecord failed");
                break;
            }
        }
        for (int k = 1; k < ns && rc == PN_OK; ++k) {
            float ms = 0.0f;
            if (hipEventSynchronize(ev[2 * k + 1]) != hipSuccess ||
                hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) != hipSuccess) {
                rc = fail(PN_EHIP, "autotune: event timing failed");
                break;
            }
            if (best == 0 || ms < best_ms) {
                best = k;
                best_ms = ms;
            }
        }
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (rc) return rc;
        pl->adj_shape = best;
        tune_cache_store(pl->g, best);
    }
    if ((rc = run(0)) || none) return rc;
    return adjoint_finish(job, st);
}

int backproject_impl(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dt,
                     int32_t out_dt, hipStream_t st)
{
    Geo pre;
    int rc = preflight(pg, batch, sino, vol, in_dt, out_dt, true, pre);
    if (rc || batch == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, &pl))) return rc;
    BpJob job;
    backproject_prepare(batch, sino, vol, pl, job);
    hipError_t e = launch_backproject(job.p, in_dt, out_dt, st);
    if (e != hipSuccess) return fail_hip(e, "backproject launch");
    return PN_OK;
}

int filter_impl(const pn_geometry *pg, int64_t batch, const void *sino, void *out, int32_t in_dt, int32_t out_dt,
                int32_t kind, hipStream_t st)
{
    if (kind != PN_FILTER_RAM_LAK && kind != PN_FILTER_SHEPP_LOGAN)
        return fail(PN_EINVAL, "filter kind %d is neither PN_FILTER_RAM_LAK nor PN_FILTER_SHEPP_LOGAN", kind);
    Geo pre;
    int rc = preflight(pg, batch, sino, out, in_dt, out_dt, true, pre);
    if (rc || batch == 0) return rc;
    if (pre.n_views == 0) return PN_OK;
    if (!out) return fail(PN_EINVAL, "output pointer is NULL");
    if (pre.nu > filter_max_cols())
        return fail(PN_EINVAL, "detector rows of %d columns: the filter handles at most %d", pre.nu, filter_max_cols());
    const double du = pg->det_spacing[1];
    if (!(du > 0.0) || !std::isfinite(du)) return fail(PN_EINVAL, "det_spacing[1] must be positive (got %g)", du);
    double pitch = du;  // pixel pitch at the rotation axis
    if (!pre.parallel) {
        if (!(pg->sid > 0.0 && pg->sdd > 0.0) || !std::isfinite(pg->sid) || !std::isfinite(pg->sdd))
            return fail(PN_EINVAL, "divergent beams need sid > 0 and sdd > 0 for the filter (got %g, %g)", pg->sid,
                        pg->sdd);
        pitch = du * pg->sid / pg->sdd;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, &pl))) return rc;
    const Geo &g = pl->g;
    FiltParams p{};
    p.tab = pl->d_tab;
    p.n_views = g.n_views;
    p.nu = g.nu;
    p.nv = g.nv;
    p.batch = (int32_t)batch;
    for (int i = 0; i < 3; ++i) p.s[i] = g.s[i];
    p.parallel = g.parallel ? 1 : 0;
    p.kind = kind == PN_FILTER_RAM_LAK ? 0 : 1;
    p.scale = (float)(M_PI / g.n_views / pitch);
    p.in = sino;
    p.out = out;
    hipError_t e = launch_filter(p, in_dt, out_dt, st);
    if (e != hipSuccess) return fail_hip(e, "filter launch");
    return PN_OK;
}

// ---------------------------------------------------- artifact simulation

int noise_impl(int64_t n, void *data, int32_t dt, double mean, double sigma, uint64_t seed, hipStream_t st)
{
    int rc;
    if (!dtype_ok(dt)) return fail(PN_EDTYPE, "unknown dtype %d", dt);
    if (n < 0) return fail(PN_EINVAL, "element count %lld is negative", (long long)n);
    if (!std::isfinite(mean) || !std::isfinite(sigma) || sigma < 0.0)
        return fail(PN_EINVAL, "mean must be finite and sigma finite and >= 0 (got %g, %g)", mean, sigma);
    if (n == 0) return PN_OK;
    if ((rc = check_ptr(data, dt, "data"))) return rc;
    NoiseParams p{};
    p.data = data;
    p.n = n;
    p.mean = mean;
    p.sigma = sigma;
    p.seed = seed;
    hipError_t e = launch_noise(p, dt, st);
    if (e != hipSuccess) return fail_hip(e, "noise launch");
    return PN_OK;
}

int ring_impl(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, void *sino, int32_t dt,
              const int32_t *columns, int32_t n_columns, double gain, int32_t v0, int32_t v1, hipStream_t st)
{
    int rc = common_checks(batch, dt, dt);
    if (rc) return rc;
    if (n_views < 0 || rows <= 0 || cols <= 0)
        return fail(PN_EINVAL, "sinogram shape views=%d rows=%d cols=%d", n_views, rows, cols);
    if (v0 < 0 || v1 < v0 || v1 > n_views)
        return fail(PN_EINVAL, "view range [%d, %d) outside [0, %d)", v0, v1, n_views);
    if (n_columns < 0 || n_columns > kRingMaxCols)
        return fail(PN_EINVAL, "%d columns: between 0 and %d may be chosen", n_columns, kRingMaxCols);
    if (n_columns > 0 && !columns) return fail(PN_EINVAL, "column list is NULL");
    if (!std::isfinite(gain)) return fail(PN_EINVAL, "gain must be finite (got %g)", gain);
    std::vector<int32_t> sel(columns, columns + n_columns);
    for (int32_t c : sel)
        if (c < 0 || c >= cols) return fail(PN_EINVAL, "column %d outside [0, %d)", c, cols);
    std::sort(sel.begin(), sel.end());
    sel.erase(std::unique(sel.begin(), sel.end()), sel.end());
    if (batch == 0 || v1 == v0 || sel.empty()) return PN_OK;
    if ((rc = check_ptr(sino, dt, "sinogram"))) return rc;
    RingParams p{};
    p.data = sino;
    p.batch = batch;
    p.n_views = n_views;
    p.rows = rows;
    p.cols = cols;
    p.v0 = v0;
    p.v1 = v1;
    p.n_sel = static_cast<int32_t>(sel.size());
    p.gain = static_cast<float>(gain);
    std::copy(sel.begin(), sel.end(), p.sel);
    hipError_t e = launch_ring(p, dt, st);
    if (e != hipSuccess) return fail_hip(e, "ring launch");
    return PN_OK;
}

int jitter_impl(int64_t n_rows, int32_t cols, const void *in, void *out, int32_t dt, int32_t max_shift,
                uint64_t seed, hipStream_t st)
{
    int rc;
    if (!dtype_ok(dt)) return fail(PN_EDTYPE, "unknown dtype %d", dt);
    if (n_rows < 0 || cols <= 0) return fail(PN_EINVAL, "shape rows=%lld cols=%d", (long long)n_rows, cols);
    if (max_shift < 0 || max_shift > 1 << 20) return fail(PN_EINVAL, "max_shift %d outside 0 .. 2^20", max_shift);
    if (n_rows > INT64_MAX / cols) return fail(PN_EINVAL, "rows x cols overflows");
    if (n_rows == 0) return PN_OK;
    if ((rc = check_ptr(in, dt, "input")) || (rc = check_ptr(out, dt, "output"))) return rc;
    const size_t bytes = (size_t)(n_rows * cols) * esize(dt);
    const char *a = static_cast<const char *>(in), *b = static_cast<const char *>(out);
    if (a < b + bytes && b < a + bytes) return fail(PN_EINVAL, "input and output overlap");
    JitterParams p{};
    p.in = in;
    p.out = out;
    p.n_rows = n_rows;
    p.cols = cols;
    p.max_shift = max_shift;
    p.seed = seed;
    hipError_t e = launch_jitter(p, dt, st);
    if (e != hipSuccess) return fail_hip(e, "jitter launch");
    return PN_OK;
}

int blur_impl(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, const void *in, void *out, int32_t dt,
              double angle_start, double angle_step, int32_t taps, hipStream_t st)
{
    int rc = common_checks(batch, dt, dt);
    if (rc) return rc;
    if (n_views < 0 || rows <= 0 || cols <= 0)
        return fail(PN_EINVAL, "sinogram shape views=%d rows=%d cols=%d", n_views, rows, cols);
    if (taps < 1 || taps > 255 || taps % 2 == 0) return fail(PN_EINVAL, "taps = %d: odd, 1 .. 255", taps);
    if (!std::isfinite(angle_start) || !std::isfinite(angle_step))
        return fail(PN_EINVAL, "angles must be finite (got %g, %g)", angle_start, angle_step);
    if (batch == 0 || n_views == 0) return PN_OK;
    if ((rc = check_ptr(in, dt, "input")) || (rc = check_ptr(out, dt, "output"))) return rc;
    const size_t bytes = (size_t)(batch * n_views) * rows * cols * esize(dt);
    const char *a = static_cast<const char *>(in), *b = static_cast<const char *>(out);
    if (a < b + bytes && b < a + bytes) return fail(PN_EINVAL, "input and output overlap");
    BlurParams p{};
    p.in = in;
    p.out = out;
    p.batch = batch;
    p.n_views = n_views;
    p.rows = rows;
    p.cols = cols;
    p.taps = taps;
    p.angle_start = angle_start;
    p.angle_step = angle_step;
    hipError_t e = launch_blur(p, dt, st);
    if (e != hipSuccess) return fail_hip(e, "gantry blur launch");
    return PN_OK;
}

// ---------------------------------------------------------- batched calls

// Validates every problem (nothing is launched on a failure) and orders
// them by estimated cost, largest first (rays x planes), so the long
// problems start first in each launch.
int batch_order(const pn_problem *probs, int32_t n, int32_t in_dt, int32_t out_dt, bool sino_is_input,
                std::vector<int32_t> &order)
{
    if (n < 0) return fail(PN_EINVAL, "negative problem count");
    if (n > 0 && !probs) return fail(PN_EINVAL, "problem array is NULL");
    std::vector<double> cost(n);
    for (int32_t i = 0; i < n; ++i) {
        Geo g;
        int rc = preflight(&probs[i].geom, 1, probs[i].in, probs[i].out, in_dt, out_dt, sino_is_input, g);
        if (rc) {
            std::string msg = t_err;
            return fail(rc, "problem %d: %s", i, msg.c_str());
        }
        cost[i] = (double)g.n_views * g.nu * g.nv * std::max(g.n[0], std::max(g.n[1], g.n[2]));
    }
    order.resize(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    return PN_OK;
}

// Builds the work list of the jobs in `idx` with `blocks(job)` workgroups
// each, starting every problem at a multiple of `align`.
template <typename P, typename Job, typename BlocksFn, typename ParamFn>
int make_batch(const std::vector<Job> &jobs, const std::vector<int> &idx, BlocksFn blocks, ParamFn param,
               int64_t align, Batch<P> &w)
{
    w.n = (int32_t)idx.size();
    int64_t at = 0;
    for (int32_t i = 0; i < w.n; ++i) {
        w.p[i] = param(jobs[idx[i]]);
        w.start[i] = (uint32_t)at;
        at += (blocks(w.p[i]) + align - 1) / align * align;
        if (at > INT32_MAX) return fail(PN_EINVAL, "batched launch too large");
    }
    w.start[w.n] = (uint32_t)at;
    return PN_OK;
}

// The problems of a batched call in work lists: `prepare(i, plan)` readies
// problem i, and `launch(pending)` runs a list of prepared problems, at
// most kMaxBatch and no plan twice.
template <typename Prepare, typename Launch>
int run_batched(const pn_problem *probs, const std::vector<int32_t> &order, Prepare prepare, Launch launch)
{
    std::vector<int32_t> pending;
    std::vector<Plan *> plans;
    for (int32_t i : order) {
        Plan *pl;
        int rc = get_plan(&probs[i].geom, &pl);
        if (rc) {
            std::string msg = t_err;
            return fail(rc, "problem %d: %s", i, msg.c_str());
        }
        const bool seen = std::find(plans.begin(), plans.end(), pl) != plans.end();
        if (seen || (int)pending.size() == kMaxBatch) {
            if ((rc = launch(pending))) return rc;
            pending.clear();
            plans.clear();
        }
        if ((rc = prepare(i, pl))) {
            std::string msg = t_err;
            return fail(rc, "problem %d: %s", i, msg.c_str());
        }
        pending.push_back(i);
        plans.push_back(pl);
    }
    return pending.empty() ? PN_OK : launch(pending);
}

int forward_batched(const pn_problem *probs, int32_t n, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    std::vector<int32_t> order;
    int rc = batch_order(probs, n, in_dt, out_dt, false, order);
    if (rc || n == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<FwdJob> jobs(n);
    std::vector<char> live(n, 0);
    auto prepare = [&](int32_t i, Plan *pl) -> int {
        bool none;
        int r = forward_prepare(&probs[i].geom, 1, probs[i].in, probs[i].out, in_dt, out_dt, st, pl, jobs[i], none);
        live[i] = !none;
        return r;
    };
    auto launch = [&](const std::vector<int32_t> &pending) -> int {
        for (int two_d = 0; two_d < 2; ++two_d) {
            std::vector<int> idx;
            for (int32_t i : pending)
                if (live[i] && jobs[i].two_d == (two_d != 0)) idx.push_back(i);
            if (idx.empty()) continue;
            Batch<FwdParams> w;
            // problems start at multiples of 8 workgroups: the kernel's
            // XCD-aware tile order stays intact
            int r = make_batch<FwdParams>(jobs, idx, [](const FwdParams &p) { return forward_blocks(p); },
                                          [](const FwdJob &j) { return j.p; }, 8, w);
            if (r) return r;
            hipError_t e = launch_forward_batch(w, two_d != 0, in_dt, out_dt, st);
            if (e != hipSuccess) return fail_hip(e, "batched forward launch");
        }
        return (int)PN_OK;
    };
    return run_batched(probs, order, prepare, launch);
}

int adjoint_batched(const pn_problem *probs, int32_t n, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    std::vector<int32_t> order;
    int rc = batch_order(probs, n, in_dt, out_dt, true, order);
    if (rc || n == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<AdjJob> jobs(n);
    std::vector<char> live(n, 0);
    auto prepare = [&](int32_t i, Plan *pl) -> int {
        bool none;
        int r = adjoint_prepare(1, probs[i].in, probs[i].out, in_dt, out_dt, st, pl, jobs[i], none);
        live[i] = !none;
        return r;
    };
    auto launch = [&](const std::vector<int32_t> &pending) -> int {
        // passes in axis order: a problem's later passes add to its earlier ones
        for (int a = 0; a < 3; ++a) {
            for (int shape = 0; shape < adjoint_shape_count(); ++shape) {  // 2-D problems use shape 0
                std::vector<int> idx;
                for (int32_t i : pending)
                    if (live[i] && jobs[i].shape == shape && jobs[i].pass[a].n_pass_views > 0) idx.push_back(i);
                if (idx.empty()) continue;
                Batch<AdjParams> w;
                int r = make_batch<AdjParams>(jobs, idx, [](const AdjParams &p) { return adjoint_blocks(p); },
                                              [a](const AdjJob &j) { return j.pass[a]; }, 1, w);
                if (r) return r;
                hipError_t e = launch_adjoint_batch(w, a, in_dt, shape, st);
                if (e != hipSuccess) return fail_hip(e, "batched adjoint launch");
            }
        }
        for (int32_t i : pending) {
            if (!live[i]) continue;
            int r = adjoint_finish(jobs[i], st);
            if (r) return r;
        }
        return (int)PN_OK;
    };
    return run_batched(probs, order, prepare, launch);
}

int backproject_batched(const pn_problem *probs, int32_t n, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    std::vector<int32_t> order;
    int rc = batch_order(probs, n, in_dt, out_dt, true, order);
    if (rc || n == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<BpJob> jobs(n);
    auto prepare = [&](int32_t i, Plan *pl) -> int {
        backproject_prepare(1, probs[i].in, probs[i].out, pl, jobs[i]);
        return PN_OK;
    };
    auto launch = [&](const std::vector<int32_t> &pending) -> int {
        for (int two_d = 0; two_d < 2; ++two_d) {
            std::vector<int> idx;
            for (int32_t i : pending)
                if (jobs[i].two_d == (two_d != 0)) idx.push_back(i);
            if (idx.empty()) continue;
            Batch<BpParams> w;
            int r = make_batch<BpParams>(jobs, idx, [](const BpParams &p) { return backproject_blocks(p); },
                                         [](const BpJob &j) { return j.p; }, 1, w);
            if (r) return r;
            hipError_t e = launch_backproject_batch(w, two_d != 0, in_dt, out_dt, st);
            if (e != hipSuccess) return fail_hip(e, "batched backproject launch");
        }
        return (int)PN_OK;
    };
    return run_batched(probs, order, prepare, launch);
}

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

// ==================================================== extern "C" ABI =====

extern "C" {

int pn_forward(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dtype,
               int32_t out_dtype, void *hip_stream)
{
    t_err.clear();
    return forward_impl(pg, batch, vol, sino, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_adjoint(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dtype,
               int32_t out_dtype, void *hip_stream)
{
    t_err.clear();
    return adjoint_impl(pg, batch, sino, vol, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_backproject(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dtype,
                   int32_t out_dtype, void *hip_stream)
{
    t_err.clear();
    return backproject_impl(pg, batch, sino, vol, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_filter(const pn_geometry *pg, int64_t batch, const void *sino, void *out, int32_t in_dtype,
              int32_t out_dtype, int32_t kind, void *hip_stream)
{
    t_err.clear();
    return filter_impl(pg, batch, sino, out, in_dtype, out_dtype, kind, static_cast<hipStream_t>(hip_stream));
}

int pn_gaussian_noise(int64_t n, void *data, int32_t dtype, double mean, double sigma, uint64_t seed,
                      void *hip_stream)
{
    t_err.clear();
    return noise_impl(n, data, dtype, mean, sigma, seed, static_cast<hipStream_t>(hip_stream));
}

int pn_gantry_blur(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, const void *in, void *out,
                   int32_t dtype, double angle_start, double angle_step, int32_t taps, void *hip_stream)
{
    t_err.clear();
    return blur_impl(batch, n_views, rows, cols, in, out, dtype, angle_start, angle_step, taps,
                     static_cast<hipStream_t>(hip_stream));
}

int pn_detector_jitter(int64_t n_rows, int32_t cols, const void *in, void *out, int32_t dtype, int32_t max_shift,
                       uint64_t seed, void *hip_stream)
{
    t_err.clear();
    return jitter_impl(n_rows, cols, in, out, dtype, max_shift, seed, static_cast<hipStream_t>(hip_stream));
}

int pn_ring_artifacts(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, void *sino, int32_t dtype,
                      const int32_t *columns, int32_t n_columns, double gain, int32_t v0, int32_t v1,
                      void *hip_stream)
{
    t_err.clear();
    return ring_impl(batch, n_views, rows, cols, sino, dtype, columns, n_columns, gain, v0, v1,
                     static_cast<hipStream_t>(hip_stream));
}

int pn_forward_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype, void *hip_stream)
{
    t_err.clear();
    return forward_batched(probs, n, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_adjoint_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype, void *hip_stream)
{
    t_err.clear();
    return adjoint_batched(probs, n, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_backproject_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype,
                           void *hip_stream)
{
    t_err.clear();
    return backproject_batched(probs, n, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_check_geometry(const pn_geometry *pg)
{
    t_err.clear();
    Geo g;
    return normalise_geometry(pg, g);
}

int pn_cone_matrices(int64_t n_views, const double *S, const double *C, const double *eu, const double *ev,
                     int64_t rows, int64_t cols, double *P_out)
{
    t_err.clear();
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
    t_err.clear();
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
    t_err.clear();
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
    t_err.clear();
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

int pn_release_caches(void)
{
    t_err.clear();
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans.clear();
    return PN_OK;
}

const char *pn_version(void) { return "pyronn_mi 0.1.0 (gfx950)"; }

}  // extern "C"
