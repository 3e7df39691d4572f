// Per-ray Joseph set-up shared by the gfx950 forward projectors (the
// LDS-staged one in pn_kernels.hip and the sampler-interpolation one in
// pn_sampler.hip): the ray's dominant axis, in-plane slopes and offsets,
// length per plane and the conservative range of planes it can sample.
// Device code only; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pn_common.hpp"

namespace pn {

// ------------------------------------------------------ ray set-up -------

// One ray's Joseph parameters for its dominant axis `axis`: in-plane
// positions at plane m are (fma(m, gf, bf), fma(m, gs, bs)) along the "fast"
// and "slow" in-plane axes; [m0, m1] is a conservative plane range outside
// which every tap is zero; ds is the ray length (mm) per plane.
struct RaySeg {
    int axis, m0, m1;
    float gf, gs, bf, bs, ds;
};

__device__ __forceinline__ int fast_axis(int a) { return a == 0 ? 1 : 0; }
__device__ __forceinline__ int slow_axis(int a) { return a == 2 ? 1 : 2; }

// Narrows [lo, hi] to the planes m where b + m*g lies in [lo_pos, hi_pos].
// The range only has to hold every plane where the ray can sample a
// non-zero tap (the caller adds a plane of slack on each side, and planes
// outside add exactly zero), so the crossings are formed with the hardware
// FP64 reciprocal (relative error about 2^-23) instead of a division.  A zero
// slope keeps or empties the whole range by the position itself.
__device__ __forceinline__ void clip_range(double b, double g, double lo_pos, double hi_pos, double &lo, double &hi)
{
    if (g == 0.0) {
        if (!(b >= lo_pos && b <= hi_pos)) { lo = 1.0; hi = 0.0; }
        return;
    }
    const double rg = __builtin_amdgcn_rcp(g);
    const double t0 = (lo_pos - b) * rg, t1 = (hi_pos - b) * rg;
    lo = fmax(lo, fmin(t0, t1));
    hi = fmin(hi, fmax(t0, t1));
}

// point_source: every ray of the view leaves the same point (B has zero u
// and v columns), so p(u, v) is the view's constant B (0, 0, 1).
__device__ __forceinline__ void ray_setup(const ViewTab &t, double u, double v, const int32_t n[3],
                                          const double s[3], bool point_source, RaySeg &r)
{
    double d[3], p[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d[i] = fma(t.A[3 * i], u, fma(t.A[3 * i + 1], v, t.A[3 * i + 2]));
        p[i] = t.B[3 * i + 2];
    }
    if (!point_source) {  // uniform; the asm keeps it a branch
        asm volatile("");
#pragma unroll
        for (int i = 0; i < 3; ++i) p[i] = fma(t.B[3 * i], u, fma(t.B[3 * i + 1], v, t.B[3 * i + 2]));
    }
    double ax = fabs(d[0]), ay = fabs(d[1]), az = fabs(d[2]);
    // dominant index-space axis; exact ties go to the lowest axis
    int a = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    int f = fast_axis(a), sl = slow_axis(a);
    // 1/d_a: hardware reciprocal refined by two Newton steps (FP64 accurate)
    const double da = d[a];
    double inv = __builtin_amdgcn_rcp(da);
    inv = inv * fma(-da, inv, 2.0);
    inv = inv * fma(-da, inv, 2.0);
    double gf = d[f] * inv, gs = d[sl] * inv;
    double bf = fma(-p[a], gf, p[f]);
    double bs = fma(-p[a], gs, p[sl]);
    // ray length per plane (mm), FP32
    const float wx = static_cast<float>(d[0]) * static_cast<float>(s[0]);
    const float wy = static_cast<float>(d[1]) * static_cast<float>(s[1]);
    const float wz = static_cast<float>(d[2]) * static_cast<float>(s[2]);
    const float ds = __builtin_amdgcn_sqrtf(fmaf(wx, wx, fmaf(wy, wy, wz * wz))) * fabsf(static_cast<float>(inv));
    double lo = 0.0, hi = static_cast<double>(n[a] - 1);
    clip_range(bf, gf, -1.0, static_cast<double>(n[f]), lo, hi);
    clip_range(bs, gs, -1.0, static_cast<double>(n[sl]), lo, hi);
    r.axis = a;
    r.gf = static_cast<float>(gf);
    r.gs = static_cast<float>(gs);
    r.bf = static_cast<float>(bf);
    r.bs = static_cast<float>(bs);
    r.ds = ds;
    if (!(lo <= hi) || !isfinite(ds)) {
        r.m0 = 1;
        r.m1 = 0;
        return;
    }
    // one plane of slack on each side: extra planes contribute exactly zero
    r.m0 = static_cast<int>(fmax(floor(lo), 0.0));
    r.m1 = static_cast<int>(fmin(ceil(hi), static_cast<double>(n[a] - 1)));
}

}  // namespace pn
