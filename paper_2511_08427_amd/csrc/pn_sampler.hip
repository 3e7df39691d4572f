// gfx950 sampler-interpolation forward projector: the ray-driven Joseph
// projector A with every bilinear tap gathered through the vector memory
// path (L1 and L2 caches) instead of being staged through LDS.  It is this
// GPU's counterpart of interpolating with a texture sampler (paper Sec. 2.1,
// interpolation: texture sampling is the faster option but needs extra
// memory, interpolation written in the kernel is the memory-efficient one).
// gfx950 has no image instructions and so no filtering hardware; the sampler
// is written out, over one of two images of the volume:
//
//  * bordered images: the zero-bordered work copies of the LDS-staged
//    projector (one per dominant axis, planes laid out for the sampling
//    direction) play the texture's part, with its extra memory and its
//    border-zero addressing: no tap is bounds-checked;
//  * the caller's volume: no extra memory, every tap bounds-checked.
//
// The interpolation weights can be rounded to multiples of 2^-B (ties
// upward), the reduced-precision weights of fixed-function filtering, so that
// their effect on A can be measured against the exact operator.
//
// Same arithmetic contract as the LDS-staged projector: FP64 per-ray set-up
// (pn_ray.hpp), positions fma(m, slope, offset) in FP32, FP32 accumulation in
// plane order, round-to-nearest-even 16-bit stores.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pn_common.hpp"
#include "pn_device.hpp"
#include "pn_ray.hpp"

namespace pn {

// One thread per ray: a workgroup takes a tile_u x tile_v tile of detector
// pixels in view_group consecutive views (one view per tile_u x tile_v
// threads).  Rays of neighbouring views cross nearly the same voxels, so
// the waves of a workgroup, which run side by side on one CU, share their
// cache lines in L1.  Consecutive workgroup ids go round-robin to the 8
// XCDs; each XCD takes every 8th tile and runs all view groups of a tile
// back to back, so its L2 holds the slab of volume those rays cross.
template <typename S, typename O, bool BORDER, bool QUANT>
__global__ __launch_bounds__(256) void forward_sampled_kernel(SampParams p)
{
    const int t = threadIdx.x;
    const int bid = blockIdx.x;
    const int tiles = p.tiles_u * p.tiles_v;
    const int tpx = (tiles + 7) >> 3;
    const int n_vg = (p.n_views + p.view_group - 1) / p.view_group;
    const int xcd = bid & 7, slot = bid >> 3;
    const int per_b = tpx * n_vg;
    const int b = slot / per_b;
    const int rem = slot - b * per_b;
    const int tile = (rem / n_vg) * 8 + xcd;
    const int tpix = p.tile_u * p.tile_v;
    const int view = (rem % n_vg) * p.view_group + t / tpix;
    if (tile >= tiles || b >= p.batch || view >= p.n_views) return;  // padding
    const int tt = t % tpix;
    const int c = (tile % p.tiles_u) * p.tile_u + tt % p.tile_u;
    const int r = (tile / p.tiles_u) * p.tile_v + tt / p.tile_u;
    if (c >= p.nu || r >= p.nv) return;

    RaySeg rs;
    rs.axis = 0;
    ray_setup(p.tab[view], static_cast<double>(c), static_cast<double>(r), p.n, p.s, p.point_source != 0, rs);
    const int a = rs.axis;
    float acc = 0.0f;
    const bool live = rs.m0 <= rs.m1 && p.img[a] != nullptr;
    if (live) {
        const int f = fast_axis(a), sl = slow_axis(a);
        const S *img = static_cast<const S *>(p.img[a]) + b * p.item[a] + p.org[a];
        // every offset within one batch item fits 32 bits (host check)
        const int32_t pl = static_cast<int32_t>(p.plane[a]), rw = static_cast<int32_t>(p.row[a]);
        const int32_t cl = BORDER ? 1 : static_cast<int32_t>(p.col[a]);
        const int32_t inf = p.n[f], ins = p.n[sl];
        const float nf = static_cast<float>(inf), ns = static_cast<float>(ins);
        const float sc = QUANT ? static_cast<float>(1 << p.weight_bits) : 1.0f;
        const float isc = QUANT ? 1.0f / sc : 1.0f;  // exact: a power of two
        // weight of the upper tap: the fraction of pos, rounded to the
        // nearest multiple of 2^-B (ties upward) when quantised.  Every step
        // is exact in FP32 (scaling by a power of two, floor, and ts - q with
        // q <= ts < q + 1), so the rounding decision is that of the FP32
        // position itself.
        auto weight = [&](float pos, float &fl) {
            fl = floorf(pos);
            float w = pos - fl;  // exact
            if constexpr (QUANT) {
                const float ts = w * sc;
                const float q = floorf(ts);
                w = (ts - q >= 0.5f ? q + 1.0f : q) * isc;
            }
            return w;
        };
        auto sample = [&](int m) {
            const float fm = static_cast<float>(m);
            // a position outside [-1, n] has both taps outside the grid;
            // clamped to -1 or n it samples exactly 0
            const float pf = fminf(fmaxf(fmaf(fm, rs.gf, rs.bf), -1.0f), nf);
            const float ps = fminf(fmaxf(fmaf(fm, rs.gs, rs.bs), -1.0f), ns);
            float ff, fs;
            const float wf = weight(pf, ff), ws = weight(ps, fs);
            const int32_t i = static_cast<int32_t>(ff), j = static_cast<int32_t>(fs);
            const int32_t o = m * pl + j * rw + i * cl;
            float v00, v01, v10, v11;
            if constexpr (BORDER) {
                v00 = to_f32(img[o]);
                v01 = to_f32(img[o + 1]);
                v10 = to_f32(img[o + rw]);
                v11 = to_f32(img[o + rw + 1]);
            } else {
                const bool f0 = static_cast<uint32_t>(i) < static_cast<uint32_t>(inf);
                const bool f1 = static_cast<uint32_t>(i + 1) < static_cast<uint32_t>(inf);
                const bool s0 = static_cast<uint32_t>(j) < static_cast<uint32_t>(ins);
                const bool s1 = static_cast<uint32_t>(j + 1) < static_cast<uint32_t>(ins);
                v00 = f0 && s0 ? to_f32(img[o]) : 0.0f;
                v01 = f1 && s0 ? to_f32(img[o + cl]) : 0.0f;
                v10 = f0 && s1 ? to_f32(img[o + rw]) : 0.0f;
                v11 = f1 && s1 ? to_f32(img[o + rw + cl]) : 0.0f;
            }
            const float lo = fmaf(wf, v01 - v00, v00);
            const float hi = fmaf(wf, v11 - v10, v10);
            return fmaf(ws, hi - lo, lo);
        };
        // four planes' taps in flight at once, summed in plane order
        int m = rs.m0;
        for (; m + 3 <= rs.m1; m += 4) {
            const float s0 = sample(m), s1 = sample(m + 1), s2 = sample(m + 2), s3 = sample(m + 3);
            acc += s0;
            acc += s1;
            acc += s2;
            acc += s3;
        }
        for (; m <= rs.m1; ++m) acc += sample(m);
    }
    O *out = static_cast<O *>(p.sino);
    out[((static_cast<int64_t>(b) * p.n_views + view) * p.nv + r) * p.nu + c] = from_f32<O>(live ? acc * rs.ds : 0.0f);
}

int64_t forward_sampled_blocks(const SampParams &p)
{
    const int64_t tiles = static_cast<int64_t>(p.tiles_u) * p.tiles_v;
    const int64_t n_vg = (p.n_views + p.view_group - 1) / p.view_group;
    return 8 * ((tiles + 7) / 8) * n_vg * static_cast<int64_t>(p.batch);
}

// Workgroup shape of the sampler: 64 x 1 pixels in 4 consecutive views (a
// wave is one row of 64 pixels of one view); 256 x 1 pixels of one view for
// 2-D problems.
void forward_sampled_tile(bool two_d, int32_t &tu, int32_t &tv, int32_t &views)
{
    tu = two_d ? 256 : 64;
    tv = 1;
    views = two_d ? 1 : 4;
}

template <typename S, typename O, bool BORDER>
static hipError_t fs_q(const SampParams &p, uint32_t blocks, hipStream_t st)
{
    if (p.weight_bits > 0) forward_sampled_kernel<S, O, BORDER, true><<<dim3(blocks), 256, 0, st>>>(p);
    else forward_sampled_kernel<S, O, BORDER, false><<<dim3(blocks), 256, 0, st>>>(p);
    return hipGetLastError();
}

template <typename S, typename O>
static hipError_t fs_b(const SampParams &p, uint32_t blocks, hipStream_t st)
{
    return p.bordered ? fs_q<S, O, true>(p, blocks, st) : fs_q<S, O, false>(p, blocks, st);
}

template <typename S>
static hipError_t fs_o(const SampParams &p, uint32_t blocks, int32_t out_dt, hipStream_t st)
{
    switch (out_dt) {
    case DT_F32: return fs_b<S, float>(p, blocks, st);
    case DT_BF16: return fs_b<S, bf16>(p, blocks, st);
    default: return fs_b<S, f16>(p, blocks, st);
    }
}

hipError_t launch_forward_sampled(const SampParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    const uint32_t blocks = static_cast<uint32_t>(forward_sampled_blocks(p));
    if (blocks == 0) return hipSuccess;
    switch (in_dt) {
    case DT_F32: return fs_o<float>(p, blocks, out_dt, st);
    case DT_BF16: return fs_o<bf16>(p, blocks, out_dt, st);
    default: return fs_o<f16>(p, blocks, out_dt, st);
    }
}

}  // namespace pn
