// gfx950 sampler-interpolation projectors: the ray-driven Joseph projector
// A and the voxel-driven back-projection with every bilinear tap gathered
// through the vector memory path (L1 and L2 caches) instead of being staged
// through LDS.  It is this
// GPU's counterpart of interpolating with a texture sampler (paper Sec. 2.1,
// interpolation: texture sampling is the faster option but needs extra
// memory, interpolation written in the kernel is the memory-efficient one).
// gfx950 has no image instructions and so no filtering hardware; the sampler
// is written out, over one of two images of the volume (of the sinogram,
// for the back-projection):
//
//  * bordered images: the zero-bordered work copies of the LDS-staged
//    projector (one per dominant axis, planes laid out for the sampling
//    direction), or a zero-bordered copy of the sinogram, play the
//    texture's part, with its extra memory and its border-zero addressing:
//    no tap is bounds-checked;
//  * the caller's volume or sinogram: no extra memory, every tap
//    bounds-checked.
//
// The interpolation weights can be rounded to multiples of 2^-B (ties
// upward), the reduced-precision weights of fixed-function filtering, so that
// their effect can be measured against the exact operators.
//
// Same arithmetic contracts as the LDS-staged kernels: for A, FP64 per-ray
// set-up (pn_ray.hpp), positions fma(m, slope, offset) in FP32, FP32
// accumulation in plane order; for the back-projection, FP32 projections
// from the view's FP32 matrix; round-to-nearest-even 16-bit stores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "pn_common.hpp"
#include "pn_device.hpp"
#include "pn_ray.hpp"

namespace pn {

// Weight of the upper tap of a position: its fraction, rounded to the
// nearest multiple of 2^-B (ties upward) when QUANT (sc = 2^B, isc = 2^-B).
// Every step is exact in FP32 (scaling by a power of two, floor, and ts - q
// with q <= ts < q + 1), so the rounding decision is that of the FP32
// position itself.  fl: the lower tap (floor of the position).
template <bool QUANT>
__device__ __forceinline__ float tap_weight(float pos, float sc, float isc, float &fl)
{
    fl = floorf(pos);
    float w = pos - fl;  // exact
    if constexpr (QUANT) {
        const float ts = w * sc;
        const float q = floorf(ts);
        w = (ts - q >= 0.5f ? q + 1.0f : q) * isc;
    }
    return w;
}

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
        auto weight = [&](float pos, float &fl) { return tap_weight<QUANT>(pos, sc, isc, fl); };
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

// The voxel-driven (W0/W)^2-weighted back-projection with sampler
// interpolation: one thread per column of kBpSampZ voxels along z, a
// workgroup per 16 x 16 x kBpSampZ block, all views in turn; every bilinear
// detector tap is a load through the caches (the LDS-staged back-projection
// stages each view's detector rectangle instead).  Positions as that
// kernel's gathers form them: U, V, W from the view's FP32 matrix, fma in
// z, the reciprocal of W, u and v clamped to [-1, n] (outside it both taps
// are off the detector).
constexpr int kBpSampZ = 8;

template <typename Q, typename O, bool BORDER, bool QUANT>
__global__ __launch_bounds__(256) void backproject_sampled_kernel(BpSampParams p)
{
    const int t = threadIdx.x;
    const int nbx = (p.n[0] + 15) / 16, nby = (p.n[1] + 15) / 16, nbz = (p.n[2] + kBpSampZ - 1) / kBpSampZ;
    int blk = blockIdx.x;
    const int bx = blk % nbx;
    blk /= nbx;
    const int by = blk % nby;
    blk /= nby;
    const int bz = blk % nbz;
    const int b = blk / nbz;
    if (b >= p.batch) return;
    const int i = bx * 16 + (t & 15), j = by * 16 + (t >> 4), k0 = bz * kBpSampZ;
    if (i >= p.n[0] || j >= p.n[1]) return;
    const Q *img = static_cast<const Q *>(p.img) + b * p.item + p.org;
    const float fi = static_cast<float>(i), fj = static_cast<float>(j), fk0 = static_cast<float>(k0);
    const float fnu = static_cast<float>(p.nu), fnv = static_cast<float>(p.nv);
    const float sc = QUANT ? static_cast<float>(1 << p.weight_bits) : 1.0f;
    const float isc = QUANT ? 1.0f / sc : 1.0f;
    const int32_t row = p.row;
    float acc[kBpSampZ];
#pragma unroll
    for (int z = 0; z < kBpSampZ; ++z) acc[z] = 0.0f;
    for (int view = 0; view < p.n_views; ++view) {
        const ViewTabF &tf = p.tabf[view];
        const Q *im = img + view * p.view;
        const float U0 = fmaf(tf.Pi[0], fi, fmaf(tf.Pi[1], fj, fmaf(tf.Pi[2], fk0, tf.Pi[3])));
        const float V0 = fmaf(tf.Pi[4], fi, fmaf(tf.Pi[5], fj, fmaf(tf.Pi[6], fk0, tf.Pi[7])));
        const float Wb = fmaf(tf.Pi[8], fi, fmaf(tf.Pi[9], fj, fmaf(tf.Pi[10], fk0, tf.Pi[11])));
#pragma unroll
        for (int z = 0; z < kBpSampZ; ++z) {
            const float fz = static_cast<float>(z);
            const float rw = __builtin_amdgcn_rcpf(fmaf(fz, tf.Pi[10], Wb));
            const float u = fminf(fmaxf(fmaf(fz, tf.Pi[2], U0) * rw, -1.0f), fnu);
            const float v = fminf(fmaxf(fmaf(fz, tf.Pi[6], V0) * rw, -1.0f), fnv);
            float fu, fv;
            const float wu = tap_weight<QUANT>(u, sc, isc, fu), wv = tap_weight<QUANT>(v, sc, isc, fv);
            const int32_t iu = static_cast<int32_t>(fu), iv = static_cast<int32_t>(fv);
            const int32_t o = iv * row + iu;
            float d00, d01, d10, d11;
            if constexpr (BORDER) {
                d00 = to_f32(im[o]);
                d01 = to_f32(im[o + 1]);
                d10 = to_f32(im[o + row]);
                d11 = to_f32(im[o + row + 1]);
            } else {
                const bool c0 = static_cast<uint32_t>(iu) < static_cast<uint32_t>(p.nu);
                const bool c1 = static_cast<uint32_t>(iu + 1) < static_cast<uint32_t>(p.nu);
                const bool r0 = static_cast<uint32_t>(iv) < static_cast<uint32_t>(p.nv);
                const bool r1 = static_cast<uint32_t>(iv + 1) < static_cast<uint32_t>(p.nv);
                d00 = c0 && r0 ? to_f32(im[o]) : 0.0f;
                d01 = c1 && r0 ? to_f32(im[o + 1]) : 0.0f;
                d10 = c0 && r1 ? to_f32(im[o + row]) : 0.0f;
                d11 = c1 && r1 ? to_f32(im[o + row + 1]) : 0.0f;
            }
            const float lo = fmaf(wu, d01 - d00, d00);
            const float hi = fmaf(wu, d11 - d10, d10);
            const float w = tf.W0 * rw;
            acc[z] = fmaf(w * w, fmaf(wv, hi - lo, lo), acc[z]);
        }
    }
    O *out = static_cast<O *>(p.vol) + b * static_cast<int64_t>(p.n[0]) * p.n[1] * p.n[2];
#pragma unroll
    for (int z = 0; z < kBpSampZ; ++z)
        if (k0 + z < p.n[2])
            out[(static_cast<int64_t>(k0 + z) * p.n[1] + j) * p.n[0] + i] = from_f32<O>(acc[z]);
}

// Zero-bordered copy of a sinogram: detector row r of image g (batch item
// times views) to row r + 1, column 1 on, of a view of `view` elements with
// rows of `row` elements (the border was cleared when the buffer was made).
template <typename Q>
__global__ __launch_bounds__(256) void pad_sino_kernel(const Q *__restrict__ in, Q *__restrict__ out, int64_t n_img,
                                                       int32_t nv, int32_t nu, int32_t row, int64_t view)
{
    for (int64_t rr = blockIdx.x; rr < n_img * nv; rr += gridDim.x) {
        const int64_t g = rr / nv;
        const int32_t r = static_cast<int32_t>(rr - g * nv);
        const Q *src = in + rr * nu;
        Q *dst = out + g * view + static_cast<int64_t>(r + 1) * row + 1;
        for (int32_t c = threadIdx.x; c < nu; c += 256) dst[c] = src[c];
    }
}

int64_t backproject_sampled_blocks(const BpSampParams &p)
{
    const int64_t nb = static_cast<int64_t>((p.n[0] + 15) / 16) * ((p.n[1] + 15) / 16) *
                       ((p.n[2] + kBpSampZ - 1) / kBpSampZ);
    return nb * p.batch;
}

hipError_t launch_pad_sino(int32_t dt, const void *in, void *out, int64_t n_img, int32_t nv, int32_t nu, int32_t row,
                           int64_t view, hipStream_t st)
{
    const int64_t rows = n_img * nv;
    if (rows <= 0) return hipSuccess;
    const dim3 grid(static_cast<uint32_t>(std::min<int64_t>(rows, 1 << 20)));
    switch (dt) {
    case DT_F32:
        pad_sino_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float *>(in), static_cast<float *>(out), n_img,
                                                     nv, nu, row, view);
        break;
    case DT_BF16:
        pad_sino_kernel<bf16><<<grid, 256, 0, st>>>(static_cast<const bf16 *>(in), static_cast<bf16 *>(out), n_img,
                                                    nv, nu, row, view);
        break;
    default:
        pad_sino_kernel<f16><<<grid, 256, 0, st>>>(static_cast<const f16 *>(in), static_cast<f16 *>(out), n_img, nv,
                                                   nu, row, view);
        break;
    }
    return hipGetLastError();
}

template <typename Q, typename O, bool BORDER>
static hipError_t bps_q(const BpSampParams &p, uint32_t blocks, hipStream_t st)
{
    if (p.weight_bits > 0) backproject_sampled_kernel<Q, O, BORDER, true><<<dim3(blocks), 256, 0, st>>>(p);
    else backproject_sampled_kernel<Q, O, BORDER, false><<<dim3(blocks), 256, 0, st>>>(p);
    return hipGetLastError();
}

template <typename Q, typename O>
static hipError_t bps_b(const BpSampParams &p, uint32_t blocks, hipStream_t st)
{
    return p.bordered ? bps_q<Q, O, true>(p, blocks, st) : bps_q<Q, O, false>(p, blocks, st);
}

template <typename Q>
static hipError_t bps_o(const BpSampParams &p, uint32_t blocks, int32_t out_dt, hipStream_t st)
{
    switch (out_dt) {
    case DT_F32: return bps_b<Q, float>(p, blocks, st);
    case DT_BF16: return bps_b<Q, bf16>(p, blocks, st);
    default: return bps_b<Q, f16>(p, blocks, st);
    }
}

hipError_t launch_backproject_sampled(const BpSampParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    const uint32_t blocks = static_cast<uint32_t>(backproject_sampled_blocks(p));
    if (blocks == 0) return hipSuccess;
    switch (in_dt) {
    case DT_F32: return bps_o<float>(p, blocks, out_dt, st);
    case DT_BF16: return bps_o<bf16>(p, blocks, out_dt, st);
    default: return bps_o<f16>(p, blocks, out_dt, st);
    }
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
