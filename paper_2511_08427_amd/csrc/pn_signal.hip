// gfx950 kernels of the CT projector library's sinogram-domain tools: the
// FBP/FDK row filter and the artifact simulators (Gaussian noise, ring
// artifacts, detector jitter, gantry motion blur).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>
#include <utility>

#include "pn_common.hpp"
#include "pn_device.hpp"

namespace pn {

// ------------------------------------------------------- FBP filter ------

// Row filter of the filtered back-projection: per detector row, the cosine
// weight of each pixel's ray (divergent beams: 1 / (|q3| |d|), q3 the last
// row of the view's 3x3 matrix, d the ray from the source to the pixel,
// q3 . d = 1) and the linear convolution with the discrete kernel g
// (Ram-Lak: g[0] = 1/4, g[k] = -1/(pi^2 k^2) for odd k, 0 for even k;
// Shepp-Logan: g[k] = -2 / (pi^2 (4 k^2 - 1))), times `scale`.
//
// Per detector row this is a product with a Toeplitz matrix, out = scale Xw
// G^T with Xw the cosine-weighted rows (rows x nu) and G[n][m] = g[n - m]
// (nu x nu): a dense contraction of 2 rows nu^2 flops, run on the matrix
// cores as v_mfma_f32_16x16x4_f32 (FP32 operands and accumulators).  A
// workgroup owns 64 rows and up to 512 output columns; each of its four
// waves 32 rows x 256 columns as 2 x 16 tiles of 16 x 16 (128 accumulators
// per lane: a block of inputs feeds 128 products, which hides the loads and
// the cosine weights; 128 columns per wave measured 0.93 against 0.86 ms).  MFMA operand layout (lane l, i = l % 16, c = l / 16): A[i][c],
// B[c][i]; the result D[4c + r][i] in register r.  The contraction runs over
// the row's inputs in blocks of 16: a lane loads the 4 consecutive inputs
// x[m0 + 4c .. m0 + 4c + 3] of each of its two rows, and MFMA step s
// contracts over m = m0 + 4c + s (the order of the terms of a product is
// free), so each step's A operand is one of those four values; the B operand
// g[n - m] comes from a table of g in LDS.  The loads of the next block are
// in flight while a block's products run.
// Ram-Lak: every even-distance tap but g[0] is zero.  A tile then holds 16
// output columns of one parity (n = n0 + 32 q + 2 i + p), which only the
// inputs of the other parity reach: two of the four steps, half the
// products.  g[0] x[n] enters through the two steps of the same parity in
// the two input blocks that cover the tile's columns, i.e. where m reaches
// n: the sum nearly cancels (the odd taps add up to -g[0]), and adding the
// large term there rather than last keeps the partial sums smaller (about
// half the FP32 error of adding it last, in a model of this summation order
// on projections of the phantoms).
constexpr int kFiltMaxCols = 1024;
constexpr int kFiltGOff = kFiltMaxCols + 16;  // g[k] at table entry k + kFiltGOff
constexpr int kFiltGN = 2 * kFiltGOff + 8;     // table entries

typedef float filt_f4 __attribute__((ext_vector_type(4)));

// Calls block(n0 + 16 i, i / 2) for i = 0 .. sizeof...(I) - 1, the tile
// pair as a compile-time constant.
template <typename B, int... I>
__device__ __forceinline__ void diag_blocks_at(B &block, int n0, std::integer_sequence<int, I...>)
{
    (block(n0 + 16 * I, std::integral_constant<int, I / 2>{}), ...);
}

// At least two waves per SIMD: the waves' 128 accumulators then live in
// VGPRs (no AGPR copies) instead of 332 registers at one wave per SIMD
// (Ram-Lak 0.56 against 0.67 ms on cone 256^3 x 360).
// TRIM: a wave whose 256 columns lie past the row returns at once (the full
// kernel is instantiated without it for rows whose last 512-column group has
// work for both waves: the early exit cost 2-4% there).
template <typename Q, typename O, int KIND, bool TRIM>
__global__ __launch_bounds__(256, 2) void filter_kernel(FiltParams p)
{
    constexpr int GOFF = kFiltGOff, GN = kFiltGN;
    __shared__ float gtab[GN];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int li = lane & 15, lc = lane >> 4;
    const int nu = p.nu;
    for (int e = t; e < GN; e += 256) {
        const int k = e - GOFF, ak = k < 0 ? -k : k;
        float g = 0.0f;
        if (ak < nu) {
            const double dk = static_cast<double>(ak);
            if (KIND == 0) {
                if (ak == 0) g = 0.25f;
                else if (ak & 1) g = static_cast<float>(-1.0 / (M_PI * M_PI * dk * dk));
            } else {
                g = static_cast<float>(-2.0 / (M_PI * M_PI * (4.0 * dk * dk - 1.0)));
            }
        }
        gtab[e] = g;
    }
    const int64_t rows = static_cast<int64_t>(p.batch) * p.n_views * p.nv;
    const int ncg = (nu + 511) >> 9;
    // 64 rows x 512 columns per workgroup: two waves of 256 columns per 32
    // rows (16 tiles of 16 x 16 per row block, 128 accumulators per lane)
    constexpr int NT = 16;        // tiles per row block of a wave
    constexpr int WROWS = 64;     // rows per workgroup
    const int64_t row0 = static_cast<int64_t>(blockIdx.x / ncg) * WROWS + 32 * (wave >> 1);
    const int n0 = static_cast<int>(blockIdx.x % ncg) * 512 + 256 * (wave & 1);

    // the lane's two input rows and their cosine weights w(m) = rq / |a m + b|
    const Q *src[2];
    bool have[2];
    float ca[2][3], cb[2][3], rq[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const int64_t row = row0 + 16 * rb + li;
        have[rb] = row < rows;
        const int64_t rr_ = have[rb] ? row : 0;
        src[rb] = static_cast<const Q *>(p.in) + rr_ * nu;
        for (int d = 0; d < 3; ++d) ca[rb][d] = cb[rb][d] = 0.0f;
        rq[rb] = 1.0f;
        if (!p.parallel) {
            const int r = static_cast<int>(rr_ % p.nv);
            const int view = static_cast<int>((rr_ / p.nv) % p.n_views);
            const ViewTab &tv = p.tab[view];
            const double rd = static_cast<double>(r);
            for (int d = 0; d < 3; ++d) {
                ca[rb][d] = static_cast<float>(tv.A[3 * d] * p.s[d]);
                cb[rb][d] = static_cast<float>((tv.A[3 * d + 1] * rd + tv.A[3 * d + 2]) * p.s[d]);
            }
            const double q0 = tv.Pi[8] / p.s[0], q1 = tv.Pi[9] / p.s[1], q2 = tv.Pi[10] / p.s[2];
            rq[rb] = static_cast<float>(1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2));
        }
    }
    // inputs m0 + 4 lc .. m0 + 4 lc + 3 of both rows: the loads are issued
    // one block ahead without a branch (an index past the row reads the
    // row's first input), the cosine weight and the zero past the row or the
    // last row are applied when the block is used
    auto fetch = [&](int m0, Q (&raw)[2][4]) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int m = m0 + 4 * lc + s;
                raw[rb][s] = src[rb][m < nu ? m : 0];
            }
    };
    auto finish = [&](int m0, const Q (&raw)[2][4], float (&xv)[2][4]) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int m = m0 + 4 * lc + s;
                float v = to_f32(raw[rb][s]);
                if (!p.parallel) {
                    const float fm = static_cast<float>(m);
                    const float d0 = fmaf(fm, ca[rb][0], cb[rb][0]);
                    const float d1 = fmaf(fm, ca[rb][1], cb[rb][1]);
                    const float d2 = fmaf(fm, ca[rb][2], cb[rb][2]);
                    v *= __builtin_amdgcn_rsqf(fmaf(d0, d0, fmaf(d1, d1, d2 * d2))) * rq[rb];
                }
                xv[rb][s] = (have[rb] && m < nu) ? v : 0.0f;
            }
    };

    filt_f4 acc[2][NT];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[rb][c] = filt_f4{0.0f, 0.0f, 0.0f, 0.0f};
    float xv[2][4];
    Q raw[2][4], rawc[2][4];
    if constexpr (KIND == 1) {
        // B of tile c at step s: g[n0 + 16 c + li - (m0 + 4 lc + s)]
        fetch(0, raw);
        __syncthreads();  // the table is written
        if constexpr (TRIM)
            if (n0 >= nu) return;  // no output column (wave-uniform; no barrier follows)
        for (int m0 = 0; m0 < nu; m0 += 16) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int s = 0; s < 4; ++s) rawc[rb][s] = raw[rb][s];
            if (m0 + 16 < nu) fetch(m0 + 16, raw);  // next block in flight
            finish(m0, rawc, xv);
            const float *gb = gtab + (GOFF + n0 + li - 4 * lc - m0 - 3);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const float bv = gb[16 * c + 3 - s];
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
                        acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[rb][s], bv, acc[rb][c], 0, 0, 0);
                }
        }
    } else {
        fetch(0, raw);
        __syncthreads();  // the table is written
        if (n0 >= nu) return;  // no output column (wave-uniform; no barrier follows)
        // tile c = 2 q + par holds n = n0 + 32 q + 2 li + par; B at step s is
        // g[n0 + 32 q + 2 li + par - (m0 + 4 lc + s)], odd distances for the
        // steps of the other parity; DQ >= 0 adds the two same-parity steps of
        // tiles 2 DQ, 2 DQ + 1 (distance 0 in the block).  The distance-0
        // blocks are separate code, not a branch around MFMAs inside one loop:
        // that kept the compiler copying all the accumulators every block.
        auto block_odd = [&](int m0, auto dq) {
            constexpr int DQ = decltype(dq)::value;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int s = 0; s < 4; ++s) rawc[rb][s] = raw[rb][s];
            fetch(m0 + 16, raw);  // next block in flight
            finish(m0, rawc, xv);
            const float *gb = gtab + (GOFF + n0 + 2 * li - 4 * lc - m0 - 3);
#pragma unroll
            for (int par = 0; par < 2; ++par)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int s = 2 * h + (1 - par);
#pragma unroll
                    for (int q = 0; q < NT / 2; ++q) {
                        const float bv = gb[32 * q + par + 3 - s];
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb)
                            acc[rb][2 * q + par] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(xv[rb][s], bv, acc[rb][2 * q + par], 0, 0, 0);
                    }
                }
            if constexpr (DQ >= 0) {
#pragma unroll
                for (int par = 0; par < 2; ++par)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int s = 2 * h + par;
                        const float bv = gb[32 * DQ + par + 3 - s];
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb)
                            acc[rb][2 * DQ + par] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(xv[rb][s], bv, acc[rb][2 * DQ + par], 0, 0, 0);
                    }
            }
        };
        // one ascending pass: the blocks before the wave's columns, the
        // sixteen that reach them at distance 0 (m0 = n0 + 32 q and
        // n0 + 32 q + 16 for tile pair q; past the row their inputs are zero),
        // then the rest
        const int mend = (nu + 15) & ~15;
        for (int m0 = 0; m0 < n0; m0 += 16) block_odd(m0, std::integral_constant<int, -1>{});
        diag_blocks_at(block_odd, n0, std::make_integer_sequence<int, NT>{});
        for (int m0 = n0 + 16 * NT; m0 < mend; m0 += 16) block_odd(m0, std::integral_constant<int, -1>{});
    }
    O *dst = static_cast<O *>(p.out);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int n = KIND == 1 ? n0 + 16 * c + li : n0 + 32 * (c >> 1) + 2 * li + (c & 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + 16 * rb + 4 * lc + r;
                if (row < rows && n < nu) dst[row * nu + n] = from_f32<O>(acc[rb][c][r] * p.scale);
            }
        }
}

template <typename Q, int KIND, bool TRIM>
static hipError_t filter_q(const FiltParams &p, uint32_t blocks, int32_t out_dt, hipStream_t st)
{
    switch (out_dt) {
    case DT_F32: filter_kernel<Q, float, KIND, TRIM><<<dim3(blocks), 256, 0, st>>>(p); break;
    case DT_BF16: filter_kernel<Q, bf16, KIND, TRIM><<<dim3(blocks), 256, 0, st>>>(p); break;
    default: filter_kernel<Q, f16, KIND, TRIM><<<dim3(blocks), 256, 0, st>>>(p); break;
    }
    return hipGetLastError();
}

template <int KIND, bool TRIM>
static hipError_t filter_k(const FiltParams &p, uint32_t blocks, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    switch (in_dt) {
    case DT_F32: return filter_q<float, KIND, TRIM>(p, blocks, out_dt, st);
    case DT_BF16: return filter_q<bf16, KIND, TRIM>(p, blocks, out_dt, st);
    default: return filter_q<f16, KIND, TRIM>(p, blocks, out_dt, st);
    }
}

int32_t filter_max_cols() { return kFiltMaxCols; }

hipError_t launch_filter(const FiltParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    const int64_t rows = static_cast<int64_t>(p.batch) * p.n_views * p.nv;
    if (rows == 0 || p.nu <= 0) return hipSuccess;
    if (p.nu > kFiltMaxCols) return hipErrorInvalidValue;
    // matrix cores: 32 rows x 512 columns per workgroup
    const int64_t blocks = (rows + 63) / 64 * ((p.nu + 511) / 512);
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const uint32_t nb = static_cast<uint32_t>(blocks);
    if (p.kind == 0) return filter_k<0, true>(p, nb, in_dt, out_dt, st);
    // the last column group's second wave (columns 256..511 of the group) idle?
    const bool trim = (p.nu - 1) % 512 < 256;
    return trim ? filter_k<1, true>(p, nb, in_dt, out_dt, st) : filter_k<1, false>(p, nb, in_dt, out_dt, st);
}

// ------------------------------------------------ artifact simulation -----

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 64 x 64 -> 128-bit multiplies; the key grows by the Weyl constants
// between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t h0 = __umul64hi(M0, c[0]), l0 = M0 * c[0];
        const uint64_t h1 = __umul64hi(M1, c[2]), l1 = M1 * c[2];
        const uint64_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = l1;
        c[2] = n2;
        c[3] = l0;
    }
}

// Additive Gaussian noise: one thread per four consecutive elements, which
// share the Philox block at counter (i / 4, 0, 0, 0) under key (seed, 0).
// Words (0, 1) and (2, 3) become Box-Muller pairs (uniforms
// ((w >> 11) + 1/2) 2^-53; the first of a pair takes the cosine).  The
// normal draws are formed in FP64, the sum in FP32.
template <typename T>
__global__ __launch_bounds__(256) void noise_kernel(NoiseParams p)
{
    const int64_t nb = (p.n + 3) / 4;
    T *d = static_cast<T *>(p.data);
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; b < nb;
         b += static_cast<int64_t>(gridDim.x) * 256) {
        uint64_t c[4] = {static_cast<uint64_t>(b), 0, 0, 0};
        philox4x64_10(c, p.seed, 0);
        double z[4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double ua = (static_cast<double>(c[2 * h] >> 11) + 0.5) * 0x1p-53;
            const double ub = (static_cast<double>(c[2 * h + 1] >> 11) + 0.5) * 0x1p-53;
            const double r = sqrt(-2.0 * log(ua));
            double sn, cs;
            sincospi(2.0 * ub, &sn, &cs);
            z[2 * h] = r * cs;
            z[2 * h + 1] = r * sn;
        }
        const int64_t e0 = b * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (e0 + q < p.n)
                d[e0 + q] = from_f32<T>(to_f32(d[e0 + q]) + static_cast<float>(p.mean + p.sigma * z[q]));
    }
}

// Ring artifacts: the chosen detector columns of views v0 .. v1 - 1 scaled
// by gain (FP32 product), one thread per touched element.
template <typename T>
__global__ __launch_bounds__(256) void ring_kernel(RingParams p)
{
    const int64_t nvs = p.v1 - p.v0;
    const int64_t total = p.batch * nvs * p.rows * p.n_sel;
    T *d = static_cast<T *>(p.data);
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * 256) {
        const int j = static_cast<int>(e % p.n_sel);
        int64_t t = e / p.n_sel;
        const int r = static_cast<int>(t % p.rows);
        t /= p.rows;
        const int v = p.v0 + static_cast<int>(t % nvs);
        const int64_t bb = t / nvs;
        const int64_t at = ((bb * p.n_views + v) * p.rows + r) * p.cols + p.sel[j];
        d[at] = from_f32<T>(to_f32(d[at]) * p.gain);
    }
}

constexpr int kJitterRows = 16;  // rows per wave and group

// Detector jitter: every detector row moved by its own integer shift s in
// -m .. m along the columns (zero where the source leaves the row).  s is
// word 0 of the Philox block at counter (row, 0, 0, 0) under key (seed, 1),
// reduced mod 2m + 1, drawn once per row.
template <typename T>
__global__ __launch_bounds__(256) void jitter_kernel(JitterParams p)
{
    // each wave moves groups of kJitterRows consecutive rows: lane l <
    // kJitterRows draws the shift of row g0 + l (one Philox block per row),
    // then the wave copies the group's rows one after the other, lanes along
    // the columns (coalesced), four columns per lane in flight at a time
    const T *__restrict__ src = static_cast<const T *>(p.in);
    T *__restrict__ dst = static_cast<T *>(p.out);
    const uint64_t span = static_cast<uint64_t>(2 * p.max_shift + 1);
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * 4;
    for (int64_t g0 = (static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6)) * kJitterRows; g0 < p.n_rows;
         g0 += waves * kJitterRows) {
        int mine = 0;
        if (lane < kJitterRows) {
            uint64_t w[4] = {static_cast<uint64_t>(g0 + lane), 0, 0, 0};
            philox4x64_10(w, p.seed, 1);
            mine = static_cast<int>(w[0] % span) - p.max_shift;
        }
        const int nrow = static_cast<int>(min(static_cast<int64_t>(kJitterRows), p.n_rows - g0));
        for (int j = 0; j < nrow; ++j) {
            const int sft = __builtin_amdgcn_readlane(mine, j);
            const T *in = src + (g0 + j) * p.cols;
            T *out = dst + (g0 + j) * p.cols;
            for (int c0 = 0; c0 < p.cols; c0 += 4 * 64) {
                T v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int c = c0 + lane + 64 * k, from = c - sft;
                    v[k] = (c < p.cols && from >= 0 && from < p.cols) ? in[from] : from_f32<T>(0.0f);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int c = c0 + lane + 64 * k;
                    if (c < p.cols) out[c] = v[k];
                }
            }
        }
    }
}

hipError_t launch_jitter(const JitterParams &p, int32_t dt, hipStream_t st);

// Gantry motion blur: every output pixel is the mean of `taps` bilinear
// samples at unit spacing along the view's acquisition direction
// (cos a, sin a) in (column, row) pixel units, zeros outside the detector;
// single-row detectors use (cos a, 0).
template <typename T>
__global__ __launch_bounds__(256) void blur_kernel(BlurParams p)
{
    // one wave per detector row (image, r): the view's direction is formed
    // once per row, the lanes run along the columns
    const int64_t n_rows = p.batch * p.n_views * p.rows;
    const T *src = static_cast<const T *>(p.in);
    T *dst = static_cast<T *>(p.out);
    const int h = (p.taps - 1) / 2;
    const float inv = 1.0f / static_cast<float>(p.taps);
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * 4;
    for (int64_t rowi = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); rowi < n_rows; rowi += waves) {
        const int r = static_cast<int>(rowi % p.rows);
        const int64_t img = rowi / p.rows;
        const int v = static_cast<int>(img % p.n_views);
        double sd, cd;
        sincos(p.angle_start + v * p.angle_step, &sd, &cd);
        // a single-row projection has no row direction: the kernel acts
        // through its column component
        const float du = static_cast<float>(cd), dv = p.rows > 1 ? static_cast<float>(sd) : 0.0f;
        const T *im = src + img * p.rows * p.cols;
        for (int c = lane; c < p.cols; c += 64) {
            float acc = 0.0f;
            for (int t = -h; t <= h; ++t) {
                // offsets from the pixel, split into whole and fractional
                // parts before the pixel index is added, so the fractions
                // keep full FP32 precision whatever the detector size
                const float tu = static_cast<float>(t) * du, tv = static_cast<float>(t) * dv;
                const float iu = floorf(tu), iv = floorf(tv);
                const float fx = tu - iu, fy = tv - iv;
                const int x0 = c + static_cast<int>(iu), y0 = r + static_cast<int>(iv);
                float s = 0.0f;
#pragma unroll
                for (int oy = 0; oy < 2; ++oy)
#pragma unroll
                    for (int ox = 0; ox < 2; ++ox) {
                        const int xi = x0 + ox, yi = y0 + oy;
                        const float w = (oy ? fy : 1.0f - fy) * (ox ? fx : 1.0f - fx);
                        if (xi >= 0 && xi < p.cols && yi >= 0 && yi < p.rows)
                            s = fmaf(w, to_f32(im[static_cast<int64_t>(yi) * p.cols + xi]), s);
                    }
                acc += s;
            }
            dst[(img * p.rows + r) * p.cols + c] = from_f32<T>(acc * inv);
        }
    }
}

// The same blur for detectors of >= 16 rows and up to 49 taps, as a
// stencil: the taps' offsets and bilinear weights depend on the view only,
// so a workgroup (one 64 x 16 pixel tile of one view) forms the <= 4 taps
// (integer offset, weight) entries once, stages the tile with its halo (zeros
// outside the detector) into LDS, and every output is a sum of LDS reads.
// Per view the taps reach at most h = (taps - 1) / 2 pixels (|cos|, |sin| <=
// 1) plus one for the bilinear corner, so the staged region is
// (16 + 2h + 2) x (64 + 2h + 2).  Each thread computes 4 rows of one column.
constexpr int kBlurTileC = 64, kBlurTileR = 16, kBlurTiledMaxHalf = 24;

template <typename T>
__global__ __launch_bounds__(256) void blur_tiled_kernel(BlurParams p)
{
    extern __shared__ float blur_lds[];
    const int h = (p.taps - 1) / 2;
    const int W = kBlurTileC + 2 * h + 2, H = kBlurTileR + 2 * h + 2;
    const int ne = 4 * p.taps;
    float *tile = blur_lds;
    float *s_w = tile + H * W;
    int *s_off = reinterpret_cast<int *>(s_w + ne);
    const int tiles_c = (p.cols + kBlurTileC - 1) / kBlurTileC, tiles_r = (p.rows + kBlurTileR - 1) / kBlurTileR;
    int64_t bid = blockIdx.x;
    const int tc = static_cast<int>(bid % tiles_c);
    bid /= tiles_c;
    const int tr = static_cast<int>(bid % tiles_r);
    const int64_t img = bid / tiles_r;
    const int v = static_cast<int>(img % p.n_views);
    const int c0 = tc * kBlurTileC, r0 = tr * kBlurTileR;
    const int t = threadIdx.x;
    const T *im = static_cast<const T *>(p.in) + img * p.rows * p.cols;
    if (t < ne) {
        // entry t: tap t / 4 (offset t / 4 - h along the direction), corner
        // (ox, oy) = (t & 1, t >> 1 & 1); offsets and fractions as the
        // per-pixel kernel forms them
        double sd, cd;
        sincos(p.angle_start + v * p.angle_step, &sd, &cd);
        const float du = static_cast<float>(cd), dv = static_cast<float>(sd);
        const int ox = t & 1, oy = (t >> 1) & 1;
        const float tf = static_cast<float>((t >> 2) - h);
        const float tu = tf * du, tv = tf * dv;
        const float iu = floorf(tu), iv = floorf(tv);
        const float fx = tu - iu, fy = tv - iv;
        s_w[t] = (oy ? fy : 1.0f - fy) * (ox ? fx : 1.0f - fx);
        s_off[t] = (static_cast<int>(iv) + oy + h) * W + static_cast<int>(iu) + ox + h;
    }
    for (int i = t; i < H * W; i += 256) {
        const int gr = r0 - h + i / W, gc = c0 - h + i % W;
        tile[i] = gr >= 0 && gr < p.rows && gc >= 0 && gc < p.cols
                      ? to_f32(im[static_cast<int64_t>(gr) * p.cols + gc])
                      : 0.0f;
    }
    __syncthreads();
    const int lx = t & 63, ly0 = (t >> 6) * 4;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int e = 0; e < ne; ++e) {
        const float w = s_w[e];
        const float *q = tile + ly0 * W + lx + s_off[e];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = fmaf(w, q[j * W], acc[j]);
    }
    const float inv = 1.0f / static_cast<float>(p.taps);
    T *dst = static_cast<T *>(p.out) + img * p.rows * p.cols;
    const int c = c0 + lx;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = r0 + ly0 + j;
        if (r < p.rows && c < p.cols) dst[static_cast<int64_t>(r) * p.cols + c] = from_f32<T>(acc[j] * inv);
    }
}

hipError_t launch_blur(const BlurParams &p, int32_t dt, hipStream_t st);

template <typename P, typename F32K, typename B16K, typename F16K>
static hipError_t launch_elementwise(const P &p, int64_t items, int32_t dt, F32K kf, B16K kb, F16K kh, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((items + 255) / 256, 256 * 32);
    if (blocks <= 0) return hipSuccess;
    const dim3 grid(static_cast<uint32_t>(blocks));
    switch (dt) {
    case DT_F32: kf<<<grid, 256, 0, st>>>(p); break;
    case DT_BF16: kb<<<grid, 256, 0, st>>>(p); break;
    default: kh<<<grid, 256, 0, st>>>(p); break;
    }
    return hipGetLastError();
}

hipError_t launch_noise(const NoiseParams &p, int32_t dt, hipStream_t st)
{
    return launch_elementwise(p, (p.n + 3) / 4, dt, noise_kernel<float>, noise_kernel<bf16>, noise_kernel<f16>, st);
}

hipError_t launch_jitter(const JitterParams &p, int32_t dt, hipStream_t st)
{
    // one wave per group of kJitterRows rows
    return launch_elementwise(p, (p.n_rows + kJitterRows - 1) / kJitterRows * 64, dt, jitter_kernel<float>,
                              jitter_kernel<bf16>, jitter_kernel<f16>, st);
}

hipError_t launch_blur(const BlurParams &p, int32_t dt, hipStream_t st)
{
    const int h = (p.taps - 1) / 2;
    if (p.rows >= kBlurTileR && h <= kBlurTiledMaxHalf) {
        // one workgroup per 64 x 16 pixel tile of a view
        const int64_t tiles = static_cast<int64_t>((p.cols + kBlurTileC - 1) / kBlurTileC) *
                              ((p.rows + kBlurTileR - 1) / kBlurTileR) * p.batch * p.n_views;
        if (tiles > 0x7fffffff) return hipErrorInvalidValue;
        const size_t lds = sizeof(float) * (static_cast<size_t>(kBlurTileC + 2 * h + 2) * (kBlurTileR + 2 * h + 2) +
                                            8 * static_cast<size_t>(p.taps));
        const dim3 grid(static_cast<uint32_t>(tiles));
        switch (dt) {
        case DT_F32: blur_tiled_kernel<float><<<grid, 256, lds, st>>>(p); break;
        case DT_BF16: blur_tiled_kernel<bf16><<<grid, 256, lds, st>>>(p); break;
        default: blur_tiled_kernel<f16><<<grid, 256, lds, st>>>(p); break;
        }
        return hipGetLastError();
    }
    // one wave per detector row
    return launch_elementwise(p, p.batch * p.n_views * p.rows * 64, dt, blur_kernel<float>, blur_kernel<bf16>,
                              blur_kernel<f16>, st);
}

hipError_t launch_ring(const RingParams &p, int32_t dt, hipStream_t st)
{
    const int64_t items = p.batch * (p.v1 - p.v0) * p.rows * p.n_sel;
    return launch_elementwise(p, items, dt, ring_kernel<float>, ring_kernel<bf16>, ring_kernel<f16>, st);
}

}  // namespace pn
