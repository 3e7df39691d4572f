// gfx950 kernels of the CT projector library: work-copy relayout, the
// ray-driven Joseph forward projector A, its exact adjoint A^T, the
// voxel-driven distance-weighted back-projection and its transpose (the
// splat projector), and the allocation-free adjoint's scratch array.  The
// FBP filter and the artifact simulators are in pn_signal.hip, the per-ray
// set-up in pn_ray.hpp.
//
// Arithmetic contract: per-ray set-up (direction, dominant axis, slopes,
// entry parameters, plane range) in FP64; the per-plane loop in FP32 with
// positions formed as fma(m, slope, offset) from the plane index m (never
// incrementally); FP32 accumulation; round-to-nearest-even on 16-bit stores.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "pn_common.hpp"
#include "pn_device.hpp"
#include "pn_ray.hpp"

namespace pn {

// Problem of a workgroup in a batched launch: the last i with start[i] <= bid
// (start[0] = 0, increasing).
template <typename P>
__device__ __forceinline__ int batch_item(const Batch<P> &w, int bid)
{
    int lo = 0, hi = w.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (static_cast<int>(w.start[mid]) <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The problem of workgroup `bid` in a device-memory work list (the search
// reads wave-uniform addresses: scalar loads).
template <typename P>
__device__ __forceinline__ int table_item(const Table<P> &w, int bid)
{
    int lo = 0, hi = w.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (static_cast<int>(w.start[mid]) <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------- relayout --------

// a = x: out[b][i][k + PADR_LO][j + PADC] = in[b][k][j][i] (tiled transpose)
template <typename S>
__global__ __launch_bounds__(256) void relayout_x_kernel(const S *__restrict__ in, S *__restrict__ out, int32_t nx,
                                                        int32_t ny, int32_t nz, int64_t out_item, int32_t out_row,
                                                        int64_t out_plane)
{
    __shared__ S tile[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int k = blockIdx.z % nz, b = blockIdx.z / nz;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const S *src = in + (static_cast<int64_t>(b) * nz + k) * ny * static_cast<int64_t>(nx);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int j = j0 + ty + 8 * q, i = i0 + tx;
        if (j < ny && i < nx) tile[ty + 8 * q][tx] = src[static_cast<int64_t>(j) * nx + i];
    }
    __syncthreads();
    S *dst = out + b * out_item + static_cast<int64_t>(k + PADR_LO) * out_row + PADC;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int i = i0 + ty + 8 * q, j = j0 + tx;
        if (j < ny && i < nx) dst[static_cast<int64_t>(i) * out_plane + j] = tile[tx][ty + 8 * q];
    }
}

// a = y: out[b][j][k + PADR_LO][i + PADC] = in[b][k][j][i]
// a = z: out[b][k][j + PADR_LO][i + PADC] = in[b][k][j][i]
template <typename S>
__global__ __launch_bounds__(256) void relayout_rows_kernel(const S *__restrict__ in, S *__restrict__ out,
                                                           int32_t nx, int32_t ny, int32_t nz, int32_t axis,
                                                           int64_t out_item, int32_t out_row, int64_t out_plane)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z % nz, b = blockIdx.z / nz;
    if (i >= nx) return;
    S v = in[((static_cast<int64_t>(b) * nz + k) * ny + j) * nx + i];
    int64_t o = axis == 1 ? static_cast<int64_t>(j) * out_plane + static_cast<int64_t>(k + PADR_LO) * out_row
                          : static_cast<int64_t>(k) * out_plane + static_cast<int64_t>(j + PADR_LO) * out_row;
    out[b * out_item + o + PADC + i] = v;
}

// ------------------------------------------------------- forward A -------

// 16-byte vector of storage elements, widened to FP32.
// A staged vector holds 4 storage elements: 16 bytes (a uint4) for FP32,
// 8 bytes (a uint2) for the 16-bit types.
template <typename S>
struct Stage {
    using T = uint2;
};
template <>
struct Stage<float> {
    using T = uint4;
};

// Widens one staged vector to 4 FP32 values.
__device__ __forceinline__ void unpack4(const uint4 v, float *o, float)
{
    o[0] = __uint_as_float(v.x);
    o[1] = __uint_as_float(v.y);
    o[2] = __uint_as_float(v.z);
    o[3] = __uint_as_float(v.w);
}
__device__ __forceinline__ void unpack4(const uint2 v, float *o, bf16)
{
    const uint32_t w[2] = {v.x, v.y};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        o[2 * i] = __uint_as_float(w[i] << 16);
        o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}
__device__ __forceinline__ void unpack4(const uint2 v, float *o, f16)
{
    const uint32_t w[2] = {v.x, v.y};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        o[2 * i] = static_cast<float>(__builtin_bit_cast(f16, static_cast<uint16_t>(w[i] & 0xffffu)));
        o[2 * i + 1] = static_cast<float>(__builtin_bit_cast(f16, static_cast<uint16_t>(w[i] >> 16)));
    }
}

template <typename S>
__device__ __forceinline__ float sample_padded(const S *__restrict__ plane, int32_t row, float pf, float ps,
                                               float nf, float ns)
{
    pf = fminf(fmaxf(pf, -1.0f), nf);
    ps = fminf(fmaxf(ps, -1.0f), ns);
    float ff = floorf(pf), fs = floorf(ps);
    float wf = pf - ff, ws = ps - fs;
    const S *q = plane + static_cast<int64_t>(static_cast<int>(fs) + PADR_LO) * row + (static_cast<int>(ff) + PADC);
    float v00 = to_f32(q[0]), v01 = to_f32(q[1]);
    float v10 = to_f32(q[row]), v11 = to_f32(q[row + 1]);
    float lo = fmaf(wf, v01 - v00, v00);
    float hi = fmaf(wf, v11 - v10, v10);
    return fmaf(ws, hi - lo, lo);
}

// Staged box of one chunk of planes: columns [f_al, f_al + nvec*VE) and rows
// [s_lo, s_lo + ns) of planes [mc, me] of the work copy.
struct Box {
    int mc, me, f_al, s_lo, nvec, ns;
    bool lds;
};

// Ray-driven forward projection.  A workgroup owns a TU x TV tile of
// detector pixels and NVW consecutive views (one pixel per thread, its ray
// in each of the views).  For each dominant axis present among the rays it
// walks the union of their plane ranges in chunks of C planes; per chunk it
// stages the box of volume that the rays can touch (bounded by the four
// corner rays of each view, whose crossings with a plane enclose those of
// every ray of the tile in between) from the padded work copy into LDS with
// 16-byte loads, and every ray then samples the chunk's planes from LDS.
// Rays of neighbouring views cross nearly the same voxels, so one staged box
// serves NVW views.  The loads of chunk i+1 are issued before chunk i is
// sampled (straight into the other LDS buffer for FP32 storage, into
// registers for 16-bit storage), and the boxes of up to 64 chunks are
// computed at once, one chunk per thread.  A box larger than RCAP x FCAP
// falls back to gathers from the work copy.
//
// A ray samples every plane of a chunk, also planes outside its own range:
// there its position lies outside [-1, n] in some in-plane axis and the
// box's zero padding makes the sample exactly 0.
//
// Workgroup order: consecutive workgroup ids go round-robin to the 8 XCDs;
// each XCD gets every 8th tile and runs the view groups of a tile back to
// back, so the workgroups resident on one XCD sample nearly the same beam of
// the volume and share its L2.
template <typename S, typename O, int TU, int TV, int C, int RCAP, int FCAP, int NVW>
__device__ __forceinline__ void forward_block(const FwdParams &p, const int bid)
{
    static_assert(TU * TV == 256, "one pixel per thread");
    static_assert(4 * NVW <= 64, "corner rays of a view group");
    constexpr int VE = 4;  // elements per staged vector
    using PreT = typename Stage<S>::T;
    constexpr int VPR = FCAP / VE;
    constexpr int RPI = 256 / VPR;
    constexpr int PLANE = RCAP * FCAP;
    constexpr int NCR = 4 * NVW;  // corner rays
    static_assert(FCAP % VE == 0 && RPI >= RCAP, "one staged row per thread and plane");
    // Two FP32 box buffers: chunk i is sampled from one while chunk i + 1
    // is staged.  FP32 storage is staged with direct global-to-LDS loads (16
    // bytes per lane, lane i of a wave at the wave's base + 16 i: thread t's
    // vector lands at float 4 t of the plane, its row-major place since a row
    // holds exactly VPR vectors); 16-bit storage with 8-byte loads into
    // registers, widened to FP32 into the other buffer once chunk i has been
    // sampled.
    constexpr bool DMA = std::is_same<S, float>::value;
    constexpr int NBUF = 2;
    static_assert(!DMA || VPR * VE == FCAP, "direct staging needs rows of exactly VPR vectors");
    __shared__ float box[NBUF][C * PLANE];
    constexpr int WIN = 64;      // chunks per window of boxes
    __shared__ int4 s_box[WIN];  // boxes of a window of chunks: f_al, s_lo, nvec | ns << 16, lds
    __shared__ float s_corner[NCR][4];
    __shared__ int s_dir[NCR];
    __shared__ int s_axes, s_m0, s_m1;

    const int t = threadIdx.x;
    const int tiles = p.tiles_u * p.tiles_v;
    const int tpx = (tiles + 7) >> 3;
    const int n_vg = (p.n_views + NVW - 1) / NVW;
    const int xcd = bid & 7;
    const int slot = bid >> 3;
    const int per_b = tpx * n_vg;
    const int b = slot / per_b;
    const int rem = slot - b * per_b;
    const int tile = (rem / n_vg) * 8 + xcd;
    const int view0 = (rem % n_vg) * NVW;
    if (tile >= tiles || b >= p.batch) return;  // padding workgroups (uniform exit)
    const int c0 = p.c_lo + (tile % p.tiles_u) * TU, r0 = p.r_lo + (tile / p.tiles_u) * TV;
    const int c = c0 + t % TU, r = r0 + t / TU;
    const bool inside = c < p.nu && r < p.nv;
    O *out = static_cast<O *>(p.sino);
    // views of the group that exist and whose window the tile meets (a
    // tile outside a view's own window sees no voxel: zeros); uniform
    bool vin[NVW];
    int wfirst = -1;
#pragma unroll
    for (int w = 0; w < NVW; ++w) {
        const int view = view0 + w;
        vin[w] = view < p.n_views;
        if (vin[w] && p.vwin) {
            const int *wn = p.vwin + 4 * view;
            if (c0 + TU <= wn[0] || c0 > wn[1] || r0 + TV <= wn[2] || r0 > wn[3]) vin[w] = false;
        }
        if (vin[w] && wfirst < 0) wfirst = w;
    }
    if (wfirst < 0) {
        if (inside)
#pragma unroll
            for (int w = 0; w < NVW; ++w)
                if (view0 + w < p.n_views)
                    out[((static_cast<int64_t>(b) * p.n_views + view0 + w) * p.nv + r) * p.nu + c] = from_f32<O>(0.0f);
        return;
    }

    // the rays' lines in registers: slopes, positions at plane 0, plane
    // range packed as m0 | m1 << 16 (empty: m0 > m1); the length per plane
    // is recomputed from the slopes at the end
    struct Line {
        float gf, gs, bf, bs;
        uint32_t rng;
        int axis;
    };
    Line seg[NVW];
    bool live[NVW];
    int amask = 0;
#pragma unroll
    for (int w = 0; w < NVW; ++w) {
        RaySeg rs;
        rs.axis = 0;
        rs.m0 = 1;
        rs.m1 = 0;
        rs.gf = rs.gs = rs.bf = rs.bs = rs.ds = 0.0f;
        if (inside && vin[w])
            ray_setup(p.tab[view0 + w], static_cast<double>(c), static_cast<double>(r), p.n, p.s, p.point_source != 0,
                      rs);
        live[w] = inside && vin[w] && rs.m0 <= rs.m1;
        seg[w].gf = rs.gf;
        seg[w].gs = rs.gs;
        seg[w].bf = rs.bf;
        seg[w].bs = rs.bs;
        seg[w].axis = rs.axis;
        seg[w].rng = live[w] ? static_cast<uint32_t>(rs.m0) | static_cast<uint32_t>(rs.m1) << 16 : 1u;
        if (live[w]) amask |= 1 << rs.axis;
    }
    if (t == 0) s_axes = 0;
    __syncthreads();
    if (amask) atomicOr(&s_axes, amask);
    __syncthreads();
    const int axes = s_axes;

    const int c1 = min(c0 + TU, p.nu) - 1, r1 = min(r0 + TV, p.nv) - 1;
    const int vr = t % VPR, rrow = t / VPR;  // this thread's vector and row of a staged plane
    float acc[NVW];
#pragma unroll
    for (int w = 0; w < NVW; ++w) acc[w] = 0.0f;
    for (int a = 0; a < 3; ++a) {
        if (!((axes >> a) & 1)) continue;
        bool part[NVW];
        int pm0 = 0x7fffffff, pm1 = -1;
#pragma unroll
        for (int w = 0; w < NVW; ++w) {
            part[w] = live[w] && seg[w].axis == a;
            if (part[w]) {
                pm0 = min(pm0, static_cast<int>(seg[w].rng & 0xffffu));
                pm1 = max(pm1, static_cast<int>(seg[w].rng >> 16));
            }
        }
        const int f = fast_axis(a), sl = slow_axis(a);
        const float nf = static_cast<float>(p.n[f]), ns = static_cast<float>(p.n[sl]);
        __syncthreads();
        if (t == 0) {
            s_m0 = 0x7fffffff;
            s_m1 = -1;
        }
        __syncthreads();
        if (pm0 <= pm1) {
            atomicMin(&s_m0, pm0);
            atomicMax(&s_m1, pm1);
        }
        if (t < NCR) {
            // corner ray t & 3 of view t >> 2, parametrised along axis a (a
            // view outside the tile's reach repeats the first one in reach)
            const int w = vin[t >> 2] ? t >> 2 : wfirst;
            const ViewTab &tab = p.tab[view0 + w];
            const double u = (t & 1) ? c1 : c0, v = ((t >> 1) & 1) ? r1 : r0;
            double d[3], q[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                d[i] = fma(tab.A[3 * i], u, fma(tab.A[3 * i + 1], v, tab.A[3 * i + 2]));
                q[i] = fma(tab.B[3 * i], u, fma(tab.B[3 * i + 1], v, tab.B[3 * i + 2]));
            }
            const double inv = 1.0 / d[a];
            const double gf = d[f] * inv, gs = d[sl] * inv;
            s_corner[t][0] = static_cast<float>(gf);
            s_corner[t][1] = static_cast<float>(fma(-q[a], gf, q[f]));
            s_corner[t][2] = static_cast<float>(gs);
            s_corner[t][3] = static_cast<float>(fma(-q[a], gs, q[sl]));
            s_dir[t] = d[a] > 0.0 ? 1 : (d[a] < 0.0 ? -1 : 0);
        }
        __syncthreads();
        const int M0 = s_m0, M1 = s_m1;
        // the corner crossings bound the tile's crossings when no ray of the
        // tile is parallel to the planes (same non-zero sign at the corners)
        bool box_ok = p.lay[a] != nullptr && s_dir[0] != 0;
#pragma unroll
        for (int k = 1; k < NCR; ++k) box_ok = box_ok && s_dir[k] == s_dir[0];
        const S *base = box_ok ? static_cast<const S *>(p.lay[a]) + b * p.lay_item[a] : nullptr;
        const int32_t row = p.lay_row[a];
        const int64_t plane = p.lay_plane[a];

        // the box of chunk [mc, min(mc + C - 1, M1)]
        auto make_box = [&](int mc) {
            Box bx;
            bx.mc = mc;
            bx.me = min(mc + C - 1, M1);
            bx.lds = box_ok;
            bx.f_al = bx.s_lo = bx.nvec = bx.ns = 0;
            if (box_ok) {
                float fmn = 3e38f, fmx = -3e38f, smn = 3e38f, smx = -3e38f;
#pragma unroll
                for (int k = 0; k < NCR; ++k) {
                    const float4 cr = *reinterpret_cast<const float4 *>(s_corner[k]);
                    const float pf0 = fmaf(static_cast<float>(bx.mc), cr.x, cr.y);
                    const float pf1 = fmaf(static_cast<float>(bx.me), cr.x, cr.y);
                    const float ps0 = fmaf(static_cast<float>(bx.mc), cr.z, cr.w);
                    const float ps1 = fmaf(static_cast<float>(bx.me), cr.z, cr.w);
                    fmn = fminf(fmn, fminf(pf0, pf1));
                    fmx = fmaxf(fmx, fmaxf(pf0, pf1));
                    smn = fminf(smn, fminf(ps0, ps1));
                    smx = fmaxf(smx, fmaxf(ps0, ps1));
                }
                // widen for FP32 rounding; a box far outside the grid
                // (which the staging fills with zeros) is cut to a size that
                // cannot overflow the integer conversions below
                fmn = fmaxf(fmn - 1e-3f, -1e6f);
                fmx = fminf(fmx + 1e-3f, 1e6f);
                smn = fmaxf(smn - 1e-3f, -1e6f);
                smx = fminf(smx + 1e-3f, 1e6f);
                const int f_lo = static_cast<int>(floorf(fmn)), f_hi = static_cast<int>(floorf(fmx)) + 1;
                bx.s_lo = static_cast<int>(floorf(smn));
                const int s_hi = static_cast<int>(floorf(smx)) + 1;
                bx.f_al = f_lo >= 0 ? f_lo / VE * VE : -((VE - 1 - f_lo) / VE) * VE;  // round down to a multiple of VE
                bx.nvec = (f_hi - bx.f_al) / VE + 1;
                bx.ns = s_hi - bx.s_lo + 1;
                bx.lds = fmn <= fmx && smn <= smx && bx.nvec <= VPR && bx.ns <= RCAP;
            }
            return bx;
        };
        // boxes of chunks wb .. wb + WIN - 1, one per thread
        auto window = [&](int wb) {
            const int mc = M0 + (wb + t) * C;
            if (t < WIN && mc <= M1) {
                const Box bx = make_box(mc);
                s_box[t] = make_int4(bx.f_al, bx.s_lo, bx.nvec | bx.ns << 16, bx.lds ? 1 : 0);
            }
        };
        auto box_at = [&](int ci, int wb) {
            const int mc = M0 + ci * C;
            if (ci - wb >= WIN) return make_box(mc);
            const int4 v = s_box[ci - wb];
            Box bx;
            bx.mc = mc;
            bx.me = min(mc + C - 1, M1);
            bx.f_al = v.x;
            bx.s_lo = v.y;
            bx.nvec = v.z & 0xffff;
            bx.ns = v.z >> 16;
            bx.lds = v.w != 0;
            return bx;
        };
        // 16-byte loads of this thread's share of a box (one row per plane);
        // rows and vectors outside the padded work copy are zeros
        const int32_t srows = p.n[sl] + PADR_LO + PADR_HI;
        PreT pre[C];
        auto issue = [&](const Box &bx) {
            if (!bx.lds || rrow >= bx.ns || vr >= bx.nvec) return;
            const int wr = bx.s_lo + PADR_LO + rrow;  // row of the work copy
            const int wc = bx.f_al + PADC + vr * VE;  // column of the work copy (multiple of VE)
            const bool in = wr >= 0 && wr < srows && wc >= 0 && wc + VE <= row;
            // a vector outside the padded copy reads the start of row 0 of
            // its plane, a zero padding row; planes past the chunk's last
            // re-read the last one (not staged)
            const S *src = base + static_cast<int64_t>(bx.mc) * plane +
                           (in ? static_cast<int64_t>(wr) * row + wc : static_cast<int64_t>(0));
            const int kmax = bx.me - bx.mc;
#pragma unroll
            for (int k = 0; k < C; ++k)
                pre[k] = *reinterpret_cast<const PreT *>(src + static_cast<int64_t>(min(k, kmax)) * plane);
        };

        // direct loads of this thread's share of a box into buffer `buf`
        auto issue_direct = [&](const Box &bx, int buf) {
            if (!bx.lds) return;  // uniform
            const bool mine = rrow < bx.ns && vr < bx.nvec;
            const int wr = bx.s_lo + PADR_LO + rrow;
            const int wc = bx.f_al + PADC + vr * VE;
            const bool in = wr >= 0 && wr < srows && wc >= 0 && wc + VE <= row;
            const S *src = base + static_cast<int64_t>(bx.mc) * plane +
                           (in ? static_cast<int64_t>(wr) * row + wc : static_cast<int64_t>(0));
            float *wave_dst = box[buf] + (t & ~63) * VE;  // the wave's first vector
            const int kmax = bx.me - bx.mc;
#if defined(__HIP_DEVICE_COMPILE__)  // a gfx950 builtin: the host pass never runs this
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (k <= kmax && mine)
                    __builtin_amdgcn_global_load_lds(src + static_cast<int64_t>(k) * plane, wave_dst + k * PLANE, 16,
                                                     0, 0);
#else
            (void)src, (void)wave_dst, (void)kmax, (void)mine;
#endif
        };

        // 16-bit storage: this thread's share of a box, widened to FP32, from
        // the registers `issue` loaded into buffer `buf` (waits for the loads)
        auto widen_store = [&](const Box &bx, int buf) {
            if (!bx.lds || rrow >= bx.ns || vr >= bx.nvec) return;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                if (bx.mc + k > bx.me) break;
                float v[VE];
                unpack4(pre[k], v, S{});
                float *dst = box[buf] + (k * RCAP + rrow) * FCAP + vr * VE;
#pragma unroll
                for (int e = 0; e < VE; e += 4)
                    *reinterpret_cast<float4 *>(dst + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
            }
        };

        // samples chunk `now` of every ray from box buffer `buf`
        auto sample_chunk = [&](const Box &now, int buf) {
#pragma unroll
            for (int w = 0; w < NVW; ++w) {
                // rays whose plane range misses the chunk sample nothing (a
                // wave whose rays all miss it skips the sampling)
                const Line &sg = seg[w];
                const int sm0 = static_cast<int>(sg.rng & 0xffffu), sm1 = static_cast<int>(sg.rng >> 16);
                if (!part[w] || sm1 < now.mc || sm0 > now.me) continue;
                if (now.lds) {
                    // box-local positions (the shifts by the integer box
                    // origin are exact): every position of the tile lies more
                    // than 1e-3 inside the box, which holds zeros outside the
                    // padded grid, so no clamp is needed; positions are >= 0,
                    // so truncation is floor.  The offset is capped to keep
                    // the reads inside the box array whatever the positions.
                    // LDS row pitch in bytes, in a VGPR (the multiply-add takes
                    // the plane offset as its one scalar operand)
                    uint32_t row_bytes = FCAP * 4;
                    asm volatile("" : "+v"(row_bytes));
                    const float fo = static_cast<float>(now.f_al), so = static_cast<float>(now.s_lo);
                    const float fmc = static_cast<float>(now.mc);
                    const float pf0 = fmaf(fmc, sg.gf, sg.bf - fo);
                    const float ps0 = fmaf(fmc, sg.gs, sg.bs - so);
                    const int kn = now.me - now.mc;
                    // taps of plane k: the reads of plane k + 1 are issued
                    // before plane k is interpolated (planes past the chunk's
                    // last read stale in-bounds LDS and are not used)
                    float tv[2][4], twf[2], tws[2];
                    float sum = 0.0f;
                    auto fetch = [&](int k, int sl_) {
                        const float pf = fmaf(static_cast<float>(k), sg.gf, pf0);
                        const float ps = fmaf(static_cast<float>(k), sg.gs, ps0);
                        twf[sl_] = __builtin_amdgcn_fractf(pf);
                        tws[sl_] = __builtin_amdgcn_fractf(ps);
                        // byte offset in the whole box array (both buffers):
                        // row and column of the tap in two ops, the buffer
                        // and plane in the uniform addend; the array's own
                        // LDS address folds into the reads' offset fields
                        uint32_t off;
                        asm("v_mad_u32_u24 %0, %1, %2, %3\n\tv_lshl_add_u32 %0, %4, 2, %0"
                            : "=&v"(off)
                            : "v"(static_cast<uint32_t>(ps)), "v"(row_bytes),
                              "s"(static_cast<uint32_t>((buf * C + k) * PLANE * 4)), "v"(static_cast<uint32_t>(pf)));
                        off = min(off, static_cast<uint32_t>((NBUF * C * PLANE - FCAP - 2) * 4));
                        asm volatile("" : "+v"(off));  // one base register for all four taps
                        const float *q = reinterpret_cast<const float *>(reinterpret_cast<const char *>(&box[0][0]) + off);
                        tv[sl_][0] = q[0];
                        tv[sl_][1] = q[1];
                        tv[sl_][2] = q[FCAP];
                        tv[sl_][3] = q[FCAP + 1];
                    };
                    auto interp = [&](int sl_) {
                        const float lo = fmaf(twf[sl_], tv[sl_][1] - tv[sl_][0], tv[sl_][0]);
                        const float hi = fmaf(twf[sl_], tv[sl_][3] - tv[sl_][2], tv[sl_][2]);
                        sum += fmaf(tws[sl_], hi - lo, lo);
                    };
                    fetch(0, 0);
                    if (kn == C - 1) {  // whole chunk (uniform): straight-line code
#pragma unroll
                        for (int k = 0; k < C; ++k) {
                            if (k + 1 < C) fetch(k + 1, (k + 1) & 1);
                            interp(k & 1);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < C; ++k) {
                            if (k > kn) break;  // uniform
                            if (k + 1 < C) fetch(k + 1, (k + 1) & 1);
                            interp(k & 1);
                        }
                    }
                    acc[w] += sum;
                } else {
                    // gathers from the padded work copy.  A copy exists for
                    // every axis a ray can take: the host builds one for each
                    // axis of the views' masks, which it finds by clipping the
                    // detector rectangle with |delta_a| >= |delta_b| - 1e-9
                    // max|delta| from the same FP64 tables the rays use here
                    // (the null test only keeps a broken mask from faulting)
                    const int ma = max(now.mc, sm0), mb = min(now.me, sm1);
                    if (p.lay[a] != nullptr) {
                        const S *lay = static_cast<const S *>(p.lay[a]) + b * p.lay_item[a];
                        for (int m = ma; m <= mb; ++m) {
                            const float fm = static_cast<float>(m);
                            acc[w] += sample_padded(lay + m * plane, row, fmaf(fm, sg.gf, sg.bf),
                                                    fmaf(fm, sg.gs, sg.bs), nf, ns);
                        }
                    }
                }
            }
        };

        int wb = 0;
        window(0);
        __syncthreads();
        Box cur = box_at(0, 0);
        if constexpr (DMA) {
            // chunk i is sampled from buffer i & 1 while chunk i + 1 goes
            // straight into the other one (last read for chunk i - 1); one
            // barrier per chunk
            issue_direct(cur, 0);
            __builtin_amdgcn_s_waitcnt(0);  // this thread's loads have reached LDS
            __syncthreads();
            for (int ci = 0, mc = M0; mc <= M1; ++ci, mc += C) {
                const int buf = ci & 1;
                const Box now = cur;
                if (mc + C <= M1) {
                    cur = box_at(ci + 1, wb);
                    issue_direct(cur, buf ^ 1);
                }
                sample_chunk(now, buf);
                if (ci + 2 - wb == WIN) {  // uniform: the next box lies past the window
                    __syncthreads();       // every box_at of this chunk has read the window
                    wb += WIN;
                    window(wb);
                }
                __builtin_amdgcn_s_waitcnt(0);  // chunk i + 1 has reached LDS
                __syncthreads();                // ... for every thread; chunk i is done
            }
        } else {
            // 16-bit storage: chunk i + 1 is loaded into registers while chunk
            // i is sampled from buffer i & 1, then widened into the other
            // buffer (last read for chunk i - 1); one barrier per chunk.
            // Iteration ci samples chunk ci (none for ci = -1) and stages
            // chunk ci + 1.
            issue(cur);
            Box smp = cur;
            for (int ci = -1, mc = M0 - C; mc <= M1; ++ci, mc += C) {
                if (ci >= 0) sample_chunk(smp, ci & 1);
                if (mc + C <= M1) {
                    smp = cur;
                    widen_store(cur, (ci + 1) & 1);
                }
                if (mc + 2 * C <= M1) {
                    cur = box_at(ci + 2, wb);
                    issue(cur);  // in flight while chunk ci + 1 is sampled
                }
                if (ci + 3 - wb == WIN) {  // uniform: the next box_at lies past the window
                    __syncthreads();       // every box_at of this iteration has read the window
                    wb += WIN;
                    window(wb);
                }
                __syncthreads();  // chunk ci + 1 is staged for every thread; chunk ci is done
            }
        }
    }
    if (!inside) return;
#pragma unroll
    for (int w = 0; w < NVW; ++w) {
        if (view0 + w >= p.n_views) continue;
        // ray length per plane (mm): one plane step moves (1, gf, gs) voxels
        // along (a, f, s)
        const int ax = seg[w].axis;
        const float sa = static_cast<float>(p.s[ax]);
        const float xf = seg[w].gf * static_cast<float>(p.s[fast_axis(ax)]);
        const float xs = seg[w].gs * static_cast<float>(p.s[slow_axis(ax)]);
        const float ds = __builtin_amdgcn_sqrtf(fmaf(xf, xf, fmaf(xs, xs, sa * sa)));
        out[((static_cast<int64_t>(b) * p.n_views + view0 + w) * p.nv + r) * p.nu + c] =
            from_f32<O>(live[w] ? acc[w] * ds : 0.0f);
    }
}

template <typename S, typename O, int TU, int TV, int C, int RCAP, int FCAP, int NVW>
__global__ __launch_bounds__(256, 5) void forward_kernel(FwdParams p)
{
    forward_block<S, O, TU, TV, C, RCAP, FCAP, NVW>(p, blockIdx.x);
}

template <typename S, typename O, int TU, int TV, int C, int RCAP, int FCAP, int NVW>
__global__ __launch_bounds__(256, 5) void forward_batch_kernel(Batch<FwdParams> w)
{
    const int i = batch_item(w, blockIdx.x);
    forward_block<S, O, TU, TV, C, RCAP, FCAP, NVW>(w.p[i], blockIdx.x - w.start[i]);
}

template <typename S, typename O, int TU, int TV, int C, int RCAP, int FCAP, int NVW>
__global__ __launch_bounds__(256, 5) void forward_table_kernel(Table<FwdParams> w)
{
    const int i = table_item(w, blockIdx.x);
    forward_block<S, O, TU, TV, C, RCAP, FCAP, NVW>(w.p[i], blockIdx.x - w.start[i]);
}

// ------------------------------------------------------- adjoint A^T -----

// Round to nearest (halves up): v_cvt_rpi_i32_f32 computes floor(x + 0.5)
// in one instruction; the compiler only forms it under fast-math.
__device__ __forceinline__ int round_fixed(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// A value known to be the same in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform_f32(float x)
{
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}

// Wave-wide helpers for the adjoint's ray-list compaction.  They are called
// with every lane of the wave active.
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Maximum over the wave: DPP exchanges within each row of 16 lanes (lane
// xor 1, xor 2, then the half-row and row mirrors leave the row maximum in
// every lane of the row), then the four row maxima in scalar registers.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0xb1, 0xf, 0xf, false)));
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x4e, 0xf, 0xf, false)));
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x141, 0xf, 0xf, false)));
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x140, 0xf, 0xf, false)));
    const uint32_t r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const uint32_t r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return max(max(r0, r1), max(r2, r3));
}

// Axes of a pass: a is the dominant (plane) axis, f and s the in-plane fast
// and slow axes.  A ray belongs to pass a when |delta_a| is the largest
// component, exact ties going to the lowest axis.
template <int A>
struct PassAxes {
    static constexpr int F = A == 0 ? 1 : 0;
    static constexpr int S = A == 2 ? 1 : 2;
    __device__ static bool dominant(double da, double df, double ds)
    {
        const double aa = fabs(da), af = fabs(df), as = fabs(ds);
        // f < a unless A == 0; s > a unless A == 2
        const bool vs_f = A == 0 ? aa >= af : aa > af;
        const bool vs_s = A == 2 ? aa > as : aa >= as;
        return vs_f && vs_s;
    }
};

// Narrows the local plane range [lo, hi] to the planes m where b + m*g lies
// in [lo_pos - 1e-3, hi_pos + 1e-3].  The FP32 rounding of the bounds moves
// a position at a boundary plane by ~|b| 2^-22, far less than the 1e-3
// widening (so no plane inside the band is dropped) and than the cell of
// margin the LDS block has beyond the band (so no tap leaves the block).
// Branch-free: a zero slope is replaced by a tiny positive one, which keeps
// or empties the whole range as the exact test would.
__device__ __forceinline__ void clip_local(float b, float g, float lo_pos, float hi_pos, float &lo, float &hi)
{
    const float gg = fabsf(g) < 1e-30f ? 1e-30f : g;
    const float rg = __builtin_amdgcn_rcpf(gg);
    const float t0 = (lo_pos - 1e-3f - b) * rg, t1 = (hi_pos + 1e-3f - b) * rg;
    lo = fmaxf(lo, ceilf(fminf(t0, t1)));
    hi = fminf(hi, floorf(fmaxf(t0, t1)));
}

// Candidate pixel boxes of the adjoint: for every block of a pass and
// every view of the pass, the pixels (integer centres) inside the detector
// bounding box of the block dilated by one voxel in-plane, i.e. of the
// projections of its 8 corners (FP32 from the rounded index-space matrix;
// the 0.01 pixel margin covers the rounding), intersected with the view's
// box of pixels whose ray may have the pass axis as dominant axis (host,
// exact, widened by one pixel) and clamped to the detector.  The projection
// of a convex box in front of the source is the convex hull of its corners'
// projections, so every ray of the pass that can sample the block has its
// pixel in the box.  Stored as 2 words: first column | first row << 16,
// columns | rows << 16 (0: empty).
struct CboxParams {
    const ViewTabF *tabf;
    const int32_t *views;
    const uint32_t *axbox;  // per view and axis: first col | row << 16, last col | row << 16
    int32_t n_pass_views, axis, nu, nv;
    int32_t n[3];
    int32_t L, TS, TF;
    int32_t blocks_a, blocks_s, blocks_f;
    uint32_t *out;
};

__global__ __launch_bounds__(256) void cbox_kernel(CboxParams p)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nb = static_cast<int64_t>(p.blocks_a) * p.blocks_s * p.blocks_f;
    if (e >= nb * p.n_pass_views) return;
    const int pv = static_cast<int>(e % p.n_pass_views);
    int blk = static_cast<int>(e / p.n_pass_views);
    const int bf_ = blk % p.blocks_f;
    blk /= p.blocks_f;
    const int bs_ = blk % p.blocks_s;
    const int ba_ = blk / p.blocks_s;
    const int a = p.axis, f = a == 0 ? 1 : 0, sl = a == 2 ? 1 : 2;
    const int a0 = ba_ * p.L, a1 = min(a0 + p.L, p.n[a]);
    const int s0 = bs_ * p.TS, s1 = min(s0 + p.TS, p.n[sl]);
    const int f0 = bf_ * p.TF, f1 = min(f0 + p.TF, p.n[f]);
    const int view = p.views[pv];
    const ViewTabF &tf = p.tabf[view];
    float umin = 3e38f, umax = -3e38f, vmin = 3e38f, vmax = -3e38f;
    for (int corner = 0; corner < 8; ++corner) {
        float ijk[3];
        ijk[a] = (corner & 1) ? static_cast<float>(a1 - 1) : static_cast<float>(a0);
        ijk[sl] = (corner & 2) ? static_cast<float>(s1) : static_cast<float>(s0 - 1);
        ijk[f] = (corner & 4) ? static_cast<float>(f1) : static_cast<float>(f0 - 1);
        const float U = fmaf(tf.Pi[0], ijk[0], fmaf(tf.Pi[1], ijk[1], fmaf(tf.Pi[2], ijk[2], tf.Pi[3])));
        const float V = fmaf(tf.Pi[4], ijk[0], fmaf(tf.Pi[5], ijk[1], fmaf(tf.Pi[6], ijk[2], tf.Pi[7])));
        const float Wc = fmaf(tf.Pi[8], ijk[0], fmaf(tf.Pi[9], ijk[1], fmaf(tf.Pi[10], ijk[2], tf.Pi[11])));
        const float rw = __builtin_amdgcn_rcpf(Wc);
        umin = fminf(umin, U * rw);
        umax = fmaxf(umax, U * rw);
        vmin = fminf(vmin, V * rw);
        vmax = fmaxf(vmax, V * rw);
    }
    // clamp before converting: the bounds are finite (W > 0 over the
    // dilated volume) but may lie far outside the detector
    const uint32_t ab0 = p.axbox[2 * (3 * static_cast<int64_t>(view) + a)];
    const uint32_t ab1 = p.axbox[2 * (3 * static_cast<int64_t>(view) + a) + 1];
    const float au0 = static_cast<float>(ab0 & 0xffffu), av0 = static_cast<float>(ab0 >> 16);
    const float au1 = static_cast<float>(ab1 & 0xffffu), av1 = static_cast<float>(ab1 >> 16);
    const int cu0 = static_cast<int>(fminf(fmaxf(ceilf(umin - 0.01f), au0), static_cast<float>(p.nu)));
    const int cu1 = static_cast<int>(fmaxf(fminf(floorf(umax + 0.01f), au1), -1.0f));
    const int cv0 = static_cast<int>(fminf(fmaxf(ceilf(vmin - 0.01f), av0), static_cast<float>(p.nv)));
    const int cv1 = static_cast<int>(fmaxf(fminf(floorf(vmax + 0.01f), av1), -1.0f));
    const bool empty = cu0 > cu1 || cv0 > cv1;
    const uint32_t w0 = empty ? 0u : static_cast<uint32_t>(cu0) | static_cast<uint32_t>(cv0) << 16;
    const uint32_t w1 = empty ? 0u : static_cast<uint32_t>(cu1 - cu0 + 1) | static_cast<uint32_t>(cv1 - cv0 + 1) << 16;
    p.out[2 * e] = w0;
    p.out[2 * e + 1] = w1;
}

hipError_t launch_cbox(const AdjParams &ap, const uint32_t *axbox, int32_t L, int32_t TS, int32_t TF, uint32_t *out,
                       hipStream_t st)
{
    CboxParams p{};
    p.tabf = ap.tabf;
    p.views = ap.views;
    p.axbox = axbox;
    p.n_pass_views = ap.n_pass_views;
    p.axis = ap.axis;
    p.nu = ap.nu;
    p.nv = ap.nv;
    for (int i = 0; i < 3; ++i) p.n[i] = ap.n[i];
    p.L = L;
    p.TS = TS;
    p.TF = TF;
    p.blocks_a = ap.blocks_a;
    p.blocks_s = ap.blocks_s;
    p.blocks_f = ap.blocks_f;
    p.out = out;
    const int64_t total = static_cast<int64_t>(ap.blocks_a) * ap.blocks_s * ap.blocks_f * ap.n_pass_views;
    if (total == 0) return hipSuccess;
    cbox_kernel<<<dim3(static_cast<uint32_t>((total + 255) / 256)), 256, 0, st>>>(p);
    return hipGetLastError();
}

// A flush period of the adjoint ends early when a batch's rays are more than
// 2^kQuietBits times quieter than the period's scale is made for.
constexpr int kQuietBits = 2;

// Each workgroup owns a block of L planes (dominant axis A) x TS rows x TF
// columns of the output.  Its FP32 sums live in registers (each thread owns
// L*TS*TF/256 voxels); per batch of candidate rays they are gathered in LDS
// as 32-bit fixed-point accumulators with a halo of two cells below and two
// above in the fast in-plane direction (SLO + 1 and SHI in the slow one):
//   phase A  each thread takes CPT candidate pixels of the detector bounding
//            box of the block (dilated by one voxel in-plane), does the
//            ray's FP64 set-up in the block's local frame and, if the ray
//            has A as dominant axis and samples the dilated block, appends
//            it to an LDS ray list (wave-aggregated compaction) with its
//            plane range cut into segments of <= K planes;
//   phase B  each thread takes segments and scatters the bilinear taps of
//            their samples with ds_add_u32.  A segment's planes are those
//            where the ray's position lies in the block dilated by one
//            voxel (the reach of a tap), so every tap lands in the block or
//            its halo (no clamp); halo cells are discarded;
//   flush    when the next batch could overflow the integers, each thread
//            moves its voxels' integer sums into its FP32 registers and
//            clears them (and once at the end).
// A ray samples a voxel's plane once with weight <= 1, and at most kcell
// rays of a view sample within one voxel of a given voxel (a per-view bound
// from the geometry), so a batch adds at most min(rays, kcell) x qmax to any
// voxel, qmax being the batch's largest |q*ds| (gathered in phase A).  The
// fixed-point scale is a power of two per flush period of the workgroup:
// the first batch of a period sets it so that kunits (a power of two,
// >= 256 and >= every kcell) times its qmax lies in [2^29, 2^30).  A batch
// whose bound would take the period's running sum past 2^30, or whose qmax
// needs a scale more than 2^kQuietBits larger (a much quieter batch), flushes
// and starts a new period at its own scale.  The rounding error of a
// contribution is therefore at most kunits 2^(kQuietBits+1) 2^-31 times the
// qmax of its own batch (round to nearest, so errors partly cancel): the
// accuracy follows the magnitude of the rays that reach the block, not the
// sinogram's global maximum, and each batch item has its own scales.
// Integer addition is exact and order-independent and the flushes happen
// at the same points in every run, so the result is deterministic.  A
// non-finite q*ds among a batch's rays turns the block's output into NaN.
//
// SLO/SHI: halo rows below/above the block in the slow in-plane direction
// besides the extra row below, 1/2 in general; 0/1 for 2-D problems, whose
// rays have z == 0 exactly (the tap at z = 0 has weight 1 and the one at
// z = 1 weight 0).
// LDS of one adjoint workgroup (declared by the kernel, so that the passes
// of a fused launch share it).
template <int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
struct AdjLds {
    static constexpr int RW = TF + 4;              // LDS row (halo: 2 before, 2 after)
    static constexpr int RP = TS + SLO + SHI + 1;  // LDS rows per plane
    // LDS plane: RP rows plus 2 or 3 padding cells, so that a plane is 2
    // cells past a multiple of 4: the two segments of one ray, 8 planes
    // apart and scattered by neighbouring lanes, then fall into different
    // LDS banks
    static constexpr int PL = RP * RW + (6 - (RP * RW) % 4) % 4;
    static constexpr int MAXR = NT * CPT;          // rays per batch
    static constexpr int MAXSEG = MAXR * ((L + 7) / 8);
    float4 s_ray[MAXR];      // gf, bf, gs, bs (block-local frame)
    int acc[L * PL];
    float s_q[MAXR];         // q * ds
    uint32_t s_seg[MAXSEG];  // slot | first local plane << 16 | planes << 24
    uint32_t s_cnt[2][2];    // [parity][rays | segments << 16, max |q*ds| bits]
};

template <typename Q, int A, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
__device__ __forceinline__ void adjoint_block(const AdjParams &p, const int bid,
                                              AdjLds<L, TS, TF, SLO, SHI, CPT, NT> &sh)
{
    using AX = PassAxes<A>;
    constexpr int F = AX::F, S = AX::S;
    constexpr int K = 8;                       // planes per segment
    constexpr int RW = TF + 4;                 // LDS row (halo: 2 before, 2 after)
    constexpr int RP = TS + SLO + SHI + 1;     // LDS rows per plane
    constexpr int PL = RP * RW + (6 - (RP * RW) % 4) % 4;  // LDS plane (padded, as AdjLds)
    constexpr int NV = L * TS * TF;            // voxels of the block
    constexpr int NQ = (NV + NT - 1) / NT;     // voxels per thread
    constexpr int MAXR = NT * CPT;             // rays per batch
    constexpr int SPR = (L + K - 1) / K;       // segments per ray, at most
    constexpr int MAXSEG = MAXR * SPR;
    static_assert(L <= 32 && SPR <= 4, "segment record packing");
    static_assert(MAXR <= 1024 && MAXSEG < 65536, "packed counters");
    static_assert(MAXSEG == AdjLds<L, TS, TF, SLO, SHI, CPT, NT>::MAXSEG && PL == AdjLds<L, TS, TF, SLO, SHI, CPT, NT>::PL,
                  "LDS layout");
    int *acc = sh.acc;
    float4 *s_ray = sh.s_ray;
    float *s_q = sh.s_q;
    uint32_t *s_seg = sh.s_seg;
    uint32_t(*s_cnt)[2] = sh.s_cnt;

    int blk = bid;
    const int bf_ = blk % p.blocks_f;
    blk /= p.blocks_f;
    const int bs_ = blk % p.blocks_s;
    blk /= p.blocks_s;
    const int ba_ = blk % p.blocks_a;
    const int b = blk / p.blocks_a;
    const int a0 = ba_ * L, a1 = min(a0 + L, p.n[A]);
    const int s0 = bs_ * TS, s1 = min(s0 + TS, p.n[S]);
    const int f0 = bf_ * TF, f1 = min(f0 + TF, p.n[F]);
    // block-local frame: local = global - origin, the origin being the
    // first halo cell.  The positions whose taps reach a voxel of the block
    // lie in the block dilated by one voxel, local [1, f1 - f0 + 2] x
    // [1, s1 - s0 + 2]; the LDS block has one more cell on every side.  2-D
    // rays sit exactly at local row 1 (band [0.5, 1.5]).
    const float flo = 1.0f, fhi = static_cast<float>(f1 - f0 + 2);
    const float slo = TS == 1 ? 0.5f : 1.0f;
    const float shi = TS == 1 ? 1.5f : static_cast<float>(s1 - s0 + 2);
    const float amaxl = static_cast<float>(a1 - a0 - 1);
    const int t = threadIdx.x, lane = t & 63;
    const int wbase = __builtin_amdgcn_readfirstlane(t & ~63);  // first thread of the wave
    // voxel spacing along the pass axis and the in-plane spacings relative to it
    const float sa = static_cast<float>(p.s[A]);
    const float sfa = static_cast<float>(p.s[F] / p.s[A]), ssa = static_cast<float>(p.s[S] / p.s[A]);
    const double oa = a0, of = f0 - 2, os = s0 - SLO - 1;

    // the voxels this thread owns: e = t + NT q, x fastest (coalesced output)
    float reg[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) reg[q] = 0.0f;
    // (a cubic block maps thread t to the same voxels in every pass: x, then
    // y, then z)
    auto cell_of = [](int e, int &la, int &ls, int &lf) {
        if (A == 0) {  // x = a, y = f, z = s
            la = e % L;
            lf = (e / L) % TF;
            ls = e / (L * TF);
        } else if (A == 1 || L != TS) {  // x = f
            lf = e % TF;
            la = (e / TF) % L;
            ls = e / (TF * L);
        } else {       // z pass of a cubic block: x = f, y = s, z = a
            lf = e % TF;
            ls = (e / TF) % TS;
            la = e / (TF * TS);
        }
    };

    for (int e = t; e < L * PL; e += NT) acc[e] = 0;
    if (t < 4) s_cnt[t >> 1][t & 1] = 0u;
    __syncthreads();

    // fixed-point scale of the current flush period, 2^ecur; `pending`
    // bounds the period's integer sums (no period open before the first
    // batch with a non-zero contribution)
    int ecur = 0;
    bool open = false, poisoned = false;
    float scale = 1.0f, inv_scale = 1.0f;
    float pending = 0.0f;
    const int ku = __builtin_amdgcn_frexp_expf(p.kunits) - 1;  // kunits = 2^ku
    auto flush = [&]() {
        // flushes are rare: recompute the cell addresses rather than keep
        // them in registers across the whole kernel
        int tt = t;
        asm volatile("" : "+v"(tt));
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int el = tt + NT * q;
            if (el < NV) {
                int la, ls, lf;
                cell_of(el, la, ls, lf);
                int *cellp = acc + la * PL + (ls + SLO + 1) * RW + lf + 2;
                reg[q] = fmaf(static_cast<float>(*cellp), inv_scale, reg[q]);
                *cellp = 0;
            }
        }
    };

    const Q *sino_b = static_cast<const Q *>(p.sino) + static_cast<int64_t>(b) * p.n_views * p.nv * p.nu;
    int parity = 0;
    // per view: its index and the block's candidate pixel box (precomputed
    // by cbox_kernel), loaded one view ahead so the loads are in flight
    // while the current view is processed
    const int nbi = p.blocks_a * p.blocks_s * p.blocks_f;
    const uint32_t *cbox = p.cbox + 2 * static_cast<int64_t>(bid % nbi) * p.n_pass_views;
    int nx_view = p.n_pass_views > 0 ? p.views[0] : 0;
    uint32_t nx_b0 = p.n_pass_views > 0 ? cbox[0] : 0u, nx_b1 = p.n_pass_views > 0 ? cbox[1] : 0u;
    for (int pv = 0; pv < p.n_pass_views; ++pv) {
        const int view = __builtin_amdgcn_readfirstlane(nx_view);
        const uint32_t b0 = __builtin_amdgcn_readfirstlane(nx_b0), b1 = __builtin_amdgcn_readfirstlane(nx_b1);
        if (pv + 1 < p.n_pass_views) {
            nx_view = p.views[pv + 1];
            nx_b0 = cbox[2 * (pv + 1)];
            nx_b1 = cbox[2 * (pv + 1) + 1];
        }
        const int cu0 = static_cast<int>(b0 & 0xffffu), cv0 = static_cast<int>(b0 >> 16);
        const int wu = static_cast<int>(b1 & 0xffffu), wv = static_cast<int>(b1 >> 16);
        if (wu == 0 || wv == 0) continue;  // uniform
        const float kcell = p.tabf[view].kcell;
        // the view's FP64 ray tables, needed rows only (uniform loads)
        const ViewTab &tv = p.tab[view];
        const double Aa0 = tv.A[3 * A], Aa1 = tv.A[3 * A + 1], Aa2 = tv.A[3 * A + 2];
        const double Af0 = tv.A[3 * F], Af1 = tv.A[3 * F + 1], Af2 = tv.A[3 * F + 2];
        const double As0 = tv.A[3 * S], As1 = tv.A[3 * S + 1], As2 = tv.A[3 * S + 2];
        // points on the rays, in the block-local frame
        const double Ba0 = tv.B[3 * A], Ba1 = tv.B[3 * A + 1], Ba2 = tv.B[3 * A + 2] - oa;
        const double Bf0 = tv.B[3 * F], Bf1 = tv.B[3 * F + 1], Bf2 = tv.B[3 * F + 2] - of;
        const double Bs0 = tv.B[3 * S], Bs1 = tv.B[3 * S + 1], Bs2 = tv.B[3 * S + 2] - os;
        const int wu_e = (wu + 1) >> 1, wu_o = wu >> 1, wv_e = (wv + 1) >> 1;
        // first candidate of the parity classes (odd column, even row),
        // (even column, odd row) and (odd column, odd row)
        const int T1 = wu_e * wv_e, T2 = T1 + wu_o * wv_e, T3 = T2 + wu_e * (wv >> 1);
        const int ncand = wu * wv;
        // below 2^20 candidates the reciprocal estimate of j / w is exact:
        // its relative error (rcp 1 ulp, product 1/2 ulp) times (j + 1/2) / w
        // stays below the 1/(2w) distance to the nearest integer
        const bool exact = ncand <= (1 << 20);
        const float rwe = __builtin_amdgcn_rcpf(static_cast<float>(wu_e));
        const float rwo = wu_o > 0 ? __builtin_amdgcn_rcpf(static_cast<float>(wu_o)) : 0.0f;
        const Q *sino_v = sino_b + static_cast<int64_t>(view) * p.nv * p.nu;
        for (int cb = 0; cb < ncand; cb += MAXR) {
            // ---- phase A: set-up of up to MAXR candidates, compacted into LDS.
            // The candidates' pixels are decoded and their sinogram values
            // requested first, so the loads are in flight during the set-up.
            int cc[CPT], cr[CPT];
            float qv[CPT];
#pragma unroll
            for (int cq = 0; cq < CPT; ++cq) {
                const int idx = cb + t + NT * cq;
                cc[cq] = -1;
                cr[cq] = 0;
                qv[cq] = 0.0f;
                if (idx < ncand) {
                    // parity classes (c - cu0, r - cv0) mod 2, each row-major
                    // (branch-free class selection)
                    const bool k1 = idx >= T1, k2 = idx >= T2, k3 = idx >= T3;
                    const int j = idx - (k3 ? T3 : (k2 ? T2 : (k1 ? T1 : 0)));
                    const bool odd_c = k3 || (k1 && !k2);
                    const int w = odd_c ? wu_o : wu_e;
                    int jq = static_cast<int>((static_cast<float>(j) + 0.5f) * (odd_c ? rwo : rwe));
                    if (!exact) {  // j, w < 2^24: the estimate is within one
                        jq -= (__mul24(jq, w) > j) ? 1 : 0;
                        jq += (__mul24(jq + 1, w) <= j) ? 1 : 0;
                    }
                    cc[cq] = cu0 + (odd_c ? 1 : 0) + 2 * (j - __mul24(jq, w));
                    cr[cq] = cv0 + (k2 ? 1 : 0) + 2 * jq;
                    // r * nu + c < 2^31 (sinogram views are validated)
                    qv[cq] = to_f32(sino_v[__umul24(static_cast<uint32_t>(cr[cq]), static_cast<uint32_t>(p.nu)) +
                                           static_cast<uint32_t>(cc[cq])]);
                }
            }
#pragma unroll
            for (int cq = 0; cq < CPT; ++cq) {
                // a wave whose candidates all lie past the end of the box
                // skips the set-up and the append (wave-uniform)
                if (cb + wbase + NT * cq >= ncand) continue;
                bool ok = false;
                float4 rec = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                float dsm = 0.0f;
                int m0 = 0, nseg = 0;
                if (cc[cq] >= 0) {
                    const double u = cc[cq], v = cr[cq];
                    const double da = fma(Aa0, u, fma(Aa1, v, Aa2));
                    const double df = fma(Af0, u, fma(Af1, v, Af2));
                    const double dsl = fma(As0, u, fma(As1, v, As2));
                    if (AX::dominant(da, df, dsl)) {
                        // 1/da: hardware reciprocal refined by two Newton steps
                        double inv = __builtin_amdgcn_rcp(da);
                        inv = inv * fma(-da, inv, 2.0);
                        inv = inv * fma(-da, inv, 2.0);
                        const double gf = df * inv, gs = dsl * inv;
                        // a point on the ray: the source for a point source
                        double pa = Ba2, pf = Bf2, ps = Bs2;
                        if (!p.point_source) {  // uniform; the asm keeps it a branch
                            asm volatile("");
                            pa = fma(Ba0, u, fma(Ba1, v, Ba2));
                            pf = fma(Bf0, u, fma(Bf1, v, Bf2));
                            ps = fma(Bs0, u, fma(Bs1, v, Bs2));
                        }
                        // in-plane position at local plane 0
                        const float bfl = static_cast<float>(fma(-pa, gf, pf));
                        const float bsl = static_cast<float>(fma(-pa, gs, ps));
                        const float gf32 = static_cast<float>(gf), gs32 = static_cast<float>(gs);
                        // ray length per plane (mm), FP32: one plane step moves
                        // (1, gf, gs) voxels along (a, f, s)
                        const float xf = gf32 * sfa, xs = gs32 * ssa;
                        dsm = __builtin_amdgcn_sqrtf(fmaf(xf, xf, fmaf(xs, xs, 1.0f))) * sa;
                        float lo = 0.0f, hi = amaxl;
                        clip_local(bfl, gf32, flo, fhi, lo, hi);
                        clip_local(bsl, gs32, slo, shi, lo, hi);
                        m0 = static_cast<int>(lo);
                        const int m1 = static_cast<int>(hi);
                        if (m0 <= m1 && isfinite(dsm)) {
                            ok = true;
                            rec = make_float4(gf32, bfl, gs32, bsl);
                            nseg = (m1 - m0 + K) / K;
                            // pack the last segment's length with the count
                            nseg |= (m1 - m0 + 1 - (nseg - 1) * K) << 8;
                        }
                    }
                }
                const float qs = ok ? qv[cq] * dsm : 0.0f;
                // wave-aggregated append (all lanes active here)
                const int ns = nseg & 0xff;
                const uint64_t mr = __ballot(ok);
                const uint64_t m1b = __ballot(ns & 1), m2b = __ballot(ns & 2), m4b = __ballot(ns & 4);
                const uint32_t nr = static_cast<uint32_t>(__popcll(mr));
                const uint32_t nsw = static_cast<uint32_t>(__popcll(m1b) + 2 * __popcll(m2b) + 4 * __popcll(m4b));
                const uint32_t qbits = wave_max_u32(ok ? __float_as_uint(fabsf(qs)) : 0u);
                uint32_t base = 0;
                if (lane == 0 && nr > 0) {
                    base = atomicAdd(&s_cnt[parity][0], nr | nsw << 16);
                    atomicMax(&s_cnt[parity][1], qbits);
                }
                base = __builtin_amdgcn_readfirstlane(base);
                if (ok) {
                    const int slot = static_cast<int>((base & 0xffff) + lane_rank(mr));
                    const int sb = static_cast<int>((base >> 16) + lane_rank(m1b) + 2 * lane_rank(m2b) +
                                                    4 * lane_rank(m4b));
                    s_ray[slot] = rec;
                    s_q[slot] = qs;
                    const int last = nseg >> 8;
                    for (int k = 0; k < ns; ++k) {
                        const int cnt = k == ns - 1 ? last : K;
                        s_seg[sb + k] = static_cast<uint32_t>(slot) | static_cast<uint32_t>(m0 + k * K) << 16 |
                                        static_cast<uint32_t>(cnt) << 24;
                    }
                }
            }
            __syncthreads();
            // ---- phase B: scatter segments (fixed point)
            const uint32_t cnts = s_cnt[parity][0];
            const int nray = static_cast<int>(cnts & 0xffff);
            const int nseg_all = static_cast<int>(cnts >> 16);
            const uint32_t qbits = s_cnt[parity][1];
            const float qmax = __uint_as_float(qbits);
            if (t < 2) s_cnt[parity ^ 1][t] = 0u;
            // a batch whose rays all carry q*ds = 0 adds nothing; a non-finite
            // q*ds poisons the block (uniform decisions: LDS values)
            if (qbits >= 0x7f800000u) poisoned = true;
            const bool live = nray > 0 && qbits != 0u && qbits < 0x7f800000u;
            if (live) {
                // the scale this batch alone would take: kunits qmax 2^eb in
                // [2^29, 2^30); the batch adds at most min(nray, kcell) x qmax
                // to a voxel
                const int eb = min(126, max(-126, 30 - ku - __builtin_amdgcn_frexp_expf(qmax)));
                const float nb = fminf(static_cast<float>(nray), kcell) * qmax;
                if (!open || pending + nb * scale > 1073741824.0f || eb > ecur + kQuietBits) {
                    if (open) {
                        flush();
                        __syncthreads();  // cells cleared before the scatter
                    }
                    ecur = eb;
                    scale = exp2f(static_cast<float>(eb));
                    inv_scale = exp2f(static_cast<float>(-eb));
                    pending = 0.0f;
                    open = true;
                }
                pending += nb * scale;
            }
            for (int se = t; se < (live ? nseg_all : 0); se += NT) {
                const uint32_t srec = s_seg[se];
                const int slot = srec & 0xffff, la0 = (srec >> 16) & 0xff, cnt = srec >> 24;
                const float4 rp = s_ray[slot];
                const float qs = s_q[slot] * scale;
                // positions at the segment's first plane, then fma(k, slope, .):
                // inside the LDS block by construction of the plane range
                const float fm0 = static_cast<float>(la0);
                const float pf0 = fmaf(fm0, rp.x, rp.y), ps0 = fmaf(fm0, rp.z, rp.w);
                const uint32_t base0 = static_cast<uint32_t>(la0 * PL * 4);
                // every segment has >= 1 plane: the first sample is taken
                // unconditionally (so the record loads are waited for once,
                // before any branch)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (k == 0 || k < cnt) {
                        const float pf = k == 0 ? pf0 : fmaf(static_cast<float>(k), rp.x, pf0);
                        const float ps = k == 0 ? ps0 : fmaf(static_cast<float>(k), rp.z, ps0);
                        const float wf = __builtin_amdgcn_fractf(pf), ws = __builtin_amdgcn_fractf(ps);
                        // positions are >= 1 up to rounding: truncation is floor.
                        // Byte offset of the tap cell in the segment's first
                        // plane, in two ops; the plane and the other three taps
                        // are immediate offsets of the LDS atomics.
                        const uint32_t is = static_cast<uint32_t>(ps), ifl = static_cast<uint32_t>(pf);
                        uint32_t off;
                        asm("v_mad_u32_u24 %0, %1, %2, %3\n\tv_lshl_add_u32 %0, %4, 2, %0"
                            : "=&v"(off)
                            : "v"(is), "s"(static_cast<uint32_t>(RW * 4)), "v"(base0), "v"(ifl));
                        int *q = reinterpret_cast<int *>(reinterpret_cast<char *>(acc) + off) + k * PL;
                        const float t1 = qs * ws, t0 = qs - t1;
                        const float c01f = t0 * wf, c11f = t1 * wf;
                        atomicAdd(q, round_fixed(t0 - c01f));
                        atomicAdd(q + 1, round_fixed(c01f));
                        atomicAdd(q + RW, round_fixed(t1 - c11f));
                        atomicAdd(q + RW + 1, round_fixed(c11f));
                    }
                }
            }
            __syncthreads();
            // halo cells are never read, so they are never cleared
            parity ^= 1;
        }
    }
    if (open) flush();
    if (poisoned)
#pragma unroll
        for (int q = 0; q < NQ; ++q) reg[q] = __int_as_float(0x7fc00000);

    // write the block; the memory-contiguous axis x runs fastest
    const int64_t item = static_cast<int64_t>(p.n[0]) * p.n[1] * p.n[2];
    float *out = p.out + b * item;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int el = t + NT * q;
        if (el >= NV) continue;
        int la, ls, lf;
        cell_of(el, la, ls, lf);
        if (a0 + la >= a1 || s0 + ls >= s1 || f0 + lf >= f1) continue;
        int ijk[3];
        ijk[A] = a0 + la;
        ijk[S] = s0 + ls;
        ijk[F] = f0 + lf;
        const int64_t o = (static_cast<int64_t>(ijk[2]) * p.n[1] + ijk[1]) * p.n[0] + ijk[0];
        out[o] = p.accumulate ? out[o] + reg[q] : reg[q];
    }
}

// 4 waves per SIMD: 128 VGPRs at most (16 voxels per thread)
template <typename Q, int A, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
__global__ __launch_bounds__(NT, 4) void adjoint_kernel(AdjParams p)
{
    __shared__ AdjLds<L, TS, TF, SLO, SHI, CPT, NT> sh;
    adjoint_block<Q, A, L, TS, TF, SLO, SHI, CPT, NT>(p, blockIdx.x, sh);
}

template <typename Q, int A, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
__global__ __launch_bounds__(NT, 4) void adjoint_batch_kernel(Batch<AdjParams> w)
{
    __shared__ AdjLds<L, TS, TF, SLO, SHI, CPT, NT> sh;
    const int i = batch_item(w, blockIdx.x);
    adjoint_block<Q, A, L, TS, TF, SLO, SHI, CPT, NT>(w.p[i], blockIdx.x - w.start[i], sh);
}

template <typename Q, int A, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
__global__ __launch_bounds__(NT, 4) void adjoint_table_kernel(Table<AdjParams> w)
{
    __shared__ AdjLds<L, TS, TF, SLO, SHI, CPT, NT> sh;
    const int i = table_item(w, blockIdx.x);
    adjoint_block<Q, A, L, TS, TF, SLO, SHI, CPT, NT>(w.p[i], blockIdx.x - w.start[i], sh);
}

// All passes of a 3-D adjoint in one launch: a workgroup owns one cubic
// block (B^3 voxels, in x, y, z block coordinates) and runs the passes
// present one after the other, each exactly as its own launch would (the
// first overwrites the block, later ones add to it, in axis order, so the
// result is bitwise that of one launch per pass).  One launch has one tail
// instead of one per pass, and a block's passes share its LDS.
template <typename Q, int B, int SLO, int SHI, int CPT, int NT>
__device__ __forceinline__ void adjoint_fused_block(const AdjFused &f, int blk, AdjLds<B, B, B, SLO, SHI, CPT, NT> &sh)
{
    const int bx = blk % f.nb[0];
    blk /= f.nb[0];
    const int by = blk % f.nb[1];
    blk /= f.nb[1];
    const int bz = blk % f.nb[2];
    const int b = blk / f.nb[2];
    bool first = true;
    // pass-local block index: ((b * blocks_a + ba) * blocks_s + bs) * blocks_f + bf
    if (f.pass[0].n_pass_views > 0) {  // a = x, f = y, s = z
        adjoint_block<Q, 0, B, B, B, SLO, SHI, CPT, NT>(
            f.pass[0], ((b * f.nb[0] + bx) * f.nb[2] + bz) * f.nb[1] + by, sh);
        first = false;
    }
    if (f.pass[1].n_pass_views > 0) {  // a = y, f = x, s = z
        if (!first) __syncthreads();   // the previous pass is done with the LDS block
        adjoint_block<Q, 1, B, B, B, SLO, SHI, CPT, NT>(
            f.pass[1], ((b * f.nb[1] + by) * f.nb[2] + bz) * f.nb[0] + bx, sh);
        first = false;
    }
    if (f.pass[2].n_pass_views > 0) {  // a = z, f = x, s = y
        if (!first) __syncthreads();
        adjoint_block<Q, 2, B, B, B, SLO, SHI, CPT, NT>(
            f.pass[2], ((b * f.nb[2] + bz) * f.nb[1] + by) * f.nb[0] + bx, sh);
    }
}

template <typename Q, int B, int SLO, int SHI, int CPT, int NT>
__global__ __launch_bounds__(NT, 4) void adjoint_fused_kernel(AdjFused f)
{
    __shared__ AdjLds<B, B, B, SLO, SHI, CPT, NT> sh;
    adjoint_fused_block<Q, B, SLO, SHI, CPT, NT>(f, blockIdx.x, sh);
}

template <typename Q, int B, int SLO, int SHI, int CPT, int NT>
__global__ __launch_bounds__(NT, 4) void adjoint_fused_table_kernel(Table<AdjFused> w)
{
    __shared__ AdjLds<B, B, B, SLO, SHI, CPT, NT> sh;
    const int i = table_item(w, blockIdx.x);
    adjoint_fused_block<Q, B, SLO, SHI, CPT, NT>(w.p[i], blockIdx.x - w.start[i], sh);
}

// ------------------------------------------------ back-projection --------

// Voxel-driven back-projection.  A workgroup owns a 16 x 16 x BZ block of
// voxels; each thread accumulates a column of BZ voxels along z in
// registers (one writer per voxel, no atomics).  Per view, the detector
// rectangle that the block's voxel centres project into (the projection of
// the block's corner box, widened by one tap) is staged into LDS, zero-
// filled outside the detector, so every bilinear tap is an unchecked LDS
// read; the next view's rectangle is loaded into registers while the
// current one is used.  The rectangles of up to 256 views are computed
// together, one view per thread, into an LDS table.  Rectangles larger than
// RCAP x CCAP fall back to bounds-checked gathers from the sinogram.
//
// Views whose projection does not depend on z (Pi_02 = Pi_22 = 0: orbits
// about z with detector columns parallel to z, such as the circular and
// helical trajectories) take a column path: W and u are constant along a
// column and v is linear in k, so the reciprocal of W, the distance weight
// and the horizontal tap address and weight are computed once per column
// and view, leaving one position, two LDS pair reads and the interpolation
// per voxel.
template <typename Q, typename O, int BZ, int RCAP, int CCAP>
__device__ __forceinline__ void backproject_block(const BpParams &p, const int bid)
{
    constexpr int BX = 16, BY = 16, CHUNK = 256;
    constexpr int NE = RCAP * CCAP;
    constexpr int PER = (NE + 255) / 256;
    __shared__ float s_det[2][NE];
    __shared__ int4 s_rect[CHUNK];
    const int t = threadIdx.x;
    const int nbx = (p.n[0] + BX - 1) / BX, nby = (p.n[1] + BY - 1) / BY, nbz = (p.n[2] + BZ - 1) / BZ;
    int blk = bid;
    const int bx = blk % nbx;
    blk /= nbx;
    const int by = blk % nby;
    blk /= nby;
    const int bz = blk % nbz;
    const int b = blk / nbz;
    const int i0 = bx * BX, j0 = by * BY, k0 = bz * BZ;
    const int i1 = min(i0 + BX, p.n[0]) - 1, j1 = min(j0 + BY, p.n[1]) - 1, k1 = min(k0 + BZ, p.n[2]) - 1;
    const int i = i0 + t % BX, j = j0 + t / BX;
    const bool own = i <= i1 && j <= j1;
    const float fi = static_cast<float>(i), fj = static_cast<float>(j), fk0 = static_cast<float>(k0);
    const Q *sino = static_cast<const Q *>(p.sino) + static_cast<int64_t>(b) * p.n_views * p.nv * p.nu;
    const float fnu = static_cast<float>(p.nu), fnv = static_cast<float>(p.nv);

    // detector rectangle of the block for one view, computed by one thread:
    // x = first column u0, y = first row v0, z = columns | rows << 16,
    // w = bit 0: some tap may be non-zero, bit 1: fits the LDS buffer
    auto rect_of = [&](int view) {
        const ViewTabF &tf = p.tabf[view];
        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float ci = static_cast<float>((c & 1) ? i1 : i0);
            const float cj = static_cast<float>((c & 2) ? j1 : j0);
            const float ck = static_cast<float>((c & 4) ? k1 : k0);
            const float U = fmaf(tf.Pi[0], ci, fmaf(tf.Pi[1], cj, fmaf(tf.Pi[2], ck, tf.Pi[3])));
            const float V = fmaf(tf.Pi[4], ci, fmaf(tf.Pi[5], cj, fmaf(tf.Pi[6], ck, tf.Pi[7])));
            const float Wc = fmaf(tf.Pi[8], ci, fmaf(tf.Pi[9], cj, fmaf(tf.Pi[10], ck, tf.Pi[11])));
            const float u = U / Wc, v = V / Wc;
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            vmin = fminf(vmin, v);
            vmax = fmaxf(vmax, v);
        }
        // voxel positions are clamped to [-1, n] (zero padding), so the
        // rectangle is clamped likewise; 0.01 px covers FP32 rounding
        umin = fminf(fmaxf(umin - 0.01f, -1.0f), fnu);
        umax = fminf(fmaxf(umax + 0.01f, -1.0f), fnu);
        vmin = fminf(fmaxf(vmin - 0.01f, -1.0f), fnv);
        vmax = fminf(fmaxf(vmax + 0.01f, -1.0f), fnv);
        const int u0 = static_cast<int>(floorf(umin)), v0 = static_cast<int>(floorf(vmin));
        const int nc = static_cast<int>(floorf(umax)) + 2 - u0, nr = static_cast<int>(floorf(vmax)) + 2 - v0;
        // entirely outside the detector: every tap is zero
        const bool any = !(umax <= -1.0f || umin >= fnu || vmax <= -1.0f || vmin >= fnv);
        const bool lds = nc <= CCAP && nr <= RCAP;
        return make_int4(u0, v0, nc | nr << 16, static_cast<int>(any) | static_cast<int>(lds) << 1);
    };
    auto rect_at = [&](int e) {
        const int4 r = s_rect[e];
        return make_int4(__builtin_amdgcn_readfirstlane(r.x), __builtin_amdgcn_readfirstlane(r.y),
                         __builtin_amdgcn_readfirstlane(r.z), __builtin_amdgcn_readfirstlane(r.w));
    };
    // the thread's elements of the LDS rectangle (row, column), fixed
    int rr[PER], cc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = t + 256 * q;
        rr[q] = e < NE ? e / CCAP : RCAP;
        cc[q] = e % CCAP;
    }
    float pre[PER];
    auto issue = [&](int view, const int4 &rc) {
        if ((rc.w & 3) != 3) return;
        const Q *img = sino + static_cast<int64_t>(view) * p.nv * p.nu;
        const int nc = rc.z & 0xffff, nr = rc.z >> 16;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int r = rc.y + rr[q], c = rc.x + cc[q];
            float v = 0.0f;
            if (rr[q] < nr && cc[q] < nc && static_cast<uint32_t>(r) < static_cast<uint32_t>(p.nv) &&
                static_cast<uint32_t>(c) < static_cast<uint32_t>(p.nu))
                v = to_f32(img[static_cast<int64_t>(r) * p.nu + c]);
            pre[q] = v;
        }
    };

    float acc[BZ];
#pragma unroll
    for (int z = 0; z < BZ; ++z) acc[z] = 0.0f;
    for (int c0 = 0; c0 < p.n_views; c0 += CHUNK) {
        const int cn = min(CHUNK, p.n_views - c0);
        // the previous chunk's table and rectangles are no longer read
        // (barrier at the end of its last view)
        if (t < cn) s_rect[t] = rect_of(c0 + t);
        __syncthreads();
        int4 cur = rect_at(0);
        issue(c0, cur);
        for (int vi = 0; vi < cn; ++vi) {
            const int view = c0 + vi, buf = vi & 1;
            if ((cur.w & 3) == 3) {
#pragma unroll
                for (int q = 0; q < PER; ++q)
                    if (t + 256 * q < NE) s_det[buf][t + 256 * q] = pre[q];
            }
            __syncthreads();  // staged rectangle visible; the other buffer is free
            const int4 now = cur;
            if (vi + 1 < cn) {
                cur = rect_at(vi + 1);
                issue(view + 1, cur);
            }
            if (own && (now.w & 1)) {
                const ViewTabF &tf = p.tabf[view];
                if (now.w & 2) {
                    const float uo = static_cast<float>(now.x), vo = static_cast<float>(now.y);
                    const int nc = now.z & 0xffff, nr = now.z >> 16;
                    const float hu = fminf(fnu - uo, static_cast<float>(nc - 1) - 1e-3f);
                    const float hv = fminf(fnv - vo, static_cast<float>(nr - 1) - 1e-3f);
                    const float lu = fmaxf(-1.0f - uo, 0.0f), lv = fmaxf(-1.0f - vo, 0.0f);
                    const float *det = s_det[buf];
                    if (BZ > 1 && tf.Pi[2] == 0.0f && tf.Pi[10] == 0.0f) {
                        // column path: u and W fixed, v linear in k
                        const float U0 = fmaf(tf.Pi[0], fi, fmaf(tf.Pi[1], fj, tf.Pi[3]));
                        const float V0 = fmaf(tf.Pi[4], fi, fmaf(tf.Pi[5], fj, fmaf(tf.Pi[6], fk0, tf.Pi[7])));
                        const float Wb = fmaf(tf.Pi[8], fi, fmaf(tf.Pi[9], fj, tf.Pi[11]));
                        const float rw = __builtin_amdgcn_rcpf(Wb);
                        const float u = __builtin_amdgcn_fmed3f(fmaf(U0, rw, -uo), lu, hu);
                        const float wu = __builtin_amdgcn_fractf(u);
                        const float *col = det + static_cast<int>(u);
                        const float dv = tf.Pi[6] * rw, v0 = fmaf(V0, rw, -vo);
                        const float w = tf.W0 * rw, w2 = w * w;
#pragma unroll
                        for (int z = 0; z < BZ; ++z) {
                            const float v = __builtin_amdgcn_fmed3f(fmaf(static_cast<float>(z), dv, v0), lv, hv);
                            const float wv = __builtin_amdgcn_fractf(v);
                            const float *q = col + __mul24(static_cast<int>(v), CCAP);
                            const float d00 = q[0], d01 = q[1], d10 = q[CCAP], d11 = q[CCAP + 1];
                            const float lo = fmaf(wu, d01 - d00, d00);
                            const float hi = fmaf(wu, d11 - d10, d10);
                            acc[z] = fmaf(w2, fmaf(wv, hi - lo, lo), acc[z]);
                        }
                    } else {
                        const float U0 = fmaf(tf.Pi[0], fi, fmaf(tf.Pi[1], fj, fmaf(tf.Pi[2], fk0, tf.Pi[3])));
                        const float V0 = fmaf(tf.Pi[4], fi, fmaf(tf.Pi[5], fj, fmaf(tf.Pi[6], fk0, tf.Pi[7])));
                        const float Wb = fmaf(tf.Pi[8], fi, fmaf(tf.Pi[9], fj, fmaf(tf.Pi[10], fk0, tf.Pi[11])));
#pragma unroll
                        for (int z = 0; z < BZ; ++z) {
                            const float fz = static_cast<float>(z);
                            const float rw = __builtin_amdgcn_rcpf(fmaf(fz, tf.Pi[10], Wb));
                            const float u = __builtin_amdgcn_fmed3f(fmaf(fmaf(fz, tf.Pi[2], U0), rw, -uo), lu, hu);
                            const float v = __builtin_amdgcn_fmed3f(fmaf(fmaf(fz, tf.Pi[6], V0), rw, -vo), lv, hv);
                            const float wu = __builtin_amdgcn_fractf(u), wv = __builtin_amdgcn_fractf(v);
                            const float *q = det + __mul24(static_cast<int>(v), CCAP) + static_cast<int>(u);
                            const float d00 = q[0], d01 = q[1], d10 = q[CCAP], d11 = q[CCAP + 1];
                            const float lo = fmaf(wu, d01 - d00, d00);
                            const float hi = fmaf(wu, d11 - d10, d10);
                            const float w = tf.W0 * rw;
                            acc[z] = fmaf(w * w, fmaf(wv, hi - lo, lo), acc[z]);
                        }
                    }
                } else {
                    const float U0 = fmaf(tf.Pi[0], fi, fmaf(tf.Pi[1], fj, fmaf(tf.Pi[2], fk0, tf.Pi[3])));
                    const float V0 = fmaf(tf.Pi[4], fi, fmaf(tf.Pi[5], fj, fmaf(tf.Pi[6], fk0, tf.Pi[7])));
                    const float Wb = fmaf(tf.Pi[8], fi, fmaf(tf.Pi[9], fj, fmaf(tf.Pi[10], fk0, tf.Pi[11])));
                    const Q *img = sino + static_cast<int64_t>(view) * p.nv * p.nu;
                    // a rolled loop: one voxel's gathers in flight keeps the
                    // register count of the LDS paths
#pragma unroll 1
                    for (int z = 0; z < BZ; ++z) {
                        const float fz = static_cast<float>(z);
                        const float Wc = fmaf(fz, tf.Pi[10], Wb);
                        const float rw = 1.0f / Wc;
                        const float u = fminf(fmaxf(fmaf(fz, tf.Pi[2], U0) * rw, -1.0f), fnu);
                        const float v = fminf(fmaxf(fmaf(fz, tf.Pi[6], V0) * rw, -1.0f), fnv);
                        const float fu = floorf(u), fv = floorf(v);
                        const float wu = u - fu, wv = v - fv;
                        const int iu = static_cast<int>(fu), iv = static_cast<int>(fv);
                        float d00 = 0.f, d01 = 0.f, d10 = 0.f, d11 = 0.f;
                        const bool c0 = iu >= 0 && iu < p.nu, c1 = iu + 1 < p.nu;
                        if (iv >= 0 && iv < p.nv) {
                            const Q *row = img + static_cast<int64_t>(iv) * p.nu;
                            if (c0) d00 = to_f32(row[iu]);
                            if (c1) d01 = to_f32(row[iu + 1]);
                        }
                        if (iv + 1 < p.nv) {
                            const Q *row = img + static_cast<int64_t>(iv + 1) * p.nu;
                            if (c0) d10 = to_f32(row[iu]);
                            if (c1) d11 = to_f32(row[iu + 1]);
                        }
                        const float lo = fmaf(wu, d01 - d00, d00);
                        const float hi = fmaf(wu, d11 - d10, d10);
                        const float w = tf.W0 * rw;
                        const float val = w * w * fmaf(wv, hi - lo, lo);
#pragma unroll
                        for (int zz = 0; zz < BZ; ++zz) acc[zz] += zz == z ? val : 0.0f;
                    }
                }
            }
            __syncthreads();  // every voxel is done with this view's rectangle
        }
    }
    if (!own) return;
    const int64_t item = static_cast<int64_t>(p.n[0]) * p.n[1] * p.n[2];
    O *out = static_cast<O *>(p.vol) + b * item;
#pragma unroll
    for (int z = 0; z < BZ; ++z) {
        const int k = k0 + z;
        if (k <= k1) out[(static_cast<int64_t>(k) * p.n[1] + j) * p.n[0] + i] = from_f32<O>(acc[z]);
    }
}

// 8 waves per SIMD: 64 VGPRs at most
template <typename Q, typename O, int BZ, int RCAP, int CCAP>
__global__ __launch_bounds__(256, BZ > 16 ? 4 : 8) void backproject_kernel(BpParams p)
{
    backproject_block<Q, O, BZ, RCAP, CCAP>(p, blockIdx.x);
}

template <typename Q, typename O, int BZ, int RCAP, int CCAP>
__global__ __launch_bounds__(256, 8) void backproject_batch_kernel(Batch<BpParams> w)
{
    const int i = batch_item(w, blockIdx.x);
    backproject_block<Q, O, BZ, RCAP, CCAP>(w.p[i], blockIdx.x - w.start[i]);
}

template <typename Q, typename O, int BZ, int RCAP, int CCAP>
__global__ __launch_bounds__(256, 8) void backproject_table_kernel(Table<BpParams> w)
{
    const int i = table_item(w, blockIdx.x);
    backproject_block<Q, O, BZ, RCAP, CCAP>(w.p[i], blockIdx.x - w.start[i]);
}

// ------------------------------------------------------ splat (BP^T) ----

// Two 32-bit fixed-point cells in one 64-bit LDS word, added with one
// ds_add_u64: the word holds lo + 2^32 hi as a signed 64-bit integer, so a
// sum of such words is (sum lo) + 2^32 (sum hi) exactly; while both sums
// stay inside (-2^31, 2^31) the halves are recovered as the low word read as
// signed and the rest shifted down.
__device__ __forceinline__ unsigned long long pair_word(int lo, int hi)
{
    return (static_cast<unsigned long long>(static_cast<uint32_t>(hi + (lo >> 31))) << 32) |
           static_cast<uint32_t>(lo);
}
__device__ __forceinline__ int lo_half(unsigned long long w) { return static_cast<int>(static_cast<uint32_t>(w)); }
__device__ __forceinline__ int hi_half(unsigned long long w)
{
    const long long sw = static_cast<long long>(w);
    return static_cast<int>((sw - lo_half(w)) >> 32);
}

// Transpose of the voxel-driven back-projection: every voxel's value times
// the distance weight (W0/W)^2 is spread over the bilinear taps of its
// projection in each view; taps off the detector are dropped.  A workgroup
// owns the same 16 x 16 x BZ block as the back-projection, its values in
// registers (a z-column of BZ voxels per thread).  Per view, the block's
// deposits collect in an LDS copy of the detector rectangle the block
// projects into (the back-projection's rectangle), as 32-bit fixed point
// with one power-of-two scale per view: the block's sum of |x| times the
// view's largest weight (W0 / min W over the block's corners)^2 stays below
// 2^30, so no cell's sum can overflow; the error of a deposit is at most
// 2^-31 of that bound: relative to the block's mass, not to its largest
// value times its voxel count.  Integer adds are exact, so the
// rectangle is independent of the order of the deposits.  The rectangle is
// then added to the FP32 sinogram with one hardware float atomic per non-zero
// pixel, which a pixel receives from every block along its ray: the result
// is not bitwise reproducible (the order of those adds varies).  The cells
// of rows r and r + 1 of a column share one 64-bit word (pair_word), so a
// deposit is two ds_add_u64 instead of four ds_add_u32, and a cell is the
// low half of its word plus the high half of the word above.  Three LDS
// rectangles rotate between views, one barrier per view: a view's rectangle
// is flushed after its barrier and cleared after the next one.  Rectangles
// larger than RCAP x CCAP, and blocks holding a non-finite value, deposit
// straight into the sinogram with one float atomic per tap.
template <typename S, int BZ, int RCAP, int CCAP>
__device__ __forceinline__ void splat_block(const SplatParams &p, const int bid)
{
    constexpr int BX = 16, BY = 16, CHUNK = 256;
    constexpr int NE = RCAP * CCAP;
    constexpr int PER = (NE + 255) / 256;
    __shared__ unsigned long long s_acc[3][NE];
    __shared__ int4 s_rect[CHUNK];
    __shared__ float s_scale[CHUNK];
    __shared__ uint32_t s_max[4];
    __shared__ float s_sum[4];
    const int t = threadIdx.x;
    const int nbx = (p.n[0] + BX - 1) / BX, nby = (p.n[1] + BY - 1) / BY, nbz = (p.n[2] + BZ - 1) / BZ;
    int blk = bid;
    const int bx = blk % nbx;
    blk /= nbx;
    const int by = blk % nby;
    blk /= nby;
    const int bz = blk % nbz;
    const int b = blk / nbz;
    const int i0 = bx * BX, j0 = by * BY, k0 = bz * BZ;
    const int i1 = min(i0 + BX, p.n[0]) - 1, j1 = min(j0 + BY, p.n[1]) - 1, k1 = min(k0 + BZ, p.n[2]) - 1;
    const int i = i0 + t % BX, j = j0 + t / BX;
    const bool own = i <= i1 && j <= j1;
    const float fi = static_cast<float>(i), fj = static_cast<float>(j), fk0 = static_cast<float>(k0);
    const float fnu = static_cast<float>(p.nu), fnv = static_cast<float>(p.nv);
    float *sino = p.sino + static_cast<int64_t>(b) * p.n_views * p.nv * p.nu;

    // the thread's voxel values, the block's max |x| and its sum of |x|.
    // Register z of a thread holds the voxel at height (z + skew) mod BZ of
    // its column, the skew varying with i and j: voxels on one ray (along x,
    // y or a diagonal) that the lanes of a wave deposit in the same step then
    // sit at different heights, so their taps fall on different detector
    // rows rather than on one LDS cell (same-address atomics serialise).
    // Neighbours along x differ by 3 heights and along y by 5 (about 2.4
    // and 4 detector rows at a magnification near 1), and with the odd row
    // stride of the rectangle the lanes' cells spread over the LDS banks.
    static_assert((BZ & (BZ - 1)) == 0, "power-of-two column");
    const int skew = (3 * i + 5 * j) & (BZ - 1);
    float x[BZ];
    uint32_t mbits = 0u;
    float asum = 0.0f;
    const S *vol = static_cast<const S *>(p.vol) + static_cast<int64_t>(b) * p.n[0] * p.n[1] * static_cast<int64_t>(p.n[2]);
#pragma unroll
    for (int z = 0; z < BZ; ++z) {
        const int k = k0 + ((z + skew) & (BZ - 1));
        x[z] = (own && k <= k1) ? to_f32(vol[(static_cast<int64_t>(k) * p.n[1] + j) * p.n[0] + i]) : 0.0f;
        mbits = max(mbits, __float_as_uint(fabsf(x[z])));
        asum += fabsf(x[z]);
    }
    mbits = wave_max_u32(mbits);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) asum += __shfl_xor(asum, o);
    if ((t & 63) == 0) {
        s_max[t >> 6] = mbits;
        s_sum[t >> 6] = asum;
    }
    for (int e = t; e < 3 * NE; e += 256) s_acc[e / NE][e % NE] = 0ull;
    __syncthreads();
    mbits = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
    if (mbits == 0u) return;                       // nothing to deposit (uniform)
    const float xsum = (s_sum[0] + s_sum[1]) + (s_sum[2] + s_sum[3]);
    // else (a non-finite value, or a sum beyond FP32): straight float atomics
    const bool finite = mbits < 0x7f800000u && xsum <= 3.0e38f;

    // detector rectangle and fixed-point scale of the block for one view
    auto rect_of = [&](int view, float &scale) {
        const ViewTabF &tf = p.tabf[view];
        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, wmin = INFINITY;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float ci = static_cast<float>((c & 1) ? i1 : i0);
            const float cj = static_cast<float>((c & 2) ? j1 : j0);
            const float ck = static_cast<float>((c & 4) ? k1 : k0);
            const float U = fmaf(tf.Pi[0], ci, fmaf(tf.Pi[1], cj, fmaf(tf.Pi[2], ck, tf.Pi[3])));
            const float V = fmaf(tf.Pi[4], ci, fmaf(tf.Pi[5], cj, fmaf(tf.Pi[6], ck, tf.Pi[7])));
            const float Wc = fmaf(tf.Pi[8], ci, fmaf(tf.Pi[9], cj, fmaf(tf.Pi[10], ck, tf.Pi[11])));
            const float u = U / Wc, v = V / Wc;
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            vmin = fminf(vmin, v);
            vmax = fmaxf(vmax, v);
            wmin = fminf(wmin, Wc);
        }
        umin = fminf(fmaxf(umin - 0.01f, -1.0f), fnu);
        umax = fminf(fmaxf(umax + 0.01f, -1.0f), fnu);
        vmin = fminf(fmaxf(vmin - 0.01f, -1.0f), fnv);
        vmax = fminf(fmaxf(vmax + 0.01f, -1.0f), fnv);
        const int u0 = static_cast<int>(floorf(umin)), v0 = static_cast<int>(floorf(vmin));
        const int nc = static_cast<int>(floorf(umax)) + 2 - u0, nr = static_cast<int>(floorf(vmax)) + 2 - v0;
        const bool any = !(umax <= -1.0f || umin >= fnu || vmax <= -1.0f || vmin >= fnv);
        const bool lds = finite && nc <= CCAP && nr <= RCAP;
        // bound of a rectangle cell's sum: a voxel deposits into a cell at
        // most once per view, with a tap weight <= 1, so no cell exceeds the
        // block's sum of |x| (W0/W)^2 (a corner's W is the smallest over the
        // convex block; 1% slack for the FP32 sums)
        const float w0 = tf.W0 / wmin;
        const float bound = xsum * w0 * w0 * 1.01f;
        const int e = min(126, max(-126, 30 - __builtin_amdgcn_frexp_expf(bound)));
        scale = exp2f(static_cast<float>(e));
        return make_int4(u0, v0, nc | nr << 16, static_cast<int>(any) | static_cast<int>(lds) << 1);
    };
    auto rect_at = [&](int e) {
        const int4 r = s_rect[e];
        return make_int4(__builtin_amdgcn_readfirstlane(r.x), __builtin_amdgcn_readfirstlane(r.y),
                         __builtin_amdgcn_readfirstlane(r.z), __builtin_amdgcn_readfirstlane(r.w));
    };
    // deposits the rectangle of view `view` (buffer buf) into the sinogram:
    // cell (r, c) is the low half of word (r, c) plus the high half of word
    // (r - 1, c).  The words read one view earlier (buffer pbuf, if that view
    // used the LDS) are cleared now: every thread has read them (barrier
    // since), and that buffer is next written two views later.
    auto flush = [&](int view, const int4 &rc, float inv, int buf, bool plds, int pbuf) {
        if (plds) {
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int e = t + 256 * q;
                if (e < NE) s_acc[pbuf][e] = 0ull;
            }
        }
        if ((rc.w & 3) != 3) return;
        const int nc = rc.z & 0xffff, nr = rc.z >> 16;
        float *img = sino + static_cast<int64_t>(view) * p.nv * p.nu;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q;
            if (e >= NE) break;
            const int rr = e / CCAP, cc = e - rr * CCAP;
            int v = lo_half(s_acc[buf][e]);
            if (rr > 0) v += hi_half(s_acc[buf][e - CCAP]);
            if (v == 0) continue;
            const int r = rc.y + rr, c = rc.x + cc;
            if (rr < nr && cc < nc && static_cast<uint32_t>(r) < static_cast<uint32_t>(p.nv) &&
                static_cast<uint32_t>(c) < static_cast<uint32_t>(p.nu))
                unsafeAtomicAdd(img + static_cast<int64_t>(r) * p.nu + c, static_cast<float>(v) * inv);
        }
    };

    bool plds = false;  // the previous view deposited into the LDS
    for (int c0 = 0; c0 < p.n_views; c0 += CHUNK) {
        const int cn = min(CHUNK, p.n_views - c0);
        __syncthreads();  // the previous chunk's table is no longer read
        if (t < cn) {
            float sc;
            s_rect[t] = rect_of(c0 + t, sc);
            s_scale[t] = sc;
        }
        __syncthreads();
        for (int vi = 0; vi < cn; ++vi) {
            const int view = c0 + vi, buf = view % 3;
            const int4 now = rect_at(vi);
            const float scale = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(s_scale[vi])));
            if (own && (now.w & 1)) {
                // the view's table entries, uniform over the workgroup, held in
                // scalar registers (one load per view, none per deposit)
                const ViewTabF &tf = p.tabf[view];
                float pi[12];
#pragma unroll
                for (int m = 0; m < 12; ++m) pi[m] = uniform_f32(tf.Pi[m]);
                const float W0 = uniform_f32(tf.W0);
                const float uo = static_cast<float>(now.x), vo = static_cast<float>(now.y);
                const int nc = now.z & 0xffff, nr = now.z >> 16;
                float *img = sino + static_cast<int64_t>(view) * p.nv * p.nu;
                const float U0 = fmaf(pi[0], fi, fmaf(pi[1], fj, fmaf(pi[2], fk0, pi[3])));
                const float V0 = fmaf(pi[4], fi, fmaf(pi[5], fj, fmaf(pi[6], fk0, pi[7])));
                const float Wb = fmaf(pi[8], fi, fmaf(pi[9], fj, fmaf(pi[10], fk0, pi[11])));
                // height (z + skew) mod BZ of register z as 16 fract(skew/BZ +
                // z/BZ): the sum is exact (multiples of 1/BZ below 2), so is the
                // fraction, and the factor BZ is folded into the coefficients
                // it multiplies (exact power-of-two scaling)
                const float fsk = static_cast<float>(skew) * (1.0f / BZ);
                auto height = [&](int z) { return __builtin_amdgcn_fractf(fsk + static_cast<float>(z) * (1.0f / BZ)); };
                if (now.w & 2) {
                    // positions relative to the rectangle, clamped to it as in
                    // the back-projection (a clamped position deposits only
                    // off the detector, which the flush drops)
                    const float hu = fminf(fnu - uo, static_cast<float>(nc - 1) - 1e-3f);
                    const float hv = fminf(fnv - vo, static_cast<float>(nr - 1) - 1e-3f);
                    const float lu = fmaxf(-1.0f - uo, 0.0f), lv = fmaxf(-1.0f - vo, 0.0f);
                    const float wsc = W0 * W0 * scale;
                    unsigned long long *acc = s_acc[buf];
                    if (BZ > 1 && pi[2] == 0.0f && pi[10] == 0.0f) {
                        // column path, the back-projection's: u and W fixed,
                        // v linear in the height
                        const float Uc = fmaf(pi[0], fi, fmaf(pi[1], fj, pi[3]));
                        const float Wc = fmaf(pi[8], fi, fmaf(pi[9], fj, pi[11]));
                        const float rw = __builtin_amdgcn_rcpf(Wc);
                        const float u = __builtin_amdgcn_fmed3f(fmaf(Uc, rw, -uo), lu, hu);
                        const float wu = __builtin_amdgcn_fractf(u);
                        const int cu = static_cast<int>(u);
                        const float dv = pi[6] * rw, v0 = fmaf(V0, rw, -vo);
                        const float dvb = dv * static_cast<float>(BZ);
                        const float w2 = rw * rw * wsc;
#pragma unroll
                        for (int z = 0; z < BZ; ++z) {
                            if (x[z] == 0.0f) continue;
                            const float v = __builtin_amdgcn_fmed3f(fmaf(height(z), dvb, v0), lv, hv);
                            const float wv = __builtin_amdgcn_fractf(v);
                            const float qs = x[z] * w2;
                            const float t1 = qs * wv, t0 = qs - t1;
                            const float c01 = t0 * wu, c11 = t1 * wu;
                            unsigned long long *q = acc + (__mul24(static_cast<int>(v), CCAP) + cu);
                            atomicAdd(q, pair_word(round_fixed(t0 - c01), round_fixed(t1 - c11)));
                            atomicAdd(q + 1, pair_word(round_fixed(c01), round_fixed(c11)));
                        }
                    } else {
                        const float p2 = pi[2] * static_cast<float>(BZ), p6 = pi[6] * static_cast<float>(BZ);
                        const float p10 = pi[10] * static_cast<float>(BZ);
#pragma unroll
                        for (int z = 0; z < BZ; ++z) {
                            if (x[z] == 0.0f) continue;
                            const float hz = height(z);
                            const float rw = __builtin_amdgcn_rcpf(fmaf(hz, p10, Wb));
                            const float u = __builtin_amdgcn_fmed3f(fmaf(fmaf(hz, p2, U0), rw, -uo), lu, hu);
                            const float v = __builtin_amdgcn_fmed3f(fmaf(fmaf(hz, p6, V0), rw, -vo), lv, hv);
                            const float wu = __builtin_amdgcn_fractf(u), wv = __builtin_amdgcn_fractf(v);
                            const float qs = x[z] * (rw * rw * wsc);
                            const float t1 = qs * wv, t0 = qs - t1;
                            const float c01 = t0 * wu, c11 = t1 * wu;
                            unsigned long long *q = acc + (__mul24(static_cast<int>(v), CCAP) + static_cast<int>(u));
                            atomicAdd(q, pair_word(round_fixed(t0 - c01), round_fixed(t1 - c11)));
                            atomicAdd(q + 1, pair_word(round_fixed(c01), round_fixed(c11)));
                        }
                    }
                } else {
                    // straight to the sinogram, bounds-checked, one atomic per tap
#pragma unroll 1
                    for (int z = 0; z < BZ; ++z) {
                        if (x[z] == 0.0f) continue;
                        const float fz = static_cast<float>((z + skew) & (BZ - 1));
                        const float Wz = fmaf(fz, pi[10], Wb);
                        const float rw = 1.0f / Wz;
                        const float u = fminf(fmaxf(fmaf(fz, pi[2], U0) * rw, -2.0f), fnu + 1.0f);
                        const float v = fminf(fmaxf(fmaf(fz, pi[6], V0) * rw, -2.0f), fnv + 1.0f);
                        const float fu = floorf(u), fv = floorf(v);
                        const float wu = u - fu, wv = v - fv;
                        const int iu = static_cast<int>(fu), iv = static_cast<int>(fv);
                        const float w = W0 * rw;
                        const float val = x[z] * w * w;
#pragma unroll
                        for (int tv = 0; tv < 2; ++tv) {
                            const int r = iv + tv;
                            if (r < 0 || r >= p.nv) continue;
                            const float a = (tv ? wv : 1.0f - wv) * val;
#pragma unroll
                            for (int tu = 0; tu < 2; ++tu) {
                                const int c = iu + tu;
                                if (c < 0 || c >= p.nu) continue;
                                unsafeAtomicAdd(img + static_cast<int64_t>(r) * p.nu + c, (tu ? wu : 1.0f - wu) * a);
                            }
                        }
                    }
                }
            }
            __syncthreads();  // this view's deposits are complete
            // flush this view's rectangle now and clear the previous view's;
            // the next view deposits into the third buffer
            flush(view, now, 1.0f / scale, buf, plds, (view + 2) % 3);
            plds = (now.w & 3) == 3;
        }
    }
}

template <typename S, int BZ, int RCAP, int CCAP>
__global__ __launch_bounds__(256, 6) void splat_kernel(SplatParams p)
{
    splat_block<S, BZ, RCAP, CCAP>(p, blockIdx.x);
}

// ------------------------------------------------------- utilities -------

__global__ __launch_bounds__(256) void fill_zero_kernel(uint32_t *__restrict__ dst, int64_t n_words)
{
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n_words;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[e] = 0u;
}

__global__ void fill_zero_bytes_kernel(uint8_t *__restrict__ dst, int32_t n)
{
    if (static_cast<int32_t>(threadIdx.x) < n) dst[threadIdx.x] = 0u;
}

template <typename O>
__global__ __launch_bounds__(256) void convert_kernel(const float *__restrict__ src, O *__restrict__ dst, int64_t n)
{
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[e] = from_f32<O>(src[e]);
}

// ----------------------------------------------------------- launchers ---

template <typename S>
static hipError_t relayout_t(const void *in, void *out, const int32_t n[3], int axis, int32_t batch, int64_t item,
                             int32_t row, int64_t plane, hipStream_t st)
{
    // grid.z carries (item, z); launch in batch chunks so that it stays <= 65535
    const int32_t chunk = n[2] > 65535 ? 1 : 65535 / n[2];
    for (int32_t b0 = 0; b0 < batch; b0 += chunk) {
        const int32_t nb = batch - b0 < chunk ? batch - b0 : chunk;
        const S *src = static_cast<const S *>(in) + static_cast<int64_t>(b0) * n[0] * n[1] * static_cast<int64_t>(n[2]);
        S *dst = static_cast<S *>(out) + b0 * item;
        if (axis == 0) {
            dim3 grid((n[0] + 31) / 32, (n[1] + 31) / 32, n[2] * nb);
            relayout_x_kernel<S><<<grid, 256, 0, st>>>(src, dst, n[0], n[1], n[2], item, row, plane);
        } else {
            dim3 grid((n[0] + 255) / 256, n[1], n[2] * nb);
            relayout_rows_kernel<S><<<grid, 256, 0, st>>>(src, dst, n[0], n[1], n[2], axis, item, row, plane);
        }
    }
    return hipGetLastError();
}

hipError_t launch_relayout(int32_t dtype, const void *in, void *out, const int32_t n[3], int axis, int32_t batch,
                           int64_t item, int32_t row, int64_t plane, hipStream_t st)
{
    switch (dtype) {
    case DT_F32: return relayout_t<float>(in, out, n, axis, batch, item, row, plane, st);
    case DT_BF16: return relayout_t<bf16>(in, out, n, axis, batch, item, row, plane, st);
    default: return relayout_t<f16>(in, out, n, axis, batch, item, row, plane, st);
    }
}

// 3-D forward: 16 x 16 pixel tiles of kFwdViews consecutive views, chunks of
// 4 planes; 2-D: 256-pixel rows of one view, chunks of 4 planes
constexpr int kFwdViews = 3;

int64_t forward_blocks(const FwdParams &p)
{
    const int64_t tiles = static_cast<int64_t>(p.tiles_u) * p.tiles_v;
    const int64_t groups = (p.n_views + p.view_group - 1) / p.view_group;
    return 8 * ((tiles + 7) / 8) * groups * p.batch;
}

// Launch dispatch: a single problem passes its parameters, a batch its work
// list; the kernel templates are the same.
template <typename S, typename O, int TU, int TV, int C, int RCAP, int FCAP, int NVW>
static void fwd_go(const FwdParams &p, uint32_t blocks, hipStream_t st)
{
    forward_kernel<S, O, TU, TV, C, RCAP, FCAP, NVW><<<dim3(blocks), 256, 0, st>>>(p);
}
template <typename S, typename O, int TU, int TV, int C, int RCAP, int FCAP, int NVW>
static void fwd_go(const Batch<FwdParams> &w, uint32_t blocks, hipStream_t st)
{
    forward_batch_kernel<S, O, TU, TV, C, RCAP, FCAP, NVW><<<dim3(blocks), 256, 0, st>>>(w);
}
template <typename S, typename O, int TU, int TV, int C, int RCAP, int FCAP, int NVW>
static void fwd_go(const Table<FwdParams> &w, uint32_t blocks, hipStream_t st)
{
    forward_table_kernel<S, O, TU, TV, C, RCAP, FCAP, NVW><<<dim3(blocks), 256, 0, st>>>(w);
}

// views per 3-D workgroup: a single call may take a tuned group of 2, work
// lists always use the default
template <typename S, typename O, typename Arg>
static hipError_t forward_t(const Arg &a, bool two_d, uint32_t blocks, hipStream_t st)
{
    if (two_d)
        fwd_go<S, O, 256, 1, 4, 3, 320, 1>(a, blocks, st);
    else if constexpr (std::is_same<Arg, FwdParams>::value) {
        if (a.view_group == 2) fwd_go<S, O, 16, 16, 4, 24, 40, 2>(a, blocks, st);
        else fwd_go<S, O, 16, 16, 4, 24, 40, kFwdViews>(a, blocks, st);
    } else {
        fwd_go<S, O, 16, 16, 4, 24, 40, kFwdViews>(a, blocks, st);
    }
    return hipGetLastError();
}

template <typename S, typename Arg>
static hipError_t forward_s(const Arg &a, bool two_d, uint32_t blocks, int32_t out_dt, hipStream_t st)
{
    switch (out_dt) {
    case DT_F32: return forward_t<S, float>(a, two_d, blocks, st);
    case DT_BF16: return forward_t<S, bf16>(a, two_d, blocks, st);
    default: return forward_t<S, f16>(a, two_d, blocks, st);
    }
}

template <typename Arg>
static hipError_t forward_any(const Arg &a, bool two_d, uint32_t blocks, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    switch (in_dt) {
    case DT_F32: return forward_s<float>(a, two_d, blocks, out_dt, st);
    case DT_BF16: return forward_s<bf16>(a, two_d, blocks, out_dt, st);
    default: return forward_s<f16>(a, two_d, blocks, out_dt, st);
    }
}

hipError_t launch_forward(const FwdParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    return forward_any(p, p.tile_v == 1, static_cast<uint32_t>(forward_blocks(p)), in_dt, out_dt, st);
}

hipError_t launch_forward_batch(const Batch<FwdParams> &w, bool two_d, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    return forward_any(w, two_d, w.start[w.n], in_dt, out_dt, st);
}

void forward_tile_shape(bool two_d, int32_t &tu, int32_t &tv, int32_t &views)
{
    if (two_d) { tu = 256; tv = 1; views = 1; }
    else { tu = 16; tv = 16; views = kFwdViews; }
}

// Compiled adjoint block shapes (planes x rows x columns, candidates per
// thread per batch); index 0 is 2-D; shape 3 runs 512 threads.
static const int32_t kAdjShapes[][4] = {{32, 1, 64, 1}, {16, 16, 16, 2}, {32, 8, 16, 1}, {16, 16, 32, 1},
                                        {32, 16, 16, 1}};
constexpr int kNumAdjShapes = 5;

int adjoint_shape_count() { return kNumAdjShapes; }

void adjoint_shape(int id, int32_t &L, int32_t &TS, int32_t &TF)
{
    L = kAdjShapes[id][0];
    TS = kAdjShapes[id][1];
    TF = kAdjShapes[id][2];
}

int64_t adjoint_blocks(const AdjParams &p)
{
    return static_cast<int64_t>(p.blocks_a) * p.blocks_s * p.blocks_f * p.batch;
}

template <typename Q, int A, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
static void adj_go(const AdjParams &p, uint32_t blocks, hipStream_t st)
{
    adjoint_kernel<Q, A, L, TS, TF, SLO, SHI, CPT, NT><<<dim3(blocks), NT, 0, st>>>(p);
}
template <typename Q, int A, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
static void adj_go(const Batch<AdjParams> &w, uint32_t blocks, hipStream_t st)
{
    adjoint_batch_kernel<Q, A, L, TS, TF, SLO, SHI, CPT, NT><<<dim3(blocks), NT, 0, st>>>(w);
}
template <typename Q, int A, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT>
static void adj_go(const Table<AdjParams> &w, uint32_t blocks, hipStream_t st)
{
    adjoint_table_kernel<Q, A, L, TS, TF, SLO, SHI, CPT, NT><<<dim3(blocks), NT, 0, st>>>(w);
}

template <typename Q, int L, int TS, int TF, int SLO, int SHI, int CPT, int NT, typename Arg>
static hipError_t adjoint_axes(const Arg &a, int axis, uint32_t blocks, hipStream_t st)
{
    switch (axis) {
    case 0: adj_go<Q, 0, L, TS, TF, SLO, SHI, CPT, NT>(a, blocks, st); break;
    case 1: adj_go<Q, 1, L, TS, TF, SLO, SHI, CPT, NT>(a, blocks, st); break;
    default:
        if constexpr (TS == 1) {
            return hipErrorInvalidValue;  // 2-D rays never have z dominant
        } else {
            adj_go<Q, 2, L, TS, TF, SLO, SHI, CPT, NT>(a, blocks, st);
        }
        break;
    }
    return hipGetLastError();
}

template <typename Q, typename Arg>
static hipError_t adjoint_q(const Arg &a, int axis, int shape, uint32_t blocks, hipStream_t st)
{
    switch (shape) {
    case 0: return adjoint_axes<Q, 32, 1, 64, 0, 1, 1, 256>(a, axis, blocks, st);
    case 1: return adjoint_axes<Q, 16, 16, 16, 1, 2, 2, 256>(a, axis, blocks, st);
    case 2: return adjoint_axes<Q, 32, 8, 16, 1, 2, 1, 256>(a, axis, blocks, st);
    case 3: return adjoint_axes<Q, 16, 16, 32, 1, 2, 1, 512>(a, axis, blocks, st);
    default: return adjoint_axes<Q, 32, 16, 16, 1, 2, 1, 512>(a, axis, blocks, st);
    }
}

template <typename Arg>
static hipError_t adjoint_any(const Arg &a, int axis, int32_t in_dt, int shape, uint32_t blocks, hipStream_t st)
{
    switch (in_dt) {
    case DT_F32: return adjoint_q<float>(a, axis, shape, blocks, st);
    case DT_BF16: return adjoint_q<bf16>(a, axis, shape, blocks, st);
    default: return adjoint_q<f16>(a, axis, shape, blocks, st);
    }
}

hipError_t launch_adjoint(const AdjParams &p, int32_t in_dt, int shape, hipStream_t st)
{
    return adjoint_any(p, p.axis, in_dt, shape, static_cast<uint32_t>(adjoint_blocks(p)), st);
}

bool adjoint_fusable(bool two_d, int shape) { return !two_d && shape == 1; }

hipError_t launch_adjoint_fused(const AdjFused &f, int32_t in_dt, hipStream_t st)
{
    const int64_t blocks = static_cast<int64_t>(f.nb[0]) * f.nb[1] * f.nb[2] * f.batch;
    if (blocks == 0) return hipSuccess;
    const dim3 grid(static_cast<uint32_t>(blocks));
    switch (in_dt) {
    case DT_F32: adjoint_fused_kernel<float, 16, 1, 2, 2, 256><<<grid, 256, 0, st>>>(f); break;
    case DT_BF16: adjoint_fused_kernel<bf16, 16, 1, 2, 2, 256><<<grid, 256, 0, st>>>(f); break;
    default: adjoint_fused_kernel<f16, 16, 1, 2, 2, 256><<<grid, 256, 0, st>>>(f); break;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_batch(const Batch<AdjParams> &w, int axis, int32_t in_dt, int shape, hipStream_t st)
{
    return adjoint_any(w, axis, in_dt, shape, w.start[w.n], st);
}

// 3-D back-projection: voxel columns of kBpDepth along z, detector
// rectangles of up to kBpRows x kBpCols pixels in LDS
constexpr int kBpDepth = 16, kBpRows = 20, kBpCols = 24;

static int bp_depth(const BpParams &p) { return p.bz == 8 || p.bz == 32 ? p.bz : kBpDepth; }

int64_t backproject_blocks(const BpParams &p)
{
    if (p.n[2] == 1) return static_cast<int64_t>((p.n[0] + 15) / 16) * ((p.n[1] + 15) / 16) * p.batch;
    const int bz = bp_depth(p);
    return static_cast<int64_t>((p.n[0] + 15) / 16) * ((p.n[1] + 15) / 16) * ((p.n[2] + bz - 1) / bz) * p.batch;
}

template <typename Q, typename O, int BZ, int RCAP, int CCAP>
static void bp_go(const BpParams &p, uint32_t blocks, hipStream_t st)
{
    backproject_kernel<Q, O, BZ, RCAP, CCAP><<<dim3(blocks), 256, 0, st>>>(p);
}
template <typename Q, typename O, int BZ, int RCAP, int CCAP>
static void bp_go(const Batch<BpParams> &w, uint32_t blocks, hipStream_t st)
{
    backproject_batch_kernel<Q, O, BZ, RCAP, CCAP><<<dim3(blocks), 256, 0, st>>>(w);
}
template <typename Q, typename O, int BZ, int RCAP, int CCAP>
static void bp_go(const Table<BpParams> &w, uint32_t blocks, hipStream_t st)
{
    backproject_table_kernel<Q, O, BZ, RCAP, CCAP><<<dim3(blocks), 256, 0, st>>>(w);
}

template <typename Q, typename O, typename Arg>
static hipError_t bp_t(const Arg &a, bool two_d, uint32_t blocks, hipStream_t st)
{
    if (two_d) {
        bp_go<Q, O, 1, 4, 64>(a, blocks, st);
    } else if constexpr (std::is_same<Arg, BpParams>::value) {
        // a single call may take a tuned block depth (rectangles of 20 rows
        // hold a 16-voxel column's projection; 36 a 32-voxel one)
        switch (bp_depth(a)) {
        case 8: bp_go<Q, O, 8, kBpRows, kBpCols>(a, blocks, st); break;
        case 32: bp_go<Q, O, 32, 36, kBpCols>(a, blocks, st); break;
        default: bp_go<Q, O, kBpDepth, kBpRows, kBpCols>(a, blocks, st); break;
        }
    } else {
        bp_go<Q, O, kBpDepth, kBpRows, kBpCols>(a, blocks, st);
    }
    return hipGetLastError();
}

template <typename Q, typename Arg>
static hipError_t bp_q(const Arg &a, bool two_d, uint32_t blocks, int32_t out_dt, hipStream_t st)
{
    switch (out_dt) {
    case DT_F32: return bp_t<Q, float>(a, two_d, blocks, st);
    case DT_BF16: return bp_t<Q, bf16>(a, two_d, blocks, st);
    default: return bp_t<Q, f16>(a, two_d, blocks, st);
    }
}

template <typename Arg>
static hipError_t bp_any(const Arg &a, bool two_d, uint32_t blocks, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    switch (in_dt) {
    case DT_F32: return bp_q<float>(a, two_d, blocks, out_dt, st);
    case DT_BF16: return bp_q<bf16>(a, two_d, blocks, out_dt, st);
    default: return bp_q<f16>(a, two_d, blocks, out_dt, st);
    }
}

hipError_t launch_backproject(const BpParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st)
{
    return bp_any(p, p.n[2] == 1, static_cast<uint32_t>(backproject_blocks(p)), in_dt, out_dt, st);
}

hipError_t launch_backproject_batch(const Batch<BpParams> &w, bool two_d, int32_t in_dt, int32_t out_dt,
                                    hipStream_t st)
{
    return bp_any(w, two_d, w.start[w.n], in_dt, out_dt, st);
}

// Launchers of device-memory work lists (`blocks`: the list's workgroups).
hipError_t launch_forward_table(const Table<FwdParams> &w, uint32_t blocks, bool two_d, int32_t in_dt,
                                int32_t out_dt, hipStream_t st)
{
    return forward_any(w, two_d, blocks, in_dt, out_dt, st);
}

hipError_t launch_adjoint_table(const Table<AdjParams> &w, uint32_t blocks, int axis, int32_t in_dt, int shape,
                                hipStream_t st)
{
    return adjoint_any(w, axis, in_dt, shape, blocks, st);
}

hipError_t launch_adjoint_fused_table(const Table<AdjFused> &w, uint32_t blocks, int32_t in_dt, hipStream_t st)
{
    if (blocks == 0) return hipSuccess;
    switch (in_dt) {
    case DT_F32: adjoint_fused_table_kernel<float, 16, 1, 2, 2, 256><<<dim3(blocks), 256, 0, st>>>(w); break;
    case DT_BF16: adjoint_fused_table_kernel<bf16, 16, 1, 2, 2, 256><<<dim3(blocks), 256, 0, st>>>(w); break;
    default: adjoint_fused_table_kernel<f16, 16, 1, 2, 2, 256><<<dim3(blocks), 256, 0, st>>>(w); break;
    }
    return hipGetLastError();
}

hipError_t launch_backproject_table(const Table<BpParams> &w, uint32_t blocks, bool two_d, int32_t in_dt,
                                    int32_t out_dt, hipStream_t st)
{
    return bp_any(w, two_d, blocks, in_dt, out_dt, st);
}

// The splat's rectangles: the back-projection's rows and an odd row stride
// of 25 words, so that the deposits of a wave, a few rows apart, fall into
// different LDS banks (measured on cone 256^3 x 360 over strides 24-37).
constexpr int kSplatCols = 25;

int64_t splat_blocks(const SplatParams &p)
{
    const int64_t bz = p.n[2] == 1 ? 1 : (p.n[2] + kBpDepth - 1) / kBpDepth;
    return static_cast<int64_t>((p.n[0] + 15) / 16) * ((p.n[1] + 15) / 16) * bz * p.batch;
}

template <typename S>
static hipError_t splat_s(const SplatParams &p, uint32_t blocks, hipStream_t st)
{
    if (p.n[2] == 1)
        splat_kernel<S, 1, 4, 64><<<dim3(blocks), 256, 0, st>>>(p);
    else
        splat_kernel<S, kBpDepth, kBpRows, kSplatCols><<<dim3(blocks), 256, 0, st>>>(p);
    return hipGetLastError();
}

hipError_t launch_splat(const SplatParams &p, int32_t in_dt, hipStream_t st)
{
    const int64_t blocks = splat_blocks(p);
    if (blocks == 0) return hipSuccess;
    switch (in_dt) {
    case DT_F32: return splat_s<float>(p, static_cast<uint32_t>(blocks), st);
    case DT_BF16: return splat_s<bf16>(p, static_cast<uint32_t>(blocks), st);
    default: return splat_s<f16>(p, static_cast<uint32_t>(blocks), st);
    }
}

hipError_t launch_fill_zero(void *dst, int64_t bytes, hipStream_t st)
{
    const int64_t words = bytes / 4;
    if (words > 0) {
        int64_t blocks = (words + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        fill_zero_kernel<<<dim3(static_cast<uint32_t>(blocks)), 256, 0, st>>>(static_cast<uint32_t *>(dst), words);
    }
    if (bytes % 4)  // a trailing 16-bit element (odd count of 16-bit values)
        fill_zero_bytes_kernel<<<1, 64, 0, st>>>(static_cast<uint8_t *>(dst) + words * 4,
                                                 static_cast<int32_t>(bytes % 4));
    return hipGetLastError();
}

hipError_t launch_convert(const float *src, void *dst, int32_t out_dt, int64_t n, hipStream_t st)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (out_dt == DT_BF16)
        convert_kernel<bf16><<<dim3(static_cast<uint32_t>(blocks)), 256, 0, st>>>(src, static_cast<bf16 *>(dst), n);
    else if (out_dt == DT_F16)
        convert_kernel<f16><<<dim3(static_cast<uint32_t>(blocks)), 256, 0, st>>>(src, static_cast<f16 *>(dst), n);
    else
        convert_kernel<float><<<dim3(static_cast<uint32_t>(blocks)), 256, 0, st>>>(src, static_cast<float *>(dst), n);
    return hipGetLastError();
}

// ------------------------------------------------ allocation-free scratch --

// Device memory of the allocation-free adjoint (pn_adjoint_noalloc): one
// array per GPU, created with the code object and held until the process
// ends.  In host code `scratch` names a host-side stand-in, not the device
// array: host code uses only the address that scratch_address() looks up.
constexpr size_t kScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t scratch_bytes() { return kScratchBytes; }

// Device address of this GPU's scratch array, looked up once per device
// (with that device current) and kept.
hipError_t scratch_address(void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace pn
