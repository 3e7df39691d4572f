// Internal types shared by the host library (pn_host.cpp) and the gfx950
// kernels (pn_kernels.hip, pn_sampler.hip, pn_signal.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>

namespace pn {

// Work copies of the volume used by the forward projector: one per dominant
// axis a, laid out [batch][n_a][rows][cols] with the in-plane "slow" axis as
// rows and the "fast" axis as columns.  a = x: rows z, cols y; a = y: rows z,
// cols x; a = z: rows y, cols x.  Rows are padded with PADR_LO zero rows
// before and PADR_HI after, columns with PADC zeros on each side, so every
// bilinear tap of a position clamped to [-1, n] is addressable.
constexpr int PADR_LO = 1;
constexpr int PADR_HI = 2;
constexpr int PADC = 8;

// Elements per row of a work copy with `nf` columns: room for PADC zeros on
// the left and for whole 16-byte vectors reaching up to column nf + 8 on the
// right, rounded to a multiple of 8 elements (16-byte aligned rows for every
// storage type).
inline int32_t work_row(int32_t nf) { return (nf + PADC + 9 + 7) / 8 * 8; }

// Per-view FP64 tables in volume index space (x, y, z order).  Built on the
// host from the view's projection matrix.
struct ViewTab {
    double A[9];   // ray direction:      delta(u, v) = A (u, v, 1)^T
    double B[9];   // a point on the ray: p(u, v)     = B (u, v, 1)^T
    double Pi[12]; // projection of index coordinates: (U,V,W) = Pi (i, j, k, 1)^T
};

// Per-view FP32 table for the voxel-driven back-projection.
struct ViewTabF {
    float Pi[12];  // as ViewTab::Pi, rounded
    float W0;      // W of the world origin (distance weight reference)
    int32_t axes;  // bit a set when some ray of the view may have dominant axis a
    float kcell;   // bound on the rays of the view that sample one voxel's 2x2 neighbourhood in one plane
    float pad;
};

enum DType : int32_t { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2 };

struct FwdParams {
    const ViewTab *tab;
    int32_t n_views, nu, nv, batch;
    int32_t n[3];          // nx, ny, nz
    double s[3];           // sx, sy, sz (mm)
    const void *lay[3];    // work copy per dominant axis (nullptr: not built)
    int64_t lay_item[3];   // elements per batch item of each copy
    int64_t lay_plane[3];  // elements per plane
    int32_t lay_row[3];    // elements per row
    void *sino;            // [batch][n_views][nv][nu]
    int32_t tile_u, tile_v;  // ray tile (tile_u * tile_v == block size)
    int32_t view_group;      // consecutive views per workgroup
    int32_t tiles_u, tiles_v;  // tiles covering the detector window [c_lo, nu) x [r_lo, nv) that is launched
    int32_t c_lo, r_lo;        // first column and row of the window
    const int32_t *vwin;       // per view: detector window of the view (c0, c1, r0, r1), or nullptr
    int32_t point_source;      // 1: every ray of a view leaves one point (B has zero u and v columns)
};

// Sampler-interpolation forward projector (pn_sampler.hip): one thread per
// ray, every tap gathered through the cache hierarchy from an "image" of the
// volume per dominant axis a.  Element (m, s, f) of image a (plane m along
// a, in-plane slow index s, fast index f) of batch item b sits at
// img[a] + b*item[a] + org[a] + m*plane[a] + s*row[a] + f*col[a].
struct SampParams {
    const ViewTab *tab;
    int32_t n_views, nu, nv, batch;
    int32_t n[3];
    double s[3];
    const void *img[3];    // per dominant axis (nullptr: no ray takes it)
    int64_t item[3], plane[3], row[3], col[3], org[3];
    void *sino;            // [batch][n_views][nv][nu]
    int32_t tile_u, tile_v, tiles_u, tiles_v;
    int32_t view_group;    // consecutive views per workgroup (tile_u * tile_v * view_group == 256)
    int32_t bordered;      // 1: images with a zero border (work copies), 0: the caller's volume, taps checked
    int32_t weight_bits;   // 0: FP32 weights; B > 0: weights rounded to multiples of 2^-B (ties up)
    int32_t point_source;  // 1: every ray of a view leaves one point (B has zero u and v columns)
};

// Sampler-interpolation back-projection (pn_sampler.hip): every bilinear
// detector tap a load through the caches.  Detector pixel (r, c) of view v
// of batch item b sits at img + b*item + v*view + org + r*row + c.
struct BpSampParams {
    const ViewTabF *tabf;
    int32_t n_views, nu, nv, batch;
    int32_t n[3];
    const void *img;       // zero-bordered copy of the sinogram, or the caller's sinogram
    int64_t item, view, org;
    int32_t row;
    int32_t bordered;      // 1: bordered copy (taps unchecked), 0: the caller's sinogram, taps checked
    int32_t weight_bits;   // 0: FP32 weights; B > 0: weights rounded to multiples of 2^-B (ties up)
    void *vol;             // [batch][nz][ny][nx]
};

struct AdjParams {
    const ViewTab *tab;
    const ViewTabF *tabf;
    float kunits;            // power of two >= every kcell: max|q ds| units a flush period holds
    const uint32_t *cbox;  // per (block, pass view) 2 words: candidate pixel box (cbox_kernel)
    const int32_t *views;  // views processed by this pass
    int32_t n_pass_views;
    int32_t axis;          // dominant axis handled by this pass
    int32_t nu, nv, n_views, batch;
    int32_t n[3];
    double s[3];
    const void *sino;      // [batch][n_views][nv][nu]
    float *out;            // FP32 [batch][nz][ny][nx]
    int32_t accumulate;    // 0: overwrite, 1: add to existing values
    int32_t blocks_a, blocks_s, blocks_f;
    int32_t point_source;  // 1: every ray of a view leaves one point (B has zero u and v columns)
};

// The passes of one 3-D adjoint in a single launch over cubic blocks:
// pass[a].n_pass_views == 0 when axis a has no views; nb: blocks along x, y, z.
struct AdjFused {
    AdjParams pass[3];
    int32_t nb[3];
    int32_t batch;
};

struct BpParams {
    const ViewTabF *tabf;
    int32_t n_views, nu, nv, batch;
    int32_t n[3];
    const void *sino;
    void *vol;
    int32_t bz;            // 3-D block depth along z (8, 16 or 32); 0: the default 16
};

// Splat projector (transpose of the voxel-driven back-projection).
struct SplatParams {
    const ViewTabF *tabf;
    int32_t n_views, nu, nv, batch;
    int32_t n[3];
    const void *vol;       // [batch][nz][ny][nx]
    float *sino;           // FP32 [batch][n_views][nv][nu], zeroed, accumulated into
};

constexpr int kRingMaxCols = 256;

struct NoiseParams {
    void *data;            // n elements, updated in place
    int64_t n;
    double mean, sigma;
    uint64_t seed;         // Philox key word 0
};

struct RingParams {
    void *data;            // [batch][n_views][rows][cols], updated in place
    int64_t batch;
    int32_t n_views, rows, cols;
    int32_t v0, v1;        // views v0 <= v < v1
    int32_t n_sel;         // distinct columns in sel
    float gain;
    int32_t sel[kRingMaxCols];
};

struct JitterParams {
    const void *in;        // [n_rows][cols]
    void *out;             // same shape, distinct buffer
    int64_t n_rows;
    int32_t cols;
    int32_t max_shift;
    uint64_t seed;         // Philox key word 0 (word 1 is 1)
};

struct BlurParams {
    const void *in;        // [batch][n_views][rows][cols]
    void *out;             // same shape, distinct buffer
    int64_t batch;
    int32_t n_views, rows, cols;
    int32_t taps;          // odd
    double angle_start, angle_step;
};

struct FiltParams {
    const ViewTab *tab;
    int32_t n_views, nu, nv, batch;
    double s[3];           // voxel spacing (index-space tables to world)
    int32_t parallel;      // 1: no cosine weights
    int32_t kind;          // 0: Ram-Lak, 1: Shepp-Logan
    float scale;           // pi / N / (pixel pitch at the rotation axis)
    const void *in;        // [batch][n_views][nv][nu]
    void *out;             // same shape
};

// Work list in device memory (a batch plan's table): workgroups
// [start[i], start[i + 1]) run problem p[i]; one launch covers any number of
// problems.
template <typename P>
struct Table {
    const P *p;
    const uint32_t *start;  // n + 1 entries
    int32_t n;
};

// Work list of a batched launch, passed by value as the kernel argument
// (no device allocation or copy, so a batched call can be captured in a
// graph): workgroups [start[i], start[i+1]) run problem i.
constexpr int kMaxBatch = 12;
template <typename P>
struct Batch {
    P p[kMaxBatch];
    uint32_t start[kMaxBatch + 1];
    int32_t n;
};

}  // namespace pn
