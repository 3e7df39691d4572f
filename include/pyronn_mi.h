/*
 * pyronn_mi.h -- C ABI of the MI355X (gfx950) CT projector library.
 *
 * The library computes the three operators of the differentiable CT layer
 * described in the PYRO-NN update (arXiv 2511.08427):
 *
 *   pn_forward      the ray-driven forward projection A (Sec. 2.1: one ray per
 *                   detector pixel, absorption values summed along it).  The
 *                   sampling rule is Joseph's: the ray is cut by every volume
 *                   plane perpendicular to its dominant index-space axis, the
 *                   volume is bilinearly interpolated in that plane with zero
 *                   padding, and the sum is scaled by the ray length per plane.
 *   pn_adjoint      the exact adjoint A^T of pn_forward (Sec. 2.2 pairs the
 *                   forward operator A with its adjoint A^T; it is the
 *                   analytic gradient of A, Sec. 2 and Sec. 2.4 "PyTorch
 *                   Integration").
 *   pn_backproject  the voxel-driven back-projection (Sec. 2.1: each voxel is
 *                   projected onto the detector and the measured values are
 *                   accumulated), with bilinear detector interpolation and the
 *                   distance weight (W0/W)^2 of the FDK algorithm, where W is
 *                   the third homogeneous coordinate of the voxel centre and
 *                   W0 that of the world origin.
 *
 * Besides them: the splat projector (pn_splat, the back-projection's
 * transpose), sampler-interpolation variants of A and of the back-projection
 * (pn_forward_sampled, pn_backproject_sampled: the texture path of Sec. 2.1
 * written out for a GPU without texture samplers), the FBP/FDK row filter,
 * sinogram artifact simulation, batched calls and batch plans, the
 * allocation-free adjoint and the trajectory helpers.
 *
 * Geometry follows the paper's description (Listing 1 and Sec. 2.1/2.3):
 * volume shape and spacing, detector shape and spacing, SID/SDD, and one
 * projection matrix per view for arbitrary trajectories (calibrated matrices
 * from real systems are accepted as they are).  The pn_*_matrices helpers
 * compose matrices from source/detector positions and detector directions
 * (Sec. 2.4 "Flexible Trajectory Modeling", after Graetz).
 *
 * Conventions
 *   volume    C-contiguous [batch][nz][ny][nx]; voxel (i,j,k) centre at world
 *             (ox + i*sx, oy + j*sy, oz + k*sz) mm.  2-D images are nz = 1.
 *   detector  C-contiguous [batch][n_views][rows][cols]; pixel (column c,
 *             row r) has image coordinates (u, v) = (c, r).  2-D: rows = 1.
 *   matrices  3-D: 3x4 row-major, (U,V,W) = P (x,y,z,1), u = U/W, v = V/W;
 *             parallel beam has last row (0,0,0,w).  2-D: 2x3 row-major,
 *             (U,W) = P (x,y,1), u = U/W; parallel beam has last row (0,0,w).
 *             A matrix is defined up to scale; the sign is normalised so that
 *             W > 0 over the volume.
 *   rays      the whole line through the pixel is integrated; the library
 *             requires the entire volume (dilated by one voxel) to lie in
 *             front of the source, so the line and the source-detector
 *             segment agree inside the support.
 *
 * Memory and streams
 *   vol/sino/in/out pointers are DEVICE pointers owned by the caller,
 *   C-contiguous, 4-byte aligned (2-byte for 16-bit types) and must not
 *   alias.  pg->proj is a HOST pointer owned by the caller; it is read during
 *   the call only.  Work is enqueued asynchronously on `hip_stream` (a
 *   hipStream_t; NULL = the default stream).  Outputs are overwritten, never
 *   accumulated into.  The library keeps a cache of per-geometry plans
 *   (per-view tables and work buffers in device memory, at most 32 plans
 *   besides pinned ones, least recently used evicted first); the first call
 *   with a new geometry allocates and uploads synchronously, later calls
 *   with an equal geometry, batch and types allocate nothing.  Two calls
 *   that use the same geometry and operator on different streams at the
 *   same time race on that plan's work buffers: order them on one stream.
 *
 * Graph capture
 *   The operator calls enqueue kernels only (no memset, copy or allocation
 *   once their plan and buffers exist), so they can be captured into a HIP
 *   graph.  Rules:
 *   - a captured call must follow an eager call with the same geometry,
 *     batch and types; a call that would allocate while its stream is
 *     capturing returns PN_EINVAL and enqueues nothing;
 *   - a plan used by a captured call is pinned: it is never evicted, and its
 *     buffers are never freed or re-purposed.  A later call on the same
 *     geometry that needs a larger buffer (a larger batch) or one laid out
 *     for another storage type gets a new buffer; the old one stays
 *     allocated for the graph until pn_release_caches;
 *   - pn_release_caches frees everything, pinned plans included: graphs that
 *     captured calls of this library must not be replayed after it;
 *   - a replay shares the plan's buffers with eager calls of the same
 *     geometry: order them on one stream.
 *
 * Errors
 *   Every function returns 0 on success or a negative PN_E* code; the text of
 *   the last error of the calling thread is returned by pn_last_error().  All
 *   argument and geometry checks happen before anything is enqueued; a fault
 *   inside a kernel surfaces at the caller's next synchronisation.
 */
#ifndef PYRONN_MI_H
#define PYRONN_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element types of volumes and sinograms (storage only; arithmetic is FP32,
 * per-ray set-up FP64) */
typedef enum { PN_F32 = 0, PN_BF16 = 1, PN_F16 = 2 } pn_dtype;

/* beam types: 2-D accepts PN_PARALLEL and PN_FAN, 3-D PN_PARALLEL and PN_CONE */
typedef enum { PN_PARALLEL = 0, PN_FAN = 1, PN_CONE = 2 } pn_beam;

enum {
    PN_OK = 0,
    PN_EINVAL = -1, /* null/misaligned pointer, bad shape, size or batch */
    PN_EDTYPE = -2, /* unknown dtype */
    PN_EGEOM = -3,  /* non-finite or singular matrix, volume not in front of the source */
    PN_EHIP = -4,   /* HIP runtime error (text from hipGetErrorString) */
    PN_ENOMEM = -5  /* device or host allocation failed */
};

typedef struct {
    int32_t ndim;           /* 2 or 3 */
    int32_t beam;           /* pn_beam */
    int64_t vol_shape[3];   /* nz, ny, nx (> 0; 2-D: nz = 1) */
    double vol_spacing[3];  /* sz, sy, sx in mm (> 0; 2-D: sz ignored) */
    double vol_origin[3];   /* z, y, x world position of voxel (0,0,0) centre;
                               NaN in an entry centres that axis on 0 */
    int64_t det_shape[2];   /* rows, cols (> 0; 2-D: rows = 1) */
    double det_spacing[2];  /* row, column pixel pitch in mm (informational) */
    double sid, sdd;        /* source-isocentre, source-detector distance (informational) */
    int64_t n_views;        /* >= 0 */
    const double *proj;     /* host: n_views matrices, 3x4 (3-D) or 2x3 (2-D) */
} pn_geometry;

/* One volume/sinogram pair of a batched call (batch size 1 each). */
typedef struct {
    pn_geometry geom;
    const void *in;
    void *out;
} pn_problem;

/* A: vol [batch][nz][ny][nx] (in_dtype) -> sino [batch][n_views][rows][cols]
 * (out_dtype).  batch >= 0; batch == 0 does nothing. */
int pn_forward(const pn_geometry *pg, int64_t batch, const void *vol, void *sino,
               int32_t in_dtype, int32_t out_dtype, void *hip_stream);

/* A with sampler interpolation (Sec. 2.1, interpolation: sampling through a
 * texture is faster but needs extra memory; interpolation written in the
 * kernel saves memory).  The same operator as pn_forward -- same rays,
 * planes and FP64 ray set-up -- but every bilinear tap is a separate load
 * through the caches instead of being staged through LDS, from the image
 * chosen by `source`:
 *   PN_SAMPLE_BORDERED  zero-bordered copies of the volume, one per dominant
 *                       axis a that occurs (the copies pn_forward builds:
 *                       8 ((n_f + 24) / 8) (n_s + 3) n_a elements per axis
 *                       and batch item, n_f and n_s the in-plane sizes, held
 *                       by the geometry's plan);
 *   PN_SAMPLE_DIRECT    the caller's volume itself, every tap bounds-checked;
 *                       no extra memory besides the view tables.
 * weight_bits = 0 interpolates with FP32 weights (the result then matches
 * pn_forward to FP32 rounding); 1 <= weight_bits <= 16 rounds each of the
 * two in-plane weights to a multiple of 2^-weight_bits, ties upward (the
 * upper tap's weight round(frac(position) * 2^B) / 2^B), the way fixed-
 * function filtering hardware quantises its weights, so that this loss of
 * precision can be measured.  Shapes, types, streams and capture rules as
 * pn_forward; additionally PN_EINVAL for an unknown source, weight_bits
 * outside [0, 16], or an image of 2^31 elements or more per batch item. */
enum { PN_SAMPLE_BORDERED = 0, PN_SAMPLE_DIRECT = 1 };
int pn_forward_sampled(const pn_geometry *pg, int64_t batch, const void *vol, void *sino,
                       int32_t in_dtype, int32_t out_dtype, int32_t source, int32_t weight_bits,
                       void *hip_stream);

/* A^T: sino [batch][n_views][rows][cols] (in_dtype) -> vol [batch][nz][ny][nx]
 * (out_dtype).  Exact transpose of pn_forward up to rounding: each block of
 * output voxels sums its rays' contributions in 32-bit fixed point whose
 * power-of-two scale follows the magnitude of those rays (the error of a
 * contribution is at most 2^-20 of the largest |q ds| among the few hundred
 * rays processed with it), then in FP32; the result is bitwise
 * reproducible.  A non-finite sinogram value turns the output blocks its
 * ray reaches into NaN (other blocks and batch items are unaffected). */
int pn_adjoint(const pn_geometry *pg, int64_t batch, const void *sino, void *vol,
               int32_t in_dtype, int32_t out_dtype, void *hip_stream);

/* pn_adjoint for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results as pn_adjoint (bitwise equal to it
 * with the default adjoint block shape, i.e. without PN_AUTOTUNE or
 * PN_ADJ_SHAPE).  It calls no hipMalloc/hipFree: its view tables, candidate
 * boxes and, for a 16-bit output, its FP32 accumulator live in one fixed
 * device array of PN_NOALLOC_SCRATCH_BYTES per GPU, created with the
 * library's code object and held until the process ends.
 *   - A call that needs more than that (large volumes, many views, a large
 *     batch with a 16-bit output) returns PN_EINVAL, says how much it needs
 *     in pn_last_error(), and enqueues nothing.  The 256^3 x 360-view cone
 *     problem fits for every output type.
 *   - The array keeps the last call's tables and boxes.  A call with the
 *     same geometry as the previous call on this GPU enqueues only the
 *     adjoint kernels; any other geometry first copies its tables from
 *     pageable host memory (the copy blocks the calling thread) and builds
 *     the boxes with a kernel.
 *   - Under stream capture only the first kind of call is accepted (else
 *     PN_EINVAL); a captured graph replays correctly only while no call
 *     with another geometry has gone through this entry point on that GPU.
 *   - Every call on one GPU uses the same array: calls that overlap in
 *     time on one GPU (other streams, other threads) race, and the caller
 *     must serialise them. */
#define PN_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
int pn_adjoint_noalloc(const pn_geometry *pg, int64_t batch, const void *sino, void *vol,
                       int32_t in_dtype, int32_t out_dtype, void *hip_stream);

/* Voxel-driven (W0/W)^2-weighted back-projection: sino -> vol, shapes as
 * pn_adjoint.  A 16-bit output may overflow (F16 max 65504) for many views;
 * request PN_F32 output in that case. */
int pn_backproject(const pn_geometry *pg, int64_t batch, const void *sino, void *vol,
                   int32_t in_dtype, int32_t out_dtype, void *hip_stream);

/* pn_backproject with sampler interpolation (Sec. 2.1, interpolation: the
 * texture path and the kernel path, as for pn_forward_sampled): the same
 * operator -- each voxel centre projected with the view's matrix, (W0/W)^2
 * weight -- with every bilinear detector tap a separate load through the
 * caches, from the image chosen by `source`:
 *   PN_SAMPLE_BORDERED  a zero-bordered copy of the sinogram (rows and
 *                       columns padded by one before and two after: extra
 *                       device memory of (rows + 3)(cols + 3) elements per
 *                       view and batch item, held by the geometry's plan);
 *   PN_SAMPLE_DIRECT    the caller's sinogram itself, every tap
 *                       bounds-checked; no extra memory.
 * weight_bits as pn_forward_sampled (0: FP32 weights, the result then
 * matches pn_backproject to FP32 rounding; 1..16: each detector weight
 * rounded to a multiple of 2^-weight_bits, ties upward).  Shapes, types,
 * streams and capture rules as pn_backproject; additionally PN_EINVAL for
 * an unknown source, weight_bits outside [0, 16], or a bordered view of
 * 2^31 elements or more. */
int pn_backproject_sampled(const pn_geometry *pg, int64_t batch, const void *sino, void *vol,
                           int32_t in_dtype, int32_t out_dtype, int32_t source, int32_t weight_bits,
                           void *hip_stream);

/* Transpose of pn_backproject (the splat projector), the analytic gradient
 * of the back-projection with respect to its sinogram (Sec. 2: gradients
 * for all operators): vol [batch][nz][ny][nx] (in_dtype) -> sino
 * [batch][n_views][rows][cols] (out_dtype), where every voxel's value times
 * (W0/W)^2 is spread over the bilinear taps of its projection (taps off the
 * detector are dropped), so that <pn_backproject(q), x> = <q, pn_splat(x)>.
 * Deposits gather per block of voxels in fixed point and are added to the
 * sinogram with float atomics: the result is not bitwise reproducible
 * (differences are FP32 rounding).  A 16-bit output is accumulated in an
 * FP32 buffer of the plan and rounded at the end. */
int pn_splat(const pn_geometry *pg, int64_t batch, const void *vol, void *sino,
             int32_t in_dtype, int32_t out_dtype, void *hip_stream);

/* Row filter of the filtered back-projection (Sec. 2.2: the reconstruction
 * is the back-projection of the sinogram filtered along detector rows by a
 * diagonal Fourier-domain filter).  out = (pi / N) (1 / a) g * (c p) along
 * every detector row, where N = n_views, a is the pixel pitch at the
 * rotation axis (det_spacing[1], times sid / sdd for fan and cone beams),
 * c the cosine of each pixel's ray to the detector normal (1 for parallel
 * beams) and g the discrete kernel: PN_FILTER_RAM_LAK (g[0] = 1/4,
 * g[k] = -1/(pi^2 k^2) for odd k, 0 otherwise) or PN_FILTER_SHEPP_LOGAN
 * (g[k] = -2/(pi^2 (4 k^2 - 1))); the convolution is linear (zero outside
 * the row), i.e. F^-1 K F with K the kernel's DFT on rows padded to twice
 * their length.  pn_backproject of the result is the FBP (parallel) or FDK
 * (fan, cone; full 2 pi orbit) reconstruction.
 * sino and out: [batch][n_views][rows][cols], device pointers, distinct
 * buffers; cols <= 1024.  Fan and cone beams need sid > 0 and sdd > 0 in the
 * geometry.  Errors: PN_EINVAL (kind, sizes, spacing, sid/sdd), PN_EGEOM. */
enum { PN_FILTER_RAM_LAK = 0, PN_FILTER_SHEPP_LOGAN = 1 };
int pn_filter(const pn_geometry *pg, int64_t batch, const void *sino, void *out, int32_t in_dtype,
              int32_t out_dtype, int32_t kind, void *hip_stream);

/* Additive Gaussian noise (Sec. 2.4, artifact simulation: electronic and
 * thermal read-out noise): data[i] += mean + sigma * z_i for 0 <= i < n, in
 * place on a device buffer of n elements of dtype.  z_i is standard normal:
 * the counter-based generator Philox4x64-10 (Salmon et al., SC'11) under
 * key (seed, 0) gives at counter (i / 4, 0, 0, 0) four words w0..w3;
 * uniforms u = ((w >> 11) + 1/2) 2^-53; Box-Muller on (u0, u1) gives z for
 * i % 4 = 0 (cosine) and 1 (sine), on (u2, u3) for 2 and 3.  The draw is
 * formed in FP64 and added in FP32; the result is a pure function of
 * (seed, i, input), so calls are reproducible and any slice of a buffer can
 * be regenerated.  Errors: PN_EINVAL (n < 0, NULL or misaligned data,
 * sigma < 0 or non-finite mean/sigma), PN_EDTYPE. */
int pn_gaussian_noise(int64_t n, void *data, int32_t dtype, double mean, double sigma, uint64_t seed,
                      void *hip_stream);

/* Detector jitter (Sec. 2.4, artifact simulation: random pixel shifts of
 * detector rows): out row g = in row g moved by an integer shift s_g along
 * the columns, out[c] = in[c - s_g], 0 where c - s_g leaves the row.
 * in and out: [n_rows][cols] device buffers of dtype that do not overlap
 * (n_rows = batch x views x detector rows).  s_g is uniform in
 * -max_shift .. max_shift: word w0 of the Philox4x64-10 block at counter
 * (g, 0, 0, 0) under key (seed, 1), s_g = (w0 mod (2 max_shift + 1)) -
 * max_shift.  Errors: PN_EINVAL (shape, 0 <= max_shift <= 2^20, NULL,
 * misaligned or overlapping buffers), PN_EDTYPE. */
int pn_detector_jitter(int64_t n_rows, int32_t cols, const void *in, void *out, int32_t dtype, int32_t max_shift,
                       uint64_t seed, void *hip_stream);

/* Gantry motion blur (Sec. 2.4, artifact simulation: a kernel turned to
 * each projection's acquisition angle): out = in convolved, per view k, with
 * a line kernel at angle a_k = angle_start + k angle_step: the mean of
 * `taps` (odd, 1 .. 255) samples at unit spacing t = -h .. h along
 * (cos a_k, sin a_k) in (column, row) pixel units, bilinear, zeros outside
 * the detector; a single-row detector (rows == 1, 2-D sinograms) has no
 * row direction and uses (cos a_k, 0).  in and out: [batch][n_views][rows][cols] device buffers of
 * dtype that do not overlap.  Errors: PN_EINVAL (shape, taps, non-finite
 * angles, NULL, misaligned or overlapping buffers), PN_EDTYPE. */
int pn_gantry_blur(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, const void *in, void *out,
                   int32_t dtype, double angle_start, double angle_step, int32_t taps, void *hip_stream);

/* Ring artifacts (Sec. 2.4: defective or miscalibrated detector elements):
 * in place on sino [batch][n_views][rows][cols] (device, dtype), every row
 * of detector columns columns[0 .. n_columns) (host array; duplicates count
 * once; n_columns <= 256) in views v0 <= v < v1 is multiplied by gain
 * (0 gives dead columns); the product is taken in FP32.  Errors: PN_EINVAL
 * (shape, view range, column out of range, too many columns, NULL pointers,
 * non-finite gain), PN_EDTYPE. */
int pn_ring_artifacts(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, void *sino, int32_t dtype,
                      const int32_t *columns, int32_t n_columns, double gain, int32_t v0, int32_t v1,
                      void *hip_stream);

/* The same operators over n independent problems of uneven sizes (each a
 * batch of one, all of the same in and out types).  Every problem is
 * validated before anything is enqueued; the problems are ordered by
 * estimated cost, largest first, and run as work lists of up to 12 problems
 * per kernel launch (per dominant axis for the adjoint).  Each problem's
 * result equals its single-problem call bit for bit.  The work lists travel
 * as kernel arguments, so these calls can be captured (the rules above);
 * for one launch per kernel group over any number of problems, replayed
 * from a graph the library captures, see the batch plans below. */
int pn_forward_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype,
                       void *hip_stream);
int pn_adjoint_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype,
                       void *hip_stream);
int pn_backproject_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype,
                           void *hip_stream);

/* Batch plans: one fixed problem set run many times (the batch axis of the
 * layers, Sec. 2.3 Listing 1; uneven problem lists).  pn_batch_create
 * validates the problems, readies their plans (pinned and held by the
 * batch plan, so pn_release_caches keeps them), builds every work buffer and
 * candidate table on a stream of its own, writes one work list per kernel
 * group into device memory (problems largest first, all of a group in ONE
 * launch) and captures the whole operator -- relayouts, fills, main
 * kernels, 16-bit conversions -- in a HIP graph.  pn_batch_run replays that
 * graph on hip_stream: it reads the problems' current input buffers and
 * overwrites their output buffers, with results equal to pn_*_batched bit
 * for bit.  The buffers of `probs` are fixed at creation: they must stay
 * allocated, and the caller changes the inputs' contents between runs, not
 * their addresses.  Problems that share a geometry share work buffers, so
 * they run in successive groups of launches.
 *   op: PN_OP_FORWARD (in = volume, out = sinogram), PN_OP_ADJOINT or
 *       PN_OP_BACKPROJECT (in = sinogram, out = volume).
 *   Errors: those of the batched calls, PN_EINVAL for n == 0 or an unknown
 *   op, PN_ENOMEM, PN_EHIP (graph capture or instantiation).
 * pn_batch_run from a device other than the creating one returns
 * PN_EINVAL.  pn_batch_destroy frees the graph and the work lists and
 * releases the plans (NULL is allowed); runs already enqueued must have
 * completed. */
typedef enum { PN_OP_FORWARD = 0, PN_OP_ADJOINT = 1, PN_OP_BACKPROJECT = 2 } pn_op;
typedef struct pn_batch pn_batch;
int pn_batch_create(int32_t op, const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype,
                    pn_batch **out);
int pn_batch_run(pn_batch *b, void *hip_stream);
int pn_batch_destroy(pn_batch *b);

/* Host-only validation of a geometry (no device work): 0 or a PN_E* code. */
int pn_check_geometry(const pn_geometry *pg);

/* Projection-matrix composition (Sec. 2.4, after Graetz), host only, FP64.
 * Vectors are arrays of n_views rows, world mm.  S: source, C: detector
 * centre (the point halfway between the outermost pixel centres), eu/ev:
 * world step from one pixel centre to the next along a row / a column.
 * Pixel (c, r) lies at C + (c - (cols-1)/2) eu + (r - (rows-1)/2) ev, and the
 * matrix maps it to (u, v) = (c, r).  Output P_out: n_views x 3x4 (2-D: 2x3).
 * Returns PN_EGEOM for a degenerate view. */
int pn_cone_matrices(int64_t n_views, const double *S, const double *C, const double *eu,
                     const double *ev, int64_t rows, int64_t cols, double *P_out);
int pn_fan_matrices(int64_t n_views, const double *S, const double *C, const double *eu,
                    int64_t cols, double *P_out);
/* parallel beams: `dir` is the ray direction instead of a source */
int pn_parallel2d_matrices(int64_t n_views, const double *dir, const double *C, const double *eu,
                           int64_t cols, double *P_out);
int pn_parallel3d_matrices(int64_t n_views, const double *dir, const double *C, const double *eu,
                           const double *ev, int64_t rows, int64_t cols, double *P_out);

/* Text of the calling thread's last error ("" if none). */
const char *pn_last_error(void);

/* Frees every cached plan and work buffer, pinned ones included (graphs
 * that captured calls of this library become invalid); the next call
 * rebuilds. */
int pn_release_caches(void);

/* Library version string. */
const char *pn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PYRONN_MI_H */
