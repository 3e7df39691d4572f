// Device side of the CT projector library's host code: the plan cache and
// work buffers, kernel launches, and the extern "C" operator entry points
// declared in include/pyronn_mi.h.  Validation and the per-view tables are
// in pn_geometry.cpp; the rules for cached device memory under graph
// capture in pn_cache.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pn_cache.hpp"
#include "pn_internal.hpp"

namespace pn {
hipError_t launch_relayout(int32_t dtype, const void *in, void *out, const int32_t n[3], int axis, int32_t batch,
                           int64_t item, int32_t row, int64_t plane, hipStream_t st);
hipError_t launch_forward(const FwdParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st);
hipError_t launch_forward_sampled(const SampParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st);
hipError_t launch_backproject_sampled(const BpSampParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st);
int64_t backproject_sampled_blocks(const BpSampParams &p);
hipError_t launch_pad_sino(int32_t dt, const void *in, void *out, int64_t n_img, int32_t nv, int32_t nu, int32_t row,
                           int64_t view, hipStream_t st);
int64_t forward_sampled_blocks(const SampParams &p);
void forward_sampled_tile(bool two_d, int32_t &tu, int32_t &tv, int32_t &views);
hipError_t launch_adjoint(const AdjParams &p, int32_t in_dt, int shape, hipStream_t st);
bool adjoint_fusable(bool two_d, int shape);
hipError_t launch_forward_table(const Table<FwdParams> &w, uint32_t blocks, bool two_d, int32_t in_dt,
                                int32_t out_dt, hipStream_t st);
hipError_t launch_adjoint_table(const Table<AdjParams> &w, uint32_t blocks, int axis, int32_t in_dt, int shape,
                                hipStream_t st);
hipError_t launch_adjoint_fused_table(const Table<AdjFused> &w, uint32_t blocks, int32_t in_dt, hipStream_t st);
hipError_t launch_backproject_table(const Table<BpParams> &w, uint32_t blocks, bool two_d, int32_t in_dt,
                                    int32_t out_dt, hipStream_t st);
hipError_t launch_adjoint_fused(const AdjFused &f, int32_t in_dt, hipStream_t st);
hipError_t launch_backproject(const BpParams &p, int32_t in_dt, int32_t out_dt, hipStream_t st);
hipError_t launch_splat(const SplatParams &p, int32_t in_dt, hipStream_t st);
int64_t splat_blocks(const SplatParams &p);
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
size_t scratch_bytes();
hipError_t scratch_address(void **out);
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

int fail_hip(hipError_t e, const char *what)
{
    return fail(PN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

// ------------------------------------------------------------- plans ------

struct HipMem {
    static bool alloc(void **p, size_t n) { return hipMalloc(p, n) == hipSuccess; }
    static void release(void *p) { (void)hipFree(p); }
};

// Retired buffers of pinned plans (pn_cache.hpp); guarded by g_mu.
BufferKeeper<HipMem> g_keeper;

struct Plan : HostTables {
    Geo g;
    int device = 0;
    // used by a call under stream capture: never evicted, buffers never
    // freed or re-purposed before pn_release_caches
    bool pinned = false;
    // batch plans (pn_batch_create) that use this plan: while any does, the
    // plan is held like a pinned one and outlives pn_release_caches
    int refs = 0;
    bool held() const { return pinned || refs > 0; }
    ViewTab *d_tab = nullptr;
    ViewTabF *d_tabf = nullptr;
    int32_t *d_views[3] = {nullptr, nullptr, nullptr};
    int32_t *d_vwin = nullptr;
    uint32_t *d_axbox = nullptr;
    // forward work copies, one per dominant axis (tag: storage type)
    DevBuf lay[3];
    int64_t lay_item[3] = {0, 0, 0}, lay_plane[3] = {0, 0, 0};
    int32_t lay_row[3] = {0, 0, 0};
    // FP32 accumulation buffers for 16-bit outputs: the adjoint's volume,
    // the splat projector's sinogram
    DevBuf acc, sacc;
    // choices of the autotuner (0: not tuned): the 3-D adjoint block shape,
    // the forward's views per workgroup, the back-projection's block depth
    int adj_shape = 0;
    int fwd_vg = 0;
    int bp_bz = 0;
    // adjoint candidate pixel boxes per pass axis (tag: block shape)
    DevBuf cbox[3];
    // zero-bordered sinogram of the sampler back-projection (tag: storage type)
    DevBuf spad;

    ~Plan()
    {
        dev_free(d_tab);
        dev_free(d_tabf);
        for (int a = 0; a < 3; ++a) dev_free(d_views[a]);
        dev_free(d_vwin);
        dev_free(d_axbox);
        for (int a = 0; a < 3; ++a) {
            g_keeper.free(lay[a]);
            g_keeper.free(cbox[a]);
        }
        g_keeper.free(acc);
        g_keeper.free(sacc);
        g_keeper.free(spad);
    }
};

std::mutex g_mu;
PlanLru<Plan> g_plans;
int g_live_batches = 0;  // batch plans not yet destroyed; guarded by g_mu
const size_t kMaxPlans = 32;

// True when work enqueued on `st` is being captured into a graph.
bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

int capture_error(const char *what)
{
    return fail(PN_EINVAL,
                "%s would allocate or re-purpose device memory while the stream is capturing: run the same call "
                "(geometry, batch, types) eagerly once before capturing it",
                what);
}

// Makes a plan buffer fit; a fresh buffer is zero-filled when `zero`.
int ensure_buf(Plan &pl, DevBuf &b, size_t need, int32_t tag, bool zero, hipStream_t st, const char *what,
               bool &fresh)
{
    fresh = false;
    switch (g_keeper.ensure(b, need, tag, pl.held(), capturing(st))) {
    case Ensure::kReady: return PN_OK;
    case Ensure::kCapturing: return capture_error(what);
    case Ensure::kNoMem: return fail(PN_ENOMEM, "%s: hipMalloc(%zu) failed", what, need);
    case Ensure::kFresh: break;
    }
    fresh = true;
    if (zero) {
        hipError_t e = launch_fill_zero(b.ptr, (int64_t)b.cap, st);
        if (e != hipSuccess) return fail_hip(e, "fill");
    }
    return PN_OK;
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
// Looks up or builds the plan of a geometry for calls on stream `st`; a
// call under capture pins the plan it uses and cannot build one.  Caller
// holds g_mu.
int get_plan(const pn_geometry *pg, hipStream_t st, Plan **out)
{
    Geo g;
    int rc = normalise_geometry(pg, g);
    if (rc) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    const bool cap = capturing(st);
    Plan *found = g_plans.find([&](const Plan &p) { return p.device == dev && p.g.same(g); });
    if (found) {
        if (cap) found->pinned = true;
        *out = found;
        return PN_OK;
    }
    if (cap) return capture_error("the first call with this geometry");
    auto pl = std::make_unique<Plan>();
    pl->g = std::move(g);
    pl->device = dev;
    build_host_tables(pl->g, *pl);
    if ((rc = upload(&pl->d_tab, pl->tab))) return rc;
    if ((rc = upload(&pl->d_tabf, pl->tabf))) return rc;
    for (int a = 0; a < 3; ++a)
        if ((rc = upload(&pl->d_views[a], pl->pass_views[a]))) return rc;
    if ((rc = upload(&pl->d_vwin, pl->vwin))) return rc;
    if ((rc = upload(&pl->d_axbox, pl->axbox))) return rc;
    *out = g_plans.insert(std::move(pl), kMaxPlans);
    return PN_OK;
}

int ensure_work_copy(Plan &pl, int a, int32_t dt, int64_t batch, hipStream_t st)
{
    const Geo &g = pl.g;
    const int f = a == 0 ? 1 : 0, sl = a == 2 ? 1 : 2;
    const int32_t row = work_row(g.n[f]);
    const int64_t plane = (int64_t)row * (g.n[sl] + PADR_LO + PADR_HI);
    const int64_t item = plane * g.n[a];
    const size_t need = (size_t)(item * batch * esize(dt));
    // padding must read as zero: a fresh copy (new, or laid out for another
    // storage type) is cleared; the interior is rewritten on every call
    bool fresh;
    int rc = ensure_buf(pl, pl.lay[a], need, dt, true, st, "work copy", fresh);
    if (rc) return rc;
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
// With PN_AUTOTUNE=1 the first 3-D single call of a plan (outside graph
// capture) times the compiled variants of its operator on the caller's
// stream and keeps the fastest for the plan: the adjoint's block shapes, the
// forward's views per workgroup (3 or 2), the back-projection's block depth
// along z (16, 8 or 32).  PN_TUNE_CACHE=<file> keeps the choices across
// processes, one line per choice: "<op> nz ny nx rows cols views beam
// value".  Different adjoint shapes round the fixed-point sums at different
// points, so with tuning on the last bits of the adjoint can differ between
// processes whose choices differ (forward and back-projection variants sum
// in the same order); without it every variant is the default one (or
// PN_ADJ_SHAPE).  Batched calls and batch plans use the defaults.

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

// The cache file holds one line per tuned choice: "<op> <geometry key>
// <value>" with op "fwd", "adj" or "bp" (lines without an op are adjoint
// choices of earlier versions).  A later line wins.
int tune_cache_lookup(const Geo &g, const char *op, int lo, int hi)
{
    const char *path = std::getenv("PN_TUNE_CACHE");
    if (!path) return 0;
    FILE *f = std::fopen(path, "r");
    if (!f) return 0;
    const std::string key = tune_key(g);
    const std::string tagged = std::string(op) + " " + key;
    char line[256];
    int found = 0;
    while (std::fgets(line, sizeof line, f)) {
        const std::string l(line);
        for (const std::string *k : {&tagged, &key}) {
            if (k == &key && std::strcmp(op, "adj") != 0) continue;
            if (l.compare(0, k->size(), *k) == 0 && l.size() > k->size() && l[k->size()] == ' ') {
                const int v = std::atoi(l.c_str() + k->size() + 1);
                if (v >= lo && v <= hi) found = v;
            }
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(const Geo &g, const char *op, int value)
{
    const char *path = std::getenv("PN_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %s %d\n", op, tune_key(g).c_str(), value);
    std::fclose(f);
}

// Times run(v) for every variant v on stream st with HIP events (one call
// each, back to back, then one synchronisation) and returns the fastest, or
// 0 with the error set.
template <typename Run>
int time_variants(const std::vector<int> &vars, Run run, hipStream_t st, int &best)
{
    best = 0;
    std::vector<hipEvent_t> ev(2 * vars.size(), nullptr);
    int rc = PN_OK;
    for (size_t k = 0; k < vars.size() && rc == PN_OK; ++k) {
        if (hipEventCreate(&ev[2 * k]) != hipSuccess || hipEventCreate(&ev[2 * k + 1]) != hipSuccess) {
            rc = fail(PN_EHIP, "autotune: hipEventCreate failed");
            break;
        }
        if (hipEventRecord(ev[2 * k], st) != hipSuccess) {
            rc = fail(PN_EHIP, "autotune: hipEventRecord failed");
            break;
        }
        if ((rc = run(vars[k]))) break;
        if (hipEventRecord(ev[2 * k + 1], st) != hipSuccess) rc = fail(PN_EHIP, "autotune: hipEventRecord failed");
    }
    float best_ms = 0.0f;
    for (size_t k = 0; k < vars.size() && rc == PN_OK; ++k) {
        float ms = 0.0f;
        if (hipEventSynchronize(ev[2 * k + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) != hipSuccess) {
            rc = fail(PN_EHIP, "autotune: event timing failed");
            break;
        }
        if (best == 0 || ms < best_ms) {
            best = vars[k];
            best_ms = ms;
        }
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// The 3-D adjoint block shape of a plan: tuned, cached, or the fixed one.
int plan_adjoint_shape(Plan *pl)
{
    if (pl->adj_shape == 0 && autotune_on()) pl->adj_shape = tune_cache_lookup(pl->g, "adj", 1, adjoint_shape_count() - 1);
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
    // every work copy is made ready before anything is launched, so a call
    // refused under capture enqueues nothing
    for (int a = 0; a < 3; ++a)
        if ((pl->axes_union >> a & 1) && (rc = ensure_work_copy(*pl, a, in_dt, batch, st))) return rc;
    for (int a = 0; a < 3; ++a) {
        p.n[a] = g.n[a];
        p.s[a] = g.s[a];
        p.lay[a] = nullptr;
        if (pl->axes_union >> a & 1) {
            hipError_t e = launch_relayout(in_dt, vol, pl->lay[a].ptr, g.n, a, (int32_t)batch, pl->lay_item[a],
                                           pl->lay_row[a], pl->lay_plane[a], st);
            if (e != hipSuccess) return fail_hip(e, "relayout launch");
            p.lay[a] = pl->lay[a].ptr;
            p.lay_item[a] = pl->lay_item[a];
            p.lay_plane[a] = pl->lay_plane[a];
            p.lay_row[a] = pl->lay_row[a];
        }
    }
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

// Launches the prepared passes of one adjoint (pass[a].n_pass_views == 0:
// no pass a): a single fused launch over cubic blocks when the block shape
// allows it, else one launch per pass axis, in axis order.
int launch_adjoint_passes(const AdjParams pass[3], const Geo &g, int64_t batch, bool two_d, int32_t in_dt, int shape,
                          hipStream_t st)
{
    hipError_t e;
    if (adjoint_fusable(two_d, shape)) {
        AdjFused f{};
        int32_t L, TS, TF;
        adjoint_shape(shape, L, TS, TF);
        for (int a = 0; a < 3; ++a) {
            f.pass[a] = pass[a];
            f.nb[a] = (g.n[a] + L - 1) / L;
        }
        f.batch = (int32_t)batch;
        if ((int64_t)f.nb[0] * f.nb[1] * f.nb[2] * batch > INT32_MAX)
            return fail(PN_EINVAL, "problem too large for one launch");
        if ((e = launch_adjoint_fused(f, in_dt, st)) != hipSuccess) return fail_hip(e, "adjoint launch");
        return PN_OK;
    }
    for (int a = 0; a < 3; ++a) {
        if (pass[a].n_pass_views == 0) continue;
        if ((e = launch_adjoint(pass[a], in_dt, shape, st)) != hipSuccess) return fail_hip(e, "adjoint launch");
    }
    return PN_OK;
}

// kunits of the adjoint: a flush period holds >= 256 units of its first
// batch's max|q ds| (and one view's worth at least), a power of two
float adjoint_kunits(const HostTables &t)
{
    float kunits = 256.0f;
    while (kunits < t.kmax) kunits *= 2.0f;
    return kunits;
}

// Parameters of the adjoint pass over dominant axis a (block shape L x TS x
// TF) of geometry g, with the device tables tab/tabf/views; cbox is set by
// the caller.
void adjoint_pass_params(const Geo &g, const HostTables &t, int a, int32_t L, int32_t TS, int32_t TF,
                         const ViewTab *tab, const ViewTabF *tabf, const int32_t *views, int64_t batch,
                         const void *sino, float *target, bool accumulate, AdjParams &p)
{
    const int f = a == 0 ? 1 : 0, sl = a == 2 ? 1 : 2;
    p = AdjParams{};
    p.tab = tab;
    p.tabf = tabf;
    p.kunits = adjoint_kunits(t);
    p.point_source = g.parallel ? 0 : 1;
    p.views = views;
    p.n_pass_views = (int32_t)t.pass_views[a].size();
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
    p.accumulate = accumulate ? 1 : 0;
    p.blocks_a = (g.n[a] + L - 1) / L;
    p.blocks_s = (g.n[sl] + TS - 1) / TS;
    p.blocks_f = (g.n[f] + TF - 1) / TF;
}

// Bytes of the candidate-box table of an adjoint pass.
size_t cbox_bytes(const AdjParams &p)
{
    return (size_t)p.blocks_a * p.blocks_s * p.blocks_f * p.n_pass_views * 8;
}

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
        bool fresh;
        int rc = ensure_buf(*pl, pl->acc, need, 0, false, st, "adjoint accumulator", fresh);
        if (rc) return rc;
        target = static_cast<float *>(pl->acc.ptr);
    }
    const bool two_d = g.ndim == 2;
    const int shape = two_d ? 0 : (force_shape ? force_shape : plan_adjoint_shape(pl));
    int32_t L, TS, TF;
    adjoint_shape(shape, L, TS, TF);
    int done = 0;
    for (int a = 0; a < 3; ++a) {
        AdjParams &p = job.pass[a];
        p = AdjParams{};
        if (pl->pass_views[a].empty()) continue;
        adjoint_pass_params(g, *pl, a, L, TS, TF, pl->d_tab, pl->d_tabf, pl->d_views[a], batch, sino, target,
                            done > 0, p);
        if (adjoint_blocks(p) > INT32_MAX) return fail(PN_EINVAL, "problem too large for one launch");
        // candidate boxes depend on the geometry and the block shape only:
        // built once per plan and shape (a kernel on the caller's stream)
        {
            bool fresh;
            int rc = ensure_buf(*pl, pl->cbox[a], cbox_bytes(p), shape, false, st, "candidate boxes", fresh);
            if (rc) return rc;
            if (fresh) {
                hipError_t e = launch_cbox(p, pl->d_axbox, L, TS, TF, static_cast<uint32_t *>(pl->cbox[a].ptr), st);
                if (e != hipSuccess) return fail_hip(e, "cbox launch");
            }
        }
        p.cbox = static_cast<const uint32_t *>(pl->cbox[a].ptr);
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
    if ((rc = get_plan(pg, st, &pl))) return rc;
    FwdJob job;
    bool none;
    if ((rc = forward_prepare(pg, batch, vol, sino, in_dt, out_dt, st, pl, job, none)) || none) return rc;
    auto run = [&](int vg) -> int {
        FwdParams p = job.p;
        p.view_group = vg;
        hipError_t e = launch_forward(p, in_dt, out_dt, st);
        return e == hipSuccess ? PN_OK : fail_hip(e, "forward launch");
    };
    if (!job.two_d && autotune_on()) {
        // views per workgroup: 3 (default) or 2, tuned once per plan
        if (pl->fwd_vg == 0) pl->fwd_vg = tune_cache_lookup(pl->g, "fwd", 2, 3);
        if (pl->fwd_vg == 0 && !capturing(st)) {
            int best = 0;
            if ((rc = time_variants({3, 2}, run, st, best))) return rc;
            pl->fwd_vg = best;
            tune_cache_store(pl->g, "fwd", best);
        }
        if (pl->fwd_vg) job.p.view_group = pl->fwd_vg;
    }
    return run(job.p.view_group);
}

// A with sampler interpolation: every tap gathered through the caches from
// the zero-bordered work copies (the ones pn_forward builds) or from the
// caller's volume with checked taps.
int forward_sampled_impl(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dt,
                         int32_t out_dt, int32_t source, int32_t wbits, hipStream_t st)
{
    if (source != PN_SAMPLE_BORDERED && source != PN_SAMPLE_DIRECT)
        return fail(PN_EINVAL, "pn_forward_sampled: unknown source %d", source);
    if (wbits < 0 || wbits > 16) return fail(PN_EINVAL, "pn_forward_sampled: weight_bits %d outside [0, 16]", wbits);
    Geo pre;
    int rc = preflight(pg, batch, vol, sino, in_dt, out_dt, false, pre);
    if (rc || batch == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, st, &pl))) return rc;
    const Geo &g = pl->g;
    if (g.n_views == 0) return PN_OK;
    SampParams p{};
    p.tab = pl->d_tab;
    p.n_views = g.n_views;
    p.nu = g.nu;
    p.nv = g.nv;
    p.batch = (int32_t)batch;
    p.bordered = source == PN_SAMPLE_BORDERED;
    p.weight_bits = wbits;
    p.point_source = g.parallel ? 0 : 1;
    const int64_t st3[3] = {1, (int64_t)g.n[0], (int64_t)g.n[0] * g.n[1]};
    for (int a = 0; a < 3; ++a) {
        p.n[a] = g.n[a];
        p.s[a] = g.s[a];
    }
    // every work copy is made ready before anything is launched, so a call
    // refused under capture enqueues nothing
    if (p.bordered)
        for (int a = 0; a < 3; ++a)
            if ((pl->axes_union >> a & 1) && (rc = ensure_work_copy(*pl, a, in_dt, batch, st))) return rc;
    for (int a = 0; a < 3; ++a) {
        if (!(pl->axes_union >> a & 1)) continue;
        const int f = a == 0 ? 1 : 0, sl = a == 2 ? 1 : 2;
        if (p.bordered) {
            p.item[a] = pl->lay_item[a];
            p.plane[a] = pl->lay_plane[a];
            p.row[a] = pl->lay_row[a];
            p.col[a] = 1;
            p.org[a] = (int64_t)PADR_LO * pl->lay_row[a] + PADC;
        } else {
            p.item[a] = st3[2] * g.n[2];
            p.plane[a] = st3[a];
            p.row[a] = st3[sl];
            p.col[a] = st3[f];
            p.org[a] = 0;
        }
        if (p.item[a] >= ((int64_t)1 << 31))
            return fail(PN_EINVAL, "pn_forward_sampled: image of %lld elements per batch item (limit 2^31 - 1)",
                        (long long)p.item[a]);
    }
    for (int a = 0; a < 3; ++a) {
        if (!(pl->axes_union >> a & 1)) continue;
        if (p.bordered) {
            hipError_t e = launch_relayout(in_dt, vol, pl->lay[a].ptr, g.n, a, (int32_t)batch, pl->lay_item[a],
                                           pl->lay_row[a], pl->lay_plane[a], st);
            if (e != hipSuccess) return fail_hip(e, "relayout launch");
            p.img[a] = pl->lay[a].ptr;
        } else {
            p.img[a] = vol;
        }
    }
    p.sino = sino;
    forward_sampled_tile(g.ndim == 2, p.tile_u, p.tile_v, p.view_group);
    p.tiles_u = (g.nu + p.tile_u - 1) / p.tile_u;
    p.tiles_v = (g.nv + p.tile_v - 1) / p.tile_v;
    if (forward_sampled_blocks(p) > INT32_MAX) return fail(PN_EINVAL, "problem too large for one launch");
    hipError_t e = launch_forward_sampled(p, in_dt, out_dt, st);
    return e == hipSuccess ? PN_OK : fail_hip(e, "sampled forward launch");
}

// The voxel-driven back-projection with sampler interpolation: every
// detector tap gathered through the caches from a zero-bordered copy of the
// sinogram (rows and columns padded by 1 before and 2 after) or from the
// caller's sinogram with checked taps.
int backproject_sampled_impl(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dt,
                             int32_t out_dt, int32_t source, int32_t wbits, hipStream_t st)
{
    if (source != PN_SAMPLE_BORDERED && source != PN_SAMPLE_DIRECT)
        return fail(PN_EINVAL, "pn_backproject_sampled: unknown source %d", source);
    if (wbits < 0 || wbits > 16)
        return fail(PN_EINVAL, "pn_backproject_sampled: weight_bits %d outside [0, 16]", wbits);
    Geo pre;
    int rc = preflight(pg, batch, sino, vol, in_dt, out_dt, true, pre);
    if (rc || batch == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, st, &pl))) return rc;
    const Geo &g = pl->g;
    BpSampParams p{};
    p.tabf = pl->d_tabf;
    p.n_views = g.n_views;
    p.nu = g.nu;
    p.nv = g.nv;
    p.batch = (int32_t)batch;
    for (int a = 0; a < 3; ++a) p.n[a] = g.n[a];
    p.weight_bits = wbits;
    p.vol = vol;
    // a call without views writes zeros and reads no image
    p.bordered = source == PN_SAMPLE_BORDERED && g.n_views > 0;
    if (p.bordered) {
        p.row = g.nu + 3;
        p.view = (int64_t)p.row * (g.nv + 3);
        p.item = p.view * g.n_views;
        p.org = (int64_t)p.row + 1;
        if (p.view >= ((int64_t)1 << 31))
            return fail(PN_EINVAL, "pn_backproject_sampled: padded view of %lld elements (limit 2^31 - 1)",
                        (long long)p.view);
        bool fresh;
        const size_t need = (size_t)(p.item * batch * esize(in_dt));
        if ((rc = ensure_buf(*pl, pl->spad, need, in_dt, true, st, "bordered sinogram", fresh))) return rc;
        hipError_t e = launch_pad_sino(in_dt, sino, pl->spad.ptr, batch * g.n_views, g.nv, g.nu, p.row, p.view, st);
        if (e != hipSuccess) return fail_hip(e, "sinogram border launch");
        p.img = pl->spad.ptr;
    } else {
        p.row = g.nu;
        p.view = (int64_t)g.nu * g.nv;
        p.item = p.view * g.n_views;
        p.org = 0;
        p.img = sino;
    }
    if (backproject_sampled_blocks(p) > INT32_MAX) return fail(PN_EINVAL, "problem too large for one launch");
    hipError_t e = launch_backproject_sampled(p, in_dt, out_dt, st);
    return e == hipSuccess ? PN_OK : fail_hip(e, "sampled back-projection launch");
}

int adjoint_impl(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dt, int32_t out_dt,
                 hipStream_t st)
{
    Geo pre;
    int rc = preflight(pg, batch, sino, vol, in_dt, out_dt, true, pre);
    if (rc || batch == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, st, &pl))) return rc;
    AdjJob job;
    bool none;
    auto run = [&](int force) -> int {
        int r = adjoint_prepare(batch, sino, vol, in_dt, out_dt, st, pl, job, none, force);
        if (r || none) return r;
        return launch_adjoint_passes(job.pass, pl->g, batch, job.two_d, in_dt, job.shape, st);
    };
    if (autotune_on() && pl->g.ndim == 3 && plan_adjoint_shape(pl) && pl->adj_shape == 0 && !capturing(st)) {
        // time every shape (each run overwrites the output), keep the fastest
        std::vector<int> vars;
        for (int k = 1; k < adjoint_shape_count(); ++k) vars.push_back(k);
        int best = 0;
        if ((rc = time_variants(vars, run, st, best))) return rc;
        pl->adj_shape = best;
        tune_cache_store(pl->g, "adj", best);
    }
    if ((rc = run(0)) || none) return rc;
    return adjoint_finish(job, st);
}

// ------------------------------------------- allocation-free adjoint ----
//
// pn_adjoint_noalloc keeps its device data in the library's fixed scratch
// array (scratch_address(), one per GPU) instead of a plan: the FP64 and
// FP32 view tables, the pass view lists, the axis boxes and the candidate
// boxes of each pass, then the FP32 accumulator of a 16-bit output.  The
// array keeps the last call's contents; the host remembers which geometry
// they belong to, per device, and re-uses them for the same geometry.

struct ScratchLayout {
    size_t tab = 0, tabf = 0, views[3] = {0, 0, 0}, axbox = 0, cbox[3] = {0, 0, 0}, acc = 0, end = 0;
};

struct NoallocState {
    bool valid = false;  // the array holds the tables and boxes of `g`
    Geo g;
    HostTables t;
    ScratchLayout lay;
};

std::mutex g_na_mu;
std::vector<NoallocState> g_na;  // per device

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int adjoint_noalloc_impl(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dt,
                         int32_t out_dt, hipStream_t st)
{
    Geo pre;
    int rc = preflight(pg, batch, sino, vol, in_dt, out_dt, true, pre);
    if (rc || batch == 0) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_na_mu);
    if ((size_t)dev >= g_na.size()) g_na.resize((size_t)dev + 1);
    NoallocState &ns = g_na[(size_t)dev];
    const bool two_d = pre.ndim == 2;
    const int shape = two_d ? 0 : adjoint_shape_3d();
    int32_t L, TS, TF;
    adjoint_shape(shape, L, TS, TF);
    const int64_t total = (int64_t)pre.n[0] * pre.n[1] * pre.n[2] * batch;
    const bool reuse = ns.valid && ns.g.same(pre);
    // host tables and the layout of the array (nothing is enqueued yet)
    HostTables fresh_t;
    ScratchLayout lay;
    const HostTables &t = reuse ? ns.t : fresh_t;
    if (reuse) {
        lay = ns.lay;
    } else {
        build_host_tables(pre, fresh_t);
        size_t off = 0;
        lay.tab = off;
        off = align256(off + sizeof(ViewTab) * t.tab.size());
        lay.tabf = off;
        off = align256(off + sizeof(ViewTabF) * t.tabf.size());
        for (int a = 0; a < 3; ++a) {
            lay.views[a] = off;
            off = align256(off + sizeof(int32_t) * t.pass_views[a].size());
        }
        lay.axbox = off;
        off = align256(off + sizeof(uint32_t) * t.axbox.size());
        for (int a = 0; a < 3; ++a) {
            lay.cbox[a] = off;
            if (t.pass_views[a].empty()) continue;
            AdjParams p;
            adjoint_pass_params(pre, t, a, L, TS, TF, nullptr, nullptr, nullptr, batch, sino, nullptr, false, p);
            off = align256(off + cbox_bytes(p));
        }
        lay.acc = off;
    }
    lay.end = lay.acc + (out_dt == PN_F32 ? 0 : (size_t)total * 4);
    if (lay.end > scratch_bytes())
        return fail(PN_EINVAL,
                    "pn_adjoint_noalloc: this geometry, batch and output type need %zu bytes of scratch; the "
                    "allocation-free entry point has %zu (use pn_adjoint)",
                    lay.end, scratch_bytes());
    if (!reuse && capturing(st))
        return fail(PN_EINVAL,
                    "pn_adjoint_noalloc: the stream is capturing and the scratch array does not hold this "
                    "geometry's tables: call it once eagerly with the same geometry first");
    void *base_v = nullptr;
    if ((e = scratch_address(&base_v)) != hipSuccess) return fail_hip(e, "scratch address");
    char *base = static_cast<char *>(base_v);
    const ViewTab *d_tab = reinterpret_cast<const ViewTab *>(base + lay.tab);
    const ViewTabF *d_tabf = reinterpret_cast<const ViewTabF *>(base + lay.tabf);
    if (!reuse) {
        // the host tables are pageable: HIP copies pageable host memory
        // synchronously, so they may go out of scope after the call
        ns.valid = false;
        auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
            if (bytes == 0) return hipSuccess;
            return hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, st);
        };
        if ((e = put(lay.tab, t.tab.data(), sizeof(ViewTab) * t.tab.size())) != hipSuccess ||
            (e = put(lay.tabf, t.tabf.data(), sizeof(ViewTabF) * t.tabf.size())) != hipSuccess ||
            (e = put(lay.axbox, t.axbox.data(), sizeof(uint32_t) * t.axbox.size())) != hipSuccess)
            return fail_hip(e, "table copy");
        for (int a = 0; a < 3; ++a)
            if ((e = put(lay.views[a], t.pass_views[a].data(), sizeof(int32_t) * t.pass_views[a].size())) !=
                hipSuccess)
                return fail_hip(e, "table copy");
        for (int a = 0; a < 3; ++a) {
            if (t.pass_views[a].empty()) continue;
            AdjParams p;
            adjoint_pass_params(pre, t, a, L, TS, TF, d_tab, d_tabf,
                                reinterpret_cast<const int32_t *>(base + lay.views[a]), batch, sino, nullptr, false, p);
            e = launch_cbox(p, reinterpret_cast<const uint32_t *>(base + lay.axbox), L, TS, TF,
                            reinterpret_cast<uint32_t *>(base + lay.cbox[a]), st);
            if (e != hipSuccess) return fail_hip(e, "cbox launch");
        }
        ns.g = pre;
        ns.t = std::move(fresh_t);
        ns.lay = lay;
        ns.valid = true;
    }
    const HostTables &tt = ns.t;
    int npass = 0;
    for (int a = 0; a < 3; ++a) npass += tt.pass_views[a].empty() ? 0 : 1;
    if (npass == 0) {
        e = launch_fill_zero(vol, total * esize(out_dt), st);
        return e == hipSuccess ? PN_OK : fail_hip(e, "fill");
    }
    float *target = out_dt == PN_F32 ? static_cast<float *>(vol) : reinterpret_cast<float *>(base + lay.acc);
    int done = 0;
    AdjParams pass[3] = {};
    for (int a = 0; a < 3; ++a) {
        if (tt.pass_views[a].empty()) continue;
        AdjParams &p = pass[a];
        adjoint_pass_params(pre, tt, a, L, TS, TF, d_tab, d_tabf,
                            reinterpret_cast<const int32_t *>(base + lay.views[a]), batch, sino, target, done > 0, p);
        if (adjoint_blocks(p) > INT32_MAX) return fail(PN_EINVAL, "problem too large for one launch");
        p.cbox = reinterpret_cast<const uint32_t *>(base + lay.cbox[a]);
        ++done;
    }
    if ((rc = launch_adjoint_passes(pass, pre, batch, two_d, in_dt, shape, st))) return rc;
    if (out_dt != PN_F32 && (e = launch_convert(target, vol, out_dt, total, st)) != hipSuccess)
        return fail_hip(e, "convert launch");
    return PN_OK;
}

int backproject_impl(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dt,
                     int32_t out_dt, hipStream_t st)
{
    Geo pre;
    int rc = preflight(pg, batch, sino, vol, in_dt, out_dt, true, pre);
    if (rc || batch == 0) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, st, &pl))) return rc;
    BpJob job;
    backproject_prepare(batch, sino, vol, pl, job);
    auto run = [&](int bz) -> int {
        BpParams p = job.p;
        p.bz = bz;
        hipError_t e = launch_backproject(p, in_dt, out_dt, st);
        return e == hipSuccess ? PN_OK : fail_hip(e, "backproject launch");
    };
    if (!job.two_d && autotune_on()) {
        // block depth along z: 16 (default), 8 or 32, tuned once per plan
        if (pl->bp_bz == 0) pl->bp_bz = tune_cache_lookup(pl->g, "bp", 8, 32);
        if (pl->bp_bz == 0 && !capturing(st)) {
            int best = 0;
            if ((rc = time_variants({16, 8, 32}, run, st, best))) return rc;
            pl->bp_bz = best;
            tune_cache_store(pl->g, "bp", best);
        }
        job.p.bz = pl->bp_bz;
    }
    return run(job.p.bz);
}

int splat_impl(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dt, int32_t out_dt,
               hipStream_t st)
{
    Geo pre;
    int rc = preflight(pg, batch, vol, sino, in_dt, out_dt, false, pre);
    if (rc || batch == 0) return rc;
    if (pre.n_views == 0) return PN_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *pl;
    if ((rc = get_plan(pg, st, &pl))) return rc;
    const Geo &g = pl->g;
    const int64_t total = (int64_t)g.n_views * g.nv * g.nu * batch;
    float *target = static_cast<float *>(sino);
    if (out_dt != PN_F32) {
        bool fresh;
        if ((rc = ensure_buf(*pl, pl->sacc, (size_t)total * 4, 0, false, st, "splat accumulator", fresh))) return rc;
        target = static_cast<float *>(pl->sacc.ptr);
    }
    SplatParams p{};
    p.tabf = pl->d_tabf;
    p.n_views = g.n_views;
    p.nu = g.nu;
    p.nv = g.nv;
    p.batch = (int32_t)batch;
    for (int a = 0; a < 3; ++a) p.n[a] = g.n[a];
    p.vol = vol;
    p.sino = target;
    if (splat_blocks(p) > INT32_MAX) return fail(PN_EINVAL, "problem too large for one launch");
    hipError_t e = launch_fill_zero(target, total * 4, st);
    if (e != hipSuccess) return fail_hip(e, "fill");
    if ((e = launch_splat(p, in_dt, st)) != hipSuccess) return fail_hip(e, "splat launch");
    if (out_dt != PN_F32 && (e = launch_convert(target, sino, out_dt, total, st)) != hipSuccess)
        return fail_hip(e, "convert launch");
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
    if ((rc = get_plan(pg, st, &pl))) return rc;
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
            std::string msg = pn_last_error();
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
int run_batched(const pn_problem *probs, const std::vector<int32_t> &order, hipStream_t st, Prepare prepare,
                Launch launch)
{
    std::vector<int32_t> pending;
    std::vector<Plan *> plans;
    for (int32_t i : order) {
        Plan *pl;
        int rc = get_plan(&probs[i].geom, st, &pl);
        if (rc) {
            std::string msg = pn_last_error();
            return fail(rc, "problem %d: %s", i, msg.c_str());
        }
        const bool seen = std::find(plans.begin(), plans.end(), pl) != plans.end();
        if (seen || (int)pending.size() == kMaxBatch) {
            if ((rc = launch(pending))) return rc;
            pending.clear();
            plans.clear();
        }
        if ((rc = prepare(i, pl))) {
            std::string msg = pn_last_error();
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
    return run_batched(probs, order, st, prepare, launch);
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
    return run_batched(probs, order, st, prepare, launch);
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
    return run_batched(probs, order, st, prepare, launch);
}

// ------------------------------------------------------- batch plans -----
//
// A batch plan fixes a problem set (geometries, buffers, types) once:
// its plans are pinned and referenced, every kernel group of the operator
// runs as ONE launch over a work list in device memory (largest problems
// first), and the whole operator -- relayouts, fills, candidate tables,
// main kernels, 16-bit conversions -- is captured in a HIP graph on a
// library stream, which pn_batch_run replays on the caller's stream.
// Problems that share a plan (same geometry) share its work buffers, so
// they go to successive groups, each group its own set of launches.

enum TableKind { TK_FWD = 0, TK_ADJ = 1, TK_FUSED = 2, TK_BP = 3 };

struct TableSlice {
    int kind = 0;
    bool two_d = false;
    int axis = 0, shape = 0;
    size_t off_p = 0, off_start = 0;  // byte offsets in the device table
    int32_t n = 0;
    uint32_t blocks = 0;
};

struct BatchGroup {
    std::vector<int32_t> probs;       // problem indices, largest first
    std::vector<TableSlice> slices;
};

}  // namespace

struct pn_batch {
    int32_t op = 0, in_dt = 0, out_dt = 0;
    int device = 0;
    std::vector<pn_problem> probs;
    std::vector<Plan *> plans;         // per problem
    std::vector<BatchGroup> groups;
    std::vector<unsigned char> host_table;
    void *d_table = nullptr;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <typename P>
void append_list(std::vector<unsigned char> &buf, const std::vector<P> &items, const std::vector<uint32_t> &start,
                 TableSlice &sl)
{
    auto align = [&](size_t a) { buf.resize((buf.size() + a - 1) / a * a); };
    align(256);
    sl.off_p = buf.size();
    buf.resize(buf.size() + sizeof(P) * items.size());
    std::memcpy(buf.data() + sl.off_p, items.data(), sizeof(P) * items.size());
    align(16);
    sl.off_start = buf.size();
    buf.resize(buf.size() + sizeof(uint32_t) * start.size());
    std::memcpy(buf.data() + sl.off_start, start.data(), sizeof(uint32_t) * start.size());
    sl.n = (int32_t)items.size();
    sl.blocks = start.back();
}

// Work list of `items` with blocks(item) workgroups each, problems starting
// at multiples of `align`.
template <typename P, typename BlocksFn>
int list_starts(const std::vector<P> &items, BlocksFn blocks, int64_t align, std::vector<uint32_t> &start)
{
    start.assign(1, 0u);
    int64_t at = 0;
    for (const P &p : items) {
        at += (blocks(p) + align - 1) / align * align;
        if (at > INT32_MAX) return fail(PN_EINVAL, "batch plan: a kernel group is too large for one launch");
        start.push_back((uint32_t)at);
    }
    return PN_OK;
}

// Prepares every problem of batch plan B on stream st (enqueueing its
// relayouts, fills and candidate tables) and either records the kernel
// groups' work lists into B.host_table (build) or launches them from the
// device table (!build).  The prepared parameters must be the same in both
// phases: they depend only on the pinned plans and the fixed buffers.
int batch_enqueue(pn_batch &B, hipStream_t st, bool build)
{
    const int n = (int)B.probs.size();
    std::vector<FwdJob> fj(B.op == PN_OP_FORWARD ? n : 0);
    std::vector<AdjJob> aj(B.op == PN_OP_ADJOINT ? n : 0);
    std::vector<BpJob> bj(B.op == PN_OP_BACKPROJECT ? n : 0);
    if (build) B.host_table.clear();
    char *dt = static_cast<char *>(B.d_table);
    for (BatchGroup &G : B.groups) {
        std::vector<char> live(n, 0);
        for (int32_t i : G.probs) {
            const pn_problem &pr = B.probs[i];
            bool none = false;
            int rc = PN_OK;
            if (B.op == PN_OP_FORWARD)
                rc = forward_prepare(&pr.geom, 1, pr.in, pr.out, B.in_dt, B.out_dt, st, B.plans[i], fj[i], none);
            else if (B.op == PN_OP_ADJOINT)
                rc = adjoint_prepare(1, pr.in, pr.out, B.in_dt, B.out_dt, st, B.plans[i], aj[i], none);
            else
                backproject_prepare(1, pr.in, pr.out, B.plans[i], bj[i]);
            if (rc) {
                std::string msg = pn_last_error();
                return fail(rc, "batch plan, problem %d: %s", i, msg.c_str());
            }
            live[i] = !none;
        }
        if (build) G.slices.clear();
        size_t k = 0;  // slice index within the group (launch phase)
        auto take = [&](int kind, bool two_d, int axis, int shape) -> TableSlice * {
            if (build) {
                G.slices.push_back(TableSlice{});
                TableSlice &sl = G.slices.back();
                sl.kind = kind;
                sl.two_d = two_d;
                sl.axis = axis;
                sl.shape = shape;
                return &sl;
            }
            if (k >= G.slices.size()) return nullptr;
            TableSlice &sl = G.slices[k++];
            if (sl.kind != kind || sl.two_d != two_d || sl.axis != axis || sl.shape != shape) return nullptr;
            return &sl;
        };
        auto mismatch = [] { return fail(PN_EINVAL, "batch plan: prepared state changed between build and capture"); };
        // one list: the items it would hold, checked against (or recorded
        // into) the table, then launched from the device table
        auto list = [&](auto items, auto blocks, int64_t align, int kind, bool two_d, int axis, int shape,
                        auto launch) -> int {
            using P = typename decltype(items)::value_type;
            if (items.empty()) return PN_OK;
            std::vector<uint32_t> start;
            int r = list_starts(items, blocks, align, start);
            if (r) return r;
            TableSlice *sl = take(kind, two_d, axis, shape);
            if (!sl) return mismatch();
            if (build) {
                append_list(B.host_table, items, start, *sl);
                return PN_OK;
            }
            if (sl->n != (int32_t)items.size() || sl->blocks != start.back() ||
                std::memcmp(B.host_table.data() + sl->off_p, items.data(), sizeof(P) * items.size()) != 0)
                return mismatch();
            Table<P> w;
            w.p = reinterpret_cast<const P *>(dt + sl->off_p);
            w.start = reinterpret_cast<const uint32_t *>(dt + sl->off_start);
            w.n = sl->n;
            hipError_t e = launch(w, sl->blocks);
            return e == hipSuccess ? PN_OK : fail_hip(e, "batch plan launch");
        };
        int rc = PN_OK;
        if (B.op == PN_OP_FORWARD) {
            for (int td = 0; td < 2 && !rc; ++td) {
                std::vector<FwdParams> items;
                for (int32_t i : G.probs)
                    if (live[i] && fj[i].two_d == (td != 0)) items.push_back(fj[i].p);
                rc = list(items, [](const FwdParams &p) { return forward_blocks(p); }, 8, TK_FWD, td != 0, 0, 0,
                          [&](const Table<FwdParams> &w, uint32_t blocks) {
                              return launch_forward_table(w, blocks, td != 0, B.in_dt, B.out_dt, st);
                          });
            }
        } else if (B.op == PN_OP_ADJOINT) {
            std::vector<AdjFused> fused;
            for (int32_t i : G.probs) {
                if (!live[i] || !adjoint_fusable(aj[i].two_d, aj[i].shape)) continue;
                const Geo &g = B.plans[i]->g;
                AdjFused f{};
                int32_t L, TS, TF;
                adjoint_shape(aj[i].shape, L, TS, TF);
                for (int a = 0; a < 3; ++a) {
                    f.pass[a] = aj[i].pass[a];
                    f.nb[a] = (g.n[a] + L - 1) / L;
                }
                f.batch = 1;
                fused.push_back(f);
            }
            rc = list(fused, [](const AdjFused &f) { return (int64_t)f.nb[0] * f.nb[1] * f.nb[2] * f.batch; }, 1,
                      TK_FUSED, false, 0, 0, [&](const Table<AdjFused> &w, uint32_t blocks) {
                          return launch_adjoint_fused_table(w, blocks, B.in_dt, st);
                      });
            // passes in axis order: a problem's later passes add to its earlier ones
            for (int a = 0; a < 3 && !rc; ++a)
                for (int shape = 0; shape < adjoint_shape_count() && !rc; ++shape) {
                    std::vector<AdjParams> items;
                    for (int32_t i : G.probs)
                        if (live[i] && !adjoint_fusable(aj[i].two_d, aj[i].shape) && aj[i].shape == shape &&
                            aj[i].pass[a].n_pass_views > 0)
                            items.push_back(aj[i].pass[a]);
                    rc = list(items, [](const AdjParams &p) { return adjoint_blocks(p); }, 1, TK_ADJ, false, a,
                              shape, [&](const Table<AdjParams> &w, uint32_t blocks) {
                                  return launch_adjoint_table(w, blocks, a, B.in_dt, shape, st);
                              });
                }
            for (int32_t i : G.probs)
                if (!rc && live[i]) rc = adjoint_finish(aj[i], st);
        } else {
            for (int td = 0; td < 2 && !rc; ++td) {
                std::vector<BpParams> items;
                for (int32_t i : G.probs)
                    if (bj[i].two_d == (td != 0)) items.push_back(bj[i].p);
                rc = list(items, [](const BpParams &p) { return backproject_blocks(p); }, 1, TK_BP, td != 0, 0, 0,
                          [&](const Table<BpParams> &w, uint32_t blocks) {
                              return launch_backproject_table(w, blocks, td != 0, B.in_dt, B.out_dt, st);
                          });
            }
        }
        if (rc) return rc;
        if (!build && k != G.slices.size()) return mismatch();
    }
    return PN_OK;
}

void batch_free(pn_batch *B)
{
    if (!B) return;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->cs) (void)hipStreamDestroy(B->cs);
    dev_free(B->d_table);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (Plan *pl : B->plans)
            if (pl) --pl->refs;
        --g_live_batches;
    }
    delete B;
}

int batch_create(int32_t op, const pn_problem *probs, int32_t n, int32_t in_dt, int32_t out_dt, pn_batch **out)
{
    if (!out) return fail(PN_EINVAL, "pn_batch_create: output pointer is NULL");
    *out = nullptr;
    if (op != PN_OP_FORWARD && op != PN_OP_ADJOINT && op != PN_OP_BACKPROJECT)
        return fail(PN_EINVAL, "pn_batch_create: unknown operator %d", op);
    std::vector<int32_t> order;
    int rc = batch_order(probs, n, in_dt, out_dt, op != PN_OP_FORWARD, order);
    if (rc) return rc;
    if (n == 0) return fail(PN_EINVAL, "pn_batch_create: no problems");
    auto *B = new pn_batch();
    B->op = op;
    B->in_dt = in_dt;
    B->out_dt = out_dt;
    B->probs.assign(probs, probs + n);
    B->plans.assign(n, nullptr);
    hipError_t e = hipGetDevice(&B->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->cs, hipStreamNonBlocking);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ++g_live_batches;
    }
    if (e != hipSuccess) {
        batch_free(B);
        return fail_hip(e, "pn_batch_create");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        std::vector<Plan *> in_group;
        for (int32_t i : order) {
            Plan *pl;
            if ((rc = get_plan(&B->probs[i].geom, B->cs, &pl))) {
                std::string msg = pn_last_error();
                rc = fail(rc, "problem %d: %s", i, msg.c_str());
                break;
            }
            ++pl->refs;
            B->plans[i] = pl;
            if (B->groups.empty() || std::find(in_group.begin(), in_group.end(), pl) != in_group.end()) {
                B->groups.emplace_back();
                in_group.clear();
            }
            B->groups.back().probs.push_back(i);
            in_group.push_back(pl);
        }
        // build: every buffer and candidate table is made on the library
        // stream (eagerly), and the work lists are recorded
        if (!rc) rc = batch_enqueue(*B, B->cs, true);
    }
    if (!rc && (e = hipStreamSynchronize(B->cs)) != hipSuccess) rc = fail_hip(e, "pn_batch_create");
    if (!rc && (e = hipMalloc(&B->d_table, std::max<size_t>(B->host_table.size(), 256))) != hipSuccess)
        rc = fail(PN_ENOMEM, "pn_batch_create: hipMalloc(%zu) failed", B->host_table.size());
    if (!rc && !B->host_table.empty() &&
        (e = hipMemcpy(B->d_table, B->host_table.data(), B->host_table.size(), hipMemcpyHostToDevice)) != hipSuccess)
        rc = fail_hip(e, "pn_batch_create: table copy");
    if (!rc) {
        // capture the operator on the library stream
        if ((e = hipStreamBeginCapture(B->cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            rc = fail_hip(e, "pn_batch_create: begin capture");
        } else {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                rc = batch_enqueue(*B, B->cs, false);
            }
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(B->cs, &g);
            B->graph = g;
            if (!rc && e != hipSuccess) rc = fail_hip(e, "pn_batch_create: end capture");
            if (!rc && (e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0)) != hipSuccess)
                rc = fail_hip(e, "pn_batch_create: graph instantiation");
        }
    }
    if (rc) {
        std::string msg = pn_last_error();
        batch_free(B);
        return fail(rc, "%s", msg.c_str());
    }
    *out = B;
    return PN_OK;
}

int batch_run(pn_batch *B, hipStream_t st)
{
    if (!B) return fail(PN_EINVAL, "pn_batch_run: batch plan is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != B->device) return fail(PN_EINVAL, "pn_batch_run: the batch plan belongs to device %d", B->device);
    if ((e = hipGraphLaunch(B->exec, st)) != hipSuccess) return fail_hip(e, "pn_batch_run: graph launch");
    return PN_OK;
}

}  // namespace

// ==================================================== extern "C" ABI =====

extern "C" {

int pn_forward(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dtype,
               int32_t out_dtype, void *hip_stream)
{
    clear_error();
    return forward_impl(pg, batch, vol, sino, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_forward_sampled(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dtype,
                       int32_t out_dtype, int32_t source, int32_t weight_bits, void *hip_stream)
{
    clear_error();
    return forward_sampled_impl(pg, batch, vol, sino, in_dtype, out_dtype, source, weight_bits,
                                static_cast<hipStream_t>(hip_stream));
}

int pn_backproject_sampled(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dtype,
                           int32_t out_dtype, int32_t source, int32_t weight_bits, void *hip_stream)
{
    clear_error();
    return backproject_sampled_impl(pg, batch, sino, vol, in_dtype, out_dtype, source, weight_bits,
                                    static_cast<hipStream_t>(hip_stream));
}

int pn_adjoint(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dtype,
               int32_t out_dtype, void *hip_stream)
{
    clear_error();
    return adjoint_impl(pg, batch, sino, vol, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_adjoint_noalloc(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dtype,
                       int32_t out_dtype, void *hip_stream)
{
    clear_error();
    return adjoint_noalloc_impl(pg, batch, sino, vol, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_backproject(const pn_geometry *pg, int64_t batch, const void *sino, void *vol, int32_t in_dtype,
                   int32_t out_dtype, void *hip_stream)
{
    clear_error();
    return backproject_impl(pg, batch, sino, vol, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_splat(const pn_geometry *pg, int64_t batch, const void *vol, void *sino, int32_t in_dtype, int32_t out_dtype,
             void *hip_stream)
{
    clear_error();
    return splat_impl(pg, batch, vol, sino, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_filter(const pn_geometry *pg, int64_t batch, const void *sino, void *out, int32_t in_dtype,
              int32_t out_dtype, int32_t kind, void *hip_stream)
{
    clear_error();
    return filter_impl(pg, batch, sino, out, in_dtype, out_dtype, kind, static_cast<hipStream_t>(hip_stream));
}

int pn_gaussian_noise(int64_t n, void *data, int32_t dtype, double mean, double sigma, uint64_t seed,
                      void *hip_stream)
{
    clear_error();
    return noise_impl(n, data, dtype, mean, sigma, seed, static_cast<hipStream_t>(hip_stream));
}

int pn_gantry_blur(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, const void *in, void *out,
                   int32_t dtype, double angle_start, double angle_step, int32_t taps, void *hip_stream)
{
    clear_error();
    return blur_impl(batch, n_views, rows, cols, in, out, dtype, angle_start, angle_step, taps,
                     static_cast<hipStream_t>(hip_stream));
}

int pn_detector_jitter(int64_t n_rows, int32_t cols, const void *in, void *out, int32_t dtype, int32_t max_shift,
                       uint64_t seed, void *hip_stream)
{
    clear_error();
    return jitter_impl(n_rows, cols, in, out, dtype, max_shift, seed, static_cast<hipStream_t>(hip_stream));
}

int pn_ring_artifacts(int64_t batch, int32_t n_views, int32_t rows, int32_t cols, void *sino, int32_t dtype,
                      const int32_t *columns, int32_t n_columns, double gain, int32_t v0, int32_t v1,
                      void *hip_stream)
{
    clear_error();
    return ring_impl(batch, n_views, rows, cols, sino, dtype, columns, n_columns, gain, v0, v1,
                     static_cast<hipStream_t>(hip_stream));
}

int pn_forward_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype, void *hip_stream)
{
    clear_error();
    return forward_batched(probs, n, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_adjoint_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype, void *hip_stream)
{
    clear_error();
    return adjoint_batched(probs, n, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_backproject_batched(const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype,
                           void *hip_stream)
{
    clear_error();
    return backproject_batched(probs, n, in_dtype, out_dtype, static_cast<hipStream_t>(hip_stream));
}

int pn_batch_create(int32_t op, const pn_problem *probs, int32_t n, int32_t in_dtype, int32_t out_dtype,
                    pn_batch **out)
{
    clear_error();
    return batch_create(op, probs, n, in_dtype, out_dtype, out);
}

int pn_batch_run(pn_batch *b, void *hip_stream)
{
    clear_error();
    return batch_run(b, static_cast<hipStream_t>(hip_stream));
}

int pn_batch_destroy(pn_batch *b)
{
    clear_error();
    batch_free(b);
    return PN_OK;
}

int pn_release_caches(void)
{
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    // plans and retired buffers that live batch plans' graphs use stay
    g_plans.remove_unless([](const Plan &p) { return p.refs > 0; });
    if (g_live_batches == 0) g_keeper.release_retired();
    return PN_OK;
}

const char *pn_version(void) { return "pyronn_mi 0.2.0 (gfx950)"; }

}  // extern "C"
