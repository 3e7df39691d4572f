// Host-side internals of the CT projector library that need no device:
// errors, argument and geometry validation, FP64 per-view tables and the
// projection-matrix composition (pn_geometry.cpp), shared by the device
// code in pn_host.cpp and by the CPU sanitizer build of the tests.  Not
// part of the public ABI.
#pragma once

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pyronn_mi.h"
#include "pn_common.hpp"

namespace pn {

// Sets the calling thread's last-error text (printf format) and returns code.
int fail(int code, const char *fmt, ...);
// Clears the calling thread's last-error text.
void clear_error();

int64_t esize(int32_t dt);
bool dtype_ok(int32_t dt);
bool inv3(const double m[9], double r[9]);

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

int normalise_geometry(const pn_geometry *pg, Geo &g);

// Per-geometry host tables: FP64 ray tables and FP32 projection tables per
// view, the dominant axes that occur, and detector windows.
struct HostTables {
    std::vector<ViewTab> tab;
    std::vector<ViewTabF> tabf;
    int32_t axes_union = 0;
    std::vector<int32_t> pass_views[3];  // views whose rays may have dominant axis a
    // largest per-view bound on the rays that sample one voxel's neighbourhood
    float kmax = 1.0f;
    // detector window that holds every ray meeting the dilated volume in
    // some view (inclusive pixel bounds; c0 > c1: no ray meets it)
    int32_t win_c0 = 0, win_c1 = -1, win_r0 = 0, win_r1 = -1;
    // the same per view (c0, c1, r0, r1)
    std::vector<int32_t> vwin;
    // per view and axis: detector box of the pixels whose ray may have that
    // dominant axis (axis_mask)
    std::vector<uint32_t> axbox;
};

int32_t axis_mask(const double A[9], int32_t nu, int32_t nv, uint32_t box[3][2]);
double cell_ray_bound(const double *Pi, const Geo &g);
void build_host_tables(const Geo &g, HostTables &t);

int check_ptr(const void *p, int32_t dt, const char *name);
int common_checks(int64_t batch, int32_t in_dt, int32_t out_dt);
int buffer_checks(const void *in, bool in_empty, const void *out, bool out_empty, int32_t in_dt, int32_t out_dt);
int preflight(const pn_geometry *pg, int64_t batch, const void *in, const void *out, int32_t in_dt, int32_t out_dt,
              bool sino_is_input, Geo &g);

}  // namespace pn
