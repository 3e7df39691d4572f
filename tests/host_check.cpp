// CPU check of the library's host logic, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py (no device):
//   * the cached-memory rules of pn_cache.hpp with a counting fake
//     allocator: buffers of plans used under graph capture are never freed
//     or re-purposed before release, pinned plans are never evicted, and
//     nothing leaks or is freed twice;
//   * argument and geometry validation, the per-view tables and the
//     projection-matrix composition entry points (pn_geometry.cpp).
// Prints "host_check OK" and exits 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <vector>

#include "../paper_2511_08427_amd/csrc/pn_cache.hpp"
#include "../paper_2511_08427_amd/csrc/pn_internal.hpp"

#define CHECK(c)                                                                       \
    do {                                                                               \
        if (!(c)) {                                                                    \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

// ------------------------------------------------------- fake allocator --

struct FakeMem {
    static std::map<void *, size_t> live;
    static int allocs, frees, fail_next;
    static bool alloc(void **p, size_t n)
    {
        if (fail_next) {
            --fail_next;
            return false;
        }
        *p = std::malloc(n);
        live[*p] = n;
        ++allocs;
        return true;
    }
    static void release(void *p)
    {
        CHECK(live.count(p) == 1);  // no double or foreign free
        live.erase(p);
        std::free(p);
        ++frees;
    }
};
std::map<void *, size_t> FakeMem::live;
int FakeMem::allocs = 0, FakeMem::frees = 0, FakeMem::fail_next = 0;

using Keeper = pn::BufferKeeper<FakeMem>;

struct FakePlan {
    int key = 0;
    bool pinned = false;
    bool held() const { return pinned; }
    pn::DevBuf buf;
    Keeper *keeper = nullptr;
    ~FakePlan() { keeper->free(buf); }
};

void check_buffers()
{
    using pn::Ensure;
    Keeper k;
    pn::DevBuf b;
    CHECK(k.ensure(b, 100, 0, false, false) == Ensure::kFresh);
    void *first = b.ptr;
    CHECK(k.ensure(b, 100, 0, false, false) == Ensure::kReady);
    CHECK(k.ensure(b, 50, 0, false, false) == Ensure::kReady && b.ptr == first);
    // unpinned: a new layout re-uses the memory, a larger size replaces it
    CHECK(k.ensure(b, 80, 1, false, false) == Ensure::kFresh && b.ptr == first && b.tag == 1);
    CHECK(k.ensure(b, 200, 1, false, false) == Ensure::kFresh && b.ptr != first);
    CHECK(FakeMem::live.size() == 1);
    // under capture nothing changes
    void *cur = b.ptr;
    CHECK(k.ensure(b, 400, 1, false, true) == Ensure::kCapturing && b.ptr == cur && b.cap == 200);
    CHECK(k.ensure(b, 150, 2, false, true) == Ensure::kCapturing && b.tag == 1);
    CHECK(k.ensure(b, 150, 1, true, true) == Ensure::kReady);
    // pinned: growing or a new layout retires the old memory, which stays allocated
    CHECK(k.ensure(b, 400, 1, true, false) == Ensure::kFresh && b.ptr != cur);
    CHECK(FakeMem::live.count(cur) == 1 && k.retired() == 1);
    void *cur2 = b.ptr;
    CHECK(k.ensure(b, 100, 3, true, false) == Ensure::kFresh && b.ptr != cur2 && FakeMem::live.count(cur2) == 1);
    CHECK(k.retired() == 2 && FakeMem::live.size() == 3);
    // a failed allocation leaves the buffer as it was
    void *cur3 = b.ptr;
    FakeMem::fail_next = 1;
    CHECK(k.ensure(b, 1000, 3, true, false) == Ensure::kNoMem && b.ptr == cur3 && b.cap == 100 && b.tag == 3);
    k.release_retired();
    CHECK(k.retired() == 0 && FakeMem::live.size() == 1 && FakeMem::live.count(cur3) == 1);
    k.free(b);
    CHECK(b.ptr == nullptr && FakeMem::live.empty());
}

void check_plans()
{
    Keeper k;
    pn::PlanLru<FakePlan> lru;
    std::vector<void *> pinned_bufs;
    for (int i = 0; i < 40; ++i) {
        auto p = std::make_unique<FakePlan>();
        p->key = i;
        p->keeper = &k;
        CHECK(k.ensure(p->buf, 64 + i, 0, false, false) == pn::Ensure::kFresh);
        if (i == 3 || i == 5) {
            p->pinned = true;
            pinned_bufs.push_back(p->buf.ptr);
        }
        lru.insert(std::move(p), 32);
        CHECK(lru.size() <= 32);
    }
    // pinned plans 3 and 5 are older than every other survivor but stay
    CHECK(lru.find([](const FakePlan &p) { return p.key == 3; }) != nullptr);
    CHECK(lru.find([](const FakePlan &p) { return p.key == 5; }) != nullptr);
    CHECK(lru.find([](const FakePlan &p) { return p.key == 9; }) == nullptr);  // evicted
    CHECK(lru.find([](const FakePlan &p) { return p.key == 10; }) != nullptr);
    for (void *q : pinned_bufs) CHECK(FakeMem::live.count(q) == 1);
    CHECK(FakeMem::live.size() == 32);
    // a limit no unpinned plan can satisfy: the pinned ones remain
    lru.trim(0);
    CHECK(lru.size() == 2);
    lru.clear();
    CHECK(FakeMem::live.empty());

    // every plan held: the list grows past its limit, and a new plan is
    // never evicted by its own insertion (its pointer stays valid)
    for (int i = 0; i < 40; ++i) {
        auto p = std::make_unique<FakePlan>();
        p->key = 100 + i;
        p->keeper = &k;
        CHECK(k.ensure(p->buf, 16, 0, false, false) == pn::Ensure::kFresh);
        FakePlan *q = lru.insert(std::move(p), 32);
        CHECK(q->key == 100 + i && FakeMem::live.count(q->buf.ptr) == 1);
        CHECK(lru.find([i](const FakePlan &f) { return f.key == 100 + i; }) == q);
        q->pinned = true;
    }
    CHECK(lru.size() == 40);
    // one unheld plan among held ones survives its insertion, and the next
    // insertion evicts it
    {
        auto p = std::make_unique<FakePlan>();
        p->key = 500;
        p->keeper = &k;
        CHECK(k.ensure(p->buf, 16, 0, false, false) == pn::Ensure::kFresh);
        CHECK(lru.insert(std::move(p), 32)->key == 500);
        auto r = std::make_unique<FakePlan>();
        r->key = 501;
        r->keeper = &k;
        CHECK(k.ensure(r->buf, 16, 0, false, false) == pn::Ensure::kFresh);
        CHECK(lru.insert(std::move(r), 32)->key == 501);
        CHECK(lru.find([](const FakePlan &f) { return f.key == 500; }) == nullptr);
        CHECK(lru.find([](const FakePlan &f) { return f.key == 501; }) != nullptr);
    }
    lru.remove_unless([](const FakePlan &f) { return f.key % 2 == 0; });
    CHECK(lru.size() == 20);
    lru.clear();
    CHECK(FakeMem::live.empty());
}

// ------------------------------------------------------ geometry ABI ------

pn_geometry cone(int64_t nz, int64_t ny, int64_t nx, int64_t rows, int64_t cols, std::vector<double> &P, int nviews)
{
    std::vector<double> S(3 * nviews), C(3 * nviews), eu(3 * nviews), ev(3 * nviews);
    for (int k = 0; k < nviews; ++k) {
        const double b = 2 * M_PI * k / nviews, c = std::cos(b), s = std::sin(b);
        S[3 * k] = 750 * c, S[3 * k + 1] = 750 * s, S[3 * k + 2] = 0;
        C[3 * k] = -450 * c, C[3 * k + 1] = -450 * s, C[3 * k + 2] = 0;
        eu[3 * k] = -s, eu[3 * k + 1] = c, eu[3 * k + 2] = 0;
        ev[3 * k] = 0, ev[3 * k + 1] = 0, ev[3 * k + 2] = 1;
    }
    P.assign(12 * nviews, 0.0);
    CHECK(pn_cone_matrices(nviews, S.data(), C.data(), eu.data(), ev.data(), rows, cols, P.data()) == PN_OK);
    pn_geometry g{};
    g.ndim = 3;
    g.beam = PN_CONE;
    g.vol_shape[0] = nz, g.vol_shape[1] = ny, g.vol_shape[2] = nx;
    for (int a = 0; a < 3; ++a) g.vol_spacing[a] = 0.5, g.vol_origin[a] = NAN;
    g.det_shape[0] = rows, g.det_shape[1] = cols;
    g.det_spacing[0] = g.det_spacing[1] = 1.0;
    g.sid = 750, g.sdd = 1200;
    g.n_views = nviews;
    g.proj = P.data();
    return g;
}

void check_geometry()
{
    std::vector<double> P;
    pn_geometry g = cone(20, 30, 40, 25, 35, P, 12);
    CHECK(pn_check_geometry(&g) == PN_OK);
    // P [S; 1] = 0 and the centre pixel's ray passes the isocentre
    for (int k = 0; k < 12; ++k) {
        const double *p = &P[12 * k];
        const double b = 2 * M_PI * k / 12, S[3] = {750 * std::cos(b), 750 * std::sin(b), 0};
        for (int r = 0; r < 3; ++r) CHECK(std::fabs(p[4 * r] * S[0] + p[4 * r + 1] * S[1] + p[4 * r + 2] * S[2] + p[4 * r + 3]) < 1e-9);
        CHECK(std::fabs(p[3] / p[11] - 17.0) < 1e-9 && std::fabs(p[7] / p[11] - 12.0) < 1e-9);
    }
    pn::Geo ng;
    CHECK(pn::normalise_geometry(&g, ng) == PN_OK);
    pn::HostTables t;
    pn::build_host_tables(ng, t);
    CHECK((int)t.tab.size() == 12 && (int)t.tabf.size() == 12 && t.vwin.size() == 48 && t.axbox.size() == 72);
    CHECK(t.axes_union == 3);  // x and y dominate in turn, z never (cone half-angle < 45 deg)
    CHECK(t.pass_views[2].empty() && !t.pass_views[0].empty() && !t.pass_views[1].empty());
    CHECK(t.kmax >= 1.0f && t.win_c0 >= 0 && t.win_c1 < 35 && t.win_r0 >= 0 && t.win_r1 < 25);
    // error paths, each with its code and a message
    auto expect = [](pn_geometry h, int code) {
        CHECK(pn_check_geometry(&h) == code);
        CHECK(pn_last_error()[0] != '\0');
    };
    pn_geometry h = g;
    h.ndim = 4;
    expect(h, PN_EINVAL);
    h = g, h.beam = PN_FAN;
    expect(h, PN_EINVAL);
    h = g, h.vol_shape[1] = 0;
    expect(h, PN_EINVAL);
    h = g, h.vol_spacing[2] = -1.0;
    expect(h, PN_EINVAL);
    h = g, h.vol_origin[0] = INFINITY;
    expect(h, PN_EINVAL);
    h = g, h.n_views = -1;
    expect(h, PN_EINVAL);
    h = g, h.proj = nullptr;
    expect(h, PN_EINVAL);
    h = g, h.det_shape[0] = 70000;
    expect(h, PN_EINVAL);
    std::vector<double> Q = P;
    Q[5] = NAN;
    h = g, h.proj = Q.data();
    expect(h, PN_EGEOM);
    Q = P;
    for (int e = 0; e < 12; ++e) Q[12 + e] = 0.0;
    h = g, h.proj = Q.data();
    expect(h, PN_EGEOM);
    // source inside the volume: shift the volume onto the source of view 0
    h = g, h.vol_origin[2] = 740.0, h.vol_origin[1] = -5.0, h.vol_origin[0] = -5.0;
    expect(h, PN_EGEOM);
    h = g, h.n_views = 0;
    CHECK(pn_check_geometry(&h) == PN_OK);
    // degenerate composition inputs
    double S[3] = {0, 0, 0}, C[3] = {1, 0, 0}, eu[3] = {0, 1, 0}, ev[3] = {0, 2, 0}, out[12];
    CHECK(pn_cone_matrices(1, S, C, eu, ev, 4, 4, out) == PN_EGEOM);
    CHECK(pn_cone_matrices(-1, S, C, eu, ev, 4, 4, out) == PN_EINVAL);
    CHECK(pn_cone_matrices(1, nullptr, C, eu, ev, 4, 4, out) == PN_EINVAL);
    double d2[2] = {1, 0}, c2[2] = {0, 0}, e2[2] = {2, 0}, o2[6];
    CHECK(pn_parallel2d_matrices(1, d2, c2, e2, 5, o2) == PN_EGEOM);
    CHECK(pn_fan_matrices(1, c2, c2, e2, 5, o2) == PN_EGEOM);
    // argument checks
    pn::Geo gg;
    float buf[4];
    CHECK(pn::preflight(&g, 1, buf, buf, PN_F32, PN_F32, false, gg) == PN_EINVAL);  // aliasing
    CHECK(pn::preflight(&g, 1, buf, nullptr, PN_F32, PN_F32, false, gg) == PN_EINVAL);
    CHECK(pn::preflight(&g, 1, (char *)buf + 1, buf + 1, PN_BF16, PN_F32, false, gg) == PN_EINVAL);
    CHECK(pn::preflight(&g, 1, buf, buf + 1, 7, PN_F32, false, gg) == PN_EDTYPE);
    CHECK(pn::preflight(&g, -1, buf, buf + 1, PN_F32, PN_F32, false, gg) == PN_EINVAL);
    CHECK(pn::preflight(&g, 0, nullptr, nullptr, PN_F32, PN_F32, false, gg) == PN_OK);
    CHECK(pn::preflight(&g, 1, buf, buf + 1, PN_F32, PN_F32, false, gg) == PN_OK);
}

int main()
{
    check_buffers();
    check_plans();
    check_geometry();
    std::printf("host_check OK\n");
    return 0;
}
