// C-ABI entry points of the EM-PIC library (declared in include/pic.h).
//
// Every call validates its arguments on the host before any launch, maps
// the caller's device pointers into kernel-argument structs, and launches
// asynchronously on the caller's stream.  The library allocates no device
// memory: scratch space comes from the caller's workspace, carved at fixed
// 256-byte-aligned offsets.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_types.hpp"

using namespace pic;

namespace {

thread_local std::string g_msg;

pic_status fail(pic_status s, const std::string &m)
{
    g_msg = m;
    return s;
}

pic_status hip_fail(hipError_t e, const char *where)
{
    g_msg = std::string(where) + ": " + hipGetErrorString(e);
    return PIC_E_DEVICE;
}

#define PIC_TRY_S(expr)                                 \
    do {                                                \
        pic_status s_ = (expr);                         \
        if (s_ != PIC_OK)                               \
            return s_;                                  \
    } while (0)

#define PIC_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess)                           \
            return hip_fail(e_, #call);                 \
    } while (0)

// ---------------------------------------------------------------------------
// optional kernel timing (pic_timing): event pairs recorded around launches
constexpr int NCAT = 7;
struct Timer {
    bool on = false;
    struct Pending {
        int cat;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double ms[NCAT] = {};
    int64_t cnt[NCAT] = {};
};
Timer g_timer;
std::mutex g_timer_mu;
// set while pic_step_noalloc runs: no timing events are created or recorded
thread_local bool g_untimed = false;

hipEvent_t timer_event()
{
    if (!g_timer.pool.empty()) {
        hipEvent_t e = g_timer.pool.back();
        g_timer.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// records an event pair around the launches made while it is alive
struct TimedScope {
    int cat;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    TimedScope(int c, hipStream_t s) : cat(c), st(s)
    {
        if (g_untimed)
            return;
        std::lock_guard<std::mutex> lk(g_timer_mu);
        if (!g_timer.on)
            return;
        a = timer_event();
        b = timer_event();
        if (a && b)
            hipEventRecord(a, st);
    }
    ~TimedScope()
    {
        if (!a || !b)
            return;
        hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(g_timer_mu);
        g_timer.pending.push_back({cat, a, b});
    }
};

void timer_flush()
{
    for (auto &p : g_timer.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_timer.ms[p.cat] += ms;
            g_timer.cnt[p.cat] += 1;
        }
        g_timer.pool.push_back(p.a);
        g_timer.pool.push_back(p.b);
    }
    g_timer.pending.clear();
}

// Error word of the calls that take no workspace (pic_gather, pic_push,
// pic_deposit): cleared on the caller's stream before their launch and read
// back after it.  One word per device, shared by those calls: calls that
// overlap on one device (other streams or threads) may see each other's
// errors.
__device__ int g_sink_err;

int *sink_err()
{
    int *p = nullptr;
    if (hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(g_sink_err)) != hipSuccess)
        return nullptr;
    return p;
}

// clears the error word on the stream (before the launch)
pic_status sink_begin(int *err, hipStream_t st)
{
    const hipError_t e = launch_fill<int>(err, 1, 0, st);
    if (e != hipSuccess)
        return hip_fail(e, "clearing the device error word");
    return PIC_OK;
}

// reads the error word back after the launch (synchronises the stream)
pic_status sink_end(int *err, hipStream_t st, const char *what)
{
    int herr = 0;
    PIC_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    PIC_HIP(hipStreamSynchronize(st));
    if (herr)
        return fail(PIC_E_STATE, what);
    return PIC_OK;
}

// Scratch of pic_step_noalloc: a static array in place of the caller's
// workspace, one copy per device (the code object's), held until the
// process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current.
static __device__ __align__(256) unsigned char scratch[PIC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // by device ordinal

pic_status scratch_address(void **out)
{
    int dev = 0;
    PIC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0)
        return fail(PIC_E_DEVICE, "hipGetDevice returned a negative ordinal");
    if ((size_t)dev >= g_scratch_ptr.size())
        g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        PIC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0)
            return fail(PIC_E_DEVICE, "static scratch array has no 256-byte aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PIC_OK;
}

// LDS bytes one workgroup may use; gfx950 has 160 KiB per CU, which is also
// what a host without a visible device assumes
int lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 160 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 160 * 1024;
    return v;
}

struct GridInfo {
    int n[3];
    int64_t ncell;
    bool filt;          // fields filtered along z before the gather
    double fw[6][4];    // the filter's taps per component
    int order;
    int dtype;
    size_t tsize;
    TileGeo tg;
    int ntiles;
    int tile_cells;
};

void region_extents(int order, TileGeo &tg)
{
    const int s = tg.slack;
    const int gl = order == 3 ? 2 : 1;   // gather halo below the tile
    for (int d = 0; d < 3; ++d) {
        tg.rf[d] = tg.t[d] + 2 * s + (order == 3 ? 4 : 2);
        tg.rj[d] = tg.t[d] + 2 * s + (order == 3 ? 5 : 3);
    }
    tg.lo_f = s + gl;
    tg.lo_j = s + gl;
    tg.jp = tg.rj[0];
}

// LDS of the tiled adjoint: its first pass holds E, B with the gather halo
// and hatE with the deposit halo, its second the FP64 accumulators of the
// six field adjoints
size_t adj_lds_for(const GridInfo &gi, const TileGeo &a)
{
    const size_t rf = (size_t)a.rf[0] * a.rf[1] * a.rf[2];
    const size_t rj = (size_t)a.rj[0] * a.rj[1] * a.rj[2];
    const size_t push = 6 * rf * gi.tsize + 3 * rj * gi.tsize + 16;
    const size_t scatter = 6 * rf * sizeof(double);
    return push > scatter ? push : scatter;
}

// regions of the tiled adjoint: the forward's tiles, with its slack when
// the adjoint regions fit the LDS and without otherwise
TileGeo adjoint_geo(const GridInfo &gi)
{
    TileGeo a = gi.tg;
    region_extents(gi.order, a);
    if (a.slack > 0 && adj_lds_for(gi, a) > (size_t)lds_limit()) {
        a.slack = 0;
        region_extents(gi.order, a);
    }
    return a;
}

size_t adj_lds_bytes(const GridInfo &gi)
{
    return adj_lds_for(gi, adjoint_geo(gi));
}

size_t lds_bytes(const GridInfo &gi)
{
    const size_t rf = (size_t)gi.tg.rf[0] * gi.tg.rf[1] * gi.tg.rf[2];
    const size_t rj = (size_t)gi.tg.jp * gi.tg.rj[1] * gi.tg.rj[2];
    // fields in the working precision, the current tile in FP64
    return ((6 * rf * gi.tsize + 15) & ~size_t(15)) + 3 * rj * sizeof(double);
}

pic_status check_grid(const pic_grid *g, GridInfo &gi)
{
    if (!g)
        return fail(PIC_E_INVALID, "grid is NULL");
    int64_t nc = 1;
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 4)
            return fail(PIC_E_INVALID, "grid n[d] must be >= 4");
        if (!(g->d[d] > 0) || !std::isfinite(g->d[d]))
            return fail(PIC_E_INVALID, "grid spacing must be positive and finite");
        gi.n[d] = g->n[d];
        nc *= g->n[d];
    }
    if (nc >= (int64_t(1) << 31))
        return fail(PIC_E_INVALID, "grid has 2^31 cells or more");
    gi.ncell = nc;
    if (!(g->dt > 0) || !(g->c > 0) || !(g->eps0 > 0) || !std::isfinite(g->dt) || !std::isfinite(g->c) ||
        !std::isfinite(g->eps0))
        return fail(PIC_E_INVALID, "dt, c and eps0 must be positive and finite");
    if (g->order != 1 && g->order != 3)
        return fail(PIC_E_UNSUPPORTED, "shape order must be 1 or 3");
    if (g->pusher != PIC_PUSH_BORIS && g->pusher != PIC_PUSH_VAY)
        return fail(PIC_E_UNSUPPORTED, "pusher must be PIC_PUSH_BORIS or PIC_PUSH_VAY");
    if (g->dtype != PIC_F32 && g->dtype != PIC_F64)
        return fail(PIC_E_UNSUPPORTED, "dtype must be PIC_F32 or PIC_F64");
    if (g->solver != PIC_SOLVER_YEE && g->solver != PIC_SOLVER_CKC)
        return fail(PIC_E_UNSUPPORTED, "solver must be PIC_SOLVER_YEE or PIC_SOLVER_CKC");
    gi.filt = g->gather_filter != nullptr;
    for (int m = 0; m < 6; ++m)
        for (int s = 0; s < 4; ++s) {
            gi.fw[m][s] = gi.filt ? g->gather_filter[4 * m + s] : (s == 0 ? 1.0 : 0.0);
            if (!std::isfinite(gi.fw[m][s]))
                return fail(PIC_E_INVALID, "gather filter taps must be finite");
        }
    if (g->solver == PIC_SOLVER_YEE) {
        const double inv = 1.0 / (g->d[0] * g->d[0]) + 1.0 / (g->d[1] * g->d[1]) + 1.0 / (g->d[2] * g->d[2]);
        if (g->c * g->dt * std::sqrt(inv) > 1.0 + 1e-12)
            return fail(PIC_E_CFL, "c dt exceeds the Yee CFL limit 1/sqrt(sum 1/d^2)");
    } else {
        const double dmin = std::min(g->d[0], std::min(g->d[1], g->d[2]));
        if (g->c * g->dt > dmin * (1.0 + 1e-12))
            return fail(PIC_E_CFL, "c dt exceeds the CKC CFL limit min(d)");
    }
    gi.order = g->order;
    gi.dtype = g->dtype;
    gi.tsize = g->dtype == PIC_F64 ? sizeof(double) : sizeof(float);
    // tiles
    bool auto_tile[3];
    for (int d = 0; d < 3; ++d) {
        int t = g->tile[d];
        auto_tile[d] = (t == 0);
        if (t == 0) {   // largest divisor of n not above 8
            t = 8;
            while (g->n[d] % t != 0)
                --t;
        }
        if (t < 1 || t > 16 || g->n[d] % t != 0)
            return fail(PIC_E_INVALID, "tile size must be in [1,16] and divide n");
        gi.tg.t[d] = t;
    }
    if (g->slack < -1 || g->slack > 2)
        return fail(PIC_E_INVALID, "slack must be -1 (automatic) or in [0,2]");
    const size_t limit = (size_t)lds_limit();
    // Automatic slack is one cell.  While the forward regions (with slack)
    // or the adjoint regions (without) do not fit one workgroup, an automatic
    // tile halves its largest dimension; only when no dimension can shrink
    // does an automatic slack drop to zero.  A smaller tile with slack beats
    // a larger one without: particles that drift out of a slack-free tile
    // between sorts take the global path.
    const bool auto_slack = g->slack < 0;
    gi.tg.slack = auto_slack ? 1 : g->slack;
    region_extents(gi.order, gi.tg);
    while (lds_bytes(gi) > limit || adj_lds_bytes(gi) > limit) {
        int dmax = -1;
        for (int d = 0; d < 3; ++d)
            if (auto_tile[d] && gi.tg.t[d] >= 4 && gi.tg.t[d] % 2 == 0 &&
                (dmax < 0 || gi.tg.t[d] > gi.tg.t[dmax] || (gi.tg.t[d] == gi.tg.t[dmax] && d > dmax)))
                dmax = d;
        if (dmax >= 0)
            gi.tg.t[dmax] /= 2;
        else if (auto_slack && gi.tg.slack > 0)
            gi.tg.slack = 0;
        else
            break;
        region_extents(gi.order, gi.tg);
    }
    if (lds_bytes(gi) > limit)
        return fail(PIC_E_UNSUPPORTED, "tile plus halo does not fit in LDS; use a smaller tile or slack");
    // On a small grid the automatic tiles halve further (not below 4 cells)
    // until there are two per CU: one workgroup per tile would otherwise
    // leave most of the 256 CUs idle.
    for (;;) {
        int64_t ntl = 1;
        for (int d = 0; d < 3; ++d)
            ntl *= gi.n[d] / gi.tg.t[d];
        if (ntl >= 512)
            break;
        int dmax = -1;
        for (int d = 0; d < 3; ++d)
            if (auto_tile[d] && gi.tg.t[d] >= 8 && gi.tg.t[d] % 2 == 0 &&
                (dmax < 0 || gi.tg.t[d] > gi.tg.t[dmax] || (gi.tg.t[d] == gi.tg.t[dmax] && d > dmax)))
                dmax = d;
        if (dmax < 0)
            break;
        gi.tg.t[dmax] /= 2;
        region_extents(gi.order, gi.tg);
    }
    // the LDS left over holds the forward tile kernel's queue of
    // cell-crossing particles (up to 1024 entries)
    {
        const size_t used = lds_bytes(gi) + sizeof(int);
        const size_t entry = 6 * gi.tsize + 2 * sizeof(int);
        const size_t room = limit > used ? (limit - used) / entry : 0;
        gi.tg.qcap = (int)(room < 1024 ? room : 1024);
    }
    int nt = 1;
    for (int d = 0; d < 3; ++d) {
        gi.tg.nt[d] = gi.n[d] / gi.tg.t[d];
        nt *= gi.tg.nt[d];
    }
    gi.ntiles = nt;
    gi.tile_cells = gi.tg.t[0] * gi.tg.t[1] * gi.tg.t[2];
    gi.tg.xcd_map = (nt % 8 == 0) ? 1 : 0;
    return PIC_OK;
}

pic_status check_species(const pic_species *s, const char *name)
{
    if (!s)
        return fail(PIC_E_INVALID, std::string(name) + " is NULL");
    if (s->n < 0 || s->n >= (int64_t(1) << 31) - 1)
        return fail(PIC_E_INVALID, std::string(name) + ": particle count must be in [0, 2^31-1)");
    if (s->n > 0)
        for (int d = 0; d < 3; ++d)
            if (!s->cell[d] || !s->off[d] || !s->u[d])
                return fail(PIC_E_INVALID, std::string(name) + ": NULL particle array");
    if (!(s->m > 0) || !std::isfinite(s->m) || !std::isfinite(s->q) || !std::isfinite(s->w0))
        return fail(PIC_E_INVALID, std::string(name) + ": m must be positive and q, w0 finite");
    return PIC_OK;
}

pic_status check_fields(const pic_fields *f, bool need_j)
{
    if (!f)
        return fail(PIC_E_INVALID, "fields is NULL");
    for (int d = 0; d < 3; ++d)
        if (!f->E[d] || !f->B[d] || (need_j && !f->J[d]))
            return fail(PIC_E_INVALID, "NULL field array");
    return PIC_OK;
}

// workspace layout
struct WsLayout {
    size_t err, counts, bsum, key, rank, slot, scell, soff, su, sw, hatE, partials, red5, old_ts, filt, lfilt,
        gcnt, glist, gflag, total;
};

// guest list slots per tile (a tile's particles that left their home region
// beyond this many go to the stray kernel)
constexpr int GUEST_CAP = 256;

size_t al(size_t x)
{
    return (x + 255) & ~size_t(255);
}

WsLayout layout(const GridInfo &gi, int64_t np)
{
    WsLayout L{};
    size_t o = 0;
    const size_t n = (size_t)(np > 0 ? np : 0);
    L.err = o;
    o += 256;
    L.counts = o;
    o += al(sizeof(int) * ((size_t)gi.ncell + 1));
    L.bsum = o;
    o += al(sizeof(int) * ((size_t)scan_blocks(gi.ncell + 1) + 1));
    L.key = o;
    o += al(sizeof(int) * n);
    L.rank = o;
    o += al(sizeof(int) * n);
    L.slot = o;
    o += al(sizeof(int) * n);
    L.scell = o;
    o += 3 * al(sizeof(int) * n);
    L.soff = o;
    o += 3 * al(gi.tsize * n);
    L.su = o;
    o += 3 * al(gi.tsize * n);
    L.sw = o;
    o += al(gi.tsize * n);
    L.hatE = o;
    o += 3 * al(gi.tsize * (size_t)gi.ncell);
    L.partials = o;
    o += al(sizeof(double) * 5 * (size_t)reduce_max_blocks());
    L.red5 = o;
    o += 256;
    L.old_ts = o;
    o += al(sizeof(int) * ((size_t)gi.ntiles + 1));
    // filtered E, B for the gather and their adjoints (only with a filter)
    L.filt = o;
    o += gi.filt ? 6 * al(gi.tsize * (size_t)gi.ncell) : 0;
    L.lfilt = o;
    o += gi.filt ? 6 * al(gi.tsize * (size_t)gi.ncell) : 0;
    // guest lists, counts and per-particle flags, two of each (by step parity)
    L.gcnt = o;
    o += 2 * al(sizeof(int) * (size_t)gi.ntiles);
    L.glist = o;
    o += 2 * al(2 * sizeof(int) * (size_t)gi.ntiles * GUEST_CAP);
    L.gflag = o;
    o += 2 * al(n);
    L.total = o;
    return L;
}

pic_status check_ws(const GridInfo &gi, int64_t np, void *ws, size_t ws_bytes, WsLayout &L)
{
    L = layout(gi, np);
    if (!ws)
        return fail(PIC_E_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(PIC_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(PIC_E_WORKSPACE, "workspace smaller than pic_workspace_bytes()");
    return PIC_OK;
}

template <typename T>
PConst<T> make_const(const pic_grid *g, const pic_species *s)
{
    PConst<T> pc{};
    for (int d = 0; d < 3; ++d) {
        pc.n[d] = g->n[d];
        pc.dtd[d] = (T)(g->dt / g->d[d]);
        const int p = (d + 1) % 3, q = (d + 2) % 3;
        pc.jk[d] = s ? (T)(-s->q / (g->dt * g->d[p] * g->d[q])) : T(0);
    }
    pc.h = s ? (T)(s->q * g->dt / (2.0 * s->m)) : T(0);
    pc.inv_c2 = (T)(1.0 / (g->c * g->c));
    pc.w0 = s ? (T)s->w0 : T(0);
    pc.lj = (T)(-g->dt / g->eps0);
    pc.vay = g->pusher == PIC_PUSH_VAY ? 1 : 0;
    return pc;
}

template <typename T>
PArr<T> parr(const pic_species *s)
{
    PArr<T> a{};
    for (int d = 0; d < 3; ++d) {
        a.cell[d] = s->cell[d];
        a.off[d] = static_cast<T *>(s->off[d]);
        a.u[d] = static_cast<T *>(s->u[d]);
    }
    a.w = static_cast<T *>(s->w);
    a.n = s->n;
    return a;
}

template <typename T>
PArr<T> parr_ws(char *ws, const WsLayout &L, const pic_species *s)
{
    PArr<T> a{};
    const size_t n = (size_t)s->n;
    for (int d = 0; d < 3; ++d) {
        a.cell[d] = reinterpret_cast<int *>(ws + L.scell + d * al(sizeof(int) * n));
        a.off[d] = reinterpret_cast<T *>(ws + L.soff + d * al(sizeof(T) * n));
        a.u[d] = reinterpret_cast<T *>(ws + L.su + d * al(sizeof(T) * n));
    }
    a.w = s->w ? reinterpret_cast<T *>(ws + L.sw) : nullptr;
    a.n = s->n;
    return a;
}

template <typename T>
FieldPtrs<T> fptrs(const pic_fields *f)
{
    FieldPtrs<T> p{};
    for (int d = 0; d < 3; ++d) {
        p.E[d] = static_cast<T *>(f->E[d]);
        p.B[d] = static_cast<T *>(f->B[d]);
        p.J[d] = static_cast<T *>(f->J[d]);
    }
    return p;
}

double src_g(const pic_source *src, int64_t step)
{
    if (!src || src->k_plane < 0 || !src->g || step < 0 || step >= src->n_g)
        return 0.0;
    return src->g[step];
}

pic_status check_source(const pic_source *src, const GridInfo &gi)
{
    if (!src || src->k_plane < 0)
        return PIC_OK;
    if (src->k_plane >= gi.n[2])
        return fail(PIC_E_INVALID, "source k_plane outside the grid");
    if (!src->amp)
        return fail(PIC_E_INVALID, "source amp is NULL");
    if (src->n_g > 0 && !src->g)
        return fail(PIC_E_INVALID, "source g is NULL");
    return PIC_OK;
}

// CKC weights of the B update's differences (alpha, beta_p, beta_q, gamma
// per difference axis), from the published closed form in pic.h.
template <typename T>
void ckc_weights(const pic_grid *g, CurlArgs<T> &a)
{
    const double dl = std::min(g->d[0], std::min(g->d[1], g->d[2]));
    double r[3];
    for (int d = 0; d < 3; ++d)
        r[d] = (dl / g->d[d]) * (dl / g->d[d]);
    const double S = r[0] * r[1] + r[1] * r[2] + r[2] * r[0];
    const double beta = (1.0 - r[0] * r[1] * r[2] / S) / 8.0;
    for (int d = 0; d < 3; ++d) {
        const int p = (d + 1) % 3, q = (d + 2) % 3;
        const double bp = r[p] * beta, bq = r[q] * beta;
        const double gm = r[p] * r[q] * (1.0 / 16.0 - r[p] * r[q] / (8.0 * S));
        a.ck[d][0] = (T)(1.0 - 2.0 * bp - 2.0 * bq - 4.0 * gm);
        a.ck[d][1] = (T)bp;
        a.ck[d][2] = (T)bq;
        a.ck[d][3] = (T)gm;
    }
    a.ckc = 1;
}

// One field step: B -= dt/2 curlE; E += dt (c^2 curlB - J/eps0) + source;
// B -= dt/2 curlE (with the CKC solver the curl of E averages transversely).
// zero_j clears J as it is consumed.
// With bh (Yee solver only): the steps of one call chained through the
// half-step B in bh, first and last marking the call's first and last step.
template <typename T>
pic_status yee_step(const pic_grid *g, const GridInfo &gi, const FieldPtrs<T> &f, const pic_source *src,
                    int64_t step, bool zero_j, hipStream_t st, T *const *bh = nullptr, bool first = true,
                    bool last = true)
{
    CurlArgs<T> b{};
    for (int d = 0; d < 3; ++d) {
        b.out[d] = f.B[d];
        b.in[d] = f.B[d];
        b.src[d] = f.E[d];
        b.n[d] = gi.n[d];
    }
    b.cx = (T)(-0.5 * g->dt / g->d[0]);
    b.cy = (T)(-0.5 * g->dt / g->d[1]);
    b.cz = (T)(-0.5 * g->dt / g->d[2]);
    b.kplane = -1;
    if (g->solver == PIC_SOLVER_CKC)
        ckc_weights<T>(g, b);
    CurlArgs<T> e{};
    for (int d = 0; d < 3; ++d) {
        e.out[d] = f.E[d];
        e.in[d] = f.E[d];
        e.src[d] = f.B[d];
        e.J[d] = f.J[d];
        e.n[d] = gi.n[d];
    }
    const double c2 = g->c * g->c;
    e.cx = (T)(c2 * g->dt / g->d[0]);
    e.cy = (T)(c2 * g->dt / g->d[1]);
    e.cz = (T)(c2 * g->dt / g->d[2]);
    e.jc = (T)(-g->dt / g->eps0);
    e.zero_j = zero_j ? 1 : 0;
    e.kplane = -1;
    if (src && src->k_plane >= 0) {
        e.kplane = src->k_plane;
        e.amp = static_cast<const T *>(src->amp);
        e.ag = (T)src_g(src, step);
    }
    if (!bh) {
        PIC_HIP(launch_curl<T>(true, b, st));
        PIC_HIP(launch_curl<T>(false, e, st));
        PIC_HIP(launch_curl<T>(true, b, st));
        return PIC_OK;
    }
    // Chained steps of one call: the second B half step of a step and the
    // first of the next use the same curl of E, so one pass writes both
    // B^{n+1} (into B, for the gather and the diagnostics) and B^{n+3/2}
    // (into bh, for the next E update) with the same arithmetic as two
    // passes; only the first step of a call computes its B^{n+1/2} alone.
    CurlArgs<T> bf = b;
    for (int d = 0; d < 3; ++d) {
        if (first) {
            b.out[d] = bh[d];
        }
        e.src[d] = bh[d];
        bf.in[d] = bh[d];
        bf.out[d] = f.B[d];
        bf.out2[d] = last ? nullptr : bh[d];
    }
    if (first)
        PIC_HIP(launch_curl<T>(true, b, st));
    PIC_HIP(launch_curl<T>(false, e, st));
    PIC_HIP(launch_curl<T>(true, bf, st));
    return PIC_OK;
}

template <typename T>
pic_status do_sort(const GridInfo &gi, const pic_species *sp, char *ws, const WsLayout &L, int *tile_start,
                   int *perm, hipStream_t st, PArr<T> &sorted, bool binned = false)
{
    int *err = reinterpret_cast<int *>(ws + L.err);
    int *counts = reinterpret_cast<int *>(ws + L.counts);
    int *bsum = reinterpret_cast<int *>(ws + L.bsum);
    int *key = reinterpret_cast<int *>(ws + L.key);
    int *rank = reinterpret_cast<int *>(ws + L.rank);
    const PArr<T> in = parr<T>(sp);
    sorted = parr_ws<T>(ws, L, sp);
    PIC_HIP(launch_fill<int>(counts, gi.ncell + 1, 0, st));
    // particles still binned by the previous sort count per tile in LDS
    if (binned)
        PIC_HIP(launch_bin_count_tile<T>(in, gi.tg, tile_start, counts, key, rank, err, st));
    else
        PIC_HIP(launch_bin_count<T>(in, gi.tg, counts, key, rank, err, st));
    PIC_HIP(launch_scan(counts, gi.ncell, bsum, st));
    // a re-sort keeps the previous binning: the scatter is staged per old tile
    int *old_start = nullptr;
    if (binned) {
        old_start = reinterpret_cast<int *>(ws + L.old_ts);
        PIC_HIP(hipMemcpyAsync(old_start, tile_start, sizeof(int) * ((size_t)gi.ntiles + 1), hipMemcpyDeviceToDevice,
                               st));
    }
    PIC_HIP(launch_tile_start(counts, gi.tile_cells, gi.ntiles, sp->n, tile_start, st));
    int *slot = reinterpret_cast<int *>(ws + L.slot);
    PIC_HIP(launch_interleave(counts, tile_start, gi.tile_cells, gi.ntiles, slot, st));
    PIC_HIP(launch_scatter<T>(in, sorted, key, rank, counts, slot, tile_start, old_start, gi.ntiles, gi.tile_cells,
                              perm, st));
    return PIC_OK;
}

template <typename T>
pic_status sort_tiles_t(const pic_grid *g, const GridInfo &gi, pic_species *sp, int32_t *tile_start, int32_t *perm,
                        void *ws, const WsLayout &L, hipStream_t st)
{
    char *w = static_cast<char *>(ws);
    int *err = reinterpret_cast<int *>(w + L.err);
    PIC_HIP(launch_fill<int>(err, 1, 0, st));
    // the state check runs before anything is reordered
    {
        int *counts = reinterpret_cast<int *>(w + L.counts);
        int *key = reinterpret_cast<int *>(w + L.key);
        int *rank = reinterpret_cast<int *>(w + L.rank);
        PIC_HIP(launch_fill<int>(counts, gi.ncell + 1, 0, st));
        PIC_HIP(launch_bin_count<T>(parr<T>(sp), gi.tg, counts, key, rank, err, st));
        int herr = 0;
        PIC_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
        PIC_HIP(hipStreamSynchronize(st));
        if (herr)
            return fail(PIC_E_STATE, "particle with a cell outside the grid or an offset outside [0,1)");
    }
    PArr<T> sorted;
    pic_status s = do_sort<T>(gi, sp, w, L, tile_start, perm, st, sorted);
    if (s != PIC_OK)
        return s;
    const size_t n = (size_t)sp->n;
    for (int d = 0; d < 3; ++d) {
        PIC_HIP(hipMemcpyAsync(sp->cell[d], sorted.cell[d], n * sizeof(int), hipMemcpyDeviceToDevice, st));
        PIC_HIP(hipMemcpyAsync(sp->off[d], sorted.off[d], n * sizeof(T), hipMemcpyDeviceToDevice, st));
        PIC_HIP(hipMemcpyAsync(sp->u[d], sorted.u[d], n * sizeof(T), hipMemcpyDeviceToDevice, st));
    }
    if (sp->w)
        PIC_HIP(hipMemcpyAsync(sp->w, sorted.w, n * sizeof(T), hipMemcpyDeviceToDevice, st));
    (void)g;
    return PIC_OK;
}

template <typename T>
pic_status reduce_t(const pic_grid *g, const GridInfo &gi, const pic_species *sp, const pic_fields *f, double *out,
                    char *ws, const WsLayout &L, hipStream_t st)
{
    const double dV = g->d[0] * g->d[1] * g->d[2];
    const double mu0 = 1.0 / (g->eps0 * g->c * g->c);
    double scale[7];
    scale[0] = 0.5 * dV * g->eps0;
    scale[1] = 0.5 * dV / mu0;
    scale[2] = sp ? sp->m * g->c * g->c : 0.0;
    scale[3] = sp ? sp->q : 0.0;
    scale[4] = sp ? sp->m : 0.0;
    scale[5] = 1.0 / (g->c * g->c);
    scale[6] = sp ? sp->w0 : 0.0;
    PArr<T> a{};
    if (sp)
        a = parr<T>(sp);
    PIC_HIP(launch_reduce<T>(sp ? &a : nullptr, fptrs<T>(f), gi.ncell, reinterpret_cast<double *>(ws + L.partials),
                             reduce_max_blocks(), scale, out, st));
    return PIC_OK;
}

// The fields the particle kernels read: the caller's, or with a gather
// filter the filtered copies in the workspace (J stays the caller's).
template <typename T>
FieldPtrs<T> gather_view(const GridInfo &gi, const FieldPtrs<T> &fp, char *w, const WsLayout &L)
{
    FieldPtrs<T> v = fp;
    if (gi.filt) {
        const size_t a = al(sizeof(T) * (size_t)gi.ncell);
        for (int d = 0; d < 3; ++d) {
            v.E[d] = reinterpret_cast<T *>(w + L.filt + d * a);
            v.B[d] = reinterpret_cast<T *>(w + L.filt + (3 + d) * a);
        }
    }
    return v;
}

// dst = filter(src) per component (add: dst += filter(src))
template <typename T>
pic_status filter_fields(const GridInfo &gi, const FieldPtrs<T> &src, const FieldPtrs<T> &dst, hipStream_t st,
                         bool add = false)
{
    for (int m = 0; m < 6; ++m) {
        const T *in = m < 3 ? src.E[m] : src.B[m - 3];
        T *out = m < 3 ? dst.E[m] : dst.B[m - 3];
        const T w[4] = {(T)gi.fw[m][0], (T)gi.fw[m][1], (T)gi.fw[m][2], (T)gi.fw[m][3]};
        PIC_HIP(launch_filter_z<T>(in, out, w, add, gi.n, st));
    }
    return PIC_OK;
}

template <typename T>
pic_status step_t(const pic_grid *g, const GridInfo &gi, pic_species *sp, pic_fields *f, const pic_source *src,
                  int64_t step0, int32_t nsteps, int32_t sort_every, int32_t *tile_start, void *ws,
                  const WsLayout &L, double *diag, hipStream_t st)
{
    char *w = static_cast<char *>(ws);
    int *err = reinterpret_cast<int *>(w + L.err);
    const PConst<T> pc = make_const<T>(g, sp);
    const FieldPtrs<T> fp = fptrs<T>(f);
    const PArr<T> user = parr<T>(sp);
    // the fields the particle kernels gather from (filtered copies with a filter)
    const FieldPtrs<T> fpp = gather_view<T>(gi, fp, w, L);
    // the list of the tile kernels' strays, in the sort's rank buffer (free
    // once the sort of the step is done), and its count
    int *stray_list = reinterpret_cast<int *>(w + L.rank);
    int *stray_cnt = reinterpret_cast<int *>(w + L.err + 64);
    // guest buffers by step parity: the lists a step builds are the next
    // step's; none are read at the first step of a call or after a sort
    // (a sort renumbers the particles)
    int *gcnt[2];
    int2 *glist[2];
    unsigned char *gflag[2];
    for (int b = 0; b < 2; ++b) {
        gcnt[b] = reinterpret_cast<int *>(w + L.gcnt + b * al(sizeof(int) * (size_t)gi.ntiles));
        glist[b] = reinterpret_cast<int2 *>(w + L.glist + b * al(2 * sizeof(int) * (size_t)gi.ntiles * GUEST_CAP));
        gflag[b] = reinterpret_cast<unsigned char *>(w + L.gflag + b * al((size_t)(sp->n > 0 ? sp->n : 0)));
    }
    // old offsets between the tile kernel's phases when it runs in place:
    // the sorted copy's offset arrays, free on a step without a sort
    T *scratch[3];
    for (int d = 0; d < 3; ++d)
        scratch[d] = reinterpret_cast<T *>(w + L.soff + d * al(gi.tsize * (size_t)(sp->n > 0 ? sp->n : 0)));
    // the half-step B of chained Yee steps, in the adjoint's hatE scratch
    // (unused by the forward step)
    T *bh[3];
    for (int d = 0; d < 3; ++d)
        bh[d] = reinterpret_cast<T *>(w + L.hatE + d * al(sizeof(T) * (size_t)gi.ncell));
    const bool chain = g->solver == PIC_SOLVER_YEE;
    PIC_HIP(launch_fill<int>(err, 1, 0, st));
    for (int d = 0; d < 3; ++d)
        PIC_HIP(launch_fill<T>(fp.J[d], gi.ncell, T(0), st));
    for (int32_t it = 0; it < nsteps; ++it) {
        const int64_t step = step0 + it;
        const bool sort_now = sort_every > 0 && (it == 0 || step % sort_every == 0);
        if (gi.filt && sp->n > 0) {
            TimedScope ts(1, st);
            PIC_TRY_S(filter_fields<T>(gi, fp, fpp, st));
        }
        // guests only where particles drift far between sorts (no re-sort, or
        // sorts more than 8 steps apart); otherwise the kernel without them
        GuestArgs ga{};
        if (sort_every == 0 || sort_every > 8) {
            const int cur = (int)(it & 1), nxt = 1 - cur;
            const bool read = it > 0 && !sort_now;
            ga.cnt = read ? gcnt[cur] : nullptr;
            ga.list = read ? glist[cur] : nullptr;
            ga.flag = read ? gflag[cur] : nullptr;
            ga.cnt_next = gcnt[nxt];
            ga.list_next = glist[nxt];
            ga.flag_next = gflag[nxt];
            ga.cap = GUEST_CAP;
            if (tile_start && sp->n > 0)
                PIC_HIP(launch_fill<int>(ga.cnt_next, gi.ntiles, 0, st));
        }
        if (sort_now && sp->n > 0) {
            PArr<T> sorted;
            {
                TimedScope ts(0, st);
                pic_status s = do_sort<T>(gi, sp, w, L, tile_start, nullptr, st, sorted, it > 0);
                if (s != PIC_OK)
                    return s;
            }
            {
                TimedScope ts(1, st);
                PIC_HIP(launch_particles_tile<T>(gi.order, pc, gi.tg, sorted, user, fpp, tile_start, stray_list,
                                                 stray_cnt, ga, scratch, err, st));
            }
            TimedScope ts(6, st);
            PIC_HIP(launch_particles_strays<T>(gi.order, pc, sorted, user, fpp, stray_list, stray_cnt, ga, err, st));
        } else if (tile_start && sp->n > 0) {
            {
                TimedScope ts(1, st);
                PIC_HIP(launch_particles_tile<T>(gi.order, pc, gi.tg, user, user, fpp, tile_start, stray_list,
                                                 stray_cnt, ga, scratch, err, st));
            }
            TimedScope ts(6, st);
            PIC_HIP(launch_particles_strays<T>(gi.order, pc, user, user, fpp, stray_list, stray_cnt, ga, err, st));
        } else {
            TimedScope ts(1, st);
            PIC_HIP(launch_particles_global<T>(gi.order, pc, user, fpp, err, st));
        }
        pic_status s;
        {
            TimedScope ts(2, st);
            s = yee_step<T>(g, gi, fp, src, step, it + 1 < nsteps, st, chain ? bh : nullptr, it == 0,
                            it + 1 == nsteps);
        }
        if (s != PIC_OK)
            return s;
        if (diag) {
            TimedScope ts(3, st);
            s = reduce_t<T>(g, gi, sp, f, diag + 5 * (int64_t)it, w, L, st);
            if (s != PIC_OK)
                return s;
        }
    }
    int herr = 0;
    PIC_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    PIC_HIP(hipStreamSynchronize(st));
    if (herr)
        return fail(PIC_E_STATE, "corrupt particle state (cell, offset, momentum or a displacement >= 1 cell)");
    return PIC_OK;
}

template <typename T>
pic_status adjoint_t(const pic_grid *g, const GridInfo &gi, const pic_species *sp, const pic_fields *f,
                     const int32_t *tile_start, const pic_source *src, int64_t step, pic_adjoint *lam, double *dA,
                     void *ws, const WsLayout &L, hipStream_t st)
{
    char *w = static_cast<char *>(ws);
    int *err = reinterpret_cast<int *>(w + L.err);
    T *hat[3], *vb[6];
    T *lE[3], *lB[3], *lx[3], *lu[3];
    const size_t np = (size_t)sp->n;
    for (int d = 0; d < 3; ++d) {
        hat[d] = reinterpret_cast<T *>(w + L.hatE + d * al(sizeof(T) * (size_t)gi.ncell));
        // the adjoints of the gathered fields pass between the two particle
        // passes in the sort's staging buffers, which the adjoint does not use
        vb[d] = reinterpret_cast<T *>(w + L.soff + d * al(sizeof(T) * np));
        vb[3 + d] = reinterpret_cast<T *>(w + L.su + d * al(sizeof(T) * np));
        lE[d] = static_cast<T *>(lam->lE[d]);
        lB[d] = static_cast<T *>(lam->lB[d]);
        lx[d] = static_cast<T *>(lam->lx[d]);
        lu[d] = static_cast<T *>(lam->lu[d]);
    }
    // with a gather filter the particle part reads the filtered fields and
    // scatters into the adjoints of the filtered fields (zeroed here), whose
    // filter transpose is added to lE, lB at the end
    const FieldPtrs<T> fpv = gather_view<T>(gi, fptrs<T>(f), w, L);
    T *glE[3], *glB[3];
    for (int d = 0; d < 3; ++d) {
        glE[d] = lE[d];
        glB[d] = lB[d];
        if (gi.filt) {
            const size_t a = al(sizeof(T) * (size_t)gi.ncell);
            glE[d] = reinterpret_cast<T *>(w + L.lfilt + d * a);
            glB[d] = reinterpret_cast<T *>(w + L.lfilt + (3 + d) * a);
        }
    }
    const double c2 = g->c * g->c;
    // hatE = lE - dt/2 curl_b(lB);  dA += g(step) hatE_x[k_plane]
    CurlArgs<T> a{};
    for (int d = 0; d < 3; ++d) {
        a.out[d] = hat[d];
        a.in[d] = lE[d];
        a.src[d] = lB[d];
        a.n[d] = gi.n[d];
    }
    a.cx = (T)(-0.5 * g->dt / g->d[0]);
    a.cy = (T)(-0.5 * g->dt / g->d[1]);
    a.cz = (T)(-0.5 * g->dt / g->d[2]);
    a.kplane = -1;
    if (src && src->k_plane >= 0 && dA) {
        a.kplane = src->k_plane;
        a.dA = dA;
        a.dag = src_g(src, step);
    }
    CurlArgs<T> b{};
    for (int d = 0; d < 3; ++d) {
        b.out[d] = lB[d];
        b.in[d] = lB[d];
        b.src[d] = hat[d];
        b.n[d] = gi.n[d];
    }
    b.cx = (T)(c2 * g->dt / g->d[0]);
    b.cy = (T)(c2 * g->dt / g->d[1]);
    b.cz = (T)(c2 * g->dt / g->d[2]);
    b.kplane = -1;
    // lE = hatE - dt/2 curl_b(lB)
    CurlArgs<T> e{};
    for (int d = 0; d < 3; ++d) {
        e.out[d] = lE[d];
        e.in[d] = hat[d];
        e.src[d] = lB[d];
        e.n[d] = gi.n[d];
    }
    e.cx = a.cx;
    e.cy = a.cy;
    e.cz = a.cz;
    e.kplane = -1;
    // transposes of the B update carry its CKC averaging (symmetric, and it
    // commutes with the differences); the E update's transpose is Yee's
    if (g->solver == PIC_SOLVER_CKC) {
        ckc_weights<T>(g, a);
        ckc_weights<T>(g, e);
    }
    PIC_HIP(launch_fill<int>(err, 1, 0, st));
    // the binning is checked on the device and reported with the state
    // errors at the end (no read-back before the launches)
    constexpr int bad_binning = 1 << 8;
    if (tile_start && sp->n > 0)
        PIC_HIP(launch_check_binning(tile_start, gi.ntiles, sp->n, err, bad_binning, st));
    {
        TimedScope tf(4, st);
        PIC_HIP(launch_curl<T>(false, a, st));   // hatE
        PIC_HIP(launch_curl<T>(true, b, st));    // lB += dt c^2 curl_f(hatE)
        PIC_HIP(launch_curl<T>(false, e, st));   // lE = hatE - dt/2 curl_b(lB)
    }
    // particles: deposit, position, Boris and gather transposes
    if (sp->n > 0) {
        TimedScope tp(5, st);
        const PConst<T> pc = make_const<T>(g, sp);
        // FP64 order 3 has no tiled transpose (the library does not build
        // one): that request takes the per-particle push and the segment-box
        // scatter with the binning, as does a tile whose regions exceed the
        // LDS.
        const bool tiled_ok = !(gi.dtype == PIC_F64 && gi.order == 3) && adj_lds_bytes(gi) <= (size_t)lds_limit();
        if (gi.filt) {
            PIC_TRY_S(filter_fields<T>(gi, fptrs<T>(f), fpv, st));
            for (int d = 0; d < 3; ++d) {
                PIC_HIP(launch_fill<T>(glE[d], gi.ncell, T(0), st));
                PIC_HIP(launch_fill<T>(glB[d], gi.ncell, T(0), st));
            }
        }
        if (tile_start && tiled_ok) {
            // Below 6 particles per cell, the particles that change cells are
            // split off (the others take the narrow window of the deposit
            // transpose) only when few do: sampled from the momenta, under 2 %
            // (a few leftover crossers per tile run alone at its end).
            bool split_sparse = false;
            if (gi.dtype == PIC_F32 && sp->n > 0 && sp->n < 6 * gi.ncell) {
                int *cnt = reinterpret_cast<int *>(w + L.err + 128);
                int64_t taken = 0;
                PIC_HIP(launch_cross_estimate<T>(pc, parr<T>(sp), int64_t(1) << 20, cnt, st, &taken));
                int hc = 0;
                PIC_HIP(hipMemcpyAsync(&hc, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
                PIC_HIP(hipStreamSynchronize(st));
                split_sparse = (int64_t)hc * 50 < taken;
            }
            PIC_HIP(launch_adjoint_tile<T>(gi.order, pc, adjoint_geo(gi), parr<T>(sp), fpv, hat, lx, lu, glE, glB,
                                           vb, tile_start, reinterpret_cast<int *>(w + L.rank),
                                           reinterpret_cast<int *>(w + L.err + 64),
                                           reinterpret_cast<int *>(w + L.key), split_sparse, err, st));
        } else {
            PIC_HIP(launch_adjoint_particles<T>(gi.order, pc, parr<T>(sp), fpv, hat, lx, lu, glE, glB, vb, tile_start,
                                                gi.ntiles, err, st));
        }
        if (gi.filt) {
            FieldPtrs<T> lsrc{}, ldst{};
            for (int d = 0; d < 3; ++d) {
                lsrc.E[d] = glE[d];
                lsrc.B[d] = glB[d];
                ldst.E[d] = lE[d];
                ldst.B[d] = lB[d];
            }
            PIC_TRY_S(filter_fields<T>(gi, lsrc, ldst, st, true));
        }
    }
    int herr = 0;
    PIC_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    PIC_HIP(hipStreamSynchronize(st));
    if (herr & bad_binning)
        return fail(PIC_E_INVALID, "tile_start is not a binning of these particles (it must run from 0 to n); "
                                   "sort them first (lam and dA are unspecified)");
    if (herr)
        return fail(PIC_E_STATE, "corrupt particle state (cell, offset, momentum or a displacement >= 1 cell)");
    return PIC_OK;
}

template <typename T>
pic_status energy_loss_t(const pic_grid *g, const GridInfo &gi, const pic_fields *f, int64_t np, double s,
                         pic_adjoint *lam, double *out, char *ws, const WsLayout &L, hipStream_t st)
{
    double *red5 = reinterpret_cast<double *>(ws + L.red5);
    PIC_TRY_S(reduce_t<T>(g, gi, nullptr, f, red5, ws, L, st));
    PIC_HIP(launch_sum2(red5, out, st));
    const double dV = g->d[0] * g->d[1] * g->d[2];
    const double mu0 = 1.0 / (g->eps0 * g->c * g->c);
    for (int d = 0; d < 3; ++d) {
        PIC_HIP(launch_scale<T>(static_cast<T *>(lam->lE[d]), static_cast<const T *>(f->E[d]), gi.ncell,
                                (T)(s * g->eps0 * dV), st));
        PIC_HIP(launch_scale<T>(static_cast<T *>(lam->lB[d]), static_cast<const T *>(f->B[d]), gi.ncell,
                                (T)(s * dV / mu0), st));
        if (np > 0) {
            PIC_HIP(launch_fill<T>(static_cast<T *>(lam->lx[d]), np, T(0), st));
            PIC_HIP(launch_fill<T>(static_cast<T *>(lam->lu[d]), np, T(0), st));
        }
    }
    return PIC_OK;
}

// Gauss-law residual: the species' charge density goes to the adjoint's
// hatE buffer (unused outside the adjoint; 3 T per cell >= one double)
template <typename T>
pic_status gauss_t(const pic_grid *g, const GridInfo &gi, const pic_species *sp, const pic_fields *f, double *out,
                   char *ws, const WsLayout &L, hipStream_t st)
{
    int *err = reinterpret_cast<int *>(ws + L.err);
    double *rho = reinterpret_cast<double *>(ws + L.hatE);
    double *red5 = reinterpret_cast<double *>(ws + L.red5);
    PIC_HIP(launch_fill<int>(err, 1, 0, st));
    PIC_HIP(launch_fill<double>(rho, gi.ncell, 0.0, st));
    PIC_TRY_S(reduce_t<T>(g, gi, sp, f, red5, ws, L, st));   // red5[3] = sum q w
    PIC_HIP(launch_gauss<T>(gi.order, parr<T>(sp), fptrs<T>(f), gi.n, g->d, sp->q, sp->w0, g->eps0, rho, red5 + 3,
                            reinterpret_cast<double *>(ws + L.partials), reduce_max_blocks(), out, err, st));
    int herr = 0;
    PIC_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    PIC_HIP(hipStreamSynchronize(st));
    if (herr)
        return fail(PIC_E_STATE, "particle with a cell outside the grid or an offset outside [0,1)");
    return PIC_OK;
}

pic_status check_vec3(void *const v[3], const char *name)
{
    if (!v)
        return fail(PIC_E_INVALID, std::string(name) + " is NULL");
    for (int d = 0; d < 3; ++d)
        if (!v[d])
            return fail(PIC_E_INVALID, std::string(name) + " has a NULL component");
    return PIC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// exported entry points

#define PIC_TRY(expr)                      \
    do {                                   \
        pic_status s_ = (expr);            \
        if (s_ != PIC_OK)                  \
            return s_;                     \
    } while (0)

extern "C" {

size_t pic_workspace_bytes(const pic_grid *grid, int64_t n_particles)
{
    GridInfo gi;
    if (check_grid(grid, gi) != PIC_OK)
        return 0;
    return layout(gi, n_particles).total;
}

int64_t pic_tile_count(const pic_grid *grid)
{
    GridInfo gi;
    if (check_grid(grid, gi) != PIC_OK)
        return 0;
    return gi.ntiles;
}

pic_status pic_tile_shape(const pic_grid *grid, int32_t *tile, int32_t *slack)
{
    GridInfo gi;
    PIC_TRY(check_grid(grid, gi));
    if (!tile || !slack)
        return fail(PIC_E_INVALID, "tile and slack must not be NULL");
    for (int d = 0; d < 3; ++d)
        tile[d] = gi.tg.t[d];
    *slack = gi.tg.slack;
    return PIC_OK;
}

pic_status pic_sort_tiles(const pic_grid *grid, pic_species *sp, int32_t *tile_start, int32_t *perm, void *ws,
                          size_t ws_bytes, void *stream)
{
    try {
        GridInfo gi;
        WsLayout L;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_species(sp, "species"));
        if (!tile_start)
            return fail(PIC_E_INVALID, "tile_start is NULL");
        PIC_TRY(check_ws(gi, sp->n, ws, ws_bytes, L));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (gi.dtype == PIC_F64)
            return sort_tiles_t<double>(grid, gi, sp, tile_start, perm, ws, L, st);
        return sort_tiles_t<float>(grid, gi, sp, tile_start, perm, ws, L, st);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_gather(const pic_grid *grid, const pic_species *sp, const pic_fields *f, void *const Ep[3],
                      void *const Bp[3], void *stream)
{
    try {
        GridInfo gi;
        PIC_TRY(check_grid(grid, gi));
        if (gi.filt)
            return fail(PIC_E_UNSUPPORTED, "pic_gather has no workspace for the gather filter (pic_step applies it)");
        PIC_TRY(check_species(sp, "species"));
        PIC_TRY(check_fields(f, false));
        PIC_TRY(check_vec3(Ep, "Ep"));
        PIC_TRY(check_vec3(Bp, "Bp"));
        int *err = sink_err();
        if (!err)
            return fail(PIC_E_DEVICE, "cannot resolve the device error word");
        hipStream_t st = static_cast<hipStream_t>(stream);
        PIC_TRY(sink_begin(err, st));
        if (gi.dtype == PIC_F64) {
            double *e[3], *b[3];
            for (int d = 0; d < 3; ++d) {
                e[d] = static_cast<double *>(Ep[d]);
                b[d] = static_cast<double *>(Bp[d]);
            }
            PIC_HIP(launch_gather<double>(gi.order, make_const<double>(grid, sp), parr<double>(sp), fptrs<double>(f),
                                          e, b, err, st));
        } else {
            float *e[3], *b[3];
            for (int d = 0; d < 3; ++d) {
                e[d] = static_cast<float *>(Ep[d]);
                b[d] = static_cast<float *>(Bp[d]);
            }
            PIC_HIP(launch_gather<float>(gi.order, make_const<float>(grid, sp), parr<float>(sp), fptrs<float>(f), e,
                                         b, err, st));
        }
        return sink_end(err, st, "particle with a cell outside the grid or an offset outside [0,1)");
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_push(const pic_grid *grid, pic_species *sp, void *const Ep[3], void *const Bp[3], void *stream)
{
    try {
        GridInfo gi;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_species(sp, "species"));
        PIC_TRY(check_vec3(Ep, "Ep"));
        PIC_TRY(check_vec3(Bp, "Bp"));
        int *err = sink_err();
        if (!err)
            return fail(PIC_E_DEVICE, "cannot resolve the device error word");
        hipStream_t st = static_cast<hipStream_t>(stream);
        PIC_TRY(sink_begin(err, st));
        if (gi.dtype == PIC_F64) {
            double *e[3], *b[3];
            for (int d = 0; d < 3; ++d) {
                e[d] = static_cast<double *>(Ep[d]);
                b[d] = static_cast<double *>(Bp[d]);
            }
            PIC_HIP(launch_push<double>(make_const<double>(grid, sp), parr<double>(sp), e, b, err, st));
        } else {
            float *e[3], *b[3];
            for (int d = 0; d < 3; ++d) {
                e[d] = static_cast<float *>(Ep[d]);
                b[d] = static_cast<float *>(Bp[d]);
            }
            PIC_HIP(launch_push<float>(make_const<float>(grid, sp), parr<float>(sp), e, b, err, st));
        }
        return sink_end(err, st, "corrupt particle state (cell, offset, momentum or a displacement >= 1 cell)");
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_deposit(const pic_grid *grid, const pic_species *before, const pic_species *after, pic_fields *f,
                       void *stream)
{
    try {
        GridInfo gi;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_species(before, "before"));
        PIC_TRY(check_species(after, "after"));
        if (before->n != after->n)
            return fail(PIC_E_INVALID, "before and after hold different particle counts");
        if (!f)
            return fail(PIC_E_INVALID, "fields is NULL");
        for (int d = 0; d < 3; ++d)
            if (!f->J[d])
                return fail(PIC_E_INVALID, "NULL current array");
        int *err = sink_err();
        if (!err)
            return fail(PIC_E_DEVICE, "cannot resolve the device error word");
        hipStream_t st = static_cast<hipStream_t>(stream);
        PIC_TRY(sink_begin(err, st));
        if (gi.dtype == PIC_F64)
            PIC_HIP(launch_deposit<double>(gi.order, make_const<double>(grid, before), parr<double>(before),
                                           parr<double>(after), fptrs<double>(f), err, st));
        else
            PIC_HIP(launch_deposit<float>(gi.order, make_const<float>(grid, before), parr<float>(before),
                                          parr<float>(after), fptrs<float>(f), err, st));
        return sink_end(err, st, "corrupt particle state or a displacement of a cell or more (its current is left out)");
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_yee(const pic_grid *grid, pic_fields *f, const pic_source *src, int64_t step, void *stream)
{
    try {
        GridInfo gi;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_fields(f, true));
        PIC_TRY(check_source(src, gi));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (gi.dtype == PIC_F64)
            return yee_step<double>(grid, gi, fptrs<double>(f), src, step, false, st);
        return yee_step<float>(grid, gi, fptrs<float>(f), src, step, false, st);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

// A binning handed in by the caller must at least span the particles: its
// first entry 0 and its last n (a binning of other particles, or an array
// never filled, would leave particles unprocessed).  Reads two ints.
pic_status check_binning(const GridInfo &gi, const int32_t *tile_start, int64_t n, hipStream_t st)
{
    int32_t ends[2] = {-1, -1};
    PIC_HIP(hipMemcpyAsync(&ends[0], tile_start, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PIC_HIP(hipMemcpyAsync(&ends[1], tile_start + gi.ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PIC_HIP(hipStreamSynchronize(st));
    if (ends[0] != 0 || ends[1] != n)
        return fail(PIC_E_INVALID, "tile_start is not a binning of these particles (it must run from 0 to n); "
                                   "sort them first");
    return PIC_OK;
}

pic_status pic_step(const pic_grid *grid, pic_species *sp, pic_fields *f, const pic_source *src, int64_t step0,
                    int32_t nsteps, int32_t sort_every, int32_t *tile_start, void *ws, size_t ws_bytes,
                    double *diag, void *stream)
{
    try {
        GridInfo gi;
        WsLayout L;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_species(sp, "species"));
        PIC_TRY(check_fields(f, true));
        PIC_TRY(check_source(src, gi));
        if (nsteps < 0)
            return fail(PIC_E_INVALID, "nsteps must be >= 0");
        if (sort_every < 0)
            return fail(PIC_E_INVALID, "sort_every must be >= 0");
        if (sort_every > 0 && !tile_start)
            return fail(PIC_E_INVALID, "sorting needs a tile_start array");
        PIC_TRY(check_ws(gi, sp->n, ws, ws_bytes, L));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (sort_every == 0 && tile_start && sp->n > 0 && nsteps > 0)
            PIC_TRY(check_binning(gi, tile_start, sp->n, st));
        if (gi.dtype == PIC_F64)
            return step_t<double>(grid, gi, sp, f, src, step0, nsteps, sort_every, tile_start, ws, L, diag, st);
        return step_t<float>(grid, gi, sp, f, src, step0, nsteps, sort_every, tile_start, ws, L, diag, st);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_step_noalloc(const pic_grid *grid, pic_species *sp, pic_fields *f, const pic_source *src,
                            int64_t step0, int32_t nsteps, int32_t sort_every, int32_t *tile_start, double *diag,
                            void *stream)
{
    try {
        GridInfo gi;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_species(sp, "species"));
        const size_t need = layout(gi, sp->n).total;
        if (need > PIC_NOALLOC_SCRATCH_BYTES)
            return fail(PIC_E_WORKSPACE, "pic_step_noalloc: this grid and particle count need " + std::to_string(need) +
                                             " bytes of scratch, more than the static " +
                                             std::to_string((size_t)PIC_NOALLOC_SCRATCH_BYTES) +
                                             " bytes; use pic_step with a workspace");
        void *ws = nullptr;
        PIC_TRY(scratch_address(&ws));
        struct Untimed {
            Untimed() { g_untimed = true; }
            ~Untimed() { g_untimed = false; }
        } untimed;
        return pic_step(grid, sp, f, src, step0, nsteps, sort_every, tile_start, ws, PIC_NOALLOC_SCRATCH_BYTES, diag,
                        stream);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_step_adjoint(const pic_grid *grid, const pic_species *state_n, const pic_fields *fields_n,
                            const int32_t *tile_start, const pic_source *src, int64_t step, pic_adjoint *lam,
                            double *dA, void *ws, size_t ws_bytes, void *stream)
{
    try {
        GridInfo gi;
        WsLayout L;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_species(state_n, "state_n"));
        PIC_TRY(check_fields(fields_n, false));
        PIC_TRY(check_source(src, gi));
        if (!lam)
            return fail(PIC_E_INVALID, "adjoint state is NULL");
        for (int d = 0; d < 3; ++d)
            if (!lam->lE[d] || !lam->lB[d] || (state_n->n > 0 && (!lam->lx[d] || !lam->lu[d])))
                return fail(PIC_E_INVALID, "NULL adjoint array");
        PIC_TRY(check_ws(gi, state_n->n, ws, ws_bytes, L));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (gi.dtype == PIC_F64)
            return adjoint_t<double>(grid, gi, state_n, fields_n, tile_start, src, step, lam, dA, ws, L, st);
        return adjoint_t<float>(grid, gi, state_n, fields_n, tile_start, src, step, lam, dA, ws, L, st);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_reduce(const pic_grid *grid, const pic_species *sp, const pic_fields *f, double *out, void *ws,
                      size_t ws_bytes, void *stream)
{
    try {
        GridInfo gi;
        WsLayout L;
        PIC_TRY(check_grid(grid, gi));
        if (sp)
            PIC_TRY(check_species(sp, "species"));
        PIC_TRY(check_fields(f, false));
        if (!out)
            return fail(PIC_E_INVALID, "out is NULL");
        PIC_TRY(check_ws(gi, sp ? sp->n : 0, ws, ws_bytes, L));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (gi.dtype == PIC_F64)
            return reduce_t<double>(grid, gi, sp, f, out, static_cast<char *>(ws), L, st);
        return reduce_t<float>(grid, gi, sp, f, out, static_cast<char *>(ws), L, st);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_gauss_residual(const pic_grid *grid, const pic_species *sp, const pic_fields *f, double *out,
                              void *ws, size_t ws_bytes, void *stream)
{
    try {
        GridInfo gi;
        WsLayout L;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_species(sp, "species"));
        PIC_TRY(check_fields(f, false));
        if (!out)
            return fail(PIC_E_INVALID, "out is NULL");
        PIC_TRY(check_ws(gi, sp->n, ws, ws_bytes, L));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (gi.dtype == PIC_F64)
            return gauss_t<double>(grid, gi, sp, f, out, static_cast<char *>(ws), L, st);
        return gauss_t<float>(grid, gi, sp, f, out, static_cast<char *>(ws), L, st);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

pic_status pic_timing(int enable, double *ms, int64_t *count, int n)
{
    std::lock_guard<std::mutex> lk(g_timer_mu);
    timer_flush();
    for (int c = 0; c < n && c < NCAT; ++c) {
        if (ms)
            ms[c] = g_timer.ms[c];
        if (count)
            count[c] = g_timer.cnt[c];
    }
    for (int c = 0; c < NCAT; ++c) {
        g_timer.ms[c] = 0.0;
        g_timer.cnt[c] = 0;
    }
    g_timer.on = enable != 0;
    return PIC_OK;
}

pic_status pic_energy_loss(const pic_grid *grid, const pic_fields *f, int64_t n_particles, double s,
                           pic_adjoint *lam, double *out, void *ws, size_t ws_bytes, void *stream)
{
    try {
        GridInfo gi;
        WsLayout L;
        PIC_TRY(check_grid(grid, gi));
        PIC_TRY(check_fields(f, false));
        if (!lam || !out)
            return fail(PIC_E_INVALID, "lam and out must not be NULL");
        if (n_particles < 0)
            return fail(PIC_E_INVALID, "n_particles must be >= 0");
        for (int d = 0; d < 3; ++d)
            if (!lam->lE[d] || !lam->lB[d] || (n_particles > 0 && (!lam->lx[d] || !lam->lu[d])))
                return fail(PIC_E_INVALID, "NULL adjoint array");
        if (!std::isfinite(s))
            return fail(PIC_E_INVALID, "seed scale must be finite");
        PIC_TRY(check_ws(gi, 0, ws, ws_bytes, L));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (gi.dtype == PIC_F64)
            return energy_loss_t<double>(grid, gi, f, n_particles, s, lam, out, static_cast<char *>(ws), L, st);
        return energy_loss_t<float>(grid, gi, f, n_particles, s, lam, out, static_cast<char *>(ws), L, st);
    } catch (...) {
        return fail(PIC_E_DEVICE, "unexpected host exception");
    }
}

const char *pic_last_error(void)
{
    return g_msg.c_str();
}

}  // extern "C"
