// Particle kernels of the EM-PIC step for gfx950.
//
//  k_particles_tile   one workgroup per tile: E and B of the tile plus the
//                     gather halo are staged in LDS, the current of the tile
//                     plus the deposit halo is accumulated in LDS with LDS
//                     atomics and flushed with one global atomic per touched
//                     value (a single-GPU analogue of the paper's guard-cell
//                     FillBoundary / SumBoundary, Sec. 2.4).  Particles are
//                     gathered, pushed, moved and deposited in one pass, so
//                     per-particle fields are never stored (Sec. 3.1).
//  k_particles_global the same fused step without tiles (global memory and
//                     global atomics, the paper's GPU deposition, Sec. 3.4.1)
//  k_gather / k_push / k_deposit   the separate operations
//  k_adjoint_push / k_adjoint_scatter_box (and their tiled forms)
//                     transpose of the particle part of a step, two passes
#include "pic_device.hpp"
#include "pic_types.hpp"

namespace pic {

// threads per tile workgroup: at 8 particles per cell and 8^3-cell tiles each
// thread takes about one cell's particles, so neighbouring lanes touch
// neighbouring LDS words
constexpr int TILE_THREADS = 512;
// FP32 fits the fused step in 128 registers, so its tiles run 16 waves per CU;
// FP64 needs more registers and runs 8
template <typename T>
struct TileThreads {
    static constexpr int value = sizeof(T) == 4 ? 1024 : 512;
};

template <typename T>
__device__ inline void gatomic_add(T *p, T v)
{
    unsafeAtomicAdd(p, v);
}

template <typename T>
__device__ inline void latomic_add(T *p, T v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline int wrap_once(int v, int n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

__device__ inline int wrap_any(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// momentum update of the push: Boris or Vay (uniform across the launch)
template <typename T>
__device__ inline void push_momentum(const PConst<T> &pc, const T *u, const T *E, const T *B, T *u1)
{
    if (pc.vay) {
        vay(pc.h, pc.inv_c2, u, E, B, u1);
    } else {
        BorisTape<T> tp;
        boris(pc.h, pc.inv_c2, u, E, B, u1, tp);
    }
}

template <typename T>
__device__ inline bool finite3(const T *u)
{
    return isfinite(u[0]) & isfinite(u[1]) & isfinite(u[2]);
}

// Load a particle and check its state; returns false (and flags err) for a
// cell outside [0,n), an offset outside [0,1) or a non-finite momentum.
// the state words of particle p, unchecked
template <typename T>
__device__ __attribute__((always_inline)) inline void load_state(const PArr<T> &in, int64_t p, int *c, T *f, T *u)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = in.cell[d][p];
        f[d] = in.off[d][p];
        u[d] = in.u[d][p];
    }
}

// true for a valid state (cell in the grid, offsets in [0,1), finite
// momentum); an invalid one sets bit 0 of the error word
template <typename T>
__device__ inline bool check_state(const int *n, const int *c, const T *f, const T *u, int *err)
{
    // no short-circuit branches: a branch between the loads of load_state
    // and their uses lets the compiler move later loads behind earlier checks
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        ok = ok & (c[d] >= 0) & (c[d] < n[d]) & (f[d] >= T(0)) & (f[d] < T(1));
    ok = ok & finite3(u);
    if (!ok)
        atomicOr(err, 1);
    return ok;
}

template <typename T>
__device__ inline bool load_particle(const PArr<T> &in, int64_t p, const int *n, int *c, T *f, T *u, int *err)
{
    load_state(in, p, c, f, u);
    return check_state(n, c, f, u, err);
}

template <typename T>
__device__ inline void copy_particle(const PArr<T> &in, const PArr<T> &out, int64_t p)
{
    if (in.cell[0] == out.cell[0])
        return;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        out.cell[d][p] = in.cell[d][p];
        out.off[d][p] = in.off[d][p];
        out.u[d][p] = in.u[d][p];
    }
    if (out.w)
        out.w[p] = in.w[p];
}

// ---------------------------------------------------------------------------
// tiles

template <typename T>
__device__ inline FieldSrc<T> global_fields(const FieldPtrs<T> &fp)
{
    FieldSrc<T> gf;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        gf.c[m] = fp.E[m];
        gf.c[3 + m] = fp.B[m];
    }
    return gf;
}

struct TileSpan {
    int t;       // logical tile index (x fastest)
    int t0[3];
    int64_t ps, pe;
};

__device__ inline TileSpan tile_span(const TileGeo &tg, const int *tile_start, int64_t N)
{
    const int ntiles = tg.nt[0] * tg.nt[1] * tg.nt[2];
    int t = blockIdx.x;
    if (tg.xcd_map)
        t = (t & 7) * (ntiles >> 3) + (t >> 3);
    TileSpan s;
    s.t = t;
    s.t0[0] = (t % tg.nt[0]) * tg.t[0];
    s.t0[1] = ((t / tg.nt[0]) % tg.nt[1]) * tg.t[1];
    s.t0[2] = (t / (tg.nt[0] * tg.nt[1])) * tg.t[2];
    int64_t ps = tile_start[t], pe = tile_start[t + 1];
    ps = ps < 0 ? 0 : (ps > N ? N : ps);
    pe = pe < ps ? ps : (pe > N ? N : pe);
    s.ps = ps;
    s.pe = pe;
    return s;
}

// cell position relative to the tile origin, periodic; true when inside
__device__ inline bool tile_local(const TileGeo &tg, const int *n, const int *t0, const int *c, int *l)
{
    bool inside = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int v = c[d] - t0[d];
        if (v < -tg.slack)
            v += n[d];
        else if (v >= tg.t[d] + tg.slack)
            v -= n[d];
        l[d] = v;
        inside = inside && v >= -tg.slack && v < tg.t[d] + tg.slack;
    }
    return inside;
}

// logical tile of a cell, and the first cell of a tile
__device__ __attribute__((always_inline)) inline int cell_tile(const TileGeo &tg, const int *c)
{
    return c[0] / tg.t[0] + tg.nt[0] * (c[1] / tg.t[1] + tg.nt[1] * (c[2] / tg.t[2]));
}

__device__ __attribute__((always_inline)) inline void tile_origin(const TileGeo &tg, int t, int *t0)
{
    t0[0] = (t % tg.nt[0]) * tg.t[0];
    t0[1] = ((t / tg.nt[0]) % tg.nt[1]) * tg.t[1];
    t0[2] = (t / (tg.nt[0] * tg.nt[1])) * tg.t[2];
}

// Status of a moved particle for the next step: 0 if its new cell c1 is in
// its home tile's region (or no list slot is free, which leaves it to the
// stray kernel), 1 once it is listed as a guest of the tile holding c1.
__device__ __attribute__((always_inline)) inline unsigned char guest_next(const GuestArgs &g, const TileGeo &tg, const int *n, int64_t p, int home,
                                           const int *home_t0, const int *c1)
{
    int l[3];
    if (tile_local(tg, n, home_t0, c1, l) || p > 0x7fffffff)
        return 0;
    const int host = cell_tile(tg, c1);
    const int slot = atomicAdd(g.cnt_next + host, 1);
    if (slot >= g.cap)
        return 0;
    g.list_next[(int64_t)host * g.cap + slot] = make_int2((int)p, home);
    return 1;
}

// Walk of a tile region (ex x ey x ez cells from t0 - lo, x fastest, LDS row
// pitch px >= ex) by the whole workgroup without integer divisions in the
// loop: a thread keeps one x (its position in a group of LX lanes, LX the
// power of two >= ex) and steps over the rows (y, z) by blockDim.x / LX,
// carrying y into z.  fn(local index, global index) runs once per cell.
// With once, every axis of the region wraps at most once around the grid
// (see region_wraps_once), else each row takes the general wrap.
template <typename Fn>
__device__ __attribute__((always_inline)) inline void region_walk(const int *n, const int *t0, int lo, int ex,
                                                                   int ey, int ez, int px, bool once, Fn &&fn)
{
    const int lb = ex > 1 ? 32 - __clz(ex - 1) : 0;
    const int x = (int)threadIdx.x & ((1 << lb) - 1);
    const int step = (int)blockDim.x >> lb;   // >= 1: regions are at most 64 cells wide
    if (x >= ex || step == 0)
        return;
    int row = (int)threadIdx.x >> lb;
    int y = row % ey, z = row / ey;
    const int sy = step % ey, sz = step / ey;
    const int gx = wrap_any(t0[0] - lo + x, n[0]);
    const int nrow = ey * ez;
    for (; row < nrow; row += step) {
        const int vy = t0[1] - lo + y, vz = t0[2] - lo + z;
        const int gy = once ? wrap_once(vy, n[1]) : wrap_any(vy, n[1]);
        const int gz = once ? wrap_once(vz, n[2]) : wrap_any(vz, n[2]);
        fn(x + px * (y + ey * z), gx + n[0] * (gy + n[1] * gz));
        y += sy;
        z += sz;
        if (y >= ey) {
            y -= ey;
            ++z;
        }
    }
}

// true when the region of extents e starting lo cells below a tile of
// extents t wraps each axis of the grid at most once (wrap_once suffices)
__device__ inline bool region_wraps_once(const int *n, const int *t, int lo, const int *e)
{
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        ok = ok && lo <= n[d] && e[d] - t[d] - lo <= n[d];
    return ok;
}

// Particles of a tile whose cell lies outside the tile's regions (they
// drifted since the binning) are left out by the tile kernels and taken by
// the stray kernels below, which first gather a chunk's strays into an LDS
// list so that they run in full waves rather than as a few divergent lanes
// of every wave.
constexpr int STRAY_THREADS = 256;
constexpr int STRAY_CHUNK = 4096;

// Collect the in-tile indices j in [j0, j0 + STRAY_CHUNK) for which
// is_stray(p) holds into the LDS list; returns the count.
template <typename Pred>
__device__ inline int collect_strays(const TileSpan &ts, int j0, int *list, int *cnt, Pred &&is_stray)
{
    if (threadIdx.x == 0)
        *cnt = 0;
    __syncthreads();
    const int np = (int)(ts.pe - ts.ps);
    const int je = np < j0 + STRAY_CHUNK ? np : j0 + STRAY_CHUNK;
    for (int j = j0 + (int)threadIdx.x; j < je; j += blockDim.x)
        if (is_stray(ts.ps + j))
            list[atomicAdd(cnt, 1)] = j;
    __syncthreads();
    const int k = *cnt;
    __syncthreads();   // every thread has the count before the next reset
    return k;
}

// A list of strays on the device, appended to by the tile kernels (one
// atomic per wave) and worked through by the stray kernels; cnt is cleared
// before the tile kernel runs.  cap >= the particle count.
struct StrayList {
    int *p;
    int *cnt;
    int cap;
};

// appends p for every lane with `want`; call with the whole wave converged
__device__ inline void stray_append(bool want, int p, const StrayList &sl)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long m = __ballot(want);
    if (m == 0)
        return;   // uniform across the wave
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader)
        base = atomicAdd(sl.cnt, __popcll(m));
    base = __shfl(base, leader);
    if (want) {
        const int i = base + __popcll(m & ((1ull << lane) - 1ull));
        if (i < sl.cap)
            sl.p[i] = p;
    }
}

// stray test from the cell (for kernels that do not move particles); an
// invalid cell is not a stray, the tile kernel flags it
template <typename T>
struct CellStray {
    const TileGeo &tg;
    const int *n;
    const TileSpan &ts;
    const PArr<T> &sp;
    __device__ bool operator()(int64_t p) const
    {
        int c[3], l[3];
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            c[d] = sp.cell[d][p];
            ok = ok && c[d] >= 0 && c[d] < n[d];
        }
        return ok && !tile_local(tg, n, ts.t0, c, l);
    }
};

// ---------------------------------------------------------------------------
// LDS queue of the cell-crossing particles of a tile.  Nearly every wave
// holds a few particles that cross a cell face, and the rim of their wider
// Esirkepov window would make every wave issue the rim's LDS atomics with
// only those lanes active.  The tile kernel deposits the particles that stay
// in their cells with the narrow window and queues the others (their
// in-tile index, local cell, cell change and old / new offsets), then
// deposits the queue in full waves.  A particle that finds the queue full
// is deposited at once.
template <typename T>
struct CrossQueue {
    int *cnt;
    int cap;
    int *j, *pk;
    T *f0, *f1;   // [3][cap]

    __device__ bool push(int jj, const int *l, const int *kap, const T *a, const T *b) const
    {
        const int i = atomicAdd(cnt, 1);
        if (i >= cap)
            return false;
        j[i] = jj;
        pk[i] = pack(l, kap);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f0[d * cap + i] = a[d];
            f1[d * cap + i] = b[d];
        }
        return true;
    }
    // local cell + 8 in 5 bits and the cell change + 1 in 2 bits per axis
    __device__ static int pack(const int *l, const int *kap)
    {
        int v = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            v |= ((l[d] + 8) | ((kap[d] + 1) << 5)) << (7 * d);
        return v;
    }
    __device__ static void unpack(int v, int *l, int *kap)
    {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int x = (v >> (7 * d)) & 127;
            l[d] = (x & 31) - 8;
            kap[d] = (x >> 5) - 1;
        }
    }
};

// Esirkepov deposit with the full window into the LDS current tile; with
// MSEL in 0..2 only that component
template <typename T, int O, int MSEL = -1>
__device__ __attribute__((always_inline)) inline void deposit_local_full(const PConst<T> &pc, const T *f0, const T *f1, const int *kap,
                                          const int *l, int lo_j, const int *sj, T w, double *sJ, int rjvol)
{
    constexpr int NW = Shape<O, T>::NW;
    EskAxis<O, T> e[3];
    T K[3];
    int jo[3][NW + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        esk_axis<O>(f0[d], f1[d], kap[d], e[d]);
        K[d] = pc.jk[d] * w;
        axis_offsets_local<NW + 1>(l[d] + lo_j, e[d].lo, sj[d], jo[d]);
    }
    esk_scatter<O, T, double, MSEL>(e, jo, K,
                                    [&](int m, int idx, double v) { latomic_add(sJ + m * rjvol + idx, v); });
}

// One particle through gather -> Boris -> move; writes the new state to
// `out` and returns the new offsets f1, the cell change kap and the weight
// w, or flags the error word and returns false for a displacement of a cell
// or more.  With LOCAL the fields come from the LDS tile (positions l[]
// relative to the tile), otherwise from global memory.
template <typename T, int O, bool LOCAL, bool WOFF = true>
__device__ __attribute__((always_inline)) inline bool particle_advance(const PConst<T> &pc, const PArr<T> &in, const PArr<T> &out,
                                        const FieldSrc<T> &fsrc, int64_t p, const int *c, const T *f,
                                        const T *u, const int *l, int lo_f, const int *sf, T *f1, int *kap,
                                        T &w, int *err)
{
    constexpr int NW = Shape<O, T>::NW;
    const int gs[3] = {1, pc.n[0], pc.n[0] * pc.n[1]};
    AxisW<O, T> aw[3];
    int on[3][NW], os[3][NW];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        axis_weights<O>(f[d], aw[d]);
        if (LOCAL) {
            axis_offsets_local<NW>(l[d] + lo_f, aw[d].bn, sf[d], on[d]);
            axis_offsets_local<NW>(l[d] + lo_f, aw[d].bs, sf[d], os[d]);
        } else {
            axis_offsets_global<NW>(c[d], aw[d].bn, pc.n[d], gs[d], on[d]);
            axis_offsets_global<NW>(c[d], aw[d].bs, pc.n[d], gs[d], os[d]);
        }
    }
    T E[3], B[3];
    gather_eb<O>(fsrc, aw, on, os, E, B);

    T u1[3];
    push_momentum(pc, u, E, B, u1);
    const T ig = T(1) / sqrt(T(1) + (u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]) * pc.inv_c2);
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T disp = pc.dtd[d] * u1[d] * ig;
        ok = ok && fabs(disp) < T(1);
        move_axis(f[d], disp, f1[d], kap[d]);
    }
    if (!ok) {
        atomicOr(err, 2);
        copy_particle(in, out, p);
        return false;
    }
    w = in.w ? in.w[p] : pc.w0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        out.cell[d][p] = wrap_once(c[d] + kap[d], pc.n[d]);
        if (WOFF)
            out.off[d][p] = f1[d];
        out.u[d][p] = u1[d];
    }
    if (out.w && out.w != in.w)
        out.w[p] = in.w[p];
    return true;
}

// The fused step on global memory (global atomics for the current).
template <typename T, int O>
__device__ __attribute__((always_inline)) inline void particle_step_global(const PConst<T> &pc, const PArr<T> &in, const PArr<T> &out,
                                            const FieldPtrs<T> &fp, int64_t p, const int *c, const T *f,
                                            const T *u, int *err)
{
    constexpr int NW = Shape<O, T>::NW;
    const int gs[3] = {1, pc.n[0], pc.n[0] * pc.n[1]};
    const int z3[3] = {0, 0, 0};
    T f1[3], w;
    int kap[3];
    if (!particle_advance<T, O, false>(pc, in, out, global_fields(fp), p, c, f, u, z3, 0, z3, f1, kap, w, err))
        return;
    EskAxis<O, T> e[3];
    T K[3];
    int jo[3][NW + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        esk_axis<O>(f[d], f1[d], kap[d], e[d]);
        K[d] = pc.jk[d] * w;
        axis_offsets_global<NW + 1>(c[d], e[d].lo, pc.n[d], gs[d], jo[d]);
    }
    esk_scatter<O, T, T>(e, jo, K, [&](int m, int idx, T v) { gatomic_add(fp.J[m] + idx, v); });
}

// ---------------------------------------------------------------------------
// Lane-shared current rows.  In the rank-major order the lanes of a wave sit
// in neighbouring cells, so a lane's window row along x overlaps the rows of
// the lanes to its left shifted by one node per lane.  A run is a maximal
// group of consecutive lanes (within one 16-lane DPP row) whose particles
// stay in their cells and lie in consecutive cells along x of one (y, z)
// row.  Each lane adds the taps of up to three lanes to its left that land
// on its first node (row shifts across lanes) and writes that node with one
// LDS atomic; the last lane of a run also writes the remaining nodes.  The
// values added are those of the per-lane scatter; only the summation order
// changes, and a wave issues far fewer lane atomics, spread over more banks.

// Row shifts within 16-lane DPP rows: K > 0 gives lane L the value of lane
// L-K, K < 0 that of lane L+|K| (0 where the source is outside the row).
template <int K>
__device__ inline int dpp_shift_int(int v)
{
    constexpr int CTRL = K > 0 ? 0x110 + K : 0x100 - K;   // row_shr:K / row_shl:-K
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}

template <int K>
__device__ inline float dpp_shift(float v)
{
    return __int_as_float(dpp_shift_int<K>(__float_as_int(v)));
}

template <int K>
__device__ inline double dpp_shift(double v, int = 0)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_shift_int<K>((int)(b & 0xffffffffLL));
    const int hi = dpp_shift_int<K>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

struct XRun {
    bool a1;     // lane L-1 belongs to this lane's run
    bool last;   // the run ends at this lane
    bool send;   // lane L+1 belongs to this lane's run
    int d;       // lanes between this one and its run's last lane (4: more, or no run)
    int len;     // at the last lane: the run's length, counted up to 4
};

// key: 0 for a lane outside the shared deposit, else a positive code of the
// first window node with x in the low bits (x - 1 is key - 1).  Call with the
// whole wave converged.
__device__ inline int xrun_key(const int *l)
{
    return (1 << 20) | (l[0] + 8) | ((l[1] + 8) << 6) | ((l[2] + 8) << 12);
}

__device__ inline XRun xrun(int key)
{
    const int k1 = dpp_shift_int<1>(key);
    const bool a1 = key != 0 && k1 == key - 1;
    const int a1i = a1 ? 1 : 0;
    const bool send = dpp_shift_int<-1>(a1i) != 0;
    const bool last = key != 0 && !send;
    // flags of the lanes to the right: bit 0 "aligned to its left", bit 1 "last"
    const int f = a1i | (last ? 2 : 0);
    const int f1 = dpp_shift_int<-1>(f), f2 = dpp_shift_int<-2>(f), f3 = dpp_shift_int<-3>(f);
    XRun r;
    r.a1 = a1;
    r.last = last;
    r.send = send;
    r.d = last ? 0
               : ((f1 & 3) == 3) ? 1
                                 : ((f1 & 1) && (f2 & 3) == 3) ? 2 : ((f1 & 1) && (f2 & 1) && (f3 & 3) == 3) ? 3 : 4;
    const int b1 = dpp_shift_int<1>(a1i), b2 = dpp_shift_int<2>(a1i);
    r.len = 1 + (a1 ? 1 + (b1 ? 1 + (b2 ? 1 : 0) : 0) : 0);
    return r;
}

// One window row of NT taps along x, starting at `row` (this lane's first
// node).  Node k of this lane collects its own tap k and, through the run,
// tap k+1 of the lane to its left, tap k+2 of the next one and so on:
// e[k] = r[k] + e_left[k+1], built from the last tap down.  Every lane writes
// e[0]; the run's last lane R holds e[1..NT-1] for the nodes past the run,
// and lane R-d writes e_R[d+1] (node X_R + d + 1) in a second instruction,
// so a row costs two LDS instructions; a run shorter than NT - 1 lanes
// leaves the rest to its last lane.  V is the type the row is summed in; the
// LDS accumulators are FP64.
template <int NT, typename V>
__device__ __attribute__((always_inline)) inline void xrow_add(double *row, const V *r, const XRun &xr)
{
    V e[NT];
    e[NT - 1] = r[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 0; --k) {
        // the sender masks, so the shift can fold into the add
        const V snd = xr.send ? e[k + 1] : V(0);
        e[k] = r[k] + dpp_shift<1>(snd);
    }
    latomic_add(row, (double)e[0]);
    if constexpr (NT >= 2) {
        V x = e[1];
        int off = xr.d == 0 ? 1 : -1;
        if constexpr (NT >= 3) {
            const V t = dpp_shift<-1>(e[2]);
            if (xr.d == 1) {
                x = t;
                off = 3;
            }
        }
        if constexpr (NT >= 4) {
            const V t = dpp_shift<-2>(e[3]);
            if (xr.d == 2) {
                x = t;
                off = 5;
            }
        }
        if constexpr (NT >= 5) {
            const V t = dpp_shift<-3>(e[4]);
            if (xr.d == 3) {
                x = t;
                off = 7;
            }
        }
        if (off > 0)
            latomic_add(row + off, (double)x);
        if (xr.last && xr.len < NT - 1) {
#pragma unroll
            for (int k = 2; k < NT; ++k)
                if (k > xr.len)
                    latomic_add(row + k, (double)e[k]);
        }
    }
}

// The same row on global memory: add(k, v) adds v to node k of this lane's
// window (the lane's own, wrapped, node indices); the run's last lane writes
// the nodes past the run itself.
template <int NT, typename V, typename AddFn>
__device__ __attribute__((always_inline)) inline void xrow_apply(const V *r, const XRun &xr, AddFn &&add)
{
    V e[NT];
    e[NT - 1] = r[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 0; --k) {
        const V snd = xr.send ? e[k + 1] : V(0);
        e[k] = r[k] + dpp_shift<1>(snd);
    }
    add(0, e[0]);
    if (xr.last) {
#pragma unroll
        for (int k = 1; k < NT; ++k)
            add(k, e[k]);
    }
}

// run key of a window starting at the unwrapped global node st (0 where the
// grid is too large to encode, which turns the sharing off)
__device__ inline int xrun_key_global(const int *st, const int *n)
{
    const long long k = 1 + (long long)(st[0] + 8) +
                        (long long)(n[0] + 16) * ((st[1] + 8) + (long long)(n[1] + 16) * (st[2] + 8));
    return k < (1LL << 31) ? (int)k : 0;
}

// Esirkepov deposit of a particle that stays in its cell, into the LDS
// current tile with lane-shared rows along x: esk_scatter_still's values,
// formed and summed along the run in the working precision and added to the
// FP64 accumulators.
template <typename T, int O>
__device__ __attribute__((always_inline)) inline void deposit_still_shared(const PConst<T> &pc, const T *f0, const T *f1, const int *l,
                                            int lo_j, const int *sj, T w, double *sJ, int rjvol, const XRun &xr)
{
    constexpr int NW = Shape<O, T>::NW;
    const T half = T(0.5), third = T(1) / T(3);
    T S0[3][NW], DS[3][NW], K[3];
    int jo[3][NW];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        esk_axis_still<O>(f0[d], f1[d], S0[d], DS[d]);
        K[d] = pc.jk[d] * w;
        axis_offsets_local<NW>(l[d] + lo_j, Shape<O, T>::NB, sj[d], jo[d]);
    }
    // P_m[a] = K_m * (running sum of DS_m), a < NW - 1
    T P[3][NW - 1];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T run = T(0);
#pragma unroll
        for (int a = 0; a < NW - 1; ++a) {
            run += DS[m][a];
            P[m][a] = K[m] * run;
        }
    }
    // C for (p, q) at (b, c), as in esk_scatter_still
    auto cw = [&](int p, int q, int b, int c) -> T {
        return S0[p][b] * (S0[q][c] + half * DS[q][c]) + DS[p][b] * (half * S0[q][c] + third * DS[q][c]);
    };
    // J_x (p = y, q = z): rows along x are the taps a
#pragma unroll
    for (int c = 0; c < NW; ++c)
#pragma unroll
        for (int b = 0; b < NW; ++b) {
            const T C = cw(1, 2, b, c);
            T r[NW - 1];
#pragma unroll
            for (int a = 0; a < NW - 1; ++a)
                r[a] = P[0][a] * C;
            xrow_add<NW - 1>(sJ + jo[1][b] + jo[2][c] + jo[0][0], r, xr);
        }
    // J_y (p = z, q = x): rows along x are the taps c
#pragma unroll
    for (int a = 0; a < NW - 1; ++a)
#pragma unroll
        for (int b = 0; b < NW; ++b) {
            T r[NW];
#pragma unroll
            for (int c = 0; c < NW; ++c)
                r[c] = P[1][a] * cw(2, 0, b, c);
            xrow_add<NW>(sJ + rjvol + jo[2][b] + jo[1][a] + jo[0][0], r, xr);
        }
    // J_z (p = x, q = y): rows along x are the taps b
#pragma unroll
    for (int a = 0; a < NW - 1; ++a)
#pragma unroll
        for (int c = 0; c < NW; ++c) {
            T r[NW];
#pragma unroll
            for (int b = 0; b < NW; ++b)
                r[b] = P[2][a] * cw(0, 1, b, c);
            xrow_add<NW>(sJ + 2 * rjvol + jo[1][c] + jo[2][a] + jo[0][0], r, xr);
        }
}

// ---------------------------------------------------------------------------
// The particles left to k_particles_strays are listed (`strays`) before they
// move: when the step runs in place their cells are overwritten, so the
// stray kernel could not tell them from the cells any more.
template <typename T, int O, bool G>
__global__ void __launch_bounds__(TileThreads<T>::value) k_particles_tile(PConst<T> pc, TileGeo tg, PArr<T> in, PArr<T> out,
                                                        FieldPtrs<T> fp, const int *__restrict__ tile_start,
                                                        StrayList strays, GuestArgs g, int *err)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sF = reinterpret_cast<T *>(smem_raw);
    const int rfx = tg.rf[0], rfy = tg.rf[1];
    const int rfvol = rfx * rfy * tg.rf[2];
    const int rjx = tg.rj[0], rjy = tg.rj[1], jpx = tg.jp;
    const int rjvol = jpx * rjy * tg.rj[2];   // rows padded to jp values
    // the current tile accumulates in FP64 (fast LDS atomics), after the fields
    double *sJ = reinterpret_cast<double *>(smem_raw + ((6 * rfvol * sizeof(T) + 15) & ~size_t(15)));
    // then the queue of cell-crossing particles: offsets, indices, count
    CrossQueue<T> cq;
    cq.cap = tg.qcap;
    cq.f0 = reinterpret_cast<T *>(sJ + 3 * rjvol);
    cq.f1 = cq.f0 + 3 * cq.cap;
    cq.j = reinterpret_cast<int *>(cq.f1 + 3 * cq.cap);
    cq.pk = cq.j + cq.cap;
    cq.cnt = cq.pk + cq.cap;
    const TileSpan ts = tile_span(tg, tile_start, in.n);
    // guests of this tile (G: the kernel also builds the next step's lists)
    const int ng = (G && g.cnt) ? (g.cnt[ts.t] < g.cap ? g.cnt[ts.t] : g.cap) : 0;
    if (ts.pe <= ts.ps && ng == 0)
        return;   // uniform across the workgroup

    const int tid = threadIdx.x, nth = blockDim.x;
    region_walk(pc.n, ts.t0, tg.lo_f, rfx, rfy, tg.rf[2], rfx, region_wraps_once(pc.n, tg.t, tg.lo_f, tg.rf),
                [&](int r, int gi) {
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        sF[m * rfvol + r] = fp.E[m][gi];
                        sF[(3 + m) * rfvol + r] = fp.B[m][gi];
                    }
                });
    for (int r = tid; r < 3 * rjvol; r += nth)
        sJ[r] = 0.0;
    if (tid == 0)
        *cq.cnt = 0;
    __syncthreads();

    FieldSrc<T> lf;
#pragma unroll
    for (int m = 0; m < 6; ++m)
        lf.c[m] = sF + m * rfvol;
    const int sf[3] = {1, rfx, rfx * rfy};
    const int sj[3] = {1, jpx, jpx * rjy};
    const int np = (int)(ts.pe - ts.ps);
    // coalesced: the tile's particles are stored rank-major (one particle
    // per cell, cell after cell, then the next rank), so consecutive lanes
    // read consecutive memory and sit in distinct neighbouring cells.  After
    // them come the tile's guests (particles binned elsewhere whose cell lies
    // in this tile), through the same path.
    for (int j0 = 0; j0 < np + ng; j0 += nth) {
        const int j = j0 + tid;
        int key = 0;   // non-zero: a particle that stays in its cell, deposited below
        int l[3] = {0, 0, 0};
        T f[3] = {T(0), T(0), T(0)}, f1[3] = {T(0), T(0), T(0)}, w = T(0);
        bool is_stray = false;
        int pst = 0;
        if (j < np + ng) {
            const bool own = j < np;
            int64_t p = ts.ps + j;
            int home = ts.t;
            if (!own) {
                const int2 e = g.list[(int64_t)ts.t * g.cap + (j - np)];
                p = e.x;
                home = e.y;
            }
            int c[3];
            T u[3];
            unsigned char st = 0, gn = 0;   // stray mark; guest status next step
            bool moved = true;             // this launch writes the particle's next status
            // The state is read together with the guest flag (one memory
            // round trip, not two).  A particle listed as a guest of another
            // tile this step is moved by that tile, possibly while this one
            // runs (the step is in place): what was read of it is dropped.
            load_state(in, p, c, f, u);
            const bool flagged = G && own && g.flag && g.flag[p];
            if (flagged) {
                moved = false;
            } else if (!check_state(pc.n, c, f, u, err)) {
                copy_particle(in, out, p);
            } else if (!tile_local(tg, pc.n, ts.t0, c, l)) {
                if (own) {
                    // outside the region and not listed as a guest: the stray
                    // kernel's (which writes its status)
                    moved = false;
                    st = 1;
                } else {
                    atomicOr(err, 2);   // cannot happen: the list was built from this cell in this call
                    copy_particle(in, out, p);
                }
            } else {
                int kap[3];
                if (particle_advance<T, O, true>(pc, in, out, lf, p, c, f, u, l, tg.lo_f, sf, f1, kap, w, err)) {
                    if ((kap[0] | kap[1] | kap[2]) == 0)
                        key = xrun_key(l);
                    else if (!cq.push((int)(p - ts.ps), l, kap, f, f1))
                        deposit_local_full<T, O>(pc, f, f1, kap, l, tg.lo_j, sj, w, sJ, rjvol);
                    // a particle that changed cells, or a guest (outside its home
                    // region), gets its status for the next step
                    if (G && ((kap[0] | kap[1] | kap[2]) || !own)) {
                        int c1[3], ht0[3] = {ts.t0[0], ts.t0[1], ts.t0[2]};
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            c1[d] = wrap_once(c[d] + kap[d], pc.n[d]);
                        if (!own)
                            tile_origin(tg, home, ht0);
                        gn = guest_next(g, tg, pc.n, p, home, ht0, c1);
                    }
                }
            }
            is_stray = own && st;
            pst = (int)p;
            if (G && moved)
                g.flag_next[p] = gn;
        }
        // the wave is converged here: list the strays, find the runs, then deposit
        stray_append(is_stray, pst, strays);
        const XRun xr = xrun(key);
        if (key != 0)
            deposit_still_shared<T, O>(pc, f, f1, l, tg.lo_j, sj, w, sJ, rjvol, xr);
    }
    __syncthreads();
    // deposit the queued cell-crossing particles in full waves, one lane per
    // particle and current component (component-major, so that a wave
    // mostly takes one component)
    const int nq = *cq.cnt < cq.cap ? *cq.cnt : cq.cap;
    for (int i = tid; i < 3 * nq; i += nth) {
        const int m = i / nq, k = i - m * nq;
        const int64_t p = ts.ps + cq.j[k];
        int l[3], kap[3];
        CrossQueue<T>::unpack(cq.pk[k], l, kap);
        T f0[3], f1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f0[d] = cq.f0[d * cq.cap + k];
            f1[d] = cq.f1[d * cq.cap + k];
        }
        const T w = in.w ? in.w[p] : pc.w0;
        if (m == 0)
            deposit_local_full<T, O, 0>(pc, f0, f1, kap, l, tg.lo_j, sj, w, sJ, rjvol);
        else if (m == 1)
            deposit_local_full<T, O, 1>(pc, f0, f1, kap, l, tg.lo_j, sj, w, sJ, rjvol);
        else
            deposit_local_full<T, O, 2>(pc, f0, f1, kap, l, tg.lo_j, sj, w, sJ, rjvol);
    }
    __syncthreads();
    region_walk(pc.n, ts.t0, tg.lo_j, rjx, rjy, tg.rj[2], jpx, region_wraps_once(pc.n, tg.t, tg.lo_j, tg.rj),
                [&](int r, int gi) {
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        const T v = (T)sJ[m * rjvol + r];
                        if (v != T(0))
                            gatomic_add(fp.J[m] + gi, v);
                    }
                });
}

// exclusive prefix sum of in[0..n) into out[0..n) by the whole workgroup;
// sh: LDS scratch of blockDim.x / 64 + 1 ints
__device__ inline void block_exclusive_scan(const int *in, int *out, int n, int *sh)
{
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wv = tid >> 6;
    const int per = (n + nth - 1) / nth, b = tid * per, e = b + per < n ? b + per : n;
    int sum = 0;
    for (int i = b; i < e; ++i)
        sum += in[i];
    int incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += v;
    }
    if (lane == 63)
        sh[wv] = incl;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < nth / 64; ++w) {
            const int v = sh[w];
            sh[w] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int run = sh[wv] + incl - sum;
    for (int i = b; i < e; ++i) {
        const int v = in[i];
        out[i] = run;
        run += v;
    }
}

// ---------------------------------------------------------------------------
// The tile step in two phases, the deposit of the particles that stay in
// their cells accumulated per cell.
//
// Phase A, one thread per particle (rank-major, coalesced): gather from the
// LDS field tile, push, move; a particle that changed cells goes to the LDS
// crossing queue (its full-window current is added per component in phase
// B; when the queue is full, at once to global memory), one that stayed is
// listed under its cell (an LDS counting sort: count per cell, scan, list)
// and when the step runs in place its old offsets are kept in scratch
// (`f0s`; else they stay in `in`) for phase B, which reads them with the
// new ones from `out`.
//
// Phase B, per current component: one thread per cell of the tile (two or
// more per cell when the workgroup has more threads than the tile has
// cells, each taking every second, ... particle of the list) sums its
// particles' narrow-window Esirkepov values in registers and adds the sum
// to the component's FP64 LDS accumulator once, with rows shared along the
// tile's rows of cells; still particles in the slack cells and the queued
// crossers follow one lane each; the component is flushed to global memory
// (one atomic per non-zero value) before the next one reuses the
// accumulator.  The per-particle values are those of the one-pass kernel
// (formed in the working precision, summed in FP64 in the LDS); only the
// order of the sums changes.  Particles are taken in chunks of `kc` (the
// list capacity); each chunk runs both phases.

template <typename T>
struct Off3 {
    T *o[3];
};

// LDS layout of k_particles_cells (byte offsets), shared by the launcher
struct CellsLds {
    size_t f, a, cnt, start, sh, keys, list, qf0, qf1, qj, qpk, qcnt, total;
};

__host__ __device__ inline CellsLds cells_lds(const TileGeo &tg, int nth, int kc, int tsize)
{
    auto al16 = [](size_t x) { return (x + 15) & ~size_t(15); };
    const size_t rf = (size_t)tg.rf[0] * tg.rf[1] * tg.rf[2];
    const size_t rj = (size_t)tg.jp * tg.rj[1] * tg.rj[2];
    const size_t tc = (size_t)tg.t[0] * tg.t[1] * tg.t[2];
    CellsLds L;
    size_t o = 0;
    L.f = o;
    o = al16(o + 6 * rf * tsize);
    L.a = o;
    o = al16(o + rj * sizeof(double));
    L.qf0 = o;
    o = al16(o + 3 * (size_t)tg.qcap * tsize);
    L.qf1 = o;
    o = al16(o + 3 * (size_t)tg.qcap * tsize);
    L.cnt = o;
    o += 4 * (tc + 1);
    L.start = o;
    o += 4 * (tc + 1);
    L.sh = o;
    o += 4 * ((size_t)nth / 64 + 4);
    L.keys = o;
    o += 4 * (size_t)kc;
    L.list = o;
    o += 4 * (size_t)kc;
    L.qj = o;
    o += 4 * (size_t)tg.qcap;
    L.qpk = o;
    o += 4 * (size_t)tg.qcap;
    L.qcnt = o;
    o += 16;
    L.total = o;
    return L;
}

// particle index of entry j of a tile's chunk list: own particles first,
// then the tile's guests
__device__ __attribute__((always_inline)) inline int64_t tile_particle(const TileSpan &ts, const GuestArgs &g, int np,
                                                                       int j)
{
    return j < np ? ts.ps + j : (int64_t)g.list[(int64_t)ts.t * g.cap + (j - np)].x;
}

// Narrow-window Esirkepov values of component M of a particle that stays in
// its cell, as rows along x: v(kz, ky, ix) for ix < NX, ky < RY, kz < RZ,
// passed to add(kz, ky, ix, value) (esk_scatter_still's values, regrouped).
template <typename T, int O, int M>
struct StillRows {
    static constexpr int NW = Shape<O, T>::NW;
    static constexpr int NX = M == 0 ? NW - 1 : NW;
    static constexpr int RY = M == 1 ? NW - 1 : NW;
    static constexpr int RZ = M == 2 ? NW - 1 : NW;
    template <typename AddFn>
    __device__ __attribute__((always_inline)) static inline void apply(const PConst<T> &pc, const T *f0, const T *f1,
                                                                       T w, AddFn &&add)
    {
        const T half = T(0.5), third = T(1) / T(3);
        T S0[3][NW], DS[3][NW];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            esk_axis_still<O>(f0[d], f1[d], S0[d], DS[d]);
        T P[NW - 1];
        {
            const T K = pc.jk[M] * w;
            T run = T(0);
#pragma unroll
            for (int a = 0; a < NW - 1; ++a) {
                run += DS[M][a];
                P[a] = K * run;
            }
        }
        // C for (p, q) at (b, c): S0p (S0q + DSq/2) + DSp (S0q/2 + DSq/3)
        auto cw = [&](int pp, int qq, int b, int c) -> T {
            return S0[pp][b] * (S0[qq][c] + half * DS[qq][c]) + DS[pp][b] * (half * S0[qq][c] + third * DS[qq][c]);
        };
        if constexpr (M == 0) {
#pragma unroll
            for (int c = 0; c < NW; ++c)
#pragma unroll
                for (int b = 0; b < NW; ++b) {
                    const T C = cw(1, 2, b, c);
#pragma unroll
                    for (int a = 0; a < NW - 1; ++a)
                        add(c, b, a, P[a] * C);
                }
        } else if constexpr (M == 1) {
#pragma unroll
            for (int b = 0; b < NW; ++b)
#pragma unroll
                for (int a = 0; a < NW - 1; ++a)
#pragma unroll
                    for (int c = 0; c < NW; ++c)
                        add(b, a, c, P[a] * cw(2, 0, b, c));
        } else {
#pragma unroll
            for (int a = 0; a < NW - 1; ++a)
#pragma unroll
                for (int c = 0; c < NW; ++c)
#pragma unroll
                    for (int b = 0; b < NW; ++b)
                        add(a, c, b, P[a] * cw(0, 1, b, c));
        }
    }
};

// Esirkepov full-window current of component M into the component's LDS
// accumulator
template <typename T, int O, int M>
__device__ __attribute__((always_inline)) inline void deposit_local_comp(const PConst<T> &pc, const T *f0, const T *f1,
                                                                         const int *kap, const int *l, int lo_j,
                                                                         const int *sj, T w, double *sA)
{
    constexpr int NW = Shape<O, T>::NW;
    EskAxis<O, T> e[3];
    T K[3];
    int jo[3][NW + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        esk_axis<O>(f0[d], f1[d], kap[d], e[d]);
        K[d] = pc.jk[d] * w;
        axis_offsets_local<NW + 1>(l[d] + lo_j, e[d].lo, sj[d], jo[d]);
    }
    esk_scatter<O, T, double, M>(e, jo, K, [&](int, int idx, double v) { latomic_add(sA + idx, v); });
}

// Esirkepov full-window current straight into global memory (a crosser
// that found the queue full)
template <typename T, int O>
__device__ __attribute__((always_inline)) inline void deposit_global_full(const PConst<T> &pc, const FieldPtrs<T> &fp,
                                                                          const int *c, const T *f0, const T *f1,
                                                                          const int *kap, T w)
{
    constexpr int NW = Shape<O, T>::NW;
    const int gs[3] = {1, pc.n[0], pc.n[0] * pc.n[1]};
    EskAxis<O, T> e[3];
    T K[3];
    int jo[3][NW + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        esk_axis<O>(f0[d], f1[d], kap[d], e[d]);
        K[d] = pc.jk[d] * w;
        axis_offsets_global<NW + 1>(c[d], e[d].lo, pc.n[d], gs[d], jo[d]);
    }
    esk_scatter<O, T, T>(e, jo, K, [&](int m, int idx, T v) { gatomic_add(fp.J[m] + idx, v); });
}

// Phase B for component M: the per-cell sums of the listed still particles,
// the still particles of the slack cells, the queued crossers; `last`
template <typename T, int O, int M>
__device__ __attribute__((always_inline)) inline void cells_component(
    const PConst<T> &pc, const TileGeo &tg, const TileSpan &ts, const GuestArgs &g, int np, const PArr<T> &in,
    const PArr<T> &out, const Off3<T> &f0s, const int *list, const int *cstart, const int *ccnt, int tc,
    const CrossQueue<T> &cq, int nq, double *sA, const int *sj, int groups)
{
    using R = StillRows<T, O, M>;
    constexpr int NB = Shape<O, T>::NB;
    const int nth = blockDim.x, tid = threadIdx.x;
    for (int lc0 = 0; lc0 < tc; lc0 += nth) {
        const int part = tc < nth ? tid / tc : 0;
        const int lc = lc0 + (tc < nth ? tid % tc : tid);
        const bool cell = part < groups && lc < tc;   // groups * tc <= nth
        int l[3] = {0, 0, 0}, s = 0, k = 0;
        if (cell) {
            l[0] = lc % tg.t[0];
            l[1] = (lc / tg.t[0]) % tg.t[1];
            l[2] = lc / (tg.t[0] * tg.t[1]);
            s = cstart[lc];
            k = ccnt[lc];
        }
        T acc[R::RZ][R::RY][R::NX];
#pragma unroll
        for (int c = 0; c < R::RZ; ++c)
#pragma unroll
            for (int b = 0; b < R::RY; ++b)
#pragma unroll
                for (int a = 0; a < R::NX; ++a)
                    acc[c][b][a] = T(0);
        // the next particle's loads are issued before this one's arithmetic
        int64_t pn = 0;
        T f0n[3] = {T(0), T(0), T(0)}, f1n[3] = {T(0), T(0), T(0)}, wn = pc.w0;
        if (part < k) {
            pn = tile_particle(ts, g, np, list[s + part]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                f0n[d] = f0s.o[d][pn];
                f1n[d] = out.off[d][pn];
            }
            if (in.w)
                wn = in.w[pn];
        }
        for (int i = part; i < k; i += groups) {
            const int64_t p = pn;
            const T f0[3] = {f0n[0], f0n[1], f0n[2]}, f1[3] = {f1n[0], f1n[1], f1n[2]}, w = wn;
            if (i + groups < k) {
                pn = tile_particle(ts, g, np, list[s + i + groups]);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    f0n[d] = f0s.o[d][pn];
                    f1n[d] = out.off[d][pn];
                }
                if (in.w)
                    wn = in.w[pn];
            }
            R::apply(pc, f0, f1, w, [&](int c, int b, int a, T v) { acc[c][b][a] += v; });
        }
        // the wave is converged here: runs of consecutive cells along x
        const XRun xr = xrun(cell ? xrun_key(l) : 0);
        if (__ballot(k > part) != 0 && cell) {
            const int x0 = l[0] + tg.lo_j + NB, y0 = l[1] + tg.lo_j + NB, z0 = l[2] + tg.lo_j + NB;
#pragma unroll
            for (int c = 0; c < R::RZ; ++c)
#pragma unroll
                for (int b = 0; b < R::RY; ++b)
                    xrow_add<R::NX>(sA + x0 + sj[1] * (y0 + b) + sj[2] * (z0 + c), acc[c][b], xr);
        }
    }
    // still particles of the slack cells, one lane each
    const int no = ccnt[tc], so = cstart[tc];
    for (int i = tid; i < no; i += nth) {
        const int64_t p = tile_particle(ts, g, np, list[so + i]);
        int c[3], l[3];
        T f0[3], f1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            c[d] = in.cell[d][p];
            f0[d] = f0s.o[d][p];
            f1[d] = out.off[d][p];
        }
        tile_local(tg, pc.n, ts.t0, c, l);
        const T w = in.w ? in.w[p] : pc.w0;
        const int x0 = l[0] + tg.lo_j + NB, y0 = l[1] + tg.lo_j + NB, z0 = l[2] + tg.lo_j + NB;
        R::apply(pc, f0, f1, w, [&](int cc, int b, int a, T v) {
            latomic_add(sA + x0 + a + sj[1] * (y0 + b) + sj[2] * (z0 + cc), (double)v);
        });
    }
    // the queued crossers of this chunk, one lane each
    for (int k = tid; k < nq; k += nth) {
        const int64_t p = ts.ps + cq.j[k];
        int l[3], kap[3];
        CrossQueue<T>::unpack(cq.pk[k], l, kap);
        T f0[3], f1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f0[d] = cq.f0[d * cq.cap + k];
            f1[d] = cq.f1[d * cq.cap + k];
        }
        const T w = in.w ? in.w[p] : pc.w0;
        deposit_local_comp<T, O, M>(pc, f0, f1, kap, l, tg.lo_j, sj, w, sA);
    }
}

template <typename T, int O, bool G>
__global__ void __launch_bounds__(TileThreads<T>::value) k_particles_cells(PConst<T> pc, TileGeo tg, PArr<T> in,
                                                                           PArr<T> out, FieldPtrs<T> fp,
                                                                           const int *__restrict__ tile_start,
                                                                           StrayList strays, GuestArgs g,
                                                                           Off3<T> f0s, int kc, int *err)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, nth = blockDim.x;
    const CellsLds Ld = cells_lds(tg, nth, kc, (int)sizeof(T));
    T *sF = reinterpret_cast<T *>(smem_raw + Ld.f);
    double *sA = reinterpret_cast<double *>(smem_raw + Ld.a);
    int *ccnt = reinterpret_cast<int *>(smem_raw + Ld.cnt);
    int *cstart = reinterpret_cast<int *>(smem_raw + Ld.start);
    int *sh = reinterpret_cast<int *>(smem_raw + Ld.sh);
    int *keys = reinterpret_cast<int *>(smem_raw + Ld.keys);
    int *list = reinterpret_cast<int *>(smem_raw + Ld.list);
    CrossQueue<T> cq;
    cq.cap = tg.qcap;
    cq.f0 = reinterpret_cast<T *>(smem_raw + Ld.qf0);
    cq.f1 = reinterpret_cast<T *>(smem_raw + Ld.qf1);
    cq.j = reinterpret_cast<int *>(smem_raw + Ld.qj);
    cq.pk = reinterpret_cast<int *>(smem_raw + Ld.qpk);
    cq.cnt = reinterpret_cast<int *>(smem_raw + Ld.qcnt);
    const int rfx = tg.rf[0], rfy = tg.rf[1];
    const int rfvol = rfx * rfy * tg.rf[2];
    const int rjx = tg.rj[0], rjy = tg.rj[1], jpx = tg.jp;
    const int rjvol = jpx * rjy * tg.rj[2];
    const int tc = tg.t[0] * tg.t[1] * tg.t[2];
    const TileSpan ts = tile_span(tg, tile_start, in.n);
    const int ng = (G && g.cnt) ? (g.cnt[ts.t] < g.cap ? g.cnt[ts.t] : g.cap) : 0;
    if (ts.pe <= ts.ps && ng == 0)
        return;   // uniform across the workgroup
    region_walk(pc.n, ts.t0, tg.lo_f, rfx, rfy, tg.rf[2], rfx, region_wraps_once(pc.n, tg.t, tg.lo_f, tg.rf),
                [&](int r, int gi) {
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        sF[m * rfvol + r] = fp.E[m][gi];
                        sF[(3 + m) * rfvol + r] = fp.B[m][gi];
                    }
                });
    for (int r = tid; r < rjvol; r += nth)
        sA[r] = 0.0;
    FieldSrc<T> lf;
#pragma unroll
    for (int m = 0; m < 6; ++m)
        lf.c[m] = sF + m * rfvol;
    const int sf[3] = {1, rfx, rfx * rfy};
    const int sj[3] = {1, jpx, jpx * rjy};
    const int np = (int)(ts.pe - ts.ps);
    for (int jb = 0; jb < np + ng; jb += kc) {
        const int je = np + ng < jb + kc ? np + ng : jb + kc;
        for (int i = tid; i <= tc; i += nth)
            ccnt[i] = 0;
        if (tid == 0)
            *cq.cnt = 0;
        __syncthreads();   // also: the field tile is staged
        // phase A
        for (int j0 = jb; j0 < je; j0 += nth) {
          const int j = j0 + tid;
          bool is_stray = false;
          int pst = 0;
          if (j < je) {
            int key = -1;
            const bool own = j < np;
            int64_t p = ts.ps + j;
            int home = ts.t;
            if (!own) {
                const int2 e = g.list[(int64_t)ts.t * g.cap + (j - np)];
                p = e.x;
                home = e.y;
            }
            int c[3], l[3];
            T f[3], u[3], f1[3], w = T(0);
            unsigned char st = 0, gn = 0;
            bool moved = true;
            // the state is read together with the guest flag; a guest of
            // another tile this step is moved by that tile (what was read of
            // it is dropped)
            load_state(in, p, c, f, u);
            const bool flagged = G && own && g.flag && g.flag[p];
            if (flagged) {
                moved = false;
            } else if (!check_state(pc.n, c, f, u, err)) {
                copy_particle(in, out, p);
            } else if (!tile_local(tg, pc.n, ts.t0, c, l)) {
                if (own) {
                    moved = false;
                    st = 1;
                } else {
                    atomicOr(err, 2);
                    copy_particle(in, out, p);
                }
            } else {
                int kap[3];
                if (particle_advance<T, O, true, false>(pc, in, out, lf, p, c, f, u, l, tg.lo_f, sf, f1, kap, w, err)) {
                    if ((kap[0] | kap[1] | kap[2]) == 0) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            out.off[d][p] = f1[d];
                            if (f0s.o[d] != in.off[d])
                                f0s.o[d][p] = f[d];
                        }
                        const bool in_tile = l[0] >= 0 && l[0] < tg.t[0] && l[1] >= 0 && l[1] < tg.t[1] &&
                                             l[2] >= 0 && l[2] < tg.t[2];
                        const int slot = in_tile ? l[0] + tg.t[0] * (l[1] + tg.t[1] * l[2]) : tc;
                        key = (slot << 16) | atomicAdd(ccnt + slot, 1);
                    } else {
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            out.off[d][p] = f1[d];
                        if (!cq.push((int)(p - ts.ps), l, kap, f, f1))
                            deposit_global_full<T, O>(pc, fp, c, f, f1, kap, w);
                    }
                    if (G && ((kap[0] | kap[1] | kap[2]) || !own)) {
                        int c1[3], ht0[3] = {ts.t0[0], ts.t0[1], ts.t0[2]};
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            c1[d] = wrap_once(c[d] + kap[d], pc.n[d]);
                        if (!own)
                            tile_origin(tg, home, ht0);
                        gn = guest_next(g, tg, pc.n, p, home, ht0, c1);
                    }
                }
            }
            is_stray = own && st;
            pst = (int)p;
            if (G && moved)
                g.flag_next[p] = gn;
            keys[j - jb] = key;
          }
          // the wave is converged here
          stray_append(is_stray, pst, strays);
        }
        __syncthreads();
        block_exclusive_scan(ccnt, cstart, tc + 1, sh);
        __syncthreads();
        for (int j = jb + tid; j < je; j += nth) {
            const int key = keys[j - jb];
            if (key >= 0)
                list[cstart[key >> 16] + (key & 0xffff)] = j;
        }
        __syncthreads();
        // phase B
        const int nq = *cq.cnt < cq.cap ? *cq.cnt : cq.cap;
        // threads per cell: each adds its sum with a row update per cell, so
        // a second thread per cell pays only from about 6 particles per cell
        // on (the chunk's count over 4 per cell, rounded)
        int groups = 1;
        if (tc < nth) {
            const int dense = (je - jb + 2 * tc) / (4 * tc);
            groups = nth / tc < dense ? nth / tc : (dense > 1 ? dense : 1);
        }
        const bool jonce = region_wraps_once(pc.n, tg.t, tg.lo_j, tg.rj);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            if (m == 0)
                cells_component<T, O, 0>(pc, tg, ts, g, np, in, out, f0s, list, cstart, ccnt, tc, cq, nq, sA, sj,
                                         groups);
            else if (m == 1)
                cells_component<T, O, 1>(pc, tg, ts, g, np, in, out, f0s, list, cstart, ccnt, tc, cq, nq, sA, sj,
                                         groups);
            else
                cells_component<T, O, 2>(pc, tg, ts, g, np, in, out, f0s, list, cstart, ccnt, tc, cq, nq, sA, sj,
                                         groups);
            __syncthreads();
            region_walk(pc.n, ts.t0, tg.lo_j, rjx, rjy, tg.rj[2], jpx, jonce, [&](int r, int gi) {
                const T v = (T)sA[r];
                sA[r] = 0.0;
                if (v != T(0))
                    gatomic_add(fp.J[m] + gi, v);
            });
            __syncthreads();
        }
    }
}

// the fused step for the listed strays, on global memory
template <typename T, int O>
__global__ void __launch_bounds__(STRAY_THREADS) k_particles_strays(PConst<T> pc, PArr<T> in, PArr<T> out,
                                                                    FieldPtrs<T> fp, StrayList strays, GuestArgs g,
                                                                    int *err)
{
    const int k = *strays.cnt < strays.cap ? *strays.cnt : strays.cap;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const int64_t p = strays.p[i];
        int c[3];
        T f[3], u[3];
        if (!load_particle(in, p, pc.n, c, f, u, err))
            copy_particle(in, out, p);
        else
            particle_step_global<T, O>(pc, in, out, fp, p, c, f, u, err);
        if (g.flag_next)
            g.flag_next[p] = 0;   // next step: the home tile's again, or a stray
    }
}

template <typename T, int O>
__global__ void __launch_bounds__(256) k_particles_global(PConst<T> pc, PArr<T> sp, FieldPtrs<T> fp, int *err)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.n)
        return;
    int c[3];
    T f[3], u[3];
    if (!load_particle(sp, p, pc.n, c, f, u, err))
        return;
    particle_step_global<T, O>(pc, sp, sp, fp, p, c, f, u, err);
}

template <typename T, int O>
__global__ void __launch_bounds__(256) k_gather(PConst<T> pc, PArr<T> sp, FieldPtrs<T> fp, T *Ex, T *Ey, T *Ez,
                                                T *Bx, T *By, T *Bz, int *err)
{
    constexpr int NW = Shape<O, T>::NW;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.n)
        return;
    int c[3];
    T f[3];
    T E[3] = {T(0), T(0), T(0)}, B[3] = {T(0), T(0), T(0)};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = sp.cell[d][p];
        f[d] = sp.off[d][p];
        ok = ok && c[d] >= 0 && c[d] < pc.n[d] && f[d] >= T(0) && f[d] < T(1);
    }
    if (!ok)
        atomicOr(err, 1);
    if (ok) {
        const int gs[3] = {1, pc.n[0], pc.n[0] * pc.n[1]};
        AxisW<O, T> aw[3];
        int on[3][NW], os[3][NW];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            axis_weights<O>(f[d], aw[d]);
            axis_offsets_global<NW>(c[d], aw[d].bn, pc.n[d], gs[d], on[d]);
            axis_offsets_global<NW>(c[d], aw[d].bs, pc.n[d], gs[d], os[d]);
        }
        FieldSrc<T> gf;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            gf.c[m] = fp.E[m];
            gf.c[3 + m] = fp.B[m];
        }
        gather_eb<O>(gf, aw, on, os, E, B);
    }
    Ex[p] = E[0];
    Ey[p] = E[1];
    Ez[p] = E[2];
    Bx[p] = B[0];
    By[p] = B[1];
    Bz[p] = B[2];
}

template <typename T>
__global__ void __launch_bounds__(256) k_push(PConst<T> pc, PArr<T> sp, const T *Ex, const T *Ey, const T *Ez,
                                              const T *Bx, const T *By, const T *Bz, int *err)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.n)
        return;
    int c[3];
    T f[3], u[3];
    if (!load_particle(sp, p, pc.n, c, f, u, err))
        return;
    const T E[3] = {Ex[p], Ey[p], Ez[p]}, B[3] = {Bx[p], By[p], Bz[p]};
    T u1[3];
    push_momentum(pc, u, E, B, u1);
    const T ig = T(1) / sqrt(T(1) + (u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]) * pc.inv_c2);
    T f1[3];
    int kap[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T disp = pc.dtd[d] * u1[d] * ig;
        ok = ok && fabs(disp) < T(1);
        move_axis(f[d], disp, f1[d], kap[d]);
    }
    if (!ok) {
        atomicOr(err, 2);
        return;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sp.cell[d][p] = wrap_once(c[d] + kap[d], pc.n[d]);
        sp.off[d][p] = f1[d];
        sp.u[d][p] = u1[d];
    }
}

template <typename T, int O>
__global__ void __launch_bounds__(256) k_deposit(PConst<T> pc, PArr<T> b, PArr<T> a, FieldPtrs<T> fp, int *err)
{
    constexpr int NW = Shape<O, T>::NW;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= b.n)
        return;
    int c0[3], c1[3], kap[3];
    T f0[3], f1[3], u[3];
    if (!load_particle(b, p, pc.n, c0, f0, u, err))
        return;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c1[d] = a.cell[d][p];
        f1[d] = a.off[d][p];
        int k = c1[d] - c0[d];
        if (k > pc.n[d] / 2)
            k -= pc.n[d];
        if (k < -(pc.n[d] / 2))
            k += pc.n[d];
        kap[d] = k;
        ok = ok && k >= -1 && k <= 1 && c1[d] >= 0 && c1[d] < pc.n[d] && f1[d] >= T(0) && f1[d] < T(1);
    }
    if (!ok) {
        atomicOr(err, 4);
        return;
    }
    const T w = b.w ? b.w[p] : pc.w0;
    const int gs[3] = {1, pc.n[0], pc.n[0] * pc.n[1]};
    EskAxis<O, T> e[3];
    T K[3];
    int jo[3][NW + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        esk_axis<O>(f0[d], f1[d], kap[d], e[d]);
        K[d] = pc.jk[d] * w;
        axis_offsets_global<NW + 1>(c0[d], e[d].lo, pc.n[d], gs[d], jo[d]);
    }
    esk_scatter<O, T, T>(e, jo, K, [&](int m, int idx, T v) { gatomic_add(fp.J[m] + idx, v); });
}

// ---------------------------------------------------------------------------
// Transpose of the particle part of one step, in two passes so that neither
// keeps the whole reverse chain live in registers.
//  pass 1 (push): the forward quantities are recomputed from the state at
//     step n with the forward device functions (gather, Boris, move), so the
//     reverse sweep follows the forward rounding; then the deposit transpose
//     (a gather of the current adjoint lj * hatE over the Esirkepov window)
//     and the position and Boris transposes.  Writes lu <- dL/du^n,
//     lx <- dL/dx^n without the gather term, and the adjoints of the
//     gathered fields (Eb, Bb) per particle.
//  pass 2 (scatter): the gather transpose of a group of three field
//     components (E or B): scatters S * vb into the component's adjoint and
//     adds vb * grad(S) . F to lx.
// With LOCAL the particle lies inside the tile's LDS regions: fields and
// hatE come from LDS and the scatter accumulates into FP64 LDS tiles;
// otherwise everything is global.
template <typename T>
struct AdjPtrs {
    const T *hat[3];   // hatE: lE - dt/2 curl_b(lB), the current adjoint is lj * hatE
    T *lx[3], *lu[3], *lE[3], *lB[3];
    T *vb[6];          // per-particle adjoints of the gathered E and B
};

// Gather transpose of one field component with staggering (SX, SY, SZ), in
// two parts.  gather_grad adds vb * grad(gathered value) to the position
// adjoint (it reads the field window); scatter_component scatters S * vb
// into the component's adjoint (FP64 LDS accumulators, rows along x shared
// between lanes as in the forward deposit, or global atomics).
template <int O, typename T, int SX, int SY, int SZ>
__device__ __attribute__((always_inline)) inline void gather_grad(const T *F, T vb, const AxisW<O, T> *aw,
                                   const T (*dn)[Shape<O, T>::NW], const T (*ds)[Shape<O, T>::NW],
                                   const int (*on)[Shape<O, T>::NW], const int (*os)[Shape<O, T>::NW], T *lxa)
{
    constexpr int NW = Shape<O, T>::NW;
    const T *wx = SX ? aw[0].ws : aw[0].wn;
    const T *wy = SY ? aw[1].ws : aw[1].wn;
    const T *wz = SZ ? aw[2].ws : aw[2].wn;
    const T *dx = SX ? ds[0] : dn[0];
    const T *dy = SY ? ds[1] : dn[1];
    const T *dz = SZ ? ds[2] : dn[2];
    const int *xo = SX ? os[0] : on[0];
    const int *yo = SY ? os[1] : on[1];
    const int *zo = SZ ? os[2] : on[2];
    T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
    for (int k = 0; k < NW; ++k)
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const int rowo = yo[j] + zo[k];
            T ax = T(0), adx = T(0);
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const T val = F[rowo + xo[i]];
                ax += wx[i] * val;
                adx += dx[i] * val;
            }
            gx += adx * wy[j] * wz[k];
            gy += ax * dy[j] * wz[k];
            gz += ax * wy[j] * dz[k];
            // finish the row here (the compiler would otherwise issue every
            // row's loads first and park them in scratch memory)
            asm volatile("" : "+v"(gx), "+v"(gy), "+v"(gz));
            __builtin_amdgcn_sched_barrier(0);
        }
    lxa[0] += vb * gx;
    lxa[1] += vb * gy;
    lxa[2] += vb * gz;
}

// The gathered value of one component and its gradient in the particle's
// offsets (in cells) in one sweep over the window: the pass-1 kernel that
// keeps the gradients in LDS reads each field value once, for the forward
// recomputation and for the position part of the gather transpose.
template <int O, typename T, int SX, int SY, int SZ>
__device__ __attribute__((always_inline)) inline T gather_value_grad(const T *F, const AxisW<O, T> *aw,
                                      const T (*dn)[Shape<O, T>::NW], const T (*ds)[Shape<O, T>::NW],
                                      const int (*on)[Shape<O, T>::NW], const int (*os)[Shape<O, T>::NW], T *g)
{
    constexpr int NW = Shape<O, T>::NW;
    const T *wx = SX ? aw[0].ws : aw[0].wn;
    const T *wy = SY ? aw[1].ws : aw[1].wn;
    const T *wz = SZ ? aw[2].ws : aw[2].wn;
    const T *dx = SX ? ds[0] : dn[0];
    const T *dy = SY ? ds[1] : dn[1];
    const T *dz = SZ ? ds[2] : dn[2];
    const int *xo = SX ? os[0] : on[0];
    const int *yo = SY ? os[1] : on[1];
    const int *zo = SZ ? os[2] : on[2];
    T v = T(0), gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
    for (int k = 0; k < NW; ++k)
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const int rowo = yo[j] + zo[k];
            T ax = T(0), adx = T(0);
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const T val = F[rowo + xo[i]];
                ax += wx[i] * val;
                adx += dx[i] * val;
            }
            const T ayz = ax * wz[k];
            v += ayz * wy[j];
            gx += adx * wy[j] * wz[k];
            gy += ayz * dy[j];
            gz += ax * wy[j] * dz[k];
            asm volatile("" : "+v"(v), "+v"(gx), "+v"(gy), "+v"(gz));
            __builtin_amdgcn_sched_barrier(0);
        }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
    return v;
}

// How the LDS scatter of a component shares rows between lanes:
//   SM_RUNS   the component's own window (its start on a staggered axis
//             depends on the half of the cell the particle is in), rows
//             shared along lane runs of equal window starts;
//   SM_WIDE   on every staggered axis the NW + 1 nodes that either half of
//             the cell can reach, the one the particle does not reach with
//             a zero weight: the window starts at a fixed node relative to
//             the cell, so all six components share one run structure and
//             lanes in consecutive cells always form runs;
//   SM_ALONE  the component's own window, one lane per particle, no sharing.
enum ScatterMode { SM_RUNS = 0, SM_WIDE = 1, SM_ALONE = 2 };

// weights of one axis on the window the scatter mode takes
template <int O, typename T, int S, int SM>
__device__ __attribute__((always_inline)) inline void scatter_axis(const AxisW<O, T> &a,
                                                                   T (&w)[Shape<O, T>::NW + (SM == SM_WIDE && S ? 1 : 0)])
{
    constexpr int NW = Shape<O, T>::NW;
    if constexpr (SM == SM_WIDE && S) {
        // the half-cell window starts at bs = NB (upper half) or NB - 1
        const bool up = a.bs == Shape<O, T>::NB;
        w[0] = up ? T(0) : a.ws[0];
#pragma unroll
        for (int i = 1; i < NW; ++i)
            w[i] = up ? a.ws[i - 1] : a.ws[i];
        w[NW] = up ? a.ws[NW - 1] : T(0);
    } else {
#pragma unroll
        for (int i = 0; i < NW; ++i)
            w[i] = S ? a.ws[i] : a.wn[i];
    }
}

template <int O, typename T, bool LOCAL, int SM, int SX, int SY, int SZ>
__device__ __attribute__((always_inline)) inline void scatter_component(T *Lglob, double *sL, T vb, const AxisW<O, T> *aw,
                                         const int (*on)[Shape<O, T>::NW], const int (*os)[Shape<O, T>::NW],
                                         const int *sf, const XRun &xr)
{
    constexpr int NW = Shape<O, T>::NW;
    if constexpr (LOCAL && SM == SM_WIDE) {
        constexpr int NX = NW + (SX ? 1 : 0), NY = NW + (SY ? 1 : 0), NZ = NW + (SZ ? 1 : 0);
        T wx[NX], wy[NY], wz[NZ];
        scatter_axis<O, T, SX, SM>(aw[0], wx);
        scatter_axis<O, T, SY, SM>(aw[1], wy);
        scatter_axis<O, T, SZ, SM>(aw[2], wz);
        // first node: the nodal window's, one node lower on a staggered axis
        const int x0 = on[0][0] - (SX ? sf[0] : 0);
        const int y0 = on[1][0] - (SY ? sf[1] : 0);
        const int z0 = on[2][0] - (SZ ? sf[2] : 0);
#pragma unroll
        for (int k = 0; k < NZ; ++k)
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const int rowo = y0 + j * sf[1] + z0 + k * sf[2];
                const T wyz = wy[j] * wz[k] * vb;
                T r[NX];
#pragma unroll
                for (int i = 0; i < NX; ++i)
                    r[i] = wx[i] * wyz;
                xrow_add<NX>(sL + rowo + x0, r, xr);   // LDS x offsets are consecutive
            }
    } else {
        const T *wx = SX ? aw[0].ws : aw[0].wn;
        const T *wy = SY ? aw[1].ws : aw[1].wn;
        const T *wz = SZ ? aw[2].ws : aw[2].wn;
        const int *xo = SX ? os[0] : on[0];
        const int *yo = SY ? os[1] : on[1];
        const int *zo = SZ ? os[2] : on[2];
#pragma unroll
        for (int k = 0; k < NW; ++k)
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const int rowo = yo[j] + zo[k];
                const T wyz = wy[j] * wz[k] * vb;
                T r[NW];
#pragma unroll
                for (int i = 0; i < NW; ++i)
                    r[i] = wx[i] * wyz;
                if constexpr (LOCAL && SM == SM_ALONE) {
#pragma unroll
                    for (int i = 0; i < NW; ++i)
                        latomic_add(sL + rowo + xo[i], (double)r[i]);
                } else if constexpr (LOCAL) {
                    xrow_add<NW>(sL + rowo + xo[0], r, xr);   // LDS x offsets are consecutive
                } else {
                    xrow_apply<NW>(r, xr, [&](int i, T v) { gatomic_add(Lglob + rowo + xo[i], v); });
                }
            }
    }
    (void)sf;
}

// lane runs packed in an int: a1 | last << 1 | send << 2 | d << 3 | len << 6
__device__ inline int xrun_pack(const XRun &r)
{
    return (r.a1 ? 1 : 0) | (r.last ? 2 : 0) | (r.send ? 4 : 0) | (r.d << 3) | (r.len << 6);
}

__device__ inline XRun xrun_unpack(int v)
{
    XRun r;
    r.a1 = (v & 1) != 0;
    r.last = (v & 2) != 0;
    r.send = (v & 4) != 0;
    r.d = (v >> 3) & 7;
    r.len = (v >> 6) & 7;
    return r;
}

// a lane on its own: no neighbour, the last of its run
constexpr int XRUN_ALONE = 2 | (1 << 6);

template <typename T, int O, bool LOCAL>
__device__ __attribute__((always_inline)) inline void adjoint_offsets(const PConst<T> &pc, const int *c, const T *f, const int *l, int lo_f,
                                       const int *sf, AxisW<O, T> *aw, int (*on)[Shape<O, T>::NW],
                                       int (*os)[Shape<O, T>::NW])
{
    constexpr int NW = Shape<O, T>::NW;
    const int gs[3] = {1, pc.n[0], pc.n[0] * pc.n[1]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        axis_weights<O>(f[d], aw[d]);
        if (LOCAL) {
            axis_offsets_local<NW>(l[d] + lo_f, aw[d].bn, sf[d], on[d]);
            axis_offsets_local<NW>(l[d] + lo_f, aw[d].bs, sf[d], os[d]);
        } else {
            axis_offsets_global<NW>(c[d], aw[d].bn, pc.n[d], gs[d], on[d]);
            axis_offsets_global<NW>(c[d], aw[d].bs, pc.n[d], gs[d], os[d]);
        }
    }
}

template <typename T>
__device__ inline void clear_vb(const AdjPtrs<T> &ap, int64_t p)
{
#pragma unroll
    for (int m = 0; m < 6; ++m)
        ap.vb[m][p] = T(0);
}

// pass 1 for one particle
//
// SST > 0: st points at this thread's slot of an LDS stash of 18 values with
// stride SST; the forward gather then also evaluates the gradients of the six
// gathered components in the particle's offsets and parks them there, and
// the position part of the gather transpose reads them back (one sweep over
// the field windows instead of two).  SST = 0: the windows are swept twice.
//
// STILL (tile kernels only): a particle that stays in its cell along every
// axis takes the narrow-window deposit transpose (the transpose of the
// forward step's still-particle deposit); one that changes cells is left
// untouched and the call returns false (the caller runs it again without
// STILL).  Otherwise the call returns true.
template <typename T, int O, bool LOCAL, int SST = 0, bool STILL = false>
__device__ __attribute__((always_inline)) inline bool adjoint_push_particle(const PConst<T> &pc, const PArr<T> &sp, const AdjPtrs<T> &ap,
                                             const FieldSrc<T> &fsrc, const T *const *hsrc, int64_t p, const int *c,
                                             const T *f, const T *u, const int *l, int lo_f, const int *sf, int lo_j,
                                             const int *sj, int *err, T *st = nullptr)
{
    static_assert(LOCAL || !STILL, "the narrow path reads tile regions");
    constexpr int NW = Shape<O, T>::NW;
    const int gs[3] = {1, pc.n[0], pc.n[0] * pc.n[1]};
    // forward recomputation: gather, Boris, position
    T E[3], B[3];
    {
        AxisW<O, T> aw[3];
        int on[3][NW], os[3][NW];
        adjoint_offsets<T, O, LOCAL>(pc, c, f, l, lo_f, sf, aw, on, os);
        if constexpr (SST > 0) {
            T dn[3][NW], ds[3][NW];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                axis_dweights<O>(f[d], dn[d], ds[d]);
            T g[3];
            auto park = [&](int m) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    st[(3 * m + k) * SST] = g[k];
            };
            // staggering: E_x(s,n,n) E_y(n,s,n) E_z(n,n,s) B_x(n,s,s) B_y(s,n,s) B_z(s,s,n)
            E[0] = gather_value_grad<O, T, 1, 0, 0>(fsrc.c[0], aw, dn, ds, on, os, g);
            park(0);
            E[1] = gather_value_grad<O, T, 0, 1, 0>(fsrc.c[1], aw, dn, ds, on, os, g);
            park(1);
            E[2] = gather_value_grad<O, T, 0, 0, 1>(fsrc.c[2], aw, dn, ds, on, os, g);
            park(2);
            B[0] = gather_value_grad<O, T, 0, 1, 1>(fsrc.c[3], aw, dn, ds, on, os, g);
            park(3);
            B[1] = gather_value_grad<O, T, 1, 0, 1>(fsrc.c[4], aw, dn, ds, on, os, g);
            park(4);
            B[2] = gather_value_grad<O, T, 1, 1, 0>(fsrc.c[5], aw, dn, ds, on, os, g);
            park(5);
        } else {
            gather_eb<O>(fsrc, aw, on, os, E, B);
        }
    }
    T f1[3];
    int kap[3];
    bool ok = true;
    {
        T u1[3];
        push_momentum(pc, u, E, B, u1);
        const T ig = T(1) / sqrt(T(1) + (u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]) * pc.inv_c2);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T disp = pc.dtd[d] * u1[d] * ig;
            ok = ok && fabs(disp) < T(1);
            move_axis(f[d], disp, f1[d], kap[d]);
        }
    }
    if (!ok) {
        atomicOr(err, 2);
        clear_vb(ap, p);
        return true;
    }
    if constexpr (STILL) {
        if ((kap[0] | kap[1] | kap[2]) != 0)
            return false;
    }
    // deposit transpose: phi = <lJ, J_p>, lJ = (-dt/eps0) hatE
    T g0[3], g1[3];
    const T w = sp.w ? sp.w[p] : pc.w0;
    if constexpr (STILL) {
        T S0[3][NW], DS[3][NW], K[3];
        int jo[3][NW];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            esk_axis_still<O>(f[d], f1[d], S0[d], DS[d]);
            K[d] = pc.jk[d] * w * pc.lj;
            axis_offsets_local<NW>(l[d] + lo_j, Shape<O, T>::NB, sj[d], jo[d]);
        }
        esk_gather_adjoint_still<O>(S0, DS, f, f1, jo, K, [&](int m, int idx) { return hsrc[m][idx]; }, g0, g1);
    } else {
        EskAxis<O, T> e[3];
        T K[3];
        int jo[3][NW + 1];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            esk_axis<O>(f[d], f1[d], kap[d], e[d]);
            K[d] = pc.jk[d] * w * pc.lj;
            if (LOCAL)
                axis_offsets_local<NW + 1>(l[d] + lo_j, e[d].lo, sj[d], jo[d]);
            else
                axis_offsets_global<NW + 1>(c[d], e[d].lo, pc.n[d], gs[d], jo[d]);
        }
        esk_gather_adjoint<O>(e, f, f1, kap, jo, K, [&](int m, int idx) { return hsrc[m][idx]; }, g0, g1);
    }
    // The momentum update again (for Boris, with its tape): only E and B stay
    // live across the deposit transpose.  The register operands keep the
    // compiler from reusing the first evaluation; the inputs and so the values
    // are the same.
    asm volatile("" : "+v"(E[0]), "+v"(E[1]), "+v"(E[2]), "+v"(B[0]), "+v"(B[1]), "+v"(B[2]));
    BorisTape<T> tp;
    T u1[3];
    if (pc.vay)
        vay(pc.h, pc.inv_c2, u, E, B, u1);
    else
        boris(pc.h, pc.inv_c2, u, E, B, u1, tp);
    const T ig = T(1) / sqrt(T(1) + (u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]) * pc.inv_c2);
    T lxb[3], v[3], lxa[3];
    T uv = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lxb[d] = ap.lx[d][p] + g1[d];   // dL/dx^{n+1} incl. the deposit
        v[d] = pc.dtd[d] * lxb[d];
        uv += u1[d] * v[d];
        lxa[d] = g0[d] + lxb[d];   // x^{n+1} = x^n + disp
    }
    // d(u/gamma)/du = I/gamma - u u^T / (gamma^3 c^2)
    T ub[3];
    const T ig3 = ig * ig * ig * pc.inv_c2 * uv;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        ub[d] = ap.lu[d][p] + v[d] * ig - u1[d] * ig3;
    T u0b[3], Eb[3], Bb[3];
    if (pc.vay)
        vay_adjoint(pc.h, pc.inv_c2, u, E, B, ub, u0b, Eb, Bb);
    else
        boris_adjoint(pc.h, pc.inv_c2, B, tp, ub, u0b, Eb, Bb);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ap.lu[d][p] = u0b[d];
        ap.vb[d][p] = Eb[d];
        ap.vb[3 + d][p] = Bb[d];
    }
    // the position part of the gather transpose: vb . grad(gathered fields).
    if constexpr (SST > 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            lxa[k] += Eb[0] * st[k * SST] + Eb[1] * st[(3 + k) * SST] + Eb[2] * st[(6 + k) * SST] +
                      Bb[0] * st[(9 + k) * SST] + Bb[1] * st[(12 + k) * SST] + Bb[2] * st[(15 + k) * SST];
    } else {
        // The weights and offsets are evaluated again; the register operands
        // keep the compiler from carrying those of the first gather across
        // the deposit transpose.
        T fr[3] = {f[0], f[1], f[2]};
        int cr[3] = {c[0], c[1], c[2]}, lr[3] = {l[0], l[1], l[2]};
        asm volatile("" : "+v"(fr[0]), "+v"(fr[1]), "+v"(fr[2]));
        asm volatile("" : "+v"(cr[0]), "+v"(cr[1]), "+v"(cr[2]), "+v"(lr[0]), "+v"(lr[1]), "+v"(lr[2]));
        AxisW<O, T> aw[3];
        int on[3][NW], os[3][NW];
        adjoint_offsets<T, O, LOCAL>(pc, cr, fr, lr, lo_f, sf, aw, on, os);
        T dn[3][NW], ds[3][NW];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            axis_dweights<O>(fr[d], dn[d], ds[d]);
        // staggering: E_x(s,n,n) E_y(n,s,n) E_z(n,n,s) B_x(n,s,s) B_y(s,n,s) B_z(s,s,n)
        gather_grad<O, T, 1, 0, 0>(fsrc.c[0], Eb[0], aw, dn, ds, on, os, lxa);
        gather_grad<O, T, 0, 1, 0>(fsrc.c[1], Eb[1], aw, dn, ds, on, os, lxa);
        gather_grad<O, T, 0, 0, 1>(fsrc.c[2], Eb[2], aw, dn, ds, on, os, lxa);
        gather_grad<O, T, 0, 1, 1>(fsrc.c[3], Bb[0], aw, dn, ds, on, os, lxa);
        gather_grad<O, T, 1, 0, 1>(fsrc.c[4], Bb[1], aw, dn, ds, on, os, lxa);
        gather_grad<O, T, 1, 1, 0>(fsrc.c[5], Bb[2], aw, dn, ds, on, os, lxa);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
        ap.lx[d][p] = lxa[d];
    return true;
}

// pass 2 for one particle: the scatter of the gather transpose for the
// components of group G (0: E, 1: B, 2: both), shared as scatter mode SM
// says.  The LDS accumulators hold the group's components at
// sL + (m - 3 G0) * rfvol (G0 = 1 for group B alone); runs[k] are the packed
// lane runs of the group's k-th component (null: none).
template <typename T, int O, bool LOCAL, int G, int SM = SM_RUNS>
__device__ __attribute__((always_inline)) inline void adjoint_scatter_particle(const PConst<T> &pc, const AdjPtrs<T> &ap, int64_t p,
                                                const int *c, const T *f, const int *l, int lo_f,
                                                const int *sf, double *sL, int rfvol, const int *runs)
{
    constexpr int NW = Shape<O, T>::NW;
    AxisW<O, T> aw[3];
    int on[3][NW], os[3][NW];
    adjoint_offsets<T, O, LOCAL>(pc, c, f, l, lo_f, sf, aw, on, os);
    constexpr int b = G == 1 ? 3 : 0;
    auto run = [&](int k) { return xrun_unpack(runs ? runs[k] : XRUN_ALONE); };
    // the group's values first: a load after a component's global atomics
    // would wait for them
    T vb[6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
        if ((m < 3 && G != 1) || (m >= 3 && G != 0))
            vb[m] = ap.vb[m][p];
    // staggering: E_x(s,n,n) E_y(n,s,n) E_z(n,n,s) B_x(n,s,s) B_y(s,n,s) B_z(s,s,n)
    if (G != 1) {
        scatter_component<O, T, LOCAL, SM, 1, 0, 0>(ap.lE[0], sL + (0 - b) * rfvol, vb[0], aw, on, os, sf, run(0));
        scatter_component<O, T, LOCAL, SM, 0, 1, 0>(ap.lE[1], sL + (1 - b) * rfvol, vb[1], aw, on, os, sf, run(1));
        scatter_component<O, T, LOCAL, SM, 0, 0, 1>(ap.lE[2], sL + (2 - b) * rfvol, vb[2], aw, on, os, sf, run(2));
    }
    if (G != 0) {
        const int k0 = G == 2 ? 3 : 0;
        scatter_component<O, T, LOCAL, SM, 0, 1, 1>(ap.lB[0], sL + (3 - b) * rfvol, vb[3], aw, on, os, sf, run(k0));
        scatter_component<O, T, LOCAL, SM, 1, 0, 1>(ap.lB[1], sL + (4 - b) * rfvol, vb[4], aw, on, os, sf,
                                                    run(k0 + 1));
        scatter_component<O, T, LOCAL, SM, 1, 1, 0>(ap.lB[2], sL + (5 - b) * rfvol, vb[5], aw, on, os, sf,
                                                    run(k0 + 2));
    }
}

// Packed lane runs of the components m0 .. m0+K-1 for a particle at cell
// position pos (local or global) with offsets f; key 0 (no sharing) for an
// inactive lane.  Call with the whole wave converged.
template <typename T, int O, int K, bool GLOBAL>
__device__ inline void component_runs(bool act, int m0, const int *pos, const T *f, const int *n, int *runs)
{
    constexpr int SX[6] = {1, 0, 0, 0, 1, 1}, SY[6] = {0, 1, 0, 1, 0, 1}, SZ[6] = {0, 0, 1, 1, 1, 0};
    int bs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        bs[d] = f[d] >= T(0.5) ? Shape<O, T>::NB : Shape<O, T>::NB - 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int m = m0 + k;
        // a lane's window of component m starts at its cell plus the
        // component's first-node offset; lanes share rows when these starts
        // are consecutive along x
        const int st[3] = {pos[0] + (SX[m] ? bs[0] : Shape<O, T>::NB), pos[1] + (SY[m] ? bs[1] : Shape<O, T>::NB),
                           pos[2] + (SZ[m] ? bs[2] : Shape<O, T>::NB)};
        const int key = act ? (GLOBAL ? xrun_key_global(st, n) : xrun_key(st)) : 0;
        runs[k] = xrun_pack(xrun(key));
    }
}

// Lane runs of the fixed (SM_WIDE) windows: every component's window starts
// at a fixed node relative to the cell, so one run structure, that of the
// cells, serves all six.  Call with the whole wave converged.
__device__ inline XRun wide_runs(bool act, const int *pos)
{
    return xrun(act ? xrun_key(pos) : 0);
}

// The length of this lane's run (counted up to 4, as at the run's last lane).
// Call with the whole wave converged.
__device__ inline int run_length(const XRun &xr)
{
    const int l1 = dpp_shift_int<-1>(xr.len), l2 = dpp_shift_int<-2>(xr.len), l3 = dpp_shift_int<-3>(xr.len);
    return xr.d == 0 ? xr.len : xr.d == 1 ? l1 : xr.d == 2 ? l2 : xr.d == 3 ? l3 : 4;
}

// A wave of the tiled adjoint scatter queues its short-run lanes (and shares
// rows on fixed windows) only while it has at most this many: a 64-lane
// wave's rows cost about 384 FP64 LDS add instructions on per-component
// windows with short runs present, about 242 on fixed windows plus about 6
// per queued lane and the fixed windows' extra arithmetic.  Measured at
// 8 ppc (256^3) and 2 ppc (512^3), FP32: 24 -> 62.8 / 177.3 ms per adjoint
// step, 32 -> 61.0 / 179.0, 48 -> 60.1 / 180.8, 64 (never the per-component
// path) -> 62.4 / 190.6.
constexpr int SCATTER_QUEUE_MAX = 32;

// Puts index j of every lane with `want` into an LDS queue (counter qcnt,
// entries qj, capacity qcap) with one atomic per wave; returns whether this
// lane's index went in, and in `any` whether the wave queued any.  Call with
// the whole wave converged.
__device__ inline bool queue_push_wave(bool want, int j, int *qcnt, int *qj, int qcap, bool &any)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long m = __ballot(want);
    any = m != 0;
    if (m == 0)
        return false;   // uniform across the wave
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader)
        base = atomicAdd(qcnt, __popcll(m));
    base = __shfl(base, leader);
    if (!want)
        return false;
    const int i = base + __popcll(m & ((1ull << lane) - 1ull));
    if (i >= qcap)
        return false;
    qj[i] = j;
    return true;
}

// positions only (pass 2): a particle that fails the check was flagged by
// pass 1 and is skipped
template <typename T>
__device__ inline bool load_position(const PArr<T> &in, int64_t p, const int *n, int *c, T *f)
{
    // all six loads first, then a check without short-circuit branches (a
    // branch between them would make each load wait for the one before)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = in.cell[d][p];
        f[d] = in.off[d][p];
    }
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        ok = ok & (c[d] >= 0) & (c[d] < n[d]) & (f[d] >= T(0)) & (f[d] < T(1));
    return ok;
}

template <typename T, int O>
// (at least two waves per SIMD: the FP64 order-3 pass sits at the 256
// registers that allow two, and one register more would halve them)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_adjoint_push(PConst<T> pc, PArr<T> sp, FieldPtrs<T> fp, AdjPtrs<T> ap, int *err)
{
    // the gathered-field gradients wait in LDS across the deposit transpose
    // (one sweep over the field windows in global memory instead of two)
    __shared__ T stash[18 * 256];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.n)
        return;
    int c[3];
    T f[3], u[3];
    if (!load_particle(sp, p, pc.n, c, f, u, err)) {
        clear_vb(ap, p);
        return;
    }
    const int z3[3] = {0, 0, 0};
    adjoint_push_particle<T, O, false, 256>(pc, sp, ap, global_fields(fp), ap.hat, p, c, f, u, z3, 0, z3, 0, z3, err,
                                            stash + threadIdx.x);
}

// Pass 2 without a binning: a workgroup takes BOX_CHUNK consecutive
// particles.  When the cells of a segment of them fit a box whose six FP64
// accumulator tiles (cells plus the gather halo) fit BOX_LDS, the segment
// scatters into LDS (rows shared between lanes) and the box is flushed with
// one global atomic per non-zero value; a segment that does not fit is
// halved, and one of BOX_THREADS particles that still does not fit scatters
// with global atomics.  Binned particles give compact boxes.
// One 512-thread workgroup per CU (the order-3 FP64 scatter needs about 250
// registers, so 8 waves per CU either way) with most of the LDS: a tile of
// binned particles that drifted a cell or two since the binning still fits.
constexpr int BOX_THREADS = 512;
constexpr int BOX_CHUNK = 2048;
constexpr int BOX_LDS = 144 * 1024;
constexpr int BOX_HEAD = 256;   // reduction scratch ahead of the accumulators
constexpr int BOX_MAX_CELLS = 40;   // box extent per axis (lane-run keys hold local coordinates below 56)
static_assert((6 * (BOX_THREADS / 64) + 3) * (int)sizeof(int) <= BOX_HEAD, "box reduction scratch");
static_assert(BOX_HEAD + BOX_LDS <= 160 * 1024, "box scatter LDS");

__device__ inline int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// cell offset from the reference cell along one axis, wrapped into [-n/2, n/2)
__device__ inline int box_rel(int c, int ref, int n)
{
    int r = c - ref;
    if (r < -(n >> 1))
        r += n;
    else if (r >= n - (n >> 1))
        r -= n;
    return r;
}

template <typename T, int O>
__global__ void __launch_bounds__(BOX_THREADS) k_adjoint_scatter_box(PConst<T> pc, PArr<T> sp, AdjPtrs<T> ap,
                                                                    const int *__restrict__ tile_start)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int(*wred)[6] = reinterpret_cast<int(*)[6]>(smem_raw);   // per-wave minima and maxima
    int *sref = reinterpret_cast<int *>(smem_raw) + 6 * (BOX_THREADS / 64);
    double *sL = reinterpret_cast<double *>(smem_raw + BOX_HEAD);   // BOX_LDS bytes
    constexpr int gl = O == 3 ? 2 : 1;   // gather halo below a cell
    constexpr int gh = O == 3 ? 4 : 2;   // nodes of the halo on both sides together
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // a workgroup's particles: one tile's range of a binning (split into
    // segments of BOX_CHUNK), or without one a fixed chunk
    int64_t base, end;
    if (tile_start) {
        base = tile_start[blockIdx.x];
        end = tile_start[blockIdx.x + 1];
        base = base < 0 ? 0 : (base > sp.n ? sp.n : base);
        end = end < base ? base : (end > sp.n ? sp.n : end);
    } else {
        base = (int64_t)blockIdx.x * BOX_CHUNK;
        end = base + BOX_CHUNK < sp.n ? base + BOX_CHUNK : sp.n;
    }
    int len = BOX_CHUNK;
    for (int64_t s0 = base; s0 < end;) {
        const int seg = (int)(end - s0 < len ? end - s0 : len);
        // reference cell: the segment's first particle, clamped into the grid
        if (tid == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int v = sp.cell[d][s0];
                sref[d] = v < 0 ? 0 : (v >= pc.n[d] ? pc.n[d] - 1 : v);
            }
        }
        __syncthreads();
        const int ref[3] = {sref[0], sref[1], sref[2]};
        int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
        for (int j = tid; j < seg; j += BOX_THREADS) {
            int c[3];
            T f[3];
            if (load_position(sp, s0 + j, pc.n, c, f)) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int r = box_rel(c[d], ref[d], pc.n[d]);
                    mn[d] = min(mn[d], r);
                    mx[d] = max(mx[d], r);
                }
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            mn[d] = wave_min(mn[d]);
            mx[d] = wave_max(mx[d]);
        }
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                wred[wv][d] = mn[d];
                wred[wv][3 + d] = mx[d];
            }
        }
        __syncthreads();
        int lo[3], rf[3];
        bool any = true;
        size_t vol = 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a = wred[0][d], b = wred[0][3 + d];
#pragma unroll
            for (int w = 1; w < BOX_THREADS / 64; ++w) {
                a = min(a, wred[w][d]);
                b = max(b, wred[w][3 + d]);
            }
            any = any && a <= b;
            lo[d] = a;
            rf[d] = any ? b - a + 1 + gh : 0;
            vol *= (size_t)rf[d];
        }
        __syncthreads();   // wred and sref are rewritten by the next segment
        if (!any) {        // no valid particle in the segment
            s0 += seg;
            continue;
        }
        const bool fits = rf[0] - gh <= BOX_MAX_CELLS && rf[1] - gh <= BOX_MAX_CELLS &&
                          rf[2] - gh <= BOX_MAX_CELLS && 6 * vol * sizeof(double) <= (size_t)BOX_LDS;
        if (!fits && len > BOX_THREADS) {
            len >>= 1;   // uniform: every thread read the same reductions
            continue;
        }
        if (fits) {
            const int rfvol = (int)vol;
            for (int r = tid; r < 6 * rfvol; r += BOX_THREADS)
                sL[r] = 0.0;
            __syncthreads();
            const int sf[3] = {1, rf[0], rf[0] * rf[1]};
            for (int j0 = 0; j0 < seg; j0 += BOX_THREADS) {
                const int j = j0 + tid;
                int c[3] = {0, 0, 0}, l[3] = {0, 0, 0};
                T f[3] = {T(0), T(0), T(0)};
                const bool act = j < seg && load_position(sp, s0 + j, pc.n, c, f);
                if (act) {
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        l[d] = box_rel(c[d], ref[d], pc.n[d]) - lo[d];   // in [0, rf - gh)
                }
                int runs[6];
                component_runs<T, O, 6, false>(act, 0, l, f, pc.n, runs);   // converged
                if (act)
                    adjoint_scatter_particle<T, O, true, 2>(pc, ap, s0 + j, c, f, l, gl, sf, sL, rfvol, runs);
            }
            __syncthreads();
            const int org[3] = {ref[0] + lo[0], ref[1] + lo[1], ref[2] + lo[2]};
            region_walk(pc.n, org, gl, rf[0], rf[1], rf[2], rf[0], false, [&](int r, int gi) {
#pragma unroll
                for (int m = 0; m < 6; ++m) {
                    const T v = (T)sL[m * rfvol + r];
                    if (v != T(0))
                        gatomic_add((m < 3 ? ap.lE[m] : ap.lB[m - 3]) + gi, v);
                }
            });
            __syncthreads();   // sL is cleared by the next segment
        } else {
            for (int j0 = 0; j0 < seg; j0 += BOX_THREADS) {
                const int j = j0 + tid;
                int c[3] = {0, 0, 0};
                T f[3] = {T(0), T(0), T(0)};
                const bool act = j < seg && load_position(sp, s0 + j, pc.n, c, f);
                int runs[6];
                component_runs<T, O, 6, true>(act, 0, c, f, pc.n, runs);   // converged
                if (act) {
                    const int z3[3] = {0, 0, 0};
                    adjoint_scatter_particle<T, O, false, 2>(pc, ap, s0 + j, c, f, z3, 0, z3, nullptr, 0, runs);
                }
            }
        }
        s0 += seg;
    }
}

// ---------------------------------------------------------------------------
// Tiled transpose: one workgroup per tile of the binning the forward sort
// produced; no slack, particles outside the tile take the global path.
template <typename T>
struct AdjThreads {
    static constexpr int value = sizeof(T) == 4 ? 1024 : 512;
};

// threads of the tiled pass 1: 512 leaves the order-3 FP32 pass 256
// registers (1024 capped it at 128 and spilled 29 to scratch; 25.9 against
// 27.1 ms at 256^3 / 8 ppc).  768 (a cap of 170, of which the FP32 pass
// takes 164) saves time at 8 ppc but costs 1 ms on the laser box, whose
// tiles hold about 1024 particles: a second batch of 768 threads runs a
// third full.  So FP32 takes 768 from 6 particles per cell on (`dense`),
// else 512, each its own instantiation (the kernel built for 768 ran the
// sparse workloads 8-20 % slower at 512 threads); FP64 (205 registers at
// order 1) stays at 512.
template <typename T>
struct PushThreads {
    static constexpr int value = 512;
    static constexpr int dense = sizeof(T) == 4 ? 768 : 512;
};

// pass 1, tiled: LDS holds E, B with the gather halo and hatE with the
// deposit halo (and, with STASH, each thread's 18 gathered-field gradients
// after them); strays are left to k_adjoint_push_strays.  The particles that
// stay in their cells take the narrow-window deposit transpose in the loop
// and those that change cells are listed in the tile's segment of crossq
// and run after it in full waves with the full window (STILL: dense tiles,
// and sparse ones where almost no particle changes cells).  Without STILL
// every particle takes the full window: in a sparse tile the leftover
// crossers would run alone at its end (512^3, 2 ppc, u_th 0.1c: 120.5 ->
// 126.1 ms per adjoint step with the split).
template <typename T, int O, int NTH, bool STASH, bool STILL>
__global__ void __launch_bounds__(NTH) k_adjoint_push_tile(PConst<T> pc, TileGeo tg, PArr<T> sp,
                                                                           FieldPtrs<T> fp, AdjPtrs<T> ap,
                                                                           const int *__restrict__ tile_start,
                                                                           StrayList strays, int *crossq, int *err)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int rfx = tg.rf[0], rfy = tg.rf[1];
    const int rfvol = rfx * rfy * tg.rf[2];
    const int rjx = tg.rj[0], rjy = tg.rj[1];
    const int rjvol = rjx * rjy * tg.rj[2];
    T *sF = reinterpret_cast<T *>(smem_raw);   // 6 * rfvol
    T *sH = sF + 6 * rfvol;                    // 3 * rjvol
    const TileSpan ts = tile_span(tg, tile_start, sp.n);
    if (ts.pe <= ts.ps)
        return;   // uniform across the workgroup
    const int tid = threadIdx.x, nth = blockDim.x;
    region_walk(pc.n, ts.t0, tg.lo_f, rfx, rfy, tg.rf[2], rfx, region_wraps_once(pc.n, tg.t, tg.lo_f, tg.rf),
                [&](int r, int gi) {
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        sF[m * rfvol + r] = fp.E[m][gi];
                        sF[(3 + m) * rfvol + r] = fp.B[m][gi];
                    }
                });
    region_walk(pc.n, ts.t0, tg.lo_j, rjx, rjy, tg.rj[2], rjx, region_wraps_once(pc.n, tg.t, tg.lo_j, tg.rj),
                [&](int r, int gi) {
#pragma unroll
                    for (int m = 0; m < 3; ++m)
                        sH[m * rjvol + r] = ap.hat[m][gi];
                });
    __syncthreads();
    FieldSrc<T> lf;
#pragma unroll
    for (int m = 0; m < 6; ++m)
        lf.c[m] = sF + m * rfvol;
    const T *lh[3] = {sH, sH + rjvol, sH + 2 * rjvol};
    const int sf[3] = {1, rfx, rfx * rfy};
    const int sj[3] = {1, rjx, rjx * rjy};
    const int np = (int)(ts.pe - ts.ps);
    // the count of the tile's cell-changing particles, after the stash
    int *ncross = reinterpret_cast<int *>(sH + 3 * rjvol + (STASH ? 18 * NTH : 0));
    if (tid == 0)
        *ncross = 0;
    __syncthreads();
    const StrayList cross{crossq + ts.ps, ncross, np};
    T *const stash = sH + 3 * rjvol + tid;
    for (int j0 = 0; j0 < np; j0 += nth) {
        const int j = j0 + tid;
        bool stray = false, crosser = false;
        if (j < np) {
            const int64_t p = ts.ps + j;
            int c[3];
            T f[3], u[3];
            if (!load_particle(sp, p, pc.n, c, f, u, err)) {
                clear_vb(ap, p);
            } else {
                int l[3];
                if (tile_local(tg, pc.n, ts.t0, c, l))
                    crosser = !adjoint_push_particle<T, O, true, STASH ? NTH : 0, STILL>(
                        pc, sp, ap, lf, lh, p, c, f, u, l, tg.lo_f, sf, tg.lo_j, sj, err, stash);
                else
                    stray = true;
            }
        }
        // the wave is converged here
        stray_append(stray, (int)(ts.ps + j), strays);
        stray_append(crosser, j, cross);
    }
    if constexpr (!STILL)
        return;
    __syncthreads();   // the list and its count are complete
    const int nc = *ncross;
    for (int k = tid; k < nc; k += nth) {
        const int64_t p = ts.ps + crossq[ts.ps + k];
        int c[3], l[3];
        T f[3], u[3];
        load_state(sp, p, c, f, u);   // checked in the loop above
        tile_local(tg, pc.n, ts.t0, c, l);
        adjoint_push_particle<T, O, true, STASH ? NTH : 0>(pc, sp, ap, lf, lh, p, c, f, u, l, tg.lo_f, sf, tg.lo_j,
                                                            sj, err, stash);
    }
}

// pass 1 for the listed strays, on global memory
template <typename T, int O>
__global__ void __launch_bounds__(STRAY_THREADS) k_adjoint_push_strays(PConst<T> pc, PArr<T> sp, FieldPtrs<T> fp,
                                                                       AdjPtrs<T> ap, StrayList strays, int *err)
{
    const FieldSrc<T> gf = global_fields(fp);
    const int z3[3] = {0, 0, 0};
    const int k = *strays.cnt < strays.cap ? *strays.cnt : strays.cap;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const int64_t p = strays.p[i];
        int c[3];
        T f[3], u[3];
        if (!load_particle(sp, p, pc.n, c, f, u, err))
            clear_vb(ap, p);
        else
            adjoint_push_particle<T, O, false>(pc, sp, ap, gf, ap.hat, p, c, f, u, z3, 0, z3, 0, z3, err);
    }
}

// pass 2 for the listed strays, both groups, on global memory
template <typename T, int O>
__global__ void __launch_bounds__(STRAY_THREADS) k_adjoint_scatter_strays(PConst<T> pc, PArr<T> sp, AdjPtrs<T> ap,
                                                                          StrayList strays)
{
    const int z3[3] = {0, 0, 0};
    const int k = *strays.cnt < strays.cap ? *strays.cnt : strays.cap;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const int64_t p = strays.p[i];
        int c[3];
        T f[3];
        if (load_position(sp, p, pc.n, c, f))
            adjoint_scatter_particle<T, O, false, 2>(pc, ap, p, c, f, z3, 0, z3, nullptr, 0, nullptr);
    }
}

// pass 2, tiled: LDS holds FP64 accumulators of the six field adjoints with
// the gather halo (no fields: the position part of the gather transpose is
// done in pass 1); they are flushed with one global atomic per non-zero
// value.  Strays are left to k_adjoint_scatter_strays.
//
// The rows are shared along lane runs on fixed windows (SM_WIDE).  A run
// shorter than a window row (particles that left their binned cell since
// the sort break the one-lane-per-cell order) would make the whole wave
// issue extra atomic instructions for its last lane, so the lanes of such
// runs put their particle in an LDS queue instead (qcap entries after the
// accumulators) and are scattered after the main loop, one lane per
// particle.
template <typename T, int O>
__global__ void __launch_bounds__(AdjThreads<T>::value) k_adjoint_scatter_tile(PConst<T> pc, TileGeo tg, PArr<T> sp,
                                                                              FieldPtrs<T> fp, AdjPtrs<T> ap,
                                                                              const int *__restrict__ tile_start,
                                                                              int qcap)
{
    constexpr int NW = Shape<O, T>::NW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int rfx = tg.rf[0], rfy = tg.rf[1];
    const int rfvol = rfx * rfy * tg.rf[2];
    double *sL = reinterpret_cast<double *>(smem_raw);   // 6 * rfvol
    int *qcnt = reinterpret_cast<int *>(sL + 6 * rfvol);
    int *qj = qcnt + 4;                                   // qcap entries
    const TileSpan ts = tile_span(tg, tile_start, sp.n);
    if (ts.pe <= ts.ps)
        return;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int r = tid; r < 6 * rfvol; r += nth)
        sL[r] = 0.0;
    if (tid == 0)
        *qcnt = 0;
    __syncthreads();
    const int sf[3] = {1, rfx, rfx * rfy};
    const int np = (int)(ts.pe - ts.ps);
    for (int j0 = 0; j0 < np; j0 += nth) {
        const int j = j0 + tid;
        int c[3] = {0, 0, 0}, l[3] = {0, 0, 0};
        T f[3] = {T(0), T(0), T(0)};
        const bool act = j < np && load_position(sp, ts.ps + j, pc.n, c, f) && tile_local(tg, pc.n, ts.t0, c, l);
        // the wave is converged here
        XRun xr = wide_runs(act, l);
        // a window row has up to NW + 1 taps: a run of fewer than NW lanes
        // leaves nodes to its last lane
        const bool shortrun = act && run_length(xr) < NW;
        if (__popcll(__ballot(shortrun)) > SCATTER_QUEUE_MAX) {
            // sparse wave (the high ranks of the rank-major order, low
            // densities): queueing would cost more than the extra atomic
            // instructions of the short runs, so the wave takes each
            // component's own window and runs
            int runs[6];
            component_runs<T, O, 6, false>(act, 0, l, f, pc.n, runs);
            if (act)
                adjoint_scatter_particle<T, O, true, 2, SM_RUNS>(pc, ap, ts.ps + j, c, f, l, tg.lo_f, sf, sL, rfvol,
                                                                  runs);
        } else {
            bool any = false;
            const bool queued = queue_push_wave(shortrun, j, qcnt, qj, qcap, any);
            const bool mine = act && !queued;
            if (any)
                xr = wide_runs(mine, l);   // the runs of the lanes that stay
            if (mine) {
                const int pr = xrun_pack(xr);
                const int runs[6] = {pr, pr, pr, pr, pr, pr};
                adjoint_scatter_particle<T, O, true, 2, SM_WIDE>(pc, ap, ts.ps + j, c, f, l, tg.lo_f, sf, sL,
                                                                  rfvol, runs);
            }
        }
    }
    __syncthreads();
    // the queued particles, one lane each
    const int nq = *qcnt < qcap ? *qcnt : qcap;
    for (int i = tid; i < nq; i += nth) {
        const int j = qj[i];
        int c[3] = {0, 0, 0}, l[3] = {0, 0, 0};
        T f[3] = {T(0), T(0), T(0)};
        if (load_position(sp, ts.ps + j, pc.n, c, f) && tile_local(tg, pc.n, ts.t0, c, l))
            adjoint_scatter_particle<T, O, true, 2, SM_ALONE>(pc, ap, ts.ps + j, c, f, l, tg.lo_f, sf, sL, rfvol,
                                                               nullptr);
    }
    __syncthreads();
    region_walk(pc.n, ts.t0, tg.lo_f, rfx, rfy, tg.rf[2], rfx, region_wraps_once(pc.n, tg.t, tg.lo_f, tg.rf),
                [&](int r, int gi) {
#pragma unroll
                    for (int m = 0; m < 6; ++m) {
                        const T v = (T)sL[m * rfvol + r];
                        if (v != T(0))
                            gatomic_add((m < 3 ? ap.lE[m] : ap.lB[m - 3]) + gi, v);
                    }
                });
    (void)fp;
}

// ---------------------------------------------------------------------------
// pass 2, tiled, accumulated per cell.  The scatter of a particle's gathered-
// field adjoints is the outer product vb wx (x) wy (x) wz on its window; the
// particles of one cell share that window (on a staggered axis the NW + 1
// nodes either half of the cell reaches, as in SM_WIDE), so one thread per
// cell of the tile sums its particles' outer products in registers, one
// component at a time, and adds the sum into the component's FP64 LDS
// accumulator once per cell with rows shared along x (the lanes of a wave
// are consecutive cells of the tile, so the runs are the tile's rows of
// cells).  Per particle this costs the weights and the multiply-adds of
// the outer product; the LDS rows are paid once per cell instead of once
// per particle.
//
// Which particles sit in which cell comes from a counting sort of the
// tile's particles in LDS (a chunk of up to `cap` at a time): count per
// cell, scan, list of in-tile indices per cell.  Particles in the tile's
// slack cells (they left the tile since the binning) are listed after the
// cells and scattered one lane each; particles beyond the slack are the
// stray kernel's.  Each component is flushed to the global field adjoint
// (one global atomic per non-zero value) before the next one reuses the
// accumulator, so the LDS holds one component at a time.
constexpr int CELL_THREADS = 512;

// One component (staggering SX, SY, SZ) of the per-cell scatter into the
// LDS accumulator sA, then its slack-cell particles one lane each.
template <typename T, int O, int SX, int SY, int SZ>
__device__ __attribute__((always_inline)) inline void cell_scatter_component(
    const PConst<T> &pc, const TileGeo &tg, const TileSpan &ts, const PArr<T> &sp, const T *__restrict__ vbm,
    const int *list, const int *cstart, const int *ccnt, int tc, double *sA, const int *sf)
{
    constexpr int NW = Shape<O, T>::NW, NB = Shape<O, T>::NB;
    constexpr int NX = NW + SX, NY = NW + SY, NZ = NW + SZ;
    const int nth = blockDim.x;
    for (int g0 = 0; g0 < tc; g0 += nth) {
        const int lc = g0 + (int)threadIdx.x;
        const bool cell = lc < tc;
        int l[3] = {0, 0, 0}, s = 0, k = 0;
        if (cell) {
            l[0] = lc % tg.t[0];
            l[1] = (lc / tg.t[0]) % tg.t[1];
            l[2] = lc / (tg.t[0] * tg.t[1]);
            s = cstart[lc];
            k = ccnt[lc];
        }
        T acc[NZ][NY][NX];
#pragma unroll
        for (int c = 0; c < NZ; ++c)
#pragma unroll
            for (int b = 0; b < NY; ++b)
#pragma unroll
                for (int a = 0; a < NX; ++a)
                    acc[c][b][a] = T(0);
        // the next particle's loads are issued before this one's arithmetic
        T fn[3] = {T(0), T(0), T(0)}, vn = T(0);
        if (k > 0) {
            const int64_t p = ts.ps + list[s];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                fn[d] = sp.off[d][p];
            vn = vbm[p];
        }
        for (int i = 0; i < k; ++i) {
            const T f[3] = {fn[0], fn[1], fn[2]}, v = vn;
            if (i + 1 < k) {
                const int64_t p = ts.ps + list[s + i + 1];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    fn[d] = sp.off[d][p];
                vn = vbm[p];
            }
            AxisW<O, T> aw[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                axis_weights<O>(f[d], aw[d]);
            T wx[NX], wy[NY], wz[NZ];
            scatter_axis<O, T, SX, SM_WIDE>(aw[0], wx);
            scatter_axis<O, T, SY, SM_WIDE>(aw[1], wy);
            scatter_axis<O, T, SZ, SM_WIDE>(aw[2], wz);
#pragma unroll
            for (int c = 0; c < NZ; ++c)
#pragma unroll
                for (int b = 0; b < NY; ++b) {
                    const T wyz = wy[b] * wz[c] * v;
#pragma unroll
                    for (int a = 0; a < NX; ++a)
                        acc[c][b][a] += wx[a] * wyz;
                }
        }
        // the wave is converged here: runs of consecutive cells along x
        const XRun xr = xrun(cell ? xrun_key(l) : 0);
        if (__ballot(k > 0) != 0 && cell) {
            const int x0 = l[0] + tg.lo_f + NB - SX;
            const int y0 = l[1] + tg.lo_f + NB - SY;
            const int z0 = l[2] + tg.lo_f + NB - SZ;
#pragma unroll
            for (int c = 0; c < NZ; ++c)
#pragma unroll
                for (int b = 0; b < NY; ++b)
                    xrow_add<NX>(sA + x0 + sf[1] * (y0 + b) + sf[2] * (z0 + c), acc[c][b], xr);
        }
    }
    // particles in the slack cells, one lane each on their own windows
    const int no = ccnt[tc], so = cstart[tc];
    for (int i = threadIdx.x; i < no; i += nth) {
        const int64_t p = ts.ps + list[so + i];
        int c[3], l[3];
        T f[3];
        load_position(sp, p, pc.n, c, f);
        tile_local(tg, pc.n, ts.t0, c, l);
        AxisW<O, T> aw[3];
        int on[3][NW], os[3][NW];
        adjoint_offsets<T, O, true>(pc, c, f, l, tg.lo_f, sf, aw, on, os);
        scatter_component<O, T, true, SM_ALONE, SX, SY, SZ>(nullptr, sA, vbm[p], aw, on, os, sf,
                                                              xrun_unpack(XRUN_ALONE));
    }
}

// With merge = 2 a workgroup takes two tiles adjacent along x (their
// particles are adjacent in the binning) and tg is the merged geometry
// (twice as wide, the same halo): at low densities the region flushed per
// particle shrinks.  A particle is placed only when it lies in the region
// of its own tile, the test by which pass 1 listed the strays.
template <typename T, int O>
__global__ void __launch_bounds__(CELL_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_adjoint_scatter_cells(PConst<T> pc, TileGeo tg, PArr<T> sp,
                                                                        AdjPtrs<T> ap,
                                                                        const int *__restrict__ tile_start, int cap,
                                                                        int merge)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int rfx = tg.rf[0], rfy = tg.rf[1];
    const int rfvol = rfx * rfy * tg.rf[2];
    const int tc = tg.t[0] * tg.t[1] * tg.t[2];
    double *sA = reinterpret_cast<double *>(smem_raw);   // rfvol: one component
    int *ccnt = reinterpret_cast<int *>(sA + rfvol);     // tc + 1 (the last: slack cells)
    int *cstart = ccnt + (tc + 1);                        // tc + 1
    int *keys = cstart + (tc + 1);                        // cap
    int *list = keys + cap;                               // cap
    int *sh = list + cap;                                 // scan scratch
    TileSpan ts = tile_span(tg, tile_start, sp.n);
    // the merged tiles' particles, and where the second tile's begin
    TileGeo to = tg;   // the geometry of one binning tile
    to.t[0] = tg.t[0] / merge;
    int64_t mid = ts.pe;
    if (merge > 1) {
        const int64_t N = sp.n;
        auto clampN = [&](int64_t v) { return v < 0 ? int64_t(0) : (v > N ? N : v); };
        ts.ps = clampN(tile_start[merge * ts.t]);
        mid = clampN(tile_start[merge * ts.t + 1]);
        ts.pe = clampN(tile_start[merge * ts.t + merge]);
        mid = mid < ts.ps ? ts.ps : (mid > ts.pe ? ts.pe : mid);
        if (ts.pe < ts.ps)
            ts.pe = ts.ps;
    }
    if (ts.pe <= ts.ps)
        return;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int sf[3] = {1, rfx, rfx * rfy};
    const int np = (int)(ts.pe - ts.ps);
    for (int r = tid; r < rfvol; r += nth)
        sA[r] = 0.0;
    for (int j0 = 0; j0 < np; j0 += cap) {
        const int je = np < j0 + cap ? np : j0 + cap;
        // counting sort of the chunk by cell
        for (int i = tid; i <= tc; i += nth)
            ccnt[i] = 0;
        __syncthreads();
        for (int j = j0 + tid; j < je; j += nth) {
            int c[3], l[3];
            T f[3];
            int key = -1;
            const int sub = ts.ps + j >= mid ? 1 : 0;   // which of the merged tiles
            const int t0s[3] = {ts.t0[0] + sub * to.t[0], ts.t0[1], ts.t0[2]};
            if (load_position(sp, ts.ps + j, pc.n, c, f) && tile_local(to, pc.n, t0s, c, l)) {
                l[0] += sub * to.t[0];
                const bool in = l[0] >= 0 && l[0] < tg.t[0] && l[1] >= 0 && l[1] < tg.t[1] && l[2] >= 0 &&
                                l[2] < tg.t[2];
                const int slot = in ? l[0] + tg.t[0] * (l[1] + tg.t[1] * l[2]) : tc;
                key = (slot << 16) | atomicAdd(ccnt + slot, 1);
            }
            keys[j - j0] = key;
        }
        __syncthreads();
        block_exclusive_scan(ccnt, cstart, tc + 1, sh);
        __syncthreads();
        for (int j = j0 + tid; j < je; j += nth) {
            const int key = keys[j - j0];
            if (key >= 0)
                list[cstart[key >> 16] + (key & 0xffff)] = j;
        }
        __syncthreads();
        const bool fonce = region_wraps_once(pc.n, tg.t, tg.lo_f, tg.rf);
        for (int m = 0; m < 6; ++m) {
            const T *vbm = ap.vb[m];
            // staggering: E_x(s,n,n) E_y(n,s,n) E_z(n,n,s) B_x(n,s,s) B_y(s,n,s) B_z(s,s,n)
            switch (m) {
            case 0: cell_scatter_component<T, O, 1, 0, 0>(pc, tg, ts, sp, vbm, list, cstart, ccnt, tc, sA, sf); break;
            case 1: cell_scatter_component<T, O, 0, 1, 0>(pc, tg, ts, sp, vbm, list, cstart, ccnt, tc, sA, sf); break;
            case 2: cell_scatter_component<T, O, 0, 0, 1>(pc, tg, ts, sp, vbm, list, cstart, ccnt, tc, sA, sf); break;
            case 3: cell_scatter_component<T, O, 0, 1, 1>(pc, tg, ts, sp, vbm, list, cstart, ccnt, tc, sA, sf); break;
            case 4: cell_scatter_component<T, O, 1, 0, 1>(pc, tg, ts, sp, vbm, list, cstart, ccnt, tc, sA, sf); break;
            default: cell_scatter_component<T, O, 1, 1, 0>(pc, tg, ts, sp, vbm, list, cstart, ccnt, tc, sA, sf); break;
            }
            __syncthreads();
            // flush the component and clear the accumulator for the next
            T *dst = m < 3 ? ap.lE[m] : ap.lB[m - 3];
            region_walk(pc.n, ts.t0, tg.lo_f, rfx, rfy, tg.rf[2], rfx, fonce, [&](int r, int gi) {
                const T v = (T)sA[r];
                sA[r] = 0.0;
                if (v != T(0))
                    gatomic_add(dst + gi, v);
            });
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned nblk(int64_t n, int b)
{
    return (unsigned)((n + b - 1) / b);
}

template <typename T>
size_t tile_lds_bytes(int, const TileGeo &tg)
{
    const size_t rf = (size_t)tg.rf[0] * tg.rf[1] * tg.rf[2];
    const size_t rj = (size_t)tg.jp * tg.rj[1] * tg.rj[2];
    return ((6 * rf * sizeof(T) + 15) & ~size_t(15)) + 3 * rj * sizeof(double) +
           (size_t)tg.qcap * (6 * sizeof(T) + 2 * sizeof(int)) + sizeof(int);
}

template <typename K>
static void allow_big_lds(K *kernel, bool &done)
{
    if (!done) {
        // allow more than the default dynamic LDS per workgroup
        hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
        done = true;
    }
}

// the two-phase tile kernel's queue entries and the list capacity left by
// its LDS; 0 when the list would hold fewer than 1024 particles
template <typename T>
int cells_chunk(const TileGeo &tg, TileGeo &tq)
{
    tq = tg;
    tq.qcap = sizeof(T) == 4 ? 512 : 256;
    const size_t fixed = cells_lds(tq, TileThreads<T>::value, 0, (int)sizeof(T)).total;
    const size_t limit = 160 * 1024;
    if (fixed >= limit)
        return 0;
    const size_t kc = (limit - fixed) / 8;
    if (kc < 1024)
        return 0;
    return (int)(kc < 16384 ? kc : 16384);
}

template <typename T, int O>
static hipError_t launch_tile_o(const PConst<T> &pc, const TileGeo &tg, const PArr<T> &in, const PArr<T> &out,
                                const FieldPtrs<T> &f, const int *tile_start, const StrayList &stray,
                                const GuestArgs &g, T *const scratch[3], int *err, hipStream_t st)
{
    static bool attr_plain = false, attr_guests = false, attr_cp = false, attr_cg = false;
    const unsigned ntiles = (unsigned)(tg.nt[0] * tg.nt[1] * tg.nt[2]);
    // The per-cell deposit pays where cells hold many particles, which share
    // one row update per cell, and where the deposit is the wide order-3
    // window in FP32: 256^3, 8 per cell, 21.2 -> 16.6 ms.  It loses at low
    // densities (the laser box, 2 per cell: 4.65 -> 5.0 ms; 512^3, 2 per
    // cell: 76.4 -> 78.2 ms), at order 1 (32^3 FP64: 0.049 -> 0.069 ms) and
    // in FP64 (213 registers: 31.0 against 30.9 ms at 256^3, 0.35 -> 0.38 ms
    // at 64^3 / 4 per cell).
    if constexpr (sizeof(T) == 4 && O == 3) {
        const int64_t ncell = (int64_t)tg.nt[0] * tg.t[0] * tg.nt[1] * tg.t[1] * tg.nt[2] * tg.t[2];
        TileGeo tq;
        const int kc = cells_chunk<T>(tg, tq);
        if (kc > 0 && in.n >= 6 * ncell) {
            // the old offsets of the particles that stay in their cells wait
            // in scratch when the step runs in place
            Off3<T> f0s;
            for (int d = 0; d < 3; ++d)
                f0s.o[d] = in.off[d] == out.off[d] ? scratch[d] : in.off[d];
            const size_t l = cells_lds(tq, TileThreads<T>::value, kc, (int)sizeof(T)).total;
            if (g.flag_next) {
                allow_big_lds(&k_particles_cells<T, O, true>, attr_cg);
                hipLaunchKernelGGL((k_particles_cells<T, O, true>), dim3(ntiles), dim3(TileThreads<T>::value), l, st,
                                   pc, tq, in, out, f, tile_start, stray, g, f0s, kc, err);
            } else {
                allow_big_lds(&k_particles_cells<T, O, false>, attr_cp);
                hipLaunchKernelGGL((k_particles_cells<T, O, false>), dim3(ntiles), dim3(TileThreads<T>::value), l, st,
                                   pc, tq, in, out, f, tile_start, stray, g, f0s, kc, err);
            }
            return hipGetLastError();
        }
    } else {
        (void)scratch;
        (void)attr_cp;
        (void)attr_cg;
    }
    const size_t lds = tile_lds_bytes<T>(O, tg);
    if (g.flag_next) {
        allow_big_lds(&k_particles_tile<T, O, true>, attr_guests);
        hipLaunchKernelGGL((k_particles_tile<T, O, true>), dim3(ntiles), dim3(TileThreads<T>::value), lds, st, pc, tg,
                           in, out, f, tile_start, stray, g, err);
    } else {
        allow_big_lds(&k_particles_tile<T, O, false>, attr_plain);
        hipLaunchKernelGGL((k_particles_tile<T, O, false>), dim3(ntiles), dim3(TileThreads<T>::value), lds, st, pc,
                           tg, in, out, f, tile_start, stray, g, err);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particles_tile(int order, const PConst<T> &pc, const TileGeo &tg, const PArr<T> &in,
                                 const PArr<T> &out, const FieldPtrs<T> &f, const int *tile_start,
                                 int *stray_list, int *stray_cnt, const GuestArgs &g, T *const scratch[3], int *err,
                                 hipStream_t st)
{
    const StrayList sl{stray_list, stray_cnt, (int)in.n};
    const hipError_t e0 = launch_fill<int>(stray_cnt, 1, 0, st);
    if (e0 != hipSuccess)
        return e0;
    return order == 1 ? launch_tile_o<T, 1>(pc, tg, in, out, f, tile_start, sl, g, scratch, err, st)
                      : launch_tile_o<T, 3>(pc, tg, in, out, f, tile_start, sl, g, scratch, err, st);
}

template <typename T>
hipError_t launch_particles_strays(int order, const PConst<T> &pc, const PArr<T> &in, const PArr<T> &out,
                                   const FieldPtrs<T> &f, int *stray_list, int *stray_cnt, const GuestArgs &g,
                                   int *err, hipStream_t st)
{
    if (in.n == 0)
        return hipSuccess;
    // a fixed grid that strides over the list (it is usually short)
    const StrayList sl{stray_list, stray_cnt, (int)in.n};
    const unsigned nb = (unsigned)(in.n < 1024 * STRAY_THREADS ? (in.n + STRAY_THREADS - 1) / STRAY_THREADS : 1024);
    if (order == 1)
        hipLaunchKernelGGL((k_particles_strays<T, 1>), dim3(nb), dim3(STRAY_THREADS), 0, st, pc, in, out, f, sl, g,
                           err);
    else
        hipLaunchKernelGGL((k_particles_strays<T, 3>), dim3(nb), dim3(STRAY_THREADS), 0, st, pc, in, out, f, sl, g,
                           err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particles_global(int order, const PConst<T> &pc, const PArr<T> &sp, const FieldPtrs<T> &f,
                                   int *err, hipStream_t st)
{
    if (sp.n == 0)
        return hipSuccess;
    if (order == 1)
        hipLaunchKernelGGL((k_particles_global<T, 1>), dim3(nblk(sp.n, 256)), dim3(256), 0, st, pc, sp, f, err);
    else
        hipLaunchKernelGGL((k_particles_global<T, 3>), dim3(nblk(sp.n, 256)), dim3(256), 0, st, pc, sp, f, err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(int order, const PConst<T> &pc, const PArr<T> &sp, const FieldPtrs<T> &f, T *const Ep[3],
                         T *const Bp[3], int *err, hipStream_t st)
{
    if (sp.n == 0)
        return hipSuccess;
    if (order == 1)
        hipLaunchKernelGGL((k_gather<T, 1>), dim3(nblk(sp.n, 256)), dim3(256), 0, st, pc, sp, f, Ep[0], Ep[1],
                           Ep[2], Bp[0], Bp[1], Bp[2], err);
    else
        hipLaunchKernelGGL((k_gather<T, 3>), dim3(nblk(sp.n, 256)), dim3(256), 0, st, pc, sp, f, Ep[0], Ep[1],
                           Ep[2], Bp[0], Bp[1], Bp[2], err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_push(const PConst<T> &pc, const PArr<T> &sp, T *const Ep[3], T *const Bp[3], int *err,
                       hipStream_t st)
{
    if (sp.n == 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_push<T>), dim3(nblk(sp.n, 256)), dim3(256), 0, st, pc, sp, Ep[0], Ep[1], Ep[2], Bp[0],
                       Bp[1], Bp[2], err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_deposit(int order, const PConst<T> &pc, const PArr<T> &before, const PArr<T> &after,
                          const FieldPtrs<T> &f, int *err, hipStream_t st)
{
    if (before.n == 0)
        return hipSuccess;
    if (order == 1)
        hipLaunchKernelGGL((k_deposit<T, 1>), dim3(nblk(before.n, 256)), dim3(256), 0, st, pc, before, after, f,
                           err);
    else
        hipLaunchKernelGGL((k_deposit<T, 3>), dim3(nblk(before.n, 256)), dim3(256), 0, st, pc, before, after, f,
                           err);
    return hipGetLastError();
}

template <typename T>
static AdjPtrs<T> adj_ptrs(T *const hatE[3], T *const lx[3], T *const lu[3], T *const lE[3], T *const lB[3],
                           T *const vb[6])
{
    AdjPtrs<T> a{};
    for (int d = 0; d < 3; ++d) {
        a.hat[d] = hatE[d];
        a.lx[d] = lx[d];
        a.lu[d] = lu[d];
        a.lE[d] = lE[d];
        a.lB[d] = lB[d];
    }
    for (int m = 0; m < 6; ++m)
        a.vb[m] = vb[m];
    return a;
}

template <typename T>
hipError_t launch_adjoint_particles(int order, const PConst<T> &pc, const PArr<T> &sp, const FieldPtrs<T> &f,
                                    T *const hatE[3], T *const lx[3], T *const lu[3], T *const lE[3],
                                    T *const lB[3], T *const vb[6], const int *tile_start, int ntiles, int *err,
                                    hipStream_t st)
{
    if (sp.n == 0)
        return hipSuccess;
    const AdjPtrs<T> ap = adj_ptrs<T>(hatE, lx, lu, lE, lB, vb);
    const unsigned nb = nblk(sp.n, 256), nc = tile_start ? (unsigned)ntiles : nblk(sp.n, BOX_CHUNK);
    static bool b1 = false, b3 = false;
    if (order == 1) {
        allow_big_lds(&k_adjoint_scatter_box<T, 1>, b1);
        hipLaunchKernelGGL((k_adjoint_push<T, 1>), dim3(nb), dim3(256), 0, st, pc, sp, f, ap, err);
        hipLaunchKernelGGL((k_adjoint_scatter_box<T, 1>), dim3(nc), dim3(BOX_THREADS), BOX_HEAD + BOX_LDS, st, pc, sp, ap,
                           tile_start);
    } else {
        allow_big_lds(&k_adjoint_scatter_box<T, 3>, b3);
        hipLaunchKernelGGL((k_adjoint_push<T, 3>), dim3(nb), dim3(256), 0, st, pc, sp, f, ap, err);
        hipLaunchKernelGGL((k_adjoint_scatter_box<T, 3>), dim3(nc), dim3(BOX_THREADS), BOX_HEAD + BOX_LDS, st, pc, sp, ap,
                           tile_start);
    }
    return hipGetLastError();
}

// LDS of the two tiled passes: pass 1 E, B (gather halo) and hatE (deposit
// halo) in the working precision; pass 2 FP64 accumulators of the six field
// adjoints (gather halo)
template <typename T>
size_t adjoint_push_lds(const TileGeo &tg)
{
    const size_t rf = (size_t)tg.rf[0] * tg.rf[1] * tg.rf[2];
    const size_t rj = (size_t)tg.rj[0] * tg.rj[1] * tg.rj[2];
    return 6 * rf * sizeof(T) + 3 * rj * sizeof(T) + 16;   // and the count of cell-changing particles
}

// dynamic LDS one workgroup of the tiled adjoint scatter may take
constexpr size_t ADJ_QUEUE_LDS = 160 * 1024;

template <typename T>
size_t adjoint_scatter_lds(const TileGeo &tg)
{
    const size_t rf = (size_t)tg.rf[0] * tg.rf[1] * tg.rf[2];
    return 6 * rf * sizeof(double);
}

template <typename T>
size_t adjoint_lds_bytes(int, const TileGeo &tg)
{
    const size_t a = adjoint_push_lds<T>(tg), b = adjoint_scatter_lds<T>(tg);
    return a > b ? a : b;
}

// Particles that would change cells at their present momenta, among runs
// of 64 consecutive particles every `stride` particles (whole cache lines
// read, one run in stride / 64): an estimate of the share of cell-changing
// particles in an adjoint step, which decides whether sparse tiles split
// them off.
template <typename T>
__global__ void __launch_bounds__(256) k_cross_estimate(PConst<T> pc, PArr<T> sp, int64_t stride, int *count)
{
    int mine = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = (i >> 6) * stride + (i & 63);
        if (p >= sp.n)
            break;
        const T u[3] = {sp.u[0][p], sp.u[1][p], sp.u[2][p]};
        const T ig = T(1) / sqrt(T(1) + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * pc.inv_c2);
        bool cross = false;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T x = sp.off[d][p] + pc.dtd[d] * u[d] * ig;
            cross = cross || !(x >= T(0) && x < T(1));
        }
        mine += cross ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1)
        mine += __shfl_down(mine, off, 64);
    if ((threadIdx.x & 63) == 0 && mine > 0)
        atomicAdd(count, mine);
}

template <typename T>
hipError_t launch_cross_estimate(const PConst<T> &pc, const PArr<T> &sp, int64_t samples, int *count,
                                 hipStream_t st, int64_t *taken)
{
    // runs of 64 at a stride that takes about `samples` particles
    const int64_t runs = (samples + 63) / 64;
    int64_t stride = runs > 0 ? (sp.n + runs - 1) / runs : sp.n;
    stride = stride < 64 ? 64 : (stride + 63) / 64 * 64;
    *taken = sp.n / stride * 64 + (sp.n % stride < 64 ? sp.n % stride : 64);
    const int64_t ns = *taken;
    const unsigned nb = (unsigned)(ns < 1024 * 256 ? (ns + 255) / 256 : 1024);
    const hipError_t e = launch_fill<int>(count, 1, 0, st);
    if (e != hipSuccess || ns == 0)
        return e;
    hipLaunchKernelGGL((k_cross_estimate<T>), dim3(nb), dim3(256), 0, st, pc, sp, stride, count);
    return hipGetLastError();
}

template <typename T, int O>
static hipError_t launch_adj_tile_o(const PConst<T> &pc, const TileGeo &tg, const PArr<T> &sp, const FieldPtrs<T> &f,
                                    const AdjPtrs<T> &ap, const int *tile_start, const StrayList &sl, int *crossq,
                                    bool split_sparse, int *err, hipStream_t st)
{
    static bool a1 = false, a1d = false, a2 = false;
    allow_big_lds(&k_adjoint_push_tile<T, O, PushThreads<T>::value, false, false>, a1);
    allow_big_lds(&k_adjoint_push_tile<T, O, PushThreads<T>::dense, false, true>, a1d);
    allow_big_lds(&k_adjoint_scatter_tile<T, O>, a2);
    const unsigned ntiles = (unsigned)(tg.nt[0] * tg.nt[1] * tg.nt[2]);
    const unsigned nth = AdjThreads<T>::value;
    const size_t l1 = adjoint_push_lds<T>(tg), l2 = adjoint_scatter_lds<T>(tg);
    // the LDS the accumulators leave holds the scatter's queue (16 bytes of
    // counter, then 4 per entry, up to 16384)
    const size_t room = l2 + 16 < ADJ_QUEUE_LDS ? (ADJ_QUEUE_LDS - l2 - 16) / 4 : 0;
    const int qcap = (int)(room < 16384 ? room : 16384);
    const size_t l2q = l2 + 16 + 4 * (size_t)qcap;
    // strays: listed by pass 1, taken by the stray kernels of both passes
    // (a fixed grid that strides over the list; it is usually short)
    const unsigned nsb = (unsigned)(sp.n < 1024 * STRAY_THREADS ? (sp.n + STRAY_THREADS - 1) / STRAY_THREADS : 1024);
    const hipError_t e0 = launch_fill<int>(sl.cnt, 1, 0, st);
    if (e0 != hipSuccess)
        return e0;
    const int64_t ncell = (int64_t)tg.nt[0] * tg.t[0] * tg.nt[1] * tg.t[1] * tg.nt[2] * tg.t[2];
    const bool dense = sp.n >= 6 * ncell;
    bool stashed = false;
    if constexpr (sizeof(T) == 4) {
        // the gradient stash: 18 values per thread after the field regions
        static bool s1 = false, s1d = false;
        const int nt = dense ? PushThreads<T>::dense : PushThreads<T>::value;
        const size_t ls = l1 + 18 * sizeof(T) * (size_t)nt;
        if (ls <= 160 * 1024) {
            if (dense) {
                allow_big_lds(&k_adjoint_push_tile<T, O, PushThreads<T>::dense, true, true>, s1d);
                hipLaunchKernelGGL((k_adjoint_push_tile<T, O, PushThreads<T>::dense, true, true>), dim3(ntiles),
                                   dim3(PushThreads<T>::dense), ls, st, pc, tg, sp, f, ap, tile_start, sl, crossq, err);
            } else if (split_sparse) {
                static bool s1s = false;
                allow_big_lds(&k_adjoint_push_tile<T, O, PushThreads<T>::value, true, true>, s1s);
                hipLaunchKernelGGL((k_adjoint_push_tile<T, O, PushThreads<T>::value, true, true>), dim3(ntiles),
                                   dim3(PushThreads<T>::value), ls, st, pc, tg, sp, f, ap, tile_start, sl, crossq, err);
            } else {
                allow_big_lds(&k_adjoint_push_tile<T, O, PushThreads<T>::value, true, false>, s1);
                hipLaunchKernelGGL((k_adjoint_push_tile<T, O, PushThreads<T>::value, true, false>), dim3(ntiles),
                                   dim3(PushThreads<T>::value), ls, st, pc, tg, sp, f, ap, tile_start, sl, crossq, err);
            }
            stashed = true;
        }
    }
    if (!stashed) {
        if (dense)
            hipLaunchKernelGGL((k_adjoint_push_tile<T, O, PushThreads<T>::dense, false, true>), dim3(ntiles),
                               dim3(PushThreads<T>::dense), l1, st, pc, tg, sp, f, ap, tile_start, sl, crossq, err);
        else
            hipLaunchKernelGGL((k_adjoint_push_tile<T, O, PushThreads<T>::value, false, false>), dim3(ntiles),
                               dim3(PushThreads<T>::value), l1, st, pc, tg, sp, f, ap, tile_start, sl, crossq, err);
    }
    hipLaunchKernelGGL((k_adjoint_push_strays<T, O>), dim3(nsb), dim3(STRAY_THREADS), 0, st, pc, sp, f, ap, sl, err);
    bool cells = false;
    if constexpr (sizeof(T) == 4) {
        // per-cell accumulation: one component's accumulators, the cell
        // counts and starts, and the chunk's keys and lists, within half the
        // LDS of a CU so that two workgroups share it
        static bool a3 = false;
        auto lds_of = [](const TileGeo &g, size_t &fixed) {
            const size_t rf = (size_t)g.rf[0] * g.rf[1] * g.rf[2];
            const size_t tc = (size_t)g.t[0] * g.t[1] * g.t[2];
            fixed = rf * sizeof(double) + 4 * (2 * (tc + 1) + CELL_THREADS / 64 + 4);
            const size_t half = 80 * 1024;
            return fixed < half ? (half - fixed) / 8 : size_t(0);
        };
        // below 6 particles per cell, pairs of tiles adjacent along x share
        // a workgroup when their regions and a chunk of 2048 fit
        TileGeo tm = tg;
        tm.t[0] = 2 * tg.t[0];
        tm.nt[0] = tg.nt[0] / 2;
        tm.rf[0] = tg.rf[0] + tg.t[0];
        tm.xcd_map = ((ntiles / 2) % 8 == 0) ? 1 : 0;
        size_t fixed = 0, fixed_m = 0;
        const size_t cap1 = lds_of(tg, fixed), cap_m = lds_of(tm, fixed_m);
        const bool merge = !dense && tg.nt[0] >= 4 && tg.nt[0] % 2 == 0 && tm.rf[0] <= 64 && cap_m >= 2048;
        const size_t cap = merge ? cap_m : cap1;
        if (cap >= 1024) {
            const int c = (int)(cap < 16384 ? cap : 16384);
            const size_t l3 = (merge ? fixed_m : fixed) + 8 * (size_t)c;
            allow_big_lds(&k_adjoint_scatter_cells<T, O>, a3);
            hipLaunchKernelGGL((k_adjoint_scatter_cells<T, O>), dim3(merge ? ntiles / 2 : ntiles), dim3(CELL_THREADS),
                               l3, st, pc, merge ? tm : tg, sp, ap, tile_start, c, merge ? 2 : 1);
            cells = true;
        }
    }
    if (!cells)
        hipLaunchKernelGGL((k_adjoint_scatter_tile<T, O>), dim3(ntiles), dim3(nth), l2q, st, pc, tg, sp, f, ap,
                           tile_start, qcap);
    hipLaunchKernelGGL((k_adjoint_scatter_strays<T, O>), dim3(nsb), dim3(STRAY_THREADS), 0, st, pc, sp, ap, sl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_tile(int order, const PConst<T> &pc, const TileGeo &tg, const PArr<T> &sp,
                               const FieldPtrs<T> &f, T *const hatE[3], T *const lx[3], T *const lu[3],
                               T *const lE[3], T *const lB[3], T *const vb[6], const int *tile_start,
                               int *stray_list, int *stray_cnt, int *crossq, bool split_sparse, int *err,
                               hipStream_t st)
{
    const StrayList sl{stray_list, stray_cnt, (int)sp.n};
    if (sp.n == 0)
        return hipSuccess;
    const AdjPtrs<T> ap = adj_ptrs<T>(hatE, lx, lu, lE, lB, vb);
    if (order == 1)
        return launch_adj_tile_o<T, 1>(pc, tg, sp, f, ap, tile_start, sl, crossq, split_sparse, err, st);
    // FP64 order 3 has no tiled form (its pass 1 needs 256 registers and
    // spills; the caller runs the per-particle kernels with the binning)
    if constexpr (sizeof(T) == 8)
        return hipErrorNotSupported;
    else
        return launch_adj_tile_o<T, 3>(pc, tg, sp, f, ap, tile_start, sl, crossq, split_sparse, err, st);
}

#define PIC_INST(T)                                                                                               \
    template size_t tile_lds_bytes<T>(int, const TileGeo &);                                                       \
    template hipError_t launch_particles_tile<T>(int, const PConst<T> &, const TileGeo &, const PArr<T> &,         \
                                                 const PArr<T> &, const FieldPtrs<T> &, const int *, int *, int *, \
                                                 const GuestArgs &, T *const[3], int *, hipStream_t);              \
    template hipError_t launch_particles_strays<T>(int, const PConst<T> &, const PArr<T> &, const PArr<T> &,       \
                                                   const FieldPtrs<T> &, int *, int *, const GuestArgs &, int *,   \
                                                   hipStream_t);                                                   \
    template hipError_t launch_particles_global<T>(int, const PConst<T> &, const PArr<T> &, const FieldPtrs<T> &,  \
                                                   int *, hipStream_t);                                            \
    template hipError_t launch_gather<T>(int, const PConst<T> &, const PArr<T> &, const FieldPtrs<T> &,            \
                                         T *const[3], T *const[3], int *, hipStream_t);                            \
    template hipError_t launch_push<T>(const PConst<T> &, const PArr<T> &, T *const[3], T *const[3], int *,        \
                                       hipStream_t);                                                               \
    template hipError_t launch_deposit<T>(int, const PConst<T> &, const PArr<T> &, const PArr<T> &,                \
                                          const FieldPtrs<T> &, int *, hipStream_t);                               \
    template hipError_t launch_adjoint_particles<T>(int, const PConst<T> &, const PArr<T> &, const FieldPtrs<T> &, \
                                                    T *const[3], T *const[3], T *const[3], T *const[3],            \
                                                    T *const[3], T *const[6], const int *, int, int *,              \
                                                    hipStream_t);                                                  \
    template size_t adjoint_lds_bytes<T>(int, const TileGeo &);                                                    \
    template hipError_t launch_adjoint_tile<T>(int, const PConst<T> &, const TileGeo &, const PArr<T> &,           \
                                               const FieldPtrs<T> &, T *const[3], T *const[3], T *const[3],        \
                                               T *const[3], T *const[3], T *const[6], const int *, int *, int *,   \
                                               int *, bool, int *, hipStream_t);                                   \
    template hipError_t launch_cross_estimate<T>(const PConst<T> &, const PArr<T> &, int64_t, int *, hipStream_t,   \
                                                 int64_t *);

PIC_INST(float)
PIC_INST(double)

}  // namespace pic
