// Grid kernels of the EM-PIC step for gfx950: the Yee curl updates (and
// their transposes), the counting sort that bins particles by tile-major
// cell (Sec. 3.4.2), and the FP64 reductions (Sec. 2.6).  All of them are
// bound by HBM bandwidth: coalesced x-fastest access, one pass per update.
#include "pic_device.hpp"
#include "pic_types.hpp"

namespace pic {

// ---------------------------------------------------------------------------
// Curl updates.  Forward differences take edge-centred vectors to faces,
// backward differences take face-centred vectors to edges (Sec. 2.4, Yee):
//   curl_f(S)_x = (S_z[j+1] - S_z)/dy - (S_y[k+1] - S_y)/dz      (cyclic)
//   curl_b(S)_x = (S_z - S_z[j-1])/dy - (S_y - S_y[k-1])/dz
// The coefficients cx, cy, cz already hold (scale / d).

// The part of an update after the curl: out = in + curl terms (+ J, source,
// source adjoint), for cell o = (i, j, k).
template <typename T>
__device__ inline void curl_finish(const CurlArgs<T> &a, int i, int j, int k, int64_t o, T dx_sy, T dx_sz, T dy_sx,
                                   T dy_sz, T dz_sx, T dz_sy)
{
    const T tx = a.cy * dy_sz - a.cz * dz_sy;
    const T ty = a.cz * dz_sx - a.cx * dx_sz;
    const T tz = a.cx * dx_sy - a.cy * dy_sx;
    T vx = a.in[0][o] + tx;
    T vy = a.in[1][o] + ty;
    T vz = a.in[2][o] + tz;
    if (a.J[0]) {
        vx += a.jc * a.J[0][o];
        vy += a.jc * a.J[1][o];
        vz += a.jc * a.J[2][o];
        if (a.zero_j) {
            a.J[0][o] = T(0);
            a.J[1][o] = T(0);
            a.J[2][o] = T(0);
        }
    }
    if (k == a.kplane) {
        if (a.amp)
            vx += a.amp[i + (int64_t)a.n[0] * j] * a.ag;
        if (a.dA)
            a.dA[i + (int64_t)a.n[0] * j] += a.dag * (double)vx;
    }
    a.out[0][o] = vx;
    a.out[1][o] = vy;
    a.out[2][o] = vz;
    if (a.out2[0]) {   // the same update again from the result (two B half steps around one E)
        a.out2[0][o] = vx + tx;
        a.out2[1][o] = vy + ty;
        a.out2[2][o] = vz + tz;
    }
}

template <typename T, bool FWD>
__global__ void __launch_bounds__(256) k_curl(CurlArgs<T> a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    if (i >= n0)
        return;
    const int64_t o = i + (int64_t)n0 * (j + (int64_t)n1 * k);
    int64_t xs, ys, zs;   // neighbour offsets (+1 for forward, -1 for backward), periodic
    if (FWD) {
        xs = (i + 1 < n0) ? 1 : 1 - n0;
        ys = (j + 1 < n1) ? n0 : (int64_t)n0 * (1 - n1);
        zs = (k + 1 < n2) ? (int64_t)n0 * n1 : (int64_t)n0 * n1 * (1 - n2);
    } else {
        xs = (i > 0) ? -1 : n0 - 1;
        ys = (j > 0) ? -(int64_t)n0 : (int64_t)n0 * (n1 - 1);
        zs = (k > 0) ? -(int64_t)n0 * n1 : (int64_t)n0 * n1 * (n2 - 1);
    }
    const T *Sx = a.src[0], *Sy = a.src[1], *Sz = a.src[2];
    // forward: S[o + s] - S[o]; backward: S[o] - S[o + s] (s the -1 offset)
    auto d = [&](const T *S, int64_t s) -> T { return FWD ? S[o + s] - S[o] : S[o] - S[o + s]; };
    curl_finish(a, i, j, k, o, d(Sy, xs), d(Sz, xs), d(Sx, ys), d(Sz, ys), d(Sx, zs), d(Sy, zs));
}

// CKC form: each difference along an axis is the weighted sum of the same
// difference at the 3 x 3 cells around it across the axis (centre alpha,
// edges beta_p / beta_q, corners gamma).  A workgroup takes a 64 x 4 x 4 block
// of cells; the three source components of the block plus one cell on every
// side (periodic) are staged in LDS, and each difference is read from there
// (54 differences per cell).
constexpr int CKC_TX = 64, CKC_TY = 4, CKC_TZ = 4;

template <typename T, bool FWD>
__global__ void __launch_bounds__(CKC_TX *CKC_TY) k_curl_ckc(CurlArgs<T> a)
{
    constexpr int LX = CKC_TX + 2, LY = CKC_TY + 2, LZ = CKC_TZ + 2, LV = LX * LY * LZ;
    __shared__ T s[3 * LV];
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int x0 = blockIdx.x * CKC_TX, y0 = blockIdx.y * CKC_TY, z0 = blockIdx.z * CKC_TZ;
    // periodic index of v >= -1 (a block can pass the end of a grid smaller
    // than itself more than once: the rare modulo)
    auto wrap = [](int v, int n) {
        v = v < 0 ? v + n : v;
        v = v >= n ? v - n : v;
        return v >= n ? v % n : v;
    };
    // every load of the staging is issued before any LDS store, so that the
    // loads overlap (divisions by compile-time constants only)
    constexpr int NTH = CKC_TX * CKC_TY, NPER = (3 * LV + NTH - 1) / NTH;
    const int tid = threadIdx.x + CKC_TX * threadIdx.y;
    T v[NPER];
#pragma unroll
    for (int t = 0; t < NPER; ++t) {
        const int r = tid + t * NTH;
        if (r < 3 * LV) {
            const int c = r / LV, q = r - c * LV;
            const int lx = q % LX, ly = (q / LX) % LY, lz = q / (LX * LY);
            const int gx = wrap(x0 - 1 + lx, n0), gy = wrap(y0 - 1 + ly, n1), gz = wrap(z0 - 1 + lz, n2);
            v[t] = a.src[c][gx + (int64_t)n0 * (gy + (int64_t)n1 * gz)];
        }
    }
#pragma unroll
    for (int t = 0; t < NPER; ++t) {
        const int r = tid + t * NTH;
        if (r < 3 * LV)
            s[r] = v[t];
    }
    __syncthreads();
    const int i = x0 + threadIdx.x, j = y0 + threadIdx.y;
    if (i >= n0 || j >= n1)
        return;   // no barrier follows
    constexpr int st[3] = {1, LX, LX * LY};
    // difference of component c along axis ax at LDS cell l, averaged across ax
    auto diff = [&](int c, int ax, int l) -> T {
        const T *S = s + c * LV;
        const int p = ax == 2 ? 0 : ax + 1, q = ax == 0 ? 2 : ax - 1;
        const int sa = FWD ? st[ax] : -st[ax];
        auto d1 = [&](int m) -> T { return FWD ? S[m + sa] - S[m] : S[m] - S[m + sa]; };
        const T *w = a.ck[ax];
        const int sp = st[p], sq = st[q];
        return w[0] * d1(l) + w[1] * (d1(l + sp) + d1(l - sp)) + w[2] * (d1(l + sq) + d1(l - sq)) +
               w[3] * (d1(l + sp + sq) + d1(l + sp - sq) + d1(l - sp + sq) + d1(l - sp - sq));
    };
    for (int tz = 0; tz < CKC_TZ; ++tz) {
        const int k = z0 + tz;
        if (k >= n2)
            break;
        const int l = (threadIdx.x + 1) + LX * ((threadIdx.y + 1) + LY * (tz + 1));
        const int64_t o = i + (int64_t)n0 * (j + (int64_t)n1 * k);
        curl_finish(a, i, j, k, o, diff(1, 0, l), diff(2, 0, l), diff(0, 1, l), diff(2, 1, l), diff(0, 2, l),
                    diff(1, 2, l));
    }
}

template <typename T>
hipError_t launch_curl(bool forward, const CurlArgs<T> &a, hipStream_t st)
{
    if (a.ckc) {
        dim3 grid((a.n[0] + CKC_TX - 1) / CKC_TX, (a.n[1] + CKC_TY - 1) / CKC_TY, (a.n[2] + CKC_TZ - 1) / CKC_TZ);
        if (forward)
            hipLaunchKernelGGL((k_curl_ckc<T, true>), grid, dim3(CKC_TX, CKC_TY), 0, st, a);
        else
            hipLaunchKernelGGL((k_curl_ckc<T, false>), grid, dim3(CKC_TX, CKC_TY), 0, st, a);
        return hipGetLastError();
    }
    const int bx = a.n[0] >= 256 ? 256 : (a.n[0] >= 128 ? 128 : 64);
    dim3 grid((a.n[0] + bx - 1) / bx, a.n[1], a.n[2]);
    if (forward)
        hipLaunchKernelGGL((k_curl<T, true>), grid, dim3(bx), 0, st, a);
    else
        hipLaunchKernelGGL((k_curl<T, false>), grid, dim3(bx), 0, st, a);
    return hipGetLastError();
}

// Symmetric filter along z (the fields before the gather): out = w0 F +
// sum_{s=1..3} w_s (F[k+s] + F[k-s]), periodic in z; add: out += that.
// One thread per cell, x fastest (coalesced; the z neighbours are whole
// planes away and come from L2).
template <typename T>
__global__ void __launch_bounds__(256) k_filter_z(const T *__restrict__ in, T *__restrict__ out, T w0, T w1, T w2,
                                                   T w3, int add, int nxy, int nz)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (int64_t)nxy * nz)
        return;
    const int k = (int)(o / nxy);
    const int64_t r = o - (int64_t)k * nxy;
    auto at = [&](int kk) -> T {
        kk = kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk);   // |shift| <= 3 < nz
        return in[r + (int64_t)kk * nxy];
    };
    T v = w0 * in[o];
    if (w1 != T(0))
        v += w1 * (at(k + 1) + at(k - 1));
    if (w2 != T(0))
        v += w2 * (at(k + 2) + at(k - 2));
    if (w3 != T(0))
        v += w3 * (at(k + 3) + at(k - 3));
    out[o] = add ? out[o] + v : v;
}

template <typename T>
hipError_t launch_filter_z(const T *in, T *out, const T w[4], bool add, const int n[3], hipStream_t st)
{
    const int64_t nc = (int64_t)n[0] * n[1] * n[2];
    if (nc == 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_filter_z<T>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, in, out, w[0], w[1],
                       w[2], w[3], add ? 1 : 0, n[0] * n[1], n[2]);
    return hipGetLastError();
}

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Sets `bit` in *err when tile_start does not run from 0 to n (a binning of
// other particles, or an array never filled).
__global__ void k_check_binning(const int *tile_start, int ntiles, int64_t n, int *err, int bit)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && (tile_start[0] != 0 || (int64_t)tile_start[ntiles] != n))
        atomicOr(err, bit);
}

hipError_t launch_check_binning(const int *tile_start, int ntiles, int64_t n, int *err, int bit, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_binning, dim3(1), dim3(64), 0, st, tile_start, ntiles, n, err, bit);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    int64_t b = (n + 255) / 256;
    if (b > 65536)
        b = 65536;
    hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)b), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

template <typename T>
__global__ void k_scale(T *out, const T *in, int64_t n, T a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a * in[i];
}

template <typename T>
hipError_t launch_scale(T *out, const T *in, int64_t n, T a, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    int64_t b = (n + 255) / 256;
    if (b > 65536)
        b = 65536;
    hipLaunchKernelGGL((k_scale<T>), dim3((unsigned)b), dim3(256), 0, st, out, in, n, a);
    return hipGetLastError();
}

__global__ void k_sum2(const double *in, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        out[0] = in[0] + in[1];
}

hipError_t launch_sum2(const double *in, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(64), 0, st, in, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Counting sort by tile-major cell key (Sec. 3.4.2).  Pass 1 computes each
// particle's key and its rank inside the key's bin with one atomic increment
// per particle; an exclusive scan of the bin counts gives bin offsets; pass 2
// scatters every particle to offset[key] + rank.

template <typename T>
__global__ void __launch_bounds__(256) k_bin_count(PArr<T> sp, TileGeo tg, int n0, int n1, int n2, int *counts,
                                                   int *key, int *rank, int *err)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.n)
        return;
    int c[3] = {sp.cell[0][p], sp.cell[1][p], sp.cell[2][p]};
    const int n[3] = {n0, n1, n2};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T f = sp.off[d][p];
        ok = ok && c[d] >= 0 && c[d] < n[d] && f >= T(0) && f < T(1);
        c[d] = c[d] < 0 ? 0 : (c[d] >= n[d] ? n[d] - 1 : c[d]);   // keep the key in range
    }
    if (!ok)
        atomicOr(err, 1);
    const int tx = c[0] / tg.t[0], ty = c[1] / tg.t[1], tz = c[2] / tg.t[2];
    const int lx = c[0] - tx * tg.t[0], ly = c[1] - ty * tg.t[1], lz = c[2] - tz * tg.t[2];
    const int tile = tx + tg.nt[0] * (ty + tg.nt[1] * tz);
    const int kk = tile * (tg.t[0] * tg.t[1] * tg.t[2]) + lx + tg.t[0] * (ly + tg.t[1] * lz);
    key[p] = kk;
    rank[p] = atomicAdd(counts + kk, 1);
}

// Counting pass for particles that are still binned by an earlier sort: one
// workgroup per tile counts its particles' current cells in an LDS
// histogram over the tile plus a margin of BC_MARGIN cells, reserves each
// non-empty cell's range with one global atomic, and hands out ranks inside
// the range.  Particles beyond the margin count with a global atomic.  Ranks
// and keys mean exactly what k_bin_count produces.
static constexpr int BC_T = 512;
static constexpr int BC_MARGIN = 2;
static constexpr int BC_GROUP = 4;   // chunks loaded ahead of their ranking

template <typename T>
__global__ void __launch_bounds__(BC_T) k_bin_count_tile(PArr<T> sp, TileGeo tg, int n0, int n1, int n2,
                                                         const int *tile_start, int *counts, int *key, int *rank,
                                                         int *err)
{
    extern __shared__ int lc[];
    const int n[3] = {n0, n1, n2};
    const int rx = tg.t[0] + 2 * BC_MARGIN, ry = tg.t[1] + 2 * BC_MARGIN, rz = tg.t[2] + 2 * BC_MARGIN;
    const int rvol = rx * ry * rz;
    const int t = blockIdx.x;
    const int tc[3] = {t % tg.nt[0], (t / tg.nt[0]) % tg.nt[1], t / (tg.nt[0] * tg.nt[1])};
    const int t0[3] = {tc[0] * tg.t[0], tc[1] * tg.t[1], tc[2] * tg.t[2]};
    const int tcells = tg.t[0] * tg.t[1] * tg.t[2];
    const int64_t N = sp.n;
    int64_t ps = tile_start[t], pe = tile_start[t + 1];
    ps = ps < 0 ? 0 : (ps > N ? N : ps);
    pe = pe < ps ? ps : (pe > N ? N : pe);
    // A particle inside the margin region lies in this tile or a neighbour
    // (tiles at least BC_MARGIN cells wide), so its key needs no division.
    // Its region cell and local rank are packed into the rank word (region
    // cells below 2^rb, ranks below 2^(31 - rb): at most 2^(31 - rb)
    // particles in the segment), so that the second pass reads nothing else.
    const int rb = 32 - __clz(rvol - 1);
    const bool packed = rb <= 20 && pe - ps <= ((int64_t)1 << (31 - rb));
    const bool nodiv = tg.t[0] >= BC_MARGIN && tg.t[1] >= BC_MARGIN && tg.t[2] >= BC_MARGIN;
    for (int r = threadIdx.x; r < rvol; r += blockDim.x)
        lc[r] = 0;
    __syncthreads();
    // pass 1: keys; local ranks (stored negative) or global ranks.  The
    // chunks of blockDim.x particles are ranked one after the other (a
    // barrier between them), so particles that kept their cell keep their
    // order and the scatter below writes long runs of consecutive slots.
    // The loads and keys of BC_GROUP chunks are taken first, so the barriers
    // separate only the LDS ranking steps.
    // (indices fit 32 bits: a species holds fewer than 2^31 particles)
    const unsigned ue = (unsigned)pe;
    for (unsigned g0 = (unsigned)ps; g0 < ue; g0 += BC_GROUP * blockDim.x) {
        // every load of the group first (no store between them, so they are
        // all in flight together), then the keys
        int cg[BC_GROUP][3];
        T fg[BC_GROUP][3];
#pragma unroll
        for (int j = 0; j < BC_GROUP; ++j) {
            const unsigned p = g0 + j * blockDim.x + threadIdx.x;
            if (p < ue) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    cg[j][d] = sp.cell[d][p];
                    fg[j][d] = sp.off[d][p];
                }
            }
        }
        int reg[BC_GROUP];   // region cell of the chunk's particle, or -1
#pragma unroll
        for (int j = 0; j < BC_GROUP; ++j) {
            const unsigned p = g0 + j * blockDim.x + threadIdx.x;
            reg[j] = -1;
            if (p < ue) {
                int c[3] = {cg[j][0], cg[j][1], cg[j][2]};
                bool ok = true;
                int v[3];
                bool inside = true;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const T f = fg[j][d];
                    ok = ok & (c[d] >= 0) & (c[d] < n[d]) & (f >= T(0)) & (f < T(1));
                    c[d] = c[d] < 0 ? 0 : (c[d] >= n[d] ? n[d] - 1 : c[d]);
                    int w = c[d] - t0[d];
                    if (w < -BC_MARGIN)
                        w += n[d];
                    else if (w >= tg.t[d] + BC_MARGIN)
                        w -= n[d];
                    v[d] = w;
                    inside = inside & (w >= -BC_MARGIN) & (w < tg.t[d] + BC_MARGIN);
                }
                if (!ok)
                    atomicOr(err, 1);
                int kk;
                if (inside && nodiv) {
                    int tile = 0, loc = 0;
#pragma unroll
                    for (int d = 2; d >= 0; --d) {
                        const int o = v[d] < 0 ? -1 : (v[d] >= tg.t[d] ? 1 : 0);
                        int td = tc[d] + o;
                        td = td < 0 ? td + tg.nt[d] : (td >= tg.nt[d] ? td - tg.nt[d] : td);
                        tile = tile * tg.nt[d] + td;
                        loc = loc * tg.t[d] + (v[d] - o * tg.t[d]);
                    }
                    kk = tile * tcells + loc;
                } else {
                    const int cx = c[0] / tg.t[0], cy = c[1] / tg.t[1], cz = c[2] / tg.t[2];
                    const int tile = cx + tg.nt[0] * (cy + tg.nt[1] * cz);
                    kk = tile * tcells + (c[0] - cx * tg.t[0]) +
                         tg.t[0] * ((c[1] - cy * tg.t[1]) + tg.t[1] * (c[2] - cz * tg.t[2]));
                }
                key[p] = kk;
                if (inside)
                    reg[j] = (v[0] + BC_MARGIN) + rx * ((v[1] + BC_MARGIN) + ry * (v[2] + BC_MARGIN));
                else
                    rank[p] = atomicAdd(counts + kk, 1);
            }
        }
#pragma unroll
        for (int j = 0; j < BC_GROUP; ++j) {
            if (g0 + j * blockDim.x >= ue)
                break;   // uniform across the workgroup
            const unsigned p = g0 + j * blockDim.x + threadIdx.x;
            if (reg[j] >= 0) {
                const int lr = atomicAdd(lc + reg[j], 1);
                rank[p] = packed ? -1 - ((lr << rb) | reg[j]) : -1 - lr;
            }
            __syncthreads();
        }
    }
    // reserve each region cell's range in the global counts
    for (int r = threadIdx.x; r < rvol; r += blockDim.x) {
        const int m = lc[r];
        if (m > 0) {
            const int gx = ((t0[0] - BC_MARGIN + r % rx) % n0 + n0) % n0;
            const int gy = ((t0[1] - BC_MARGIN + (r / rx) % ry) % n1 + n1) % n1;
            const int gz = ((t0[2] - BC_MARGIN + r / (rx * ry)) % n2 + n2) % n2;
            const int cx = gx / tg.t[0], cy = gy / tg.t[1], cz = gz / tg.t[2];
            const int tile = cx + tg.nt[0] * (cy + tg.nt[1] * cz);
            const int kk = tile * tcells + (gx - cx * tg.t[0]) +
                           tg.t[0] * ((gy - cy * tg.t[1]) + tg.t[1] * (gz - cz * tg.t[2]));
            lc[r] = atomicAdd(counts + kk, m);
        }
    }
    __syncthreads();
    // pass 2: local rank + the range base
    for (int64_t p = ps + threadIdx.x; p < pe; p += blockDim.x) {
        const int rk = rank[p];
        if (rk < 0) {
            const int v = -1 - rk;
            if (packed) {
                rank[p] = lc[v & ((1 << rb) - 1)] + (v >> rb);
            } else {
                int l[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    int c = sp.cell[d][p];
                    c = c < 0 ? 0 : (c >= n[d] ? n[d] - 1 : c);
                    int w = c - t0[d];
                    if (w < -BC_MARGIN)
                        w += n[d];
                    else if (w >= tg.t[d] + BC_MARGIN)
                        w -= n[d];
                    l[d] = w + BC_MARGIN;
                }
                rank[p] = lc[l[0] + rx * (l[1] + ry * l[2])] + v;
            }
        }
    }
}

template <typename T>
hipError_t launch_bin_count_tile(const PArr<T> &sp, const TileGeo &tg, const int *tile_start, int *counts, int *key,
                                 int *rank, int *err, hipStream_t st)
{
    if (sp.n == 0)
        return hipSuccess;
    const int n0 = tg.t[0] * tg.nt[0], n1 = tg.t[1] * tg.nt[1], n2 = tg.t[2] * tg.nt[2];
    const size_t lds = sizeof(int) * (size_t)(tg.t[0] + 2 * BC_MARGIN) * (tg.t[1] + 2 * BC_MARGIN) *
                       (tg.t[2] + 2 * BC_MARGIN);
    const unsigned ntiles = (unsigned)(tg.nt[0] * tg.nt[1] * tg.nt[2]);
    hipLaunchKernelGGL((k_bin_count_tile<T>), dim3(ntiles), dim3(BC_T), lds, st, sp, tg, n0, n1, n2, tile_start,
                       counts, key, rank, err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bin_count(const PArr<T> &sp, const TileGeo &tg, int *counts, int *key, int *rank, int *err,
                            hipStream_t st)
{
    if (sp.n == 0)
        return hipSuccess;
    const int n0 = tg.t[0] * tg.nt[0], n1 = tg.t[1] * tg.nt[1], n2 = tg.t[2] * tg.nt[2];
    hipLaunchKernelGGL((k_bin_count<T>), dim3((unsigned)((sp.n + 255) / 256)), dim3(256), 0, st, sp, tg, n0, n1, n2,
                       counts, key, rank, err);
    return hipGetLastError();
}

// Order inside a tile: rank-major ("interleaved"), i.e. the first particle of
// every non-empty cell in cell order, then the second particle of every cell
// holding at least two, and so on.  Consecutive particles then sit in
// consecutive cells, so a wave that reads them with coalesced loads has its
// lanes in distinct neighbouring cells (distinct LDS addresses for the same
// stencil offset).  One workgroup per tile computes the in-tile slot of
// every (cell, rank) pair from the cell offsets of the counting sort:
//   slot(c, r) = sum_{r' < r} #{cells with count > r'} + #{c' < c : count(c') > r}
// written to slot_of[offset(c) + r].
static constexpr int IL_T = 512;

__device__ inline int block_excl_scan_512(int v, int *sh, int &total)
{
    // inclusive scan inside each wave, then over the eight wave totals
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < IL_T / 64; ++w) {
            const int t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[IL_T / 64] = run;
    }
    __syncthreads();
    const int res = sh[wv] + x - v;
    total = sh[IL_T / 64];
    __syncthreads();
    return res;
}

// PER cells per thread, contiguous (a compile-time count, so that the
// per-cell registers are indexed statically in the loop over rank levels)
template <int PER>
__global__ void __launch_bounds__(IL_T) k_interleave(const int *offsets, const int *tile_start, int tile_cells,
                                                     int *slot_of)
{
    __shared__ int sh[IL_T / 64 + 1];
    __shared__ int smax;
    const int t = blockIdx.x;
    const int64_t c0 = (int64_t)t * tile_cells;
    constexpr int per = PER;
    const int tend = tile_start[t + 1];
    int cnt[PER], off[PER];
    int mymax = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) {
        const int lc = threadIdx.x * per + i;
        cnt[i] = 0;
        off[i] = 0;
        if (lc < tile_cells) {
            off[i] = offsets[c0 + lc];
            const int nxt = (lc + 1 < tile_cells) ? offsets[c0 + lc + 1] : tend;
            cnt[i] = nxt - off[i];
            mymax = cnt[i] > mymax ? cnt[i] : mymax;
        }
    }
    if (threadIdx.x == 0)
        smax = 0;
    __syncthreads();
    atomicMax(&smax, mymax);
    __syncthreads();
    const int levels = smax;
    int base = 0;
    for (int r = 0; r < levels; ++r) {
        int mine = 0;
#pragma unroll
        for (int i = 0; i < per; ++i)
            mine += cnt[i] > r ? 1 : 0;
        int total = 0;
        int pos = block_excl_scan_512(mine, sh, total) + base;
#pragma unroll
        for (int i = 0; i < per; ++i)
            if (cnt[i] > r)
                slot_of[off[i] + r] = pos++;
        base += total;
    }
}

hipError_t launch_interleave(const int *offsets, const int *tile_start, int tile_cells, int ntiles, int *slot_of,
                             hipStream_t st)
{
    if (tile_cells > 8 * IL_T)
        return hipErrorInvalidValue;
    const dim3 g((unsigned)ntiles), b(IL_T);
    if (tile_cells <= IL_T)
        hipLaunchKernelGGL(k_interleave<1>, g, b, 0, st, offsets, tile_start, tile_cells, slot_of);
    else if (tile_cells <= 2 * IL_T)
        hipLaunchKernelGGL(k_interleave<2>, g, b, 0, st, offsets, tile_start, tile_cells, slot_of);
    else if (tile_cells <= 4 * IL_T)
        hipLaunchKernelGGL(k_interleave<4>, g, b, 0, st, offsets, tile_start, tile_cells, slot_of);
    else
        hipLaunchKernelGGL(k_interleave<8>, g, b, 0, st, offsets, tile_start, tile_cells, slot_of);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(PArr<T> in, PArr<T> out, const int *key, const int *rank,
                                                 const int *offsets, const int *slot_of, const int *tile_start,
                                                 int tile_cells, int *perm)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= in.n)
        return;
    const int k = key[p];
    const int64_t q = (int64_t)tile_start[k / tile_cells] + slot_of[(int64_t)offsets[k] + rank[p]];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        out.cell[d][q] = in.cell[d][p];
        out.off[d][q] = in.off[d][p];
        out.u[d][q] = in.u[d][p];
    }
    if (in.w)
        out.w[q] = in.w[p];
    if (perm)
        perm[q] = (int)p;
}

// Tile-staged scatter for a re-sort.  One workgroup per old tile moves that
// tile's particles.  Between sorts particles enter and leave cells, which
// shifts the ranks inside most cells, so even the particles that stay in the
// tile land at slots scattered over its new segment.  The workgroup places
// them into an LDS image of the segment, one array at a time, and writes the
// image out with coalesced stores of only the slots it filled; particles
// bound for another tile are stored directly.  A tile whose old or new
// segment exceeds SCT_CAP particles stores every particle directly.
static constexpr int SCT_T = 1024;
static constexpr int SCT_CAP = 8192;   // a multiple of SCT_T

static constexpr int SCT_PER = SCT_CAP / SCT_T;

template <typename V>
__device__ inline void sct_array(const V *src, V *dst, int64_t ps, int np, int ws, int wn, const int *qb,
                                 V *img, const unsigned char *mark)
{
    // all of a thread's loads are issued before its stores
    V v[SCT_PER];
#pragma unroll
    for (int k = 0; k < SCT_PER; ++k) {
        const int j = threadIdx.x + k * SCT_T;
        if (j < np)
            v[k] = src[ps + j];
    }
#pragma unroll
    for (int k = 0; k < SCT_PER; ++k) {
        const int j = threadIdx.x + k * SCT_T;
        if (j < np) {
            const int q = qb[j];
            const int rel = q - ws;
            if (rel >= 0 && rel < wn)
                img[rel] = v[k];
            else
                dst[q] = v[k];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < wn; i += blockDim.x)
        if (mark[i])
            dst[ws + i] = img[i];
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(SCT_T) k_scatter_tile(PArr<T> in, PArr<T> out, const int *key, const int *rank,
                                                        const int *offsets, const int *slot_of,
                                                        const int *tile_start, const int *old_start, int tile_cells,
                                                        int *perm)
{
    extern __shared__ __align__(16) unsigned char sct_raw[];
    void *img = sct_raw;                                                  // SCT_CAP values of T (or int)
    int *qb = reinterpret_cast<int *>(sct_raw + SCT_CAP * sizeof(T));    // destination of each particle
    unsigned char *mark = sct_raw + SCT_CAP * (sizeof(T) + 4);           // image slots this workgroup fills
    const int t = blockIdx.x;
    const int64_t N = in.n;
    int64_t ps = old_start[t], pe = old_start[t + 1];
    ps = ps < 0 ? 0 : (ps > N ? N : ps);
    pe = pe < ps ? ps : (pe > N ? N : pe);
    const int np = (int)(pe - ps);
    const int ws = tile_start[t], wn = tile_start[t + 1] - ws;
    if (np == 0)
        return;
    auto dest = [&](int64_t p) {
        const int k = key[p];
        return tile_start[k / tile_cells] + slot_of[(int64_t)offsets[k] + rank[p]];
    };
    if (np > SCT_CAP || wn > SCT_CAP || wn < 0) {   // uniform across the workgroup
        for (int j = threadIdx.x; j < np; j += blockDim.x) {
            const int64_t p = ps + j;
            const int q = dest(p);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                out.cell[d][q] = in.cell[d][p];
                out.off[d][q] = in.off[d][p];
                out.u[d][q] = in.u[d][p];
            }
            if (in.w)
                out.w[q] = in.w[p];
            if (perm)
                perm[q] = (int)p;
        }
        return;
    }
    for (int i = threadIdx.x; i < wn; i += blockDim.x)
        mark[i] = 0;
    {
        // the dependent loads of a thread's particles proceed side by side
        int k[SCT_PER], o[SCT_PER];
#pragma unroll
        for (int e = 0; e < SCT_PER; ++e) {
            const int j = threadIdx.x + e * SCT_T;
            k[e] = j < np ? key[ps + j] : 0;
        }
#pragma unroll
        for (int e = 0; e < SCT_PER; ++e) {
            const int j = threadIdx.x + e * SCT_T;
            o[e] = j < np ? offsets[k[e]] + rank[ps + j] : 0;
        }
#pragma unroll
        for (int e = 0; e < SCT_PER; ++e) {
            const int j = threadIdx.x + e * SCT_T;
            if (j < np)
                qb[j] = tile_start[k[e] / tile_cells] + slot_of[o[e]];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < np; j += blockDim.x) {
        const int rel = qb[j] - ws;
        if (rel >= 0 && rel < wn)
            mark[rel] = 1;
    }
    __syncthreads();
    int *ii = static_cast<int *>(img);
    T *ti = static_cast<T *>(img);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sct_array<int>(in.cell[d], out.cell[d], ps, np, ws, wn, qb, ii, mark);
        sct_array<T>(in.off[d], out.off[d], ps, np, ws, wn, qb, ti, mark);
        sct_array<T>(in.u[d], out.u[d], ps, np, ws, wn, qb, ti, mark);
    }
    if (in.w)
        sct_array<T>(in.w, out.w, ps, np, ws, wn, qb, ti, mark);
    if (perm) {
        for (int j = threadIdx.x; j < np; j += blockDim.x) {
            const int rel = qb[j] - ws;
            if (rel >= 0 && rel < wn)
                ii[rel] = (int)(ps + j);
            else
                perm[qb[j]] = (int)(ps + j);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < wn; i += blockDim.x)
            if (mark[i])
                perm[ws + i] = ii[i];
    }
}

template <typename T>
hipError_t launch_scatter(const PArr<T> &in, const PArr<T> &out, const int *key, const int *rank,
                          const int *offsets, const int *slot_of, const int *tile_start, const int *old_start,
                          int ntiles, int tile_cells, int *perm, hipStream_t st)
{
    if (in.n == 0)
        return hipSuccess;
    if (old_start) {
        static bool attr = false;
        const size_t lds = (size_t)SCT_CAP * (sizeof(T) + 5);
        if (!attr) {
            hipFuncSetAttribute(reinterpret_cast<const void *>(&k_scatter_tile<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            attr = true;
        }
        hipLaunchKernelGGL((k_scatter_tile<T>), dim3((unsigned)ntiles), dim3(SCT_T), lds, st, in, out, key, rank,
                           offsets, slot_of, tile_start, old_start, tile_cells, perm);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_scatter<T>), dim3((unsigned)((in.n + 255) / 256)), dim3(256), 0, st, in, out, key, rank,
                       offsets, slot_of, tile_start, tile_cells, perm);
    return hipGetLastError();
}

// Exclusive scan of int32 in three passes (block sums, scan of the sums,
// block-local rescan with the block offset).  Each block covers SCAN_CHUNK
// elements, 16 per thread.
static constexpr int SCAN_T = 256;
static constexpr int SCAN_PER = 16;
static constexpr int SCAN_CHUNK = SCAN_T * SCAN_PER;

int64_t scan_blocks(int64_t n)
{
    return (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
}

// inclusive block scan of one value per thread; returns the block total
__device__ inline int block_incl_scan(int v, int *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int add = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    return sh[tid];
}

__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(const int *data, int64_t n, int *bsum)
{
    __shared__ int sh[SCAN_T];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
    int s = 0;
#pragma unroll
    for (int e = 0; e < SCAN_PER; ++e)
        if (base + e < n)
            s += data[base + e];
    const int incl = block_incl_scan(s, sh);
    if (threadIdx.x == SCAN_T - 1)
        bsum[blockIdx.x] = incl;
}

// one workgroup scans the block sums (exclusive), chunk by chunk
__global__ void __launch_bounds__(SCAN_T) k_scan_top(int *bsum, int64_t nb)
{
    __shared__ int sh[SCAN_T];
    int carry = 0;
    for (int64_t base = 0; base < nb; base += (int64_t)SCAN_T * SCAN_PER) {
        const int64_t b0 = base + (int64_t)threadIdx.x * SCAN_PER;
        int loc[SCAN_PER];
        int s = 0;
#pragma unroll
        for (int e = 0; e < SCAN_PER; ++e) {
            loc[e] = (b0 + e < nb) ? bsum[b0 + e] : 0;
            s += loc[e];
        }
        const int incl = block_incl_scan(s, sh);
        int run = carry + incl - s;
#pragma unroll
        for (int e = 0; e < SCAN_PER; ++e) {
            if (b0 + e < nb)
                bsum[b0 + e] = run;
            run += loc[e];
        }
        const int total = sh[SCAN_T - 1];
        __syncthreads();
        carry += total;
    }
}

__global__ void __launch_bounds__(SCAN_T) k_scan_down(int *data, int64_t n, const int *bsum)
{
    __shared__ int sh[SCAN_T];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
    int loc[SCAN_PER];
    int s = 0;
#pragma unroll
    for (int e = 0; e < SCAN_PER; ++e) {
        loc[e] = (base + e < n) ? data[base + e] : 0;
        s += loc[e];
    }
    const int incl = block_incl_scan(s, sh);
    int run = bsum[blockIdx.x] + incl - s;
#pragma unroll
    for (int e = 0; e < SCAN_PER; ++e) {
        if (base + e < n)
            data[base + e] = run;
        run += loc[e];
    }
}

hipError_t launch_scan(int *data, int64_t n, int *bsum, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t nb = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, st, data, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_T), 0, st, data, n, bsum);
    return hipGetLastError();
}

__global__ void k_tile_start(const int *offsets, int tile_cells, int ntiles, int64_t np, int *tile_start)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles)
        tile_start[t] = offsets[(int64_t)t * tile_cells];
    else if (t == ntiles)
        tile_start[t] = (int)np;
}

hipError_t launch_tile_start(const int *offsets, int tile_cells, int ntiles, int64_t np, int *tile_start,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_tile_start, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0, st, offsets,
                       tile_cells, ntiles, np, tile_start);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 reductions in one pass over cells and particles (Sec. 2.6: several
// reductions in a single launch).  Blocks [0, nbf) sum |E|^2 and |B|^2 over
// cells, blocks [nbf, nbf+nbp) sum w (gamma-1), w and w u_z over particles;
// each block writes its five partial sums, and one final block adds them in
// block order (deterministic) and applies the physical scale factors.

static constexpr int RED_T = 256;
static constexpr int RED_U = 4;   // elements per thread and iteration of k_reduce
static constexpr int RED_MAX_BLOCKS = 4096;

int reduce_max_blocks()
{
    return RED_MAX_BLOCKS;
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline void block_sum5(double *v, double *sh, double *dst)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0)
            sh[wv * 5 + k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double s = 0;
        for (int w = 0; w < RED_T / 64; ++w)
            s += sh[w * 5 + threadIdx.x];
        dst[threadIdx.x] = s;
    }
}

template <typename T>
__global__ void __launch_bounds__(RED_T) k_reduce(PArr<T> sp, int has_sp, FieldPtrs<T> f, int64_t ncell, int nbf,
                                                  int nbp, double inv_c2, double w0, double *partials)
{
    __shared__ double sh[(RED_T / 64) * 5];
    double v[5] = {0, 0, 0, 0, 0};
    // RED_U strided elements per iteration, all loaded before any is used
    // (one element per iteration leaves too few loads in flight); the last
    // fewer than RED_U one at a time
    if ((int)blockIdx.x < nbf) {
        const int64_t stride = (int64_t)nbf * RED_T;
        auto add = [&](const T *e, const T *b) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double ed = (double)e[m], bd = (double)b[m];
                v[0] += ed * ed;
                v[1] += bd * bd;
            }
        };
        int64_t i = (int64_t)blockIdx.x * RED_T + threadIdx.x;
        for (; i + (RED_U - 1) * stride < ncell; i += RED_U * stride) {
            T e[RED_U][3], b[RED_U][3];
#pragma unroll
            for (int k = 0; k < RED_U; ++k)
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    e[k][m] = f.E[m][i + k * stride];
                    b[k][m] = f.B[m][i + k * stride];
                }
#pragma unroll
            for (int k = 0; k < RED_U; ++k)
                add(e[k], b[k]);
        }
        for (; i < ncell; i += stride) {
            const T e[3] = {f.E[0][i], f.E[1][i], f.E[2][i]}, b[3] = {f.B[0][i], f.B[1][i], f.B[2][i]};
            add(e, b);
        }
    } else if (has_sp) {
        const int bb = blockIdx.x - nbf;
        const int64_t stride = (int64_t)nbp * RED_T;
        auto add = [&](const T *u, double w) {
            const double ux = u[0], uy = u[1], uz = u[2];
            const double uu = (ux * ux + uy * uy + uz * uz) * inv_c2;
            const double gm = sqrt(1.0 + uu);
            v[2] += w * uu / (gm + 1.0);   // gamma - 1 without cancellation
            v[3] += w;
            v[4] += w * uz;
        };
        int64_t p = (int64_t)bb * RED_T + threadIdx.x;
        if (sp.w) {
            for (; p + (RED_U - 1) * stride < sp.n; p += RED_U * stride) {
                T u[RED_U][3], w[RED_U];
#pragma unroll
                for (int k = 0; k < RED_U; ++k) {
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        u[k][d] = sp.u[d][p + k * stride];
                    w[k] = sp.w[p + k * stride];
                }
#pragma unroll
                for (int k = 0; k < RED_U; ++k)
                    add(u[k], (double)w[k]);
            }
        } else {
            for (; p + (RED_U - 1) * stride < sp.n; p += RED_U * stride) {
                T u[RED_U][3];
#pragma unroll
                for (int k = 0; k < RED_U; ++k)
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        u[k][d] = sp.u[d][p + k * stride];
#pragma unroll
                for (int k = 0; k < RED_U; ++k)
                    add(u[k], w0);
            }
        }
        for (; p < sp.n; p += stride) {
            const T u[3] = {sp.u[0][p], sp.u[1][p], sp.u[2][p]};
            add(u, sp.w ? (double)sp.w[p] : w0);
        }
    }
    block_sum5(v, sh, partials + 5 * (int64_t)blockIdx.x);
}

__global__ void __launch_bounds__(RED_T) k_reduce_final(const double *partials, int nb, double s0, double s1,
                                                        double s2, double s3, double s4, double *out)
{
    __shared__ double sh[(RED_T / 64) * 5];
    // each thread sums a contiguous range of blocks in order
    const int per = (nb + RED_T - 1) / RED_T;
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x * per; b < (threadIdx.x + 1) * per && b < nb; ++b)
#pragma unroll
        for (int k = 0; k < 5; ++k)
            v[k] += partials[5 * b + k];
    __shared__ double tot[5];
    block_sum5(v, sh, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = s0 * tot[0];
        out[1] = s1 * tot[1];
        out[2] = s2 * tot[2];
        out[3] = s3 * tot[3];
        out[4] = s4 * tot[4];
    }
}

template <typename T>
hipError_t launch_reduce(const PArr<T> *sp, const FieldPtrs<T> &f, int64_t ncell, double *partials, int max_blocks,
                         const double scale[7], double *out, hipStream_t st)
{
    // scale[0..4]: factors of the five sums; scale[5] = 1/c^2; scale[6] = w0
    int nbf = (int)((ncell + RED_T * 8 - 1) / (RED_T * 8));
    int nbp = sp ? (int)((sp->n + RED_T * 8 - 1) / (RED_T * 8)) : 0;
    const int half = max_blocks / 2;
    nbf = nbf < 1 ? 1 : (nbf > half ? half : nbf);
    nbp = nbp > half ? half : nbp;
    PArr<T> s{};
    if (sp)
        s = *sp;
    hipLaunchKernelGGL((k_reduce<T>), dim3(nbf + nbp), dim3(RED_T), 0, st, s, sp ? 1 : 0, f, ncell, nbf, nbp,
                       scale[5], scale[6], partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_T), 0, st, partials, nbf + nbp, scale[0], scale[1], scale[2],
                       scale[3], scale[4], out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gauss-law residual (diagnostic).  The species' charge density at the nodes
// with the order-O B-spline, rho(i,j,k) = sum_p q w_p S S S / dV, accumulated
// in FP64 (weights evaluated in FP64 from the offsets) with global atomics;
// then, per node, r = div E - (rho + rho_bg)/eps0 with the backward
// differences that take edge fields to nodes and the immobile neutralising
// background rho_bg = -(sum_p q w_p)/(ncell dV), summed as r^2,
// ((rho + rho_bg)/eps0)^2 and rho.

template <typename T, int O>
__global__ void __launch_bounds__(256) k_rho(PArr<T> sp, int nx, int ny, int nz, double qdv, double w0, double *rho,
                                             int *err)
{
    using S = Shape<O, double>;
    constexpr int NW = S::NW;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.n)
        return;
    const int n[3] = {nx, ny, nz};
    int c[3];
    double wt[3][NW];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = sp.cell[d][p];
        const T f = sp.off[d][p];
        ok = ok && c[d] >= 0 && c[d] < n[d] && f >= T(0) && f < T(1);
        S::w((double)f, wt[d]);
    }
    if (!ok) {
        atomicOr(err, 1);
        return;
    }
    const double qw = qdv * (sp.w ? (double)sp.w[p] : w0);
    int ix[NW], iy[NW], iz[NW];
#pragma unroll
    for (int a = 0; a < NW; ++a) {
        int v = c[0] + S::NB + a;
        ix[a] = v < 0 ? v + nx : (v >= nx ? v - nx : v);
        v = c[1] + S::NB + a;
        iy[a] = v < 0 ? v + ny : (v >= ny ? v - ny : v);
        v = c[2] + S::NB + a;
        iz[a] = v < 0 ? v + nz : (v >= nz ? v - nz : v);
    }
#pragma unroll
    for (int k = 0; k < NW; ++k)
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const double wyz = qw * wt[1][j] * wt[2][k];
            const int64_t row = (int64_t)nx * (iy[j] + (int64_t)ny * iz[k]);
#pragma unroll
            for (int i = 0; i < NW; ++i)
                atomicAdd(rho + row + ix[i], wyz * wt[0][i]);
        }
}

template <typename T>
__global__ void __launch_bounds__(RED_T) k_gauss(FieldPtrs<T> f, const double *rho, const double *qsum, int nx,
                                                 int ny, int nz, double idx, double idy, double idz, double bg_scale,
                                                 double inv_eps0, double *partials)
{
    __shared__ double sh[(RED_T / 64) * 5];
    const int64_t nxy = (int64_t)nx * ny, ncell = nxy * nz;
    const double bg = bg_scale * qsum[0];   // -(sum q w)/(ncell dV)
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t o = (int64_t)blockIdx.x * RED_T + threadIdx.x; o < ncell; o += (int64_t)gridDim.x * RED_T) {
        const int i = (int)(o % nx), j = (int)((o / nx) % ny), k = (int)(o / nxy);
        const int64_t ox = i > 0 ? o - 1 : o + nx - 1;
        const int64_t oy = j > 0 ? o - nx : o + nxy - nx;
        const int64_t oz = k > 0 ? o - nxy : o + ncell - nxy;
        const double div = ((double)f.E[0][o] - (double)f.E[0][ox]) * idx +
                           ((double)f.E[1][o] - (double)f.E[1][oy]) * idy +
                           ((double)f.E[2][o] - (double)f.E[2][oz]) * idz;
        const double rt = (rho[o] + bg) * inv_eps0;
        const double r = div - rt;
        v[0] += r * r;
        v[1] += rt * rt;
        v[2] += rho[o];
    }
    block_sum5(v, sh, partials + 5 * (int64_t)blockIdx.x);
}

__global__ void __launch_bounds__(RED_T) k_gauss_final(const double *partials, int nb, double dV, double *out)
{
    __shared__ double sh[(RED_T / 64) * 5];
    __shared__ double tot[5];
    const int per = (nb + RED_T - 1) / RED_T;
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x * per; b < (threadIdx.x + 1) * per && b < nb; ++b)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            v[k] += partials[5 * b + k];
    block_sum5(v, sh, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = sqrt(tot[0]);
        out[1] = sqrt(tot[1]);
        out[2] = tot[2] * dV;
    }
}

template <typename T>
hipError_t launch_gauss(int order, const PArr<T> &sp, const FieldPtrs<T> &f, const int n[3], const double d[3],
                        double q, double w0, double eps0, double *rho, const double *qsum, double *partials,
                        int max_blocks, double *out, int *err, hipStream_t st)
{
    const double dV = d[0] * d[1] * d[2];
    const int64_t ncell = (int64_t)n[0] * n[1] * n[2];
    if (sp.n > 0) {
        const unsigned nb = (unsigned)((sp.n + 255) / 256);
        if (order == 3)
            hipLaunchKernelGGL((k_rho<T, 3>), dim3(nb), dim3(256), 0, st, sp, n[0], n[1], n[2], q / dV, w0, rho, err);
        else
            hipLaunchKernelGGL((k_rho<T, 1>), dim3(nb), dim3(256), 0, st, sp, n[0], n[1], n[2], q / dV, w0, rho, err);
    }
    int nb = (int)((ncell + RED_T * 8 - 1) / (RED_T * 8));
    nb = nb < 1 ? 1 : (nb > max_blocks ? max_blocks : nb);
    hipLaunchKernelGGL((k_gauss<T>), dim3(nb), dim3(RED_T), 0, st, f, rho, qsum, n[0], n[1], n[2], 1.0 / d[0],
                       1.0 / d[1], 1.0 / d[2], -1.0 / ((double)ncell * dV), 1.0 / eps0, partials);
    hipLaunchKernelGGL(k_gauss_final, dim3(1), dim3(RED_T), 0, st, partials, nb, dV, out);
    return hipGetLastError();
}

#define PIC_GINST(T)                                                                                             \
    template hipError_t launch_curl<T>(bool, const CurlArgs<T> &, hipStream_t);                                   \
    template hipError_t launch_filter_z<T>(const T *, T *, const T[4], bool, const int[3], hipStream_t);         \
    template hipError_t launch_fill<T>(T *, int64_t, T, hipStream_t);                                             \
    template hipError_t launch_scale<T>(T *, const T *, int64_t, T, hipStream_t);                                 \
    template hipError_t launch_bin_count<T>(const PArr<T> &, const TileGeo &, int *, int *, int *, int *,         \
                                            hipStream_t);                                                         \
    template hipError_t launch_bin_count_tile<T>(const PArr<T> &, const TileGeo &, const int *, int *, int *,     \
                                                 int *, int *, hipStream_t);                                      \
    template hipError_t launch_scatter<T>(const PArr<T> &, const PArr<T> &, const int *, const int *, const int *, \
                                          const int *, const int *, const int *, int, int, int *, hipStream_t);   \
    template hipError_t launch_reduce<T>(const PArr<T> *, const FieldPtrs<T> &, int64_t, double *, int,           \
                                         const double[7], double *, hipStream_t);                                 \
    template hipError_t launch_gauss<T>(int, const PArr<T> &, const FieldPtrs<T> &, const int[3], const double[3], \
                                        double, double, double, double *, const double *, double *, int, double *, \
                                        int *, hipStream_t);

PIC_GINST(float)
PIC_GINST(double)
template hipError_t launch_fill<int>(int *, int64_t, int, hipStream_t);

}  // namespace pic
