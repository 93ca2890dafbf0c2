// Kernel-argument structs and launcher declarations shared by the HIP
// translation units of the library (host and device side).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pic {

// Per-step constants of the particle update, in the working precision T.
template <typename T>
struct PConst {
    int n[3];
    T dtd[3];      // dt / d_d: displacement in cells per unit velocity
    T h;           // q dt / (2 m)
    T inv_c2;      // 1 / c^2
    T jk[3];       // -q / (dt d_p d_q): Esirkepov prefactor per unit weight
    T w0;          // weight when the species has no weight array
    T lj;          // -dt / eps0: current adjoint from the field adjoint
    int vay;       // momentum update: 0 Boris, 1 Vay
};

// Structure-of-arrays particle storage.
template <typename T>
struct PArr {
    int *cell[3];
    T *off[3];
    T *u[3];
    T *w;          // may be null
    int64_t n;
};

template <typename T>
struct FieldPtrs {
    T *E[3], *B[3], *J[3];
};

// Tile decomposition of the grid and the LDS regions of one tile: fields
// with the gather halo (lo_f cells below, extent rf) and current with the
// deposit halo (lo_j, rj).  `slack` extra cells on each side keep particles
// that drifted since the last sort on the LDS path.
struct TileGeo {
    int t[3];      // tile size in cells
    int nt[3];     // tiles per direction
    int slack;
    int lo_f, rf[3];
    int lo_j, rj[3];
    int jp;        // row pitch of the forward kernel's LDS current tile (>= rj[0])
    int xcd_map;   // spread consecutive tiles so each XCD gets a contiguous block
    int qcap;      // entries of the tile kernel's LDS queue of cell-crossing particles
};

// Arguments of the curl-update kernel:
//   out = in + (cx,cy,cz)-weighted curl(src)  [forward or backward differences]
//         + jc * J                       (J may be null; zero_j clears J)
//   out_x[kplane] += amp * ag            (plane source, amp may be null)
//   dA[i + n0 j] += dag * out_x[kplane]  (source adjoint, dA may be null)
//   with ckc set, every difference is the CKC transverse average of the
//   differences at the 3x3 neighbours across its axis
template <typename T>
struct CurlArgs {
    T *out[3];
    T *out2[3];       // non-null: out2 = out + the same curl terms (no J or source)
    const T *in[3];
    const T *src[3];
    T cx, cy, cz;
    T *J[3];
    T jc;
    int zero_j;
    const T *amp;
    T ag;
    int kplane;
    double *dA;
    double dag;
    int n[3];
    int ckc;          // differences averaged over transverse neighbours (CKC)
    T ck[3][4];       // per difference axis a: alpha, beta_p, beta_q, gamma (p = a+1, q = a+2)
};

// Guests: a particle whose cell, after a step, lies outside the region
// (tile + slack) of its binned ("home") tile is handed to the tile that holds
// its cell for the next step, whose kernel moves it with its LDS fields and
// current; without a free list slot it goes to the stray kernel instead.
// Lists and flags are double-buffered by step.
struct GuestArgs {
    const int *cnt;              // guests per tile this step (null: no guests this step)
    const int2 *list;            // [tile * cap + i]: (particle, home tile)
    const unsigned char *flag;   // per particle: 1 = handled by a host tile this step (null: none)
    int *cnt_next;               // guests per tile next step, zeroed before the launch
    int2 *list_next;
    unsigned char *flag_next;    // written for every particle the launch moves
    int cap;                     // list slots per tile
};

// ---------------------------------------------------------------------------
// launchers (return hipSuccess or the launch error)

// stray_list (int[n]) and stray_cnt (one int, cleared by the launcher):
// the particles the tile kernel leaves to the stray kernel; scratch: three
// T[n] arrays that hold old offsets between the two-phase kernel's phases
// when in and out are the same arrays
template <typename T>
hipError_t launch_particles_tile(int order, const PConst<T> &pc, const TileGeo &tg, const PArr<T> &in,
                                 const PArr<T> &out, const FieldPtrs<T> &f, const int *tile_start,
                                 int *stray_list, int *stray_cnt, const GuestArgs &g, T *const scratch[3], int *err,
                                 hipStream_t st);
// the particles the tile kernel listed, on global memory
template <typename T>
hipError_t launch_particles_strays(int order, const PConst<T> &pc, const PArr<T> &in, const PArr<T> &out,
                                   const FieldPtrs<T> &f, int *stray_list, int *stray_cnt, const GuestArgs &g,
                                   int *err, hipStream_t st);
template <typename T>
hipError_t launch_particles_global(int order, const PConst<T> &pc, const PArr<T> &sp, const FieldPtrs<T> &f,
                                   int *err, hipStream_t st);
template <typename T>
hipError_t launch_gather(int order, const PConst<T> &pc, const PArr<T> &sp, const FieldPtrs<T> &f, T *const Ep[3],
                         T *const Bp[3], int *err, hipStream_t st);
template <typename T>
hipError_t launch_push(const PConst<T> &pc, const PArr<T> &sp, T *const Ep[3], T *const Bp[3], int *err,
                       hipStream_t st);
template <typename T>
hipError_t launch_deposit(int order, const PConst<T> &pc, const PArr<T> &before, const PArr<T> &after,
                          const FieldPtrs<T> &f, int *err, hipStream_t st);
// adjoint launchers: vb[6] is per-particle scratch (T[n] each) that carries
// the adjoints of the gathered E and B from the first pass to the second
// (the per-particle passes; with tile_start, a binning of sp, the scatter
// takes one tile's particles per workgroup)
template <typename T>
hipError_t launch_adjoint_particles(int order, const PConst<T> &pc, const PArr<T> &sp, const FieldPtrs<T> &f,
                                    T *const hatE[3], T *const lx[3], T *const lu[3], T *const lE[3],
                                    T *const lB[3], T *const vb[6], const int *tile_start, int ntiles, int *err,
                                    hipStream_t st);
template <typename T>
size_t tile_lds_bytes(int order, const TileGeo &tg);
template <typename T>
size_t adjoint_lds_bytes(int order, const TileGeo &tg);
// stray_list: int[n] scratch, stray_cnt: one int of scratch (cleared by the
// launcher): the particles outside their tile's region, listed by the first
// pass for the stray kernels; crossq: int[n] scratch, where the first pass
// lists each tile's particles that change cells (in the tile's segment);
// split_sparse: below 6 particles per cell too, run those separately (the
// particles that stay in their cells take the narrow window)
template <typename T>
hipError_t launch_adjoint_tile(int order, const PConst<T> &pc, const TileGeo &tg, const PArr<T> &sp,
                               const FieldPtrs<T> &f, T *const hatE[3], T *const lx[3], T *const lu[3],
                               T *const lE[3], T *const lB[3], T *const vb[6], const int *tile_start,
                               int *stray_list, int *stray_cnt, int *crossq, bool split_sparse, int *err,
                               hipStream_t st);
// count[0] = the particles, among about `samples` of them (runs of 64
// spread over the arrays; *taken = how many), whose offsets would leave
// [0,1) after a move with their present momenta (count cleared first)
template <typename T>
hipError_t launch_cross_estimate(const PConst<T> &pc, const PArr<T> &sp, int64_t samples, int *count,
                                 hipStream_t st, int64_t *taken);

template <typename T>
hipError_t launch_curl(bool forward, const CurlArgs<T> &a, hipStream_t st);
// sets `bit` in *err when tile_start[0] != 0 or tile_start[ntiles] != n
hipError_t launch_check_binning(const int *tile_start, int ntiles, int64_t n, int *err, int bit, hipStream_t st);
// out = (add ? out : 0) + symmetric z filter of in with taps w[0..3] (periodic)
template <typename T>
hipError_t launch_filter_z(const T *in, T *out, const T w[4], bool add, const int n[3], hipStream_t st);
template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t st);
template <typename T>
hipError_t launch_scale(T *out, const T *in, int64_t n, T a, hipStream_t st);
hipError_t launch_sum2(const double *in, double *out, hipStream_t st);
template <typename T>
hipError_t launch_bin_count(const PArr<T> &sp, const TileGeo &tg, int *counts, int *key, int *rank, int *err,
                            hipStream_t st);
template <typename T>
hipError_t launch_bin_count_tile(const PArr<T> &sp, const TileGeo &tg, const int *tile_start, int *counts, int *key,
                                 int *rank, int *err, hipStream_t st);
// old_start (the binning before this sort, or null): with it the scatter is
// staged per old tile in LDS
template <typename T>
hipError_t launch_scatter(const PArr<T> &in, const PArr<T> &out, const int *key, const int *rank,
                          const int *offsets, const int *slot_of, const int *tile_start, const int *old_start,
                          int ntiles, int tile_cells, int *perm, hipStream_t st);
hipError_t launch_interleave(const int *offsets, const int *tile_start, int tile_cells, int ntiles, int *slot_of,
                             hipStream_t st);
hipError_t launch_scan(int *data, int64_t n, int *block_sums, hipStream_t st);
hipError_t launch_tile_start(const int *offsets, int tile_cells, int ntiles, int64_t nparticles, int *tile_start,
                             hipStream_t st);
template <typename T>
hipError_t launch_reduce(const PArr<T> *sp, const FieldPtrs<T> &f, int64_t ncell, double *partials,
                         int max_blocks, const double scale[7], double *out, hipStream_t st);

// Gauss-law residual: rho (double[ncell], zeroed by the caller) receives the
// species' nodal charge density; qsum points at the species' total charge
// sum q w (device); out[0] = |div E - rho_total/eps0|_2 over the nodes,
// out[1] = |rho_total/eps0|_2, out[2] = sum of rho dV (the species' charge),
// rho_total including the uniform neutralising background.
template <typename T>
hipError_t launch_gauss(int order, const PArr<T> &sp, const FieldPtrs<T> &f, const int n[3], const double d[3],
                        double q, double w0, double eps0, double *rho, const double *qsum, double *partials,
                        int max_blocks, double *out, int *err, hipStream_t st);

// blocks used by the scan for n elements, and by the reduction
int64_t scan_blocks(int64_t n);
int reduce_max_blocks();

}  // namespace pic
