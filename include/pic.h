/*
 * pic355 — electromagnetic particle-in-cell time step for MI355X (gfx950).
 *
 * C ABI of the hot path.  The operations follow the paper's statement of the
 * PIC problem ("Porting WarpX to GPU-accelerated platforms", arXiv
 * 2101.12149): relativistic charged macro-particles coupled to Maxwell's
 * equations (Sec. 1); one particle container per species holding per-particle
 * arrays (Sec. 2.2); field components on the Yee staggering, B on cell faces
 * and E, J on cell edges (Sec. 2.4); and the particle operations field
 * gathering, particle pushing and current deposition (Sec. 2.2), with the
 * Yee FDTD solver, Esirkepov deposition and third-order shapes (Sec. 4.1.1),
 * energy-conserving gathering (Sec. 4.2) and particle binning / sorting by a
 * counting sort (Sec. 3.4.2).
 *
 * Conventions shared by every entry point
 *   - Every array pointer is a DEVICE pointer owned by the caller.  Structs
 *     are host memory and are only read during the call.  The library never
 *     keeps a pointer after returning and never allocates device memory.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream), except where a status has to be read back: pic_sort_tiles,
 *     pic_gather, pic_push, pic_deposit, pic_step and pic_step_adjoint read a
 *     device error word at their end and so synchronise the stream.
 *   - Grid: n[3] cells, periodic in all three directions, spacing d[3].
 *     Field arrays hold n0*n1*n2 values, x fastest: index i + n0*(j + n1*k).
 *     Staggering of element [i,j,k] (in cells):
 *       E_x, J_x (i+1/2, j, k)   E_y, J_y (i, j+1/2, k)   E_z, J_z (i, j, k+1/2)
 *       B_x (i, j+1/2, k+1/2)    B_y (i+1/2, j, k+1/2)    B_z (i+1/2, j+1/2, k)
 *   - Particle position in cell units x/d = cell + off with cell an int32 in
 *     [0, n) and off in [0, 1) of the grid dtype (split precision).  u = gamma v.
 *   - dtype PIC_F32: fields, offsets, momenta, weights and source map are
 *     float; PIC_F64: double.  Energy/charge reductions are always FP64.
 *   - State at step n is (x^n, u^{n-1/2}, E^n, B^n).
 *
 * Errors: every argument check is synchronous and runs before any launch; on
 * a non-OK status from these checks no output has been touched.  Corrupt
 * particle state is found on the device (a cell outside [0,n), an offset
 * outside [0,1), a non-finite momentum, a displacement of a cell or more in
 * one step): the calls that read the error word back return PIC_E_STATE
 * after their kernels ran, the offending particles left unchanged (or, in
 * pic_deposit, their current left out) and the others processed.
 * pic_gather, pic_push and pic_deposit have no workspace and share one error
 * word per device: two of these calls that overlap on one device (other
 * streams or host threads) may report each other's state errors.
 * pic_last_error() returns a thread-local message.  No C++ exception crosses
 * this ABI.
 */
#ifndef PIC355_PIC_H
#define PIC355_PIC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define PIC_API __attribute__((visibility("default")))
#else
#define PIC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIC_OK = 0,
    PIC_E_INVALID = 1,     /* null pointer, bad size, inconsistent argument */
    PIC_E_CFL = 2,         /* c dt beyond the solver's stability limit */
    PIC_E_UNSUPPORTED = 3, /* order not in {1,3}, dtype unknown, tile too big */
    PIC_E_WORKSPACE = 4,   /* workspace missing or smaller than pic_workspace_bytes */
    PIC_E_STATE = 5,       /* corrupt particle state found on the device */
    PIC_E_DEVICE = 6       /* a HIP call failed */
} pic_status;

typedef enum { PIC_F32 = 0, PIC_F64 = 1 } pic_dtype;

/* Momentum update of the particle push.
 *   PIC_PUSH_BORIS  relativistic Boris rotation: half electric kick, magnetic
 *                   rotation, half electric kick.
 *   PIC_PUSH_VAY    Vay's pusher (J.-L. Vay, Phys. Plasmas 15, 056701, 2008),
 *                   which the paper runs for relativistic beams (Sec. 4.2): the
 *                   magnetic force takes the mean of the old and new velocity,
 *                   u1 - u0 = (q dt/m) E + (q dt/2m) (u0/g0 + u1/g1) x B,
 *                   solved in closed form; a particle in crossed fields with
 *                   E + v x B = 0 keeps its momentum exactly.
 * Both are followed by the same position update with gamma(u1). */
typedef enum { PIC_PUSH_BORIS = 0, PIC_PUSH_VAY = 1 } pic_pusher;

/* Field solver of the leapfrog step.
 *   PIC_SOLVER_YEE  Yee's FDTD (Sec. 4.1.1); stable for c dt <= 1/sqrt(sum 1/d^2).
 *   PIC_SOLVER_CKC  Cole-Karkkainen-Cowan FDTD, the paper's solver for the
 *                   accelerator stage (Sec. 4.2): the E update keeps Yee's
 *                   differences, the B update averages each difference along
 *                   axis a over its transverse neighbours with weights alpha_a
 *                   (centre), beta_ap, beta_aq (edges), gamma_a (corners); with
 *                   delta = min d, r_a = (delta/d_a)^2, S = sum of r_a r_b (a<b):
 *                   beta = (1 - r_x r_y r_z/S)/8, beta_ap = r_p beta,
 *                   gamma_a = r_p r_q (1/16 - r_p r_q/(8S)),
 *                   alpha_a = 1 - 2 beta_ap - 2 beta_aq - 4 gamma_a
 *                   (7/12, 1/12, 1/48 for cubic cells); stable for c dt <= delta. */
typedef enum { PIC_SOLVER_YEE = 0, PIC_SOLVER_CKC = 1 } pic_solver;

typedef struct {
    int32_t n[3];     /* cells per direction (periodic) */
    double d[3];      /* cell size */
    double dt;        /* time step */
    double c;         /* speed of light */
    double eps0;      /* vacuum permittivity; mu0 = 1/(eps0 c^2) */
    int32_t order;    /* shape-function order: 1 (cloud in cell) or 3 (cubic) */
    int32_t dtype;    /* pic_dtype */
    int32_t tile[3];  /* sort/tile size in cells, each in [1,16] dividing n;
                         0 = automatic: the largest divisor of n not above 8,
                         halved (not below 4) while the tile's LDS regions do
                         not fit or the grid holds fewer than 512 tiles */
    int32_t slack;    /* cells of halo slack around a tile for particles that
                         drifted since the last sort; -1 = automatic */
    int32_t pusher;   /* pic_pusher; anything else is PIC_E_UNSUPPORTED */
    int32_t solver;   /* pic_solver; anything else is PIC_E_UNSUPPORTED */
    const double *gather_filter; /* NULL, or HOST double[6][4]: a filter of the
                         fields before the gather (the place of the paper's
                         Godfrey filter, Sec. 4.2), see below */
} pic_grid;
/* Gather filter.  With gather_filter != NULL, pic_step and pic_step_adjoint
 * gather E and B through a symmetric stencil along z, per component m
 * (E_x, E_y, E_z, B_x, B_y, B_z), w = gather_filter + 4 m:
 *   F~(i,j,k) = w[0] F(i,j,k) + sum_{s=1..3} w[s] (F(i,j,k+s) + F(i,j,k-s)),
 * periodic; the fields themselves are not changed, and the adjoint adds the
 * filter's transpose (itself) of the gathered-field adjoints to lam->lE,
 * lam->lB.  The taps are the caller's (Godfrey's tables, a binomial filter,
 * ...); they must be finite.  The filtered fields and their adjoints take six
 * more field arrays each in the workspace.  pic_gather has no workspace and
 * refuses a grid with a filter (PIC_E_UNSUPPORTED). */

typedef struct {
    int64_t n;          /* number of particles */
    int32_t *cell[3];   /* int32[n] cell index per direction */
    void *off[3];       /* T[n] in-cell offset in [0,1) */
    void *u[3];         /* T[n] momentum per mass, gamma v */
    void *w;            /* T[n] weights, or NULL for the constant w0 (sorted
                           along with the other arrays) */
    double w0;          /* weight used when w == NULL */
    double q, m;        /* charge and mass of one physical particle */
} pic_species;

typedef struct {
    void *E[3], *B[3], *J[3];   /* T[n0*n1*n2] each */
} pic_fields;

typedef struct {
    int32_t k_plane;    /* < 0: no source */
    const void *amp;    /* T[n0*n1] device map, x fastest */
    const double *g;    /* HOST double[n_g]; g[step] multiplies the map */
    int64_t n_g;        /* steps outside [0, n_g) use g = 0 */
} pic_source;
/* A soft source: after the E update of step `step`,
 * E_x[i, j, k_plane] += amp[i + n0*j] * g[step].  The paper's laser stage
 * (Sec. 4.2) injects a laser; this plane source is the periodic-box stand-in. */

typedef struct {
    void *lx[3];   /* T[n] dL/d(position in cell units) */
    void *lu[3];   /* T[n] dL/du */
    void *lE[3];   /* T[n0*n1*n2] dL/dE */
    void *lB[3];   /* T[n0*n1*n2] dL/dB */
} pic_adjoint;

/* Bytes of device workspace needed by pic_sort_tiles, pic_step,
 * pic_step_adjoint and pic_reduce for this grid and particle count. */
PIC_API size_t pic_workspace_bytes(const pic_grid *grid, int64_t n_particles);

/* Number of tiles the library uses for this grid (the length of tile_start
 * is this plus one); 0 if the grid is invalid.  With tile[d] == 0 the tile
 * edge starts at 8 and is halved until the LDS regions fit one workgroup. */
PIC_API int64_t pic_tile_count(const pic_grid *grid);

/* The tile edge in cells per direction (tile[3]) and the slack in cells
 * (*slack) that the library uses for this grid, resolving the automatic
 * choices of pic_grid.tile and pic_grid.slack.  Tile t of tile_start covers
 * the cells tile[d] * (t_x, t_y, t_z) onwards, t = t_x + nx (t_y + ny t_z)
 * with n[d] / tile[d] tiles per direction.  Host-only. */
PIC_API pic_status pic_tile_shape(const pic_grid *grid, int32_t *tile, int32_t *slack);

/* Particle binning and sorting by counting sort (Sec. 3.4.2: binning computes
 * a permutation that assigns particles to bins; sorting reorders the data).
 * Bins are cells grouped by tile: tiles of grid->tile cells in lexicographic
 * (x fastest) order.  Inside a tile the order is rank-major: the first
 * particle of every non-empty cell (cells x fastest), then the second
 * particle of every cell holding two or more, and so on, so that consecutive
 * particles sit in neighbouring cells.  Which particle of a cell counts as
 * first is not specified.  Reorders every array of `sp` in place, writes tile_start[t] = first particle of tile t for
 * t in [0, ntiles] (tile_start[ntiles] = n), and, if perm != NULL,
 * perm[j] = index before the sort of the particle now at j.
 * tile_start: int32[ntiles+1] device.  perm: int32[n] device or NULL.
 * Particles with a cell outside [0,n) or an offset outside [0,1) make the
 * call return PIC_E_STATE (this call synchronises the stream to read it). */
PIC_API pic_status pic_sort_tiles(const pic_grid *grid, pic_species *sp, int32_t *tile_start, int32_t *perm,
                          void *ws, size_t ws_bytes, void *stream);

/* Field gather (Sec. 3.1, Sec. 4.2): E and B at every particle, each
 * component interpolated from its own staggered location with the
 * order-`order` B-spline in all three directions.  Ep, Bp: T[n] x 3 outputs
 * (zero for a particle with a corrupt cell or offset, and PIC_E_STATE).
 * Synchronises the stream to read the device error word. */
PIC_API pic_status pic_gather(const pic_grid *grid, const pic_species *sp, const pic_fields *f, void *const Ep[3],
                      void *const Bp[3], void *stream);

/* Relativistic Boris (or Vay, per grid->pusher) push u^{n-1/2} -> u^{n+1/2}
 * with the given per-particle fields, then the position update
 * x += dt u/gamma with periodic wrap.  A particle with corrupt state or a
 * displacement of a cell or more is left unchanged (PIC_E_STATE).
 * Synchronises the stream to read the device error word. */
PIC_API pic_status pic_push(const pic_grid *grid, pic_species *sp, void *const Ep[3], void *const Bp[3], void *stream);

/* Esirkepov charge-conserving current deposition (Sec. 3.4.1, 4.1.1):
 * J += current of the particles moving from `before` to `after` (same n,
 * same order of particles, displacement below one cell per direction).
 * A particle with corrupt state in either, or that moved more than one cell
 * along an axis, deposits nothing (PIC_E_STATE).  Synchronises the stream to
 * read the device error word. */
PIC_API pic_status pic_deposit(const pic_grid *grid, const pic_species *before, const pic_species *after, pic_fields *f,
                       void *stream);

/* One Yee FDTD step (Sec. 2.4, 4.1.1): B -= dt/2 curl E; E += dt (c^2 curl B
 * - J/eps0); source; B -= dt/2 curl E.  J is read, not modified. */
PIC_API pic_status pic_yee(const pic_grid *grid, pic_fields *f, const pic_source *src, int64_t step, void *stream);

/* nsteps full PIC steps from step index step0: [sort] -> gather + Boris push
 * + position update + Esirkepov deposit (one fused tile kernel, Sec. 3.1) ->
 * Yee update.  Sorting happens before the first step of the call and before
 * every step whose index is a multiple of sort_every when sort_every > 0;
 * with sort_every == 0 the binning already in tile_start is used (it must
 * run from 0 to n, else PIC_E_INVALID; particles that left their tile since
 * take the stray path), and with tile_start == NULL as well the particles are
 * processed without tiles.
 * On return J holds the current of the last step.  diag (optional, device
 * double[nsteps][5]) receives pic_reduce's five values after every step.
 * Synchronises the stream at the end to read the device error word. */
PIC_API pic_status pic_step(const pic_grid *grid, pic_species *sp, pic_fields *f, const pic_source *src, int64_t step0,
                    int32_t nsteps, int32_t sort_every, int32_t *tile_start, void *ws, size_t ws_bytes,
                    double *diag, void *stream);

/* Bytes of the static scratch array pic_step_noalloc uses in place of a
 * workspace (one per device, held until the process ends). */
#define PIC_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* pic_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, checks, kernels and results as pic_step without ws and
 * ws_bytes.  Its scratch is a static device array of
 * PIC_NOALLOC_SCRATCH_BYTES per device (128 MiB: enough for
 * pic_workspace_bytes of a 64^3 grid with 4 particles per cell in FP64);
 * a grid and particle count that need more return PIC_E_WORKSPACE before
 * anything is launched.  The call allocates nothing, neither device memory
 * nor timing events (pic_timing does not see it); the device address of the
 * array is looked up once per device, on the first call with that device
 * current.  Every call on one device shares that device's array, which keeps
 * the last call's contents (the call clears what it needs): calls that
 * overlap on one device, from other streams or host threads, race and give
 * wrong results.  Like pic_step it synchronises the stream at the end. */
PIC_API pic_status pic_step_noalloc(const pic_grid *grid, pic_species *sp, pic_fields *f, const pic_source *src,
                                   int64_t step0, int32_t nsteps, int32_t sort_every, int32_t *tile_start,
                                   double *diag, void *stream);

/* Hand-written adjoint of step `step`: state_n / fields_n are the inputs of
 * that forward step (no sort in between); lam holds dL/d(state n+1) on entry
 * and dL/d(state n) on return; dA (device double[n0*n1], or NULL) accumulates
 * dL/d(source map).  Field part: transpose of the Yee step (the periodic
 * forward difference is minus the transpose of the backward one).  Particle
 * part: transpose of the deposit (a gather of the current adjoint), of the
 * position update, of the Boris push and of the gather (a scatter).
 * tile_start (int32[ntiles+1], or NULL): a binning of state_n's particles
 * from pic_sort_tiles or pic_step (running from 0 to n, else
 * PIC_E_INVALID, found on the device and returned at the end of the call:
 * lam and dA are then unspecified); with it the particle part runs one
 * workgroup per tile with the fields, the field adjoint and the scatter
 * accumulators in LDS, without it one thread per particle on global memory.
 * The result does not depend on the choice beyond rounding. */
PIC_API pic_status pic_step_adjoint(const pic_grid *grid, const pic_species *state_n, const pic_fields *fields_n,
                                    const int32_t *tile_start, const pic_source *src, int64_t step,
                                    pic_adjoint *lam, double *dA, void *ws, size_t ws_bytes, void *stream);

/* Field-energy loss and the seed of the reverse sweep: out[0] (device double)
 * receives L = U_E + U_B (pic_reduce's out[0] + out[1]); lam->lE = s eps0 dV E,
 * lam->lB = s dV B / mu0 (the gradient of s L), and lam->lx, lam->lu are
 * zeroed for n_particles particles.  s scales the seed (the incoming
 * gradient of a composite loss).  Needs the workspace. */
PIC_API pic_status pic_energy_loss(const pic_grid *grid, const pic_fields *f, int64_t n_particles, double s,
                                   pic_adjoint *lam, double *out, void *ws, size_t ws_bytes, void *stream);

/* FP64 reductions (Sec. 2.6): out[0] = dV/2 sum eps0|E|^2,
 * out[1] = dV/2 sum |B|^2/mu0, out[2] = sum w m c^2 (gamma-1),
 * out[3] = sum q w, out[4] = sum w m u_z.  sp may be NULL (out[2..4] = 0).
 * out: device double[5].  Needs the workspace. */
PIC_API pic_status pic_reduce(const pic_grid *grid, const pic_species *sp, const pic_fields *f, double *out, void *ws,
                      size_t ws_bytes, void *stream);

/* Gauss-law residual, a diagnostic of charge conservation (Sec. 2.6
 * reductions, FP64): the species' charge density at the nodes with the
 * order-`order` B-spline, rho(i,j,k) = sum_p q w_p S(x-i) S(y-j) S(z-k) / dV,
 * accumulated in FP64 (shape weights evaluated in FP64 from the offsets),
 * plus the immobile neutralising background -(sum_p q w_p)/(ncell dV); the
 * divergence of E at the nodes with the backward differences that take
 * edge fields to nodes, div E(i,j,k) = sum_d (E_d[i,j,k] - E_d[.. - 1 along
 * d]) / d_d (periodic).  out (device double[3]):
 *   out[0] = sqrt(sum over nodes (div E - rho/eps0)^2),
 *   out[1] = sqrt(sum over nodes (rho/eps0)^2)  (rho with the background),
 *   out[2] = sum over nodes rho dV (the species' charge).
 * With Esirkepov's deposit and the Yee update the residual field does not
 * change from step to step beyond rounding (no Poisson solve is needed).
 * The deposit uses per-particle global atomics (a diagnostic, not the hot
 * path).  Needs the workspace; a particle with a cell outside [0,n) or an
 * offset outside [0,1) is left out and the call returns PIC_E_STATE (it
 * synchronises the stream to read the error word). */
PIC_API pic_status pic_gauss_residual(const pic_grid *grid, const pic_species *sp, const pic_fields *f, double *out,
                                      void *ws, size_t ws_bytes, void *stream);

/* Kernel timing with HIP events recorded on the caller's stream around the
 * launches of pic_step and pic_step_adjoint, by category:
 *   0 sort (binning + scan + scatter)   1 fused particle (tile) kernel
 *   2 Yee field update                  3 FP64 reductions
 *   4 adjoint field transposes          5 adjoint particle kernels
 *   6 particles outside their tile's region (stray kernel)
 * Completes the pending measurements (synchronising on their events),
 * writes the accumulated milliseconds and launch counts of the first n
 * categories to ms / count (either may be NULL), resets the accumulators and
 * then turns timing on (enable != 0) or off.  Off by default. */
PIC_API pic_status pic_timing(int enable, double *ms, int64_t *count, int n);

/* Message for the last non-OK status of the calling thread. */
PIC_API const char *pic_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PIC355_PIC_H */
