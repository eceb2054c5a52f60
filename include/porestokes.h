/*
 * porestokes.h -- C ABI of the MI355X (gfx950) pseudo-unsteady Stokes
 * permeability solver.
 *
 * Method (Krach, Ruf, Steeb, "POREMAPS", arXiv 2407.19868):
 *   - binary voxel image in, solid/pore (§5.1; here: nonzero byte = solid);
 *   - staggered MAC grid, face velocities u, v, w and cell pressure p (§4 "Grid");
 *   - no-slip / no-penetration at voxel faces touching solid (§4), second
 *     derivatives across the flow from the neighbourhood cases of App. B;
 *   - artificial-compressibility pseudo-time stepping of the nondimensional
 *     equations (§3, App. A), velocity then pressure each sweep (Algorithm 1);
 *   - drive: a mean pressure gradient G along the load axis, periodic
 *     fluctuation p~ (§4 "Simulation parametrization", Fig. 2);
 *   - Darcy: k_{i,j} = mu q_i / h_j from three load cases (§4 eq. darcy,
 *     eq. cases_pressure; App. C), off-diagonals averaged for k_sym (App. C).
 *
 * Conventions shared by every call
 *   Layout:     every 3-D array is [nz][ny][nx], x fastest, dense, no padding.
 *               u[c] is the x-face between cells c - e_x and c (likewise v, w);
 *               p[c] is the cell-centre pressure fluctuation p~.
 *               All domains are periodic on all three axes.
 *   Pointers:   "device" pointers are HIP device memory of the context's GPU
 *               (e.g. torch tensor data_ptr()); "host" pointers are CPU memory.
 *               The caller owns every pointer it passes; the library never
 *               frees them.  Device field pointers must be 8-byte aligned.
 *   Streams:    `stream` is a hipStream_t (NULL = default stream).  All device
 *               work of a call is ordered on it.  Calls that return numbers on
 *               the host (solve, tensor, batch, residual) synchronise that
 *               stream before returning; pm_preprocess and pm_face_codes only
 *               enqueue work.  pm_iterate returns after its sweeps are done
 *               (it releases its scratch buffers, which waits for the GPU).
 *   Errors:     every call returns pm_status.  Argument errors are detected
 *               before any device write.  The text of the last error is kept
 *               per context (pm_last_error).  No C++ exception crosses the ABI.
 *   Threads:    one context per host thread.
 *   Units:      fields are in the solver's nondimensional units: lengths in
 *               voxels, nu = 1/re, drive G (default 1 per voxel).  k is
 *               returned in physical units: k[vx^2] * voxel_size^2.  The
 *               viscosity mu cancels from k (the paper fixes Re); it only
 *               scales a physical velocity, v_phys = v * voxel_size^2 / (mu re)
 *               per unit applied pressure gradient.
 */
#ifndef PORESTOKES_H
#define PORESTOKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PM_OK = 0,             /* converged / success                                   */
    PM_ERR_ARG = 1,        /* invalid argument; nothing was written                 */
    PM_ERR_OOM = 2,        /* device allocation failed or exceeds the context cap   */
    PM_ERR_DEVICE = 3,     /* HIP runtime error                                     */
    PM_NOT_CONVERGED = 4,  /* max_sweeps reached; results are those of the last check */
    PM_DIVERGED = 5,       /* non-finite residual or r > 1e3 * min(r)               */
    PM_ERR_NO_FLOW = 6     /* no solid voxel, or no fluid face normal to the load axis */
} pm_status;

typedef enum {
    PM_FP64 = 0,    /* FP64 fields and arithmetic                                      */
    PM_FP32 = 1,    /* FP32 fields and arithmetic, FP64 reductions                     */
    PM_FP32_DC = 2  /* FP32 phase until the residual stalls at its rounding floor,
                       then an FP64 defect correction until tol (pm_params.dc_form:
                       FP32 sweeps of the correction, or FP64 sweeps).  An FP32
                       phase that meets the stop rule first (with stop_rule 1:
                       eps_q < tol at a check where r reached a new minimum)
                       hands over to FP64 sweeps, which must meet it again;
                       eps_q < tol at other checks ends the FP32 phase as the
                       floor does                                               */
} pm_precision;

typedef enum {
    PM_KERNEL_AUTO = 0,   /* fused kernel, tile from the autotuner / defaults         */
    PM_KERNEL_FUSED = 1,  /* one pass per sweep: pressure of sweep n and velocity of
                             sweep n+1 fused, LDS-staged tiles streamed along z       */
    PM_KERNEL_SIMPLE = 2  /* two passes per sweep (velocity, pressure), one thread per
                             cell, no LDS; the same per-face arithmetic               */
} pm_kernel;

/* Solver parameters.  pm_params_default fills the paper's values (§4). */
typedef struct {
    double re;          /* Reynolds number; nu = 1/re.          default 0.01 (§4)    */
    double c2;          /* artificial compressibility c*^2.     default 1.5e6 (§4)   */
    double dt;          /* pseudo-time step.                    default 2^-12        */
    double tol;         /* stop when r < tol (or eps_q < tol).  default 1e-8         */
    double drive;       /* mean pressure gradient G per voxel.  default 1 (§4)       */
    int64_t max_sweeps; /*                                      default 10^7         */
    int32_t check_every;/* residual check every M sweeps.       default 100          */
    int32_t precision;  /* pm_precision.                        default PM_FP64      */
    int32_t stop_rule;  /* 0: r < tol; 1: eps_q < tol (relative change of |q|
                           between checks, the paper's criterion §7.1)              */
    int32_t warm_start; /* 1: start from the fields passed in (else from rest)       */
    int32_t kernel;     /* pm_kernel.                           default AUTO         */
    int32_t tile_x;     /* fused-kernel tile override (0 = auto); (tile_x, tile_y)   */
    int32_t tile_y;     /* one of 128x8, 64x8, 64x16, 32x8, 32x16                   */
    int32_t zchunk;     /* planes per workgroup along z (0 = auto)                   */
    int32_t graphs;     /* 1: each block of check_every sweeps (plus its reduction
                           and copy-back) is captured once as HIP graphs (the
                           two-sweep launches, then the rest) and replayed; 0:
                           launched directly.                    default 1            */
    int32_t autotune;   /* 1: before solving, time the fused-kernel decompositions
                           on each new (shape, precision) and keep the fastest in
                           the context (see pm_autotune).        default 0            */
    int32_t progress;   /* > 0: every `progress` checks, print one line (sweeps,
                           active instances, largest residual) to stderr; for
                           long solves.                          default 0            */
    int32_t pore_cleanup; /* 1: before sweeping, the pore voxels of components that
                           do not wind around the domain along the load axis are
                           treated as solid (see pm_pores): they carry no flow at
                           the fixed point, so k is unchanged, and their slow
                           transients leave the residual.  An axis along which
                           nothing winds is PM_ERR_NO_FLOW without sweeps.  Fields
                           of the removed voxels are returned as 0.  default 0 */
    int32_t outer_walls;  /* bit i (1 << i): no-slip, no-penetration walls at both ends
                           of axis i instead of the periodic connection (§4 lists
                           such outer walls beside periodic ones).  Realised
                           exactly by sweeping the mask with one solid layer
                           appended along each wall axis: a wall lies half a voxel
                           beyond the first and the last layer, and every stencil
                           position beyond it is solid (so the App. B cases 7 and 8
                           never arise).  Fields are returned on the caller's grid;
                           k is the mean flux over the caller's voxels.  A load
                           axis with walls carries no through-flow: that solve is
                           PM_ERR_NO_FLOW without sweeps.  Solves only (pm_iterate
                           and pm_residual reject it).            default 0 */
    int32_t dc_form;    /* how PM_FP32_DC continues once the FP32 iterate s0 sits at
                           its rounding floor: 0 correction form: s0 is kept in
                           FP64, d0 = T(s0) - s0 is formed once by an FP64 sweep T
                           and stored in FP32, and FP32 sweeps iterate the
                           correction e <- A e + d0 (A: the sweep without the
                           drive; the fixed point is s* - s0) until s0 + e meets
                           the stop rule; if the correction reaches its own
                           rounding floor first, or the 16 B/voxel for d0 cannot be
                           allocated, s0 + e continues in FP64.  1: the FP32
                           iterate is promoted and FP64 sweeps continue.  default 0 */
    int32_t tblock;     /* sweeps per HBM pass of the fused kernel: 1, or 2 (temporal
                           blocking: two sweeps per read and write of the fields;
                           the first sweep of a solve, the sweep of each residual
                           check and the correction form run as single sweeps); 0:
                           the autotuned choice for the shape, else 1.  Results are
                           bitwise the same for every value.     default 0            */
    int32_t tile2_x;    /* two-sweep kernel output tile override (0 = auto);         */
    int32_t tile2_y;    /* (tile2_x, tile2_y) one of 64x10, 64x8, 64x6, 32x24, 32x12,
                           32x8                                                      */
    int32_t zchunk2;    /* planes per two-sweep workgroup along z (0 = auto)         */
    int32_t fixed_pressure; /* §4 (boundary conditions; Fig. 2 p_in, p_out): the
                           pressure is fixed along the drive while the flux stays
                           periodic.  1 holds p~ on the cell layer x_axis = 0 at
                           its starting value (0 from rest), so the pressure is
                           p_in there and p_out = p_in - G n one period later;
                           that layer's mass balance is not imposed and its
                           cells are left out of the residual's divergence sum.
                           0: p~ periodic and free everywhere.     default 0        */
    int32_t persistent; /* 1: small instances (both field sets and the codes within
                           3 MiB) run each block of check_every - 1 sweeps as one
                           persistent launch, instance j of up to 8 on XCD j, 32x16
                           tiles, at most 32 workgroups per instance, a barrier in
                           the XCD's L2 between sweeps (solves, tensors and batches;
                           results are bitwise the same).  On MI355X, against one
                           launch per sweep with 32x8 tiles and one-plane chunks,
                           it is no faster: 32^3 FP64 solve 7.0 against 5.4 us
                           per sweep, three 32^3 load cases 10.9 against
                           10.1-11.2 ms.  0: one launch per sweep.  default 0    */
} pm_params;

/* Residual history: one record per check.  Host arrays of length cap owned by
 * the caller (q has 3*cap entries); n is set to the number of records written
 * (at most cap; later records are dropped). */
typedef struct {
    int64_t cap;
    int64_t n;
    int64_t *sweep;  /* sweep count of the record                                  */
    double *resid;   /* r = sqrt(S_F + S_D) / (G sqrt(N_f))                         */
    double *eps_q;   /* | |q_n| - |q_prev| | / |q_n|  (inf at the first record)      */
    double *q;       /* mean face velocity q_x, q_y, q_z of the state (3 per record)  */
} pm_history;

typedef struct pm_ctx pm_ctx;

/* Fill *p with the defaults listed in pm_params. */
void pm_params_default(pm_params *p);

/* Text for a status code (static storage). */
const char *pm_status_string(pm_status s);

/* Create a context on HIP device `hip_device`.  mem_cap_bytes bounds the
 * context's own device allocations (0 = no bound); a call that would exceed
 * it returns PM_ERR_OOM.  *out receives the context. */
pm_status pm_create(int hip_device, size_t mem_cap_bytes, pm_ctx **out);

/* Free the context and its device scratch.  NULL is ignored. */
void pm_destroy(pm_ctx *ctx);

/* Device memory the library allocates for a call (stencil codes, the second
 * field set, partial sums) is not freed when the call returns: the context
 * keeps it for reuse by later calls, so that repeated solves of one size do
 * not map and unmap pages each time.  A request takes a kept block when one
 * is at most 1/8 larger.  Kept blocks count against mem_cap_bytes and are
 * returned to the device when an allocation would exceed the cap or fails,
 * by pm_trim, and by pm_destroy.  pm_trim returns them now (PM_ERR_ARG for a
 * NULL context). */
pm_status pm_trim(pm_ctx *ctx);

/* Message of the last error on this context ("" if none).  Valid until the next call. */
const char *pm_last_error(const pm_ctx *ctx);

/* Device bytes currently held by the context, kept blocks included. */
size_t pm_mem_used(const pm_ctx *ctx);

/*
 * Face flags ("Evaluate neighborhood", Algorithm 1; §4): a face is solid iff
 * either adjacent voxel is solid.  mask: device uint8 [nz][ny][nx].
 * bits: device uint32 [3][nz][ny][ceil(nx/32)]; plane k holds the k-faces,
 * bit b of word w is x = 32 w + b; padding bits are 0.
 */
pm_status pm_preprocess(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                        int64_t nz, uint32_t *bits);

/*
 * Per-cell stencil codes used by the sweep (App. B neighbourhood cases).
 * codes: device uint32 [nz][ny][nx].  For component k (bit offset 8 k):
 *   bits 0-2  code along the first perpendicular axis (x->y, y->x, z->x),
 *   bits 3-5  code along the second perpendicular axis (x->z, y->z, z->y),
 *   bit  6    face solid.
 * A 3-bit code is L | R<<1 | F<<2 with L / R = solid face at offset -1 / +1
 * (wall half a voxel away) and F = solid face at offset +2 (if only L) or -2
 * (if only R), i.e. a wall 3/2 voxels away.  Cases: none = 6, L = 4, R = 5,
 * L+F = 2, R+F = 3, L+R = 1.
 */
pm_status pm_face_codes(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                        int64_t nz, uint32_t *codes);

/*
 * Run exactly `count` sweeps on the state (u, v, w, p) in place, load axis
 * `axis` (0 x, 1 y, 2 z).  Fields are device arrays of nx*ny*nz doubles
 * (params->precision PM_FP64) or floats (PM_FP32); PM_FP32_DC is rejected.
 * Faces touching solid are set to 0 first.  Returns once the sweeps are
 * complete (the call's scratch buffers are freed on return).
 */
pm_status pm_iterate(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                     int64_t nz, int axis, const pm_params *params, void *u, void *v, void *w,
                     void *p, int64_t count);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pm_iterate
 * without any allocation.  Same arguments, checks and results as pm_iterate
 * (bitwise), for grids whose packed stencil codes (2 B per voxel) and second
 * field set (4 values per voxel in the call's precision) fit, with a 1 KiB
 * table, in PM_STATIC_SCRATCH_BYTES: up to about 1.97 M voxels in PM_FP64
 * (125^3) and 3.72 M in PM_FP32 (155^3).  Larger grids are rejected with PM_ERR_ARG before
 * any device work.  The scratch is one static device array per GPU, held from
 * the moment the library is loaded on that GPU until the process ends, and
 * shared by every call on it: calls on one GPU whose sweeps overlap in time
 * (different streams or threads) race on it and must be serialised by the
 * caller.  Every byte a call reads from it, the call writes first.  The call
 * returns once its sweeps are complete; pm_last_stats reports no timing for it.
 */
#define PM_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
pm_status pm_iterate_static(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                            int64_t nz, int axis, const pm_params *params, void *u, void *v, void *w,
                            void *p, int64_t count);

/*
 * Residual sums of a state, computed in FP64 on the GPU: out[0] = S_F (sum of
 * squared momentum residuals over fluid faces), out[1] = S_D (sum of squared
 * nu*div v over cells), out[2..4] = sums of u, v, w over all faces.  Fields as
 * in pm_iterate.  out is a host array of 5 doubles.  Synchronises the stream.
 */
pm_status pm_residual(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                      int64_t nz, int axis, const pm_params *params, const void *u,
                      const void *v, const void *w, const void *p, double out[5]);

/*
 * One load case (Algorithm 1; eq. cases_pressure): iterate from rest (or from
 * the given fields with warm_start) until the stop rule, with checks every
 * check_every sweeps.  Fields: device arrays of nx*ny*nz doubles (PM_FP64,
 * PM_FP32_DC) or floats (PM_FP32); on return they hold the state at the last
 * check.  hist: host, may be NULL.  k_col (host, 3 doubles): k_{i,axis} in
 * voxel_size^2 units, i = x, y, z.  sweeps_done (host, may be NULL).
 * Returns PM_OK, PM_NOT_CONVERGED, PM_DIVERGED, PM_ERR_NO_FLOW or an error.
 */
pm_status pm_solve(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                   int64_t nz, double voxel_size, double mu, int axis, const pm_params *params,
                   void *u, void *v, void *w, void *p, pm_history *hist, double k_col[3],
                   int64_t *sweeps_done);

/*
 * Full tensor (§2 eq. 3dK; App. C): the three load cases x, y, z solved as one
 * batch when their device buffers fit beside each other (within the context
 * cap and the device's free memory), else one after another; each load case
 * gives the same result either way (pm_stats.tensor_cases_at_once tells which
 * ran).  k (host, 9 doubles, row-major k[i*3+j] = k_ij, column j from load
 * axis j) and k_sym = (k + k^T)/2 (host, 9).  hist: host array of 3 histories
 * or NULL.  sweeps: host array of 3 or NULL.  Fields are kept internally.
 */
pm_status pm_tensor(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                    int64_t nz, double voxel_size, double mu, const pm_params *params,
                    double k[9], double k_sym[9], pm_history *hist, int64_t sweeps[3]);

/* One instance of a batch: a (mask, load axis) solve. */
typedef struct {
    const uint8_t *mask;   /* device uint8 [nz][ny][nx]                              */
    int64_t nx, ny, nz;
    double voxel_size, mu;
    int32_t axis;
    int32_t pad;
    void *u, *v, *w, *p;   /* device fields (as in pm_solve), or all NULL: internal  */
    pm_history *hist;      /* host, may be NULL                                      */
    double k_col[3];       /* out                                                    */
    int64_t sweeps;        /* out                                                    */
    int32_t status;        /* out: pm_status of this instance                        */
    int32_t pad2;
} pm_instance;

/*
 * Batched solves (many masks of uneven sizes and load axes, e.g. clogging or
 * compression series and the three load cases of each): every sweep of all
 * active instances is one launch; an instance that meets its stop rule stops
 * being swept while the others continue.  Each instance gets its own status;
 * the call returns the worst one (error > DIVERGED > NO_FLOW > NOT_CONVERGED > OK).
 */
pm_status pm_solve_batch(pm_ctx *ctx, void *stream, pm_instance *inst, int32_t n,
                         const pm_params *params);

/*
 * Autotuner: time the fused sweep for each supported decomposition on this
 * mask and precision (PM_FP64 or PM_FP32), from rest: the single-step tiles
 * (128x8, 64x8, 32x8, 32x16, 64x16) with z-chunks of 16..128 planes, and the
 * two-step kernel (two sweeps per pass, pm_params.tblock) with output tiles
 * 64x10, 64x8, 64x6, 32x24, 32x12, 32x8 and its z-chunks, each priced per sweep.  The
 * fastest choice is kept for the shape (nx, ny, nz) in the context; later
 * solves of that shape use it unless params fix a tile or tblock.  If the
 * environment variable PORESTOKES_TUNE_CACHE names a file, choices are loaded
 * from it at pm_create and written back here (a flat JSON object
 * "NXxNYxNZ:f64" -> [tile_x, tile_y, zchunk, tblock, tile2_x, tile2_y, zchunk2]).
 * best (host, 7 ints, may be NULL) receives the choice in that order.
 * Synchronises the stream.
 */
pm_status pm_autotune(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny,
                      int64_t nz, int precision, int32_t best[7]);

/* Timing of the sweep kernels of the last pm_iterate / pm_solve / pm_tensor /
 * pm_solve_batch call on a context, measured with HIP events recorded on the
 * call's stream around each run of consecutive sweep launches (in a solve: a
 * block of check_every sweeps plus its final reduction and 40-byte copy-back
 * per instance). */
typedef struct {
    int64_t sweep_launches;  /* sweep-kernel launches                                  */
    int64_t voxel_updates;   /* voxels swept, summed over launches (all instances)     */
    double sweep_ms;         /* GPU time spanned by those launches                     */
    double total_ms;         /* host wall time of the call                             */
    int32_t tile_x, tile_y, zchunk;  /* decomposition of the last instance             */
    int32_t precision;       /* pm_precision of the last sweep launch (PM_FP64/PM_FP32) */
    int64_t peak_bytes;      /* most device memory the call had in use at once (the
                                library's own allocations, not the caller's buffers,
                                not blocks kept idle for later calls)                    */
    int32_t tblock;          /* sweeps per pass of the last sweep launch (pm_params.tblock) */
    int32_t tensor_cases_at_once; /* pm_tensor: 3 when the three load cases ran as one
                                batch, 1 when they did not fit beside each other and
                                ran one after another (then the counts and times are
                                summed over the three calls); 0 for other calls         */
    int32_t dc_promoted_for_memory; /* PM_FP32_DC instances whose correction form could
                                not allocate its defect field and continued as FP64
                                sweeps instead (dc_form 1 behaviour)                     */
    int32_t reserved;
    int64_t t2_launches;     /* two-step launches among sweep_launches (tblock 2)         */
    int64_t t2_voxels;       /* voxels those launches passed over (each advanced 2 sweeps) */
    double t2_ms;            /* GPU time spanned by the runs of consecutive two-step launches
                                (HIP events on the call's stream)                         */
    int64_t pers_launches;   /* persistent launches among sweep_launches (pm_params.persistent) */
    int64_t pers_sweeps;     /* instance-sweeps done inside them                          */
} pm_stats;

/* Copy the statistics of the last call into *out (host). */
pm_status pm_last_stats(const pm_ctx *ctx, pm_stats *out);

/*
 * Mirroring (§5.1 pre-processing, which mirrors a sample to make it periodic;
 * the mirrored samples of §7.1): the sample followed by its mirror image along every
 * axis i with bit i of `axes`, so that the periodic cell is continuous across
 * its boundaries.  out: device uint8 [mz][my][mx], m_i = 2 n_i for mirrored axes,
 * n_i otherwise; out at coordinate c >= n_i equals the sample at 2 n_i - 1 - c.
 * Only enqueues work.  Errors: PM_ERR_ARG (NULL pointers, axes outside 0..7,
 * dims too large after doubling).
 */
pm_status pm_mirror(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int axes,
                    uint8_t *out);

/* ------------------------------------------------------------ pore space
 *
 * Connectivity of the pore space (§5.1: pre-processing removes disconnected
 * pore space; the solver assumes percolation).  Pore voxels (mask byte 0) are
 * connected through shared faces, across the periodic boundaries too.  A
 * component percolates along axis j when it holds a closed path that winds
 * around the domain along j (in the periodically repeated space it reaches a
 * copy of its start shifted along j).  Only such components carry flow under
 * a drive along j: in any other, p = G x_j balances the drive with v = 0.
 */
typedef struct {
    int64_t n_pore;                   /* pore voxels                                    */
    int64_t n_components;             /* pore components                                */
    int32_t percolates[3];            /* axis j: some component winds along j           */
    int32_t reserved;
    int64_t n_flowing[3];             /* pore voxels of components winding along j      */
    int64_t n_flowing_components[3];  /* components winding along j                     */
} pm_pore_info;

/*
 * mask: device uint8 [nz][ny][nx].  labels: device int64 [nz][ny][nx] or NULL;
 * receives for each pore voxel the smallest linear index of its component, -1
 * for solid voxels.  flow: device uint8 [nz][ny][nx] or NULL; bit j (value
 * 1 << j) set for pore voxels of components winding along j, 0 elsewhere.
 * info: host, required.  Scratch: about 17 bytes per voxel.  Synchronises the
 * stream.  Errors: PM_ERR_ARG (NULL mask or info, bad dims, misaligned labels),
 * PM_ERR_OOM, PM_ERR_DEVICE.
 */
pm_status pm_pores(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                   int64_t *labels, uint8_t *flow, pm_pore_info *info);

/* ------------------------------------------------------------ principal axes
 *
 * Post-processing of a permeability tensor (host computation, no context, no
 * GPU).  The principal permeabilities are the eigenvalues of the symmetric
 * part k_sym = (k + k^T)/2 (the off-diagonals averaged as in App. C; §2
 * eq. 3dK_eigen), the principal axes its unit eigenvectors, and the material
 * class follows §2 from which of them are equal.
 */
typedef enum { PM_ISOTROPIC = 0, PM_TRANSVERSE = 1, PM_ORTHOTROPIC = 2 } pm_aniso_class;

typedef struct {
    double k_sym[9];   /* (k + k^T) / 2, row-major                                    */
    double lambda[3];  /* principal permeabilities k_I <= k_II <= k_III                */
    double R[9];       /* rotation tensor, row-major, R[k*3+i] = cos(e_k, e~_i): column
                          i is the unit principal axis of lambda[i].  Columns 0 and 1
                          have their largest-magnitude component positive, column 2 =
                          column 0 x column 1 (det R = +1).  Axes of equal values are
                          any orthonormal basis of their eigenspace.                 */
    int32_t cls;       /* pm_aniso_class                                               */
    int32_t distinct;  /* PM_TRANSVERSE: index (0..2) into lambda of the value that
                          differs from the equal pair; -1 otherwise                    */
    double ratio;      /* anisotropy ratio k_III / k_I (+inf when k_I <= 0)           */
} pm_principal;

/*
 * k: host, 9 doubles, row-major k[i*3+j] = k_ij (as pm_tensor returns).
 * Two principal values a, b count as equal when |a - b| <= rel_tol * max(|a|, |b|)
 * (the paper's classes are exact equalities; rel_tol >= 0 sets the resolution).
 * Class: PM_ISOTROPIC if k_I and k_III are equal; else PM_TRANSVERSE if k_I = k_II
 * or k_II = k_III (both: the pair with the smaller relative gap); else
 * PM_ORTHOTROPIC.  Errors: PM_ERR_ARG for NULL pointers, a negative or non-finite
 * rel_tol or a non-finite entry of k.
 */
pm_status pm_principal_axes(const double k[9], double rel_tol, pm_principal *out);

/*
 * Principal directions within the plane of axes a and b (a != b, 0..2), the
 * reduced two-dimensional evaluation of §6.4: with s = (k_ab + k_ba) / 2,
 *   phi = atan2(2 s, k_bb - k_aa) / 2   (radians, in (-pi/2, pi/2]),
 * so that sin(phi) e_a + cos(phi) e_b is the principal axis of the larger value
 * lam[1] of the 2x2 block [[k_aa, s], [s, k_bb]]: the angle between e_b and that
 * axis.  For k_bb > k_aa this is (1/2) arctan(2 s / (k_bb - k_aa)), §6.4's formula
 * read with the difference of the diagonal entries in the denominator.  lam (host, 2): eigenvalues of the
 * block, lam[0] <= lam[1].  Errors: PM_ERR_ARG for NULL pointers, bad or equal
 * axes, non-finite entries.
 */
pm_status pm_plane_angle(const double k[9], int a, int b, double *phi, double lam[2]);

#ifdef __cplusplus
}
#endif

#endif /* PORESTOKES_H */
