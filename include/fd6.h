/*
 * fd6.h -- C ABI of the MI355X (gfx950) library for the per-substep kernel of
 * a sixth-order finite-difference solver for isothermal compressible
 * hydrodynamics (Pekkila, Vaisala, Kapyla, Kapyla, Anjum 2017, "Methods for
 * compressible fluid simulation on GPUs using high-order finite differences").
 *
 * What one step computes (paper section / equation / algorithm):
 *   state        lnrho, ux, uy, uz on an nx*ny*nz periodic grid with a ghost
 *                zone of R = 3 cells (Sec. 2.3, Sec. 4)
 *   right-hand   D lnrho/Dt = -div u                          eq. continuity
 *   side         D u/Dt = -cs^2 grad lnrho + nu (lap u + (1/3) grad div u
 *                         + 2 S . grad lnrho), f = 0          eq. navierstokes
 *                S_ij = (d_j u_i + d_i u_j)/2 - (1/3) delta_ij div u  eq. tensor
 *   derivatives  sixth-order central first, second and bidiagonal mixed
 *                differences, eqs. first_derivatives, second_derivatives
 *                (prefactor 1/(180 dx^2)), mixed_derivatives (Sec. 2.3); the
 *                19-point variant forms grad div u as D1 of the divergence
 *                field (eq. 19-point_mixed_derivatives, Sec. 4.2, Appendix A)
 *   time step    2N-storage RK3, eq. 2N-RK_scheme (Sec. 2.4), substeps as in
 *                Algorithm 2 (55 points) or Algorithm 3 (19 points), with the
 *                Williamson coefficients alpha = (0, -5/9, -153/128),
 *                beta = (1/3, 15/16, 8/15)
 *
 * Conventions for every entry point
 *   - Return value: FD6_OK (0) or a negative fd6_status.  No C++ exception
 *     crosses this boundary.  An argument error (FD6_EINVAL) leaves the
 *     handle unchanged.  After FD6_EHIP, fd6_last_error() holds the HIP text.
 *   - Host field arrays are compact FP64, nx*ny*nz values, C order [z][y][x]
 *     (x fastest).  "_device" variants take device pointers with the same
 *     layout; they are read or written on the handle's stream.
 *   - Device memory: the caller allocates one workspace of
 *     fd6_workspace_bytes() bytes, 256-byte aligned, and keeps it alive until
 *     fd6_destroy().  The library borrows it and allocates no device memory.
 *   - Streams: work is enqueued on the hipStream_t given at creation (or by
 *     fd6_set_stream); NULL means the default stream.  fd6_rk3_step is
 *     asynchronous; calls that return host data synchronise the stream.
 *   - Handles are not thread-safe; distinct handles are independent.
 */
#ifndef FD6_H
#define FD6_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FD6_ABI_VERSION 1

typedef enum {
    FD6_OK = 0,
    FD6_EINVAL = -1,       /* bad argument (null pointer, size, parameter) */
    FD6_ESTATE = -2,       /* step/get/reduce before set_params + init_fields */
    FD6_ENOMEM = -3,       /* workspace smaller than fd6_workspace_bytes() */
    FD6_EHIP = -4,         /* a HIP call failed; see fd6_last_error() */
    FD6_ENONFINITE = -5,   /* fd6_reduce found NaN or Inf in the state */
    FD6_EUNSUPPORTED = -6  /* valid but not implemented combination */
} fd6_status;

/* Storage and arithmetic precision of the state (Sec. 5 compares single and
 * double precision).  FD6_FP32_ACC64 stores the state in FP32 and keeps the
 * RK3 register w and the RK3 update arithmetic in FP64. */
typedef enum { FD6_FP64 = 0, FD6_FP32 = 1, FD6_FP32_ACC64 = 2 } fd6_precision;

/* Discretisation: 55-point single pass (Sec. 4.1, Algorithm 2) or 19-point
 * two pass (Sec. 4.2, Algorithm 3). */
typedef enum { FD6_55P = 0, FD6_19P = 1 } fd6_variant;

/* Device layout of the state and of the RK3 register (fd6_desc.flags).
 * Default (0): one array per field.  FD6_LAYOUT_AOS: the four values of a grid
 * point adjacent (array of structures, the alternative Sec. 7 proposes to
 * save the partial memory segments of the x halos), so the sweep kernels move
 * each point with 16-byte accesses.  Results are bit for bit those of the
 * default layout.  The layout is internal: host and device field arrays at
 * this boundary keep the compact per-field layout either way.  Supported for
 * the 55-point method and the z-sweep shapes whose loader goes through
 * registers (fd6_set_tile and fd6_batch_set_schedule return FD6_EUNSUPPORTED
 * for the others); an ensemble takes one layout for all its boxes. */
#define FD6_LAYOUT_AOS 1

typedef struct {
    int32_t nx, ny, nz;  /* interior points, 6 <= n <= 4096 each */
    int32_t precision;   /* fd6_precision */
    int32_t variant;     /* fd6_variant */
    int32_t flags;       /* 0 or FD6_LAYOUT_AOS */
} fd6_desc;

/* Physical and numerical parameters: viscosity nu >= 0, sound speed cs >= 0,
 * grid spacings dx, dy, dz > 0 (delta_i = L_i / N_i, Sec. 2.3), time step
 * dt > 0.  All finite. */
typedef struct {
    double nu, cs, dx, dy, dz, dt;
} fd6_params;

/* FP64 global diagnostics of the state: mass = dV sum exp(lnrho), kinetic
 * energy = dV sum exp(lnrho)|u|^2/2, sum of lnrho, max |u|, and the number
 * of grid points holding a non-finite value in any field.  When that number
 * is not zero, mass and kinetic energy are NaN.  Sums are in FP64 in a fixed
 * order (bitwise reproducible); exp is evaluated to within 2 ulp. */
typedef struct {
    double mass, kinetic_energy, sum_lnrho, umax;
    int64_t nonfinite;
} fd6_reductions;

typedef struct fd6_box fd6_box;

/* Library ABI version (FD6_ABI_VERSION). */
int fd6_abi_version(void);

/* Static text for a status code. */
const char *fd6_status_string(int status);

/* Device workspace needed by a box described by desc. */
int fd6_workspace_bytes(const fd6_desc *desc, size_t *bytes);

/* Create a box in the caller's workspace.  d_workspace: device pointer,
 * 256-byte aligned, at least fd6_workspace_bytes() bytes; stream: a
 * hipStream_t or NULL.  On success *out owns no device memory of its own. */
int fd6_create(const fd6_desc *desc, void *d_workspace, size_t bytes, void *stream,
               fd6_box **out);

/* Release the handle (the workspace stays the caller's). NULL is accepted. */
int fd6_destroy(fd6_box *box);

/* Replace the stream used by subsequent calls. */
int fd6_set_stream(fd6_box *box, void *stream);

/* Set nu, cs, dx, dy, dz, dt (validated as described above). */
int fd6_set_params(fd6_box *box, const fd6_params *params);

/* Load the state from host FP64 arrays (converted to the storage precision
 * with round-to-nearest-even); resets the RK3 register. Synchronises. */
int fd6_init_fields(fd6_box *box, const double *lnrho, const double *ux, const double *uy,
                    const double *uz);

/* Same from device FP64 arrays; asynchronous on the box's stream. */
int fd6_init_fields_device(fd6_box *box, const double *lnrho, const double *ux,
                           const double *uy, const double *uz);

/* Advance nsteps >= 0 full RK3 steps (3 substeps each: periodic boundary
 * condition, then the fused right-hand side + 2N-RK3 update, Algorithm 2; or
 * the two passes of Algorithm 3).  The z-sweep kernels resolve the periodic
 * images while loading their tiles; kernels that read the 3-cell ghost zone
 * are preceded by the periodic ghost pass.  Asynchronous on the box's
 * stream. */
int fd6_rk3_step(fd6_box *box, int32_t nsteps);

/* Advance nsteps >= 1 steps like fd6_rk3_step and enqueue the FP64
 * diagnostics of the final state (layout of fd6_reduce_device) into the
 * device buffer d_out5.  Asynchronous. */
int fd6_rk3_step_reduce(fd6_box *box, int32_t nsteps, double *d_out5);

/* Copy the state to host FP64 arrays.  Synchronises. */
int fd6_get_fields(fd6_box *box, double *lnrho, double *ux, double *uy, double *uz);

/* Copy the state to device FP64 arrays.  Asynchronous. */
int fd6_get_fields_device(fd6_box *box, double *lnrho, double *ux, double *uy, double *uz);

/* FP64 diagnostics of the current state, deterministic (fixed reduction
 * order).  Synchronises.  Returns FD6_ENONFINITE (with *out filled) when
 * out->nonfinite > 0. */
int fd6_reduce(fd6_box *box, fd6_reductions *out);

/* Same diagnostics written asynchronously, on the box's stream, to a device
 * buffer of 5 doubles: mass, kinetic energy, sum lnrho, max |u|, non-finite
 * count (as a double).  For use inside a timed or captured sequence. */
int fd6_reduce_device(fd6_box *box, double *d_out5);

/* Right-hand side d/dt (lnrho, ux, uy, uz) of the current state, evaluated by
 * the same kernels as a substep (precision of the box), to host FP64 arrays.
 * Overwrites the RK3 register, which holds no state between full steps
 * because alpha(1) = 0.  Synchronises. */
int fd6_rhs(fd6_box *box, double *r_lnrho, double *r_ux, double *r_uy, double *r_uz);

/* Kernel shape of the substep kernels (both methods): 0 = direct kernels, one
 * thread per point with every tap read through the caches from the ghost
 * zone, which a separate pass refreshes; 1 .. fd6_tile_count()-1 = z-sweep
 * kernels (periodic images resolved by their loaders, no ghost pass) with
 * different xy tile shapes, load pipelines and cache policies (most shapes
 * stream the new state and the RK register past the caches; the last ones
 * keep them cached, which pays when the whole state fits in the device's
 * last-level cache).  Results agree up to rounding order (the z-sweep shapes
 * bit for bit with each other); the choice only changes speed (see the
 * autotuner).  FD6_EINVAL for an index out of range; FD6_EUNSUPPORTED for a
 * shape the box's layout does not take (FD6_LAYOUT_AOS).  Default: 6 (64 x 8,
 * two planes ahead) for FP32 state, 8 (32 x 8, two planes ahead) for FP64. */
int fd6_tile_count(void);
int fd6_set_tile(fd6_box *box, int32_t tile);

/* Length in z-planes of the chunk one workgroup of a z-sweep kernel sweeps
 * (each chunk re-reads 6 planes): 0 (default) lets the library choose enough
 * workgroups to fill the device; values above nz mean whole columns.  Results
 * do not depend on it (bit for bit).  FD6_EINVAL if zchunk < 0. */
int fd6_set_zchunk(fd6_box *box, int32_t zchunk);

/* The current kernel shape and z-chunk length (set or tuned). */
int fd6_get_schedule(const fd6_box *box, int32_t *tile, int32_t *zchunk);

/* Autotuner of the kernel shape and z-chunk length (a speed choice only):
 * times every z-sweep shape the box's layout takes with the automatic
 * z-chunk, then z-chunk lengths 64, 128, 256 (those below nz) and nz for the
 * fastest shape -- one warm-up and 2 timed steps each, every step with its
 * FP64 diagnostics as fd6_rk3_step_reduce computes them, HIP events on the
 * box's stream -- and keeps the fastest pair.  Advances the state by 3 steps
 * per candidate: call it before the fields of the actual run are set, or set
 * them again afterwards.  cache_path as for fd6_batch_tune (key: device name,
 * grid, precision, method, layout).  FD6_ESTATE before parameters and fields
 * are set.  Synchronises. */
int fd6_tune(fd6_box *box, const char *cache_path);

/* The candidates the box's last fd6_tune call timed, in order: kernel shape,
 * z-chunk length and milliseconds per step (the mean of its timed steps).
 * Fills min(cap, count) entries of the three arrays and sets *n = count (0
 * when the last call took a cached choice or no call was made).  cap = 0
 * with NULL arrays queries the count.  FD6_EINVAL for null handle or n,
 * cap < 0, or cap > 0 with a null array. */
int fd6_get_tune_log(const fd6_box *box, int32_t *tiles, int32_t *zchunks, float *ms,
                     int32_t cap, int32_t *n);

/* External force of the momentum equation: one Fourier mode of eq.
 * (forcing), Sec. 6,
 *   f(x) = Re{ N f_k exp(i k.x + i phase) },  N = f0 cs sqrt(|k| cs / dt),
 *   f_k = (k x e) / sqrt(|k|^2 - (k.e)^2),
 * evaluated at grid point (i, j, k) as x = (i dx, j dy, k dz) and added to the
 * momentum right-hand side of every substep until changed.  The method draws
 * k (from an isotropic shell of wave vectors of the box), the unit vector e
 * and the phase afresh at every time step; those draws are the caller's:
 * call fd6_set_forcing before each fd6_rk3_step(box, 1).  k should be a wave
 * vector of the periodic box (k_x nx dx a multiple of 2 pi, likewise y, z)
 * for f to be periodic.  N uses the box's current cs and dt (fd6_set_params).
 * f = NULL switches the force off.  FD6_EINVAL for non-finite values, k = 0,
 * |e| != 1 (within 1e-6), e parallel to k, or f0 < 0.  Not available for the
 * batched ensemble. */
typedef struct {
    double kx, ky, kz; /* wave vector (radians per unit length) */
    double ex, ey, ez; /* unit vector, not parallel to k */
    double f0;         /* magnitude */
    double phase;      /* radians */
} fd6_forcing;
int fd6_set_forcing(fd6_box *box, const fd6_forcing *f);

/* Temporal blocking of substeps 1 and 2 (the paper's discussion of Sec. 7
 * proposes it): with enable != 0 every step runs substeps 1 and 2 as ONE
 * launch in which a workgroup sweeps substep 1 over its 16 x 16 output tile
 * and a 3-column ring, keeps that substep's new state and RK3 register on
 * chip (LDS), and sweeps substep 2 of the tile from them; substep 3 follows
 * as usual.  The substep-1 state and register never reach HBM (112 -> 48
 * bytes per point for the two substeps, FP32), at the price of substep 1 on
 * 22 x 22 / (16 x 16) = 1.9 times the columns.  Results are bit for bit
 * those of the plain launches.  An experimental schedule, off by default:
 * on MI355X at 512^3 the plain launches are 8.5 times faster (the fused
 * kernel spills the registers of its two column states to scratch memory
 * and does 1.7 times their arithmetic).  FP32 precision
 * and the 55-point method only (FD6_EUNSUPPORTED otherwise); ignored while a
 * force is set.  Drops captured steps when it changes. */
int fd6_set_fused_substeps(fd6_box *box, int32_t enable);

/* Graph mode (Algorithm 2 as one HIP graph per step): with enable != 0,
 * fd6_rk3_step and fd6_rk3_step_reduce capture one full step (three substeps,
 * and for the reducing variant the diagnostics of the last step, with d_out
 * recorded) per starting state set on a private stream the first time they
 * need it, and then replay it on the box's stream.  Results are bit for bit
 * those of the launch-by-launch path.  Captured steps are dropped by
 * fd6_set_params, fd6_set_tile, fd6_set_zchunk and disabling; a different
 * d_out re-captures the reducing step.  Event timing (fd6_set_timing)
 * bypasses graphs.  Default: off. */
int fd6_set_graph(fd6_box *box, int32_t enable);

/* Kernel timing with HIP events recorded on the box's stream around every
 * launch of the main substep kernel(s) (55-point fused kernel; both passes of
 * the 19-point method) and of the ghost fill.  enable != 0 starts (and
 * resets) collection, 0 stops it.  fd6_get_timing synchronises and returns
 * the summed milliseconds and launch counts since collection started. */
int fd6_set_timing(fd6_box *box, int enable);
int fd6_get_timing(fd6_box *box, double *kernel_ms, int64_t *kernel_launches, double *ghost_ms,
                   int64_t *ghost_launches);

/* Text of the last error on this handle ("" if none). */
const char *fd6_last_error(const fd6_box *box);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * diagnostics of fd6_reduce_device computed from four caller-owned compact
 * device arrays (nx*ny*nz values each, [z][y][x], x fastest), without a box
 * and without any allocation.  precision: FD6_FP64 for double arrays,
 * FD6_FP32 or FD6_FP32_ACC64 for float arrays.  dx, dy, dz > 0 give the cell
 * volume of the mass and kinetic-energy sums.  d_out5: device buffer of 5
 * doubles (mass, kinetic energy, sum lnrho, max |u|, non-finite count),
 * written asynchronously on `stream` (a hipStream_t or NULL).  The same
 * kernels and the same fixed summation order as fd6_reduce_device, so a box
 * holding the same values gives the same result.
 * Scratch: the partial sums live in a static device array of the library
 * (1024 x 8 doubles = 64 KiB per device, kept until the process ends; its
 * address is looked up once per device, on the first call with that device
 * current).  Every call on a device shares that array: calls that overlap on
 * one device (different streams or threads) race and must be serialised by
 * the caller.  Nothing needs clearing between calls.
 * FD6_EINVAL for null pointers, an unknown precision, non-positive or
 * non-finite spacings, or a grid dimension outside 1..4096 (the largest grid
 * the fixed partial count is sized for); FD6_EHIP if a HIP call fails. */
int fd6_reduce_fields_static(int32_t nx, int32_t ny, int32_t nz, int32_t precision,
                             const void *lnrho, const void *ux, const void *uy,
                             const void *uz, double dx, double dy, double dz, void *stream,
                             double *d_out5);

/* ---------------------------------------------------------------------------
 * Batched ensemble: n independent periodic boxes of possibly different sizes
 * and parameters, all with the same precision and the 55-point method,
 * advanced together.  Each substep is ONE persistent kernel launch over the
 * tile-chunks of every box (longest first); a full step (3 substeps) is
 * replayed from a captured HIP graph.  Per-box geometry, pointers,
 * coefficients and time steps live in device memory inside the workspace.
 * Per grid point the arithmetic is that of the single-box z-sweep kernel with
 * the same tile shape, so each box's result equals a single-box run bit for
 * bit.  Conventions (status codes, host layout, workspace ownership, stream)
 * as for fd6_box.
 * ------------------------------------------------------------------------- */
typedef struct fd6_batch fd6_batch;

/* Workspace for n boxes described by descs[0..n-1] (same precision and the
 * same flags, else FD6_EINVAL; variant FD6_55P, else FD6_EUNSUPPORTED). */
int fd6_batch_workspace_bytes(int32_t n, const fd6_desc *descs, size_t *bytes);

/* Create the ensemble in the caller's workspace (256-byte aligned). */
int fd6_batch_create(int32_t n, const fd6_desc *descs, void *d_workspace, size_t bytes,
                     void *stream, fd6_batch **out);
int fd6_batch_destroy(fd6_batch *batch);

/* Parameters of every box: per_box[0..n-1], validated like fd6_set_params.
 * Uploads the device descriptors (synchronises). */
int fd6_batch_set_params(fd6_batch *batch, const fd6_params *per_box);

/* State of box `box` from host FP64 arrays; resets its RK3 register. */
int fd6_batch_init_fields(fd6_batch *batch, int32_t box, const double *lnrho, const double *ux,
                          const double *uy, const double *uz);

/* Kernel shape (1 .. fd6_tile_count()-1, a z-sweep shape) and work
 * distribution of the persistent launch.  zchunk >= 0: each box's z range is
 * split evenly into chunks of at most zchunk planes (0 = whole boxes;
 * otherwise zchunk >= 8, since every chunk re-reads 6 planes), the chunks
 * sorted longest first and dealt to the workgroups in turn.
 * zchunk = FD6_BATCH_BALANCED: the tile columns of all boxes cut into one run
 * of equal cost per workgroup (a column is split only where a run ends).
 * zchunk = FD6_BATCH_PACKED: whole tile columns, longest first, each dealt to
 * the least-loaded workgroup; a column that would take its workgroup past a
 * target cost (chosen by the library near the mean cost) is split there.
 * Rebuilds the work lists and drops any captured graph.  FD6_EINVAL for a
 * shape out of range, zchunk < 0 other than FD6_BATCH_BALANCED and
 * FD6_BATCH_PACKED, or 0 < zchunk < 8;
 * FD6_EUNSUPPORTED for a shape the ensemble's layout does not take.  A
 * refused call leaves the schedule in force (and fd6_batch_get_schedule's
 * answer) unchanged.  Default: shape 8 (32 x 8, two planes ahead), chunks of
 * at most 64 planes. */
#define FD6_BATCH_BALANCED (-1)
#define FD6_BATCH_PACKED (-2)
int fd6_batch_set_schedule(fd6_batch *batch, int32_t tile, int32_t zchunk);

/* Autotuner of the ensemble schedule (the shape and chunk choice is the
 * caller's tuning concern, not the method's): times every z-sweep shape the
 * ensemble's layout takes with z-chunk lengths 0 (whole boxes), 32, 48 and 64,
 * FD6_BATCH_BALANCED and FD6_BATCH_PACKED, in two passes over the candidates
 * (each trial 10 warm-up steps, since the step time settles only after a
 * change of schedule, then 8 timed steps, HIP events on the ensemble's
 * stream; a candidate's time is its faster trial), and keeps the fastest.
 * Advances every box by 36 steps per candidate: call it before the fields of
 * the actual run are set, or set them again afterwards.
 * cache_path (may be NULL) names a text file of "key tile zchunk" lines,
 * keyed by device name, precision, layout and box shapes: a cached entry is
 * applied without timing, a new result is appended (a file that cannot be
 * opened is ignored).  FD6_ESTATE before parameters
 * and fields are set.  If a trial fails, the schedule in force before the
 * call is restored and the failure returned.  Synchronises. */
int fd6_batch_tune(fd6_batch *batch, const char *cache_path);

/* The current schedule (set or tuned). */
int fd6_batch_get_schedule(const fd6_batch *batch, int32_t *tile, int32_t *zchunk);

/* enable != 0 (default): steps replay a captured graph of the 3 substeps;
 * 0: the same kernels are launched directly. */
int fd6_batch_set_graph(fd6_batch *batch, int32_t enable);

/* Advance every box by nsteps full RK3 steps.  Asynchronous. */
int fd6_batch_step(fd6_batch *batch, int32_t nsteps);

/* State of box `box` to host FP64 arrays.  Synchronises. */
int fd6_batch_get_fields(fd6_batch *batch, int32_t box, double *lnrho, double *ux, double *uy,
                         double *uz);

/* FP64 diagnostics of every box into per_box[0..n-1] (as fd6_reduce).
 * Synchronises; FD6_ENONFINITE if any box holds a non-finite value. */
int fd6_batch_reduce(fd6_batch *batch, fd6_reductions *per_box);

const char *fd6_batch_last_error(const fd6_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* FD6_H */
