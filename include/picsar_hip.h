/*
 * picsar_hip.h -- C ABI of the MI355X (gfx950) 2.5D axisymmetric PIC step.
 *
 * The library advances the particle-in-cell step of Belyaev, "PICsar"
 * (arXiv 1407.1810) on one GPU: the Yee/FDTD field update in integral form
 * on the body-fitted (r, theta) mesh (App. A), the relativistic Vay or Boris
 * push with field gather (Sec. 3.3), the charge-conserving Villasenor-Buneman
 * deposit (Sec. 2, Sec. 3.3), the 1-2-1 current filter with its polar remap
 * (App. B), conducting walls and the lossy absorbing layer (Sec. 3.4), the
 * analytic initial fields with spin-up (Sec. 5.2) and surface pair injection
 * (Sec. 5.3).
 *
 * Conventions shared by every entry point
 *  - Every call returns a pic_status and never throws; pic_last_error()
 *    holds the message of the last failure of a context.
 *  - All pointers in these signatures are HOST pointers owned by the
 *    caller; the library copies from / into them.  All device memory is
 *    owned by the context and freed by pic_destroy().
 *  - Units: Lorentz-Heaviside, time step dt = 1, lengths in code units, c in
 *    length units per step.  Momenta u = gamma v / c in the local
 *    (r, theta, phi) basis.  Particle weights w are signed macro charges.
 *  - Grid: nr x nth cells; radial nodes i = 0..nr (conductors at 0 and nr),
 *    meridional nodes j = 0..nth (poles at 0 and nth).  Fields follow the
 *    staggering of eq. (offseteq), Sec. 3.1.  Field arrays exchanged through
 *    the ABI are row-major [i][j] (j fastest) with these extents:
 *       PIC_ER  (i+1/2, j)      nr     x (nth+1)
 *       PIC_ETH (i, j+1/2)      (nr+1) x nth
 *       PIC_EPH (i, j)          (nr+1) x (nth+1)
 *       PIC_BR  (i, j+1/2)      (nr+1) x nth
 *       PIC_BTH (i+1/2, j)      nr     x (nth+1)
 *       PIC_BPH (i+1/2, j+1/2)  nr     x nth
 *       PIC_FR, PIC_FTH, PIC_FPH: the face charges deposited in the last step
 *       (charge crossing each dual face during the step, after filtering),
 *       shaped like ER, ETH, EPH with g = 2*n_filt + 3 extra ghost rows on
 *       each radial side (first row is i = -g).
 *    pic_field_shape() returns the extents.
 *  - Particles cross the ABI as FP64 absolute grid coordinates (x radial in
 *    [-(n_filt+1), nr+n_filt+1], y meridional in [0, nth]).  Inside, a
 *    particle is an int32 cell plus an in-cell offset of the context's
 *    precision: an FP32 context rounds the offset (x - floor(x)), the
 *    momenta and the weight to FP32 once, on the way in.
 *  - pic_step() enqueues on the context's stream and synchronises before it
 *    returns, so that device-side errors (CFL, capacity) are reported by
 *    the call that caused them.  Without stage timing the launches of one
 *    step are captured into HIP graphs, one with the particle sort and one
 *    without (used on steps where no run is due to sort), and replayed;
 *    with timing on they are enqueued one by one between HIP events.
 */
#ifndef PICSAR_HIP_H
#define PICSAR_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,     /* bad argument or descriptor */
    PIC_ENOMEM = -2,     /* device allocation failed */
    PIC_ECFL = -3,       /* a particle moved one cell or more in a step */
    PIC_ECAPACITY = -4,  /* particle store full (inject or injection) */
    PIC_ENAN = -5,       /* non-finite value found by a diagnostic */
    PIC_EDEVICE = -6,    /* HIP runtime error */
    PIC_ESTATE = -7      /* call out of order (e.g. step before init) */
} pic_status;

enum { PIC_R_LOG = 0, PIC_R_LIN = 1 };            /* Sec. 3.2: xi = r0 ln(r/r0) or r */
enum { PIC_TH_EQAREA = 0, PIC_TH_LIN = 1 };       /* Sec. 3.2: theta_A = -cos(theta) or theta */
enum { PIC_FP64 = 0, PIC_FP32 = 1 };
enum { PIC_VAY = 0, PIC_BORIS = 1 };              /* Sec. 3.3 */
enum { PIC_BG_NONE = 0, PIC_BG_UNIFORM_BZ = 1, PIC_BG_MONOPOLE = 2, PIC_BG_DIPOLE = 3,
       PIC_BG_DIPOLE_COROT = 4 };
enum { PIC_ER = 0, PIC_ETH = 1, PIC_EPH = 2, PIC_BR = 3, PIC_BTH = 4, PIC_BPH = 5,
       PIC_FR = 6, PIC_FTH = 7, PIC_FPH = 8 };
enum { PIC_FLAG_IDS = 1 };                        /* carry a uint64 id per particle */

/* Grid, numerics and storage.  tile_r, tile_th and sort_interval choose the
 * counting-sort tile and how often particles are re-sorted (0 = default);
 * they change speed, never results beyond float reordering. */
typedef struct {
    int32_t nr, nth;          /* cells; 2 <= nr <= 16000, 4 <= nth <= 8191 */
    double r_in, r_out;       /* conductor radii, 0 < r_in < r_out */
    int32_t r_kind, th_kind;  /* PIC_R_*, PIC_TH_* */
    double c;                 /* light speed, length units per step */
    int32_t n_filt;           /* 1-2-1 filter passes, 0..8 (App. B) */
    int32_t absorb_cells;     /* lossy layer width in cells, 0 = off, at most nr (Sec. 3.4.1) */
    double sigma_max;         /* sigma* at the outer conductor, eq. (EBcond) */
    int32_t precision;        /* PIC_FP64 | PIC_FP32 */
    int32_t mover;            /* PIC_VAY | PIC_BORIS */
    int64_t particle_capacity;/* maximum particles held at once, below 2^31 */
    int32_t tile_r, tile_th;  /* sort tile in cells (0 = 8 x 8) */
    int32_t sort_interval;    /* steps between sorts (0 = 4; < 0 = never) */
    int32_t flags;            /* PIC_FLAG_* */
    int32_t chunk_ppt;        /* particles per thread of a push work-group: 4, 8, 16 (0 = 8) */
} pic_grid_desc;

/* Analytic initial fields and injection (Sec. 5.2, 5.3, 4.3). */
typedef struct {
    int32_t bg_kind;          /* PIC_BG_* */
    double B0;                /* field at r_in (monopole, dipole) or uniform B_z */
    double omega;             /* final angular velocity of the inner conductor */
    double t_spin;            /* linear spin-up time (0 = none) */
    double q_over_m;          /* |q/m| of all macro-particles */
    double f_inj;             /* fraction of the surface charge released per step */
    double q_inj;             /* |charge| of one injected macro-particle */
    int32_t inject;           /* 1: surface injection on (monopole / dipole only) */
    uint64_t seed;            /* key of the Philox4x64-10 injection stream */
} pic_phys_desc;

/* Create a context on HIP device `device`.  hip_stream is a hipStream_t to
 * enqueue on (for example the caller's current stream) or NULL, in which
 * case the context creates and owns a stream of default priority. */
pic_status pic_create(pic_ctx **out, int device, void *hip_stream);

/* Allocate and initialise the grid (fields zero), the particle store, the
 * diagnostic planes and the metric tables: the stretched coordinates of
 * Sec. 3.2 (xi = r0 ln(r / r0), theta_A = -cos theta, or their linear
 * options) and the area and line elements of App. A eq. (linearea), formed
 * in FP64 on the host and kept in FP64 on the device for the field update
 * in either precision (the push reads the radii in the context's
 * precision).  Once per context; PIC_ESTATE if called twice, PIC_EINVAL for
 * an invalid descriptor, PIC_ENOMEM if the device memory runs out (nothing
 * is then kept).  pic_init_grid is the same call under a second name. */
pic_status pic_init(pic_ctx *ctx, const pic_grid_desc *grid, const pic_phys_desc *phys);
pic_status pic_init_grid(pic_ctx *ctx, const pic_grid_desc *grid, const pic_phys_desc *phys);

/* Append n macro-particles: the state of Sec. 3.3 (position in grid
 * coordinates, momentum u = gamma v / c in the local (r, theta, phi) basis,
 * signed macro charge w, all host FP64 arrays of length n); id may be NULL,
 * then ids are the storage slots in order of arrival.  Each particle is
 * stored as an int32 cell plus in-cell offsets (rounded once to FP32 in an
 * FP32 context).  PIC_EINVAL if a position lies outside the ranges above
 * or a momentum or weight is not finite, PIC_ECAPACITY if the store would
 * overflow (nothing is then appended in either case). */
pic_status pic_inject_particles(pic_ctx *ctx, int64_t n, const double *x, const double *y,
                                const double *ur, const double *ut, const double *up,
                                const double *w, const uint64_t *id);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation): the same append as
 * pic_inject_particles, with the same arguments, results and errors, staged
 * through a fixed block of device memory that the library holds on each GPU
 * for the life of the process instead of memory allocated per call; it
 * calls no allocating routine.  At most 65536 particles per call
 * (PIC_EINVAL beyond).  Like pic_inject_particles it reads the particle
 * count back and waits for the context's stream, so it cannot be recorded
 * into a graph.  All contexts on one GPU share that block: calls that
 * overlap on one GPU (from several host threads) race and must be
 * serialised by the caller. */
pic_status pic_inject_particles_noalloc(pic_ctx *ctx, int64_t n, const double *x, const double *y,
                                        const double *ur, const double *ut, const double *up, const double *w,
                                        const uint64_t *id);

/* Advance n_steps steps: half Faraday, gather + push + deposit, half
 * Faraday, filter, Ampere with the conducting walls and the polar caps of
 * eq. (erpolarupdate), lossy layer, surface injection; particles are
 * re-sorted every sort_interval steps. */
pic_status pic_step(pic_ctx *ctx, int32_t n_steps);

/* Field component comp (PIC_*) converted to FP64 into host[cap]. */
pic_status pic_field_shape(pic_ctx *ctx, int32_t comp, int32_t *rows, int32_t *cols, int32_t *row0);
pic_status pic_get_field(pic_ctx *ctx, int32_t comp, double *host, int64_t cap);
/* Overwrite one E or B component from host FP64 data (rows x cols). */
pic_status pic_set_field(pic_ctx *ctx, int32_t comp, const double *host, int64_t n);

/* Live particles in storage order: the particle state of Sec. 3.3 as FP64
 * absolute grid coordinates (cell index plus offset), local momenta,
 * weights and ids, into host arrays of cap entries.  Any output pointer may
 * be NULL.  *n_out receives the count; PIC_EINVAL if cap is smaller
 * (nothing is written then). */
pic_status pic_get_particles(pic_ctx *ctx, double *x, double *y, double *ur, double *ut, double *up,
                             double *w, uint64_t *id, int64_t cap, int64_t *n_out);

/* The positions of the same particles, in the same order, exactly as stored
 * (Sec. 3.3 particle state; the int32 cell and the in-cell offsets of the
 * context's precision, converted to FP64 without rounding): radial and
 * meridional cell index ci, cj, and offsets fx = x - ci in [0, 1), fy =
 * y - cj in [0, 1] (1 only in the last meridional cell, at the pole).  An
 * FP64 absolute coordinate rounds the offset of a particle at cell index N
 * to about 1e-16 N; these do not.  Any output pointer may be NULL; cap and
 * n_out as for pic_get_particles. */
pic_status pic_get_particle_cells(pic_ctx *ctx, int32_t *ci, int32_t *cj, double *fx, double *fy, int64_t cap,
                                  int64_t *n_out);

/* Moments and diagnostics:
 *  PIC_MOM_COUNTS: out[0..4] = live particles, injected total, deleted
 *                  total, step index, particle-steps advanced since init;
 *                  out[5] (if cap >= 6) = push chunks whose cells did not fit
 *                  the LDS planes and went through global memory
 *  PIC_MOM_GAUSS:  Gauss diagnostic in FP64 (Sec. 2 eq. (maxti), App. B
 *                  eq. (multfiltcharge)): out[0..N) = closed-surface flux
 *                  G of E out of each dual cell, out[N..2N) = the
 *                  n_filt-filtered bilinear particle charge Qbar of that
 *                  node, N = (nr+1)*(nth+1) row-major; rows 0 and nr of the
 *                  flux are zero (surface nodes)
 *  PIC_MOM_GAUSS_RES: the same residual R = G - Qbar reduced on the device
 *                  in FP64 over the interior nodes below the lossy layer,
 *                  1 <= i <= nr-1-absorb_cells, all j (the layer damps E
 *                  and so does not conserve R; Sec. 3.4.1), 9 values:
 *                  out[0] = max |R - R0|, out[1] =
 *                  sqrt(sum (R - R0)^2), out[2] = max |R|, out[3] =
 *                  sqrt(sum R^2), out[4] = max of the unfiltered absolute
 *                  node charge sum_p |w_p| W(node; x_p) (the scale of a
 *                  drift when the net charge vanishes), out[5] = max |G|,
 *                  out[6] = nodes reduced, out[7] = non-finite values met
 *                  on any interior node, out[8] = step index at which R0
 *                  was recorded.  R0
 *                  is the residual of the first Gauss evaluation (this kind
 *                  or PIC_MOM_GAUSS) after pic_init, pic_load, particles
 *                  added from the host or a field set from the host; it
 *                  stays on the device, so that the drift R - R0 is exactly
 *                  the charge-conservation error of the steps since then
 *  PIC_MOM_RHO_Q:  the n_filt-filtered bilinear node charge Qbar alone
 *                  (N values, as the second half of PIC_MOM_GAUSS)
 *  PIC_MOM_CARRY:  fractional injection count per theta node (nth+1)
 *  PIC_MOM_STAGE_MS: mean device time per step, in ms, of each stage over
 *                  the steps of the last pic_step call (out[0..8] = sort,
 *                  first faraday, push, filter, ampere, absorb, inject,
 *                  zeroing, whole step), from HIP events recorded on the
 *                  context stream -- only when timing is on
 *  PIC_MOM_POYNTING: spindown luminosity (Sec. 5.4), out[i] for
 *                  i = 0..nr-1 = the Poynting flux c (E x B)_r, in FP64,
 *                  of the total field (plasma field plus the analytic
 *                  initial field at the current step) through the sphere
 *                  of radial half-node i + 1/2: per meridional cell
 *                  E_theta averaged over its two radial nodes, E_phi over
 *                  its four corners, B_theta over its two meridional
 *                  nodes, B_phi at its own point, times the cell's face
 *                  2 pi r(i+1/2)^2 (cos theta_j - cos theta_j+1) (nr) */
enum { PIC_MOM_COUNTS = 0, PIC_MOM_GAUSS = 1, PIC_MOM_CARRY = 2, PIC_MOM_STAGE_MS = 3, PIC_MOM_POYNTING = 4,
       PIC_MOM_GAUSS_RES = 5, PIC_MOM_RHO_Q = 6 };
/* Every kind copies into the caller's out[cap] (PIC_EINVAL if cap is below
 * the size given above).  PIC_MOM_GAUSS, PIC_MOM_GAUSS_RES and
 * PIC_MOM_POYNTING return PIC_ENAN, after writing out, when the reduction
 * met a non-finite field value or particle charge.  The diagnostic planes
 * are allocated by pic_init; no kind allocates device memory. */
pic_status pic_get_moments(pic_ctx *ctx, int32_t kind, double *out, int64_t cap);

/* Set the step index (time t = index * dt) and the injection carry, so a
 * run can be resumed from a saved state. */
pic_status pic_set_step_index(pic_ctx *ctx, int64_t step);
pic_status pic_set_carry(pic_ctx *ctx, const double *carry, int64_t n);

/* Turn per-stage device timing (HIP events on the context stream) on/off. */
pic_status pic_set_timing(pic_ctx *ctx, int32_t on);

/* Change the counting-sort tile (tile_r x tile_th cells, each >= 1) and the
 * steps between sorts (> 0, or < 0 for never) of a live context; the next
 * step sorts.  Speed only: results change by float reordering at most.
 * PIC_EINVAL for a zero interval or a tile side outside 1..4096. */
pic_status pic_set_sort(pic_ctx *ctx, int32_t tile_r, int32_t tile_th, int32_t sort_interval);

/* Per-run autotuning of the sort: for each of n_cand candidates
 * cand[3q..3q+2] = (tile_r, tile_th, sort_interval) the context takes one
 * step with it and then `steps` more (rounded up to whole sort periods),
 * timed with HIP events; the candidate with the least device time per
 * particle-step is kept and written to best[0..2], its time in ns per
 * particle-step to *best_ns (may be NULL).  The tuning steps are real
 * steps of the run (its state and step index advance). */
pic_status pic_autotune(pic_ctx *ctx, const int32_t *cand, int32_t n_cand, int32_t steps, int32_t *best,
                        double *best_ns);

/* Checkpoint and resume, for runs longer than one process (the paper's
 * rotator runs last tens of thousands of steps).  pic_save writes the whole
 * state of an initialised context to the file `path` (created or
 * truncated): its grid and physics descriptors (with the sort tile,
 * interval and chunk size in use), step index and counters, the
 * fixed-point deposit scale, the injection carry, the nine field planes and
 * the filtered face charges, and every particle slot as stored -- int32
 * cell, offsets, momenta and weight in the context's precision, ids -- so
 * that nothing passes through an FP64 conversion.  pic_load restores such
 * a file into a context made by pic_create and not initialised, which then
 * continues the run from the same bits.  The file is this library's own
 * format (a versioned header, then the arrays, host byte order).
 * PIC_ESTATE for pic_save before pic_init or pic_load after it; PIC_EINVAL
 * for a null path, a file that cannot be opened, written or read whole, a
 * file that is not a checkpoint of this version, or one whose descriptors,
 * counters, cells or offsets are out of range; PIC_ECAPACITY if its
 * particles exceed its capacity; PIC_EDEVICE for HIP errors. */
pic_status pic_save(pic_ctx *ctx, const char *path);
pic_status pic_load(pic_ctx *ctx, const char *path);

/* Message of the last failed call on ctx (empty if none). */
const char *pic_last_error(const pic_ctx *ctx);

/* Release every resource of the context.  A context that belongs to a
 * batch must outlive the batch. */
void pic_destroy(pic_ctx *ctx);

/* ------------------------------------------------------------------
 * Batches: many independent runs advanced together (the ensemble of
 * uneven runs of one precision on one device).  Every kernel of a step
 * serves all runs of the batch at once -- field kernels over the
 * concatenated work-groups of all grids, the push over the concatenated
 * particle chunks of all runs -- so small runs fill the GPU together and a
 * step costs one launch sequence, captured once into a HIP graph and
 * replayed.  Each run keeps its own grid, physics, tile, sort interval and
 * particle store (those of its context); the push uses the chunk_ppt of
 * the first run.  Results are those of stepping each context on its own,
 * up to the order of floating-point atomic additions.
 * ------------------------------------------------------------------ */
typedef struct pic_batch pic_batch;

/* Group n initialised contexts (same device, same precision, no context
 * twice) into *out.  The contexts stay valid for pic_get_* and may still be
 * stepped alone; they must not be stepped concurrently with the batch and
 * must outlive it.  hip_stream as in pic_create.  PIC_EINVAL for an empty
 * or mixed list, PIC_ESTATE for a context without pic_init. */
pic_status pic_batch_create(pic_ctx *const *runs, int32_t n, void *hip_stream, pic_batch **out);

/* Advance every run of the batch by n_steps steps and synchronise.  A
 * device error (CFL, injection capacity) of any run is reported with the
 * index of the first run that raised it; all runs have then taken the
 * steps. */
pic_status pic_batch_step(pic_batch *b, int32_t n_steps);

/* Device time in ms of the last pic_batch_step, from HIP events on the
 * batch stream around its launches. */
pic_status pic_batch_elapsed_ms(pic_batch *b, double *ms);

/* Per-stage device timing of batch steps, as pic_set_timing /
 * PIC_MOM_STAGE_MS for a context: with timing on the launches are enqueued
 * one by one between HIP events instead of replaying the graph;
 * pic_batch_stage_ms writes the 9 stage means of the last pic_batch_step
 * (cap >= 9). */
pic_status pic_batch_set_timing(pic_batch *b, int32_t on);
pic_status pic_batch_stage_ms(pic_batch *b, double *out, int64_t cap);

/* Message of the last failed call on b (empty if none). */
const char *pic_batch_last_error(const pic_batch *b);

/* Release the batch (not its contexts). */
void pic_batch_destroy(pic_batch *b);

#ifdef __cplusplus
}
#endif
#endif
