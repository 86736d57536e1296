/*
 * pabd.h -- C ABI of the MI355X (gfx950) library for projective affine body
 * dynamics (PABD): affine bodies joined by peridynamic bonds, advanced by the
 * semi-implicit successive-substitution global/local iteration of the paper
 * "Projective Affine Body Dynamics for Multibody Systems" (Algorithm 1).
 *
 * Conventions
 *  - Every call returns a pabd_status; no exception crosses the ABI.  After a
 *    failure pabd_last_error() returns a thread-local message.
 *  - All host arrays are owned by the caller.  Descriptor arrays are copied at
 *    create/admit time; output arrays are written in full.  Read-back is always
 *    double precision.  Row-major; SI units; A is 3x3 with rows a1, a2, a3 so that
 *    a material point x maps to y = A x + c (Sec. 3).
 *  - Handles are owned by the library and freed with *_destroy.  A handle is not
 *    thread safe; use one host thread and one stream per handle.
 *  - hip_stream arguments are hipStream_t values passed as void* (NULL = the
 *    library's own stream of the handle).  Work is enqueued asynchronously;
 *    read-back calls synchronise the handle's stream.
 *  - Device memory is allocated by the library (hipMalloc) at create/admit time
 *    and released at destroy/release; stepping allocates nothing.
 */
#ifndef PABD_H
#define PABD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PABD_OK = 0,
  PABD_E_INVALID = -1,  /* malformed argument or descriptor */
  PABD_E_OOM = -2,      /* device allocation failed or budget exceeded */
  PABD_E_DEVICE = -3,   /* HIP runtime error */
  PABD_E_DIVERGED = -4, /* non-finite state or contact capacity overflow */
  PABD_E_BUSY = -5,     /* batch has no free slot or HBM budget for the scene */
  PABD_E_NOTFOUND = -6  /* slot not in use */
} pabd_status;

/* body shapes (shape_param: box half extents; sphere radius in [0]) */
#define PABD_SHAPE_BOX 0
#define PABD_SHAPE_SPHERE 1
/* body flags */
#define PABD_FLAG_PINNED 1u     /* kinematic: infinite mass, never updated, v = w = 0 */
#define PABD_FLAG_NO_CONTACT 2u /* never takes part in collision detection */
/* bond types */
#define PABD_BOND_QUADRATIC 0 /* Psi = 1/2 kappa (d - l)^2 (Sec. 5.2.2); l = 0: ball joint */
#define PABD_BOND_DRIVEN 1    /* ball joint whose j-side anchor is turned by theta(t) */
/* augmented Lagrangian (Sec. 5.2.2): Psi = 1/2 kappa_j C^2 + lambda_j C with the signed
 * elongation C = d - l (l > 0 required); kappa is kappa_start.  Every iteration
 * lambda_j += kappa_j C and kappa_j += al_beta |C| (C at the iterate the forces use);
 * every step kappa_j = max(al_gamma kappa_j, kappa_start), lambda_j *= al_alpha al_gamma.
 * The multiplier's tension beyond kappa l is treated implicitly (weight
 * kappa + (lambda - kappa l)/d).  Scenes with such bonds run on the flat path. */
#define PABD_BOND_AUGMENTED 3
/* polynomial bond (Sec. 4.2.1): Psi = kappa / p (d - l)^p, p = order[] even in [2, 12];
 * phi = kappa (d - l)^{p-1} split by the signs of its binomial terms (non-negative terms
 * implicit, the rest explicit); p = 2 is the quadratic bond.  Flat path. */
#define PABD_BOND_POLYNOMIAL 4
/* slider bond (the slider joint of Sec. 5.1, whose energy the paper does not print;
 * read as a point-on-line bond): Psi = 1/2 kappa dist(y_i, L_j)^2 with L_j the line
 * through x_j along the axis drive[0..2] (both in j's material frame, world if
 * j = -1; the axis need not be unit; rest_len must be 0 or NULL).  Every iteration
 * the line-side anchor is the foot of the perpendicular from y_i^k onto L_j at q^k,
 * and the bond acts as a ball joint between x_i and that point of j: the point
 * side's weight stays at x_i, the line side's moves with the foot.  A prismatic
 * joint is three such bonds from non-collinear points to parallel lines.  Flat path. */
#define PABD_BOND_SLIDER 5
/* precision of bond and body arithmetic; the block factorisation and the
 * convergence-residual reductions are always FP64 */
#define PABD_FP32 0
#define PABD_FP64 1

/*
 * Scene description: the statement of the problem of Sec. 4 -- bodies with mass
 * m and affine moment Pi0 = int rho x x^T dV of the generalised mass matrix
 * M = diag(m I, Pi0, Pi0, Pi0) (Sec. 4.1.1), given directly (mass, Pi0) or
 * derived from a uniform density and the body's shape; initial q (c0, A0) and
 * velocities; bonds with material anchors and energy parameters (Sec. 4.2.1,
 * Sec. 5.2.2); gravity; time step h; and the number K of global/local
 * iterations per step (Algorithm 1).  The shape is also the body's contact
 * geometry.
 *
 * Validation (PABD_E_INVALID): h > 0, K >= 1; every free body needs m > 0 and
 * a symmetric positive definite Pi0; A0 must be a rotation (|A0^T A0 - I|_F <=
 * 1e-6 and det A0 > 0); bond endpoints in range (-1 = world), no bond from a
 * body to itself, kappa > 0, rest length >= 0.
 */
typedef struct {
  int32_t n_bodies;
  const int32_t *shape;       /* [N] PABD_SHAPE_* */
  const double *shape_param;  /* [N*3] */
  const double *density;      /* [N] kg/m^3 (> 0 unless pinned) */
  const uint8_t *flags;       /* [N] PABD_FLAG_* or NULL */
  const int32_t *group;       /* [N] bodies sharing a nonzero group never collide; or NULL */
  const double *c0;           /* [N*3] centre of mass */
  const double *A0;           /* [N*9] rotation, row-major */
  const double *v0, *w0;      /* [N*3] linear / angular (world) velocity, or NULL */
  int32_t n_bonds;
  const int32_t *bond_i;      /* [B] */
  const int32_t *bond_j;      /* [B] -1 = world (x_j then in world coordinates) */
  const int32_t *bond_type;   /* [B] PABD_BOND_* or NULL (all quadratic) */
  const double *x_i, *x_j;    /* [B*3] material anchors */
  const double *kappa;        /* [B] stiffness > 0 */
  const double *rest_len;     /* [B] rest length >= 0, or NULL */
  const double *drive;        /* [B*13] driven bonds: axis3 pivot3 base3 theta0 amp freq phase;
                               * slider bonds: the line axis in [0..2] */
  double gravity[3];
  double h;                   /* time step > 0 */
  double t0;                  /* time at the start of the first step */
  int32_t iters;              /* K >= 1 */
  int32_t contact_enable;     /* build contact bonds every step */
  double mu;                  /* Coulomb friction coefficient */
  double contact_kappa_scale; /* kappa_c = scale * m / h^2, m the heavier free mass */
  double contact_margin;      /* base detection margin (m) */
  int32_t n_planes;
  const double *planes;       /* [P*4] unit normal n and offset o: free side n.y >= o */
  int32_t max_contacts_per_body; /* capacity of contact ends per body (> 0 if contacts) */
  int32_t precision;          /* PABD_FP32 or PABD_FP64 */
  double al_beta, al_alpha, al_gamma; /* augmented-bond constants (the paper: 1e4, 0.99, 0.999) */
  const int32_t *order;       /* [B] order p of polynomial bonds, or NULL */
  /* optional generalised mass (Sec. 4.1.1), overriding what density and shape
   * give: mass [N] in kg, Pi0 [N*6] = int rho x x^T dV in kg m^2 as the packed
   * symmetric (00, 01, 02, 11, 12, 22) in the body's material frame.  Either may
   * be NULL (then that part comes from density and shape); pinned bodies may
   * give anything (their mass never enters a step). */
  const double *mass;
  const double *Pi0;
} pabd_scene_desc;

typedef struct pabd_scene pabd_scene;
typedef struct pabd_batch pabd_batch;

const char *pabd_last_error(void);
/* Device memory of scenes and batches created from now on: alloc(bytes, ctx) must
 * return device memory of the current device, aligned to 256 bytes, or NULL (then
 * the create or admit fails with PABD_E_OOM); release(ptr, ctx) returns it.  A
 * scene or batch releases its memory only at destroy, after the device is idle,
 * and keeps the allocator that was in force at its creation.  alloc = NULL
 * restores hipMalloc / hipFree.  Not thread-safe: set it before creating handles.
 * (For a caching allocator such as PyTorch's.) */
pabd_status pabd_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                               void (*release)(void *ptr, void *ctx), void *ctx);
/* number of HIP devices visible (0 without a GPU); never fails */
int32_t pabd_device_count(void);

/* ---- plain path: one scene, one kernel launch per iteration --------------- */

/* Validate the descriptor, take m and Pi0 per body (given, or from density and
 * shape: Sec. 4.1.1), build the bond incidence lists in (body, bond id) order,
 * upload, and factor every body's 12x12 block H = M + h^2 sum w J^T J in FP64
 * by its closed-form inverse (Sec. 4.2.1 block matrix; Sec. 4.3).  *out is a
 * library-owned handle (NULL on failure). */
pabd_status pabd_scene_create(const pabd_scene_desc *desc, pabd_scene **out);
/* Wait for the device, then free the handle and its device memory. */
pabd_status pabd_scene_destroy(pabd_scene *s);
/* Advance nsteps steps of Algorithm 1: collision detection on q^n (contact
 * bonds, Sec. 4.2), prediction, K Jacobi iterations of the body-wise global
 * update (Sec. 4.2.1) each followed by the local polar projection (Sec. 4.2.2),
 * and velocity recovery (Sec. 4.4).  Enqueued on hip_stream; returns at once. */
pabd_status pabd_scene_step(pabd_scene *s, int32_t nsteps, void *hip_stream);
/* Copy the state q^n = (c, A) and velocities (v, w) of Algorithm 1 to the host
 * (c [N*3], A [N*9], v [N*3], w [N*3]; any may be NULL) after the device is
 * idle.  Returns PABD_E_DIVERGED (state still copied) if a step produced a
 * non-finite state or overflowed contact capacity. */
pabd_status pabd_scene_read_state(pabd_scene *s, double *c, double *A, double *v, double *w);
/* FP64 convergence residual of the last iteration of the last step,
 * rho = ||q^K - q^{K-1}||_M / ||q^{K-1}||_M over the scene's free bodies (the
 * relative change that the stopping test of Algorithm 1 reads; K is fixed
 * here, so it is reported, not tested).  0 before the first step. */
pabd_status pabd_scene_residual(const pabd_scene *s, double *rho_last);
/* The same residual for every iteration k of the last step (out[k], k < cap;
 * iterations other than the last are recorded only with debug bit1 set, else
 * reported as 0); writes K to *k_out. */
pabd_status pabd_scene_residuals(pabd_scene *s, double *out, int32_t cap, int32_t *k_out);
/* Contact bonds built by the last step's collision detection (the contact bonds
 * of Sec. 4.2; geometry as read: the owner's point x_i, the partner's surface
 * point x_j, the normal and kappa_c), in a canonical order (i, j, feature).
 * Arrays of length cap (any may be NULL); *n_out is the total count. */
pabd_status pabd_scene_contacts(pabd_scene *s, int32_t cap, int32_t *ci, int32_t *cj,
                                int32_t *feature, double *xi, double *xj, double *normal,
                                double *kappa, int32_t *n_out);
/* Augmented-Lagrangian state (kappa_j, lambda_j of Sec. 5.2.2) of every bond
 * after the last step, from its i-side end ([B] each, any may be NULL; other
 * bond kinds report kappa and 0). */
pabd_status pabd_scene_bond_state(pabd_scene *s, double *kappa, double *lambda);
/* Device bytes the scene needs (admission bound for the batch); 0 for an
 * invalid descriptor. */
size_t pabd_scene_bytes(const pabd_scene_desc *desc);
/* Debug switches: bit0 = skip the local step (the global step of Sec. 4.2.1
 * alone, a block Jacobi iteration), bit1 = record the residual of every
 * iteration. */
pabd_status pabd_scene_set_debug(pabd_scene *s, int32_t flags);
/* Fault injection for tests: overwrite one component of one body's state q^n
 * or velocity (field 0..2 = c, 3..11 = A row-major, 12..14 = v, 15..17 = w)
 * after the device is idle.  PABD_E_INVALID for a body or field out of range. */
pabd_status pabd_debug_poke(pabd_scene *s, int32_t body, int32_t field, double value);
/* The same call under its earlier name. */
pabd_status pabd_scene_poke(pabd_scene *s, int32_t body, int32_t field, double value);
/* How often the local step (Sec. 4.2.2) fell back from Newton's iteration to
 * the nearest proper rotation U diag(1, 1, det U V^T) V^T of the SVD, since
 * create: *svd counts body-iterations whose A^{k+1/2} had a determinant that
 * was not safely positive or whose Newton iteration did not converge, and
 * *det_nonpositive those among them with det A^{k+1/2} <= 0 (either pointer may
 * be NULL). */
pabd_status pabd_scene_polar_fallbacks(const pabd_scene *s, int64_t *svd, int64_t *det_nonpositive);
/* the hipStream_t of the handle, as void* */
void *pabd_scene_stream(pabd_scene *s);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): pabd_scene_create, nsteps calls'
 * worth of pabd_scene_step and pabd_scene_read_state in one call, with every
 * device array of the scene taken from a static array of the library
 * (PABD_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends) instead of
 * hipMalloc; no device or pinned host memory is allocated.  The same kernels
 * in the same order as the plain path, so the results equal those of
 * create + step + read_state bit for bit.  desc as for pabd_scene_create;
 * outputs as for pabd_scene_read_state (caller-owned host arrays, any may be
 * NULL); work runs on hip_stream (NULL = the null stream) and the call returns
 * when it is done.  PABD_E_OOM, before the device is touched, when the scene
 * needs more than the static array; PABD_E_DIVERGED as read_state.  Every call
 * on one GPU uses that GPU's one array (its contents are left from the last
 * call; what must start at zero is cleared by the call): calls that overlap on
 * one GPU, from several threads or streams, race. */
#define PABD_NOALLOC_SCRATCH_BYTES (64u << 20)
pabd_status pabd_scene_run_noalloc(const pabd_scene_desc *desc, int32_t nsteps, double *c, double *A,
                                   double *v, double *w, void *hip_stream);

/* ---- batched / served path ------------------------------------------------- */

/* A batch keeps many independent scenes resident and advances all of them one
 * step per pabd_batch_step, in one replay of a captured HIP graph whose kernels
 * read the device scene table (admission changes data, not the graph).  Scenes
 * without contacts and with few bodies are packed into workgroup tiles that run
 * the whole step (prediction, K iterations, velocity recovery) from LDS.
 * All scenes of a batch share its precision. */
pabd_status pabd_batch_create(int32_t max_slots, size_t hbm_budget, int32_t precision,
                              pabd_batch **out);
pabd_status pabd_batch_destroy(pabd_batch *b);
/* Admit a scene for nsteps steps.  PABD_E_BUSY if no slot or not enough of the
 * HBM budget is free right now; the scene then stays outside (retry later). */
pabd_status pabd_batch_admit(pabd_batch *b, const pabd_scene_desc *desc, int32_t nsteps,
                             int32_t *slot);
/* One step of every resident scene that has steps left. */
pabd_status pabd_batch_step(pabd_batch *b, void *hip_stream);
/* nsteps steps (1..PABD_MAX_STEPS_PER_LAUNCH) of every resident scene, each
 * scene stopping at its own step count: the same result as nsteps calls of
 * pabd_batch_step.  Tiled scenes run all nsteps in one launch of the tile
 * kernel (a tile's bodies are loaded once and stored after every step);
 * flat-path scenes take one launch sequence per step.  Nothing can be admitted,
 * released or read between the steps of one call.  PABD_E_INVALID for nsteps
 * out of range. */
#define PABD_MAX_STEPS_PER_LAUNCH 256
pabd_status pabd_batch_steps(pabd_batch *b, int32_t nsteps, void *hip_stream);
/* Slots whose scenes finished all their steps (host bookkeeping, no sync). */
pabd_status pabd_batch_poll(pabd_batch *b, int32_t *done, int32_t cap, int32_t *n_done);
/* State of the scene in slot, as pabd_scene_read_state (PABD_E_DIVERGED when
 * that scene, and only it, produced a non-finite state or overflowed its
 * contact capacity; PABD_E_NOTFOUND for a slot not in use). */
pabd_status pabd_batch_read_state(pabd_batch *b, int32_t slot, double *c, double *A, double *v,
                                  double *w);
/* Residual of the scene in slot, as pabd_scene_residual. */
pabd_status pabd_batch_residual(pabd_batch *b, int32_t slot, double *rho_last);
/* Free the slot and its share of the HBM budget (the scene's state is lost). */
pabd_status pabd_batch_release(pabd_batch *b, int32_t slot);
/* Slots whose scene has failed, after the device is idle: slots[k] and its
 * health bits codes[k] (bit0 = non-finite state, bit1 = contact capacity
 * overflow), k < cap; *n_out is the total count.  Other scenes of the batch are
 * unaffected by a failed one (scenes never read each other's data). */
pabd_status pabd_batch_faults(pabd_batch *b, int32_t *slots, int32_t *codes, int32_t cap,
                              int32_t *n_out);
/* Fault injection for tests: as pabd_debug_poke, on body `body` of the scene in
 * slot (takes effect at the next step). */
pabd_status pabd_batch_poke(pabd_batch *b, int32_t slot, int32_t body, int32_t field, double value);
/* As pabd_scene_polar_fallbacks, for the scene in slot (counted since admit). */
pabd_status pabd_batch_polar_fallbacks(pabd_batch *b, int32_t slot, int64_t *svd,
                                       int64_t *det_nonpositive);
/* Steps taken so far by the scene in slot. */
pabd_status pabd_batch_steps_done(pabd_batch *b, int32_t slot, int32_t *steps);
/* Time candidate tile sizes on the resident scenes (their state is saved and
 * restored): the tile kernel alone, event-timed at the steps per launch the
 * batch last ran (10 before any), best of three; keep the fastest and write the
 * chosen tile size. */
pabd_status pabd_batch_autotune(pabd_batch *b, int32_t *tile_bodies);
/* Force a tile size (32, 64, 128 or 256 bodies; 0 = automatic). */
pabd_status pabd_batch_set_tile(pabd_batch *b, int32_t tile_bodies);
void *pabd_batch_stream(pabd_batch *b);
/* Block until all work enqueued on the batch's stream has finished. */
pabd_status pabd_batch_sync(pabd_batch *b);
/* Measurement: launch the tile kernel alone reps times, nsteps steps per
 * launch, on the batch's stream between two HIP events (after one untimed
 * launch) and return the average duration of one launch in ms (0 if no scene
 * is tiled).  Advances the tiled scenes like (reps + 1) * nsteps extra steps
 * would. */
pabd_status pabd_batch_time_tile_kernel(pabd_batch *b, int32_t reps, int32_t nsteps,
                                        double *avg_ms);
/* Bodies, tiles and tile size currently in the batch. */
pabd_status pabd_batch_layout(pabd_batch *b, int32_t *n_bodies, int32_t *n_tiles,
                              int32_t *tile_bodies);
/* Bytes of HBM budget in use / free. */
pabd_status pabd_batch_memory(pabd_batch *b, size_t *used, size_t *budget);

/* ---- launch schedules and the tuner --------------------------------------- */

/* How the work of Algorithm 1's iterations is laid out on the device.  The
 * body-wise update of Sec. 4.2.1 sums one term per bond end of a body; the
 * schedule says how many lanes share those ends and how many bodies share a
 * workgroup.  Results under any schedule agree with the oracle to the same
 * bounds; different schedules add a body's terms in different orders, so their
 * bits may differ (the same schedule repeats the same bits). */
typedef struct pabd_schedule {
  int32_t tile_bodies;   /* batches: bodies per workgroup of the tile kernel, 32, 64, 128
                            or 256 (0 for a plain scene, which has no tiles) */
  int32_t contact_lanes; /* lanes that share a contact body's ends on the flat path:
                            1, 2, 4, 8 or 16 (other bodies take one lane each) */
  int32_t group_waves;   /* wavefronts per workgroup of the flat-path iteration: 1, 2
                            or 4 */
  int32_t from_cache;    /* output of the tuners: 1 when the schedule came from the
                            tuning cache instead of timing */
} pabd_schedule;

/* flags of the tuners: time the candidates even when the cache holds the key */
#define PABD_TUNE_FORCE 1

/* Pick a batch's schedule by timing, on the scenes resident now (their state,
 * bond states, health bits and residuals are saved first and restored after
 * every candidate, so the scenes continue as if the call had not been made).
 * First the tile size: when every scene is one the tile kernel can take, the
 * sizes that hold the largest, timed on the tile kernel alone (as
 * pabd_batch_autotune); otherwise every size whose placement fits, timed as
 * whole batch steps (a smaller tile moves the larger chains to the flat path).
 * Then, when contact scenes run on the flat path, contact_lanes from {1, 2, 4,
 * 8, 16}; then, when any scene runs on the flat path, group_waves from {1, 2,
 * 4}.  Whole batch steps are one graph replay each, timed with HIP events,
 * best of three rounds of four steps from the saved state; a candidate
 * replaces the schedule in force only when it is more than 3 % faster.  The
 * result is kept in a per-process cache under (device architecture, precision, size bucket): the
 * bit lengths of the body counts of the scenes the tile kernel can take (joint
 * scenes without contacts, driven or variable bonds), of the contact scenes
 * and of the other scenes, the bit length of the largest contact capacity, and
 * the smallest tile size that holds the largest scene the tile kernel can
 * take.  A later call with the same key applies the cached schedule without
 * timing (unless flags has PABD_TUNE_FORCE).  Writes the schedule in force to
 * *out (may be NULL).  Blocks until the device is idle, and steps the scenes
 * only inside the saved-and-restored timing rounds.  PABD_E_INVALID for a null
 * batch; PABD_E_DEVICE when a device call fails and PABD_E_OOM when a re-placed
 * layout does not fit (then the batch's state is undefined: release its
 * scenes). */
pabd_status pabd_batch_tune(pabd_batch *b, int32_t flags, pabd_schedule *out);
/* Apply a schedule to a batch (tile_bodies 0 leaves the tile size as it is;
 * from_cache is ignored): a new tile size re-places every scene, keeping its
 * state and bond states; the next step recaptures its graph.  PABD_E_INVALID
 * for a value outside the sets above or a null argument. */
pabd_status pabd_batch_set_schedule(pabd_batch *b, const pabd_schedule *s);
pabd_status pabd_batch_get_schedule(const pabd_batch *b, pabd_schedule *out);
/* The same for a plain scene: contact_lanes, then group_waves, each timed over
 * whole steps from the saved state (with the same 3 % margin).  A scene whose
 * whole step runs in the resident kernel (small scenes) has no flat-path launch to tune: the call
 * writes the schedule in force and times nothing.  Cache key: (device
 * architecture, precision, bit length of the body count, contact flag, bit
 * length of the contact capacity). */
pabd_status pabd_scene_tune(pabd_scene *s, int32_t flags, pabd_schedule *out);
/* (tile_bodies and from_cache are ignored; a scene reads back tile_bodies 0;
 * errors as for the batch) */
pabd_status pabd_scene_set_schedule(pabd_scene *s, const pabd_schedule *sch);
pabd_status pabd_scene_get_schedule(const pabd_scene *s, pabd_schedule *out);
/* Empty the tuning cache / number of entries in it. */
void pabd_tune_cache_clear(void);
int32_t pabd_tune_cache_size(void);

/* ---- measurement ------------------------------------------------------------ */

/* Device-wide streaming copy of `bytes` (rounded down to 16-byte units) between
 * two library-owned buffers, timed with HIP events over `reps` launches on the
 * library's probe stream: the achievable-HBM-bandwidth reference and the
 * calibration kernel for hardware traffic counters.  Writes GB/s of read+write
 * traffic (2 * bytes per launch) and the average launch duration in ms. */
pabd_status pabd_hbm_copy_probe(size_t bytes, int32_t reps, double *gbps, double *avg_ms);

#ifdef __cplusplus
}
#endif

#endif
