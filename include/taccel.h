/* taccel: incremental-potential-contact (IPC) time step of a tetrahedral neo-Hookean gel
 * pad in contact with affine (ABD) rigid bodies, on AMD Instinct MI355X (gfx950).
 *
 * Method: Taccel, arXiv 2504.12908.  One call of taccel_step / taccel_batch_step advances
 * every scene by one backward-Euler step, x^{n+1} = argmin E(x) with
 *   E = 1/2 |x - x^n - h v^n|^2_M + h^2 (Phi_neoHookean + E_ext) + h^2 kappa sum_k b(d_k)
 * plus the affine-body terms and kinematic constraints (Sec. 3.2 Eq. 1, Sec. 3.3 Eq. 3-5,
 * Sec. 3.4 Eq. 6; App. A.1-A.5; barrier App. A.3 Eq. A6).  The minimiser is found by Newton's
 * method (element Hessians projected to positive semidefinite away from the minimiser, exact
 * near it) with preconditioned CG (block Jacobi plus a rigid-mode coarse level), additive CCD
 * and a backtracking line search.
 *
 * Conventions: SI units; 0-based int32 indices; arrays written [n][k] are row-major,
 * host memory unless a name ends in _device.  Inputs are borrowed for the duration of the
 * call and copied; the library owns all device state of a scene/batch until destroy.  No
 * exceptions cross this boundary.  A scene or batch is not thread-safe; distinct objects on
 * distinct streams are.
 */
#ifndef TACCEL_H
#define TACCEL_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TACCEL_OK = 0,
  TACCEL_ERR_ARG = 1,              /* bad sizes, indices, degenerate/inverted tets, open body */
  TACCEL_ERR_HIP = 2,              /* HIP runtime failure (message in taccel_last_error) */
  TACCEL_NOT_CONVERGED = 3,        /* Newton did not reach the tolerance in max_newton iterations */
  TACCEL_LINESEARCH_FAILED = 4,    /* step size fell below 1e-12 */
  TACCEL_AL_FAILED = 5,            /* kinematic targets not met after max_al rounds */
  TACCEL_NAN = 6,                  /* non-finite gradient or singular preconditioner */
  TACCEL_INFEASIBLE_TARGET = 7,    /* moving Dirichlet targets would collide or invert */
  TACCEL_ERR_OOM = 8,              /* device allocation failed */
  TACCEL_INFEASIBLE = 9,           /* initial state interpenetrates or is inverted */
  TACCEL_CANCELLED = 10            /* server request dropped by taccel_server_destroy */
} taccel_status;

/* MIXED: FP32 Hessian blocks, assembly, SpMV and PCG; FP64 positions, gradient, contact,
 * CCD and convergence test.  A batch with more than one scene must use FP64 or
 * FP64_REFINED (ERR_ARG).
 * FP64_REFINED: every term, block and the assembly as in FP64 mode; the PCG iterations run
 * on an FP32 copy of the FP64 system (half the bytes per sparse product), and the FP64
 * residual of the system decides whether another FP32 pass solves for a correction
 * (mixed-precision iterative refinement, the stronger-solver item of the paper's stated PCG
 * bottleneck, Sec. 7), so the Newton direction meets the FP64 tolerance. */
typedef enum { TACCEL_FP64 = 0, TACCEL_MIXED = 1, TACCEL_FP64_REFINED = 2 } taccel_precision;

/* Soft body (the gel pad): nv rest vertices, nt tets of positive orientation.
 * dirichlet[i]: 0 free, 1 fixed, 2 moving (position prescribed each step); NULL = all free.
 * Young's modulus E, Poisson ratio nu (neo-Hookean, Sec. 3.1), density rho (lumped mass). */
typedef struct {
  int32_t nv;
  const double* verts;      /* [nv][3] rest = initial positions */
  int32_t nt;
  const int32_t* tets;      /* [nt][4] */
  const uint8_t* dirichlet; /* [nv] or NULL */
  double youngs, poisson, density;
} taccel_soft_desc;

/* Affine body (Sec. 3.3): closed, outward-oriented triangle mesh given by its world vertex
 * positions at creation.  Mass properties come from its enclosed volume.  prescribed = 1:
 * the body follows a kinematic target each step (augmented Lagrangian, Sec. 3.4). */
typedef struct {
  int32_t nv;
  const double* verts;   /* [nv][3] */
  int32_t nf;
  const int32_t* tris;   /* [nf][3], local indices */
  double density;
  int32_t prescribed;
} taccel_body_desc;

typedef struct {
  double h;           /* time step (s) */
  double dhat;        /* barrier activation distance (m) */
  double kappa;       /* barrier stiffness */
  double kappa_s;     /* affine-body ARAP stiffness (Pa) */
  double newton_tol;  /* Newton stops when max |dx| <= newton_tol * h * L (L: rest bbox diag) */
  double gravity[3];
  int32_t max_newton; /* per Newton loop; 0 -> 100 */
  int32_t max_al;     /* augmented-Lagrangian rounds; 0 -> 30 */
  int32_t max_pcg;    /* 0 -> 10000 */
  double pcg_eta;     /* relative residual of PCG; 0 -> 1e-4 (FP64, FP64_REFINED) or 1e-3
                         (MIXED) */
  int32_t precision;  /* taccel_precision.  MIXED: Hessian blocks, their assembly, the sparse
                         product and the whole PCG in FP32 (FP32 accumulation); positions,
                         gradients, energies, distances, barrier, CCD, line search and the
                         Newton test in FP64.  All scenes of a batch share one precision. */
  double friction;    /* Coulomb coefficient mu of the lagged friction potential D (Taccel
                         App. A.3); 0: frictionless (no friction work at all).  >= 0. */
  double eps_v;       /* velocity threshold (m/s) between static and sliding friction in the
                         mollifier f1; must be > 0 when friction > 0. */
  int32_t pcg_forcing; /* 0: every Newton system is solved to pcg_eta.  1: inexact Newton with
                         Eisenstat-Walker forcing terms (the paper's relaxed convergence
                         tolerances, Sec. 7): the first iteration of each Newton loop is
                         solved to 0.01, iteration k to 0.9 (g_k'D^-1 g_k)/(g_k-1'D^-1 g_k-1)
                         (not below 0.9 eta_k-1^2 when that exceeds 0.1), clamped to
                         [pcg_eta, 0.01].  The converged state meets the same Newton test. */
} taccel_params;

typedef struct {
  taccel_soft_desc soft;
  int32_t n_bodies;
  const taccel_body_desc* bodies;
  taccel_params params;
} taccel_scene_desc;

/* Device memory and stream.  alloc/free may be NULL (then hipMalloc/hipFree).  stream NULL:
 * the library creates a non-blocking stream of default priority for the object.  The device
 * work of a scene/batch is ordered on that stream (the PCG loop is replayed from a HIP graph
 * captured on it, so it must not be the legacy null stream); inside a Newton iteration two
 * more streams of the object's own (default priority) take part of the derivative work and
 * are joined back to it by events before anything later depends on them, so every call still
 * returns with its work complete. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
  void* stream; /* hipStream_t */
} taccel_runtime;

/* Kinematic targets for one step of one scene.
 * body_targets: [n_bodies][12] = (t[3], A row-major[9]); a creation-pose vertex X0 of a
 *   prescribed body is to be at A X0 + t at the end of the step (ignored for free bodies).
 * dirichlet_targets: [n_moving][3] end-of-step positions of the vertices flagged 2, in
 *   increasing vertex order.  Either pointer may be NULL if there is nothing to prescribe. */
typedef struct {
  const double* body_targets;
  const double* dirichlet_targets;
} taccel_targets;

typedef struct {
  int32_t status;        /* taccel_status of this scene */
  int32_t newton_iters;  /* summed over the step's Newton loops */
  int32_t al_rounds;     /* Newton loops of the step */
  int32_t pcg_iters;     /* summed PCG iterations */
  int32_t n_active;      /* contact pairs with d < dhat in the last Newton iteration */
  int32_t ls_halvings;   /* summed line-search halvings */
  double step_ms;        /* wall time of the call (batch: same for all scenes) */
} taccel_step_stats;

typedef enum {
  TACCEL_FIELD_X = 0,    /* double[nv][3] soft-vertex positions */
  TACCEL_FIELD_V = 1,    /* double[nv][3] soft-vertex velocities */
  TACCEL_FIELD_Q = 2,    /* double[n_bodies][12] body maps (t, A row-major) of creation pose */
  TACCEL_FIELD_QDOT = 3, /* double[n_bodies][12] their rates */
  TACCEL_FIELD_BODY_X = 4, /* double[sum body nv][3] body vertex world positions (read only) */
  TACCEL_FIELD_CONTACTS = 5, /* int32[n_active][5] (read only): the contact pairs closer than
                            dhat at the current positions (Sec. 3.2 Eq. 2: the active set of
                            the barrier sum), each as kind (0 point-triangle, 1 edge-edge) and
                            four world vertex ids (soft vertices 0..nv-1, then the body
                            vertices in order) in the order of taccel_debug_candidates, the
                            records sorted.  Its size changes with the state: ask
                            taccel_state_bytes first. */
  TACCEL_FIELD_STATS = 6 /* taccel_step_stats of the scene's last step (read only; zeros
                            before the first step and after a reset) */
} taccel_field;

typedef struct taccel_scene taccel_scene;
typedef struct taccel_batch taccel_batch;

/* Create one scene.  rt may be NULL.  Errors: ARG (bad sizes/indices, degenerate or
 * inverted tets, body without positive volume), INFEASIBLE (some admissible contact pair is
 * at distance 0), OOM, HIP. */
taccel_status taccel_scene_create(const taccel_scene_desc* d, const taccel_runtime* rt,
                                  taccel_scene** out);
/* Advance one time step (synchronous: returns after the device work is done).  targets may
 * be NULL when nothing is prescribed.  On a failure status the scene is rolled back to the
 * start of the step; stats (nullable) is filled in any case. */
taccel_status taccel_step(taccel_scene* s, const taccel_targets* targets, taccel_step_stats* stats);
/* Copy a field to caller-owned host memory; bytes must equal the field size (else ARG). */
taccel_status taccel_state_read(const taccel_scene* s, taccel_field f, void* dst, size_t bytes);
/* Overwrite X, V, Q or QDOT (reset / resume).  The augmented-Lagrangian multipliers of the
 * prescribed bodies (Sec. 3.4, App. A.5), which otherwise carry over from one accepted step to
 * the next as a starting guess, are cleared by a write of Q and by a failed step. */
taccel_status taccel_state_write(taccel_scene* s, taccel_field f, const void* src, size_t bytes);
void taccel_scene_destroy(taccel_scene* s);
/* Current size in bytes of a field (CONTACTS: computed from the current positions). */
taccel_status taccel_state_bytes(const taccel_scene* s, taccel_field f, size_t* bytes);
/* Device-pointer variant of taccel_state_read: writes the same bytes to device memory dst
 * (on this scene's device), in an operation ordered on the scene's stream, and returns after
 * it completes.  Fields X, V, Q, QDOT and BODY_X; ARG for a size mismatch or another field. */
taccel_status taccel_state_read_device(const taccel_scene* s, taccel_field f, void* dst,
                                       size_t bytes);
/* Back to the creation state (the paper's API resets environments, Sec. 4.3): rest positions,
 * zero velocities, every body at its creation pose at rest, multipliers cleared, STATS zero. */
taccel_status taccel_scene_reset(taccel_scene* s);

/* n independent scenes solved together: every stage is one launch over all scenes,
 * reductions are per scene, a scene that fails is rolled back without affecting others. */
taccel_status taccel_batch_create(const taccel_scene_desc* descs, int32_t n,
                                  const taccel_runtime* rt, taccel_batch** out);
/* targets: [n] (NULL = none); per_scene (nullable): [n] statuses; stats (nullable): [n].
 * Returns OK if every scene succeeded, else the first failing scene's status. */
taccel_status taccel_batch_step(taccel_batch* b, const taccel_targets* targets,
                                taccel_status* per_scene, taccel_step_stats* stats);
taccel_status taccel_batch_read(const taccel_batch* b, int32_t scene, taccel_field f, void* dst,
                                size_t bytes);
taccel_status taccel_batch_write(taccel_batch* b, int32_t scene, taccel_field f, const void* src,
                                 size_t bytes);
taccel_status taccel_batch_state_bytes(const taccel_batch* b, int32_t scene, taccel_field f,
                                      size_t* bytes);
taccel_status taccel_batch_read_device(const taccel_batch* b, int32_t scene, taccel_field f,
                                       void* dst, size_t bytes);
/* taccel_scene_reset for the scenes with mask[k] != 0 ([n] host bytes; NULL: all scenes). */
taccel_status taccel_batch_reset(taccel_batch* b, const uint8_t* mask);
void taccel_batch_destroy(taccel_batch* b);

/* ---- Tactile outputs of the current state (Taccel Sec. 4.2) ----------------------------
 * Markers: marker k lies on the soft-body triangle tris[k][0..2] (the caller's soft vertex
 * ids) at barycentric coordinates bary[k][0..2] (each in [0, 1]).  Writes its current
 * position pos[k][3] = sum_u bary[k][u] x[tris[k][u]] and its flow flow[k][3] = pos[k] minus
 * the same combination of the rest positions.  All arrays are host memory of m entries;
 * TACCEL_ERR_ARG for an id out of range or a coordinate outside [0, 1]. */
taccel_status taccel_markers(const taccel_scene* s, int32_t m, const int32_t* tris,
                             const double* bary, double* pos, double* flow);
taccel_status taccel_batch_markers(const taccel_batch* b, int32_t scene, int32_t m,
                                   const int32_t* tris, const double* bary, double* pos,
                                   double* flow);

/* Image plane of a depth map: pixel (i, j) (row i < height, column j < width) is the ray from
 * origin + (j + 1/2) pixel axis_u + (i + 1/2) pixel axis_v along axis_n = axis_u x axis_v.
 * axis_u and axis_v must be orthonormal (to 1e-9); width * height <= 2^26. */
typedef struct {
  double origin[3];
  double axis_u[3];
  double axis_v[3];
  double pixel;  /* pixel pitch (m) */
  int32_t width, height;
} taccel_camera;

/* Depth and normal maps of the deformed surface given by ntri triangles tris[ntri][3] (the
 * caller's soft vertex ids; e.g. the pad's coated face), seen orthographically from the
 * camera's image plane.  A triangle covers a pixel when the pixel centre lies in its
 * projection onto the plane (edges included).  depth[i][j] is the smallest ray parameter
 * over the covering triangles (+inf where none covers); normal[i][j][3] is the unit normal
 * of the covering triangle that attains it (the lowest index on ties), turned to face the
 * image plane (normal . axis_n <= 0), zero where none covers.  The coverage and depth
 * arithmetic is plain IEEE FP64 without fused multiply-add, so any evaluation of the same
 * expressions reproduces every pixel bit for bit.  depth: [height][width], normal:
 * [height][width][3], host memory. */
taccel_status taccel_depth_map(const taccel_scene* s, const taccel_camera* cam, int32_t ntri,
                               const int32_t* tris, double* depth, double* normal);
taccel_status taccel_batch_depth_map(const taccel_batch* b, int32_t scene,
                                     const taccel_camera* cam, int32_t ntri,
                                     const int32_t* tris, double* depth, double* normal);

/* ---- Serving: continuous batching of time-step requests -------------------------------
 * A request is one scene plus a script of n_steps per-step targets (a rollout, e.g. one
 * tactile press-and-slide episode, Sec. 5).  Requests are admitted in arrival order into
 * cohorts: a cohort is one resident batch (as taccel_batch_*) with its own stream and host
 * thread that advances all its unfinished requests by one step per call; a request that
 * finishes or fails stops being stepped while the others go on, and the cohort's device
 * memory is released with its last request.  A new cohort is formed whenever requests are
 * waiting, fewer than max_cohorts run, and the estimated footprint of the requests taken fits
 * hbm_budget_bytes minus what running cohorts hold, so cohorts formed at different times
 * run concurrently.  Waiting requests also take the slots that finished requests leave in a
 * running cohort (FP64 cohorts): at a step boundary its unfinished requests and the newly
 * admitted ones (same precision, within the cohort's reservation) form a new batch into which
 * the unfinished requests' state moves bit for bit.  A request's results are bitwise the same
 * as stepping its scene alone with taccel_step.  All calls are thread-safe. */
typedef struct {
  double hbm_budget_bytes; /* device memory the server may hold (> 0) */
  int32_t max_cohort;      /* requests per cohort (<= 0: 64) */
  int32_t max_cohorts;     /* cohorts running at once (<= 0: 8) */
  double coalesce_ms;      /* wait before forming a cohort so near-simultaneous arrivals
                              share it (<= 0: 1 ms) */
} taccel_server_params;

typedef struct {
  uint64_t req_id;
  int32_t status;      /* OK, or the status of the failing step (the request stops there),
                          ERR_OOM (can never fit the budget), INFEASIBLE, CANCELLED, ... */
  int32_t n_steps;     /* steps requested */
  int32_t steps_done;  /* steps attempted (the last one failed if status != OK) */
  double wait_ms;      /* submit -> admission into a cohort */
  double run_ms;       /* admission -> completion */
  double mean_step_ms; /* per-step latency of the cohort calls that stepped this request */
  double max_step_ms;
} taccel_completion;

typedef struct taccel_server taccel_server;

/* rt (nullable): alloc/free/ctx apply to every cohort; rt->stream is ignored (each cohort
 * creates its own).  Errors: ARG. */
taccel_status taccel_server_create(const taccel_server_params* p, const taccel_runtime* rt,
                                   taccel_server** out);
/* Queue a request; d and per_step ([n_steps], NULL if nothing is prescribed) are copied.
 * The scene is checked on the host now (ARG and its message, nothing queued); checks that
 * need the device (INFEASIBLE) are reported through its completion. */
taccel_status taccel_server_submit(taccel_server* s, const taccel_scene_desc* d, int32_t n_steps,
                                   const taccel_targets* per_step, uint64_t* req_id);
/* Move up to cap completions (in completion order) into out, waiting up to wait_ms for the
 * first one if none is ready; *n = number written. */
taccel_status taccel_server_poll(taccel_server* s, taccel_completion* out, int32_t cap, int32_t* n,
                                 int32_t wait_ms);
/* Final state of a completed request: fields X, V, Q, QDOT as taccel_state_read (after the
 * last successful step).  ARG if unknown, unfinished or released, or on a size mismatch. */
taccel_status taccel_server_read(taccel_server* s, uint64_t req_id, taccel_field f, void* dst,
                                 size_t bytes);
/* Wall time of each step call of a completed request: up to cap values, *n = steps. */
taccel_status taccel_server_step_latencies(taccel_server* s, uint64_t req_id, double* out,
                                           int32_t cap, int32_t* n);
/* Forget a completed request (its final state and latencies). */
taccel_status taccel_server_release(taccel_server* s, uint64_t req_id);
/* Requests waiting for admission, cohorts running, the device bytes reserved by the running
 * cohorts (a cohort reserves the estimated footprint of its requests, or what its creation
 * took if more; its buffers may grow with its contacts up to that and no further: a step that
 * would need more fails its requests with ERR_OOM, so the reservations never pass the budget)
 * and the peak of the bytes the cohorts actually held (any pointer may be NULL). */
taccel_status taccel_server_info(taccel_server* s, int32_t* queued, int32_t* running_cohorts,
                                 double* used_bytes, double* peak_bytes);
/* Cancel queued requests, stop running cohorts after their current step (their requests
 * complete as CANCELLED), wait for all threads and free everything. */
void taccel_server_destroy(taccel_server* s);

/* Thread-local text of the last error of this thread (empty if none). */
const char* taccel_last_error(void);
const char* taccel_status_str(taccel_status s);

/* ---- Element evaluators (run the solver's own device code; for tests) -------------------
 * Neo-Hookean tets: rest, x [n][4][3]; outputs e [n] (V Psi), g [n][12], H and Hp [n][12][12]
 * (unprojected / projected Hessian of V Psi).  Any output may be NULL. */
taccel_status taccel_debug_fem(int32_t n, const double* rest, const double* x, double youngs,
                               double poisson, double* e, double* g, double* H, double* Hp);
/* Barrier pairs: kinds [n] (0 point-triangle, 1 edge-edge), x [n][4][3] in local order
 * (PT: p,t0,t1,t2; EE: a0,a1,b0,b1), mollifier_eps [n] (EE: 1e-3 |a|^2_rest |b|^2_rest).
 * Outputs kappa*m*b(d), gradient, Hessians, distance type.  Any output may be NULL. */
taccel_status taccel_debug_barrier(int32_t n, const int32_t* kinds, const double* x,
                                   const double* mollifier_eps, double dhat, double kappa,
                                   double* e, double* g, double* H, double* Hp, int32_t* types);
/* Friction potential of n pairs (Taccel App. A.3).  Per pair: kind, the start-of-step
 * configuration xn [n][12] from which the lagged data are taken (closest-point weights of
 * the closest features, unit normal, lambda = -kappa m b'(d) with m the edge-edge mollifier
 * value for mollifier_eps [n]) and the current configuration x [n][12].  Outputs lambda [n]
 * (0 for a pair not closer than dhat), the energy mu lambda f0(|u|) [n], its gradient
 * [n][12] and Hessian [n][12][12] (no h^2 factor; u is the tangential part of the change of
 * the closest-point difference), with eps_v_h = eps_v * h.  All arrays are host memory. */
taccel_status taccel_debug_friction(int32_t n, const int32_t* kinds, const double* xn,
                                    const double* x, const double* mollifier_eps, double dhat,
                                    double kappa, double mu, double eps_v_h, double* lambda,
                                    double* e, double* g, double* H);
/* Additive CCD of n pairs moving linearly by p: largest safe fraction t in [0,1]. */
taccel_status taccel_debug_ccd(int32_t n, const int32_t* kinds, const double* x, const double* p,
                               double gap_ratio, int32_t max_iter, double* t);
/* ARAP term |A - R(A)|^2 of n 3x3 matrices (row-major): e, g [n][9], H, Hp [n][9][9]. */
taccel_status taccel_debug_arap(int32_t n, const double* A, double* e, double* g, double* H,
                                double* Hp);
/* Newton system of the scene's first Newton iteration of its next step (Sec. 3.2 Eq. 1 with
 * Sec. 3.3-3.4 and App. A.2-A.5: the incremental potential with barrier, affine-body and
 * constraint terms): the step is begun as taccel_step would begin it with these targets
 * (prediction, moving Dirichlet vertices, body targets, bodies already on their target
 * fixed), the pairs closer than dhat are found, and the gradient and the projected Hessian
 * are assembled exactly as the solver assembles them; then the scene is put back where it was
 * (its carried multipliers cleared, as after a failed step).  Nodes are numbered in the
 * caller's terms: soft vertex i is node i, body b has nodes nv + 4b + (0: its centre-of-mass
 * position p, 1-3: the columns c1, c2, c3 of its affine map).  grad [nv + 4 nb][3]
 * (nullable) is zero at nodes that are not unknowns (fixed or moving vertices, fixed bodies);
 * the Hessian comes as 3x3 blocks (row node, column node, 9 values row-major), sorted by
 * (row, column), both nodes unknowns, duplicates summed: up to cap of them are written and
 * *n_blocks gets their number.  Single scene only; ARG otherwise, INFEASIBLE_TARGET when the
 * targets cannot be reached. */
taccel_status taccel_debug_system(taccel_scene* s, const taccel_targets* t, double* grad,
                                  int32_t* brow, int32_t* bcol, double* bval, int32_t cap,
                                  int32_t* n_blocks);
/* Broad phase of a scene on given world positions P0 (and P1 for the swept test, or NULL):
 * world vertex ids are soft vertices 0..nv-1 then body vertices in order.  Writes up to cap
 * candidates as 5 int32 (kind, four world ids: PT point + sorted triangle; EE sorted edges,
 * smaller edge first) and the total count to *n. */
taccel_status taccel_debug_candidates(taccel_scene* s, const double* P0, const double* P1,
                                      int32_t* out, int32_t cap, int32_t* n);

/* ---- Measurement --------------------------------------------------------------------
 * Process-wide timing, off by default (it adds synchronisations).  taccel_profile_enable(flags):
 * bit 0 turns on the kernel timings "spmv" and "pcg", bit 1 the phase timings.  While enabled:
 *   "spmv": on every Newton iteration, 16 back-to-back launches of the PCG sparse-product
 *     kernel on that iteration's matrix are timed between two events on the object's stream
 *     (their outputs are recomputed by the solve); query returns the summed milliseconds, the
 *     number of launches and the summed algorithmic bytes (values, indices and vectors the
 *     product must move once);
 *   "pcg": the PCG iterations of every solve (after initialisation) between two events;
 *     query returns the summed milliseconds and iterations (largest count per solve);
 *   "refine" (FP64_REFINED, counted while bit 0 is on): query returns 0 ms, the number of
 *     FP32 passes as launches and the number of Newton directions they solved as
 *     algorithmic_bytes (passes per direction = launches / that count);
 *   "candidates", "derivatives", "solve", "check", "ccd", "line_search": host wall time of
 *     each phase of a Newton iteration (static candidates and narrow phase; element
 *     derivatives, assembly and preconditioner; PCG; convergence test; swept candidates and
 *     CCD; line search and update), each ended by a stream synchronisation; query returns
 *     the summed milliseconds and the number of Newton iterations. */
void taccel_profile_enable(int32_t on);
void taccel_profile_reset(void);
taccel_status taccel_profile_query(const char* kernel, double* total_ms, int64_t* launches,
                                   double* algorithmic_bytes);
/* hipDeviceSynchronize on the current device. */
taccel_status taccel_device_synchronize(void);

#ifdef __cplusplus
}
#endif
#endif
