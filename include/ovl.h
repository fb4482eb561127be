/* ovl.h - C ABI of the MI355X overlapping-partition rigid-body stepper.
 *
 * The library steps rigid bodies with the overlapping-partition method of
 * Kale & Kry, "Distributed Simulation of Large Multi-body Systems"
 * (arXiv 2403.17261).  The paper's workers become independent sub-solves
 * ("partitions") on one GPU; every step runs, on the device:
 *   contacts (Alg. 1 getContacts) -> constraint graph (section 5.1) ->
 *   overlap sets (section 4, Eq. 9-10; Alg. 2-3 read as a k-hop halo) ->
 *   geodesic weights (section 5.3, Eq. 15-16, Alg. 5) -> per-partition MLCP
 *   rows (section 3, Eq. 1-7) -> graph colouring -> projected Gauss-Seidel ->
 *   integration -> blending of the overlap bodies (section 5.2, Eq. 11-14,
 *   Alg. 4), which also resets every replica for the next step (Alg. 1).
 *
 * Conventions
 *  - All pointers are plain host pointers unless a `*_is_device` flag says
 *    otherwise.  Input arrays are borrowed for the duration of the call and
 *    copied; the library never keeps a caller pointer.
 *  - A body state is 13 float32 in the paper's order (section 4, Eq. 8):
 *    position x(3), rotation quaternion q(4, scalar first), linear velocity
 *    v(3), angular velocity w(3), all in the world frame.  State arrays are
 *    row-major [n_bodies][13].
 *  - Bodies are sorted by scene id; the scenes of one world never interact.
 *    Partition ids are global: scene s owns the contiguous range
 *    [base_s, base_s + parts_per_scene[s]) with base_s the sum of the earlier
 *    scenes' counts.  A scene has 1..64 partitions.
 *  - Every call returns an ovl_status; no exception crosses the ABI.  The
 *    text of the last error of a world is returned by ovl_last_error().
 *  - A world belongs to one host thread and one HIP stream.
 */
#ifndef OVL_H
#define OVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OVL_OK = 0,
  OVL_ERR_INVALID_ARG = 1, /* a size, index or flag is out of range */
  OVL_ERR_OOM = 2,         /* device allocation failed */
  OVL_ERR_CAPACITY = 3,    /* a per-step buffer overflowed and could not be grown */
  OVL_ERR_NONFINITE = 4,   /* a step produced NaN/Inf; the state stays at the last good step */
  OVL_ERR_DEVICE = 5,      /* a HIP call failed */
  OVL_NOT_CONVERGED = 6    /* informational: some partition hit the iteration cap in adaptive mode */
} ovl_status;

typedef struct ovl_world ovl_world;

/* Scene content of a world (section 4: the set of non-static bodies plus
 * static bodies of infinite mass).  Bodies are spheres (shape 0, isotropic
 * inertia) or capsules (shape 1: the segment of half-length halflen along the
 * body z axis swept by the radius; inertia symmetric about body z). */
typedef struct {
  int32_t n_bodies;            /* N >= 0 */
  int32_t n_scenes;            /* S >= 1 */
  int32_t n_joints;            /* J >= 0 */
  const int32_t* scene;        /* [N] scene id, nondecreasing */
  const int32_t* shape;        /* [N] 0 = sphere, 1 = capsule */
  const float* radius;         /* [N] > 0 */
  const float* halflen;        /* [N] capsule half-length > 0; unused for spheres (may be NULL without capsules) */
  const float* mass;           /* [N] > 0 */
  const float* inertia;        /* [N*3] body-frame principal moments (sphere: all equal; capsule: I_x = I_y) */
  const float* state;          /* [N*13] initial states */
  const float* mu;             /* [S] Coulomb friction coefficient (section 3, Eq. 5-7) */
  const float* margin;         /* [S] contact margin: a pair is in contact when its gap < margin */
  const int32_t* plane_off;    /* [S+1] planes of scene s: [plane_off[s], plane_off[s+1]) */
  const float* planes;         /* [P*4] static planes n.x = c (n unit, pointing to the free side) */
  const int32_t* ssph_off;     /* [S+1] */
  const float* ssph;           /* [Q*4] static spheres: centre(3), radius */
  const int32_t* joint_ab;     /* [J*2] ball joints between two bodies of one scene, sorted by scene */
  const float* joint_anchor;   /* [J*6] body-frame anchor on body a, then on body b */
} ovl_world_desc;

enum { OVL_MODE_FIXED = 0, OVL_MODE_ADAPTIVE = 1 };
enum { OVL_WARM_NONE = 0, OVL_WARM_PLAIN = 1, OVL_WARM_LEARNED = 2 };
/* Blend weights of the overlap bodies: geodesic (section 5.3, Eq. 15-16,
 * Alg. 5) or equal 1/|W| (the naive weights section 5.3 compares against). */
enum { OVL_WEIGHTS_GEODESIC = 0, OVL_WEIGHTS_EQUAL = 1 };
/* Interface coupling between partitions (section 7 names it as a way to
 * couple the workers' solutions beyond the overlap, after [BW97]).
 * OVL_COUPLING_PREV_IMPULSE: a constraint of the step between two dynamic
 * bodies of which only one is active in partition i is left out of i's solve
 * (section 4); with this option its impulse of the previous step still acts
 * on the body inside i, as a fixed impulse added to the body's free velocity
 * v + h M^-1 f before the warm start and the sweeps.  The impulse is the one
 * the constraint left, at the end of the previous step, in the partition
 * with the lowest id among those active in both of its bodies (found by the
 * warm start's key; a contact's friction is carried as a world vector,
 * projected on the new tangents and clipped to the new friction box, its
 * normal impulse clamped to >= 0); none if that partition did not solve it
 * then.  The features of the learned warm start see the coupled velocity.
 * OVL_COUPLING_MASS_SPLIT: the workers share the mass of an overlap body
 * (section 2 relates the blend to the mass splitting of [TBV12]).  The
 * replica of an overlap body in partition i carries the share w_i of the
 * body's mass and inertia, w_i being its blend weight (inverse mass and
 * inverse inertia divided by w_i; a replica of weight 0 keeps the whole
 * body), in the rows, the sweeps, the residuals and the learned features.
 * The blend sum_i w_i v_i then applies the sum of the partitions' impulses
 * to the whole body, so a partitioned step conserves momentum where the
 * constraint impulses are equal and opposite. */
enum { OVL_COUPLING_NONE = 0, OVL_COUPLING_PREV_IMPULSE = 1, OVL_COUPLING_MASS_SPLIT = 2 };

/* Parameters of the warm-start network 12 -> 64 -> 64 -> 3 (ReLU), flat:
 * W1[12][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3], input index first. */
#define OVL_MLP_PARAMS 5187

/* Step parameters.  Eq. 2's compliance C is cfm * identity; its
 * stabilisation term is applied as erp * phi / h for penetrations and phi / h
 * for open gaps.  Adaptive mode stops a partition's Gauss-Seidel sweeps when
 * the largest |A_rr * delta lambda_r| of a sweep is <= tol (m/s), capped at
 * max_iters; fixed mode runs exactly max_iters sweeps. */
typedef struct {
  float dt;           /* time step h (s) */
  float gravity[3];   /* m/s^2 */
  float cfm;          /* >= 0 */
  float erp;          /* in [0, 1] */
  float tol;          /* adaptive stop threshold, m/s */
  int32_t max_iters;  /* >= 1 (cap 100000) */
  int32_t mode;       /* OVL_MODE_* */
  int32_t warmstart;  /* OVL_WARM_* */
  uint32_t seed;      /* colouring priority seed */
  int32_t weights;    /* OVL_WEIGHTS_* */
  int32_t coupling;   /* OVL_COUPLING_* */
} ovl_params;

/* Device context: the stream every kernel runs on (NULL = the null stream)
 * and optional allocation callbacks (NULL = hipMalloc/hipFree).  The Python
 * binding passes PyTorch's current stream and caching allocator. */
typedef struct {
  void* stream;                                  /* hipStream_t */
  void* (*alloc)(size_t bytes, void* user);      /* returns device memory or NULL */
  void (*free)(void* ptr, void* user);
  void* user;
} ovl_device_ctx;

/* Per-call statistics of the last step (totals where marked). */
typedef struct {
  int64_t n_contacts;      /* contacts found (Alg. 1 getContacts) */
  int64_t n_copies;        /* constraint copies summed over partitions */
  int64_t n_replicas;      /* body replicas summed over partitions */
  int64_t n_overlap;       /* bodies active in >= 2 partitions (the overlap set O, Eq. 10) */
  int32_t max_colours;     /* largest colour count of a partition */
  int32_t max_iters;       /* largest sweep count of a partition */
  int32_t n_unconverged;   /* partitions that hit the cap in adaptive mode */
  int32_t steps;           /* steps run by the call */
  int64_t iters_total;     /* total over the call's steps of the largest sweep count */
  float resid_sweep;       /* largest last-sweep residual max |A_rr dlambda| over partitions (m/s) */
  float resid_exact;       /* natural-map residual of the final iterate (computed when requested) */
  int64_t n_lb_changes;    /* contacts whose load-balancing rule changed a worker set (last step) */
  /* computed with resid_exact (last step): the natural-map residual summed over
   * every row of every partition (the paper's total residual, section 6), and
   * the largest and the summed norm |C| of the ball joints at the blended state */
  double resid_exact_sum;
  double joint_violation_max;
  double joint_violation_sum;
} ovl_step_stats;

/* Create a world from a scene description.  Every body starts in partition 0
 * of its scene (one partition per scene) until ovl_set_partitions is called.
 * On success *out owns all device buffers until ovl_destroy_world.
 * Errors: INVALID_ARG (bad sizes, a shape other than 0 or 1, a capsule without
 * a positive half-length, sphere inertia not isotropic or capsule inertia not
 * symmetric about body z, joints across scenes or unsorted), OOM, DEVICE. */
ovl_status ovl_create_world(const ovl_world_desc* desc, const ovl_params* params, const ovl_device_ctx* ctx,
                            ovl_world** out);

/* Release every buffer of the world.  NULL is ignored. */
void ovl_destroy_world(ovl_world* w);

/* Replace the step parameters (takes effect at the next step). */
ovl_status ovl_set_params(ovl_world* w, const ovl_params* params);

/* Set the base partition of every body (the paper's initial partitioning,
 * section 5.1 and 5.4).  owner[b] is a global partition id inside its scene's
 * range; parts_per_scene[s] in [1, 64].  halo_k >= 1 is the overlap depth: a
 * body is active in every partition that owns a body within halo_k hops of
 * it in the constraint graph (halo_k = 1 puts exactly the interface bodies in
 * the overlap set; halo_k = gamma + 1 for the paper's growth depth gamma).
 * beta in [1, 16] is the geodesic search depth of Alg. 5.  Takes effect at
 * the next step.  Errors: INVALID_ARG. */
ovl_status ovl_set_partitions(ovl_world* w, const int32_t* owner, int64_t n_bodies, const int32_t* parts_per_scene,
                              int32_t n_scenes, int32_t halo_k, int32_t beta);

/* Dynamic load balancing (section 5.4: Alg. 6 with the bridge test of
 * Alg. 7).  enable = 0: every step's worker sets are the halo of the owners
 * (ovl_set_partitions).  enable = 1: the worker sets are carried from step to
 * step; each step first updates them from its contacts between two dynamic
 * bodies (as CONTACT_KEY lists them), taken in key order:
 *   - bodies A, B with disjoint sets: the set of smaller load (number of
 *     bodies active in it, summed over its workers; a tie goes to A) is
 *     activated on the other body, and every vertex within `depth` hops of
 *     that body in the step's constraint graph is activated in both sets;
 *   - an overlap body meeting a single-worker body keeps only the shared
 *     workers unless its neighbours span more than one worker (a bridge);
 *   - two bodies with equal sets both keep only its least loaded worker
 *     (ties: the lowest partition).
 * depth in [0, 64] is the paper's growth depth gamma.  sets (host, n_sets =
 * n_bodies, or NULL) gives the starting sets as local partition bits, each
 * non-empty and inside its scene's partitions; NULL starts every body in its
 * owner only (the naive start of section 5.4).  Copied.  The sets carried
 * forward are those of the last step that committed; ovl_set_partitions
 * restarts them from the owners.  halo_k is not used while enabled.
 * Errors: INVALID_ARG, OOM, DEVICE. */
ovl_status ovl_set_load_balance(ovl_world* w, int32_t enable, int32_t depth, const uint64_t* sets, int64_t n_sets);

/* Run n_steps steps.  Asynchronous on the world's stream when stats is NULL
 * (errors then surface at the next synchronising call); with stats non-NULL
 * the call synchronises, fills *stats for the last step and, if a per-step
 * buffer overflowed, grows the buffers and re-runs the steps that did not
 * commit.  compute_exact_residual != 0 also fills stats->resid_exact.
 * Errors: CAPACITY, NONFINITE (state kept at the last good step), DEVICE;
 * NOT_CONVERGED is informational (the state advanced). */
ovl_status ovl_step(ovl_world* w, int32_t n_steps, ovl_step_stats* stats, int32_t compute_exact_residual);

/* Replace the warm-start cache (checkpoint restore of the impulses the next
 * step starts from; plain warm start, reading R16).  n entries, strictly
 * increasing in (part, kind, key), as ovl_read_debug exports them
 * (CACHE_PART, CACHE_KIND, CACHE_KEY, CACHE_VAL): part a global partition id,
 * kind 0 joint (key = joint index, val = its three impulses, 0) or 1 contact
 * (key = (a<<32)|(bcode<<1)|sub, val = lambda_n and the friction impulse as a
 * world vector).  Host arrays, copied.  INVALID_ARG (unsorted, bad partition
 * or kind, non-finite value), CAPACITY (n above the copy capacity), DEVICE. */
ovl_status ovl_write_cache(ovl_world* w, const int32_t* part, const int32_t* kind, const uint64_t* key,
                           const float* val, int64_t n);

/* Copy the blended states, [n_bodies][13] float32, into dst (host, or device
 * when dst_is_device != 0).  Synchronises the stream.  Errors: INVALID_ARG
 * (n_bodies differs), a pending CAPACITY/NONFINITE error, DEVICE. */
ovl_status ovl_read_state(ovl_world* w, float* dst, int64_t n_bodies, int32_t dst_is_device);

/* Overwrite the states (checkpoint restore, bulk reset).  src as in
 * ovl_read_state.  Non-finite values are rejected (INVALID_ARG).  The
 * warm-start cache is cleared unless keep_cache != 0. */
ovl_status ovl_write_state(ovl_world* w, const float* src, int64_t n_bodies, int32_t src_is_device,
                           int32_t keep_cache);

/* Wait for all work queued on the world's stream. */
ovl_status ovl_synchronize(ovl_world* w);

/* Debug/parity export of the last step's intermediate results.  Writes at
 * most capacity_bytes into dst (host) and the element count into *count
 * (a NULL dst only queries the count).  Synchronises.  Fields and layouts:
 *   CONTACT_KEY   u64 [C]  (a<<32)|(bcode<<1)|sub, sorted; bcode = b for a
 *                          body b > a, N + plane index, N + P + sphere index
 *   CONTACT_GEOM  f32 [C*8]  n(3), phi, l_a, l_b, s_a, t_b: the lever arms to the contact
 *                           point are r_a = s_a u_a + l_a n and r_b = t_b u_b - l_b n, with u the
 *                           body z axis at the start of the step (s_a = t_b = 0 for spheres)
 *   ADJ_OFF       i32 [N+1]; ADJ i32 [adj_off[N]] (per vertex sorted, unique,
 *                          padded slots hold -1)
 *   MASK          u64 [N]  local partition bits of every body
 *   PART_REP_OFF  i32 [G+1]; REP_BODY i32 [R] partition-major, bodies ascending
 *   REP_D         i32 [R]  geodesic distance (0 = none within beta), partition-major
 *   REP_W         f32 [R]  blend weight, partition-major
 *   PART_COPY_OFF i32 [G+1]; COPY_KIND i32 [M] (0 joint, 1 contact); COPY_KEY u64 [M]
 *   COPY_IA, COPY_IB i32 [M] local replica indices (-1 static); COPY_COLOUR i32 [M]
 *   COPY_LAMBDA0, COPY_LAMBDA f32 [M*3] warm start and final impulses, uid order
 *   REP_STATE     f32 [R*13] replica states after integration, partition-major
 *   PART_ITERS    i32 [G]; PART_RESID f32 [G]
 *   CACHE         packed warm-start cache of the last step, uid order:
 *                 CACHE_PART i32 [M], CACHE_KIND i32 [M], CACHE_KEY u64 [M], CACHE_VAL f32 [M*4]
 *   PART_COL_OFF  i32 [G*65] colour offsets (relative to the partition start)
 *   COPY_FEAT, COPY_LAMBDAL, PART_GUARD, PART_RHO0: see below
 */
enum {
  OVL_DBG_CONTACT_KEY = 0,
  OVL_DBG_CONTACT_GEOM,
  OVL_DBG_ADJ_OFF,
  OVL_DBG_ADJ,
  OVL_DBG_MASK,
  OVL_DBG_PART_REP_OFF,
  OVL_DBG_REP_BODY,
  OVL_DBG_REP_D,
  OVL_DBG_REP_W,
  OVL_DBG_PART_COPY_OFF,
  OVL_DBG_COPY_KIND,
  OVL_DBG_COPY_KEY,
  OVL_DBG_COPY_IA,
  OVL_DBG_COPY_IB,
  OVL_DBG_COPY_COLOUR,
  OVL_DBG_COPY_LAMBDA0,
  OVL_DBG_COPY_LAMBDA,
  OVL_DBG_REP_STATE,
  OVL_DBG_PART_ITERS,
  OVL_DBG_PART_RESID,
  OVL_DBG_CACHE_PART,
  OVL_DBG_CACHE_KIND,
  OVL_DBG_CACHE_KEY,
  OVL_DBG_CACHE_VAL,
  OVL_DBG_PART_COL_OFF,
  OVL_DBG_COPY_FEAT,      /* f32 [M*13] features and impulse scale (feature export or learned mode) */
  OVL_DBG_COPY_LAMBDAL,   /* f32 [M*3] learned start, uid order (learned mode) */
  OVL_DBG_PART_GUARD,     /* i32 [G] 1 when the learned start was kept */
  OVL_DBG_PART_RHO0,      /* f32 [G*2] initial residual of the plain and the learned start */
  OVL_DBG_REP_CPL,        /* f32 [R*6] interface-coupling impulse per replica (dv, dw), partition-major */
  OVL_DBG_NFIELDS
};
ovl_status ovl_read_debug(ovl_world* w, int32_t field, void* dst, int64_t capacity_bytes, int64_t* count);

/* Warm-start mode of the following steps (not in the paper; a solver
 * accelerator).  OVL_WARM_PLAIN: the previous step's impulses of the same
 * (partition, kind, key).  OVL_WARM_LEARNED: for contacts, the network's
 * prediction from twelve per-contact features (BF16 matrix-core inference),
 * projected on the contact's bounds; per partition it is kept only when its
 * initial natural-map residual is below the plain start's, else the plain
 * start is used (the guard).  params: OVL_MLP_PARAMS floats (learned mode
 * only; copied).  ovl_params.warmstart is overridden.  Errors: INVALID_ARG. */
ovl_status ovl_set_warmstart(ovl_world* w, int32_t mode, const float* params, int64_t n_params);

/* Write the per-contact features during the following steps (1) or not (0);
 * needed by ovl_collect_training_rows. */
ovl_status ovl_set_feature_export(ovl_world* w, int32_t enable);

/* Training rows of the last step's contact copies (uid order): features
 * [n][12] and targets [n][3] = final impulses (n, t1, t2) / s, with s the
 * copy's impulse scale.  Host buffers of capacity_rows rows; *n_rows gets the
 * count (NULL buffers only query it).  Errors: INVALID_ARG (no features
 * exported, buffers too small). */
ovl_status ovl_collect_training_rows(ovl_world* w, float* features, float* targets, int64_t capacity_rows,
                                     int64_t* n_rows);

/* Force the learned/plain choice of every partition of the next steps
 * (parity checks of the guard); choice[g] in {-1 decide, 0 plain, 1 learned};
 * NULL clears it. */
ovl_status ovl_force_guard(ovl_world* w, const int32_t* choice, int32_t n_parts);

/* Trainer of the warm-start network on the device (FP32, Adam with
 * beta1 0.9, beta2 0.999, eps 1e-8; deterministic).  Rows are features
 * [n][12] and targets [n][3]; the loss is their mean squared error. */
typedef struct ovl_mlp ovl_mlp;
ovl_status ovl_mlp_create(const float* params, int64_t n_params, const ovl_device_ctx* ctx, ovl_mlp** out);
void ovl_mlp_destroy(ovl_mlp* m);
/* One Adam step on a batch; x, t on the host, or on the device when on_device != 0. */
ovl_status ovl_mlp_train_step(ovl_mlp* m, const float* x, const float* t, int64_t n, float lr, int32_t on_device,
                              float* loss);
/* Gradient (OVL_MLP_PARAMS floats, host) and loss of a batch without an update. */
ovl_status ovl_mlp_gradient(ovl_mlp* m, const float* x, const float* t, int64_t n, int32_t on_device, float* grad,
                            float* loss);
ovl_status ovl_mlp_get_params(ovl_mlp* m, float* out, int64_t n_params);
const char* ovl_mlp_last_error(const ovl_mlp* m);
/* BF16 matrix-core inference of the network on host rows x [n][12] -> y [n][3]
 * (the kernel the learned warm start uses). */
ovl_status ovl_mlp_infer(const float* params, int64_t n_params, const float* x, int64_t n, float* y);

/* Gradient and loss of a batch, like ovl_mlp_gradient, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc): no trainer handle, nothing allocated, no
 * synchronisation.  All pointers are device memory on the current device:
 * params [OVL_MLP_PARAMS], rows x [n][12] and targets t [n][3] (read); grad
 * [OVL_MLP_PARAMS] and loss [1] (written: the gradient of the mean squared
 * error and that error, the same bits ovl_mlp_gradient returns for the same
 * rows).  The work is queued on `stream` (a hipStream_t; NULL: the null
 * stream); results are there once the stream reaches it.  The blocks' partial
 * sums live in one fixed array per device, alive until the process ends, of
 * room for OVL_MLP_STATIC_ROWS rows (about 1.3 MB): every call on a device uses
 * the same array, so calls that overlap on one device (other streams, other
 * host threads) race and must be ordered by the caller.  Errors, with nothing
 * queued: INVALID_ARG (NULL pointer, n <= 0), CAPACITY (n above
 * OVL_MLP_STATIC_ROWS), DEVICE; the text is ovl_mlp_last_error(NULL). */
#define OVL_MLP_STATIC_ROWS 8192
ovl_status ovl_mlp_gradient_static(const float* params, const float* x, const float* t, int64_t n, float* grad,
                                   float* loss, void* stream);

/* Force the sweep count of every partition of the next step (parity checks
 * of adaptive runs); iters == NULL clears it.  [G] entries, each >= 0. */
ovl_status ovl_force_iters(ovl_world* w, const int32_t* iters, int32_t n_parts);

/* Cumulative counters of a world since its creation (synchronises). */
typedef struct {
  int64_t steps;              /* committed steps */
  int64_t sweeps_max_total;   /* sum over steps of the largest sweep count of a partition */
  int64_t sweeps_part_total;  /* sum over steps and partitions of the sweep counts */
  int64_t unconverged_total;  /* partitions that hit the cap in adaptive mode */
  int64_t pgs_bytes;          /* algorithmic bytes of all Gauss-Seidel sweeps: per sweep and constraint
                                 copy 220 B (two bodies), 164 B (one body and a static), 192 B (joint) */
  int64_t pgs_launches;       /* solver launches timed with HIP events (profiling on) */
  double pgs_ms;              /* their summed duration, ms, measured on the world's stream */
  int64_t steps_capped;       /* steps in which a partition hit the cap unconverged (adaptive mode) */
  int64_t pgs_ops;            /* algorithmic FP32 operations of all Gauss-Seidel sweeps (add, multiply,
                                 fused multiply-add, min, max each one): per sweep and constraint copy 88
                                 (sphere contact, two bodies), 74 (one body and a static), 63 (ball joint,
                                 three rows); capsule contacts are counted as sphere contacts */
} ovl_counters;
ovl_status ovl_get_counters(ovl_world* w, ovl_counters* out);

/* ---- launch configuration of the solve, HIP graph replay, autotuner ----
 * (spec pattern: many uneven scenes and partitions in one persistent,
 * graph-captured launch with autotuned block and tile sizes)
 *
 * pgs_block / pgs_lds_reps: threads per partition workgroup and the number of
 *   replicas whose velocities the workgroup keeps in LDS (larger partitions
 *   run in a global-memory variant).  Supported pairs: (1024, 4800),
 *   (512, 2400), (256, 1200), (256, 2400); default (1024, 4800).
 * persistent: 0 = one workgroup per partition, largest partitions dispatched
 *   first; 1 = as many workgroups as fit on the device at once, each taking
 *   partitions (largest first) from an atomic queue until it is empty.
 * graph: 1 = ovl_step captures one step into a HIP graph and replays it;
 *   the graph is captured again whenever a parameter, the partitioning or a
 *   buffer changes.  Steps that force sweep counts, compute the exact
 *   residual or are profiled run without the graph.
 * The configuration changes no result: every configuration computes the
 * same bits. */
typedef struct {
  int32_t pgs_block;
  int32_t pgs_lds_reps;
  int32_t persistent;
  int32_t graph;
} ovl_launch_cfg;

/* INVALID_ARG for an unsupported pair or a flag other than 0/1. */
ovl_status ovl_set_launch(ovl_world* w, const ovl_launch_cfg* cfg);
ovl_status ovl_get_launch(const ovl_world* w, ovl_launch_cfg* cfg);
/* Writes up to cap candidate configurations the autotuner tries (graph = 0)
 * into out (may be NULL) and returns their number. */
int32_t ovl_launch_candidates(ovl_launch_cfg* out, int32_t cap);
/* Autotuner: runs the contacts, graph, colouring and rows of ONE step, then
 * times the Gauss-Seidel solve of that step `trials` times (1..100) with each
 * candidate configuration on the same inputs (the minimum counts), checks
 * that all candidates produce identical replica states and sweep counts
 * (DEVICE error otherwise), keeps the fastest (graph flag unchanged) and
 * finishes the step with it: the world advances by exactly one step.
 * chosen (nullable) receives the configuration, ms (nullable, n_ms >=
 * ovl_launch_candidates(NULL, 0)) the time of each candidate in the order of
 * ovl_launch_candidates.  INVALID_ARG while a forced sweep count is pending. */
ovl_status ovl_autotune(ovl_world* w, int32_t trials, ovl_launch_cfg* chosen, float* ms, int32_t n_ms);

/* Turn HIP-event timing of the solver kernel on (1) or off (0).  Events are
 * recorded on the world's stream around every Gauss-Seidel launch and summed
 * by ovl_get_counters. */
ovl_status ovl_profile(ovl_world* w, int32_t enable);

/* Last error text of the world (never NULL; "" when none).  NULL world:
 * the last error of a failed ovl_create_world on this thread. */
const char* ovl_last_error(const ovl_world* w);

/* Library version string. */
const char* ovl_version(void);

#ifdef __cplusplus
}
#endif
#endif
