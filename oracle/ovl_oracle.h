/* Oracle for the overlapping-partition rigid-body step (TEST INFRASTRUCTURE ONLY).
 *
 * A plain, slow, sequential, double-precision CPU implementation of one step of
 * the overlapping-partition method of Kale & Kry, "Distributed Simulation of
 * Large Multi-body Systems" (arXiv 2403.17261):
 *   contacts -> constraint graph (section 5.1) -> overlap sets (section 4 Eq. 9-10,
 *   Alg. 2-3 as a k-hop halo) -> geodesic weights (section 5.3, Eq. 15-16, Alg. 5)
 *   -> per-partition MLCP rows (section 3, Eq. 1-7) -> colour order -> projected
 *   Gauss-Seidel -> integration -> blending (section 5.2, Eq. 11-14, Alg. 4).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library.
 */
#ifndef OVL_ORACLE_H
#define OVL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_bodies, n_scenes, n_joints;
  const int32_t* scene;        /* [N] nondecreasing */
  const int32_t* shape;        /* [N] 0 = sphere, 1 = capsule along body z (halflen > 0) */
  const float* radius;         /* [N] */
  const float* halflen;        /* [N] */
  const float* mass;           /* [N] */
  const float* inertia;        /* [N*3] body-frame principal moments */
  const float* mu;             /* [S] */
  const float* margin;         /* [S] */
  const int32_t* plane_off;    /* [S+1] */
  const float* planes;         /* [P*4] n.x = c */
  const int32_t* ssph_off;     /* [S+1] */
  const float* ssph;           /* [Q*4] centre, radius */
  const int32_t* joint_ab;     /* [J*2] */
  const float* joint_anchor;   /* [J*6] body-frame anchor on a, then on b */
} orc_scene;

typedef struct {
  double dt, gx, gy, gz, cfm, erp, tol;
  int32_t max_iters, adaptive, warmstart, halo_k, beta, brute_force_contacts;
  uint32_t seed;
  int32_t learned;              /* 1: learned warm start for contacts, guarded per partition */
  const float* mlp;             /* [ORC_MLP_PARAMS] W1[12][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3] */
  const int32_t* forced_guard;  /* [G] or NULL: 1 learned, 0 plain, -1 decide */
  /* Dynamic load balancing (section 5.4, Alg. 6-7).  lb_masks NULL: the
   * worker sets are the k-hop halo of the owners.  Otherwise they are carried
   * from the previous step (lb_masks, local partition bits per body) and the
   * step updates them with the rules of Alg. 6 applied to every contact of
   * the step between two dynamic bodies, in key order (Alg. 1 passes the
   * step's whole contact list; a contact handled by the first rule in one
   * step meets the third rule in the next). */
  const uint64_t* lb_masks;
  int32_t lb_depth;             /* growth depth gamma of Alg. 6 (>= 0) */
  /* 1: every overlap body blends its replicas with equal weights 1/|W|, the
   * naive choice section 5.3 compares the geodesic weights against */
  int32_t equal_weights;
  /* 1: interface coupling by the previous step's constraint impulses (the
   * coupling section 7 proposes, after [BW97]).  A constraint of the step
   * between two dynamic bodies with exactly one of them active in partition i
   * is cut from that partition's solve; its impulse of the previous step, as
   * the partition with the lowest id among those active in both bodies left
   * it (cache key as for the warm start, friction carried as a world vector,
   * projected and clipped as the warm start does), acts on the body inside
   * P_i as a fixed impulse added to its free velocity before the solve.
   * 2: mass splitting at the interface (section 2 relates the blend to the
   * mass splitting of [TBV12]: the workers share a body's mass).  The replica
   * of an overlap body in partition i carries the share w_i of its mass and
   * of its inertia (inverse mass and inverse inertia divided by its blend
   * weight w_i; a replica of weight 0 keeps the whole body), so that the
   * blend sum_i w_i v_i equals the body's free velocity plus the sum of the
   * partitions' impulses applied to the whole body. */
  int32_t coupling;
  /* Threads for the projected Gauss-Seidel solves (1: sequential).  The
   * partitions are independent sub-solves (section 4: one worker each), so
   * solving them on several threads, one partition per thread at a time,
   * gives the same bits as the sequential loop. */
  int32_t threads;
} orc_params;

#define ORC_MLP_IN 12
#define ORC_MLP_HID 64
#define ORC_MLP_OUT 3
#define ORC_MLP_PARAMS (12 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3)

typedef struct {
  int64_t n;
  const int32_t* part;   /* global partition id */
  const int32_t* kind;   /* 0 joint, 1 contact */
  const uint64_t* key;   /* joint id, or contact key */
  const float* val;      /* [n*4]: contact (lambda_n, friction impulse world xyz); joint (lx, ly, lz, 0) */
} orc_cache;

typedef struct orc_result orc_result;

enum orc_field {
  ORC_CONTACT_KEY = 0,   /* u64 [C]   (a<<32) | (bcode<<1) | sub */
  ORC_CONTACT_N,         /* f64 [C*3] normal from body a towards b */
  ORC_CONTACT_PHI,       /* f64 [C]   signed gap */
  ORC_CONTACT_RA,        /* f64 [C*3] lever arm of a */
  ORC_CONTACT_RB,        /* f64 [C*3] lever arm of b */
  ORC_ADJ_OFF,           /* i32 [N+1] */
  ORC_ADJ,               /* i32 [2E] sorted, unique per vertex */
  ORC_MASK,              /* u64 [N]   local partition bits */
  ORC_PART_REP_OFF,      /* i32 [G+1] */
  ORC_REP_BODY,          /* i32 [R]   partition-major, bodies ascending */
  ORC_REP_D,             /* i32 [R]   geodesic distance to the partition's pure bodies (0 = not found) */
  ORC_REP_W,             /* f64 [R]   blend weight */
  ORC_PART_COPY_OFF,     /* i32 [G+1] */
  ORC_COPY_KIND,         /* i32 [M] */
  ORC_COPY_KEY,          /* u64 [M] */
  ORC_COPY_IA,           /* i32 [M]   local replica index */
  ORC_COPY_IB,           /* i32 [M]   local replica index or -1 (static) */
  ORC_COPY_COLOUR,       /* i32 [M] */
  ORC_COPY_DIR,          /* f64 [M*9] row directions (3 rows x 3) */
  ORC_COPY_RA,           /* f64 [M*3] */
  ORC_COPY_RB,           /* f64 [M*3] */
  ORC_COPY_ARR,          /* f64 [M*3] diagonal A_rr */
  ORC_COPY_BIAS,         /* f64 [M*3] */
  ORC_COPY_MU,           /* f64 [M]   (joint: 0) */
  ORC_COPY_LAMBDA0,      /* f64 [M*3] warm start */
  ORC_COPY_LAMBDA,       /* f64 [M*3] final impulses */
  ORC_REP_VT,            /* f64 [R*6] velocity before the solve (gravity applied, no warm start) */
  ORC_REP_INVM,          /* f64 [R] */
  ORC_REP_INVI,          /* f64 [R*9] world inverse inertia */
  ORC_REP_STATE,         /* f64 [R*13] replica state after integration */
  ORC_STATE,             /* f64 [N*13] blended state */
  ORC_PART_ITERS,        /* i32 [G] */
  ORC_PART_RESID,        /* f64 [G] in-sweep residual of the last sweep */
  ORC_CACHE_PART,        /* i32 [M] warm-start cache for the next step (uid order) */
  ORC_CACHE_KIND,        /* i32 [M] */
  ORC_CACHE_KEY,         /* u64 [M] */
  ORC_CACHE_VAL,         /* f32 [M*4] */
  ORC_STATS,             /* f64 [8]: exact residual, sum residual, joint violation, n_overlap,
                                      max colours, max iters, error code, unconverged partitions */
  ORC_COPY_FEAT,         /* f64 [M*13] contact features (12) and impulse scale s (joints: zeros) */
  ORC_COPY_LAMBDAL,      /* f64 [M*3] learned warm start (contacts; joints: plain) */
  ORC_PART_GUARD,        /* i32 [G] 1 when the learned start was kept */
  ORC_PART_RHO0,         /* f64 [G*2] initial residual of the plain and of the learned start */
  ORC_COPY_DEG,          /* i32 [M] conflict degree */
  ORC_REP_CPL,           /* f64 [R*6] interface-coupling impulse per replica (dv, dw); zeros without coupling */
  ORC_NFIELDS
};

orc_result* orc_step(const orc_scene* sc, const float* state, const int32_t* owner,
                     const int32_t* parts_per_scene, const orc_params* prm, const orc_cache* cache,
                     const int32_t* forced_iters);
void orc_free(orc_result* r);
int64_t orc_len(const orc_result* r, int32_t field);
const void* orc_ptr(const orc_result* r, int32_t field);
const char* orc_error(const orc_result* r);

/* Building blocks exposed for the pins. */
uint32_t orc_fmix32(uint32_t h);
void orc_tangents(const double n[3], double t1[3], double t2[3]);
void orc_blend(int32_t n, const double* states, const double* w, double* out);
float orc_bf16(float x);
void orc_mlp_infer(const float* params, const double* x12, double* y3);

#ifdef __cplusplus
}
#endif
#endif
