// Internal declarations of the ovl library (device buffers and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace ovl {

constexpr int kMaxParts = 64;        // partitions per scene (u64 membership mask)
constexpr int kMaxColours = 64;      // colours per partition (u64 used-colour mask)
constexpr int kColStride = kMaxColours + 1;
// Gauss-Seidel launch configurations (threads per partition workgroup, replicas
// whose velocities fit in LDS, two float4 each): 1, 2, 4 and 2 workgroups per CU
constexpr int kPgsCfgCount = 4;
constexpr int kPgsCfgBlock[kPgsCfgCount] = {1024, 512, 256, 256};
constexpr int kPgsCfgReps[kPgsCfgCount] = {4800, 2400, 1200, 2400};
// the sweeps' record loads may run up to one workgroup past a partition's last
// slot (lanes past a colour's end), so the record arrays carry this many spare slots
constexpr int kSlotPad = 1024;
static_assert(kSlotPad >= kPgsCfgBlock[0] && kSlotPad >= kPgsCfgBlock[1] && kSlotPad >= kPgsCfgBlock[2] &&
                  kSlotPad >= kPgsCfgBlock[3],
              "the record arrays must be padded by the largest solver workgroup");
constexpr int kBlock = 256;          // generic per-item kernels
constexpr int kKeep = 16;            // contact keys per body kept between the two narrow-phase passes
constexpr int kLbLdsCap = 12288;     // load balancing: scenes up to this many bodies keep their sets in LDS
// warm-start network 12 -> 64 -> 64 -> 3
constexpr int kMlpIn = 12, kMlpHid = 64, kMlpOut = 3;
constexpr int kMlpParams = kMlpIn * kMlpHid + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpHid * kMlpOut + kMlpOut;
constexpr int kMlpWb = 16 * 64 + 64 * 64 + 64 * 16;  // padded bfloat16 weight tiles
constexpr int kMlpBias = 64 + 64 + 16;
constexpr int kFeatStride = 16;      // 12 features, impulse scale s, padding

// device scalar slots
enum Scal {
  SC_NCONTACT = 0,   // contacts found
  SC_NADJ,           // adjacency entries
  SC_NREP,           // replicas
  SC_NCOPY,          // constraint copies
  SC_FLAGS,          // error flags (bit set = failure of this step)
  SC_PREV_NCOPY,     // copies in the warm-start cache
  SC_COMMITTED,      // steps whose blend committed
  SC_NJCOPY,         // joint copies
  SC_NCCOPY,         // contact copies
  SC_NOVERLAP,       // bodies in >= 2 partitions
  SC_LB_CHANGES,     // contacts whose load-balancing rule changed a worker set
  SC_COUNT = 16
};

enum Flag {
  F_CONTACT_CAP = 1,
  F_ADJ_CAP = 2,
  F_REP_CAP = 4,
  F_COPY_CAP = 8,
  F_COLOUR_CAP = 16,
  F_NONFINITE = 32,
};

// Everything a kernel may touch.  Passed by value to every kernel.
struct WP {
  // sizes and capacities
  int32_t N, S, J, P, Q, G, T;   // bodies, scenes, joints, planes, static spheres, partitions, hash buckets
  int32_t Ccap, Mcap, Rcap, Acap;
  float cs;                      // grid cell edge
  // parameters
  float dt, gx, gy, gz, cfm, erp, tol;
  int32_t max_iters, adaptive, warmstart, halo_k, beta;
  int32_t equal_w;               // 1: equal blend weights instead of geodesic ones
  int32_t couple;                // 1: previous-step impulses of cut constraints act on the partition's bodies
  int32_t msplit;                // 1: an overlap replica carries the share w of its body's mass and inertia
  uint32_t seed;
  int32_t forced;                // 1: part_force_iters holds each partition's sweep count
  // static body data
  const int32_t* b_scene;
  const float* b_radius;
  const float* b_invm;
  const float* b_invI;          // spheres: 1/I; capsules: 1/I_perp (about a transverse axis)
  const float* b_half;          // capsule half-length (0 for a sphere)
  const float* b_dI;            // capsules: 1/I_axis - 1/I_perp (0 for a sphere)
  int32_t has_caps;             // 1 when some body is a capsule
  // scenes
  const float* s_mu;
  const float* s_margin;
  const int32_t* s_plane_off;
  const float* planes;          // [P*4]
  const int32_t* s_ssph_off;
  const float* ssph;            // [Q*4]
  const int32_t* s_body_off;    // [S+1]
  const int32_t* s_joint_off;   // [S+1]
  const int32_t* s_part_base;   // [S+1]
  // joints
  const int32_t* j_ab;          // [J*2]
  const float* j_anchor;        // [J*6]
  const int32_t* jadj_off;      // [N+1] joint partners per body, sorted
  const int32_t* jadj;
  const int32_t* jinc_off;      // [N+1] joints of each body, by joint index
  const int32_t* jinc;
  // partitions
  const int32_t* owner_local;   // [N] owner - base of the body's scene
  const int32_t* part_force_iters;  // [G]
  // canonical state, component-major [13][N]
  float* st;
  // grid
  int32_t* cell;                // [3N]
  uint32_t* bucket;             // [N]
  int32_t* bcount;              // [T+1]
  int32_t* bstart;              // [T+1]
  int32_t* bfill;               // [T]
  int32_t* bbody;               // [N] bodies in bucket order
  int4* srt_cell;               // [N] bucket order: cell x, y, z and body
  float4* srt_pos;              // [N] bucket order: centre and radius
  // contacts
  int32_t* ccount;              // [N+1]
  int32_t* coff;                // [N+1]
  uint32_t* c_bkey;             // [Ccap] (bcode<<1)|sub
  uint32_t* c_keep;             // [N*kKeep] contact keys found by the count pass
  int32_t* c_a;                 // [Ccap]
  float* c_geom;                // [8][Ccap]: n(3), phi, l_a, l_b, s_a, t_b: lever arms
                                //   r_a = s_a u_a + l_a n, r_b = t_b u_b - l_b n (u: capsule axis)
  // graph
  int32_t* deg;                 // [N+1]
  int32_t* adj_off;             // [N+1]
  int32_t* adj;                 // [Acap]
  int32_t* adj_fill;            // [N]
  // masks
  uint64_t* mask;               // [N]
  uint64_t* mask_tmp;           // [N]
  uint64_t* reach;              // [N]
  uint64_t* reach_tmp;          // [N]
  // replicas
  int32_t* rep_cnt;             // [N+1]
  int32_t* rep_off_bm;          // [N+1]
  int32_t* rep_D_bm;            // [Rcap]
  int32_t* rep_pm_of_bm;        // [Rcap]
  int32_t* rep_body_pm;         // [Rcap]
  int32_t* part_rep_off;        // [G+1]
  float* rst;                   // [13][Rcap] replica states after integration
  float* rep_w_bm;              // [Rcap] blend weight (body-major)
  // masked compaction scratch: set 0 bodies, 1 joints, 2 contacts
  int32_t* mc_blk[3];           // [(nblk+1)*64] per-block counts, then exclusive prefixes
  int32_t* mc_rank0[3];         // [(S+1)*64] rank of each scene start per bit
  int32_t* mc_psize[3];         // [G+1] items per partition
  const int32_t* part_scene;    // [G]
  const int32_t* part_bit;      // [G] local bit of the partition in its scene
  int32_t* g_tmp;               // [G+1]
  // copies (uid order)
  int32_t* part_copy_off;       // [G+1]
  int32_t* cp_src;              // [Mcap] joint index, or contact index + J
  int32_t* cp_part;             // [Mcap]
  int32_t* cp_ia;               // [Mcap]
  int32_t* cp_ib;               // [Mcap]
  int32_t* cp_colour;           // [Mcap]
  int32_t* cp_slot;             // [Mcap]
  int32_t* cp_inv;              // [Mcap] slot -> copy (scratch of the slot order)
  int32_t* inc_off;             // [2*Rcap] replica -> first incident copy, then incident-copy counts
  int32_t* inc;                 // [2*Mcap]
  int32_t* part_col_off;        // [G*65]
  int32_t* part_ncol;           // [G]
  // rows (slot order = colour-sorted within each partition)
  //   contact: rec0 = (n, a_duff), rec1 = (l_a, l_b, bias_n, mu), rec2 = (1/A_n, 1/A_t, A_n, A_t)
  //            (a sphere contact has A_t1 = A_t2 = A_t)
  //   joint:   rec0 = (r_a, bias_x), rec1 = (r_b, bias_y), rec2 = (1/A_x, 1/A_y, 1/A_z, bias_z)
  //   contact touching a capsule (kGenFlag): rec1 = (A_n, 0, bias_n, mu),
  //   rec2 = (1/A_n, 1/A_t1, 1/A_t2, 0), and r_gen holds the full lever arms (r_a, A_t1), (r_b, A_t2)
  float4* r_rec;                // [3][Mcap]
  float4* r_gen;                // [2][Mcap] (only with capsules)
  int2* r_ids;                  // [Mcap] (local replica a | kJointFlag | kGenFlag, local replica b or -1)
  float4* rep_ax;               // [Rcap] capsule axis u and 1/I_axis - 1/I_perp of each replica
  float4* rep_cpl;              // [2*Rcap] interface-coupling impulse per replica: (dv, 0), then (dw, 0)
  float* rep_isc;               // [Rcap] mass splitting: inverse mass and inertia factor 1/w per replica
  float2* rep_im;               // [Rcap] inverse mass and inverse inertia of each replica (with that factor)
  float4* r_lam;                // [Mcap] impulses (3 used)
  float4* r_lam0;               // [Mcap] warm-start impulses
  float4* rep_v4;               // [2*Rcap] velocity storage of partitions too large for LDS
  // learned warm start
  int32_t learned;              // 1: learned start for contacts, guarded per partition
  int32_t feat_on;              // 1: write the per-copy features
  float* r_feat;                // [Mcap][kFeatStride] uid order
  float4* r_lamL;               // [Mcap] learned start, slot order
  const uint16_t* mlp_wb;       // [kMlpWb]
  const float* mlp_bias;        // [kMlpBias]
  int32_t* part_guard;          // [G] 1 when the learned start was kept
  float* part_rho0;             // [G*2] initial residual of the plain and of the learned start
  const int32_t* part_force_guard;  // [G] -1 decide, 0 plain, 1 learned
  int32_t force_guard;
  // warm-start cache (uid order of the last committed step)
  int32_t* wc_part;             // [Mcap]
  int32_t* wc_kind;             // [Mcap]
  uint64_t* wc_key;             // [Mcap]
  float* wc_val;                // [4][Mcap]
  uint64_t* wc_k64;             // [Mcap] search key of each entry: kind << 63 | key
  int32_t* wc_off;              // [G+1] entries of partition p: [wc_off[p], wc_off[p+1])
  // Gauss-Seidel schedule
  int32_t* part_order;          // [G] partitions by descending copy count
  int32_t* pgs_queue;           // [2] work counters of the persistent kernels (LDS, global)
  int32_t pgs_cfg;              // index into kPgsCfg*
  int32_t pgs_persistent;       // 1: resident workgroups take partitions from the queue
  int32_t pgs_grid[2];          // resident workgroups of the two persistent kernels
  int32_t n_cu;                 // compute units of the device
  // per-partition results
  int32_t* part_iters;          // [G]
  int32_t* part_nstatic;        // [G] contact copies with a static body
  float* part_resid;            // [G]
  float* part_rsum;             // [G] natural-map residual summed over the partition's rows
  float* joint_viol;            // [J] |C| of every ball joint at the blended state
  float* stat_f;                // [4]: exact residual
  int64_t* stat_i64;            // [8]: 0 sum over steps of the largest sweep count, 1 unconverged partitions,
                                //      2 algorithmic bytes of the sweeps, 3 sweeps summed over partitions,
                                //      4 committed steps, 5 steps with a capped partition, 6 algorithmic
                                //      FP32 operations of the sweeps
  // dynamic load balancing: worker sets carried from step to step
  int32_t lb_on;                // 1: sets carried and updated from each step's contacts; 0: k-hop halo
  int32_t lb_depth;             // growth depth of the inter-worker rule
  int32_t lb_lds_max;           // largest scene of at most kLbLdsCap bodies (LDS layout size), 0 if none
  int32_t lb_big;               // 1: some scene has more than kLbLdsCap bodies
  uint64_t* lb_mask;            // [N] sets of the last committed step
  int32_t* lb_queue;            // [N] growth BFS queue
  uint32_t* lb_visit;           // [N/32+1] growth BFS visited bits of scenes kept in global memory
  uint32_t* lb_bridge;          // [N/32+1] bridge bits (Alg. 7) of scenes kept in global memory
  // scalars
  int32_t* scal;                // [SC_COUNT]
};

constexpr int32_t kJointFlag = 0x40000000;
constexpr int32_t kGenFlag = 0x20000000;    // a row touching a capsule: full lever arms and inertia

inline int nblocks(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// ---- launchers (each returns hipSuccess or the launch error) ----
// utilities
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);
// exclusive scan of n ints: out[0..n] (out[n] = total); optional copy of the total to *total
hipError_t scan_excl(const int32_t* in, int32_t* out, int64_t n, int32_t* total, int32_t* scratch,
                     hipStream_t s);
size_t scan_scratch_ints(int64_t n);

// collision (broad + narrow phase)
hipError_t launch_collide(const WP& w, int32_t* scan_scratch, hipStream_t s);
// graph, overlap sets, replicas, geodesic distances, constraint copies
hipError_t launch_graph(const WP& w, int32_t* scan_scratch, hipStream_t s);
// solve of a step in three phases: (1) partition order, colouring, rows, warm
// start; (2) projected Gauss-Seidel with integration of the replicas; (3) exact
// residual (optional), blending, warm-start cache, commit
hipError_t launch_solve_pre(const WP& w, hipStream_t s);
hipError_t launch_pgs(const WP& w, hipStream_t s, hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);
hipError_t launch_solve_post(const WP& w, hipStream_t s, bool exact_residual);
// resident solver workgroups per compute unit (LDS and global-memory variants)
// of launch configuration cfg, for the variant a world with (caps, split) runs
hipError_t pgs_occupancy(int cfg, bool caps, bool split, int* per_cu_lds, int* per_cu_glob);
hipError_t launch_reset_lambda(const WP& w, hipStream_t s);
hipError_t launch_digest(const WP& w, unsigned long long* out, hipStream_t s);

// Algorithmic bytes of one Gauss-Seidel sweep per constraint copy: the row
// record and impulses plus the two bodies' velocity read/write and mass data.
constexpr int64_t kBytesDynDyn = 220;
constexpr int64_t kBytesStatic = 164;
constexpr int64_t kBytesJoint = 192;
// Algorithmic FP32 operations of one sweep per constraint copy (each add,
// multiply, fused multiply-add, min and max counted once; the row formulas of
// the sweep): a sphere contact rebuilds its tangents (11), forms the relative
// velocity terms and the three projected updates (n, t1, t2) and applies the
// impulse to both bodies (88); with a static body the second body's terms drop
// out (74); a ball joint solves its three axis rows in turn (63).
constexpr int64_t kOpsDynDyn = 88;
constexpr int64_t kOpsStatic = 74;
constexpr int64_t kOpsJoint = 63;
hipError_t pgs_set_attributes();
// dynamic load balancing (between the graph and the replica table; commit after the blend)
hipError_t launch_balance(const WP& w, hipStream_t s);
hipError_t launch_balance_commit(const WP& w, hipStream_t s);
hipError_t lb_set_attributes();
hipError_t launch_mlp_world(const WP& w, hipStream_t s);
void mlp_pack(const float* params, std::vector<uint16_t>& wb, std::vector<float>& bias);

}  // namespace ovl
