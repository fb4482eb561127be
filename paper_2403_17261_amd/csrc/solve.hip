// Per-partition solve of a step: colouring, rows + warm start, projected
// Gauss-Seidel sweeps, integration, blending and the warm-start cache.
//
//  * Colouring: inside a partition two constraint copies conflict when they
//    share a non-static body.  Jones-Plassmann with priority
//    (fmix32(uid ^ seed), uid): a copy is coloured once every conflicting copy
//    of higher priority is, taking the smallest colour none of them uses.  The
//    result equals sequential greedy colouring in descending priority, so it
//    is unique.  The copies are then renumbered colour by colour (uid order
//    inside a colour); these "slots" are where the rows live.  Gauss-Seidel
//    in colour order is an ordering of the paper's sequential solve: copies of
//    one colour touch disjoint bodies, so they can run at once.
//  * Rows (section 3, Eq. 1-7): three per copy.  Contact: normal n, tangents
//    t1, t2 (Duff et al. 2017 basis); normal impulse >= 0; friction box
//    |lambda_t| <= mu lambda_n; bias phi/h for an open gap, erp*phi/h for a
//    penetration (Eq. 2's stabilisation), none for friction.  Ball joint: the
//    three world axes, unbounded, bias erp*C/h.  A_rr = J_r M^-1 J_r^T + cfm.
//  * Warm start: the previous step's impulses of the same
//    (partition, kind, key); friction is carried as a world vector, projected
//    on the new tangents and clipped to the new box.
//  * Interface coupling (optional, section 7's proposal after [BW97]): a
//    constraint left out of a partition because one of its dynamic bodies is
//    not active there still pushes the body that is, with its impulse of the
//    previous step, added to that replica's free velocity.
//  * Gauss-Seidel: one workgroup per partition (the paper's worker); replica
//    velocities and inverse masses stay in LDS; colours are separated by
//    workgroup barriers.  Adaptive mode stops when a sweep's largest
//    |A_rr * delta lambda| is <= tol.
//  * Integration: x += h v; q <- normalise(q + h/2 (0, w) q).
//  * Blend (Alg. 4, Eq. 11-14): weights from the geodesic distances (Eq. 15-16),
//    replicas in ascending partition id, quaternions sign-aligned with the
//    first one and renormalised.  A body with one replica keeps its state.
#include "ovl_internal.h"

#include <algorithm>
#include <type_traits>
#include "wave.h"

// No implicit fused multiply-add in this file: every fused operation is written
// out with fmaf.  The sweeps are compiled in several variants (velocities in LDS
// or in global memory, block sizes); with the fusions fixed in the source every
// variant rounds the same way, so every launch configuration gives the same bits.
#pragma clang fp contract(off)

namespace ovl {

namespace {

struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)); }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)), fmaf(a.x, b.y, -(a.y * b.x))};
}
__device__ __forceinline__ f3 add(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 sub(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 scale(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
// c + a s and c - a s, fused per component
__device__ __forceinline__ f3 madd(f3 c, f3 a, float s) { return {fmaf(a.x, s, c.x), fmaf(a.y, s, c.y), fmaf(a.z, s, c.z)}; }
__device__ __forceinline__ f3 msub(f3 c, f3 a, float s) {
  return {fmaf(-a.x, s, c.x), fmaf(-a.y, s, c.y), fmaf(-a.z, s, c.z)};
}

__device__ __forceinline__ bool step_failed(const WP& w) {
  return __hip_atomic_load(&w.scal[SC_FLAGS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Duff et al., "Building an Orthonormal Basis, Revisited" (JCGT 2017): the
// only branch is the sign of n_z.  tangents() returns the basis' coefficient
// a = -1/(s + n_z), which the rows store so the sweeps rebuild t1, t2 with no
// division.
__device__ __forceinline__ void tangents_from(f3 n, float a, f3& t1, f3& t2) {
  const float s = copysignf(1.0f, n.z);
  const float b = n.x * n.y * a;
  const float sx = s * n.x;
  t1 = mk(fmaf(sx * n.x, a, 1.0f), s * b, -sx);
  t2 = mk(b, fmaf(n.y * n.y, a, s), -n.y);
}

__device__ __forceinline__ float tangents(f3 n, f3& t1, f3& t2) {
  const float a = -1.0f / (copysignf(1.0f, n.z) + n.z);
  tangents_from(n, a, t1, t2);
  return a;
}

// 1/A of a sphere contact's rows: the hardware reciprocal (within one ulp).
// The row assembly stores it and the sphere-only sweeps form it again from
// the replicas' inverse masses; both use this, so both give the same bits.
__device__ __forceinline__ float row_rcp(float a) { return __builtin_amdgcn_rcpf(a); }

// (1/A_n, 1/A_t, A_n, A_t) of a sphere contact between bodies of inverse
// masses ima, imb and inverse inertias iia, iib, with lever arms la, lb
// (lia = iia la, lib = iib lb): A_n = m_a^-1 + m_b^-1 + cfm and
// A_t = A_n + l_a^2 I_a^-1 + l_b^2 I_b^-1.  The row assembly and the
// sphere-only sweeps both call it, so both give the same bits.
__device__ __forceinline__ float4 sphere_row_masses(float ima, float imb, float la, float lia, float lb, float lib,
                                                    float cfm) {
  const float An = ima + imb + cfm;
  const float At = fmaf(la, lia, fmaf(lb, lib, An));
  return make_float4(row_rcp(An), row_rcp(At), An, At);
}

__device__ __forceinline__ f3 quat_rotate(float qw, float qx, float qy, float qz, f3 v) {
  float nn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= nn;
  qx *= nn;
  qy *= nn;
  qz *= nn;
  f3 r0 = mk(1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy));
  f3 r1 = mk(2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx));
  f3 r2 = mk(2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy));
  return mk(dot(r0, v), dot(r1, v), dot(r2, v));
}

// capsule axis u = R(q) e_z of body b from the canonical state
__device__ __forceinline__ f3 body_axis(const WP& w, int b) {
  const int N = w.N;
  return quat_rotate(w.st[3 * N + b], w.st[4 * N + b], w.st[5 * N + b], w.st[6 * N + b], mk(0.0f, 0.0f, 1.0f));
}

// world inverse inertia of an axisymmetric body applied to x:
// I^-1 x = x / I_perp + (1/I_axis - 1/I_perp) (u.x) u
__device__ __forceinline__ f3 inv_inertia(float ii, f3 u, float dI, f3 x) {
  return madd(scale(x, ii), u, dI * dot(u, x));
}

// Blend weight (Eq. 15-16) of a replica at geodesic distance D of a body in
// n > 1 partitions, given the sum of 1/D over the body's replicas: 1/D
// normalised, uniform where no search reached a partition or with equal weights.
__device__ __forceinline__ float inv_dist_sum(const WP& w, int bm0, int n) {
  float sum = 0.0f;
  for (int k = 0; k < n; ++k) {
    const int D = w.rep_D_bm[bm0 + k];
    sum += D > 0 ? 1.0f / (float)D : 0.0f;
  }
  return sum;
}

__device__ __forceinline__ float blend_weight(const WP& w, int D, float sum, int n) {
  return (sum > 0.0f && !w.equal_w) ? (D > 0 ? 1.0f / (float)D : 0.0f) / sum : 1.0f / (float)n;
}

// mass splitting: factor on the inverse mass and inverse inertia of the
// replica with local index r of partition p (1 without splitting)
__device__ __forceinline__ float rep_split(const WP& w, int p, int r) {
  return w.msplit ? w.rep_isc[w.part_rep_off[p] + r] : 1.0f;
}

// lever arms of contact c: r_a = s_a u_a + l_a n, r_b = t_b u_b - l_b n
__device__ __forceinline__ void contact_arms(const WP& w, int c, int a, int b, f3 n, f3& ra, f3& rb) {
  const int64_t CC = w.Ccap;
  const float la = w.c_geom[4 * CC + c], lb = w.c_geom[5 * CC + c];
  const float sa = w.c_geom[6 * CC + c], tb = w.c_geom[7 * CC + c];
  ra = scale(n, la);
  rb = scale(n, -lb);
  if (sa != 0.0f) ra = add(ra, scale(body_axis(w, a), sa));
  if (tb != 0.0f && b >= 0) rb = add(rb, scale(body_axis(w, b), tb));
}

__device__ __forceinline__ bool prio_gt(uint32_t ha, int ua, uint32_t hb, int ub) {
  return ha > hb || (ha == hb && ua > ub);
}

// ------------------------------------------------------------ colouring ----

// f(l) for the local copy indices inc[k0 .. k1) of an incidence list in LDS,
// four entries read at a time so that their loads (and f's own reads) overlap
// instead of forming one dependent chain per neighbour.
template <class F>
__device__ __forceinline__ void for_incident(const uint16_t* inc, int k0, int k1, F f) {
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    const int l0 = inc[k], l1 = inc[k + 1], l2 = inc[k + 2], l3 = inc[k + 3];
    f(l0);
    f(l1);
    f(l2);
    f(l3);
  }
  for (; k < k1; ++k) f(inc[k]);
}

constexpr int kColBS = 1024;
constexpr int kColLds = 16384;  // partitions with at most this many copies colour in LDS (7 B per copy)
constexpr int kColRepLds = 8192;  // ... and at most this many replicas (incidence offsets in LDS)
// Small partitions colour in a 256-thread workgroup with 39 KB of LDS, four to
// a compute unit, when there are more partitions than compute units (many
// scenes at once).  At most 16 copies per thread.
constexpr int kColSmallBS = 256;
constexpr int kColSmallCopies = 4096;
constexpr int kColSmallReps = 4096;

// BS threads; partitions of at most kCopies copies and kReps replicas colour
// in LDS.  kSmall: this instantiation takes only the partitions that fit the
// small one (kColSmallCopies, kColSmallReps); the large one takes the rest
// when split is set, else every partition.
template <int BS, int kCopies, int kReps, bool kSmall>
__global__ __launch_bounds__(BS) void k_colour(WP w, int split) {
  __shared__ int lds_i[(BS / 64)];
  __shared__ int ccount[kMaxColours];
  __shared__ int col_off[kColStride];
  __shared__ int running[kMaxColours];
  __shared__ int wcnt[(BS / 64)][kMaxColours];
  __shared__ int any_s;
  __shared__ signed char col_lds[kCopies];
  __shared__ uint32_t wait_lds[kCopies / 2];  // two 16-bit counters per word
  __shared__ uint16_t inc_l[2 * kCopies];     // incidence lists: local copy indices
  __shared__ uint16_t ioff_l[kReps + 1];  // per local replica, into inc_l
  const int p = w.part_order[blockIdx.x];  // largest partitions first
  const int tid = threadIdx.x;
  {
    const int nc = w.part_copy_off[p + 1] - w.part_copy_off[p], nrp = w.part_rep_off[p + 1] - w.part_rep_off[p];
    const bool small = nc <= kColSmallCopies && nrp <= kColSmallReps;
    if (kSmall ? !small : (split && small)) return;  // uniform
  }
  if (tid == 0) any_s = (w.scal[SC_FLAGS] & (F_CONTACT_CAP | F_ADJ_CAP | F_REP_CAP | F_COPY_CAP)) ? 1 : 0;
  __syncthreads();
  if (any_s) return;
  const int u0 = w.part_copy_off[p], u1 = w.part_copy_off[p + 1];
  const int r0 = w.part_rep_off[p], r1 = w.part_rep_off[p + 1];
  const int nr = r1 - r0;
  if (tid == 0) w.part_nstatic[p] = 0;
  int* inc_cnt = w.inc_off + w.Rcap;  // second half of inc_off holds the counts
  // Incidence lists of the partition's replicas: in LDS (16-bit local indices)
  // when the partition fits, else in global memory.  The per-replica counts
  // also go to global memory (the conflict-degree feature reads them).
  // The LDS path keeps 16-bit wait counters: every replica must touch fewer
  // than 2^14 copies so that a copy's count stays below 2^15.  Uniform.
  bool in_lds = u1 - u0 <= kCopies && nr <= kReps;
  if (in_lds) {
    for (int i = tid; i < (nr + 1) / 2; i += BS) wait_lds[i] = 0u;
    __syncthreads();
    for (int u = u0 + tid; u < u1; u += BS) {
      const int ia = w.cp_ia[u], ib = w.cp_ib[u];
      atomicAdd(&wait_lds[ia >> 1], 1u << (16 * (ia & 1)));
      if (ib >= 0) atomicAdd(&wait_lds[ib >> 1], 1u << (16 * (ib & 1)));
    }
    __syncthreads();
    bool busy = false;
    for (int r = tid; r < nr; r += BS) {
      const int c = (wait_lds[r >> 1] >> (16 * (r & 1))) & 0xffff;
      busy |= c >= (1 << 14);
      inc_cnt[r0 + r] = c;
    }
    in_lds = !__syncthreads_or(busy);
  }
  if (in_lds) {
    int carry = 0;
    for (int base = 0; base < nr; base += BS) {
      const int r = base + tid;
      const int v = r < nr ? (wait_lds[r >> 1] >> (16 * (r & 1))) & 0xffff : 0;
      int tot;
      const int pre = block_excl_scan<BS>(v, lds_i, tot);
      if (r < nr) ioff_l[r] = (uint16_t)(carry + pre);
      carry += tot;
    }
    if (tid == 0) ioff_l[nr] = (uint16_t)carry;
    __syncthreads();
    for (int i = tid; i < (nr + 1) / 2; i += BS) wait_lds[i] = 0u;
    __syncthreads();
    for (int u = u0 + tid; u < u1; u += BS) {
      const int ia = w.cp_ia[u], ib = w.cp_ib[u];
      const int ka = (atomicAdd(&wait_lds[ia >> 1], 1u << (16 * (ia & 1))) >> (16 * (ia & 1))) & 0xffff;
      inc_l[ioff_l[ia] + ka] = (uint16_t)(u - u0);
      if (ib >= 0) {
        const int kb = (atomicAdd(&wait_lds[ib >> 1], 1u << (16 * (ib & 1))) >> (16 * (ib & 1))) & 0xffff;
        inc_l[ioff_l[ib] + kb] = (uint16_t)(u - u0);
      }
    }
    __syncthreads();
    for (int u = u0 + tid; u < u1; u += BS) col_lds[u - u0] = -1;
    for (int i = tid; i < (u1 - u0 + 1) / 2; i += BS) wait_lds[i] = 0u;
    __syncthreads();
  } else {
    for (int r = tid; r < nr; r += BS) inc_cnt[r0 + r] = 0;
    __syncthreads();
    for (int u = u0 + tid; u < u1; u += BS) {
      atomicAdd(&inc_cnt[r0 + w.cp_ia[u]], 1);
      int ib = w.cp_ib[u];
      if (ib >= 0) atomicAdd(&inc_cnt[r0 + ib], 1);
    }
    __syncthreads();
    for (int u = u0 + tid; u < u1; u += BS) w.cp_colour[u] = -1;
    {
      int carry = 2 * u0;
      for (int base = 0; base < nr; base += BS) {
        int r = base + tid;
        int v = r < nr ? inc_cnt[r0 + r] : 0;
        int tot;
        int pre = block_excl_scan<BS>(v, lds_i, tot);
        if (r < nr) {
          w.inc_off[r0 + r] = carry + pre;
          inc_cnt[r0 + r] = 0;
        }
        carry += tot;
      }
    }
    __syncthreads();
    for (int u = u0 + tid; u < u1; u += BS) {
      int ia = r0 + w.cp_ia[u];
      w.inc[w.inc_off[ia] + atomicAdd(&inc_cnt[ia], 1)] = u;
      int ib = w.cp_ib[u];
      if (ib >= 0) w.inc[w.inc_off[r0 + ib] + atomicAdd(&inc_cnt[r0 + ib], 1)] = u;
    }
    __syncthreads();
  }
  // Jones-Plassmann.  In LDS (the common case): every copy counts its
  // conflicting copies of higher priority; each round colours the copies whose
  // count is zero (an independent set: of two conflicting copies the lower one
  // still counts the higher), then those copies release their lower-priority
  // neighbours.  Every neighbour list is read twice in all, not once per round.
  // Otherwise (larger partitions) the same rounds run on global colours, each
  // round rechecking the uncoloured copies.
  bool overflow = false;
  auto pick = [&](uint64_t used) -> int {
    if (used == ~0ull) {
      overflow = true;
      return kMaxColours - 1;
    }
    return __ffsll((unsigned long long)~used) - 1;
  };
  if (in_lds) {
    const int per = (u1 - u0 + BS - 1) / BS;  // copies per thread, at most 16
    uint32_t todo = 0;
    for (int j = 0; j < per; ++j) {
      const int u = u0 + tid + j * BS;
      if (u >= u1) break;
      todo |= 1u << j;
      const uint32_t hu = fmix32((uint32_t)u ^ w.seed);
      int n = 0;
      const int ends[2] = {w.cp_ia[u], w.cp_ib[u]};
      for (int e = 0; e < 2; ++e) {
        if (ends[e] < 0) continue;
        for_incident(inc_l, ioff_l[ends[e]], ioff_l[ends[e] + 1], [&](int l) {
          const int o = u0 + l;
          if (o != u && prio_gt(fmix32((uint32_t)o ^ w.seed), o, hu, u)) ++n;
        });
      }
      atomicAdd(&wait_lds[(u - u0) >> 1], (uint32_t)n << (16 * ((u - u0) & 1)));
    }
    __syncthreads();
    // each round colours at least the highest-priority uncoloured copy, so at
    // most u1 - u0 rounds run; the bound only guards against a broken count
    for (int round = 0;; ++round) {
      if (round > u1 - u0) {
        overflow = true;
        break;
      }
      // the thread's copies whose higher-priority neighbours are all coloured:
      // their counters read together rather than one after another
      uint32_t ready = 0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if ((todo >> j) & 1u) {
          const int ul = tid + j * BS;
          const uint32_t wv = wait_lds[ul >> 1] >> (16 * (ul & 1));
          ready |= ((wv & 0xffffu) == 0 ? 1u : 0u) << j;
        }
      }
      uint32_t now = 0;
      for (uint32_t t = ready; t; t &= t - 1) {
        const int j = __ffs(t) - 1;
        const int u = u0 + tid + j * BS;
        uint64_t used = 0;
        const int ends[2] = {w.cp_ia[u], w.cp_ib[u]};
        for (int e = 0; e < 2; ++e) {
          if (ends[e] < 0) continue;
          for_incident(inc_l, ioff_l[ends[e]], ioff_l[ends[e] + 1], [&](int l) {
            const int co = col_lds[l];
            if (co >= 0) used |= 1ull << co;
          });
        }
        col_lds[u - u0] = (signed char)pick(used);
        now |= 1u << j;
      }
      todo &= ~now;
      __syncthreads();
      for (uint32_t t = now; t; t &= t - 1) {
        const int j = __ffs(t) - 1;
        const int u = u0 + tid + j * BS;
        const uint32_t hu = fmix32((uint32_t)u ^ w.seed);
        const int ends[2] = {w.cp_ia[u], w.cp_ib[u]};
        for (int e = 0; e < 2; ++e) {
          if (ends[e] < 0) continue;
          for_incident(inc_l, ioff_l[ends[e]], ioff_l[ends[e] + 1], [&](int l) {
            const int o = u0 + l;
            if (o != u && prio_gt(hu, u, fmix32((uint32_t)o ^ w.seed), o))
              atomicSub(&wait_lds[(o - u0) >> 1], 1u << (16 * ((o - u0) & 1)));
          });
        }
      }
      if (!__syncthreads_or(todo != 0)) break;
    }
  } else {
    for (;;) {
      bool pending = false;
      for (int u = u0 + tid; u < u1; u += BS) {
        if (__hip_atomic_load(&w.cp_colour[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= 0) continue;
        const uint32_t hu = fmix32((uint32_t)u ^ w.seed);
        uint64_t used = 0;
        bool ready = true;
        int ends[2] = {r0 + w.cp_ia[u], w.cp_ib[u] >= 0 ? r0 + w.cp_ib[u] : -1};
        for (int e = 0; e < 2 && ready; ++e) {
          if (ends[e] < 0) continue;
          const int k0 = w.inc_off[ends[e]], k1 = k0 + inc_cnt[ends[e]];
          for (int k = k0; k < k1; ++k) {
            int o = w.inc[k];
            if (o == u) continue;
            int co = __hip_atomic_load(&w.cp_colour[o], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (co >= 0) {
              used |= 1ull << co;
            } else if (prio_gt(fmix32((uint32_t)o ^ w.seed), o, hu, u)) {
              ready = false;
              break;
            }
          }
        }
        if (ready)
          __hip_atomic_store(&w.cp_colour[u], pick(used), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          pending = true;
      }
      if (!__syncthreads_or(pending)) break;
    }
  }
  if (__syncthreads_or(overflow) && tid == 0) atomicOr(&w.scal[SC_FLAGS], F_COLOUR_CAP);
  if (in_lds)  // a copy left uncoloured by the round bound gets a valid colour (the step is flagged)
    for (int u = u0 + tid; u < u1; u += BS) w.cp_colour[u] = col_lds[u - u0] < 0 ? kMaxColours - 1 : col_lds[u - u0];
  __syncthreads();
  // colour histogram and offsets
  if (tid < kMaxColours) {
    ccount[tid] = 0;
    running[tid] = 0;
  }
  __syncthreads();
  for (int u = u0 + tid; u < u1; u += BS) atomicAdd(&ccount[w.cp_colour[u]], 1);
  __syncthreads();
  if (tid == 0) {
    int acc = 0, ncol = 0;
    for (int k = 0; k < kMaxColours; ++k) {
      col_off[k] = acc;
      acc += ccount[k];
      if (ccount[k]) ncol = k + 1;
    }
    col_off[kMaxColours] = acc;
    w.part_ncol[p] = ncol;
  }
  __syncthreads();
  if (tid < kColStride) w.part_col_off[p * kColStride + tid] = col_off[tid];
  // stable slots: rank inside the colour in uid order
  const int wave = tid >> 6;
  for (int base = u0; base < u1; base += BS) {
    const int u = base + tid;
    const int col = u < u1 ? w.cp_colour[u] : -1;
    wcnt[wave][lane_id()] = 0;
    __syncthreads();
    uint64_t present = col >= 0 ? (1ull << col) : 0ull;
    present = wave_or(present);
    int myrank = 0;
    for (uint64_t bb = present; bb; bb &= bb - 1) {
      int k = __ffsll((unsigned long long)bb) - 1;
      uint64_t bal = ballot64(col == k);
      if (col == k) myrank = __popcll(bal & lanemask_lt());
      if (lane_id() == 0) wcnt[wave][k] = __popcll(bal);
    }
    __syncthreads();
    if (col >= 0) {
      int pre = 0;
      for (int q = 0; q < wave; ++q) pre += wcnt[q][col];
      w.cp_slot[u] = u0 + col_off[col] + running[col] + pre + myrank;
    }
    __syncthreads();
    if (tid < kMaxColours) {
      int t = 0;
      for (int q = 0; q < (BS / 64); ++q) t += wcnt[q][tid];
      running[tid] += t;
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------- rows ----

// Warm-start cache lookup: the previous step's entries of partition `part`
// are [wc_off[part], wc_off[part+1]), sorted by kind << 63 | key.  n: the
// number of entries (0: no cache).
__device__ __forceinline__ int cache_find(const WP& w, int n, int part, int kind, uint64_t key) {
  if (n <= 0) return -1;
  const uint64_t k = ((uint64_t)kind << 63) | key;
  int lo = w.wc_off[part], hi = w.wc_off[part + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (w.wc_k64[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < w.wc_off[part + 1] && w.wc_k64[lo] == k) return lo;
  return -1;
}

// ----------------------------------------------------- interface coupling ----
// One thread per body v.  For each partition i that v is active in and one of
// v's constraint-graph neighbours is not, the constraints of v whose other
// body is outside P_i are cut from i's solve.  Each one's impulse of the
// previous step (cache entry of the lowest partition active in both bodies,
// converted as the warm start converts it) acts on v as F at v's lever arm:
// dv = F/m, dw = I^-1 (r x F), F = -sum_r lambda_r d_r on body a and
// +sum_r lambda_r d_r on body b.  Summed per replica in constraint-list order
// (joints by index, then contacts by key: those where v is body b come first,
// their body a being smaller) into rep_cpl.
__device__ __forceinline__ void couple_add(const WP& w, int v, f3 F, f3 r, f3& dv, f3& dw) {
  const float im = w.b_invm[v], ii = w.b_invI[v];
  const f3 u = w.has_caps ? body_axis(w, v) : mk(0.0f, 0.0f, 1.0f);
  const float dI = w.has_caps ? w.b_dI[v] : 0.0f;
  dv = add(dv, scale(F, im));
  dw = add(dw, inv_inertia(ii, u, dI, cross(r, F)));
}

__device__ __forceinline__ bool couple_contact(const WP& w, int prevM, int pb, uint64_t mv, int v, int c, f3& dv,
                                               f3& dw) {
  const int64_t MC = w.Mcap, CC = w.Ccap;
  const int a = w.c_a[c];
  const uint32_t bk = w.c_bkey[c];
  const int b = (int)(bk >> 1);
  const int o = a == v ? b : a;
  const uint64_t both = mv & w.mask[o];
  if (!both) return false;
  const int hit = cache_find(w, prevM, pb + __builtin_ctzll(both), 1, ((uint64_t)a << 32) | bk);
  if (hit < 0) return false;
  const f3 n = mk(w.c_geom[c], w.c_geom[CC + c], w.c_geom[2 * CC + c]);
  f3 t1, t2;
  tangents(n, t1, t2);
  const float ln = fmaxf(w.wc_val[hit], 0.0f);
  const f3 fw = mk(w.wc_val[MC + hit], w.wc_val[2 * MC + hit], w.wc_val[3 * MC + hit]);
  const float bnd = w.s_mu[w.b_scene[a]] * ln;
  const float l1 = fminf(fmaxf(dot(fw, t1), -bnd), bnd);
  const float l2 = fminf(fmaxf(dot(fw, t2), -bnd), bnd);
  const f3 P = add(add(scale(n, ln), scale(t1, l1)), scale(t2, l2));
  f3 ra, rb;
  contact_arms(w, c, a, b, n, ra, rb);
  if (a == v)
    couple_add(w, v, scale(P, -1.0f), ra, dv, dw);
  else
    couple_add(w, v, P, rb, dv, dw);
  return true;
}

__global__ void k_couple(WP w) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N || step_failed(w)) return;
  const int N = w.N;
  const uint64_t m = w.mask[v];
  const int n = __popcll(m);
  const int bm0 = w.rep_off_bm[v];
  const int64_t RC = w.Rcap;
  for (int k = 0; k < n; ++k) {
    const int r = w.rep_pm_of_bm[bm0 + k];
    w.rep_cpl[r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    w.rep_cpl[RC + r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  const int prevM = w.scal[SC_PREV_NCOPY];
  if (prevM <= 0 || w.adj_off[N] > w.Acap) return;
  const int a0 = w.adj_off[v], a1 = w.adj_off[v + 1];
  uint64_t cut = 0;
  for (int k = a0; k < a1; ++k) {
    const int u = w.adj[k];
    if (u >= 0) cut |= m & ~w.mask[u];
  }
  if (!cut) return;
  const int pb = w.s_part_base[w.b_scene[v]];
  // A constraint's impulse on v is found once and added to every replica of
  // v in whose partition the constraint is cut (cm: those partitions' bits);
  // each replica's sum still runs in constraint-list order.
  auto add_to = [&](uint64_t cm, f3 dv, f3 dw) {
    for (uint64_t bits = cm; bits; bits &= bits - 1) {
      const int i = __builtin_ctzll(bits);
      const int r = w.rep_pm_of_bm[bm0 + __popcll(m & ((1ull << i) - 1))];
      const float4 a = w.rep_cpl[r], b = w.rep_cpl[RC + r];
      w.rep_cpl[r] = make_float4(a.x + dv.x, a.y + dv.y, a.z + dv.z, 0.0f);
      w.rep_cpl[RC + r] = make_float4(b.x + dw.x, b.y + dw.y, b.z + dw.z, 0.0f);
    }
  };
  // ball joints (rows along -e_k: the impulse on body a is +lambda)
  for (int e = w.jinc_off[v]; e < w.jinc_off[v + 1]; ++e) {
    const int j = w.jinc[e];
    const int ja = w.j_ab[2 * j], jb = w.j_ab[2 * j + 1];
    const int o = ja == v ? jb : ja;
    const uint64_t mo = w.mask[o], cm = m & ~mo, both = m & mo;
    if (!cm || !both) continue;
    const int hit = cache_find(w, prevM, pb + __builtin_ctzll(both), 0, (uint64_t)j);
    if (hit < 0) continue;
    const int64_t MC = w.Mcap;
    const f3 lam = mk(w.wc_val[hit], w.wc_val[MC + hit], w.wc_val[2 * MC + hit]);
    const float* an = w.j_anchor + 6 * j + (ja == v ? 0 : 3);
    const f3 r = quat_rotate(w.st[3 * N + v], w.st[4 * N + v], w.st[5 * N + v], w.st[6 * N + v],
                             mk(an[0], an[1], an[2]));
    f3 dv = mk(0.0f, 0.0f, 0.0f), dw = mk(0.0f, 0.0f, 0.0f);
    couple_add(w, v, ja == v ? lam : scale(lam, -1.0f), r, dv, dw);
    add_to(cm, dv, dw);
  }
  // contacts whose body a is a smaller neighbour u (adjacency is sorted, -1 padded)
  for (int k = a0; k < a1; ++k) {
    const int u = w.adj[k];
    if (u < 0 || u >= v) break;
    const uint64_t cm = m & ~w.mask[u];
    if (!cm) continue;
    for (int c = w.coff[u]; c < w.coff[u + 1]; ++c)
      if ((w.c_bkey[c] >> 1) == (uint32_t)v) {
        f3 dv = mk(0.0f, 0.0f, 0.0f), dw = mk(0.0f, 0.0f, 0.0f);
        if (couple_contact(w, prevM, pb, m, v, c, dv, dw)) add_to(cm, dv, dw);
      }
  }
  // contacts whose body a is v
  for (int c = w.coff[v]; c < w.coff[v + 1]; ++c) {
    const uint32_t o = w.c_bkey[c] >> 1;
    if (o >= (uint32_t)N) continue;
    const uint64_t cm = m & ~w.mask[o];
    if (!cm) continue;
    f3 dv = mk(0.0f, 0.0f, 0.0f), dw = mk(0.0f, 0.0f, 0.0f);
    if (couple_contact(w, prevM, pb, m, v, c, dv, dw)) add_to(cm, dv, dw);
  }
}

// Features of a contact copy for the learned warm start (joints: zeros).
// Velocities are those at the start of the solve (v~ = v + h g); the velocity
// scale is g h and the impulse scale s = g h / (1/m_a + 1/m_b):
//   n (3), relative contact-point velocity in (n, t1, t2) / (g h) (3),
//   gap / margin, (1/m_a, 1/m_b) / (1/m_a + 1/m_b) (2), the plain start
//   (lambda_n, |lambda_t|) / s (2), conflict degree / 16; then s.
__device__ void write_features(const WP& w, int u, int src, int p, float l0, float l1, float l2) {
  float* f = w.r_feat + (int64_t)u * kFeatStride;
  if (src < w.J) {
    for (int k = 0; k < kFeatStride; ++k) f[k] = 0.0f;
    return;
  }
  const int N = w.N;
  const int c = src - w.J;
  const int a = w.c_a[c];
  const uint32_t bk = w.c_bkey[c];
  const int b = (bk >> 1) < (uint32_t)N ? (int)(bk >> 1) : -1;
  const int64_t CC = w.Ccap;
  const f3 n = mk(w.c_geom[c], w.c_geom[CC + c], w.c_geom[2 * CC + c]);
  const float phi = w.c_geom[3 * CC + c];
  f3 ra, rb;
  contact_arms(w, c, a, b, n, ra, rb);
  f3 t1, t2;
  tangents(n, t1, t2);
  const float h = w.dt;
  const f3 hg = mk(h * w.gx, h * w.gy, h * w.gz);
  const int r0 = w.part_rep_off[p];
  f3 va = add(mk(w.st[7 * N + a], w.st[8 * N + a], w.st[9 * N + a]), hg);
  f3 wa = mk(w.st[10 * N + a], w.st[11 * N + a], w.st[12 * N + a]);
  if (w.couple) {
    const float4 cv = w.rep_cpl[r0 + w.cp_ia[u]], cw = w.rep_cpl[w.Rcap + r0 + w.cp_ia[u]];
    va = add(va, mk(cv.x, cv.y, cv.z));
    wa = add(wa, mk(cw.x, cw.y, cw.z));
  }
  f3 pa = add(va, cross(wa, ra));
  f3 pb = mk(0, 0, 0);
  const float ima = w.b_invm[a] * rep_split(w, p, w.cp_ia[u]);
  float imb = 0.0f;
  if (b >= 0) {
    f3 vb = add(mk(w.st[7 * N + b], w.st[8 * N + b], w.st[9 * N + b]), hg);
    f3 wb = mk(w.st[10 * N + b], w.st[11 * N + b], w.st[12 * N + b]);
    if (w.couple) {
      const float4 cv = w.rep_cpl[r0 + w.cp_ib[u]], cw = w.rep_cpl[w.Rcap + r0 + w.cp_ib[u]];
      vb = add(vb, mk(cv.x, cv.y, cv.z));
      wb = add(wb, mk(cw.x, cw.y, cw.z));
    }
    pb = add(vb, cross(wb, rb));
    imb = w.b_invm[b] * rep_split(w, p, w.cp_ib[u]);
  }
  const f3 vr = sub(pb, pa);
  const float g = sqrtf(w.gx * w.gx + w.gy * w.gy + w.gz * w.gz);
  const float vs = g * h > 0.0f ? g * h : 1.0f;
  const float sim = vs / (ima + imb);
  const float margin = w.s_margin[w.b_scene[a]];
  const int* inc_cnt = w.inc_off + w.Rcap;
  int deg = inc_cnt[r0 + w.cp_ia[u]] - 1;
  if (b >= 0) deg += inc_cnt[r0 + w.cp_ib[u]] - 1;
  f[0] = n.x;
  f[1] = n.y;
  f[2] = n.z;
  f[3] = dot(vr, n) / vs;
  f[4] = dot(vr, t1) / vs;
  f[5] = dot(vr, t2) / vs;
  f[6] = margin > 0.0f ? phi / margin : phi;
  f[7] = ima / (ima + imb);
  f[8] = imb / (ima + imb);
  f[9] = l0 / sim;
  f[10] = sqrtf(l1 * l1 + l2 * l2) / sim;
  f[11] = (float)deg / 16.0f;
  f[12] = sim;
  f[13] = f[14] = f[15] = 0.0f;
}

// Ids of a copy in 32 bits: local replica a (bits 0-13), joint (14), capsule
// rows (15), local replica b + 1 (bits 16-31; 0 = static).  Stored, as bits,
// in the fourth component of the copy's impulse, which the sweeps load anyway.
constexpr int kPackReps = 16384;

__device__ __forceinline__ float pack_ids(int2 id) {
  const uint32_t ia = (uint32_t)(id.x & ~(kJointFlag | kGenFlag));
  const uint32_t pk = ia | ((id.x & kJointFlag) ? 0x4000u : 0u) | ((id.x & kGenFlag) ? 0x8000u : 0u) |
                      ((uint32_t)(id.y + 1) << 16);
  return __uint_as_float(pk);
}

__global__ void k_rows(WP w) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int M = w.part_copy_off[w.G];
  if (u >= M || u >= w.Mcap || step_failed(w)) return;
  const int N = w.N;
  const int slot = w.cp_slot[u];
  const int src = w.cp_src[u];
  const int p = w.cp_part[u];
  const int64_t MC = w.Mcap;
  float l0 = 0.0f, l1 = 0.0f, l2 = 0.0f;
  const int prevM = w.scal[SC_PREV_NCOPY];
  const bool warm = w.warmstart && prevM > 0;
  if (src < w.J) {
    const int a = w.j_ab[2 * src], b = w.j_ab[2 * src + 1];
    const float* an = w.j_anchor + 6 * src;
    const f3 ra = quat_rotate(w.st[3 * N + a], w.st[4 * N + a], w.st[5 * N + a], w.st[6 * N + a],
                              mk(an[0], an[1], an[2]));
    const f3 rb = quat_rotate(w.st[3 * N + b], w.st[4 * N + b], w.st[5 * N + b], w.st[6 * N + b],
                              mk(an[3], an[4], an[5]));
    // C = (x_a + r_a) - (x_b + r_b), grouped so that the difference of the two
    // nearby centres is taken first (exact in float) instead of cancelling two
    // rounded sums of large coordinates
    const f3 dx = mk(w.st[a] - w.st[b], w.st[N + a] - w.st[N + b], w.st[2 * N + a] - w.st[2 * N + b]);
    const f3 C = add(dx, sub(ra, rb));
    const float k = w.erp / w.dt;
    const float sa = rep_split(w, p, w.cp_ia[u]), sb = rep_split(w, p, w.cp_ib[u]);
    const float ima = w.b_invm[a] * sa, iia = w.b_invI[a] * sa, imb = w.b_invm[b] * sb, iib = w.b_invI[b] * sb;
    float Ax, Ay, Az;
    const bool gen = w.has_caps && (w.b_half[a] > 0.0f || w.b_half[b] > 0.0f);
    if (!gen) {
      // rows along -e_x, -e_y, -e_z: |r x e_k|^2 = |r|^2 - r_k^2
      const float raa = dot(ra, ra), rbb = dot(rb, rb);
      Ax = ima + imb + iia * (raa - ra.x * ra.x) + iib * (rbb - rb.x * rb.x) + w.cfm;
      Ay = ima + imb + iia * (raa - ra.y * ra.y) + iib * (rbb - rb.y * rb.y) + w.cfm;
      Az = ima + imb + iia * (raa - ra.z * ra.z) + iib * (rbb - rb.z * rb.z) + w.cfm;
    } else {
      const f3 ua = body_axis(w, a), ub = body_axis(w, b);
      const float dIa = w.b_dI[a] * sa, dIb = w.b_dI[b] * sb;
      float Ak[3];
      for (int e = 0; e < 3; ++e) {
        const f3 ek = mk(e == 0 ? 1.0f : 0.0f, e == 1 ? 1.0f : 0.0f, e == 2 ? 1.0f : 0.0f);
        const f3 ca = cross(ra, ek), cb = cross(rb, ek);
        Ak[e] = ima + imb + dot(ca, inv_inertia(iia, ua, dIa, ca)) + dot(cb, inv_inertia(iib, ub, dIb, cb)) + w.cfm;
      }
      Ax = Ak[0];
      Ay = Ak[1];
      Az = Ak[2];
    }
    w.r_rec[slot] = make_float4(ra.x, ra.y, ra.z, k * C.x);
    w.r_rec[MC + slot] = make_float4(rb.x, rb.y, rb.z, k * C.y);
    w.r_rec[2 * MC + slot] = make_float4(1.0f / Ax, 1.0f / Ay, 1.0f / Az, k * C.z);
    w.r_ids[slot] = make_int2(w.cp_ia[u] | kJointFlag | (gen ? kGenFlag : 0), w.cp_ib[u]);
    if (warm) {
      const int hit = cache_find(w, prevM, p, 0, (uint64_t)src);
      if (hit >= 0) {
        l0 = w.wc_val[hit];
        l1 = w.wc_val[MC + hit];
        l2 = w.wc_val[2 * MC + hit];
      }
    }
  } else {
    const int c = src - w.J;
    const int a = w.c_a[c];
    const uint32_t bk = w.c_bkey[c];
    const int b = (bk >> 1) < (uint32_t)N ? (int)(bk >> 1) : -1;
    const int64_t CC = w.Ccap;
    const f3 n = mk(w.c_geom[c], w.c_geom[CC + c], w.c_geom[2 * CC + c]);
    const float phi = w.c_geom[3 * CC + c];
    const float la = w.c_geom[4 * CC + c], lb = w.c_geom[5 * CC + c];
    f3 t1, t2;
    const float ad = tangents(n, t1, t2);
    if (b < 0) atomicAdd(&w.part_nstatic[p], 1);
    const float bias = phi > 0.0f ? phi / w.dt : w.erp * phi / w.dt;
    const float mu = w.s_mu[w.b_scene[a]];
    const float sa = rep_split(w, p, w.cp_ia[u]), sb = b >= 0 ? rep_split(w, p, w.cp_ib[u]) : 0.0f;
    const float ima = w.b_invm[a] * sa, iia = w.b_invI[a] * sa;
    const float imb = b >= 0 ? w.b_invm[b] * sb : 0.0f, iib = b >= 0 ? w.b_invI[b] * sb : 0.0f;
    const bool gen = w.has_caps && (w.b_half[a] > 0.0f || (b >= 0 && w.b_half[b] > 0.0f));
    if (!gen) {
      // sphere contact: r_a = l_a n, r_b = -l_b n, so r x n = 0 and |r x t|^2 = l^2
      w.r_rec[slot] = make_float4(n.x, n.y, n.z, ad);
      w.r_rec[MC + slot] = make_float4(la, lb, bias, mu);
      w.r_rec[2 * MC + slot] = sphere_row_masses(ima, imb, la, iia * la, lb, iib * lb, w.cfm);
      w.r_ids[slot] = make_int2(w.cp_ia[u], b >= 0 ? w.cp_ib[u] : -1);
    } else {
      // capsule contact: full lever arms, A_rr = m_a^-1 + m_b^-1 + sum (r x d).I^-1 (r x d)
      f3 ra, rb;
      contact_arms(w, c, a, b, n, ra, rb);
      if (b < 0) rb = mk(0.0f, 0.0f, 0.0f);
      const f3 ua = body_axis(w, a), ub = b >= 0 ? body_axis(w, b) : mk(0.0f, 0.0f, 0.0f);
      const float dIa = w.b_dI[a] * sa, dIb = b >= 0 ? w.b_dI[b] * sb : 0.0f;
      const f3 dirs[3] = {n, t1, t2};
      float Ad[3];
      for (int e = 0; e < 3; ++e) {
        const f3 ca = cross(ra, dirs[e]), cb = cross(rb, dirs[e]);
        Ad[e] = ima + imb + dot(ca, inv_inertia(iia, ua, dIa, ca)) + dot(cb, inv_inertia(iib, ub, dIb, cb)) + w.cfm;
      }
      w.r_rec[slot] = make_float4(n.x, n.y, n.z, ad);
      w.r_rec[MC + slot] = make_float4(Ad[0], 0.0f, bias, mu);
      w.r_rec[2 * MC + slot] = make_float4(1.0f / Ad[0], 1.0f / Ad[1], 1.0f / Ad[2], 0.0f);
      w.r_gen[slot] = make_float4(ra.x, ra.y, ra.z, Ad[1]);
      w.r_gen[MC + slot] = make_float4(rb.x, rb.y, rb.z, Ad[2]);
      w.r_ids[slot] = make_int2(w.cp_ia[u] | kGenFlag, b >= 0 ? w.cp_ib[u] : -1);
    }
    if (warm) {
      const int hit = cache_find(w, prevM, p, 1, ((uint64_t)a << 32) | bk);
      if (hit >= 0) {
        const float* v = w.wc_val;
        const float ln = fmaxf(v[hit], 0.0f);
        const f3 fw = mk(v[MC + hit], v[2 * MC + hit], v[3 * MC + hit]);
        const float bnd = mu * ln;
        l0 = ln;
        l1 = fminf(fmaxf(dot(fw, t1), -bnd), bnd);
        l2 = fminf(fmaxf(dot(fw, t2), -bnd), bnd);
      }
    }
  }
  // partitions with fewer than kPackReps replicas carry the ids in the impulse's fourth component
  const float pk = w.part_rep_off[p + 1] - w.part_rep_off[p] < kPackReps ? pack_ids(w.r_ids[slot]) : 0.0f;
  w.r_lam0[slot] = make_float4(l0, l1, l2, pk);
  w.r_lam[slot] = make_float4(l0, l1, l2, pk);
  if (w.feat_on) write_features(w, u, src, p, l0, l1, l2);
}

// ---------------------------------------------------------- Gauss-Seidel ----
// Replica velocity storage: two float4 per replica, (v, 1/m) and (w, 1/I), in
// two arrays `stride` apart (so consecutive replicas are 16 B apart and random
// gathers spread over all LDS banks): in LDS, or for partitions too large for
// LDS in the partition's slice of rep_v4 (stride Rcap).
struct Vel {
  float4* p;
  int stride;
};

struct Rec {
  float4 r0, r1, r2, lam;
  float4 g0, g1;  // capsule rows only: (r_a, A_t1), (r_b, A_t2)
  int2 id;        // raw ids as stored
  int ia, ib;
  bool joint, gen;
};

// Issue the loads of a record without using them, so a prefetch does not wait
// for its data (decode() reads the ids when the record is solved).  kCaps: the
// world has capsules; the lever-arm records are then always loaded.
// packed: the partition has fewer than kPackReps replicas, and the impulse's
// fourth component carries the ids (pack_ids), so r_ids is not read.
template <bool kCaps>
__device__ __forceinline__ void fetch_rec(const WP& w, int slot, Rec& R, bool packed) {
  const int64_t MC = w.Mcap;
  R.r0 = w.r_rec[slot];
  R.r1 = w.r_rec[MC + slot];
  R.r2 = w.r_rec[2 * MC + slot];
  if (!packed) R.id = w.r_ids[slot];
  R.lam = w.r_lam[slot];
  if (kCaps) {
    R.g0 = w.r_gen[slot];
    R.g1 = w.r_gen[MC + slot];
  }
}

template <bool kCaps>
__device__ __forceinline__ void decode(Rec& R, bool packed) {
  if (packed) {
    const uint32_t pk = __float_as_uint(R.lam.w);
    R.ia = (int)(pk & 0x3fffu);
    R.joint = (pk & 0x4000u) != 0;
    R.gen = kCaps && (pk & 0x8000u) != 0;
    R.ib = (int)(pk >> 16) - 1;
    return;
  }
  R.joint = (R.id.x & kJointFlag) != 0;
  R.gen = kCaps && (R.id.x & kGenFlag) != 0;
  R.ia = R.id.x & ~(kJointFlag | kGenFlag);
  R.ib = R.id.y;
}

template <bool kCaps>
__device__ __forceinline__ void load_rec(const WP& w, int slot, Rec& R, bool packed = false) {
  fetch_rec<kCaps>(w, slot, R, packed);
  decode<kCaps>(R, packed);
}

// The record arrays of one partition, from its first slot: the sweeps address
// a slot by its 32-bit byte offset from these scalar bases (one vector
// instruction per slot for all of its loads and its impulse store).
struct Slots {
  const char *r0, *r1, *r2, *ids, *g0, *g1;
  char* lam;
};

__device__ __forceinline__ Slots slots_of(const WP& w, int s0) {
  // s0 is the same in every lane; taking it from the first lane keeps the
  // bases in scalar registers
  const int64_t u = __builtin_amdgcn_readfirstlane(s0);
  const int64_t MC = w.Mcap;
  Slots S;
  S.r0 = reinterpret_cast<const char*>(w.r_rec + u);
  S.r1 = reinterpret_cast<const char*>(w.r_rec + MC + u);
  S.r2 = reinterpret_cast<const char*>(w.r_rec + 2 * MC + u);
  S.ids = reinterpret_cast<const char*>(w.r_ids + u);
  S.g0 = reinterpret_cast<const char*>(w.r_gen + u);
  S.g1 = reinterpret_cast<const char*>(w.r_gen + MC + u);
  S.lam = reinterpret_cast<char*>(w.r_lam + u);
  return S;
}

// fetch_rec for the slot at local index base + tid of the partition (see
// fetch_rec): `base` is the same in every lane, so its byte offset joins the
// scalar bases, and toff = 16 tid is the lane's vector offset.  Lanes may read
// up to a workgroup past the last slot: the record arrays are padded by
// kSlotPad slots.  kCompact (sphere contacts only) leaves out the third row
// record (the row masses), which do_slot forms again from the replicas.
template <bool kCaps, bool kCompact = false>
__device__ __forceinline__ void fetch_lane(const Slots& S, int base, uint32_t toff, Rec& R, bool packed) {
  // one 32-bit vector offset from the partition's scalar bases for all the loads
  const uint32_t o = ((uint32_t)base << 4) + toff;
  R.r0 = *reinterpret_cast<const float4*>(S.r0 + o);
  R.r1 = *reinterpret_cast<const float4*>(S.r1 + o);
  if (!kCompact) R.r2 = *reinterpret_cast<const float4*>(S.r2 + o);
  if (!packed) R.id = *reinterpret_cast<const int2*>(S.ids + (o >> 1));
  R.lam = *reinterpret_cast<const float4*>(S.lam + o);
  if (kCaps) {
    R.g0 = *reinterpret_cast<const float4*>(S.g0 + o);
    R.g1 = *reinterpret_cast<const float4*>(S.g1 + o);
  }
}

struct Bod {
  f3 v, w;
  float im, ii;
};

__device__ __forceinline__ Bod ld_body(Vel V, int r) {
  const float4 a = V.p[r], b = V.p[r + V.stride];
  return {mk(a.x, a.y, a.z), mk(b.x, b.y, b.z), a.w, b.w};
}

// the inverse mass and inertia never change during the solve: only v and w are stored
__device__ __forceinline__ void st_body(Vel V, int r, const Bod& B) {
  float* a = reinterpret_cast<float*>(V.p + r);
  float* b = reinterpret_cast<float*>(V.p + r + V.stride);
  a[0] = B.v.x;
  a[1] = B.v.y;
  a[2] = B.v.z;
  b[0] = B.w.x;
  b[1] = B.w.y;
  b[2] = B.w.z;
}

__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Contact (three rows n, t1, t2).  With r_a = l_a n and r_b = -l_b n:
//   J_n v  = n.(v_b - v_a)
//   J_t1 v = t1.(v_b - v_a) - t2.(l_a w_a + l_b w_b)
//   J_t2 v = t2.(v_b - v_a) + t1.(l_a w_a + l_b w_b)
// and the impulse dl of a row moves v_a by -dl/m_a d, v_b by +dl/m_b d, and the
// spins by the matching lever-arm terms.  For such a contact the three rows
// are decoupled (J_i M^-1 J_j^T = 0 for i != j): an impulse on one row leaves
// the other rows' velocities unchanged.  Solving the rows in order n, t1, t2
// therefore only needs the velocities before the contact, and the three
// impulses are applied together.  `solve` false applies lam as given (warm
// start) instead of projecting.  r2 = (1/A_n, 1/A_t, A_n, A_t); kCompact forms
// it here from the bodies' inverse masses instead (see sphere_row_masses).
//
// The tangents are never formed.  With s = sign(n_z), a the record's basis
// coefficient and m = (a n_x, a n_y, -1), the basis of tangents_from is
// t1 = e_x + s n_x m and t2 = s e_y + n_y m, so for any vector v
//   n.v = h + n_z v_z,  t1.v = v_x + s n_x k,  t2.v = s v_y + n_y k,
// with h = n_x v_x + n_y v_y and k = m.v = a h - v_z; and the impulse vectors
//   P = n d0 + t1 d1 + t2 d2 = (n_x r + d1, n_y r + s d2, n_z d0 - c),
//   Q = t2 d1 - t1 d2 = (a n_x e - d2, a n_y e + s d1, -e),
// with c = s n_x d1 + n_y d2, r = d0 + a c and e = n_y d1 - s n_x d2.
template <bool solve, bool kCompact = false>
__device__ __forceinline__ void contact_rows(const Rec& R, Bod& A, Bod& B, float cfm, float4& lam, float& rl,
                                             float4 r2) {
  const f3 n = mk(R.r0.x, R.r0.y, R.r0.z);
  const float a = R.r0.w;
  const float s = copysignf(1.0f, n.z), sx = s * n.x;
  const float la = R.r1.x, lb = R.r1.y, bias = R.r1.z, mu = R.r1.w;
  const float lia = A.ii * la, lib = B.ii * lb;
  if (kCompact) r2 = sphere_row_masses(A.im, B.im, la, lia, lb, lib, cfm);
  float d0, d1, d2;
  if (solve) {
    const f3 dv = sub(B.v, A.v);
    const f3 sw = madd(scale(B.w, lb), A.w, la);
    const float h1 = fmaf(n.y, dv.y, n.x * dv.x), k1 = fmaf(a, h1, -dv.z);
    const float h2 = fmaf(n.y, sw.y, n.x * sw.x), k2 = fmaf(a, h2, -sw.z);
    // normal
    const float un = fmaf(cfm, lam.x, fmaf(n.z, dv.z, h1) + bias);
    const float ln = fmaxf(fmaf(-un, r2.x, lam.x), 0.0f);
    d0 = ln - lam.x;
    lam.x = ln;
    // friction box of the new normal impulse
    const float hi = mu * ln;
    const float u1 = fmaf(cfm, lam.y, fmaf(sx, k1, dv.x) - fmaf(n.y, k2, s * sw.y));
    const float l1 = fminf(fmaxf(fmaf(-u1, r2.y, lam.y), -hi), hi);
    d1 = l1 - lam.y;
    lam.y = l1;
    const float u2 = fmaf(cfm, lam.z, fmaf(n.y, k1, s * dv.y) + fmaf(sx, k2, sw.x));
    const float l2 = fminf(fmaxf(fmaf(-u2, r2.y, lam.z), -hi), hi);
    d2 = l2 - lam.z;
    lam.z = l2;
    rl = fmaxf(rl, fmaxf(fabsf(d0) * r2.z, fmaxf(fabsf(d1), fabsf(d2)) * r2.w));
  } else {
    d0 = lam.x;
    d1 = lam.y;
    d2 = lam.z;
  }
  const float c = fmaf(n.y, d2, sx * d1), r = fmaf(a, c, d0);
  const float e = fmaf(n.y, d1, -(sx * d2)), ae = a * e;
  const f3 P = mk(fmaf(n.x, r, d1), fmaf(n.y, r, s * d2), fmaf(n.z, d0, -c));
  const f3 Q = mk(fmaf(n.x, ae, -d2), fmaf(n.y, ae, s * d1), -e);
  A.v = msub(A.v, P, A.im);
  B.v = madd(B.v, P, B.im);
  A.w = msub(A.w, Q, lia);
  B.w = msub(B.w, Q, lib);
}

// Ball joint, rows along -e_k: J_k v = (v_a + w_a x r_a - v_b - w_b x r_b)_k;
// the impulse dl of row k moves v_a by +dl/m_a e_k and w_a by +dl I_a^-1 (r_a x e_k),
// and body b the opposite way.  The rows are written out per axis so that no
// product with a zero component of e_k is formed.
__device__ __forceinline__ f3 cross_axis(f3 r, int k) {
  // r x e_k
  return k == 0 ? mk(0.0f, r.z, -r.y) : (k == 1 ? mk(-r.z, 0.0f, r.x) : mk(r.y, -r.x, 0.0f));
}

// v_k += a b (fused)
__device__ __forceinline__ void add_axis(f3& v, int k, float a, float b) {
  if (k == 0)
    v.x = fmaf(a, b, v.x);
  else if (k == 1)
    v.y = fmaf(a, b, v.y);
  else
    v.z = fmaf(a, b, v.z);
}

template <bool solve, bool kGen = false>
__device__ __forceinline__ void joint_rows(const Rec& R, Bod& A, Bod& B, float cfm, float4& lam, float& rl,
                                           float4 axA = float4{}, float4 axB = float4{}) {
  const f3 ra = mk(R.r0.x, R.r0.y, R.r0.z), rb = mk(R.r1.x, R.r1.y, R.r1.z);
  const float bias[3] = {R.r0.w, R.r1.w, R.r2.w};
  const float invd[3] = {R.r2.x, R.r2.y, R.r2.z};
  float* l = &lam.x;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float dl;
    if (solve) {
      // (v_a + w_a x r_a - v_b - w_b x r_b)_k
      const f3 ca = cross(A.w, ra), cb = cross(B.w, rb);
      const float vr = k == 0 ? (A.v.x + ca.x) - (B.v.x + cb.x)
                              : (k == 1 ? (A.v.y + ca.y) - (B.v.y + cb.y) : (A.v.z + ca.z) - (B.v.z + cb.z));
      const float wv = fmaf(cfm, l[k], vr + bias[k]);
      const float nl = fmaf(-wv, invd[k], l[k]);
      dl = nl - l[k];
      l[k] = nl;
      rl = fmaxf(rl, fabsf(dl) * rcp_fast(invd[k]));
    } else {
      dl = l[k];
    }
    add_axis(A.v, k, A.im, dl);
    add_axis(B.v, k, -B.im, dl);
    const f3 xa = cross_axis(ra, k), xb = cross_axis(rb, k);
    if (kGen) {
      A.w = madd(A.w, inv_inertia(A.ii, mk(axA.x, axA.y, axA.z), axA.w, xa), dl);
      B.w = msub(B.w, inv_inertia(B.ii, mk(axB.x, axB.y, axB.z), axB.w, xb), dl);
    } else {
      const float sa = A.ii * dl, sb = B.ii * dl;
      // only the two nonzero components of r x e_k
      if (k == 0) {
        A.w.y = fmaf(sa, xa.y, A.w.y);
        A.w.z = fmaf(sa, xa.z, A.w.z);
        B.w.y = fmaf(-sb, xb.y, B.w.y);
        B.w.z = fmaf(-sb, xb.z, B.w.z);
      } else if (k == 1) {
        A.w.x = fmaf(sa, xa.x, A.w.x);
        A.w.z = fmaf(sa, xa.z, A.w.z);
        B.w.x = fmaf(-sb, xb.x, B.w.x);
        B.w.z = fmaf(-sb, xb.z, B.w.z);
      } else {
        A.w.x = fmaf(sa, xa.x, A.w.x);
        A.w.y = fmaf(sa, xa.y, A.w.y);
        B.w.x = fmaf(-sb, xb.x, B.w.x);
        B.w.y = fmaf(-sb, xb.y, B.w.y);
      }
    }
  }
}

// Contact touching a capsule: rows d = n, t1, t2 with full lever arms,
//   J_d v = d.(v_b - v_a) + w_b.(r_b x d) - w_a.(r_a x d),
// and the impulse dl moves v_a by -dl/m_a d, w_a by -dl I_a^-1 (r_a x d), and
// body b the opposite way.  axA, axB: (capsule axis, 1/I_axis - 1/I_perp).
template <bool solve>
__device__ __forceinline__ void gen_contact_rows(const Rec& R, Bod& A, Bod& B, float cfm, float4& lam, float& rl,
                                                 float4 axA, float4 axB) {
  const f3 n = mk(R.r0.x, R.r0.y, R.r0.z);
  f3 t1, t2;
  tangents_from(n, R.r0.w, t1, t2);
  const f3 ra = mk(R.g0.x, R.g0.y, R.g0.z), rb = mk(R.g1.x, R.g1.y, R.g1.z);
  const f3 ua = mk(axA.x, axA.y, axA.z), ub = mk(axB.x, axB.y, axB.z);
  const float bias = R.r1.z, mu = R.r1.w;
  float* l = &lam.x;
  const float invd[3] = {R.r2.x, R.r2.y, R.r2.z};
  const float Arr[3] = {R.r1.x, R.g0.w, R.g1.w};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const f3 d = k == 0 ? n : (k == 1 ? t1 : t2);
    const f3 ca = cross(ra, d), cb = cross(rb, d);
    float dl;
    if (solve) {
      const float vr = dot(d, sub(B.v, A.v)) + dot(cb, B.w) - dot(ca, A.w);
      const float wv = fmaf(cfm, l[k], vr + (k == 0 ? bias : 0.0f));
      const float hi = k == 0 ? INFINITY : mu * l[0];
      const float lo = k == 0 ? 0.0f : -hi;
      const float nl = fminf(fmaxf(fmaf(-wv, invd[k], l[k]), lo), hi);
      dl = nl - l[k];
      l[k] = nl;
      rl = fmaxf(rl, fabsf(dl) * Arr[k]);
    } else {
      dl = l[k];
    }
    A.v = msub(A.v, d, A.im * dl);
    B.v = madd(B.v, d, B.im * dl);
    A.w = msub(A.w, inv_inertia(A.ii, ua, axA.w, ca), dl);
    B.w = madd(B.w, inv_inertia(B.ii, ub, axB.w, cb), dl);
  }
}

// A static second body in the sweeps of partitions held in global memory: a
// zero velocity and zero inverse mass and inertia, never written.
__device__ float4 g_zero_body[2];

// One copy: gather its bodies, solve (or, with solve false, apply) its rows,
// scatter the velocities, store the impulses at lam_out.  kSweep: the second
// body is always loaded, a static one as a zero body: at index -1 of V when
// the velocities are in LDS (kLds), from g_zero_body otherwise, so that the
// arithmetic is the same in both and no lane branches on it before the store.
// A zero body stays zero in LDS because a zero inverse mass adds only zeros.
// kCompact: every copy is a sphere contact and its record has no row masses;
// they are formed from the replicas' inverse masses exactly as the row
// assembly forms them (the same operations in the same order), so the bits
// are those of the stored record.
template <bool solve, bool kCaps = false, bool kSweep = false, bool kLds = false, bool kCompact = false>
__device__ __forceinline__ float4 do_slot(const WP& w, Vel V, Rec& R, float& rl, int r0 = 0) {
  Bod A = ld_body(V, R.ia);
  Bod B;
  const bool hasB = R.ib >= 0;
  if (kSweep && kLds) {
    B = ld_body(V, R.ib);
  } else if (kSweep) {
    const float4* zl = hasB ? V.p + R.ib : g_zero_body;
    const float4* za = hasB ? V.p + R.ib + V.stride : g_zero_body + 1;
    const float4 a = *zl, b = *za;
    B = {mk(a.x, a.y, a.z), mk(b.x, b.y, b.z), a.w, b.w};
  } else if (hasB) {
    B = ld_body(V, R.ib);
  } else {
    B = {mk(0, 0, 0), mk(0, 0, 0), 0.0f, 0.0f};
  }
  // The record's registers are only read (the new impulses go to L): a record
  // loaded one colour ahead then stays in the registers it was loaded into.
  float4 L = R.lam;
  if (kCompact) {
    contact_rows<solve, true>(R, A, B, w.cfm, L, rl, float4{});
  } else if (kCaps && R.gen) {
    const float4 axA = w.rep_ax[r0 + R.ia];
    const float4 axB = hasB ? w.rep_ax[r0 + R.ib] : float4{};
    if (R.joint)
      joint_rows<solve, true>(R, A, B, w.cfm, L, rl, axA, axB);
    else
      gen_contact_rows<solve>(R, A, B, w.cfm, L, rl, axA, axB);
  } else if (R.joint) {
    joint_rows<solve>(R, A, B, w.cfm, L, rl);
  } else {
    contact_rows<solve>(R, A, B, w.cfm, L, rl, R.r2);
  }
  st_body(V, R.ia, A);
  if ((kSweep && kLds) || hasB) st_body(V, R.ib, B);
  return L;
}

// a sweep never changes the fourth component of an impulse (the packed ids):
// only x, y, z are stored
__device__ __forceinline__ void store_lam(char* p, float4 L) {
  *reinterpret_cast<float3*>(p) = make_float3(L.x, L.y, L.z);
}

// s_waitcnt operand (gfx9 encoding) that waits for every vector-memory access
// of the wave to complete and leaves the other counters free.
constexpr int kWaitVmem0 = 0x0F70;

// Workgroup barrier after which other waves read replica velocities this wave
// wrote.  In LDS the barrier's wait for the wave's LDS operations orders them.
// In global memory (partitions above the LDS tile) the workgroup barrier does
// not wait for the wave's stores, so the wave waits for them first.
template <bool kLds>
__device__ __forceinline__ void vel_sync() {
  if (!kLds) __builtin_amdgcn_s_waitcnt(kWaitVmem0);
  __syncthreads();
}

// replica velocities with gravity applied (v~ = v + h g), plus the interface
// coupling impulse when that option is on, and inverse masses (the replica's
// share of them under mass splitting, kSplit)
template <int BS, bool kSplit>
__device__ void load_replicas(const WP& w, Vel V, int r0, int nr) {
  const int N = w.N;
  const float hgx = w.dt * w.gx, hgy = w.dt * w.gy, hgz = w.dt * w.gz;
  for (int r = threadIdx.x; r < nr; r += BS) {
    const int b = w.rep_body_pm[r0 + r];
    float2 im;
    if constexpr (kSplit)
      im = w.rep_im[r0 + r];
    else
      im = make_float2(w.b_invm[b], w.b_invI[b]);
    float4 lin = make_float4(w.st[7 * N + b] + hgx, w.st[8 * N + b] + hgy, w.st[9 * N + b] + hgz, im.x);
    float4 ang = make_float4(w.st[10 * N + b], w.st[11 * N + b], w.st[12 * N + b], im.y);
    if (w.couple) {
      const float4 cv = w.rep_cpl[r0 + r], cw = w.rep_cpl[w.Rcap + r0 + r];
      lin.x += cv.x;
      lin.y += cv.y;
      lin.z += cv.z;
      ang.x += cw.x;
      ang.y += cw.y;
      ang.z += cw.z;
    }
    V.p[r] = lin;
    V.p[r + V.stride] = ang;
  }
}

// natural-map residual of one copy's three rows at the given velocities
__device__ float copy_residual(const Rec& R, const Bod& A, const Bod& B, float cfm) {
  float vr[3], bias[3], lo[3], hi[3];
  const float* l = &R.lam.x;
  if (R.joint) {
    const f3 ra = mk(R.r0.x, R.r0.y, R.r0.z), rb = mk(R.r1.x, R.r1.y, R.r1.z);
    const f3 d = sub(add(A.v, cross(A.w, ra)), add(B.v, cross(B.w, rb)));
    vr[0] = d.x;
    vr[1] = d.y;
    vr[2] = d.z;
    bias[0] = R.r0.w;
    bias[1] = R.r1.w;
    bias[2] = R.r2.w;
    for (int k = 0; k < 3; ++k) {
      lo[k] = -INFINITY;
      hi[k] = INFINITY;
    }
  } else {
    const f3 n = mk(R.r0.x, R.r0.y, R.r0.z);
    f3 t1, t2;
    tangents_from(n, R.r0.w, t1, t2);
    const f3 dv = sub(B.v, A.v);
    if (R.gen) {
      const f3 ra = mk(R.g0.x, R.g0.y, R.g0.z), rb = mk(R.g1.x, R.g1.y, R.g1.z);
      vr[0] = dot(n, dv) + dot(cross(rb, n), B.w) - dot(cross(ra, n), A.w);
      vr[1] = dot(t1, dv) + dot(cross(rb, t1), B.w) - dot(cross(ra, t1), A.w);
      vr[2] = dot(t2, dv) + dot(cross(rb, t2), B.w) - dot(cross(ra, t2), A.w);
    } else {
      const f3 sw = madd(scale(B.w, R.r1.y), A.w, R.r1.x);
      vr[0] = dot(n, dv);
      vr[1] = dot(t1, dv) - dot(t2, sw);
      vr[2] = dot(t2, dv) + dot(t1, sw);
    }
    bias[0] = R.r1.z;
    bias[1] = bias[2] = 0.0f;
    lo[0] = 0.0f;
    hi[0] = INFINITY;
    hi[1] = hi[2] = R.r1.w * l[0];
    lo[1] = lo[2] = -hi[1];
  }
  // sphere contacts keep one 1/A for both tangents (the record's z, w hold A_n, A_t)
  const float invd[3] = {R.r2.x, R.r2.y, (R.joint || R.gen) ? R.r2.z : R.r2.y};
  float e = 0.0f;
  for (int k = 0; k < 3; ++k) {
    const float wv = fmaf(cfm, l[k], vr[k] + bias[k]);
    const float pr = fminf(fmaxf(fmaf(-wv, invd[k], l[k]), lo[k]), hi[k]);
    e = fmaxf(e, fabsf(l[k] - pr) / invd[k]);
  }
  return e;
}

// Initial residual of a start (plain, or learned for contacts): apply it in
// solve order, take the largest natural-map residual of the partition's rows,
// then restore v~.  Uniform over the workgroup.
template <int BS, bool kCaps, bool kSplit, bool kLds>
__device__ float start_residual(const WP& w, Vel V, int s0, int ncol, const int* coff, int r0, int nr,
                                bool learned, float* red) {
  const int tid = threadIdx.x;
  const bool packed = nr < kPackReps;
  float unused = 0.0f;
  for (int c = 0; c < ncol; ++c) {
    const int e = s0 + coff[c + 1];
    for (int slot = s0 + coff[c] + tid; slot < e; slot += BS) {
      Rec R;
      load_rec<kCaps>(w, slot, R, packed);
      if (learned && !R.joint) R.lam = w.r_lamL[slot];
      if (R.lam.x != 0.0f || R.lam.y != 0.0f || R.lam.z != 0.0f) do_slot<false, kCaps>(w, V, R, unused, r0);
    }
    vel_sync<kLds>();
  }
  float e = 0.0f;
  for (int slot = s0 + tid; slot < s0 + coff[ncol]; slot += BS) {
    Rec R;
    load_rec<kCaps>(w, slot, R, packed);
    if (learned && !R.joint) R.lam = w.r_lamL[slot];
    const Bod A = ld_body(V, R.ia);
    Bod B = {mk(0, 0, 0), mk(0, 0, 0), 0.0f, 0.0f};
    if (R.ib >= 0) B = ld_body(V, R.ib);
    e = fmaxf(e, copy_residual(R, A, B, w.cfm));
  }
  e = block_max<BS>(e, red);
  load_replicas<BS, kSplit>(w, V, r0, nr);
  vel_sync<kLds>();
  return e;
}

// One colour of a sweep, solved by the workgroup: each thread solves the
// colour's slot at its own index (its record `cur`, loaded one colour ahead)
// and, in colours larger than the workgroup, the slots BS, 2 BS, ... further
// on; meanwhile the first slot of the next colour (local range [n0, n1), never
// empty) is loaded into `nxt`.  Every lane issues that load (lanes past the
// colour's end read slots after it, which they never use), so each wave issues
// the same loads in every pass and the wait for `cur` can leave the new loads
// in flight.  All record addresses are a scalar base plus the lane's offset
// toff = 16 tid.  Ends with the workgroup barrier between colours.
template <int BS, bool kCaps, bool kLds, bool kCompact>
__device__ __forceinline__ void colour_pass(const WP& w, Vel V, const Slots& S, int b0, int b1, int n0, int n1,
                                            bool prefetch, Rec& cur, bool& has_cur, Rec& nxt, bool& has_nxt,
                                            int first, float& rl, int r0, bool packed, uint32_t toff,
                                            int* over = nullptr, float tol = 0.0f) {
  const int tid = threadIdx.x;
  has_nxt = prefetch && n0 + tid < n1;
  fetch_lane<kCaps, kCompact>(S, n0, toff, nxt, packed);
  // the thread's second slot of a colour larger than the workgroup: loaded once
  // the first one is decoded, so that its loads run during the first one's rows
  const int k2 = b0 + first;
  const bool has2 = tid < b1 - k2;
  // Wait here for `cur` (loaded one colour ahead, before the loads just issued
  // for `nxt`), ahead of the second slot's loads: a wait placed after those
  // would also hold back the prefetch.  (With separate record ids, 4, 5 or 7
  // loads per record, this waits for one prefetch load too.)
  constexpr int kFetchLoads = kCaps ? 6 : (kCompact ? 3 : 4);
  __builtin_amdgcn_s_waitcnt(kWaitVmem0 | kFetchLoads);
  decode<kCaps>(cur, packed);
  Rec R2;
  if (has2) fetch_lane<kCaps, kCompact>(S, k2, toff, R2, packed);
  // both slots' impulses are stored after both are solved, so that the wait for
  // the second slot's loads does not also wait for the first slot's store
  float4 Lc, L2;
  if (has_cur) Lc = do_slot<true, kCaps, true, kLds, kCompact>(w, V, cur, rl, r0);
  if (has2) {
    decode<kCaps>(R2, packed);
    L2 = do_slot<true, kCaps, true, kLds, kCompact>(w, V, R2, rl, r0);
  }
  if (has_cur) store_lam(S.lam + (((uint32_t)b0 << 4) + toff), Lc);
  if (has2) store_lam(S.lam + (((uint32_t)k2 << 4) + toff), L2);
  for (int k = k2 + BS; k < b1; k += BS) {
    if (tid < b1 - k) {
      Rec R;
      fetch_lane<kCaps, kCompact>(S, k, toff, R, packed);
      decode<kCaps>(R, packed);
      store_lam(S.lam + (((uint32_t)k << 4) + toff), do_slot<true, kCaps, true, kLds, kCompact>(w, V, R, rl, r0));
    }
  }
  // the last colour of an adaptive sweep: a wave with a residual above the
  // tolerance marks the sweep (read after the barrier)
  if (over != nullptr && __ballot(rl > tol) != 0 && lane_id() == 0) *over = 1;
  vel_sync<kLds>();
}

// Solve one partition with a workgroup of BS threads.  V holds its replica
// velocities (LDS, or its slice of rep_v4 for the global variant).
template <int BS, bool kCaps, bool kSplit, bool kLds>
__device__ void solve_partition(const WP& w, int p, Vel V, int* coff, float* red, int* over) {
  const int tid = threadIdx.x;
  const int N = w.N;
  const int r0 = w.part_rep_off[p];
  const int nr = w.part_rep_off[p + 1] - r0;
  const int s0 = w.part_copy_off[p];
  const int ncol = w.part_ncol[p];
  const bool packed = nr < kPackReps;  // uniform: ids from the impulses' fourth component
  if (tid < kColStride) coff[tid] = w.part_col_off[p * kColStride + tid];
  if (tid < 3) over[tid] = 0;
  if (kLds && tid == 0) {
    // the zero body at index -1 (a static second body in the sweeps)
    V.p[-1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    V.p[V.stride - 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  load_replicas<BS, kSplit>(w, V, r0, nr);
  vel_sync<kLds>();
  float rl = 0.0f;
  if (w.learned) {
    // keep the learned start only when its initial residual is below the plain start's
    const float rho_p = start_residual<BS, kCaps, kSplit, kLds>(w, V, s0, ncol, coff, r0, nr, false, red);
    const float rho_l = start_residual<BS, kCaps, kSplit, kLds>(w, V, s0, ncol, coff, r0, nr, true, red);
    bool use = rho_l < rho_p;
    if (w.force_guard && w.part_force_guard[p] >= 0) use = w.part_force_guard[p] != 0;
    if (use)
      for (int slot = s0 + tid; slot < s0 + coff[ncol]; slot += BS)
        if (!(w.r_ids[slot].x & kJointFlag)) {
          const float4 L = w.r_lamL[slot];
          w.r_lam[slot] = make_float4(L.x, L.y, L.z, w.r_lam[slot].w);
        }
    if (tid == 0) {
      w.part_guard[p] = use ? 1 : 0;
      w.part_rho0[2 * p] = rho_p;
      w.part_rho0[2 * p + 1] = rho_l;
    }
    // the learned starts just stored are read below by other threads
    __builtin_amdgcn_s_waitcnt(kWaitVmem0);
    __syncthreads();
  }
  // warm-start impulses enter in solve order
  for (int c = 0; c < ncol; ++c) {
    const int e = s0 + coff[c + 1];
    for (int slot = s0 + coff[c] + tid; slot < e; slot += BS) {
      Rec R;
      load_rec<kCaps>(w, slot, R, packed);
      if (R.lam.x != 0.0f || R.lam.y != 0.0f || R.lam.z != 0.0f) do_slot<false, kCaps>(w, V, R, rl, r0);
    }
    vel_sync<kLds>();
  }
  // sweeps; the first slot of the next colour is loaded while the current colour is solved
  const int cap = w.forced ? w.part_force_iters[p] : w.max_iters;
  int it = 0;
  float rho = 0.0f;
  // A world of spheres alone (no joints, no capsules) sweeps with three loads
  // per record instead of four: the row masses are formed from the replicas.
  auto sweeps = [&](auto compact) {
    constexpr bool kCompact = decltype(compact)::value;
    // With a single colour the next record would be the current one, read before
    // its impulses are stored: then nothing is prefetched and every slot is
    // loaded where it is solved.
    const int first = ncol == 1 ? 0 : BS;
    // colour offsets: lane k of cv0 holds coff[k], cv1 the last one; read with readlane
    const int cv0 = coff[lane_id()];
    const int cv1 = __builtin_amdgcn_readfirstlane(coff[kColStride - 1]);
    auto co = [&](int k) { return k < 64 ? __builtin_amdgcn_readlane(cv0, k) : cv1; };
    const Slots S = slots_of(w, s0);
    // two record sets used in turn: one is solved while the next colour's first
    // slot is loaded into the other, so no record is ever copied between them
    Rec ra, rb;
    bool ha = ncol > 1 && co(0) + tid < co(1), hb = false;
    const uint32_t toff = (uint32_t)tid << 4;
    if (ncol > 0) fetch_lane<kCaps, kCompact>(S, co(0), toff, ra, packed);
    // Nothing may still be in flight into the first set when the loop is entered:
    // otherwise the wait placed before its first use would also hold back the
    // next colour's prefetch in every pass.
    __builtin_amdgcn_s_waitcnt(0);
    if (ncol == 0) {
      // no rows: every sweep is empty (a zero residual stops adaptive sweeps after one)
      it = (!w.forced && w.adaptive) ? min(cap, 1) : max(cap, 0);
    } else if (cap > 0) {
      int c = 0;
      rl = 0.0f;
      // Adaptive sweeps stop once no slot's residual exceeds the tolerance: the
      // last colour of sweep s marks over[s mod 3] if one does (three flags in
      // turn, so that clearing the flag of sweep s + 2 after sweep s never races
      // with a read or a mark).  The residual itself is reduced once, at the end.
      const bool check = !w.forced && w.adaptive;
      int k3 = 0;
      // after colour c: the end of a sweep may stop
      auto next_colour = [&]() {
        if (++c < ncol) return false;
        c = 0;
        ++it;
        bool stop = it >= cap;
        if (check) {
          stop = stop || over[k3] == 0;
          if (tid == 0) over[k3 == 0 ? 2 : k3 - 1] = 0;
          k3 = k3 == 2 ? 0 : k3 + 1;
        }
        if (stop) rho = block_max<BS>(rl, red);
        rl = 0.0f;
        return stop;
      };
      // [b0, b1): the current colour's slots, carried from the previous pass, so
      // that a pass reads one new offset
      const int co0 = co(0);
      int b0 = co0, b1 = co(1);
      for (;;) {
        {
          const int cn = c + 1 < ncol ? c + 1 : 0;
          const int n0 = cn == 0 ? co0 : b1, n1 = co(cn + 1);
          colour_pass<BS, kCaps, kLds, kCompact>(w, V, S, b0, b1, n0, n1, ncol > 1, ra, ha, rb, hb, first, rl, r0,
                                                 packed, toff, check && c == ncol - 1 ? over + k3 : nullptr, w.tol);
          b0 = n0;
          b1 = n1;
        }
        if (next_colour()) break;
        {
          const int cn = c + 1 < ncol ? c + 1 : 0;
          const int n0 = cn == 0 ? co0 : b1, n1 = co(cn + 1);
          colour_pass<BS, kCaps, kLds, kCompact>(w, V, S, b0, b1, n0, n1, ncol > 1, rb, hb, ra, ha, first, rl, r0,
                                                 packed, toff, check && c == ncol - 1 ? over + k3 : nullptr, w.tol);
          b0 = n0;
          b1 = n1;
        }
        if (next_colour()) break;
      }
    }
  };
  if (!kCaps && w.J == 0)
    sweeps(std::true_type{});
  else
    sweeps(std::false_type{});
  // integrate and write the replica states
  const float h = w.dt;
  bool bad = false;
  for (int r = tid; r < nr; r += BS) {
    const int b = w.rep_body_pm[r0 + r];
    const Bod B = ld_body(V, r);
    const float x = fmaf(h, B.v.x, w.st[b]);
    const float y = fmaf(h, B.v.y, w.st[N + b]);
    const float z = fmaf(h, B.v.z, w.st[2 * N + b]);
    float qw = w.st[3 * N + b], qx = w.st[4 * N + b], qy = w.st[5 * N + b], qz = w.st[6 * N + b];
    const float wx = B.w.x, wy = B.w.y, wz = B.w.z;
    const float dw = -fmaf(wz, qz, fmaf(wy, qy, wx * qx));
    const float dx = fmaf(wx, qw, fmaf(wy, qz, -(wz * qy)));
    const float dy = fmaf(wy, qw, fmaf(wz, qx, -(wx * qz)));
    const float dz = fmaf(wz, qw, fmaf(wx, qy, -(wy * qx)));
    const float hh = 0.5f * h;
    qw = fmaf(hh, dw, qw);
    qx = fmaf(hh, dx, qx);
    qy = fmaf(hh, dy, qy);
    qz = fmaf(hh, dz, qz);
    const float nn = 1.0f / sqrtf(fmaf(qz, qz, fmaf(qy, qy, fmaf(qx, qx, qw * qw))));
    const float out[13] = {x, y, z, qw * nn, qx * nn, qy * nn, qz * nn, B.v.x, B.v.y, B.v.z, B.w.x, B.w.y, B.w.z};
#pragma unroll
    for (int k = 0; k < 13; ++k) {
      bad |= !isfinite(out[k]);
      w.rst[(int64_t)k * w.Rcap + r0 + r] = out[k];
    }
  }
  if (__syncthreads_or(bad) && tid == 0) atomicOr(&w.scal[SC_FLAGS], F_NONFINITE);
  if (tid == 0) {
    w.part_iters[p] = it;
    w.part_resid[p] = rho;
  }
  __syncthreads();  // coff and red are reused by the workgroup's next partition
}

// Projected Gauss-Seidel over the partitions, largest first (part_order).
// kLds: velocities in LDS, for the partitions with at most kReps replicas;
// otherwise velocities in global memory, for the larger ones.  Either one
// workgroup per partition, or (w.pgs_persistent) a grid of resident
// workgroups that take partitions from an atomic queue until it is empty.
template <int BS, int kReps, bool kLds, bool kCaps, bool kSplit>
__global__ __launch_bounds__(BS) void k_pgs(WP w) {
  extern __shared__ float4 sm4[];
  __shared__ int coff[kColStride];
  __shared__ float red[BS / 64];
  __shared__ int over[3];
  __shared__ int failed_s, item_s;
  const int tid = threadIdx.x;
  // one read of the failure flag per workgroup, so the early exit is uniform
  if (tid == 0) failed_s = step_failed(w) ? 1 : 0;
  __syncthreads();
  if (failed_s) {
    for (int p = blockIdx.x * BS + tid; p < w.G; p += gridDim.x * BS) {
      w.part_iters[p] = 0;
      w.part_resid[p] = 0.0f;
    }
    return;
  }
  int32_t* queue = w.pgs_queue + (kLds ? 0 : 1);
  for (int k = blockIdx.x;;) {
    if (w.pgs_persistent) {
      if (tid == 0) item_s = atomicAdd(queue, 1);
      __syncthreads();
      k = item_s;
      __syncthreads();
    }
    if (k >= w.G) break;
    const int p = w.part_order[k];
    const int nr = w.part_rep_off[p + 1] - w.part_rep_off[p];
    if (kLds == (nr <= kReps)) {  // otherwise the other variant handles this partition
      // LDS: [0][v, 1/m of kReps replicas][0][w, 1/I of kReps replicas], indexed from the
      // first replica, so index -1 of either array is a zero entry
      const Vel V = kLds ? Vel{sm4 + 1, kReps + 1} : Vel{w.rep_v4 + w.part_rep_off[p], w.Rcap};
      solve_partition<BS, kCaps, kSplit, kLds>(w, p, V, coff, red, over);
    }
    if (!w.pgs_persistent) break;
  }
}

// Partitions in descending order of constraint copies (ties: ascending id),
// by counting ranks: every workgroup reads all keys into LDS and ranks its
// slice of the partitions.  More than kOrderMax partitions keep their
// natural order.
constexpr int kOrderBS = 256;
constexpr int kOrderMax = 8192;

__global__ __launch_bounds__(kOrderBS) void k_part_order(WP w) {
  __shared__ int key[kOrderMax];
  const int G = w.G;
  const int p = blockIdx.x * kOrderBS + threadIdx.x;
  if (G > kOrderMax) {
    if (p < G) w.part_order[p] = p;
    return;
  }
  for (int q = threadIdx.x; q < G; q += kOrderBS) key[q] = w.part_copy_off[q + 1] - w.part_copy_off[q];
  __syncthreads();
  if (p < G) {
    const int kp = key[p];
    int rank = 0;
    for (int q = 0; q < G; ++q) {
      const int kq = key[q];
      rank += (kq > kp || (kq == kp && q < p)) ? 1 : 0;
    }
    w.part_order[rank] = p;
  }
}

// Inverse mass and inverse inertia of every replica, partition-major, for the
// sweeps.  With mass splitting a replica of an overlap body carries the share
// w of the body that the blend will give it: both are divided by w (a replica
// of weight 0 keeps the whole body), and the factor 1/w is kept for the rows.
__global__ void k_rep_mass(WP w) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N || step_failed(w)) return;
  const int n = __popcll(w.mask[v]);
  const int bm0 = w.rep_off_bm[v];
  const float im = w.b_invm[v], ii = w.b_invI[v];
  const float sum = w.msplit && n > 1 ? inv_dist_sum(w, bm0, n) : 0.0f;
  for (int k = 0; k < n; ++k) {
    float s = 1.0f;
    if (w.msplit && n > 1) {
      const float wt = blend_weight(w, w.rep_D_bm[bm0 + k], sum, n);
      s = wt > 0.0f ? 1.0f / wt : 1.0f;
    }
    const int r = w.rep_pm_of_bm[bm0 + k];
    if (w.msplit) w.rep_isc[r] = s;
    w.rep_im[r] = make_float2(im * s, ii * s);
  }
}

// capsule axis and inertia difference of every replica (read by capsule rows)
__global__ void k_rep_axis(WP w) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= w.Rcap || w.G <= 0 || r >= w.part_rep_off[w.G] || step_failed(w)) return;
  const int b = w.rep_body_pm[r];
  float4 ax = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (w.b_half[b] > 0.0f) {
    const f3 u = body_axis(w, b);
    ax = make_float4(u.x, u.y, u.z, w.b_dI[b] * (w.msplit ? w.rep_isc[r] : 1.0f));
  }
  w.rep_ax[r] = ax;
}

// ------------------------------------------------------- blend + cache ----

__global__ void k_blend(WP w) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N || step_failed(w)) return;
  const int N = w.N;
  const int64_t RC = w.Rcap;
  const uint64_t m = w.mask[v];
  const int n = __popcll(m);
  const int bm0 = w.rep_off_bm[v];
  if (n == 1) {
    const int r = w.rep_pm_of_bm[bm0];
#pragma unroll
    for (int k = 0; k < 13; ++k) w.st[k * N + v] = w.rst[k * RC + r];
    w.rep_w_bm[bm0] = 1.0f;
    return;
  }
  const float sum = inv_dist_sum(w, bm0, n);
  float acc[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) acc[k] = 0.0f;
  float q0[4];
  for (int k = 0; k < n; ++k) {
    const float wt = blend_weight(w, w.rep_D_bm[bm0 + k], sum, n);
    w.rep_w_bm[bm0 + k] = wt;
    const int r = w.rep_pm_of_bm[bm0 + k];
    float s[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) s[c] = w.rst[c * RC + r];
    if (k == 0) {
      q0[0] = s[3];
      q0[1] = s[4];
      q0[2] = s[5];
      q0[3] = s[6];
    } else if (s[3] * q0[0] + s[4] * q0[1] + s[5] * q0[2] + s[6] * q0[3] < 0.0f) {
      s[3] = -s[3];
      s[4] = -s[4];
      s[5] = -s[5];
      s[6] = -s[6];
    }
#pragma unroll
    for (int c = 0; c < 13; ++c) acc[c] += wt * s[c];
  }
  const float nn = 1.0f / sqrtf(acc[3] * acc[3] + acc[4] * acc[4] + acc[5] * acc[5] + acc[6] * acc[6]);
  acc[3] *= nn;
  acc[4] *= nn;
  acc[5] *= nn;
  acc[6] *= nn;
#pragma unroll
  for (int k = 0; k < 13; ++k) w.st[k * N + v] = acc[k];
}

__global__ void k_cache(WP w) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int M = w.part_copy_off[w.G];
  if (u >= M || u >= w.Mcap || step_failed(w)) return;
  const int64_t MC = w.Mcap;
  const int slot = w.cp_slot[u];
  const int src = w.cp_src[u];
  const float4 l = w.r_lam[slot];
  w.wc_part[u] = w.cp_part[u];
  if (src < w.J) {
    w.wc_kind[u] = 0;
    w.wc_key[u] = (uint64_t)src;
    w.wc_k64[u] = (uint64_t)src;
    w.wc_val[u] = l.x;
    w.wc_val[MC + u] = l.y;
    w.wc_val[2 * MC + u] = l.z;
    w.wc_val[3 * MC + u] = 0.0f;
  } else {
    const int c = src - w.J;
    w.wc_kind[u] = 1;
    w.wc_key[u] = ((uint64_t)w.c_a[c] << 32) | w.c_bkey[c];
    w.wc_k64[u] = (1ull << 63) | w.wc_key[u];
    const float4 r0 = w.r_rec[slot];
    f3 t1, t2;
    tangents_from(mk(r0.x, r0.y, r0.z), r0.w, t1, t2);
    const f3 fw = add(scale(t1, l.y), scale(t2, l.z));
    w.wc_val[u] = l.x;
    w.wc_val[MC + u] = fw.x;
    w.wc_val[2 * MC + u] = fw.y;
    w.wc_val[3 * MC + u] = fw.z;
  }
}

// Commit of a step (one workgroup): the warm-start cache becomes this step's,
// and the per-partition sweep counts are summed into the counters.
constexpr int kCommitBS = 1024;

__global__ __launch_bounds__(kCommitBS) void k_commit(WP w) {
  __shared__ int failed_s;
  __shared__ long long part[5][kCommitBS / 64];
  if (threadIdx.x == 0) failed_s = w.scal[SC_FLAGS] != 0;
  __syncthreads();
  if (failed_s) return;
  // the cache written by k_cache is indexed by this step's partition ranges
  for (int g = threadIdx.x; g <= w.G; g += kCommitBS) w.wc_off[g] = w.part_copy_off[g];
  int mx = 0;
  long long unconv = 0, bytes = 0, sweeps = 0, ops = 0;
  for (int g = threadIdx.x; g < w.G; g += kCommitBS) {
    const int it = w.part_iters[g];
    mx = max(mx, it);
    if (w.adaptive && !w.forced && it >= w.max_iters && w.part_resid[g] > w.tol) ++unconv;
    const int64_t nj = w.mc_psize[1][g], nc = w.mc_psize[2][g], ns = w.part_nstatic[g];
    bytes += (int64_t)it * ((nc - ns) * kBytesDynDyn + ns * kBytesStatic + nj * kBytesJoint);
    ops += (int64_t)it * ((nc - ns) * kOpsDynDyn + ns * kOpsStatic + nj * kOpsJoint);
    sweeps += it;
  }
  long long v[5] = {mx, unconv, bytes, sweeps, ops};
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const long long o = __shfl_xor(v[k], d, 64);
      v[k] = k == 0 ? max(v[k], o) : v[k] + o;
    }
  if (lane_id() == 0)
    for (int k = 0; k < 5; ++k) part[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < kCommitBS / 64; ++i) {
      t[0] = max(t[0], part[0][i]);
      for (int k = 1; k < 5; ++k) t[k] += part[k][i];
    }
    w.scal[SC_PREV_NCOPY] = w.part_copy_off[w.G];
    w.scal[SC_COMMITTED] += 1;
    w.stat_i64[0] += t[0];
    w.stat_i64[1] += t[1];
    w.stat_i64[2] += t[2];
    w.stat_i64[3] += t[3];
    w.stat_i64[4] += 1;
    w.stat_i64[5] += t[1] > 0 ? 1 : 0;
    w.stat_i64[6] += t[4];
  }
}

// natural-map residual of the final iterate, one workgroup per partition: for
// every row, A_rr |lambda - clamp(lambda - w/A_rr, lo, hi)| with w the row's
// constraint velocity at the final velocities
__global__ __launch_bounds__(256) void k_exact_resid(WP w) {
  __shared__ float red[4];
  __shared__ int failed_s;
  const int p = blockIdx.x;
  if (threadIdx.x == 0) failed_s = step_failed(w) ? 1 : 0;
  __syncthreads();
  if (failed_s) return;
  const int r0 = w.part_rep_off[p];
  const int s0 = w.part_copy_off[p], s1 = w.part_copy_off[p + 1];
  const int64_t RC = w.Rcap;
  float e = 0.0f, esum = 0.0f;
  for (int slot = s0 + threadIdx.x; slot < s1; slot += 256) {
    Rec R;
    if (w.has_caps)
      load_rec<true>(w, slot, R);
    else
      load_rec<false>(w, slot, R);
    Bod A, B;
    const int ra_ = r0 + R.ia;
    A.v = mk(w.rst[7 * RC + ra_], w.rst[8 * RC + ra_], w.rst[9 * RC + ra_]);
    A.w = mk(w.rst[10 * RC + ra_], w.rst[11 * RC + ra_], w.rst[12 * RC + ra_]);
    B.v = mk(0, 0, 0);
    B.w = mk(0, 0, 0);
    if (R.ib >= 0) {
      const int rb_ = r0 + R.ib;
      B.v = mk(w.rst[7 * RC + rb_], w.rst[8 * RC + rb_], w.rst[9 * RC + rb_]);
      B.w = mk(w.rst[10 * RC + rb_], w.rst[11 * RC + rb_], w.rst[12 * RC + rb_]);
    }
    float vr[3], invd[3], bias[3], lo[3], hi[3];
    const float* l = &R.lam.x;
    if (R.joint) {
      const f3 ra = mk(R.r0.x, R.r0.y, R.r0.z), rb = mk(R.r1.x, R.r1.y, R.r1.z);
      const f3 d = sub(add(A.v, cross(A.w, ra)), add(B.v, cross(B.w, rb)));
      vr[0] = d.x;
      vr[1] = d.y;
      vr[2] = d.z;
      bias[0] = R.r0.w;
      bias[1] = R.r1.w;
      bias[2] = R.r2.w;
      for (int k = 0; k < 3; ++k) {
        lo[k] = -INFINITY;
        hi[k] = INFINITY;
      }
    } else {
      const f3 n = mk(R.r0.x, R.r0.y, R.r0.z);
      f3 t1, t2;
      tangents_from(n, R.r0.w, t1, t2);
      const f3 dv = sub(B.v, A.v);
      if (R.gen) {
        const f3 ra = mk(R.g0.x, R.g0.y, R.g0.z), rb = mk(R.g1.x, R.g1.y, R.g1.z);
        vr[0] = dot(n, dv) + dot(cross(rb, n), B.w) - dot(cross(ra, n), A.w);
        vr[1] = dot(t1, dv) + dot(cross(rb, t1), B.w) - dot(cross(ra, t1), A.w);
        vr[2] = dot(t2, dv) + dot(cross(rb, t2), B.w) - dot(cross(ra, t2), A.w);
      } else {
        const f3 sw = add(scale(A.w, R.r1.x), scale(B.w, R.r1.y));
        vr[0] = dot(n, dv);
        vr[1] = dot(t1, dv) - dot(t2, sw);
        vr[2] = dot(t2, dv) + dot(t1, sw);
      }
      bias[0] = R.r1.z;
      bias[1] = bias[2] = 0.0f;
      lo[0] = 0.0f;
      hi[0] = INFINITY;
      hi[1] = hi[2] = R.r1.w * l[0];
      lo[1] = lo[2] = -hi[1];
    }
    invd[0] = R.r2.x;
    invd[1] = R.r2.y;
    invd[2] = (R.joint || R.gen) ? R.r2.z : R.r2.y;
    for (int k = 0; k < 3; ++k) {
      const float wv = vr[k] + bias[k] + w.cfm * l[k];
      const float pr = fminf(fmaxf(l[k] - wv * invd[k], lo[k]), hi[k]);
      e = fmaxf(e, fabsf(l[k] - pr) / invd[k]);
      esum += fabsf(l[k] - pr) / invd[k];
    }
  }
  e = block_max<256>(e, red);
  if (threadIdx.x == 0) atomicMax((int*)&w.stat_f[0], __float_as_int(e));
  // summed residual in a fixed order: waves, then the block
  esum = wave_sum_f(esum);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x >> 6] = esum;
  __syncthreads();
  if (threadIdx.x == 0) w.part_rsum[p] = (red[0] + red[1]) + (red[2] + red[3]);
}

// |C| of every ball joint at the blended state (section 6 reports joint violation)
__global__ void k_joint_viol(WP w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= w.J || step_failed(w)) return;
  const int N = w.N;
  const int a = w.j_ab[2 * j], b = w.j_ab[2 * j + 1];
  const float* an = w.j_anchor + 6 * j;
  float d[3];
  const int bod[2] = {a, b};
  float p[2][3];
  for (int s = 0; s < 2; ++s) {
    const int v = bod[s];
    const float qw = w.st[3 * N + v], qx = w.st[4 * N + v], qy = w.st[5 * N + v], qz = w.st[6 * N + v];
    const float ax = an[3 * s], ay = an[3 * s + 1], az = an[3 * s + 2];
    // R(q) a = a + 2 qw (u x a) + 2 u x (u x a), u = (qx, qy, qz)
    const float cx = qy * az - qz * ay, cy = qz * ax - qx * az, cz = qx * ay - qy * ax;
    const float ex = qy * cz - qz * cy, ey = qz * cx - qx * cz, ez = qx * cy - qy * cx;
    p[s][0] = w.st[0 * N + v] + ax + 2.0f * (qw * cx + ex);
    p[s][1] = w.st[1 * N + v] + ay + 2.0f * (qw * cy + ey);
    p[s][2] = w.st[2 * N + v] + az + 2.0f * (qw * cz + ez);
  }
  for (int k = 0; k < 3; ++k) d[k] = p[0][k] - p[1][k];
  w.joint_viol[j] = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

}  // namespace

namespace {

template <int BS, int R>
hipError_t set_attrs_t() {
  hipError_t e = hipSuccess;
  const int lds = 2 * (R + 1) * (int)sizeof(float4);
  const void* fns[4] = {(const void*)k_pgs<BS, R, true, false, false>, (const void*)k_pgs<BS, R, true, true, false>,
                        (const void*)k_pgs<BS, R, true, false, true>, (const void*)k_pgs<BS, R, true, true, true>};
  for (const void* f : fns)
    if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds))) return e;
  return e;
}

// resident workgroups per compute unit of the variants launch_pgs_t runs
template <int BS, int R, bool kCaps, bool kSplit>
hipError_t occupancy_v(int* per_cu_lds, int* per_cu_glob) {
  const size_t lds = 2 * ((size_t)R + 1) * sizeof(float4);
  hipError_t e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu_lds, k_pgs<BS, R, true, kCaps, kSplit>, BS, lds)))
    return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu_glob, k_pgs<BS, R, false, kCaps, kSplit>, BS, 0);
}

template <int BS, int R>
hipError_t occupancy_t(bool caps, bool split, int* per_cu_lds, int* per_cu_glob) {
  if (caps) return split ? occupancy_v<BS, R, true, true>(per_cu_lds, per_cu_glob)
                         : occupancy_v<BS, R, true, false>(per_cu_lds, per_cu_glob);
  return split ? occupancy_v<BS, R, false, true>(per_cu_lds, per_cu_glob)
               : occupancy_v<BS, R, false, false>(per_cu_lds, per_cu_glob);
}

template <int BS, int R>
hipError_t launch_pgs_t(const WP& w, hipStream_t s) {
  const size_t lds = 2 * ((size_t)R + 1) * sizeof(float4);
  const int g0 = w.pgs_persistent ? std::min(w.G, w.pgs_grid[0]) : w.G;
  const int g1 = w.pgs_persistent ? std::min(w.G, w.pgs_grid[1]) : w.G;
  hipError_t e;
  if (w.pgs_persistent && (e = fill_i32(w.pgs_queue, 0, 2, s))) return e;
  // mass splitting reads the replicas' inverse masses from their own array
  // (a variant of its own, so the default sweeps keep their per-body loads)
  if (w.has_caps && w.msplit) {
    k_pgs<BS, R, true, true, true><<<g0, BS, lds, s>>>(w);
    if ((e = hipGetLastError())) return e;
    k_pgs<BS, R, false, true, true><<<g1, BS, 0, s>>>(w);
  } else if (w.has_caps) {
    k_pgs<BS, R, true, true, false><<<g0, BS, lds, s>>>(w);
    if ((e = hipGetLastError())) return e;
    k_pgs<BS, R, false, true, false><<<g1, BS, 0, s>>>(w);
  } else if (w.msplit) {
    k_pgs<BS, R, true, false, true><<<g0, BS, lds, s>>>(w);
    if ((e = hipGetLastError())) return e;
    k_pgs<BS, R, false, false, true><<<g1, BS, 0, s>>>(w);
  } else {
    k_pgs<BS, R, true, false, false><<<g0, BS, lds, s>>>(w);
    if ((e = hipGetLastError())) return e;
    k_pgs<BS, R, false, false, false><<<g1, BS, 0, s>>>(w);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t pgs_set_attributes() {
  hipError_t e;
  if ((e = set_attrs_t<1024, 4800>())) return e;
  if ((e = set_attrs_t<512, 2400>())) return e;
  if ((e = set_attrs_t<256, 1200>())) return e;
  return set_attrs_t<256, 2400>();
}

hipError_t pgs_occupancy(int cfg, bool caps, bool split, int* per_cu_lds, int* per_cu_glob) {
  switch (cfg) {
    case 0: return occupancy_t<1024, 4800>(caps, split, per_cu_lds, per_cu_glob);
    case 1: return occupancy_t<512, 2400>(caps, split, per_cu_lds, per_cu_glob);
    case 2: return occupancy_t<256, 1200>(caps, split, per_cu_lds, per_cu_glob);
    case 3: return occupancy_t<256, 2400>(caps, split, per_cu_lds, per_cu_glob);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------- slot order in a colour ----
// The copies of one colour share no replica, so any order of their slots gives
// the same sweep.  The order is chosen for the solver's LDS gathers: thread t
// of a colour reads replicas ia and ib of slot t, and 16 consecutive threads
// read without bank conflicts when their ia (and their ib) differ modulo 16
// (a replica's 16 B velocity entry sits in bank group ia mod 16).  Copies are
// grouped by d = (ia - ib) mod 16 (16 for a static second body), and inside a
// group dealt out round-robin over ia mod 16: each round then holds distinct
// ia residues, and, d being fixed, distinct ib residues.  Ranks are taken in
// the previous (uid) order, so the result is deterministic.
constexpr int kSpreadBS = 1024;
constexpr int kSpreadWaves = kSpreadBS / 64;
constexpr int kSpreadKeys = 17 * 16;

__global__ __launch_bounds__(kSpreadBS) void k_slot_spread(WP w) {
  __shared__ int tab[kSpreadWaves][kSpreadKeys];
  __shared__ int run[kSpreadWaves][kSpreadKeys];
  __shared__ int base[kSpreadWaves][18];
  __shared__ int coff[kColStride];
  __shared__ int skip_s;
  const int p = blockIdx.x, tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  if (tid == 0) skip_s = (w.scal[SC_FLAGS] & (F_CONTACT_CAP | F_ADJ_CAP | F_REP_CAP | F_COPY_CAP)) ? 1 : 0;
  __syncthreads();
  if (skip_s) return;
  // Partitions whose velocities do not fit the solver's LDS tile gather from
  // global memory, where the uid order's locality is worth more: they keep it.
  const int nr = w.part_rep_off[p + 1] - w.part_rep_off[p];
  const int tile = w.pgs_cfg == 0 ? kPgsCfgReps[0] : (w.pgs_cfg == 1 ? kPgsCfgReps[1]
                                                     : (w.pgs_cfg == 2 ? kPgsCfgReps[2] : kPgsCfgReps[3]));
  if (nr > tile) return;
  const int u0 = w.part_copy_off[p], u1 = w.part_copy_off[p + 1];
  const int ncol = w.part_ncol[p];
  if (tid < kColStride) coff[tid] = w.part_col_off[p * kColStride + tid];
  for (int u = u0 + tid; u < u1; u += kSpreadBS) w.cp_inv[w.cp_slot[u]] = u;
  __syncthreads();
  int* T = tab[wave];
  int* Rn = run[wave];
  int* Bs = base[wave];
  auto key_of = [&](int u) {
    const int ia = w.cp_ia[u], ib = w.cp_ib[u];
    const int d = ib < 0 ? 16 : ((ia - ib) & 15);
    return d * 16 + (ia & 15);
  };
  for (int c = wave; c < ncol; c += kSpreadWaves) {
    const int cb = u0 + coff[c], n = coff[c + 1] - coff[c];
    for (int k = lane; k < kSpreadKeys; k += 64) {
      T[k] = 0;
      Rn[k] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < n; i += 64) atomicAdd(&T[key_of(w.cp_inv[cb + i])], 1);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    // group sizes and starts: lane d < 17 sums its group
    int nd = 0;
    if (lane < 17)
      for (int r = 0; r < 16; ++r) nd += T[lane * 16 + r];
    const int inc = wave_incl_scan(nd);
    if (lane < 17) Bs[lane] = inc - nd;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int i0 = 0; i0 < n; i0 += 64) {
      const int i = i0 + lane;
      const bool valid = i < n;
      const int u = valid ? w.cp_inv[cb + i] : -1;
      const int key = valid ? key_of(u) : 511;
      // lanes holding the same key (nine ballots over its bits)
      uint64_t peers = ~0ull;
#pragma unroll
      for (int b = 0; b < 9; ++b) {
        const uint64_t bal = __ballot((key >> b) & 1);
        peers &= ((key >> b) & 1) ? bal : ~bal;
      }
      const int rank = __popcll(peers & lanemask_lt());
      const int j = valid ? Rn[key] + rank : 0;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
      if (valid && rank == 0) Rn[key] += __popcll(peers);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        const int d = key >> 4, r = key & 15;
        int pos = Bs[d];
        for (int q = 0; q < 16; ++q) {
          const int cq = T[d * 16 + q];
          pos += min(cq, j) + ((q < r && cq > j) ? 1 : 0);
        }
        w.cp_slot[u] = cb + pos;
      }
    }
  }
}

hipError_t launch_solve_pre(const WP& w, hipStream_t s) {
  hipError_t e;
  if (w.couple && w.N > 0) {
    k_couple<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.N > 0) {
    k_rep_mass<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.G > 0) {
    k_part_order<<<nblocks(w.G, kOrderBS), kOrderBS, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
    // with more partitions than compute units the small ones colour several
    // to a compute unit; otherwise every partition has a compute unit of its own
    const int split = w.G > w.n_cu ? 1 : 0;
    k_colour<kColBS, kColLds, kColRepLds, false><<<w.G, kColBS, 0, s>>>(w, split);
    if (split) k_colour<kColSmallBS, kColSmallCopies, kColSmallReps, true><<<w.G, kColSmallBS, 0, s>>>(w, split);
    k_slot_spread<<<w.G, kSpreadBS, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.Mcap > 0) {
    k_rows<<<nblocks(w.Mcap, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.learned) {
    if ((e = launch_mlp_world(w, s))) return e;
  }
  if (w.has_caps && w.Rcap > 0) {
    k_rep_axis<<<nblocks(w.Rcap, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  return hipSuccess;
}

hipError_t launch_pgs(const WP& w, hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end) {
  if (w.G <= 0) return hipSuccess;
  hipError_t e;
  if (ev_begin && (e = hipEventRecord(ev_begin, s))) return e;
  switch (w.pgs_cfg) {
    case 0: e = launch_pgs_t<1024, 4800>(w, s); break;
    case 1: e = launch_pgs_t<512, 2400>(w, s); break;
    case 2: e = launch_pgs_t<256, 1200>(w, s); break;
    case 3: e = launch_pgs_t<256, 2400>(w, s); break;
    default: e = hipErrorInvalidValue;
  }
  if (e) return e;
  if (ev_end && (e = hipEventRecord(ev_end, s))) return e;
  return hipSuccess;
}

hipError_t launch_solve_post(const WP& w, hipStream_t s, bool exact_residual) {
  hipError_t e;
  if (exact_residual && w.G > 0) {
    if ((e = fill_i32((int32_t*)w.stat_f, 0, 1, s))) return e;
    k_exact_resid<<<w.G, 256, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.N > 0) {
    k_blend<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (exact_residual && w.J > 0) {
    k_joint_viol<<<nblocks(w.J, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.Mcap > 0) {
    k_cache<<<nblocks(w.Mcap, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  k_commit<<<1, kCommitBS, 0, s>>>(w);
  if ((e = hipGetLastError())) return e;
  if (w.lb_on) return launch_balance_commit(w, s);
  return hipSuccess;
}

// reset the impulses to the warm start (to time the solve again on the same inputs)
__global__ void k_reset_lambda(WP w) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < w.Mcap) w.r_lam[u] = w.r_lam0[u];
}

// order-independent 64-bit digest of the replica states and sweep counts
__global__ void k_digest(WP w, unsigned long long* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int R = w.G > 0 ? w.part_rep_off[w.G] : 0;
  unsigned long long acc = 0;
  if (i < R) {
    for (int k = 0; k < 13; ++k) {
      const uint32_t bits = __float_as_uint(w.rst[(int64_t)k * w.Rcap + i]);
      acc += (unsigned long long)fmix32(bits ^ fmix32((uint32_t)(13 * i + k))) << (k & 31);
    }
  }
  if (i < w.G) acc += (unsigned long long)fmix32((uint32_t)w.part_iters[i] ^ 0x9e3779b9u) << 7;
  if (acc) atomicAdd(out, acc);
}

hipError_t launch_reset_lambda(const WP& w, hipStream_t s) {
  if (w.Mcap <= 0) return hipSuccess;
  k_reset_lambda<<<nblocks(w.Mcap, kBlock), kBlock, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_digest(const WP& w, unsigned long long* out, hipStream_t s) {
  hipError_t e;
  if ((e = fill_u64((uint64_t*)out, 0, 1, s))) return e;
  const int n = std::max(w.Rcap, w.G);
  if (n > 0) k_digest<<<nblocks(n, kBlock), kBlock, 0, s>>>(w, out);
  return hipGetLastError();
}

}  // namespace ovl
