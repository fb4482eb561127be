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
//  * Gauss-Seidel: one workgroup per partition (the paper's worker); replica
//    velocities and inverse masses stay in LDS; colours are separated by
//    workgroup barriers.  Adaptive mode stops when a sweep's largest
//    |A_rr * delta lambda| is <= tol.
//  * Integration: x += h v; q <- normalise(q + h/2 (0, w) q).
//  * Blend (Alg. 4, Eq. 11-14): weights from the geodesic distances (Eq. 15-16),
//    replicas in ascending partition id, quaternions sign-aligned with the
//    first one and renormalised.  A body with one replica keeps its state.
#include "ovl_internal.h"
#include "wave.h"

namespace ovl {

namespace {

struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ f3 add(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 sub(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 scale(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }

__device__ __forceinline__ bool step_failed(const WP& w) {
  return __hip_atomic_load(&w.scal[SC_FLAGS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Duff et al., "Building an Orthonormal Basis, Revisited" (JCGT 2017)
__device__ __forceinline__ void tangents(f3 n, f3& t1, f3& t2) {
  float s = copysignf(1.0f, n.z);
  float a = -1.0f / (s + n.z);
  float b = n.x * n.y * a;
  t1 = mk(1.0f + s * n.x * n.x * a, s * b, -s * n.x);
  t2 = mk(b, s + n.y * n.y * a, -n.y);
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

__device__ __forceinline__ bool prio_gt(uint32_t ha, int ua, uint32_t hb, int ub) {
  return ha > hb || (ha == hb && ua > ub);
}

// ------------------------------------------------------------ colouring ----

constexpr int kColBS = 1024;
constexpr int kColWaves = kColBS / 64;

__global__ __launch_bounds__(kColBS) void k_colour(WP w) {
  __shared__ int lds_i[kColWaves];
  __shared__ int ccount[kMaxColours];
  __shared__ int col_off[kColStride];
  __shared__ int running[kMaxColours];
  __shared__ int wcnt[kColWaves][kMaxColours];
  __shared__ int any_s;
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid == 0) any_s = (w.scal[SC_FLAGS] & (F_CONTACT_CAP | F_ADJ_CAP | F_REP_CAP | F_COPY_CAP)) ? 1 : 0;
  __syncthreads();
  if (any_s) return;
  const int u0 = w.part_copy_off[p], u1 = w.part_copy_off[p + 1];
  const int r0 = w.part_rep_off[p], r1 = w.part_rep_off[p + 1];
  const int nr = r1 - r0;
  if (tid == 0) w.part_nstatic[p] = 0;
  int* inc_cnt = w.inc_off + w.Rcap;  // second half of inc_off holds the counts
  // incidence lists of the partition's replicas
  for (int r = tid; r < nr; r += kColBS) inc_cnt[r0 + r] = 0;
  __syncthreads();
  for (int u = u0 + tid; u < u1; u += kColBS) {
    atomicAdd(&inc_cnt[r0 + w.cp_ia[u]], 1);
    int ib = w.cp_ib[u];
    if (ib >= 0) atomicAdd(&inc_cnt[r0 + ib], 1);
    w.cp_colour[u] = -1;
  }
  __syncthreads();
  {
    int carry = 2 * u0;
    for (int base = 0; base < nr; base += kColBS) {
      int r = base + tid;
      int v = r < nr ? inc_cnt[r0 + r] : 0;
      int tot;
      int pre = block_excl_scan<kColBS>(v, lds_i, tot);
      if (r < nr) {
        w.inc_off[r0 + r] = carry + pre;
        inc_cnt[r0 + r] = 0;
      }
      carry += tot;
    }
  }
  __syncthreads();
  for (int u = u0 + tid; u < u1; u += kColBS) {
    int ia = r0 + w.cp_ia[u];
    w.inc[w.inc_off[ia] + atomicAdd(&inc_cnt[ia], 1)] = u;
    int ib = w.cp_ib[u];
    if (ib >= 0) w.inc[w.inc_off[r0 + ib] + atomicAdd(&inc_cnt[r0 + ib], 1)] = u;
  }
  __syncthreads();
  // Jones-Plassmann rounds
  bool overflow = false;
  for (;;) {
    bool pending = false;
    for (int u = u0 + tid; u < u1; u += kColBS) {
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
      if (ready) {
        int c;
        if (used == ~0ull) {
          overflow = true;
          c = kMaxColours - 1;
        } else {
          c = __ffsll((unsigned long long)~used) - 1;
        }
        __hip_atomic_store(&w.cp_colour[u], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        pending = true;
      }
    }
    if (!__syncthreads_or(pending)) break;
  }
  if (__syncthreads_or(overflow) && tid == 0) atomicOr(&w.scal[SC_FLAGS], F_COLOUR_CAP);
  // colour histogram and offsets
  if (tid < kMaxColours) {
    ccount[tid] = 0;
    running[tid] = 0;
  }
  __syncthreads();
  for (int u = u0 + tid; u < u1; u += kColBS) atomicAdd(&ccount[w.cp_colour[u]], 1);
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
  for (int base = u0; base < u1; base += kColBS) {
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
      for (int q = 0; q < kColWaves; ++q) t += wcnt[q][tid];
      running[tid] += t;
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------- rows ----

__device__ __forceinline__ int cache_find(const WP& w, int n, int part, int kind, uint64_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int pm = w.wc_part[mid], km = w.wc_kind[mid];
    uint64_t xm = w.wc_key[mid];
    bool less = pm < part || (pm == part && (km < kind || (km == kind && xm < key)));
    if (less)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < n && w.wc_part[lo] == part && w.wc_kind[lo] == kind && w.wc_key[lo] == key) return lo;
  return -1;
}

__global__ void k_rows(WP w) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int M = w.part_copy_off[w.G];
  if (u >= M || u >= w.Mcap || step_failed(w)) return;
  const int N = w.N;
  const int slot = w.cp_slot[u];
  const int src = w.cp_src[u];
  const int p = w.cp_part[u];
  int a, b;
  f3 d[3], ra, rb;
  float bias[3], mu;
  int kind;
  uint64_t key;
  if (src < w.J) {
    kind = 0;
    key = (uint64_t)src;
    a = w.j_ab[2 * src];
    b = w.j_ab[2 * src + 1];
    const float* an = w.j_anchor + 6 * src;
    ra = quat_rotate(w.st[3 * N + a], w.st[4 * N + a], w.st[5 * N + a], w.st[6 * N + a], mk(an[0], an[1], an[2]));
    rb = quat_rotate(w.st[3 * N + b], w.st[4 * N + b], w.st[5 * N + b], w.st[6 * N + b], mk(an[3], an[4], an[5]));
    f3 xa = mk(w.st[a], w.st[N + a], w.st[2 * N + a]);
    f3 xb = mk(w.st[b], w.st[N + b], w.st[2 * N + b]);
    f3 C = sub(add(xa, ra), add(xb, rb));
    d[0] = mk(-1, 0, 0);
    d[1] = mk(0, -1, 0);
    d[2] = mk(0, 0, -1);
    const float k = w.erp / w.dt;
    bias[0] = k * C.x;
    bias[1] = k * C.y;
    bias[2] = k * C.z;
    mu = -1.0f;
  } else {
    kind = 1;
    const int c = src - w.J;
    a = w.c_a[c];
    const uint32_t bk = w.c_bkey[c];
    key = ((uint64_t)a << 32) | bk;
    b = (bk >> 1) < (uint32_t)N ? (int)(bk >> 1) : -1;
    const int64_t C = w.Ccap;
    d[0] = mk(w.c_geom[c], w.c_geom[C + c], w.c_geom[2 * C + c]);
    const float phi = w.c_geom[3 * C + c];
    ra = mk(w.c_geom[4 * C + c], w.c_geom[5 * C + c], w.c_geom[6 * C + c]);
    rb = mk(w.c_geom[7 * C + c], w.c_geom[8 * C + c], w.c_geom[9 * C + c]);
    tangents(d[0], d[1], d[2]);
    if (b < 0) atomicAdd(&w.part_nstatic[p], 1);
    bias[0] = phi > 0.0f ? phi / w.dt : w.erp * phi / w.dt;
    bias[1] = 0.0f;
    bias[2] = 0.0f;
    mu = w.s_mu[w.b_scene[a]];
  }
  const float ima = w.b_invm[a], iia = w.b_invI[a];
  const float imb = b >= 0 ? w.b_invm[b] : 0.0f, iib = b >= 0 ? w.b_invI[b] : 0.0f;
  const int64_t MC = w.Mcap;
  w.r_ia[slot] = w.cp_ia[u];
  w.r_ib[slot] = w.cp_ib[u];
  float* f = w.r_f;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    f3 aa = cross(ra, d[r]);
    float A = ima + iia * dot(aa, aa);
    if (b >= 0) {
      f3 ab = cross(rb, d[r]);
      A += imb + iib * dot(ab, ab);
    }
    A += w.cfm;
    f[(RF_D0 + 3 * r) * MC + slot] = d[r].x;
    f[(RF_D0 + 3 * r + 1) * MC + slot] = d[r].y;
    f[(RF_D0 + 3 * r + 2) * MC + slot] = d[r].z;
    f[(RF_INVD + r) * MC + slot] = 1.0f / A;
    f[(RF_BIAS + r) * MC + slot] = bias[r];
  }
  f[(RF_RA + 0) * MC + slot] = ra.x;
  f[(RF_RA + 1) * MC + slot] = ra.y;
  f[(RF_RA + 2) * MC + slot] = ra.z;
  f[(RF_RB + 0) * MC + slot] = rb.x;
  f[(RF_RB + 1) * MC + slot] = rb.y;
  f[(RF_RB + 2) * MC + slot] = rb.z;
  f[RF_MU * MC + slot] = mu;
  // warm start
  float l0 = 0.0f, l1 = 0.0f, l2 = 0.0f;
  const int prevM = w.scal[SC_PREV_NCOPY];
  if (w.warmstart && prevM > 0) {
    int hit = cache_find(w, prevM, p, kind, key);
    if (hit >= 0) {
      const float* v = w.wc_val;
      if (kind == 0) {
        l0 = v[hit];
        l1 = v[MC + hit];
        l2 = v[2 * MC + hit];
      } else {
        float ln = fmaxf(v[hit], 0.0f);
        f3 fw = mk(v[MC + hit], v[2 * MC + hit], v[3 * MC + hit]);
        float bnd = mu * ln;
        l0 = ln;
        l1 = fminf(fmaxf(dot(fw, d[1]), -bnd), bnd);
        l2 = fminf(fmaxf(dot(fw, d[2]), -bnd), bnd);
      }
    }
  }
  w.r_lam0[slot] = l0;
  w.r_lam0[MC + slot] = l1;
  w.r_lam0[2 * MC + slot] = l2;
  w.r_lam[slot] = l0;
  w.r_lam[MC + slot] = l1;
  w.r_lam[2 * MC + slot] = l2;
}

// ---------------------------------------------------------- Gauss-Seidel ----

// replica velocity storage: LDS (component-major [8][nr]) or, for partitions
// too large for LDS, the partition's own slice of the replica-state array
template <bool kLds>
struct Vel;

template <>
struct Vel<true> {
  float* s;
  int n;
  __device__ __forceinline__ float* ptr(int comp, int r) const { return s + comp * n + r; }
};

template <>
struct Vel<false> {
  float* s;  // rst + r0 ; component stride Rcap
  int64_t stride;
  __device__ __forceinline__ float* ptr(int comp, int r) const { return s + comp * stride + r; }
};
// components: 0..2 v, 3..5 w, 6 invm, 7 invI

struct Row3 {
  f3 d[3];
  f3 ra, rb;
  float invd[3], bias[3], mu;
  int ia, ib;
};

__device__ __forceinline__ void load_row(const WP& w, int slot, Row3& R) {
  const int64_t MC = w.Mcap;
  const float* f = w.r_f;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    R.d[r] = mk(f[(RF_D0 + 3 * r) * MC + slot], f[(RF_D0 + 3 * r + 1) * MC + slot], f[(RF_D0 + 3 * r + 2) * MC + slot]);
    R.invd[r] = f[(RF_INVD + r) * MC + slot];
    R.bias[r] = f[(RF_BIAS + r) * MC + slot];
  }
  R.ra = mk(f[RF_RA * MC + slot], f[(RF_RA + 1) * MC + slot], f[(RF_RA + 2) * MC + slot]);
  R.rb = mk(f[RF_RB * MC + slot], f[(RF_RB + 1) * MC + slot], f[(RF_RB + 2) * MC + slot]);
  R.mu = f[RF_MU * MC + slot];
  R.ia = w.r_ia[slot];
  R.ib = w.r_ib[slot];
}

struct Body6 {
  f3 v, w;
  float im, ii;
};

template <class V>
__device__ __forceinline__ Body6 load_body(const V& V_, int r) {
  Body6 b;
  b.v = mk(*V_.ptr(0, r), *V_.ptr(1, r), *V_.ptr(2, r));
  b.w = mk(*V_.ptr(3, r), *V_.ptr(4, r), *V_.ptr(5, r));
  b.im = *V_.ptr(6, r);
  b.ii = *V_.ptr(7, r);
  return b;
}

template <class V>
__device__ __forceinline__ void store_vel(const V& V_, int r, const Body6& b) {
  *V_.ptr(0, r) = b.v.x;
  *V_.ptr(1, r) = b.v.y;
  *V_.ptr(2, r) = b.v.z;
  *V_.ptr(3, r) = b.w.x;
  *V_.ptr(4, r) = b.w.y;
  *V_.ptr(5, r) = b.w.z;
}

// apply impulse dl of row r
__device__ __forceinline__ void apply(Body6& A, Body6& B, bool hasB, const Row3& R, int r, f3 angA, f3 angB,
                                      float dl) {
  A.v = sub(A.v, scale(R.d[r], A.im * dl));
  A.w = sub(A.w, scale(angA, A.ii * dl));
  if (hasB) {
    B.v = add(B.v, scale(R.d[r], B.im * dl));
    B.w = add(B.w, scale(angB, B.ii * dl));
  }
}

template <bool kLds>
__global__ __launch_bounds__(kPgsBlock) void k_pgs(WP w) {
  extern __shared__ float sm[];
  __shared__ int coff[kColStride];
  __shared__ float red[kPgsBlock / 64];
  __shared__ int failed_s;
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  // one read of the failure flag per workgroup, so the early exit is uniform
  if (tid == 0) failed_s = step_failed(w) ? 1 : 0;
  __syncthreads();
  if (failed_s) {
    if (tid == 0) {
      w.part_iters[p] = 0;
      w.part_resid[p] = 0.0f;
    }
    return;
  }
  const int N = w.N;
  const int r0 = w.part_rep_off[p];
  const int nr = w.part_rep_off[p + 1] - r0;
  if (kLds != (nr <= kLdsReps)) return;  // the other variant handles this partition
  const int s0 = w.part_copy_off[p];
  const int ncol = w.part_ncol[p];
  if (tid < kColStride) coff[tid] = w.part_col_off[p * kColStride + tid];
  Vel<kLds> V;
  if constexpr (kLds) {
    V.s = sm;
    V.n = nr;
  } else {
    V.s = w.rst + r0;
    V.stride = w.Rcap;
  }
  // load replica velocities (gravity applied: v~ = v + h g) and inverse masses
  const float hgx = w.dt * w.gx, hgy = w.dt * w.gy, hgz = w.dt * w.gz;
  for (int r = tid; r < nr; r += kPgsBlock) {
    const int b = w.rep_body_pm[r0 + r];
    *V.ptr(0, r) = w.st[7 * N + b] + hgx;
    *V.ptr(1, r) = w.st[8 * N + b] + hgy;
    *V.ptr(2, r) = w.st[9 * N + b] + hgz;
    *V.ptr(3, r) = w.st[10 * N + b];
    *V.ptr(4, r) = w.st[11 * N + b];
    *V.ptr(5, r) = w.st[12 * N + b];
    *V.ptr(6, r) = w.b_invm[b];
    *V.ptr(7, r) = w.b_invI[b];
  }
  __syncthreads();
  const int64_t MC = w.Mcap;
  // warm-start impulses enter in solve order
  for (int c = 0; c < ncol; ++c) {
    const int e = s0 + coff[c + 1];
    for (int slot = s0 + coff[c] + tid; slot < e; slot += kPgsBlock) {
      float l[3] = {w.r_lam[slot], w.r_lam[MC + slot], w.r_lam[2 * MC + slot]};
      if (l[0] == 0.0f && l[1] == 0.0f && l[2] == 0.0f) continue;
      Row3 R;
      load_row(w, slot, R);
      const bool hasB = R.ib >= 0;
      Body6 A = load_body(V, R.ia);
      Body6 B;
      if (hasB) B = load_body(V, R.ib);
#pragma unroll
      for (int r = 0; r < 3; ++r) apply(A, B, hasB, R, r, cross(R.ra, R.d[r]), cross(R.rb, R.d[r]), l[r]);
      store_vel(V, R.ia, A);
      if (hasB) store_vel(V, R.ib, B);
    }
    __syncthreads();
  }
  // sweeps
  const int cap = w.forced ? w.part_force_iters[p] : w.max_iters;
  int it = 0;
  float rho = 0.0f;
  while (it < cap) {
    float rl = 0.0f;
    for (int c = 0; c < ncol; ++c) {
      const int e = s0 + coff[c + 1];
      for (int slot = s0 + coff[c] + tid; slot < e; slot += kPgsBlock) {
        Row3 R;
        load_row(w, slot, R);
        float l[3] = {w.r_lam[slot], w.r_lam[MC + slot], w.r_lam[2 * MC + slot]};
        const bool hasB = R.ib >= 0;
        Body6 A = load_body(V, R.ia);
        Body6 B;
        if (hasB) B = load_body(V, R.ib);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const f3 angA = cross(R.ra, R.d[r]);
          const f3 angB = cross(R.rb, R.d[r]);
          float vr = -dot(R.d[r], A.v) - dot(angA, A.w);
          if (hasB) vr += dot(R.d[r], B.v) + dot(angB, B.w);
          const float wv = vr + R.bias[r] + w.cfm * l[r];
          float lo, hi;
          if (R.mu < 0.0f) {
            lo = -INFINITY;
            hi = INFINITY;
          } else if (r == 0) {
            lo = 0.0f;
            hi = INFINITY;
          } else {
            hi = R.mu * l[0];
            lo = -hi;
          }
          const float nl = fminf(fmaxf(l[r] - wv * R.invd[r], lo), hi);
          const float dl = nl - l[r];
          l[r] = nl;
          apply(A, B, hasB, R, r, angA, angB, dl);
          rl = fmaxf(rl, fabsf(dl) / R.invd[r]);
        }
        store_vel(V, R.ia, A);
        if (hasB) store_vel(V, R.ib, B);
        w.r_lam[slot] = l[0];
        w.r_lam[MC + slot] = l[1];
        w.r_lam[2 * MC + slot] = l[2];
      }
      __syncthreads();
    }
    rho = block_max<kPgsBlock>(rl, red);
    ++it;
    if (!w.forced && w.adaptive && rho <= w.tol) break;
  }
  // integrate and write the replica states
  const float h = w.dt;
  bool bad = false;
  for (int r = tid; r < nr; r += kPgsBlock) {
    const int b = w.rep_body_pm[r0 + r];
    Body6 B = load_body(V, r);
    float x = w.st[b] + h * B.v.x;
    float y = w.st[N + b] + h * B.v.y;
    float z = w.st[2 * N + b] + h * B.v.z;
    float qw = w.st[3 * N + b], qx = w.st[4 * N + b], qy = w.st[5 * N + b], qz = w.st[6 * N + b];
    const float wx = B.w.x, wy = B.w.y, wz = B.w.z;
    const float dw = -(wx * qx + wy * qy + wz * qz);
    const float dx = wx * qw + (wy * qz - wz * qy);
    const float dy = wy * qw + (wz * qx - wx * qz);
    const float dz = wz * qw + (wx * qy - wy * qx);
    qw += 0.5f * h * dw;
    qx += 0.5f * h * dx;
    qy += 0.5f * h * dy;
    qz += 0.5f * h * dz;
    const float nn = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    float out[13] = {x, y, z, qw * nn, qx * nn, qy * nn, qz * nn, B.v.x, B.v.y, B.v.z, B.w.x, B.w.y, B.w.z};
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
  float sum = 0.0f;
  for (int k = 0; k < n; ++k) {
    const int D = w.rep_D_bm[bm0 + k];
    sum += D > 0 ? 1.0f / (float)D : 0.0f;
  }
  float acc[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) acc[k] = 0.0f;
  float q0[4];
  for (int k = 0; k < n; ++k) {
    const int D = w.rep_D_bm[bm0 + k];
    const float wt = sum > 0.0f ? (D > 0 ? 1.0f / (float)D : 0.0f) / sum : 1.0f / (float)n;
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
  const float l0 = w.r_lam[slot], l1 = w.r_lam[MC + slot], l2 = w.r_lam[2 * MC + slot];
  w.wc_part[u] = w.cp_part[u];
  if (src < w.J) {
    w.wc_kind[u] = 0;
    w.wc_key[u] = (uint64_t)src;
    w.wc_val[u] = l0;
    w.wc_val[MC + u] = l1;
    w.wc_val[2 * MC + u] = l2;
    w.wc_val[3 * MC + u] = 0.0f;
  } else {
    const int c = src - w.J;
    w.wc_kind[u] = 1;
    w.wc_key[u] = ((uint64_t)w.c_a[c] << 32) | w.c_bkey[c];
    const float* f = w.r_f;
    f3 t1 = mk(f[(RF_D0 + 3) * MC + slot], f[(RF_D0 + 4) * MC + slot], f[(RF_D0 + 5) * MC + slot]);
    f3 t2 = mk(f[(RF_D0 + 6) * MC + slot], f[(RF_D0 + 7) * MC + slot], f[(RF_D0 + 8) * MC + slot]);
    f3 fw = add(scale(t1, l1), scale(t2, l2));
    w.wc_val[u] = l0;
    w.wc_val[MC + u] = fw.x;
    w.wc_val[2 * MC + u] = fw.y;
    w.wc_val[3 * MC + u] = fw.z;
  }
}

__global__ void k_commit(WP w) {
  if (threadIdx.x || blockIdx.x) return;
  if (w.scal[SC_FLAGS] != 0) return;
  w.scal[SC_PREV_NCOPY] = w.part_copy_off[w.G];
  w.scal[SC_COMMITTED] += 1;
  int mx = 0, unconv = 0;
  int64_t bytes = 0, sweeps = 0;
  for (int g = 0; g < w.G; ++g) {
    const int it = w.part_iters[g];
    mx = max(mx, it);
    if (w.adaptive && !w.forced && it >= w.max_iters && w.part_resid[g] > w.tol) ++unconv;
    const int64_t nj = w.mc_psize[1][g], nc = w.mc_psize[2][g], ns = w.part_nstatic[g];
    bytes += (int64_t)it * ((nc - ns) * kBytesDynDyn + ns * kBytesStatic + nj * kBytesJoint);
    sweeps += it;
  }
  w.stat_i64[0] += mx;
  w.stat_i64[1] += unconv;
  w.stat_i64[2] += bytes;
  w.stat_i64[3] += sweeps;
  w.stat_i64[4] += 1;
}

// natural-map residual of the final iterate, one workgroup per partition
__global__ __launch_bounds__(256) void k_exact_resid(WP w) {
  __shared__ float red[4];
  __shared__ int failed_s;
  const int p = blockIdx.x;
  if (threadIdx.x == 0) failed_s = step_failed(w) ? 1 : 0;
  __syncthreads();
  if (failed_s) return;
  const int r0 = w.part_rep_off[p];
  const int s0 = w.part_copy_off[p], s1 = w.part_copy_off[p + 1];
  const int64_t MC = w.Mcap, RC = w.Rcap;
  float e = 0.0f;
  for (int slot = s0 + threadIdx.x; slot < s1; slot += 256) {
    Row3 R;
    load_row(w, slot, R);
    float l[3] = {w.r_lam[slot], w.r_lam[MC + slot], w.r_lam[2 * MC + slot]};
    const int ra_ = r0 + R.ia;
    f3 va = mk(w.rst[7 * RC + ra_], w.rst[8 * RC + ra_], w.rst[9 * RC + ra_]);
    f3 wa = mk(w.rst[10 * RC + ra_], w.rst[11 * RC + ra_], w.rst[12 * RC + ra_]);
    f3 vb = mk(0, 0, 0), wb = mk(0, 0, 0);
    if (R.ib >= 0) {
      const int rb_ = r0 + R.ib;
      vb = mk(w.rst[7 * RC + rb_], w.rst[8 * RC + rb_], w.rst[9 * RC + rb_]);
      wb = mk(w.rst[10 * RC + rb_], w.rst[11 * RC + rb_], w.rst[12 * RC + rb_]);
    }
    for (int r = 0; r < 3; ++r) {
      f3 angA = cross(R.ra, R.d[r]), angB = cross(R.rb, R.d[r]);
      float vr = -dot(R.d[r], va) - dot(angA, wa) + dot(R.d[r], vb) + dot(angB, wb);
      float wv = vr + R.bias[r] + w.cfm * l[r];
      float lo = -INFINITY, hi = INFINITY;
      if (R.mu >= 0.0f) {
        if (r == 0)
          lo = 0.0f;
        else {
          hi = R.mu * l[0];
          lo = -hi;
        }
      }
      float pr = fminf(fmaxf(l[r] - wv * R.invd[r], lo), hi);
      e = fmaxf(e, fabsf(l[r] - pr) / R.invd[r]);
    }
  }
  e = block_max<256>(e, red);
  if (threadIdx.x == 0) atomicMax((int*)&w.stat_f[0], __float_as_int(e));
}

}  // namespace

hipError_t pgs_set_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)k_pgs<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     8 * kLdsReps * (int)sizeof(float));
  return e;
}

hipError_t launch_solve(const WP& w, int32_t* sc, hipStream_t s, bool exact_residual, hipEvent_t ev_pgs_begin,
                        hipEvent_t ev_pgs_end) {
  (void)sc;
  hipError_t e;
  if (w.G > 0) {
    k_colour<<<w.G, kColBS, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.Mcap > 0) {
    k_rows<<<nblocks(w.Mcap, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.G > 0) {
    if (ev_pgs_begin && (e = hipEventRecord(ev_pgs_begin, s))) return e;
    k_pgs<true><<<w.G, kPgsBlock, 8 * kLdsReps * sizeof(float), s>>>(w);
    if ((e = hipGetLastError())) return e;
    k_pgs<false><<<w.G, kPgsBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
    if (ev_pgs_end && (e = hipEventRecord(ev_pgs_end, s))) return e;
  }
  if (exact_residual && w.G > 0) {
    if ((e = fill_i32((int32_t*)w.stat_f, 0, 1, s))) return e;
    k_exact_resid<<<w.G, 256, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.N > 0) {
    k_blend<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if (w.Mcap > 0) {
    k_cache<<<nblocks(w.Mcap, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  k_commit<<<1, 1, 0, s>>>(w);
  return hipGetLastError();
}

}  // namespace ovl
