// Dynamic load balancing of the worker sets (section 5.4): Alg. 6 over the
// step's contacts, with the bridge test of Alg. 7.
//
// The worker sets W_b (one u64 of local partition bits per body) are carried
// from the last committed step.  Every contact of the step between two
// dynamic bodies is taken in key order (statics are not vertices of the
// constraint graph).  The rules are order dependent: an activation changes the
// loads the next decision reads, and any rule changes the sets the next
// contacts see.  One wavefront per scene therefore walks the scene's contacts
// with a 64-wide window: every lane tests whether the rule of its contact
// would change anything in the current state.  Contacts before the first lane
// that would are no-ops in sequence too (nothing before them changes the
// state), so the window skips them, applies that one contact with the whole
// wavefront, and restarts right after it.  The result is the sequential one.
// Scenes are independent and run as separate workgroups.
//
// Readings (the same as stated by the oracle):
//   * the load of a set of workers is the number of bodies active in them,
//     summed over the set's workers;
//   * a tie in the first rule goes to the first body's side;
//   * "smallest load" ties go to the lowest worker index;
//   * the growth BFS reaches every vertex within the depth, its root included.
#include "ovl_internal.h"
#include "wave.h"

namespace ovl {
namespace {

constexpr int kLbBS = 64;  // one wavefront per scene

// worker sets of the last committed step
__global__ void k_lb_begin(WP w) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < w.N) w.mask[v] = w.lb_mask[v];
}

// Where a scene's sets, growth queue and visited bits live: LDS for scenes of
// up to kLbLdsCap bodies, else the global copies.  Indices are scene-local;
// visited bit of local vertex v = bit (v + vb) of vis.
struct LbMem {
  uint64_t* m;
  int32_t* q;
  uint32_t* vis;
  int vb;
};

// sum of the loads of the workers in `set` (lane k holds worker k's load)
__device__ __forceinline__ long long set_load(uint64_t set, int my_load) {
  long long v = ((set >> lane_id()) & 1ull) ? (long long)my_load : 0ll;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ void activate(const LbMem& L, int* load, uint64_t set, int v) {
  const uint64_t old = L.m[v];
  const uint64_t add = set & ~old;
  if (lane_id() == 0) L.m[v] = old | add;
  if ((add >> lane_id()) & 1ull) load[lane_id()] += 1;
  __syncthreads();
}

__device__ __forceinline__ void deactivate(const LbMem& L, int* load, uint64_t set, int v) {
  const uint64_t old = L.m[v];
  const uint64_t rem = set & old;
  if (lane_id() == 0) L.m[v] = old & ~rem;
  if ((rem >> lane_id()) & 1ull) load[lane_id()] -= 1;
  __syncthreads();
}

// Alg. 7 by one lane: the union of the neighbours' sets spans more than one worker
__device__ __forceinline__ bool bridge_lane(const WP& w, const LbMem& L, int b0, int n, int v) {
  uint64_t acc = 0;
  const int o1 = w.adj_off[b0 + v + 1];
  for (int k = w.adj_off[b0 + v]; k < o1; ++k) {
    const int u = w.adj[k] - b0;
    if (u >= 0 && u < n) acc |= L.m[u];
  }
  return __popcll(acc) > 1;
}

// Alg. 7 by the whole wavefront
__device__ __forceinline__ bool bridge_wave(const WP& w, const LbMem& L, int b0, int n, int v) {
  const int o0 = w.adj_off[b0 + v], o1 = w.adj_off[b0 + v + 1];
  uint64_t acc = 0;
  for (int k = o0 + lane_id(); k < o1; k += 64) {
    const int u = w.adj[k] - b0;
    if (u >= 0 && u < n) acc |= L.m[u];
  }
  return __popcll(wave_or(acc)) > 1;
}

// Would the rule of contact (a, b) change any set in the current state?  (One
// lane.)  The first rule always adds workers; the bridge rules remove at least
// one; the last rule removes workers exactly when the common set has several.
__device__ __forceinline__ bool rule_changes(const WP& w, const LbMem& L, int b0, int n, int a, int b) {
  const uint64_t WA = L.m[a], WB = L.m[b];
  if ((WA & WB) == 0ull) return true;
  const int pa = __popcll(WA), pb = __popcll(WB);
  if (pa > 1 && pb == 1 && !bridge_lane(w, L, b0, n, a)) return true;
  if (pb > 1 && pa == 1 && !bridge_lane(w, L, b0, n, b)) return true;
  if (WA == WB) return pa > 1;
  return false;
}

// Growth of the first rule: every vertex within `depth` hops of root (root
// included) is activated in `set`.
__device__ void grow(const WP& w, const LbMem& L, int* load, int* tail, int b0, int n, int root, uint64_t set,
                     int depth) {
  const int lane = lane_id();
  if (lane == 0) {
    L.q[0] = root;
    atomicOr(&L.vis[(root + L.vb) >> 5], 1u << ((root + L.vb) & 31));
    *tail = 1;
  }
  __syncthreads();
  int lo = 0, hi = 1;
  for (int d = 0; d < depth && lo < hi; ++d) {
    for (int i = lo + lane; i < hi; i += 64) {
      const int v = L.q[i];
      const int o1 = w.adj_off[b0 + v + 1];
      for (int k = w.adj_off[b0 + v]; k < o1; ++k) {
        const int u = w.adj[k] - b0;
        if (u < 0 || u >= n) continue;
        const uint32_t bit = 1u << ((u + L.vb) & 31);
        if (!(atomicOr(&L.vis[(u + L.vb) >> 5], bit) & bit)) L.q[atomicAdd(tail, 1)] = u;
      }
    }
    __syncthreads();
    lo = hi;
    hi = *tail;
    __syncthreads();
  }
  for (int i = lane; i < hi; i += 64) {
    const int v = L.q[i];
    const uint64_t old = L.m[v];
    const uint64_t add = set & ~old;
    L.m[v] = old | add;
    for (uint64_t t = add; t; t &= t - 1) atomicAdd(&load[__builtin_ctzll(t)], 1);
    atomicAnd(&L.vis[(v + L.vb) >> 5], ~(1u << ((v + L.vb) & 31)));
  }
  __syncthreads();
}

// Alg. 6 for one contact, by the whole wavefront (a, b uniform)
__device__ void apply_rule(const WP& w, const LbMem& L, int* load, int* tail, int b0, int n, int a, int b) {
  const int lane = lane_id();
  const uint64_t WA = L.m[a], WB = L.m[b];
  if ((WA & WB) == 0ull) {
    // Figure 9 (i), (ii): the lighter side becomes aware of the other body
    const long long la = set_load(WA, load[lane]), lb = set_load(WB, load[lane]);
    int root;
    if (la <= lb) {
      activate(L, load, WA, b);
      root = b;
    } else {
      activate(L, load, WB, a);
      root = a;
    }
    grow(w, L, load, tail, b0, n, root, WA | WB, w.lb_depth);
  } else if (__popcll(WA) > 1 && __popcll(WB) == 1 && !bridge_wave(w, L, b0, n, a)) {
    deactivate(L, load, WA & ~WB, a);  // Figure 9 (iii); (iv) is the bridge case
  } else if (__popcll(WB) > 1 && __popcll(WA) == 1 && !bridge_wave(w, L, b0, n, b)) {
    deactivate(L, load, WB & ~WA, b);
  } else if (WA == WB) {
    // Figure 9 (v): both keep only the least loaded of their workers
    long long key = ((WA >> lane) & 1ull) ? (((long long)load[lane] << 6) | lane) : 0x7fffffffffffffffll;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const long long o = __shfl_xor(key, d, 64);
      key = o < key ? o : key;
    }
    const uint64_t keep = 1ull << (key & 63);
    deactivate(L, load, WA & ~keep, a);
    deactivate(L, load, WB & ~keep, b);
  }
}

// (local a, local b) of contact i of the scene, or (-1, -1) past the end or for a static
__device__ __forceinline__ int2 contact_pair(const WP& w, int i, int c1, int b0) {
  if (i >= c1) return make_int2(-1, -1);
  const int bc = (int)(w.c_bkey[i] >> 1);
  if (bc >= w.N) return make_int2(-1, -1);
  return make_int2(w.c_a[i] - b0, bc - b0);
}

template <bool kLds>
__global__ __launch_bounds__(kLbBS) void k_load_balance(WP w) {
  extern __shared__ uint64_t lds_m[];
  __shared__ int load[kMaxParts];
  __shared__ int tail;
  const int s = blockIdx.x, lane = lane_id();
  if (w.scal[SC_FLAGS] != 0) return;
  const int b0 = w.s_body_off[s], b1 = w.s_body_off[s + 1], n = b1 - b0;
  if (kLds != (n <= kLbLdsCap)) return;
  const int c0 = w.coff[b0], c1 = w.coff[b1];
  if (c0 >= c1) return;  // no contact: the carried sets stand
  const int np = w.s_part_base[s + 1] - w.s_part_base[s];
  LbMem L;
  if (kLds) {
    L.m = lds_m;
    L.q = (int32_t*)(lds_m + w.lb_lds_max);
    L.vis = (uint32_t*)(L.q + w.lb_lds_max);
    L.vb = 0;
  } else {
    L.m = w.mask + b0;
    L.q = w.lb_queue + b0;
    L.vis = w.lb_visit;
    L.vb = b0;
  }
  // sets into place; per-worker loads by ballot (lane k counts worker k)
  int my_load = 0;
  for (int i0 = 0; i0 < n; i0 += 4 * 64) {
    uint64_t m[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 64 + lane;
      m[u] = i < n ? w.lb_mask[b0 + i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 64 + lane;
      if (kLds && i < n) L.m[i] = m[u];
      for (int k = 0; k < np; ++k) {
        const int c = __popcll(__ballot((m[u] >> k) & 1ull));
        if (lane == k) my_load += c;
      }
    }
  }
  if (kLds)
    for (int i = lane; i < (n + 31) / 32; i += 64) L.vis[i] = 0u;
  load[lane] = my_load;
  __syncthreads();

  // the window: lane l holds contacts cb + l (x0) and cb + 64 + l (x1)
  int cb = c0;
  int2 x0 = contact_pair(w, cb + lane, c1, b0);
  int2 x1 = contact_pair(w, cb + 64 + lane, c1, b0);
  int c = c0;
  while (c < c1) {
    while (c >= cb + 64) {
      x0 = x1;
      cb += 64;
      x1 = contact_pair(w, cb + 64 + lane, c1, b0);
    }
    const int src = c - cb + lane;  // 0..127
    const int sl = src & 63;
    const int a0 = __shfl(x0.x, sl, 64), bb0 = __shfl(x0.y, sl, 64);
    const int a1 = __shfl(x1.x, sl, 64), bb1 = __shfl(x1.y, sl, 64);
    const int a = src < 64 ? a0 : a1, b = src < 64 ? bb0 : bb1;
    const bool live = a >= 0 && a < n && b >= 0 && b < n;
    const uint64_t fire = __ballot(live && rule_changes(w, L, b0, n, a, b));
    if (fire == 0ull) {
      c += 64;
      continue;
    }
    const int j = __builtin_ctzll(fire);
    apply_rule(w, L, load, &tail, b0, n, __shfl(a, j, 64), __shfl(b, j, 64));
    c += j + 1;
  }
  if (kLds)
    for (int i = lane; i < n; i += 64) w.mask[b0 + i] = L.m[i];
}

// after a committed step: its sets are carried
__global__ void k_lb_commit(WP w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < w.N && w.scal[SC_FLAGS] == 0) w.lb_mask[i] = w.mask[i];
}

}  // namespace

size_t lb_lds_bytes(int n) { return (size_t)n * (sizeof(uint64_t) + sizeof(int32_t)) + (size_t)((n + 31) / 32) * 4; }

hipError_t lb_set_attributes() {
  return hipFuncSetAttribute((const void*)k_load_balance<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lb_lds_bytes(kLbLdsCap));
}

hipError_t launch_balance(const WP& w, hipStream_t s) {
  if (w.N <= 0) return hipSuccess;
  k_lb_begin<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
  if (w.lb_lds_max > 0) k_load_balance<true><<<w.S, kLbBS, lb_lds_bytes(w.lb_lds_max), s>>>(w);
  if (w.lb_big) k_load_balance<false><<<w.S, kLbBS, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_balance_commit(const WP& w, hipStream_t s) {
  if (w.N <= 0) return hipSuccess;
  k_lb_commit<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
  return hipGetLastError();
}

}  // namespace ovl
