// Dynamic load balancing of the worker sets (section 5.4): Alg. 6 over the
// step's contacts, with the bridge test of Alg. 7.
//
// The worker sets W_b (one u64 of local partition bits per body) are carried
// from the last committed step.  Every contact of the step between two
// dynamic bodies is taken in key order (statics are not vertices of the
// constraint graph).  The rules are order dependent: an activation changes the
// loads the next decision reads, and any rule changes the sets the next
// contacts see.  One wavefront per scene therefore walks the scene's contacts
// with a 64-wide window (the other wavefronts of the workgroup only help to
// stage the scene in LDS): every lane tests whether the rule of its contact
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

constexpr int kLbBS = 256;   // four wavefronts stage a scene; the first applies the rules
constexpr int kLbLdsBytes = 152 * 1024;
constexpr int kLbChunks = 8;   // contacts fetched per global round trip: 8 x 64

// orders this wavefront's LDS and global accesses (the rules run in one wavefront)
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// worker sets of the last committed step
__global__ void k_lb_begin(WP w) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < w.N) w.mask[v] = w.lb_mask[v];
}

// Where a scene's sets, bit arrays and constraint graph live: LDS for scenes
// of up to kLbLdsCap bodies (the adjacency too, as 16-bit local ids, when it
// fits), else global memory.  Indices are scene-local: the visited and bridge
// bits of vertex v are bit (v + vb) of vis and brg; its neighbours are nbr(k)
// for k in [off[v], off[v + 1]) (negative: an empty slot).  The growth queue is
// the scene's slice of a global array.
//
// brg holds Alg. 7 for every body of the scene: set when the union of the
// neighbours' sets has more than one worker.  It is computed once when the
// scene is staged and recomputed around every body whose set changes, so the
// rules read it in one access.
struct LbMem {
  uint64_t* m;
  int32_t* q;
  uint32_t* vis;
  uint32_t* brg;
  int vb;
  const int32_t* off;
  const uint16_t* nb16;
  const int32_t* nb32;
  int nsub;
  __device__ __forceinline__ int nbr(int k) const {
    if (nb16) {
      const int u = nb16[k];
      return u == 0xFFFF ? -1 : u;
    }
    return nb32[k] - nsub;
  }
  __device__ __forceinline__ bool bridge(int v) const { return (brg[(v + vb) >> 5] >> ((v + vb) & 31)) & 1u; }
};

// Alg. 7 from the neighbours' sets, by one lane
__device__ __forceinline__ bool bridge_of(const LbMem& L, int n, int v) {
  uint64_t acc = 0;
  const int o1 = L.off[v + 1];
  for (int k = L.off[v]; k < o1; ++k) {
    const int u = L.nbr(k);
    if (u >= 0 && u < n) acc |= L.m[u];
  }
  return __popcll(acc) > 1;
}

__device__ __forceinline__ void set_bridge(const LbMem& L, int v, bool on) {
  const uint32_t bit = 1u << ((v + L.vb) & 31);
  if (on)
    atomicOr(&L.brg[(v + L.vb) >> 5], bit);
  else
    atomicAnd(&L.brg[(v + L.vb) >> 5], ~bit);
}

// the set of x changed: the bridge bits of its neighbours follow (one wavefront)
__device__ __forceinline__ void refresh_around(const LbMem& L, int n, int x) {
  const int o1 = L.off[x + 1];
  for (int k = L.off[x] + lane_id(); k < o1; k += 64) {
    const int y = L.nbr(k);
    if (y >= 0 && y < n) set_bridge(L, y, bridge_of(L, n, y));
  }
}

// sum of the loads of the workers in `set` (every lane computes it)
__device__ __forceinline__ long long set_load(uint64_t set, const int* load) {
  long long v = 0;
  for (; set; set &= set - 1) v += load[__builtin_ctzll(set)];
  return v;
}

__device__ __forceinline__ void activate(const LbMem& L, int* load, int n, uint64_t set, int v) {
  const uint64_t old = L.m[v];
  const uint64_t add = set & ~old;
  if (lane_id() == 0) L.m[v] = old | add;
  if ((add >> lane_id()) & 1ull) load[lane_id()] += 1;
  wave_fence();
  if (add) {
    refresh_around(L, n, v);
    wave_fence();
  }
}

__device__ __forceinline__ void deactivate(const LbMem& L, int* load, int n, uint64_t set, int v) {
  const uint64_t old = L.m[v];
  const uint64_t rem = set & old;
  if (lane_id() == 0) L.m[v] = old & ~rem;
  if ((rem >> lane_id()) & 1ull) load[lane_id()] -= 1;
  wave_fence();
  if (rem) {
    refresh_around(L, n, v);
    wave_fence();
  }
}

// Would the rule of contact (a, b) change any set in the current state?  (One
// lane.)  The first rule always adds workers; the bridge rules remove at least
// one; the last rule removes workers exactly when the common set has several.
__device__ __forceinline__ bool rule_changes(const LbMem& L, int a, int b) {
  const uint64_t WA = L.m[a], WB = L.m[b];
  if ((WA & WB) == 0ull) return true;
  const int pa = __popcll(WA), pb = __popcll(WB);
  if (pa > 1 && pb == 1 && !L.bridge(a)) return true;
  if (pb > 1 && pa == 1 && !L.bridge(b)) return true;
  if (WA == WB) return pa > 1;
  return false;
}

// Growth of the first rule: every vertex within `depth` hops of root (root
// included) is activated in `set`.
__device__ void grow(const LbMem& L, int* load, int* tail, int n, int root, uint64_t set, int depth) {
  const int lane = lane_id();
  if (lane == 0) {
    L.q[0] = root;
    atomicOr(&L.vis[(root + L.vb) >> 5], 1u << ((root + L.vb) & 31));
    *tail = 1;
  }
  wave_fence();
  int lo = 0, hi = 1;
  for (int d = 0; d < depth && lo < hi; ++d) {
    for (int i = lo + lane; i < hi; i += 64) {
      const int v = L.q[i];
      const int o1 = L.off[v + 1];
      for (int k = L.off[v]; k < o1; ++k) {
        const int u = L.nbr(k);
        if (u < 0 || u >= n) continue;
        const uint32_t bit = 1u << ((u + L.vb) & 31);
        if (!(atomicOr(&L.vis[(u + L.vb) >> 5], bit) & bit)) L.q[atomicAdd(tail, 1)] = u;
      }
    }
    wave_fence();
    lo = hi;
    hi = *tail;
    wave_fence();
  }
  for (int i = lane; i < hi; i += 64) {
    const int v = L.q[i];
    const uint64_t old = L.m[v];
    const uint64_t add = set & ~old;
    L.m[v] = old | add;
    for (uint64_t t = add; t; t &= t - 1) atomicAdd(&load[__builtin_ctzll(t)], 1);
    atomicAnd(&L.vis[(v + L.vb) >> 5], ~(1u << ((v + L.vb) & 31)));
  }
  wave_fence();
  for (int i = 0; i < hi; ++i) refresh_around(L, n, L.q[i]);
  wave_fence();
}

// Alg. 6 for one contact, by the whole wavefront (a, b uniform)
__device__ void apply_rule(const LbMem& L, int* load, int* tail, int n, int depth, int a, int b) {
  const uint64_t WA = L.m[a], WB = L.m[b];
  if ((WA & WB) == 0ull) {
    // Figure 9 (i), (ii): the lighter side becomes aware of the other body
    const long long la = set_load(WA, load), lb = set_load(WB, load);
    int root;
    if (la <= lb) {
      activate(L, load, n, WA, b);
      root = b;
    } else {
      activate(L, load, n, WB, a);
      root = a;
    }
    grow(L, load, tail, n, root, WA | WB, depth);
  } else if (__popcll(WA) > 1 && __popcll(WB) == 1 && !L.bridge(a)) {
    deactivate(L, load, n, WA & ~WB, a);  // Figure 9 (iii); (iv) is the bridge case
  } else if (__popcll(WB) > 1 && __popcll(WA) == 1 && !L.bridge(b)) {
    deactivate(L, load, n, WB & ~WA, b);
  } else if (WA == WB) {
    // Figure 9 (v): both keep only the least loaded of their workers (ties: lowest index)
    int best = -1, best_load = 0;
    for (uint64_t t = WA; t; t &= t - 1) {
      const int k = __builtin_ctzll(t), l = load[k];
      if (best < 0 || l < best_load) {
        best = k;
        best_load = l;
      }
    }
    const uint64_t keep = 1ull << best;
    deactivate(L, load, n, WA & ~keep, a);
    deactivate(L, load, n, WB & ~keep, b);
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
  const int s = blockIdx.x, t = threadIdx.x, lane = lane_id();
  if (w.scal[SC_FLAGS] != 0) return;
  const int b0 = w.s_body_off[s], b1 = w.s_body_off[s + 1], n = b1 - b0;
  if (kLds != (n <= kLbLdsCap)) return;
  const int c0 = w.coff[b0], c1 = w.coff[b1];
  if (c0 >= c1) return;  // no contact: the carried sets stand
  const int np = w.s_part_base[s + 1] - w.s_part_base[s];
  const int a0 = w.adj_off[b0], na = w.adj_off[b1] - a0;
  LbMem L;
  L.q = w.lb_queue + b0;
  bool adj_lds = false;
  int32_t* off_l = nullptr;
  uint16_t* nb_l = nullptr;
  if (kLds) {
    const int nm = w.lb_lds_max;
    L.m = lds_m;
    L.vis = (uint32_t*)(lds_m + nm);
    L.brg = L.vis + (nm + 31) / 32;
    off_l = (int32_t*)(L.brg + (nm + 31) / 32);
    nb_l = (uint16_t*)(off_l + nm + 1);
    adj_lds = (int64_t)((char*)(nb_l + na) - (char*)lds_m) <= kLbLdsBytes;
    L.vb = 0;
    L.off = off_l;
    L.nb16 = adj_lds ? nb_l : nullptr;
    L.nb32 = w.adj + a0;
    L.nsub = b0;
  } else {
    L.m = w.mask + b0;
    L.vis = w.lb_visit;
    L.brg = w.lb_bridge;
    L.vb = b0;
    L.off = w.adj_off + b0;
    L.nb16 = nullptr;
    L.nb32 = w.adj;
    L.nsub = b0;
  }
  if (t < kMaxParts) load[t] = 0;
  __syncthreads();
  // stage the scene: sets, per-worker loads (ballots), scene-relative adjacency
  int my_load = 0;
  for (int i0 = 0; i0 < n; i0 += 4 * kLbBS) {
    uint64_t m[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * kLbBS + t;
      m[u] = i < n ? w.lb_mask[b0 + i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * kLbBS + t;
      if (kLds && i < n) L.m[i] = m[u];
      for (int k = 0; k < np; ++k) {
        const int c = __popcll(__ballot((m[u] >> k) & 1ull));
        if (lane == k) my_load += c;
      }
    }
  }
  if (lane < np) atomicAdd(&load[lane], my_load);
  if (kLds) {
    for (int i = t; i < (n + 31) / 32; i += kLbBS) L.vis[i] = 0u;
    for (int i0 = 0; i0 <= n; i0 += 4 * kLbBS) {
      int o[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * kLbBS + t;
        o[u] = i <= n ? w.adj_off[b0 + i] - a0 : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * kLbBS + t;
        if (i <= n) off_l[i] = o[u];
      }
    }
    if (adj_lds)
      for (int i0 = 0; i0 < na; i0 += 8 * kLbBS) {
        int e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u * kLbBS + t;
          e[u] = i < na ? w.adj[a0 + i] : -1;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u * kLbBS + t;
          if (i < na) nb_l[i] = (uint16_t)(e[u] < 0 ? 0xFFFF : e[u] - b0);
        }
      }
  }
  __syncthreads();
  // Alg. 7 for every body of the scene
  for (int v = t; v < n; v += kLbBS) set_bridge(L, v, bridge_of(L, n, v));
  __syncthreads();

  if (t < 64) {
    // The contacts are read kLbChunks x 64 at a time (lane l holds contact
    // cb + 64 k + l in x[k]); a window runs from c to the end of its chunk.
    int2 x[kLbChunks];
    int cb = c0;
#pragma unroll
    for (int k = 0; k < kLbChunks; ++k) x[k] = contact_pair(w, cb + 64 * k + lane, c1, b0);
    int c = c0, changes = 0;
    while (c < c1) {
      if (c >= cb + 64 * kLbChunks) {
        cb += 64 * kLbChunks;
#pragma unroll
        for (int k = 0; k < kLbChunks; ++k) x[k] = contact_pair(w, cb + 64 * k + lane, c1, b0);
      }
      const int rel = c - cb, kc = rel >> 6, off = rel & 63;
      int2 xk = x[0];
#pragma unroll
      for (int k = 1; k < kLbChunks; ++k)
        if (k == kc) xk = x[k];
      const int src = off + lane;
      const int a = __shfl(xk.x, src & 63, 64), b = __shfl(xk.y, src & 63, 64);
      const bool live = src < 64 && a >= 0 && a < n && b >= 0 && b < n;
      const uint64_t fire = __ballot(live && rule_changes(L, a, b));
      if (fire == 0ull) {
        c += 64 - off;
        continue;
      }
      const int j = __builtin_ctzll(fire);
      apply_rule(L, load, &tail, n, w.lb_depth, __shfl(a, j, 64), __shfl(b, j, 64));
      c += j + 1;
      ++changes;
    }
    if (lane == 0 && changes) atomicAdd(&w.scal[SC_LB_CHANGES], changes);
  }
  __syncthreads();
  if (kLds)
    for (int i = t; i < n; i += kLbBS) w.mask[b0 + i] = L.m[i];
}

// after a committed step: its sets are carried
__global__ void k_lb_commit(WP w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < w.N && w.scal[SC_FLAGS] == 0) w.lb_mask[i] = w.mask[i];
}

}  // namespace

hipError_t lb_set_attributes() {
  return hipFuncSetAttribute((const void*)k_load_balance<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kLbLdsBytes);
}

hipError_t launch_balance(const WP& w, hipStream_t s) {
  if (w.N <= 0) return hipSuccess;
  k_lb_begin<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
  if (w.lb_lds_max > 0) k_load_balance<true><<<w.S, kLbBS, kLbLdsBytes, s>>>(w);
  if (w.lb_big) k_load_balance<false><<<w.S, kLbBS, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_balance_commit(const WP& w, hipStream_t s) {
  if (w.N <= 0) return hipSuccess;
  k_lb_commit<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
  return hipGetLastError();
}

}  // namespace ovl
