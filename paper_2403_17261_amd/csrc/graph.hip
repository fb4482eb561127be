// Constraint graph, overlap sets, replica table, geodesic distances and the
// per-partition constraint lists of a step.
//
//  * Constraint graph (section 5.1): vertices are the non-static bodies; an
//    edge joins two bodies that share a joint or a contact.  Built as CSR:
//    degrees (joints, then contacts by atomics), scan, fill, then each
//    vertex's list sorted and de-duplicated (slots freed by duplicates hold
//    -1).  Only the set of neighbours matters to the consumers below.
//  * Overlap sets (section 4, Eq. 9-10; Alg. 2-3 read as a k-hop halo): a
//    64-bit mask of local partition bits per body, seeded with the owner bit
//    and widened by k rounds of "OR of the neighbours' masks".  A body with
//    two or more bits is in the overlap set O.
//  * Replica table: body-major slots (scan of the popcounts), plus a stable
//    partition-major order (bodies ascending inside each partition) built by
//    a masked compaction: per-256-item block and bit counts, a column scan
//    over blocks, the rank of every scene's first item per bit, and a scatter
//    that ranks items inside a block with wave64 ballots.
//  * Geodesic distances (section 5.3, Eq. 16, Alg. 5): a multi-source BFS in
//    beta rounds starting from the bodies that are active in one partition
//    only; the round in which partition i's bit first reaches an overlap body
//    o is D(o, i).
//  * Constraint copies: partition p solves every joint and contact whose
//    non-static bodies are all active in p.  The same masked compaction lists
//    them per partition in uid order: joints by index, then contacts by key.
#include "ovl_internal.h"
#include "wave.h"

namespace ovl {

namespace {

__device__ __forceinline__ int clampi(int x, int hi) { return x < hi ? x : hi; }
__device__ __forceinline__ int n_contacts(const WP& w) { return clampi(w.scal[SC_NCONTACT], w.Ccap); }
__device__ __forceinline__ bool adj_ok(const WP& w) { return w.adj_off[w.N] <= w.Acap; }
__device__ __forceinline__ bool rep_ok(const WP& w) { return w.rep_off_bm[w.N] <= w.Rcap; }

// ---------------------------------------------------------------- graph ----

__global__ void k_deg_init(WP w) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < w.N) w.deg[v] = w.jadj_off[v + 1] - w.jadj_off[v];
}

__global__ void k_deg_contacts(WP w) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_contacts(w)) return;
  uint32_t b = w.c_bkey[c] >> 1;
  if (b < (uint32_t)w.N) {
    atomicAdd(&w.deg[w.c_a[c]], 1);
    atomicAdd(&w.deg[b], 1);
  }
}

__global__ void k_adj_joints(WP w) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N) return;
  if (!adj_ok(w)) {
    if (v == 0) atomicOr(&w.scal[SC_FLAGS], F_ADJ_CAP);
    return;
  }
  int o = w.adj_off[v];
  int j0 = w.jadj_off[v], j1 = w.jadj_off[v + 1];
  for (int k = j0; k < j1; ++k) w.adj[o + k - j0] = w.jadj[k];
  w.adj_fill[v] = j1 - j0;
}

__global__ void k_adj_contacts(WP w) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_contacts(w) || !adj_ok(w)) return;
  uint32_t b = w.c_bkey[c] >> 1;
  if (b < (uint32_t)w.N) {
    int a = w.c_a[c];
    w.adj[w.adj_off[a] + atomicAdd(&w.adj_fill[a], 1)] = (int)b;
    w.adj[w.adj_off[b] + atomicAdd(&w.adj_fill[b], 1)] = a;
  }
}

__global__ void k_adj_sort(WP w) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N || !adj_ok(w)) return;
  int o0 = w.adj_off[v], o1 = w.adj_off[v + 1];
  for (int i = o0 + 1; i < o1; ++i) {
    int k = w.adj[i];
    int j = i - 1;
    while (j >= o0 && w.adj[j] > k) {
      w.adj[j + 1] = w.adj[j];
      --j;
    }
    w.adj[j + 1] = k;
  }
  int u = o0;
  for (int i = o0; i < o1; ++i)
    if (i == o0 || w.adj[i] != w.adj[u - 1]) w.adj[u++] = w.adj[i];
  for (int i = u; i < o1; ++i) w.adj[i] = -1;
}

// ------------------------------------------------------- overlap masks ----

__global__ void k_mask_init(WP w) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < w.N) w.mask[v] = 1ull << w.owner_local[v];
}

// dst[v] = src[v] | OR of src over the neighbours of v
__device__ __forceinline__ uint64_t or_neighbours(const WP& w, const uint64_t* src, int v) {
  uint64_t m = src[v];
  if (adj_ok(w)) {
    const int o1 = w.adj_off[v + 1];
    for (int k = w.adj_off[v]; k < o1; ++k) {
      int u = w.adj[k];
      if (u >= 0) m |= src[u];
    }
  }
  return m;
}

__global__ void k_or_round(WP w, const uint64_t* __restrict__ src, uint64_t* __restrict__ dst) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < w.N) dst[v] = or_neighbours(w, src, v);
}

__global__ void k_copy_u64(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, int n) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) dst[v] = src[v];
}

__global__ void k_rep_count(WP w) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N) return;
  int c = __popcll(w.mask[v]);
  w.rep_cnt[v] = c;
  if (c >= 2) atomicAdd(&w.scal[SC_NOVERLAP], 1);
}

// ------------------------------------------------- geodesic distances ----

__global__ void k_reach_init(WP w) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N) return;
  uint64_t m = w.mask[v];
  w.reach[v] = __popcll(m) == 1 ? m : 0ull;
}

__global__ void k_reach_round(WP w, const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, int round) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= w.N) return;
  uint64_t m = or_neighbours(w, src, v);
  dst[v] = m;
  uint64_t mv = w.mask[v];
  if (__popcll(mv) < 2 || !rep_ok(w)) return;
  uint64_t fresh = m & mv & ~src[v];
  const int base = w.rep_off_bm[v];
  while (fresh) {
    int b = __ffsll((unsigned long long)fresh) - 1;
    fresh &= fresh - 1;
    w.rep_D_bm[base + __popcll(mv & ((1ull << b) - 1ull))] = round;
  }
}

// -------------------------------------------------- masked compaction ----
// Items with a mask of local partition bits are listed per global partition
// (scene base + bit), stably (item order inside each partition).  Items are
// sorted by scene.

constexpr int kMcBS = 256;

struct BodyItems {
  static constexpr int set = 0;
  __device__ static int count(const WP& w) { return w.N; }
  __device__ static int scene_start(const WP& w, int s) { return w.s_body_off[s]; }
  __device__ static void get(const WP& w, int i, uint64_t& m, int& s) {
    m = w.mask[i];
    s = w.b_scene[i];
  }
  __device__ static void put(const WP& w, int i, uint64_t m, int bit, int g, int pos) {
    const int slot = w.rep_off_bm[i] + __popcll(m & ((1ull << bit) - 1ull));
    if (pos >= w.Rcap || slot >= w.Rcap) return;
    w.rep_body_pm[pos] = i;
    w.rep_pm_of_bm[slot] = pos;
  }
};

// local replica index of body v in global partition g (local bit `bit`)
__device__ __forceinline__ int local_rep(const WP& w, int v, int bit, int g) {
  uint64_t mv = w.mask[v];
  return w.rep_pm_of_bm[w.rep_off_bm[v] + __popcll(mv & ((1ull << bit) - 1ull))] - w.part_rep_off[g];
}

struct JointItems {
  static constexpr int set = 1;
  __device__ static int count(const WP& w) { return w.J; }
  __device__ static int scene_start(const WP& w, int s) { return w.s_joint_off[s]; }
  __device__ static void get(const WP& w, int i, uint64_t& m, int& s) {
    int a = w.j_ab[2 * i], b = w.j_ab[2 * i + 1];
    m = w.mask[a] & w.mask[b];
    s = w.b_scene[a];
  }
  __device__ static void put(const WP& w, int i, uint64_t, int bit, int g, int pos) {
    if (pos >= w.Mcap || !rep_ok(w)) return;
    int a = w.j_ab[2 * i], b = w.j_ab[2 * i + 1];
    w.cp_src[pos] = i;
    w.cp_part[pos] = g;
    w.cp_ia[pos] = local_rep(w, a, bit, g);
    w.cp_ib[pos] = local_rep(w, b, bit, g);
  }
};

struct ContactItems {
  static constexpr int set = 2;
  __device__ static int count(const WP& w) { return n_contacts(w); }
  __device__ static int scene_start(const WP& w, int s) { return clampi(w.coff[w.s_body_off[s]], n_contacts(w)); }
  __device__ static void get(const WP& w, int i, uint64_t& m, int& s) {
    int a = w.c_a[i];
    uint32_t b = w.c_bkey[i] >> 1;
    m = w.mask[a] & (b < (uint32_t)w.N ? w.mask[b] : ~0ull);
    s = w.b_scene[a];
  }
  __device__ static void put(const WP& w, int i, uint64_t, int bit, int g, int pos) {
    if (pos >= w.Mcap || !rep_ok(w)) return;
    int a = w.c_a[i];
    uint32_t b = w.c_bkey[i] >> 1;
    w.cp_src[pos] = w.J + i;
    w.cp_part[pos] = g;
    w.cp_ia[pos] = local_rep(w, a, bit, g);
    w.cp_ib[pos] = b < (uint32_t)w.N ? local_rep(w, (int)b, bit, g) : -1;
  }
};

template <class I>
__global__ __launch_bounds__(kMcBS) void k_mc_count(WP w) {
  __shared__ int cnt[64];
  if (threadIdx.x < 64) cnt[threadIdx.x] = 0;
  __syncthreads();
  int i = blockIdx.x * kMcBS + threadIdx.x;
  if (i < I::count(w)) {
    uint64_t m;
    int s;
    I::get(w, i, m, s);
    while (m) {
      atomicAdd(&cnt[__ffsll((unsigned long long)m) - 1], 1);
      m &= m - 1;
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) w.mc_blk[I::set][blockIdx.x * 64 + threadIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of every bit column over the blocks; row nblk gets the totals
__global__ __launch_bounds__(kMcBS) void k_mc_colscan(int32_t* blk, int nblk) {
  __shared__ int lds[kMcBS / 64];
  const int bit = blockIdx.x;
  int carry = 0;
  for (int base = 0; base < nblk; base += kMcBS) {
    int i = base + threadIdx.x;
    int v = i < nblk ? blk[i * 64 + bit] : 0;
    int tot;
    int pre = block_excl_scan<kMcBS>(v, lds, tot);
    if (i < nblk) blk[i * 64 + bit] = carry + pre;
    carry += tot;
  }
  if (threadIdx.x == 0) blk[nblk * 64 + bit] = carry;
}

// rank (count of earlier items with the bit) of every scene's first item, and of the end
template <class I>
__global__ void k_mc_rank0(WP w) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (w.S + 1) * 64) return;
  int s = t >> 6, bit = t & 63;
  int n = I::count(w);
  int start = s == w.S ? n : clampi(I::scene_start(w, s), n);
  int blk = start / kMcBS;
  int r = w.mc_blk[I::set][blk * 64 + bit];
  for (int i = blk * kMcBS; i < start; ++i) {
    uint64_t m;
    int sc;
    I::get(w, i, m, sc);
    r += (int)((m >> bit) & 1ull);
  }
  w.mc_rank0[I::set][t] = r;
}

__global__ void k_mc_psize(WP w, int set) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= w.G) return;
  int s = w.part_scene[g], b = w.part_bit[g];
  w.mc_psize[set][g] = w.mc_rank0[set][(s + 1) * 64 + b] - w.mc_rank0[set][s * 64 + b];
}

template <class I>
__global__ __launch_bounds__(kMcBS) void k_mc_scatter(WP w, const int32_t* __restrict__ base0,
                                                      const int32_t* __restrict__ base1) {
  __shared__ unsigned long long bor;
  __shared__ int wcnt[kMcBS / 64][64];
  const int i = blockIdx.x * kMcBS + threadIdx.x;
  const int wave = threadIdx.x >> 6;
  uint64_t m = 0;
  int s = 0;
  if (i < I::count(w)) I::get(w, i, m, s);
  if (threadIdx.x == 0) bor = 0ull;
  __syncthreads();
  if (m) atomicOr(&bor, (unsigned long long)m);
  __syncthreads();
  const uint64_t B = bor;
  for (uint64_t bb = B; bb; bb &= bb - 1) {
    int b = __ffsll((unsigned long long)bb) - 1;
    uint64_t bal = ballot64((m >> b) & 1ull);
    if (lane_id() == 0) wcnt[wave][b] = __popcll(bal);
  }
  __syncthreads();
  const int* blkpre = w.mc_blk[I::set] + blockIdx.x * 64;
  for (uint64_t bb = B; bb; bb &= bb - 1) {
    int b = __ffsll((unsigned long long)bb) - 1;
    uint64_t bal = ballot64((m >> b) & 1ull);
    if ((m >> b) & 1ull) {
      int pre = 0;
      for (int k = 0; k < wave; ++k) pre += wcnt[k][b];
      int rank = blkpre[b] + pre + __popcll(bal & lanemask_lt()) - w.mc_rank0[I::set][s * 64 + b];
      int g = w.s_part_base[s] + b;
      int pos = base0[g] + (base1 ? base1[g] : 0) + rank;
      I::put(w, i, m, b, g, pos);
    }
  }
}

__global__ void k_sum2(const int32_t* a, const int32_t* b, int32_t* out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

__global__ void k_check_reps(WP w) {
  if (threadIdx.x || blockIdx.x) return;
  if (w.rep_off_bm[w.N] > w.Rcap) atomicOr(&w.scal[SC_FLAGS], F_REP_CAP);
}

__global__ __launch_bounds__(1024) void k_check_copies(WP w) {
  __shared__ int red[16];
  int nj = 0;
  for (int g = threadIdx.x; g < w.G; g += 1024) nj += w.mc_psize[1][g];
  nj = block_sum<1024>(nj, red);
  if (threadIdx.x == 0) {
    if (w.part_copy_off[w.G] > w.Mcap) atomicOr(&w.scal[SC_FLAGS], F_COPY_CAP);
    w.scal[SC_NJCOPY] = nj;
    w.scal[SC_NCCOPY] = w.part_copy_off[w.G] - nj;
  }
}

__global__ void k_zero_scal(WP w) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    w.scal[SC_NOVERLAP] = 0;
    w.scal[SC_LB_CHANGES] = 0;
  }
}

template <class I>
hipError_t mc_count(const WP& w, int nitems_cap, hipStream_t s, int32_t* scan_scratch) {
  int nblk = nblocks(nitems_cap, kMcBS);
  if (nblk > 0) k_mc_count<I><<<nblk, kMcBS, 0, s>>>(w);
  k_mc_colscan<<<64, kMcBS, 0, s>>>(w.mc_blk[I::set], nblk);
  k_mc_rank0<I><<<nblocks((w.S + 1) * 64, 128), 128, 0, s>>>(w);
  if (w.G > 0) k_mc_psize<<<nblocks(w.G, 128), 128, 0, s>>>(w, I::set);
  (void)scan_scratch;
  return hipGetLastError();
}

template <class I>
hipError_t mc_scatter(const WP& w, int nitems_cap, const int32_t* base0, const int32_t* base1, hipStream_t s) {
  int nblk = nblocks(nitems_cap, kMcBS);
  if (nblk > 0) k_mc_scatter<I><<<nblk, kMcBS, 0, s>>>(w, base0, base1);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_graph(const WP& w, int32_t* sc, hipStream_t s) {
  hipError_t e;
  const int nb = nblocks(w.N, kBlock);
  const int ncb = nblocks(w.Ccap, kBlock);
  k_zero_scal<<<1, 1, 0, s>>>(w);
  // constraint graph CSR
  if (w.N > 0) k_deg_init<<<nb, kBlock, 0, s>>>(w);
  if (w.Ccap > 0) k_deg_contacts<<<ncb, kBlock, 0, s>>>(w);
  if ((e = hipGetLastError())) return e;
  if ((e = scan_excl(w.deg, w.adj_off, w.N, &w.scal[SC_NADJ], sc, s))) return e;
  if (w.N > 0) {
    k_adj_joints<<<nb, kBlock, 0, s>>>(w);
    if (w.Ccap > 0) k_adj_contacts<<<ncb, kBlock, 0, s>>>(w);
    k_adj_sort<<<nb, kBlock, 0, s>>>(w);
    if (w.lb_on) {
      // worker sets carried from the last step, updated from this step's contacts
      if ((e = launch_balance(w, s))) return e;
    } else {
      // overlap masks: k rounds of neighbour OR
      k_mask_init<<<nb, kBlock, 0, s>>>(w);
      uint64_t* a = w.mask;
      uint64_t* b = w.mask_tmp;
      for (int r = 0; r < w.halo_k; ++r) {
        k_or_round<<<nb, kBlock, 0, s>>>(w, a, b);
        uint64_t* t = a;
        a = b;
        b = t;
      }
      if (a != w.mask) k_copy_u64<<<nb, kBlock, 0, s>>>(a, w.mask, w.N);
    }
    k_rep_count<<<nb, kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  // replica table
  if ((e = scan_excl(w.rep_cnt, w.rep_off_bm, w.N, &w.scal[SC_NREP], sc, s))) return e;
  if ((e = mc_count<BodyItems>(w, w.N, s, sc))) return e;
  if ((e = scan_excl(w.mc_psize[0], w.part_rep_off, w.G, nullptr, sc, s))) return e;
  k_check_reps<<<1, 1, 0, s>>>(w);
  if ((e = mc_scatter<BodyItems>(w, w.N, w.part_rep_off, nullptr, s))) return e;
  // geodesic distances: beta rounds of a multi-source BFS from the single-partition bodies
  if ((e = fill_i32(w.rep_D_bm, 0, w.Rcap, s))) return e;
  if (w.N > 0) {
    k_reach_init<<<nb, kBlock, 0, s>>>(w);
    uint64_t* a = w.reach;
    uint64_t* b = w.reach_tmp;
    for (int r = 1; r <= w.beta; ++r) {
      k_reach_round<<<nb, kBlock, 0, s>>>(w, a, b, r);
      uint64_t* t = a;
      a = b;
      b = t;
    }
    if ((e = hipGetLastError())) return e;
  }
  // constraint copies: joints then contacts per partition
  if ((e = mc_count<JointItems>(w, w.J, s, sc))) return e;
  if ((e = mc_count<ContactItems>(w, w.Ccap, s, sc))) return e;
  if (w.G > 0) k_sum2<<<nblocks(w.G, kBlock), kBlock, 0, s>>>(w.mc_psize[1], w.mc_psize[2], w.g_tmp, w.G);
  if ((e = scan_excl(w.g_tmp, w.part_copy_off, w.G, &w.scal[SC_NCOPY], sc, s))) return e;
  k_check_copies<<<1, 1024, 0, s>>>(w);
  if ((e = mc_scatter<JointItems>(w, w.J, w.part_copy_off, nullptr, s))) return e;
  if ((e = mc_scatter<ContactItems>(w, w.Ccap, w.part_copy_off, w.mc_psize[1], s))) return e;
  return hipGetLastError();
}

}  // namespace ovl
