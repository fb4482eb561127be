// Device primitives: fills and a three-pass exclusive scan (tile reduce, scan of
// the tile sums in one workgroup, tile scan + carry).  wave64 shuffles do the
// in-wave scans; LDS carries the four wave totals of a 256-thread block.
#include "ovl_internal.h"
#include "wave.h"

namespace ovl {

namespace {

constexpr int kScanBS = 256;
constexpr int kScanIPT = 4;
constexpr int kScanTile = kScanBS * kScanIPT;

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(kScanBS) void k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                         int32_t* __restrict__ partial) {
  __shared__ int lds[kScanBS / 64];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanIPT;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanIPT; ++k)
    if (base + k < n) s += in[base + k];
  int tot = block_sum<kScanBS>(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBS) void k_scan_partials(int32_t* __restrict__ partial, int nblk,
                                                           int32_t* __restrict__ out_total_slot,
                                                           int32_t* __restrict__ total) {
  __shared__ int lds[kScanBS / 64];
  int carry = 0;
  for (int base = 0; base < nblk; base += kScanTile) {
    int v[kScanIPT];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanIPT; ++k) {
      int i = base + threadIdx.x * kScanIPT + k;
      v[k] = i < nblk ? partial[i] : 0;
      s += v[k];
    }
    int tile_total;
    int pre = block_excl_scan<kScanBS>(s, lds, tile_total);
    int run = carry + pre;
#pragma unroll
    for (int k = 0; k < kScanIPT; ++k) {
      int i = base + threadIdx.x * kScanIPT + k;
      if (i < nblk) partial[i] = run;
      run += v[k];
    }
    carry += tile_total;
  }
  if (threadIdx.x == 0) {
    *out_total_slot = carry;
    if (total) *total = carry;
  }
}

__global__ __launch_bounds__(kScanBS) void k_scan_apply(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                        int64_t n, const int32_t* __restrict__ partial) {
  __shared__ int lds[kScanBS / 64];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanIPT;
  int v[kScanIPT];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanIPT; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  int tile_total;
  int run = partial[blockIdx.x] + block_excl_scan<kScanBS>(s, lds, tile_total);
#pragma unroll
  for (int k = 0; k < kScanIPT; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

__global__ void k_scan_empty(int32_t* out, int32_t* total) {
  out[0] = 0;
  if (total) *total = 0;
}

}  // namespace

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int g = nblocks(n, kBlock);
  if (g > 4096) g = 4096;
  k_fill_i32<<<g, kBlock, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int g = nblocks(n, kBlock);
  if (g > 4096) g = 4096;
  k_fill_u64<<<g, kBlock, 0, s>>>(p, v, n);
  return hipGetLastError();
}

size_t scan_scratch_ints(int64_t n) { return (size_t)nblocks(n, kScanTile) + 1; }

hipError_t scan_excl(const int32_t* in, int32_t* out, int64_t n, int32_t* total, int32_t* scratch, hipStream_t s) {
  if (n <= 0) {
    k_scan_empty<<<1, 1, 0, s>>>(out, total);
    return hipGetLastError();
  }
  int nblk = nblocks(n, kScanTile);
  k_scan_reduce<<<nblk, kScanBS, 0, s>>>(in, n, scratch);
  k_scan_partials<<<1, kScanBS, 0, s>>>(scratch, nblk, out + n, total);
  k_scan_apply<<<nblk, kScanBS, 0, s>>>(in, out, n, scratch);
  return hipGetLastError();
}

}  // namespace ovl
