// Learned warm start: a 12 -> 64 -> 64 -> 3 ReLU network that predicts a
// contact's impulses (normalised by the impulse scale s) from twelve features
// of the problem at the start of the step.
//
//  * Training (FP32, deterministic): k_mlp_grad runs forward and backward for
//    a block of 128 samples with weights and activations in LDS and writes
//    the block's gradient; k_mlp_adam sums the block gradients in a fixed
//    order and applies Adam.  No floating-point atomics.
//  * Inference (BF16 matrix cores, FP32 accumulation): one wave evaluates 16
//    contacts with v_mfma_f32_16x16x16_bf16 tiles, the weights held in its
//    registers; activations pass through the wave's LDS between layers
//    (bfloat16).  The world-side kernel writes the projected prediction into
//    the learned-start slot of every contact copy.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ovl.h"
#include "ovl_internal.h"
#include "wave.h"

namespace ovl {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// bfloat16 of a float, round to nearest, ties to even (NaN/Inf kept)
__host__ __device__ inline uint16_t to_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Device copy of a network for the matrix engine: bfloat16 weights padded to
// 16-wide tiles (W1 [16][64], W2 [64][64], W3 [64][16]) and float biases.
void mlp_pack(const float* P, std::vector<uint16_t>& wb, std::vector<float>& bias) {
  const float* W1 = P;
  const float* b1 = W1 + kMlpIn * kMlpHid;
  const float* W2 = b1 + kMlpHid;
  const float* b2 = W2 + kMlpHid * kMlpHid;
  const float* W3 = b2 + kMlpHid;
  const float* b3 = W3 + kMlpHid * kMlpOut;
  wb.assign(kMlpWb, 0);
  for (int k = 0; k < kMlpIn; ++k)
    for (int j = 0; j < kMlpHid; ++j) wb[k * 64 + j] = to_bf16(W1[k * kMlpHid + j]);
  for (int k = 0; k < 64; ++k)
    for (int j = 0; j < 64; ++j) wb[1024 + k * 64 + j] = to_bf16(W2[k * kMlpHid + j]);
  for (int k = 0; k < 64; ++k)
    for (int o = 0; o < kMlpOut; ++o) wb[1024 + 4096 + k * 16 + o] = to_bf16(W3[k * kMlpOut + o]);
  bias.assign(kMlpBias, 0.0f);
  for (int j = 0; j < 64; ++j) {
    bias[j] = b1[j];
    bias[64 + j] = b2[j];
  }
  for (int o = 0; o < kMlpOut; ++o) bias[128 + o] = b3[o];
}

namespace {

constexpr int kInfBS = 256;  // 4 waves, 16 rows each

// Operand layout of the 16x16x16 bf16 instruction: lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16], j = 0..3.
//
// A lane's share of the packed network as matrix-core operands: its B
// fragments of the three layers and the biases of its output columns, read
// once and kept in registers for every tile the wave evaluates.
struct MlpLane {
  bf16x4 w1[4], w2[4][4], w3[4];
  float b1[4], b2[4], b3;
};

__device__ __forceinline__ void mlp_lane_load(MlpLane& n, const uint16_t* wb, const float* bias) {
  const int l = lane_id();
  const int row = l & 15, q = l >> 4;
  for (int t = 0; t < 4; ++t) {
    for (int j = 0; j < 4; ++j) n.w1[t][j] = (short)wb[(4 * q + j) * 64 + 16 * t + row];
    n.b1[t] = bias[16 * t + row];
    n.b2[t] = bias[64 + 16 * t + row];
  }
  for (int ks = 0; ks < 4; ++ks)
    for (int t = 0; t < 4; ++t)
      for (int j = 0; j < 4; ++j) n.w2[ks][t][j] = (short)wb[1024 + (16 * ks + 4 * q + j) * 64 + 16 * t + row];
  for (int ks = 0; ks < 4; ++ks)
    for (int j = 0; j < 4; ++j) n.w3[ks][j] = (short)wb[1024 + 4096 + (16 * ks + 4 * q + j) * 16 + row];
  n.b3 = bias[128 + row];
}

// the LDS written by this wave is complete and visible to its other lanes
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Evaluate 16 rows with the network in registers.  `a` is the lane's A
// operand of the first layer: row l%16, features 4(l/16) .. +3 as bfloat16
// (zero-padded to 16).  h1, h2 ([16][64] bfloat16) and y ([16][4] float, the
// three outputs of each row) are this wave's LDS.  Only the wave takes part.
__device__ void mlp_rows(const MlpLane& n, bf16x4 a, uint16_t* h1, uint16_t* h2, float* y) {
  const int l = lane_id();
  const int row = l & 15, q = l >> 4;
  // layer 1: [16 x 16] x [16 x 64]
  for (int t = 0; t < 4; ++t) {
    f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, n.w1[t], c, 0, 0, 0);
    const int col = 16 * t + row;
    for (int j = 0; j < 4; ++j) h1[(4 * q + j) * 64 + col] = to_bf16(fmaxf(c[j] + n.b1[t], 0.0f));
  }
  wave_lds_sync();
  // layer 2: [16 x 64] x [64 x 64]
  f32x4 acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int ks = 0; ks < 4; ++ks) {
    bf16x4 a2;
    for (int j = 0; j < 4; ++j) a2[j] = (short)h1[row * 64 + 16 * ks + 4 * q + j];
    for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, n.w2[ks][t], acc[t], 0, 0, 0);
  }
  for (int t = 0; t < 4; ++t) {
    const int col = 16 * t + row;
    for (int j = 0; j < 4; ++j) h2[(4 * q + j) * 64 + col] = to_bf16(fmaxf(acc[t][j] + n.b2[t], 0.0f));
  }
  wave_lds_sync();
  // layer 3: [16 x 64] x [64 x 16] (3 outputs used)
  f32x4 o = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int ks = 0; ks < 4; ++ks) {
    bf16x4 a3;
    for (int j = 0; j < 4; ++j) a3[j] = (short)h2[row * 64 + 16 * ks + 4 * q + j];
    o = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, n.w3[ks], o, 0, 0, 0);
  }
  if (row < kMlpOut)
    for (int j = 0; j < 4; ++j) y[(4 * q + j) * 4 + row] = o[j] + n.b3;
  wave_lds_sync();
}

struct InferLds {
  uint16_t wb[kMlpWb];
  float bias[kMlpBias];
  uint16_t h1[4][16 * 64];
  uint16_t h2[4][16 * 64];
  float y[4][16 * 4];
};

// the packed network into LDS (whole workgroup, then a barrier)
__device__ void load_net(InferLds& s, const uint16_t* wb, const float* bias) {
  for (int i = threadIdx.x; i < kMlpWb; i += kInfBS) s.wb[i] = wb[i];
  for (int i = threadIdx.x; i < kMlpBias; i += kInfBS) s.bias[i] = bias[i];
  __syncthreads();
}

// A operand of the first layer for row i of a [n][stride] float feature matrix
__device__ __forceinline__ bf16x4 mlp_input(const float* X, int64_t stride, int i, int n) {
  const int q = lane_id() >> 4;
  bf16x4 a;
  for (int j = 0; j < 4; ++j) {
    const int k = 4 * q + j;
    a[j] = (short)((i < n && k < kMlpIn) ? to_bf16(X[(int64_t)i * stride + k]) : 0);
  }
  return a;
}

// standalone inference: X [n][12] float -> Y [n][3] float
__global__ __launch_bounds__(kInfBS) void k_mlp_infer(const uint16_t* __restrict__ wb, const float* __restrict__ bias,
                                                      const float* __restrict__ X, int n, float* __restrict__ Y) {
  __shared__ InferLds s;
  load_net(s, wb, bias);
  const int wv = threadIdx.x >> 6, l = lane_id();
  const int base = (blockIdx.x * 4 + wv) * 16;
  MlpLane net;
  mlp_lane_load(net, s.wb, s.bias);
  mlp_rows(net, mlp_input(X, kMlpIn, base + (l & 15), n), s.h1[wv], s.h2[wv], s.y[wv]);
  if (l < 16 && base + l < n)
    for (int o = 0; o < kMlpOut; ++o) Y[(int64_t)(base + l) * kMlpOut + o] = s.y[wv][l * 4 + o];
}

// world: learned start of every contact copy (uid order in, slot order out).
// A persistent grid: every workgroup stages the network in LDS once, each of
// its waves takes the network into registers and then evaluates tiles of 16
// copies with a grid stride, on its own (no workgroup barrier in the loop).
constexpr int kInfWorldBlocks = 1024;

__global__ __launch_bounds__(kInfBS) void k_mlp_world(WP w) {
  __shared__ InferLds s;
  if (w.scal[SC_FLAGS] != 0) return;
  const int M = min(w.part_copy_off[w.G], w.Mcap);
  if (blockIdx.x * 64 >= M) return;
  load_net(s, w.mlp_wb, w.mlp_bias);
  const int wv = threadIdx.x >> 6, l = lane_id();
  MlpLane net;
  mlp_lane_load(net, s.wb, s.bias);
  for (int tile = blockIdx.x * 4 + wv; tile * 16 < M; tile += gridDim.x * 4) {
    const int base = tile * 16;
    // the copy of lane l < 16: its slot and impulse scale, loaded ahead of the rows
    int slot = -1;
    float sc = 0.0f;
    const int u = base + l;
    if (l < 16 && u < M && w.cp_src[u] >= w.J) {
      slot = w.cp_slot[u];
      sc = w.r_feat[(int64_t)u * kFeatStride + 12];
    }
    mlp_rows(net, mlp_input(w.r_feat, kFeatStride, base + (l & 15), M), s.h1[wv], s.h2[wv], s.y[wv]);
    if (slot >= 0) {
      const float mu = w.r_rec[w.Mcap + slot].w;
      const float ln = fmaxf(s.y[wv][l * 4] * sc, 0.0f);
      const float bnd = mu * ln;
      const float l1 = fminf(fmaxf(s.y[wv][l * 4 + 1] * sc, -bnd), bnd);
      const float l2 = fminf(fmaxf(s.y[wv][l * 4 + 2] * sc, -bnd), bnd);
      w.r_lamL[slot] = make_float4(ln, l1, l2, 0.0f);
    }
    wave_lds_sync();  // y is rewritten by the next tile
  }
}

// ------------------------------------------------------------ training ----

constexpr int kTrBS = 256;
constexpr int kTrRows = 128;

struct TrainLds {
  float P[kMlpParams];
  float X[kTrRows * kMlpIn];
  float H1[kTrRows * kMlpHid];
  float H2[kTrRows * kMlpHid];
  float D[kTrRows * kMlpHid];
  float DY[kTrRows * kMlpOut];
  float red[kTrBS / 64];
};

// Forward and backward of one block of up to 128 samples; writes the block's
// summed gradient (of the mean squared error over n_total samples) and its
// summed squared error.
__global__ __launch_bounds__(kTrBS) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ X,
                                                    const float* __restrict__ T, int n, float* __restrict__ gpart,
                                                    float* __restrict__ lpart) {
  extern __shared__ float smem[];
  TrainLds& s = *reinterpret_cast<TrainLds*>(smem);
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * kTrRows;
  const int nr = min(kTrRows, n - r0);
  const float* W1 = s.P;
  const float* b1 = W1 + kMlpIn * kMlpHid;
  const float* W2 = b1 + kMlpHid;
  const float* b2 = W2 + kMlpHid * kMlpHid;
  const float* W3 = b2 + kMlpHid;
  const float* b3 = W3 + kMlpHid * kMlpOut;
  for (int i = tid; i < kMlpParams; i += kTrBS) s.P[i] = params[i];
  for (int i = tid; i < kTrRows * kMlpIn; i += kTrBS) {
    const int r = i / kMlpIn;
    s.X[i] = r < nr ? X[(int64_t)(r0 + r) * kMlpIn + i % kMlpIn] : 0.0f;
  }
  __syncthreads();
  for (int i = tid; i < kTrRows * kMlpHid; i += kTrBS) {
    const int r = i / kMlpHid, j = i % kMlpHid;
    float a = b1[j];
    for (int k = 0; k < kMlpIn; ++k) a += s.X[r * kMlpIn + k] * W1[k * kMlpHid + j];
    s.H1[i] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  for (int i = tid; i < kTrRows * kMlpHid; i += kTrBS) {
    const int r = i / kMlpHid, j = i % kMlpHid;
    float a = b2[j];
    for (int k = 0; k < kMlpHid; ++k) a += s.H1[r * kMlpHid + k] * W2[k * kMlpHid + j];
    s.H2[i] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  const float scale = 2.0f / ((float)n * kMlpOut);
  float se = 0.0f;
  for (int i = tid; i < kTrRows * kMlpOut; i += kTrBS) {
    const int r = i / kMlpOut, o = i % kMlpOut;
    float a = b3[o];
    for (int k = 0; k < kMlpHid; ++k) a += s.H2[r * kMlpHid + k] * W3[k * kMlpOut + o];
    float d = 0.0f;
    if (r < nr) {
      d = a - T[(int64_t)(r0 + r) * kMlpOut + o];
      se += d * d;
    }
    s.DY[i] = scale * d;
  }
  __syncthreads();
  float* g = gpart + (int64_t)blockIdx.x * kMlpParams;
  float* gW1 = g;
  float* gb1 = gW1 + kMlpIn * kMlpHid;
  float* gW2 = gb1 + kMlpHid;
  float* gb2 = gW2 + kMlpHid * kMlpHid;
  float* gW3 = gb2 + kMlpHid;
  float* gb3 = gW3 + kMlpHid * kMlpOut;
  // layer 3 gradients and dH2
  for (int i = tid; i < kMlpHid * kMlpOut; i += kTrBS) {
    const int j = i / kMlpOut, o = i % kMlpOut;
    float a = 0.0f;
    for (int r = 0; r < kTrRows; ++r) a += s.H2[r * kMlpHid + j] * s.DY[r * kMlpOut + o];
    gW3[i] = a;
  }
  if (tid < kMlpOut) {
    float a = 0.0f;
    for (int r = 0; r < kTrRows; ++r) a += s.DY[r * kMlpOut + tid];
    gb3[tid] = a;
  }
  for (int i = tid; i < kTrRows * kMlpHid; i += kTrBS) {
    const int r = i / kMlpHid, j = i % kMlpHid;
    float a = 0.0f;
    for (int o = 0; o < kMlpOut; ++o) a += s.DY[r * kMlpOut + o] * W3[j * kMlpOut + o];
    s.D[i] = s.H2[i] > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  // layer 2 gradients, then dH1 (stored over H2)
  for (int i = tid; i < kMlpHid * kMlpHid; i += kTrBS) {
    const int k = i / kMlpHid, j = i % kMlpHid;
    float a = 0.0f;
    for (int r = 0; r < kTrRows; ++r) a += s.H1[r * kMlpHid + k] * s.D[r * kMlpHid + j];
    gW2[i] = a;
  }
  if (tid < kMlpHid) {
    float a = 0.0f;
    for (int r = 0; r < kTrRows; ++r) a += s.D[r * kMlpHid + tid];
    gb2[tid] = a;
  }
  __syncthreads();
  for (int i = tid; i < kTrRows * kMlpHid; i += kTrBS) {
    const int r = i / kMlpHid, k = i % kMlpHid;
    float a = 0.0f;
    for (int j = 0; j < kMlpHid; ++j) a += s.D[r * kMlpHid + j] * W2[k * kMlpHid + j];
    s.H2[i] = s.H1[i] > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  for (int i = tid; i < kMlpIn * kMlpHid; i += kTrBS) {
    const int k = i / kMlpHid, j = i % kMlpHid;
    float a = 0.0f;
    for (int r = 0; r < kTrRows; ++r) a += s.X[r * kMlpIn + k] * s.H2[r * kMlpHid + j];
    gW1[i] = a;
  }
  if (tid < kMlpHid) {
    float a = 0.0f;
    for (int r = 0; r < kTrRows; ++r) a += s.H2[r * kMlpHid + tid];
    gb1[tid] = a;
  }
  se = wave_sum_f(se);
  if (lane_id() == 0) s.red[tid >> 6] = se;
  __syncthreads();
  if (tid == 0) lpart[blockIdx.x] = s.red[0] + s.red[1] + s.red[2] + s.red[3];
}

// Sum of the block gradients in block order; with update != 0 an Adam step.
__global__ void k_mlp_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ gpart, int nblk, float* __restrict__ grad_out, int update,
                           float lr, float b1, float b2, float c1, float c2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += gpart[(int64_t)b * kMlpParams + i];
  if (grad_out) grad_out[i] = g;
  if (!update) return;
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// The mean squared error of a batch from the blocks' summed squared errors:
// summed in block order in double and divided by the element count, the same
// arithmetic as the host does for the trainer's gradient.
__global__ void k_mlp_loss(const float* __restrict__ lpart, int nblk, int64_t n, float* __restrict__ loss) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double sse = 0.0;
  for (int b = 0; b < nblk; ++b) sse += lpart[b];
  *loss = (float)(sse / ((double)n * kMlpOut));
}

// Partial results of ovl_mlp_gradient_static: each block's gradient, then each
// block's summed squared error.  One copy per device, alive until the process
// ends; host code reaches it only through the address kept per device below.
constexpr int kStaticBlocks = OVL_MLP_STATIC_ROWS / kTrRows;
static __device__ __align__(256) float scratch[kStaticBlocks * kMlpParams + kStaticBlocks];

}  // namespace

hipError_t launch_mlp_world(const WP& w, hipStream_t s) {
  if (w.Mcap <= 0) return hipSuccess;
  k_mlp_world<<<std::min(nblocks(w.Mcap, 64), kInfWorldBlocks), kInfBS, 0, s>>>(w);
  return hipGetLastError();
}

}  // namespace ovl

using namespace ovl;

struct ovl_mlp {
  hipStream_t stream = nullptr;
  float* params = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* gpart = nullptr;
  float* lpart = nullptr;
  float* grad = nullptr;
  float* xbuf = nullptr;
  float* tbuf = nullptr;
  int64_t cap_rows = 0;
  int nblk_cap = 0;
  int64_t t = 0;
  std::string err;
};

namespace {

thread_local std::string g_mlp_error;
// the last error of ovl_mlp_gradient_static (a fixed text; nothing allocated)
thread_local const char* g_static_error = nullptr;

// Device address of `scratch`, taken once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

float* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    // the gradient kernel's LDS is above the default limit
    if (hipFuncSetAttribute((const void*)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(TrainLds)) != hipSuccess)
      return nullptr;
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_ptr[dev];
}

bool mlp_reserve(ovl_mlp* M, int64_t n) {
  const int nblk = (int)((n + kTrRows - 1) / kTrRows);
  if (nblk > M->nblk_cap) {
    (void)hipFree(M->gpart);
    (void)hipFree(M->lpart);
    M->gpart = M->lpart = nullptr;
    if (hipMalloc(&M->gpart, (size_t)nblk * kMlpParams * sizeof(float)) != hipSuccess) return false;
    if (hipMalloc(&M->lpart, (size_t)nblk * sizeof(float)) != hipSuccess) return false;
    M->nblk_cap = nblk;
  }
  if (n > M->cap_rows) {
    (void)hipFree(M->xbuf);
    (void)hipFree(M->tbuf);
    M->xbuf = M->tbuf = nullptr;
    if (hipMalloc(&M->xbuf, (size_t)n * kMlpIn * sizeof(float)) != hipSuccess) return false;
    if (hipMalloc(&M->tbuf, (size_t)n * kMlpOut * sizeof(float)) != hipSuccess) return false;
    M->cap_rows = n;
  }
  return true;
}

ovl_status mlp_run(ovl_mlp* M, const float* x, const float* t, int64_t n, int32_t on_device, bool update, float lr,
                   float* grad_host, float* loss) {
  if (n <= 0 || n > (1 << 26)) {
    M->err = "n out of range";
    return OVL_ERR_INVALID_ARG;
  }
  if (!x || !t) {
    M->err = "NULL input";
    return OVL_ERR_INVALID_ARG;
  }
  if (!mlp_reserve(M, n)) {
    M->err = "device allocation failed";
    return OVL_ERR_OOM;
  }
  const float* dx = x;
  const float* dt = t;
  if (!on_device) {
    if (hipMemcpyAsync(M->xbuf, x, (size_t)n * kMlpIn * sizeof(float), hipMemcpyHostToDevice, M->stream) ||
        hipMemcpyAsync(M->tbuf, t, (size_t)n * kMlpOut * sizeof(float), hipMemcpyHostToDevice, M->stream)) {
      M->err = "upload failed";
      return OVL_ERR_DEVICE;
    }
    dx = M->xbuf;
    dt = M->tbuf;
  }
  const int nblk = (int)((n + kTrRows - 1) / kTrRows);
  k_mlp_grad<<<nblk, kTrBS, sizeof(TrainLds), M->stream>>>(M->params, dx, dt, (int)n, M->gpart, M->lpart);
  float c1 = 1.0f, c2 = 1.0f;
  if (update) {
    M->t += 1;
    c1 = (float)(1.0 - std::pow(0.9, (double)M->t));
    c2 = (float)(1.0 - std::pow(0.999, (double)M->t));
  }
  k_mlp_adam<<<nblocks(kMlpParams, 256), 256, 0, M->stream>>>(M->params, M->m, M->v, M->gpart, nblk, M->grad,
                                                              update ? 1 : 0, lr, 0.9f, 0.999f, c1, c2, 1e-8f);
  if (hipGetLastError() != hipSuccess) {
    M->err = "launch failed";
    return OVL_ERR_DEVICE;
  }
  std::vector<float> lp(nblk);
  if (hipMemcpyAsync(lp.data(), M->lpart, nblk * sizeof(float), hipMemcpyDeviceToHost, M->stream) ||
      (grad_host &&
       hipMemcpyAsync(grad_host, M->grad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, M->stream)) ||
      hipStreamSynchronize(M->stream)) {
    M->err = "copy failed";
    return OVL_ERR_DEVICE;
  }
  if (loss) {
    double sse = 0.0;
    for (float v : lp) sse += v;
    *loss = (float)(sse / ((double)n * kMlpOut));
  }
  return OVL_OK;
}

}  // namespace

extern "C" {

ovl_status ovl_mlp_create(const float* params, int64_t n_params, const ovl_device_ctx* ctx, ovl_mlp** out) {
  g_mlp_error.clear();
  if (!out || !params || n_params != kMlpParams) {
    g_mlp_error = "bad arguments (the network has " + std::to_string(kMlpParams) + " parameters)";
    return OVL_ERR_INVALID_ARG;
  }
  *out = nullptr;
  for (int64_t i = 0; i < n_params; ++i)
    if (!std::isfinite(params[i])) {
      g_mlp_error = "non-finite parameter";
      return OVL_ERR_INVALID_ARG;
    }
  ovl_mlp* M = new ovl_mlp();
  if (ctx) M->stream = (hipStream_t)ctx->stream;
  if (hipMalloc(&M->params, kMlpParams * sizeof(float)) || hipMalloc(&M->m, kMlpParams * sizeof(float)) ||
      hipMalloc(&M->v, kMlpParams * sizeof(float)) || hipMalloc(&M->grad, kMlpParams * sizeof(float))) {
    ovl_mlp_destroy(M);
    g_mlp_error = "device allocation failed";
    return OVL_ERR_OOM;
  }
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(TrainLds)) != hipSuccess) {
      ovl_mlp_destroy(M);
      g_mlp_error = "could not raise the LDS limit of the training kernel";
      return OVL_ERR_DEVICE;
    }
    attr = true;
  }
  std::vector<float> z(kMlpParams, 0.0f);
  if (hipMemcpy(M->params, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice) ||
      hipMemcpy(M->m, z.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice) ||
      hipMemcpy(M->v, z.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice)) {
    ovl_mlp_destroy(M);
    g_mlp_error = "upload failed";
    return OVL_ERR_DEVICE;
  }
  *out = M;
  return OVL_OK;
}

void ovl_mlp_destroy(ovl_mlp* M) {
  if (!M) return;
  (void)hipStreamSynchronize(M->stream);
  for (float* p : {M->params, M->m, M->v, M->gpart, M->lpart, M->grad, M->xbuf, M->tbuf}) (void)hipFree(p);
  delete M;
}

ovl_status ovl_mlp_train_step(ovl_mlp* M, const float* x, const float* t, int64_t n, float lr, int32_t on_device,
                              float* loss) {
  if (!M) return OVL_ERR_INVALID_ARG;
  if (!(lr > 0.0f) || !std::isfinite(lr)) {
    M->err = "lr must be > 0";
    return OVL_ERR_INVALID_ARG;
  }
  return mlp_run(M, x, t, n, on_device, true, lr, nullptr, loss);
}

ovl_status ovl_mlp_gradient(ovl_mlp* M, const float* x, const float* t, int64_t n, int32_t on_device, float* grad,
                            float* loss) {
  if (!M || !grad) return OVL_ERR_INVALID_ARG;
  return mlp_run(M, x, t, n, on_device, false, 0.0f, grad, loss);
}

ovl_status ovl_mlp_get_params(ovl_mlp* M, float* out, int64_t n) {
  if (!M || !out || n != kMlpParams) return OVL_ERR_INVALID_ARG;
  if (hipStreamSynchronize(M->stream) || hipMemcpy(out, M->params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost)) {
    M->err = "copy failed";
    return OVL_ERR_DEVICE;
  }
  return OVL_OK;
}

const char* ovl_mlp_last_error(const ovl_mlp* M) {
  if (M) return M->err.c_str();
  return g_static_error ? g_static_error : g_mlp_error.c_str();
}

ovl_status ovl_mlp_gradient_static(const float* params, const float* x, const float* t, int64_t n, float* grad,
                                   float* loss, void* stream) {
  g_static_error = nullptr;
  if (!params || !x || !t || !grad || !loss) {
    g_static_error = "ovl_mlp_gradient_static: NULL pointer";
    return OVL_ERR_INVALID_ARG;
  }
  if (n <= 0) {
    g_static_error = "ovl_mlp_gradient_static: n must be positive";
    return OVL_ERR_INVALID_ARG;
  }
  if (n > OVL_MLP_STATIC_ROWS) {
    g_static_error = "ovl_mlp_gradient_static: n exceeds OVL_MLP_STATIC_ROWS (8192 rows)";
    return OVL_ERR_CAPACITY;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    g_static_error = "ovl_mlp_gradient_static: no current device";
    return OVL_ERR_DEVICE;
  }
  float* sp = scratch_on(dev);
  if (!sp) {
    g_static_error = "ovl_mlp_gradient_static: could not reach the device's partial-result array";
    return OVL_ERR_DEVICE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nblk = (int)((n + kTrRows - 1) / kTrRows);
  float* gpart = sp;
  float* lpart = sp + (int64_t)kStaticBlocks * kMlpParams;
  k_mlp_grad<<<nblk, kTrBS, sizeof(TrainLds), s>>>(params, x, t, (int)n, gpart, lpart);
  k_mlp_adam<<<nblocks(kMlpParams, 256), 256, 0, s>>>(nullptr, nullptr, nullptr, gpart, nblk, grad, 0, 0.0f, 0.9f,
                                                      0.999f, 1.0f, 1.0f, 1e-8f);
  k_mlp_loss<<<1, 64, 0, s>>>(lpart, nblk, n, loss);
  if (hipGetLastError() != hipSuccess) {
    g_static_error = "ovl_mlp_gradient_static: launch failed";
    return OVL_ERR_DEVICE;
  }
  return OVL_OK;
}

ovl_status ovl_mlp_infer(const float* params, int64_t n_params, const float* x, int64_t n, float* y) {
  if (!params || n_params != kMlpParams || (n > 0 && (!x || !y)) || n < 0 || n > (1 << 26))
    return OVL_ERR_INVALID_ARG;
  if (n == 0) return OVL_OK;
  std::vector<uint16_t> wb;
  std::vector<float> bias;
  mlp_pack(params, wb, bias);
  uint16_t* dwb = nullptr;
  float *dbias = nullptr, *dx = nullptr, *dy = nullptr;
  ovl_status st = OVL_OK;
  if (hipMalloc(&dwb, wb.size() * 2) || hipMalloc(&dbias, bias.size() * 4) || hipMalloc(&dx, (size_t)n * kMlpIn * 4) ||
      hipMalloc(&dy, (size_t)n * kMlpOut * 4)) {
    st = OVL_ERR_OOM;
  } else if (hipMemcpy(dwb, wb.data(), wb.size() * 2, hipMemcpyHostToDevice) ||
             hipMemcpy(dbias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice) ||
             hipMemcpy(dx, x, (size_t)n * kMlpIn * 4, hipMemcpyHostToDevice)) {
    st = OVL_ERR_DEVICE;
  } else {
    k_mlp_infer<<<nblocks(n, 64), kInfBS>>>(dwb, dbias, dx, (int)n, dy);
    if (hipGetLastError() || hipDeviceSynchronize() ||
        hipMemcpy(y, dy, (size_t)n * kMlpOut * 4, hipMemcpyDeviceToHost))
      st = OVL_ERR_DEVICE;
  }
  (void)hipFree(dwb);
  (void)hipFree(dbias);
  (void)hipFree(dx);
  (void)hipFree(dy);
  return st;
}

}  // extern "C"
