// Contacts of a step (the main server's getContacts of Alg. 1): uniform-grid
// broad phase plus sphere narrow phase.
//
// Broad phase: every body goes into a hashed grid cell of edge `cs` (at least
// 2% wider than the largest contact distance, so float rounding of the cell
// index can never separate two bodies in contact by more than one cell);
// counting sort by bucket (atomic counts, scan, atomic scatter).  Order inside
// a bucket does not matter: a candidate b is accepted only from the one
// neighbour cell that equals b's own cell, so every pair is seen once.
//
// Narrow phase: a pair (a < b, same scene, not joined by a joint) is in
// contact when its gap is below the scene margin.  The test runs in double on
// the float state with a fixed operation order and no contraction, so the
// contact list is identical to any other implementation that follows the
// same order.  Static planes and static spheres of the scene are tested per
// body.  Contact records (normal from a to b, gap, lever-arm lengths to the
// midpoint of the two surface points) are computed in double, stored as float.
//
// Output order: per body a ascending, keys (bcode<<1 | sub) ascending, so the
// whole list is sorted by (a<<32)|(bcode<<1)|sub without a global sort: a
// count pass, a scan, then a write pass that sorts each body's short segment.
#include "ovl_internal.h"
#include "wave.h"

namespace ovl {

namespace {

__device__ __forceinline__ uint32_t cell_hash(int s, int x, int y, int z) {
  return ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349663u) ^ ((uint32_t)z * 83492791u) ^
         ((uint32_t)s * 2654435761u);
}

__device__ __forceinline__ int cell_coord(float x, float inv_cs) {
  float c = floorf(x * inv_cs);
  c = fminf(fmaxf(c, -1.0e9f), 1.0e9f);
  return (c == c) ? (int)c : 0;
}

__global__ void k_cells(WP w) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w.N) return;
  float inv = 1.0f / w.cs;
  int cx = cell_coord(w.st[0 * w.N + i], inv);
  int cy = cell_coord(w.st[1 * w.N + i], inv);
  int cz = cell_coord(w.st[2 * w.N + i], inv);
  w.cell[i] = cx;
  w.cell[w.N + i] = cy;
  w.cell[2 * w.N + i] = cz;
  uint32_t b = cell_hash(w.b_scene[i], cx, cy, cz) & (uint32_t)(w.T - 1);
  w.bucket[i] = b;
  atomicAdd(&w.bcount[b], 1);
}

__global__ void k_scatter(WP w) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w.N) return;
  uint32_t b = w.bucket[i];
  int pos = w.bstart[b] + atomicAdd(&w.bfill[b], 1);
  w.bbody[pos] = i;
}

// FP64 contact predicates, evaluated exactly as written (no contraction).
__device__ __forceinline__ bool pred_spheres(double xa, double ya, double za, double ra, double xb, double yb,
                                             double zb, double rb, double m, double* d) {
#pragma clang fp contract(off)
  double dx = xb - xa;
  double dy = yb - ya;
  double dz = zb - za;
  double d2 = dx * dx;
  d2 = d2 + dy * dy;
  d2 = d2 + dz * dz;
  double s = ra + rb;
  s = s + m;
  d[0] = dx;
  d[1] = dy;
  d[2] = dz;
  d[3] = d2;
  return d2 < s * s;
}

__device__ __forceinline__ bool pred_plane(double xa, double ya, double za, double ra, const float* pl, double m,
                                           double* phi_out) {
#pragma clang fp contract(off)
  double sd = (double)pl[0] * xa;
  sd = sd + (double)pl[1] * ya;
  sd = sd + (double)pl[2] * za;
  sd = sd - (double)pl[3];
  double phi = sd - ra;
  *phi_out = phi;
  return phi < m;
}

__device__ __forceinline__ bool jointed(const WP& w, int a, int b) {
  for (int k = w.jadj_off[a]; k < w.jadj_off[a + 1]; ++k)
    if (w.jadj[k] == b) return true;
  return false;
}

// Enumerate every contact of body a with bodies b > a and with statics.
// f(bkey) is called once per contact, in no particular order.
template <class F>
__device__ __forceinline__ void for_each_contact(const WP& w, int a, F&& f) {
  const int N = w.N;
  const int s = w.b_scene[a];
  const double m = (double)w.s_margin[s];
  const double xa = w.st[a], ya = w.st[N + a], za = w.st[2 * N + a], ra = w.b_radius[a];
  const int cx = w.cell[a], cy = w.cell[N + a], cz = w.cell[2 * N + a];
  const bool has_joints = w.jadj_off[a + 1] > w.jadj_off[a];
  double d[4];
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int nx = cx + dx, ny = cy + dy, nz = cz + dz;
        uint32_t h = cell_hash(s, nx, ny, nz) & (uint32_t)(w.T - 1);
        const int k1 = w.bstart[h + 1];
        for (int k = w.bstart[h]; k < k1; ++k) {
          const int b = w.bbody[k];
          if (b <= a) continue;
          if (w.cell[b] != nx || w.cell[N + b] != ny || w.cell[2 * N + b] != nz || w.b_scene[b] != s) continue;
          if (has_joints && jointed(w, a, b)) continue;
          if (pred_spheres(xa, ya, za, ra, w.st[b], w.st[N + b], w.st[2 * N + b], w.b_radius[b], m, d))
            f((uint32_t)b << 1);
        }
      }
  for (int j = w.s_plane_off[s]; j < w.s_plane_off[s + 1]; ++j) {
    double phi;
    if (pred_plane(xa, ya, za, ra, w.planes + 4 * j, m, &phi)) f((uint32_t)(N + j) << 1);
  }
  for (int j = w.s_ssph_off[s]; j < w.s_ssph_off[s + 1]; ++j) {
    const float* c = w.ssph + 4 * j;
    if (pred_spheres(xa, ya, za, ra, c[0], c[1], c[2], c[3], m, d)) f((uint32_t)(N + w.P + j) << 1);
  }
}

__global__ void k_contact_count(WP w) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= w.N) return;
  int n = 0;
  for_each_contact(w, a, [&](uint32_t) { ++n; });
  w.ccount[a] = n;
}

// geometry of one contact in double, stored as float: normal from a towards b,
// gap, and the lever-arm lengths: both arms point at the midpoint of the two
// surface points (r_a = l_a n, r_b = -l_b n), so a contact's impulse pair
// carries no net angular momentum
__device__ void contact_geometry(const WP& w, int a, uint32_t bkey, float* g /*6*/) {
  const int N = w.N;
  const uint32_t bc = bkey >> 1;
  const double xa = w.st[a], ya = w.st[N + a], za = w.st[2 * N + a], ra = w.b_radius[a];
  double n[3], phi, la, lb;
  if (bc < (uint32_t)N || bc >= (uint32_t)(N + w.P)) {
    double xb, yb, zb, rb;
    if (bc < (uint32_t)N) {
      xb = w.st[bc];
      yb = w.st[N + bc];
      zb = w.st[2 * N + bc];
      rb = w.b_radius[bc];
    } else {
      const float* c = w.ssph + 4 * (bc - N - w.P);
      xb = c[0];
      yb = c[1];
      zb = c[2];
      rb = c[3];
    }
    double d[4];
    pred_spheres(xa, ya, za, ra, xb, yb, zb, rb, 0.0, d);
    double dist = sqrt(d[3]);
    if (d[3] > 0.0) {
      n[0] = d[0] / dist;
      n[1] = d[1] / dist;
      n[2] = d[2] / dist;
    } else {
      n[0] = 0.0;
      n[1] = 0.0;
      n[2] = 1.0;
    }
    phi = dist - ra - rb;
    la = ra + 0.5 * phi;
    lb = rb + 0.5 * phi;
  } else {
    const float* pl = w.planes + 4 * (bc - N);
    pred_plane(xa, ya, za, ra, pl, 0.0, &phi);
    n[0] = -(double)pl[0];
    n[1] = -(double)pl[1];
    n[2] = -(double)pl[2];
    la = ra + 0.5 * phi;
    lb = 0.0;
  }
  g[0] = (float)n[0];
  g[1] = (float)n[1];
  g[2] = (float)n[2];
  g[3] = (float)phi;
  g[4] = (float)la;
  g[5] = (float)lb;
}

__global__ void k_contact_write(WP w) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= w.N) return;
  const int o0 = w.coff[a];
  const int o1 = w.coff[a + 1];
  if (o1 > w.Ccap) {
    if (o0 < w.Ccap || a == 0) atomicOr(&w.scal[SC_FLAGS], F_CONTACT_CAP);
    return;
  }
  int p = o0;
  for_each_contact(w, a, [&](uint32_t bkey) {
    if (p < o1) w.c_bkey[p++] = bkey;
  });
  // insertion sort of the body's short segment
  for (int i = o0 + 1; i < o1; ++i) {
    uint32_t k = w.c_bkey[i];
    int j = i - 1;
    while (j >= o0 && w.c_bkey[j] > k) {
      w.c_bkey[j + 1] = w.c_bkey[j];
      --j;
    }
    w.c_bkey[j + 1] = k;
  }
  for (int i = o0; i < o1; ++i) {
    float g[6];
    contact_geometry(w, a, w.c_bkey[i], g);
    w.c_a[i] = a;
#pragma unroll
    for (int k = 0; k < 6; ++k) w.c_geom[(int64_t)k * w.Ccap + i] = g[k];
  }
}

}  // namespace

hipError_t launch_collide(const WP& w, int32_t* scan_scratch, hipStream_t s) {
  hipError_t e;
  if ((e = fill_i32(w.bcount, 0, w.T + 1, s))) return e;
  if ((e = fill_i32(w.bfill, 0, w.T, s))) return e;
  if (w.N > 0) {
    k_cells<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if ((e = scan_excl(w.bcount, w.bstart, w.T, nullptr, scan_scratch, s))) return e;
  if (w.N > 0) {
    k_scatter<<<nblocks(w.N, kBlock), kBlock, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
    k_contact_count<<<nblocks(w.N, 128), 128, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  if ((e = scan_excl(w.ccount, w.coff, w.N, &w.scal[SC_NCONTACT], scan_scratch, s))) return e;
  if (w.N > 0) {
    k_contact_write<<<nblocks(w.N, 128), 128, 0, s>>>(w);
    if ((e = hipGetLastError())) return e;
  }
  return hipSuccess;
}

}  // namespace ovl
