// Contacts of a step (the main server's getContacts of Alg. 1): uniform-grid
// broad phase plus sphere and capsule narrow phase.
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
// body.  A capsule is the segment x + s u (|s| <= half-length, u the body z
// axis) swept by its radius: a pair involving one is tested on the closest
// points of the two segments; against a plane each end of the segment is a
// contact of its own (sub 0 for the end at -hl, 1 for +hl).  Contact records
// (normal from a to b, gap, lever arms to the midpoint of the two surface
// points) are computed in double, stored as float.
//
// Output order: per body a ascending, keys (bcode<<1 | sub) ascending, so the
// whole list is sorted by (a<<32)|(bcode<<1)|sub without a global sort: a
// count pass, a scan, then a write pass that sorts each body's short segment.
#include "ovl_internal.h"
#include "wave.h"

namespace ovl {

namespace {

// Spatial hash of a grid cell: the three large primes of Teschner et al.,
// "Optimized Spatial Hashing for Collision Detection of Deformable Objects"
// (VMV 2003), XOR-combined; the scene index is mixed in with Knuth's
// multiplicative constant 2654435761 (TAOCP vol. 3, section 6.4).
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

// Bodies in bucket order, with a packed copy of what the neighbour scan reads
// (cell, body; centre, radius), so a bucket is one or two cache lines.
__global__ void k_scatter(WP w) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w.N) return;
  const int N = w.N;
  uint32_t b = w.bucket[i];
  int pos = w.bstart[b] + atomicAdd(&w.bfill[b], 1);
  w.bbody[pos] = i;
  w.srt_cell[pos] = make_int4(w.cell[i], w.cell[N + i], w.cell[2 * N + i], i);
  w.srt_pos[pos] = make_float4(w.st[i], w.st[N + i], w.st[2 * N + i], w.b_radius[i]);
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

// Capsule axis from the float quaternion in double, not renormalised, in this
// exact order: u = (2 (qx qz + qw qy), 2 (qy qz - qw qx), 1 - 2 (qx qx + qy qy)).
__device__ __forceinline__ void capsule_axis(const float* st, int N, int i, double* u) {
#pragma clang fp contract(off)
  const double qw = st[3 * N + i], qx = st[4 * N + i], qy = st[5 * N + i], qz = st[6 * N + i];
  double s;
  s = qx * qz;
  s = s + qw * qy;
  u[0] = 2.0 * s;
  s = qy * qz;
  s = s - qw * qx;
  u[1] = 2.0 * s;
  s = qx * qx;
  s = s + qy * qy;
  u[2] = 1.0 - 2.0 * s;
}

__device__ __forceinline__ double dot3d(const double* a, const double* b) {
#pragma clang fp contract(off)
  double d = a[0] * b[0];
  d = d + a[1] * b[1];
  d = d + a[2] * b[2];
  return d;
}

__device__ __forceinline__ double clamp_sym(double x, double h) { return x < -h ? -h : (x > h ? h : x); }

// Closest points of the segments x_a + s u_a (|s| <= ha) and x_b + t u_b
// (|t| <= hb), ha or hb possibly 0.  With r = x_a - x_b the stationary point
// solves a s - b t = -c, -b s + e t = f (a = u_a.u_a, e = u_b.u_b, b = u_a.u_b,
// c = u_a.r, f = u_b.r); s is clamped, t follows from s and is clamped, and s
// is recomputed if t was.  Near-parallel segments (a e - b^2 <= 1e-9 a e):
// s is the middle of the stretch of A covered by B's projection, or the end
// of A nearest to it when they do not overlap.
__device__ __forceinline__ void segment_closest(const double* xa, const double* ua, double ha, const double* xb,
                                                const double* ub, double hb, double& s_out, double& t_out) {
#pragma clang fp contract(off)
  const double r[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
  double s = 0.0, t = 0.0;
  if (ha > 0.0 && hb > 0.0) {
    const double a = dot3d(ua, ua), e = dot3d(ub, ub), b = dot3d(ua, ub);
    const double c = dot3d(ua, r), f = dot3d(ub, r);
    double den = a * e;
    den = den - b * b;
    if (den > 1e-9 * (a * e)) {
      double num = b * f;
      num = num - c * e;
      s = clamp_sym(num / den, ha);
    } else {
      const double wv = fabs(b) * hb;
      const double lo = (-wv - c) / a, hi = (wv - c) / a;
      const double l2 = lo > -ha ? lo : -ha, h2 = hi < ha ? hi : ha;
      s = l2 <= h2 ? 0.5 * (l2 + h2) : clamp_sym(-c / a, ha);
    }
    double tn = b * s;
    tn = tn + f;
    t = tn / e;
    if (t < -hb || t > hb) {
      t = clamp_sym(t, hb);
      double sn = b * t;
      sn = sn - c;
      s = clamp_sym(sn / a, ha);
    }
  } else if (hb > 0.0) {
    t = clamp_sym(dot3d(ub, r) / dot3d(ub, ub), hb);
  } else if (ha > 0.0) {
    s = clamp_sym(-dot3d(ua, r) / dot3d(ua, ua), ha);
  }
  s_out = s;
  t_out = t;
}

// Gap test of two swept segments: d = (x_b + t u_b) - (x_a + s u_a), same
// order as the sphere test on it.  d[0..2] the vector, d[3] its square, st[0..1] = (s, t).
__device__ __forceinline__ bool pred_swept(const double* xa, const double* ua, double ha, double ra, const double* xb,
                                           const double* ub, double hb, double rb, double m, double* d, double* st) {
#pragma clang fp contract(off)
  double s, t;
  segment_closest(xa, ua, ha, xb, ub, hb, s, t);
  double pa[3], pb[3];
  for (int k = 0; k < 3; ++k) {
    pa[k] = xa[k] + s * ua[k];
    pb[k] = xb[k] + t * ub[k];
  }
  st[0] = s;
  st[1] = t;
  return pred_spheres(pa[0], pa[1], pa[2], ra, pb[0], pb[1], pb[2], rb, m, d);
}

// One end of a capsule against a plane (sub 0: x - hl u, sub 1: x + hl u).
__device__ __forceinline__ bool pred_cap_plane(const double* xa, const double* u, double hl, double ra, int sub,
                                               const float* pl, double m, double* phi_out) {
#pragma clang fp contract(off)
  double e[3];
  for (int k = 0; k < 3; ++k) {
    const double hu = hl * u[k];
    e[k] = sub ? xa[k] + hu : xa[k] - hu;
  }
  return pred_plane(e[0], e[1], e[2], ra, pl, m, phi_out);
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
  const double ha = w.has_caps ? (double)w.b_half[a] : 0.0;
  const double pa[3] = {xa, ya, za};
  double ua[3] = {0.0, 0.0, 0.0};
  if (ha > 0.0) capsule_axis(w.st, N, a, ua);
  double d[4], stp[2];
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int nx = cx + dx, ny = cy + dy, nz = cz + dz;
        uint32_t h = cell_hash(s, nx, ny, nz) & (uint32_t)(w.T - 1);
        const int k1 = w.bstart[h + 1];
        for (int k = w.bstart[h]; k < k1; ++k) {
          const int4 ck = w.srt_cell[k];
          const int b = ck.w;
          if (b <= a || ck.x != nx || ck.y != ny || ck.z != nz) continue;
          if (w.b_scene[b] != s) continue;
          if (has_joints && jointed(w, a, b)) continue;
          const float4 pr = w.srt_pos[k];
          const double hb = w.has_caps ? (double)w.b_half[b] : 0.0;
          bool hit;
          if (ha == 0.0 && hb == 0.0) {
            hit = pred_spheres(xa, ya, za, ra, pr.x, pr.y, pr.z, pr.w, m, d);
          } else {
            const double pb[3] = {pr.x, pr.y, pr.z};
            double ub[3] = {0.0, 0.0, 0.0};
            if (hb > 0.0) capsule_axis(w.st, N, b, ub);
            hit = pred_swept(pa, ua, ha, ra, pb, ub, hb, pr.w, m, d, stp);
          }
          if (hit) f((uint32_t)b << 1);
        }
      }
  for (int j = w.s_plane_off[s]; j < w.s_plane_off[s + 1]; ++j) {
    double phi;
    if (ha == 0.0) {
      if (pred_plane(xa, ya, za, ra, w.planes + 4 * j, m, &phi)) f((uint32_t)(N + j) << 1);
    } else {
      for (int sub = 0; sub < 2; ++sub)
        if (pred_cap_plane(pa, ua, ha, ra, sub, w.planes + 4 * j, m, &phi)) f(((uint32_t)(N + j) << 1) | sub);
    }
  }
  for (int j = w.s_ssph_off[s]; j < w.s_ssph_off[s + 1]; ++j) {
    const float* c = w.ssph + 4 * j;
    bool hit;
    if (ha == 0.0) {
      hit = pred_spheres(xa, ya, za, ra, c[0], c[1], c[2], c[3], m, d);
    } else {
      const double pc[3] = {c[0], c[1], c[2]}, zero[3] = {0.0, 0.0, 0.0};
      hit = pred_swept(pa, ua, ha, ra, pc, zero, 0.0, c[3], m, d, stp);
    }
    if (hit) f((uint32_t)(N + w.P + j) << 1);
  }
}

// Both passes walk the bodies in grid-bucket order (bbody), so the lanes of a
// wavefront search neighbouring cells and share their cache lines.  The count
// pass keeps the first kKeep keys of each body; the write pass copies them and
// searches again only for bodies with more contacts.
__global__ void k_contact_count(WP w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w.N) return;
  const int a = w.bbody[i];
  uint32_t* keep = w.c_keep + (int64_t)a * kKeep;
  int n = 0;
  for_each_contact(w, a, [&](uint32_t bkey) {
    if (n < kKeep) keep[n] = bkey;
    ++n;
  });
  w.ccount[a] = n;
}

// geometry of one contact in double, stored as float: normal from a towards b,
// gap, and the lever arms to the midpoint of the two surface points,
// r_a = s_a u_a + l_a n and r_b = t_b u_b - l_b n (s_a = t_b = 0 for spheres),
// so a contact's impulse pair carries no net angular momentum
__device__ void contact_geometry(const WP& w, int a, uint32_t bkey, float* g /*8*/) {
  const int N = w.N;
  const uint32_t bc = bkey >> 1;
  const int sub = (int)(bkey & 1u);
  const double xa = w.st[a], ya = w.st[N + a], za = w.st[2 * N + a], ra = w.b_radius[a];
  const double ha = w.has_caps ? (double)w.b_half[a] : 0.0;
  const double pa[3] = {xa, ya, za};
  double ua[3] = {0.0, 0.0, 0.0};
  if (ha > 0.0) capsule_axis(w.st, N, a, ua);
  double n[3], phi, la, lb, sa = 0.0, tb = 0.0;
  if (bc < (uint32_t)N || bc >= (uint32_t)(N + w.P)) {
    double pb[3], rb, hb = 0.0;
    double ub[3] = {0.0, 0.0, 0.0};
    if (bc < (uint32_t)N) {
      pb[0] = w.st[bc];
      pb[1] = w.st[N + bc];
      pb[2] = w.st[2 * N + bc];
      rb = w.b_radius[bc];
      hb = w.has_caps ? (double)w.b_half[bc] : 0.0;
      if (hb > 0.0) capsule_axis(w.st, N, (int)bc, ub);
    } else {
      const float* c = w.ssph + 4 * (bc - N - w.P);
      pb[0] = c[0];
      pb[1] = c[1];
      pb[2] = c[2];
      rb = c[3];
    }
    double d[4];
    if (ha == 0.0 && hb == 0.0) {
      pred_spheres(xa, ya, za, ra, pb[0], pb[1], pb[2], rb, 0.0, d);
    } else {
      double stp[2];
      pred_swept(pa, ua, ha, ra, pb, ub, hb, rb, 0.0, d, stp);
      sa = stp[0];
      tb = stp[1];
    }
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
    if (ha == 0.0) {
      pred_plane(xa, ya, za, ra, pl, 0.0, &phi);
    } else {
      pred_cap_plane(pa, ua, ha, ra, sub, pl, 0.0, &phi);
      sa = sub ? ha : -ha;
    }
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
  g[6] = (float)sa;
  g[7] = (float)tb;
}

__global__ void k_contact_write(WP w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w.N) return;
  const int a = w.bbody[i];
  const int o0 = w.coff[a];
  const int o1 = w.coff[a + 1];
  if (o1 > w.Ccap) {
    if (o0 < w.Ccap || a == 0) atomicOr(&w.scal[SC_FLAGS], F_CONTACT_CAP);
    return;
  }
  if (o1 - o0 <= kKeep) {
    const uint32_t* keep = w.c_keep + (int64_t)a * kKeep;
    for (int k = 0; k < o1 - o0; ++k) w.c_bkey[o0 + k] = keep[k];
  } else {
    int p = o0;
    for_each_contact(w, a, [&](uint32_t bkey) {
      if (p < o1) w.c_bkey[p++] = bkey;
    });
  }
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
    float g[8];
    contact_geometry(w, a, w.c_bkey[i], g);
    w.c_a[i] = a;
#pragma unroll
    for (int k = 0; k < 8; ++k) w.c_geom[(int64_t)k * w.Ccap + i] = g[k];
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
