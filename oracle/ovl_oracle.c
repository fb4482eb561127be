/* Oracle for the overlapping-partition rigid-body step (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, sequential, double-precision CPU code that follows the method of
 * Kale & Kry (arXiv 2403.17261) step by step for one time step.  It is meant to
 * be read against the paper, not to be fast.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg load it; it shares no code with
 * the GPU library.
 *
 * Where the paper leaves a detail open the reading taken here is stated at the
 * place it is used (the same readings bind the GPU library).
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -shared -fPIC (no fast-math), so
 * every double operation is a single IEEE round-to-nearest operation.
 */
#include "ovl_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

struct orc_result {
  void* ptr[ORC_NFIELDS];
  int64_t len[ORC_NFIELDS];
  char err[256];
};

static void* xalloc(size_t n) {
  void* p = calloc(n ? n : 1, 1);
  if (!p) {
    fprintf(stderr, "oracle: out of memory\n");
    abort();
  }
  return p;
}

static void* xgrow(void* p, size_t n) {
  void* q = realloc(p, n ? n : 1);
  if (!q) {
    fprintf(stderr, "oracle: out of memory\n");
    abort();
  }
  return q;
}

static void put(orc_result* r, int f, void* p, int64_t n) {
  r->ptr[f] = p;
  r->len[f] = n;
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double* a, const double* b, double* o) {
  double x = a[1] * b[2] - a[2] * b[1];
  double y = a[2] * b[0] - a[0] * b[2];
  double z = a[0] * b[1] - a[1] * b[0];
  o[0] = x;
  o[1] = y;
  o[2] = z;
}

static void mat3_vec(const double* m, const double* v, double* o) {
  for (int i = 0; i < 3; ++i) o[i] = m[3 * i] * v[0] + m[3 * i + 1] * v[1] + m[3 * i + 2] * v[2];
}

static int popcount64(uint64_t x) {
  int c = 0;
  while (x) {
    x &= x - 1;
    ++c;
  }
  return c;
}

static int lowest_bit(uint64_t x) {
  int i = 0;
  while (!(x & 1)) {
    x >>= 1;
    ++i;
  }
  return i;
}

/* MurmurHash3 32-bit finaliser (Appleby, public domain).  Used only to give
 * every constraint copy a deterministic pseudo-random colouring priority. */
uint32_t orc_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

/* Orthonormal tangent pair for unit normal n: the branch-on-sign(n_z)
 * construction of Duff et al., "Building an Orthonormal Basis, Revisited"
 * (JCGT 6(1), 2017).  The only branch is the sign of n_z, which is decided
 * exactly in any precision, so both implementations pick the same branch. */
void orc_tangents(const double n[3], double t1[3], double t2[3]) {
  double s = copysign(1.0, n[2]);
  double a = -1.0 / (s + n[2]);
  double b = n[0] * n[1] * a;
  t1[0] = 1.0 + s * n[0] * n[0] * a;
  t1[1] = s * b;
  t1[2] = -s * n[0];
  t2[0] = b;
  t2[1] = s + n[1] * n[1] * a;
  t2[2] = -n[1];
}

/* rotation matrix of a unit quaternion (w, x, y, z) */
static void quat_to_mat(const double* q, double* R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  double nn = sqrt(w * w + x * x + y * y + z * z);
  w /= nn;
  x /= nn;
  y /= nn;
  z /= nn;
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------------------------------- */
/* contacts: the list of touching pairs the main server finds each step       */
/* (Alg. 1 getContacts).  Reading: a pair is in contact when its gap is below */
/* the scene margin; the test is evaluated in double on the float state with  */
/* a fixed operation order so that every implementation agrees exactly.       */
/* ------------------------------------------------------------------------- */

typedef struct {
  uint64_t key;
  double n[3], phi, ra[3], rb[3];
} contact;

typedef struct {
  contact* c;
  int64_t n, cap;
} contact_list;

static void cl_push(contact_list* l, const contact* c) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 256;
    l->c = (contact*)xgrow(l->c, (size_t)l->cap * sizeof(contact));
  }
  l->c[l->n++] = *c;
}

static uint64_t contact_key(int64_t a, int64_t bcode, int sub) {
  return ((uint64_t)a << 32) | ((uint64_t)bcode << 1) | (uint64_t)sub;
}

/* sphere centre xa (radius ra) against a sphere centre xb (radius rb): FP64 test */
static int sphere_sphere(const float* xa, float ra, const float* xb, float rb, float margin, contact* out) {
  double dx = (double)xb[0] - (double)xa[0];
  double dy = (double)xb[1] - (double)xa[1];
  double dz = (double)xb[2] - (double)xa[2];
  double d2 = dx * dx;
  d2 = d2 + dy * dy;
  d2 = d2 + dz * dz;
  double s = (double)ra + (double)rb;
  s = s + (double)margin;
  if (!(d2 < s * s)) return 0;
  double dist = sqrt(d2);
  if (d2 > 0.0) {
    out->n[0] = dx / dist;
    out->n[1] = dy / dist;
    out->n[2] = dz / dist;
  } else {
    out->n[0] = 0.0;
    out->n[1] = 0.0;
    out->n[2] = 1.0;
  }
  out->phi = dist - (double)ra - (double)rb;
  /* reading: both lever arms point at the midpoint of the two surface points,
   * so the pair of impulses carries no net angular momentum */
  double la = (double)ra + 0.5 * out->phi, lb = (double)rb + 0.5 * out->phi;
  for (int k = 0; k < 3; ++k) {
    out->ra[k] = la * out->n[k];
    out->rb[k] = -lb * out->n[k];
  }
  return 1;
}

static int sphere_plane(const float* xa, float ra, const float* pl, float margin, contact* out) {
  double sd = (double)pl[0] * (double)xa[0];
  sd = sd + (double)pl[1] * (double)xa[1];
  sd = sd + (double)pl[2] * (double)xa[2];
  sd = sd - (double)pl[3];
  double phi = sd - (double)ra;
  if (!(phi < (double)margin)) return 0;
  out->phi = phi;
  for (int k = 0; k < 3; ++k) {
    out->n[k] = -(double)pl[k];
    out->ra[k] = ((double)ra + 0.5 * phi) * out->n[k];
    out->rb[k] = 0.0;
  }
  return 1;
}

/* Capsules (shape 1): a segment of half-length hl along the body z axis,
 * swept by the radius.  Reading: the world axis is computed from the float
 * quaternion in double without renormalisation, in this exact order, so every
 * implementation gets the same bits:
 *   u = (2 (qx qz + qw qy), 2 (qy qz - qw qx), 1 - 2 (qx qx + qy qy)). */
static void capsule_axis(const float* q, double* u) {
  double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
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

static double clamp_sym(double x, double h) { return x < -h ? -h : (x > h ? h : x); }

/* Closest points of two segments x_a + s u_a (|s| <= ha) and x_b + t u_b
 * (|t| <= hb); ha or hb may be 0 (a sphere centre).  Minimising
 * |r + s u_a - t u_b|^2 with r = x_a - x_b gives the 2x2 system
 *   a s - b t = -c,   -b s + e t = f
 * (a = u_a.u_a, e = u_b.u_b, b = u_a.u_b, c = u_a.r, f = u_b.r).  s is taken
 * from it and clamped, t follows from s and is clamped, and s is recomputed
 * when t was clamped.  Reading for (near-)parallel segments, where the system
 * is singular: s is the middle of the stretch of A that B's projection covers
 * (or the nearest end of A when they do not overlap). */
static void segment_closest(const double* xa, const double* ua, double ha, const double* xb, const double* ub,
                            double hb, double* s_out, double* t_out) {
  double r[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
  double s = 0.0, t = 0.0;
  if (ha > 0.0 && hb > 0.0) {
    double a = dot3(ua, ua), e = dot3(ub, ub), b = dot3(ua, ub);
    double c = dot3(ua, r), f = dot3(ub, r);
    double den = a * e - b * b;
    if (den > 1e-9 * (a * e)) {
      s = clamp_sym((b * f - c * e) / den, ha);
    } else {
      double w = fabs(b) * hb;
      double lo = (-w - c) / a, hi = (w - c) / a;
      double l2 = lo > -ha ? lo : -ha, h2 = hi < ha ? hi : ha;
      s = l2 <= h2 ? 0.5 * (l2 + h2) : clamp_sym(-c / a, ha);
    }
    t = (b * s + f) / e;
    if (t < -hb || t > hb) {
      t = clamp_sym(t, hb);
      s = clamp_sym((b * t - c) / a, ha);
    }
  } else if (hb > 0.0) {
    t = clamp_sym(dot3(ub, r) / dot3(ub, ub), hb);
  } else if (ha > 0.0) {
    s = clamp_sym(-dot3(ua, r) / dot3(ua, ua), ha);
  }
  *s_out = s;
  *t_out = t;
}

/* Contact of two swept segments (at least one a capsule, or a capsule and a
 * static sphere).  Same gap test as for spheres, on the closest points; the
 * lever arms point at the midpoint of the two surface points:
 *   r_a = s u_a + (ra + phi/2) n,   r_b = t u_b - (rb + phi/2) n. */
static int swept_pair(const float* xa_f, const double* ua, double ha, float ra_f, const float* xb_f,
                      const double* ub, double hb, float rb_f, float margin, contact* out) {
  double xa[3] = {xa_f[0], xa_f[1], xa_f[2]}, xb[3] = {xb_f[0], xb_f[1], xb_f[2]};
  double s, t;
  segment_closest(xa, ua, ha, xb, ub, hb, &s, &t);
  double pa[3], pb[3];
  for (int k = 0; k < 3; ++k) {
    pa[k] = xa[k] + s * ua[k];
    pb[k] = xb[k] + t * ub[k];
  }
  double dx = pb[0] - pa[0];
  double dy = pb[1] - pa[1];
  double dz = pb[2] - pa[2];
  double d2 = dx * dx;
  d2 = d2 + dy * dy;
  d2 = d2 + dz * dz;
  double sr = (double)ra_f + (double)rb_f;
  sr = sr + (double)margin;
  if (!(d2 < sr * sr)) return 0;
  double dist = sqrt(d2);
  if (d2 > 0.0) {
    out->n[0] = dx / dist;
    out->n[1] = dy / dist;
    out->n[2] = dz / dist;
  } else {
    out->n[0] = 0.0;
    out->n[1] = 0.0;
    out->n[2] = 1.0;
  }
  out->phi = dist - (double)ra_f - (double)rb_f;
  double la = (double)ra_f + 0.5 * out->phi, lb = (double)rb_f + 0.5 * out->phi;
  for (int k = 0; k < 3; ++k) {
    out->ra[k] = s * ua[k] + la * out->n[k];
    out->rb[k] = t * ub[k] - lb * out->n[k];
  }
  return 1;
}

/* Capsule against a plane: each end of the segment is tested like a sphere
 * centre (sub 0 for the end at -hl, sub 1 for +hl). */
static int capsule_plane_end(const float* xa_f, const double* u, double hl, float ra, int sub, const float* pl,
                             float margin, contact* out) {
  double e[3];
  for (int k = 0; k < 3; ++k) {
    double hu = hl * u[k];
    e[k] = sub ? (double)xa_f[k] + hu : (double)xa_f[k] - hu;
  }
  double sd = (double)pl[0] * e[0];
  sd = sd + (double)pl[1] * e[1];
  sd = sd + (double)pl[2] * e[2];
  sd = sd - (double)pl[3];
  double phi = sd - (double)ra;
  if (!(phi < (double)margin)) return 0;
  out->phi = phi;
  for (int k = 0; k < 3; ++k) {
    out->n[k] = -(double)pl[k];
    out->ra[k] = (sub ? hl : -hl) * u[k] + ((double)ra + 0.5 * phi) * out->n[k];
    out->rb[k] = 0.0;
  }
  return 1;
}

/* any pair of dynamic bodies: the sphere test when both are spheres */
static int body_pair(const orc_scene* sc, const float* st, int64_t a, int64_t b, contact* out) {
  float m = sc->margin[sc->scene[a]];
  const float* xa = st + 13 * a;
  const float* xb = st + 13 * b;
  if (sc->shape[a] == 0 && sc->shape[b] == 0) return sphere_sphere(xa, sc->radius[a], xb, sc->radius[b], m, out);
  double ua[3] = {0, 0, 0}, ub[3] = {0, 0, 0};
  double ha = 0.0, hb = 0.0;
  if (sc->shape[a] == 1) {
    capsule_axis(xa + 3, ua);
    ha = sc->halflen[a];
  }
  if (sc->shape[b] == 1) {
    capsule_axis(xb + 3, ub);
    hb = sc->halflen[b];
  }
  return swept_pair(xa, ua, ha, sc->radius[a], xb, ub, hb, sc->radius[b], m, out);
}

typedef struct {
  int64_t* k;
  int64_t n;
} pairset;

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

static int cmp_contact(const void* a, const void* b) {
  uint64_t x = ((const contact*)a)->key, y = ((const contact*)b)->key;
  return (x > y) - (x < y);
}

static int jointed(const pairset* js, int64_t a, int64_t b) {
  int64_t lo = a < b ? a : b, hi = a < b ? b : a;
  int64_t key = (lo << 32) | hi;
  return bsearch(&key, js->k, (size_t)js->n, sizeof(int64_t), cmp_i64) != NULL;
}

/* contacts of body a with statics of its scene (planes, then static spheres) */
static void static_contacts(const orc_scene* sc, int64_t a, const float* xa, int64_t P, contact_list* out) {
  int s = sc->scene[a];
  float m = sc->margin[s];
  contact c;
  const int cap = sc->shape[a] == 1;
  double u[3] = {0, 0, 0}, zero[3] = {0, 0, 0};
  if (cap) capsule_axis(xa + 3, u);
  for (int64_t j = sc->plane_off[s]; j < sc->plane_off[s + 1]; ++j) {
    if (!cap) {
      if (sphere_plane(xa, sc->radius[a], sc->planes + 4 * j, m, &c)) {
        c.key = contact_key(a, sc->n_bodies + j, 0);
        cl_push(out, &c);
      }
      continue;
    }
    for (int sub = 0; sub < 2; ++sub)
      if (capsule_plane_end(xa, u, sc->halflen[a], sc->radius[a], sub, sc->planes + 4 * j, m, &c)) {
        c.key = contact_key(a, sc->n_bodies + j, sub);
        cl_push(out, &c);
      }
  }
  for (int64_t j = sc->ssph_off[s]; j < sc->ssph_off[s + 1]; ++j) {
    const float* cs = sc->ssph + 4 * j;
    int hit = cap ? swept_pair(xa, u, sc->halflen[a], sc->radius[a], cs, zero, 0.0, cs[3], m, &c)
                  : sphere_sphere(xa, sc->radius[a], cs, cs[3], m, &c);
    if (hit) {
      c.key = contact_key(a, sc->n_bodies + P + j, 0);
      cl_push(out, &c);
    }
  }
}

typedef struct {
  int64_t cell[4]; /* scene, cx, cy, cz */
  int64_t body;
} cellent;

static int cmp_cell(const void* a, const void* b) {
  const cellent* x = (const cellent*)a;
  const cellent* y = (const cellent*)b;
  for (int i = 0; i < 4; ++i)
    if (x->cell[i] != y->cell[i]) return x->cell[i] < y->cell[i] ? -1 : 1;
  return (x->body > y->body) - (x->body < y->body);
}

static int64_t cell_lower(const cellent* e, int64_t n, const int64_t* key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    int c = 0;
    for (int i = 0; i < 4 && !c; ++i)
      if (e[mid].cell[i] != key[i]) c = e[mid].cell[i] < key[i] ? -1 : 1;
    if (c < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

static void find_contacts(const orc_scene* sc, const float* st, const pairset* js, int brute,
                          contact_list* out) {
  const int64_t N = sc->n_bodies;
  const int64_t P = sc->plane_off[sc->n_scenes];
  contact_list tmp = {0};
  if (brute) {
    for (int64_t a = 0; a < N; ++a) {
      tmp.n = 0;
      for (int64_t b = a + 1; b < N && sc->scene[b] == sc->scene[a]; ++b) {
        contact c;
        if (jointed(js, a, b)) continue;
        if (body_pair(sc, st, a, b, &c)) {
          c.key = contact_key(a, b, 0);
          cl_push(&tmp, &c);
        }
      }
      static_contacts(sc, a, st + 13 * a, P, &tmp);
      qsort(tmp.c, (size_t)tmp.n, sizeof(contact), cmp_contact);
      for (int64_t i = 0; i < tmp.n; ++i) cl_push(out, &tmp.c[i]);
    }
  } else {
    /* the oracle's own uniform grid: cells of edge 2*r_max + margin_max, with
     * r the bounding radius (radius + half-length for a capsule) */
    double rmax = 0.0, mmax = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      double rb = (double)sc->radius[i] + (sc->shape[i] == 1 ? (double)sc->halflen[i] : 0.0);
      if (rb > rmax) rmax = rb;
    }
    for (int s = 0; s < sc->n_scenes; ++s)
      if (sc->margin[s] > mmax) mmax = sc->margin[s];
    double cs = 2.0 * rmax + mmax;
    if (cs <= 0) cs = 1.0;
    cellent* e = (cellent*)xalloc((size_t)N * sizeof(cellent));
    for (int64_t i = 0; i < N; ++i) {
      e[i].cell[0] = sc->scene[i];
      for (int k = 0; k < 3; ++k) e[i].cell[k + 1] = (int64_t)floor((double)st[13 * i + k] / cs);
      e[i].body = i;
    }
    qsort(e, (size_t)N, sizeof(cellent), cmp_cell);
    int64_t* home = (int64_t*)xalloc((size_t)N * sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) home[e[i].body] = i;
    for (int64_t a = 0; a < N; ++a) {
      tmp.n = 0;
      const cellent* ea = &e[home[a]];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int64_t key[4] = {ea->cell[0], ea->cell[1] + dx, ea->cell[2] + dy, ea->cell[3] + dz};
            for (int64_t i = cell_lower(e, N, key); i < N; ++i) {
              if (e[i].cell[0] != key[0] || e[i].cell[1] != key[1] || e[i].cell[2] != key[2] ||
                  e[i].cell[3] != key[3])
                break;
              int64_t b = e[i].body;
              contact c;
              if (b <= a || jointed(js, a, b)) continue;
              if (body_pair(sc, st, a, b, &c)) {
                c.key = contact_key(a, b, 0);
                cl_push(&tmp, &c);
              }
            }
          }
      static_contacts(sc, a, st + 13 * a, P, &tmp);
      qsort(tmp.c, (size_t)tmp.n, sizeof(contact), cmp_contact);
      for (int64_t i = 0; i < tmp.n; ++i) cl_push(out, &tmp.c[i]);
    }
    free(home);
    free(e);
  }
  free(tmp.c);
}

/* ------------------------------------------------------------------------- */
/* constraint graph (section 5.1): vertices are the non-static bodies, an     */
/* edge joins two bodies that share a joint or a contact; statics are left out */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t* off; /* N+1 */
  int32_t* adj;
} graph;

static void build_graph(const orc_scene* sc, const contact_list* cl, graph* g) {
  const int64_t N = sc->n_bodies;
  int64_t ne = 0;
  int64_t* e = (int64_t*)xalloc((size_t)(2 * (cl->n + sc->n_joints) + 1) * sizeof(int64_t));
  for (int64_t i = 0; i < cl->n; ++i) {
    int64_t a = (int64_t)(cl->c[i].key >> 32), b = (int64_t)((cl->c[i].key >> 1) & 0x7fffffff);
    if (b >= N) continue;
    e[ne++] = (a << 32) | b;
    e[ne++] = (b << 32) | a;
  }
  for (int64_t j = 0; j < sc->n_joints; ++j) {
    int64_t a = sc->joint_ab[2 * j], b = sc->joint_ab[2 * j + 1];
    e[ne++] = (a << 32) | b;
    e[ne++] = (b << 32) | a;
  }
  qsort(e, (size_t)ne, sizeof(int64_t), cmp_i64);
  g->off = (int32_t*)xalloc((size_t)(N + 1) * sizeof(int32_t));
  g->adj = (int32_t*)xalloc((size_t)(ne + 1) * sizeof(int32_t));
  int64_t m = 0;
  for (int64_t i = 0; i < ne; ++i) {
    if (i > 0 && e[i] == e[i - 1]) continue; /* duplicate edge */
    int64_t v = e[i] >> 32;
    g->off[v + 1]++;
    g->adj[m++] = (int32_t)(e[i] & 0xffffffff);
  }
  for (int64_t v = 0; v < N; ++v) g->off[v + 1] += g->off[v];
  free(e);
}

/* breadth-first search from `src` to depth `maxd`; writes the visited
 * vertices and their hop counts (getBFSVertices of the paper) */
typedef struct {
  int32_t* stamp;
  int32_t* dist;
  int32_t* queue;
  int32_t cur;
} bfs_ws;

static int64_t bfs(const graph* g, int32_t src, int maxd, bfs_ws* w) {
  int64_t head = 0, tail = 0;
  w->cur++;
  w->stamp[src] = w->cur;
  w->dist[src] = 0;
  w->queue[tail++] = src;
  while (head < tail) {
    int32_t v = w->queue[head++];
    if (w->dist[v] >= maxd) continue;
    for (int32_t i = g->off[v]; i < g->off[v + 1]; ++i) {
      int32_t u = g->adj[i];
      if (w->stamp[u] == w->cur) continue;
      w->stamp[u] = w->cur;
      w->dist[u] = w->dist[v] + 1;
      w->queue[tail++] = u;
    }
  }
  return tail;
}

/* ------------------------------------------------------------------------- */
/* step                                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t part, kind, ia, ib, colour;
  int64_t id; /* joint index or contact index */
  uint64_t key;
  int64_t uid;
  double dir[9], ra[3], rb[3], arr[3], invd[3], bias[3], mu;
  double anga[9], angb[9], ka[9], kb[9];
  double lam[3], lam0[3], laml[3];
  double feat[13];
  int32_t deg;
} copy_t;

typedef struct {
  uint32_t h;
  int64_t uid;
  int64_t idx;
} prio_t;

static int cmp_prio_desc(const void* a, const void* b) {
  const prio_t* x = (const prio_t*)a;
  const prio_t* y = (const prio_t*)b;
  if (x->h != y->h) return x->h > y->h ? -1 : 1;
  return x->uid > y->uid ? -1 : (x->uid < y->uid);
}

typedef struct {
  int32_t colour;
  int64_t uid;
  int64_t idx;
} order_t;

static int cmp_order(const void* a, const void* b) {
  const order_t* x = (const order_t*)a;
  const order_t* y = (const order_t*)b;
  if (x->colour != y->colour) return x->colour < y->colour ? -1 : 1;
  return (x->uid > y->uid) - (x->uid < y->uid);
}

/* cache lookup: entries sorted by (part, kind, key) */
static int64_t cache_find(const orc_cache* c, int32_t part, int32_t kind, uint64_t key) {
  int64_t lo = 0, hi = c->n;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    int cmp;
    if (c->part[mid] != part)
      cmp = c->part[mid] < part ? -1 : 1;
    else if (c->kind[mid] != kind)
      cmp = c->kind[mid] < kind ? -1 : 1;
    else if (c->key[mid] != key)
      cmp = c->key[mid] < key ? -1 : 1;
    else
      return mid;
    if (cmp < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  return -1;
}

typedef struct {
  double x[3], q[4], v[3], w[3];
  double invm, invi[9];
  double vt[6];
  double cpl[6]; /* coupling impulse of the previous step's cut constraints, as (dv, dw) */
  int32_t body;
} replica;

/* apply an impulse of size dl along a row to the velocities of its bodies */
static void apply_row(replica* A, replica* B, const copy_t* c, int r, double dl) {
  for (int k = 0; k < 3; ++k) {
    A->v[k] -= A->invm * dl * c->dir[3 * r + k];
    A->w[k] -= dl * c->ka[3 * r + k];
  }
  if (B) {
    for (int k = 0; k < 3; ++k) {
      B->v[k] += B->invm * dl * c->dir[3 * r + k];
      B->w[k] += dl * c->kb[3 * r + k];
    }
  }
}

/* constraint velocity J_r v of one row */
static double row_velocity(const replica* A, const replica* B, const copy_t* c, int r) {
  double s = -dot3(c->dir + 3 * r, A->v) - dot3(c->anga + 3 * r, A->w);
  if (B) s += dot3(c->dir + 3 * r, B->v) + dot3(c->angb + 3 * r, B->w);
  return s;
}

static void row_bounds(const copy_t* c, int r, double* lo, double* hi) {
  if (c->kind == 0) {
    *lo = -INFINITY;
    *hi = INFINITY;
  } else if (r == 0) {
    *lo = 0.0;
    *hi = INFINITY;
  } else {
    /* box friction: limits follow the current normal impulse */
    *lo = -c->mu * c->lam[0];
    *hi = c->mu * c->lam[0];
  }
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Blending of one body's replica states (Alg. 4, Eq. 11-14).  Replicas come
 * in ascending partition id; a quaternion whose dot product with the first
 * replica's is negative is negated before the weighted sum; the summed
 * quaternion is normalised.  A body with one replica keeps its state. */
void orc_blend(int32_t n, const double* states, const double* w, double* out) {
  if (n == 1) {
    for (int k = 0; k < 13; ++k) out[k] = states[k];
    return;
  }
  double q0[4] = {states[3], states[4], states[5], states[6]};
  double acc[13];
  for (int k = 0; k < 13; ++k) acc[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    const double* st = states + 13 * i;
    double qi[4] = {st[3], st[4], st[5], st[6]};
    if (i > 0 && qi[0] * q0[0] + qi[1] * q0[1] + qi[2] * q0[2] + qi[3] * q0[3] < 0.0)
      for (int k = 0; k < 4; ++k) qi[k] = -qi[k];
    for (int k = 0; k < 3; ++k) {
      acc[k] += w[i] * st[k];
      acc[7 + k] += w[i] * st[7 + k];
      acc[10 + k] += w[i] * st[10 + k];
    }
    for (int k = 0; k < 4; ++k) acc[3 + k] += w[i] * qi[k];
  }
  double nn = sqrt(acc[3] * acc[3] + acc[4] * acc[4] + acc[5] * acc[5] + acc[6] * acc[6]);
  for (int k = 0; k < 4; ++k) acc[3 + k] /= nn;
  for (int k = 0; k < 13; ++k) out[k] = acc[k];
}

/* Copy a start (plain, or learned for contacts) into lambda and apply it to
 * the velocities in solve order. */
static void apply_start(replica* rp, copy_t* cp, const order_t* od, int64_t nm, int learned) {
  for (int64_t t = 0; t < nm; ++t) {
    copy_t* c = &cp[od[t].idx];
    replica* A = &rp[c->ia];
    replica* B = c->ib >= 0 ? &rp[c->ib] : NULL;
    const double* l0 = learned ? c->laml : c->lam0;
    for (int r = 0; r < 3; ++r) {
      c->lam[r] = l0[r];
      if (l0[r] != 0.0) apply_row(A, B, c, r, l0[r]);
    }
  }
}

/* Natural-map residual of a start (max over the partition's rows); the
 * velocities are restored to v~ afterwards. */
static double start_residual(replica* rp, int64_t nr, copy_t* cp, const order_t* od, int64_t nm, int learned,
                             double cfm) {
  apply_start(rp, cp, od, nm, learned);
  double e = 0.0;
  for (int64_t t = 0; t < nm; ++t) {
    copy_t* c = &cp[od[t].idx];
    replica* A = &rp[c->ia];
    replica* B = c->ib >= 0 ? &rp[c->ib] : NULL;
    for (int r = 0; r < 3; ++r) {
      double w = row_velocity(A, B, c, r) + c->bias[r] + cfm * c->lam[r];
      double lo, hi;
      row_bounds(c, r, &lo, &hi);
      double x = c->arr[r] * fabs(c->lam[r] - clampd(c->lam[r] - w * c->invd[r], lo, hi));
      if (x > e) e = x;
    }
  }
  for (int64_t r = 0; r < nr; ++r)
    for (int k = 0; k < 3; ++k) {
      rp[r].v[k] = rp[r].vt[k];
      rp[r].w[k] = rp[r].vt[3 + k];
    }
  return e;
}

/* bfloat16 rounding of a float (round to nearest, ties to even), returned as float */
float orc_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  memcpy(&x, &u, 4);
  return x;
}

/* The warm-start network 12 -> 64 -> 64 -> 3 with ReLU, evaluated the way a
 * bfloat16 matrix engine does: inputs, weights and hidden activations rounded
 * to bfloat16, products accumulated exactly (here in double), biases in
 * float. */
void orc_mlp_infer(const float* P, const double* x12, double* y3) {
  const float* W1 = P;
  const float* b1 = W1 + ORC_MLP_IN * ORC_MLP_HID;
  const float* W2 = b1 + ORC_MLP_HID;
  const float* b2 = W2 + ORC_MLP_HID * ORC_MLP_HID;
  const float* W3 = b2 + ORC_MLP_HID;
  const float* b3 = W3 + ORC_MLP_HID * ORC_MLP_OUT;
  double x[ORC_MLP_IN], h1[ORC_MLP_HID], h2[ORC_MLP_HID];
  for (int k = 0; k < ORC_MLP_IN; ++k) x[k] = orc_bf16((float)x12[k]);
  for (int j = 0; j < ORC_MLP_HID; ++j) {
    double acc = 0.0;
    for (int k = 0; k < ORC_MLP_IN; ++k) acc += x[k] * orc_bf16(W1[k * ORC_MLP_HID + j]);
    double v = acc + b1[j];
    h1[j] = orc_bf16((float)(v > 0.0 ? v : 0.0));
  }
  for (int j = 0; j < ORC_MLP_HID; ++j) {
    double acc = 0.0;
    for (int k = 0; k < ORC_MLP_HID; ++k) acc += h1[k] * orc_bf16(W2[k * ORC_MLP_HID + j]);
    double v = acc + b2[j];
    h2[j] = orc_bf16((float)(v > 0.0 ? v : 0.0));
  }
  for (int o = 0; o < ORC_MLP_OUT; ++o) {
    double acc = 0.0;
    for (int k = 0; k < ORC_MLP_HID; ++k) acc += h2[k] * orc_bf16(W3[k * ORC_MLP_OUT + o]);
    y3[o] = acc + b3[o];
  }
}

/* local index of body v among the replicas of partition p (bodies ascending) */
static int32_t local_rep(const int32_t* prep, const int32_t* rep_body, int32_t p, int32_t v) {
  int32_t lo = prep[p], hi = prep[p + 1];
  while (lo < hi) {
    int32_t mid = (lo + hi) / 2;
    if (rep_body[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < prep[p + 1] && rep_body[lo] == v) ? lo - prep[p] : -1;
}

/* ------------------------------------------------------------------------- */
/* dynamic load balancing (section 5.4): Alg. 6 with the bridge test Alg. 7  */
/* ------------------------------------------------------------------------- */

/* A worker's load is the number of bodies active in it; the load of a set of
 * workers (Alg. 6 line 5) is read as the sum of its workers' loads.  Workers
 * are the local partition bits of a scene; load[] is indexed by global id. */
typedef struct {
  uint64_t* mask;
  int64_t* load;
  const int32_t* pbase;
  const int32_t* scene;
} lb_state;

static void lb_activate(lb_state* st, uint64_t set, int32_t v) {
  uint64_t add = set & ~st->mask[v];
  st->mask[v] |= add;
  for (; add; add &= add - 1) st->load[st->pbase[st->scene[v]] + lowest_bit(add)]++;
}

static void lb_deactivate(lb_state* st, uint64_t set, int32_t v) {
  uint64_t rem = set & st->mask[v];
  st->mask[v] &= ~rem;
  for (; rem; rem &= rem - 1) st->load[st->pbase[st->scene[v]] + lowest_bit(rem)]--;
}

static int64_t lb_set_load(const lb_state* st, uint64_t set, int s) {
  int64_t l = 0;
  for (; set; set &= set - 1) l += st->load[st->pbase[s] + lowest_bit(set)];
  return l;
}

/* Alg. 7: a body bridges workers when its graph neighbours span more than one */
static int lb_bridge(const lb_state* st, const graph* g, int32_t b) {
  uint64_t w = 0;
  for (int32_t k = g->off[b]; k < g->off[b + 1]; ++k) w |= st->mask[g->adj[k]];
  return popcount64(w) > 1;
}

/* Alg. 6 over the step's contacts, in key order.  Readings: ties in line 5 go
 * to A's side (the test is <=); "smallest load" ties go to the lowest worker
 * index; the BFS vertices of line 12 include the root. */
static void load_balance(lb_state* st, const graph* g, const contact_list* cl, int64_t N, int depth, bfs_ws* ws) {
  for (int64_t i = 0; i < cl->n; ++i) {
    uint64_t key = cl->c[i].key;
    int32_t A = (int32_t)(key >> 32);
    int64_t B64 = (int64_t)((key >> 1) & 0x7fffffff);
    if (B64 >= N) continue; /* statics are not in the graph */
    int32_t B = (int32_t)B64;
    int s = st->scene[A];
    uint64_t WA = st->mask[A], WB = st->mask[B];
    if ((WA & WB) == 0) {
      /* Fig. 9 (i), (ii): make one worker aware of the other body */
      int32_t root;
      if (lb_set_load(st, WA, s) <= lb_set_load(st, WB, s)) {
        lb_activate(st, WA, B);
        root = B;
      } else {
        lb_activate(st, WB, A);
        root = A;
      }
      int64_t nv = bfs(g, root, depth, ws);
      for (int64_t q = 0; q < nv; ++q) lb_activate(st, WA | WB, ws->queue[q]);
    } else if (popcount64(WA) > 1 && popcount64(WB) == 1 && !lb_bridge(st, g, A)) {
      lb_deactivate(st, WA & ~WB, A); /* Fig. 9 (iii), (iv) */
    } else if (popcount64(WB) > 1 && popcount64(WA) == 1 && !lb_bridge(st, g, B)) {
      lb_deactivate(st, WB & ~WA, B);
    } else if (WA == WB) {
      /* Fig. 9 (v): keep both bodies only in the least loaded of their workers */
      int best = -1;
      int64_t bl = 0;
      for (uint64_t t = WA; t; t &= t - 1) {
        int b = lowest_bit(t);
        int64_t l = st->load[st->pbase[s] + b];
        if (best < 0 || l < bl) {
          best = b;
          bl = l;
        }
      }
      lb_deactivate(st, WA & ~(1ull << best), A);
      lb_deactivate(st, WB & ~(1ull << best), B);
    }
  }
}

orc_result* orc_step(const orc_scene* sc, const float* state, const int32_t* owner,
                     const int32_t* parts_per_scene, const orc_params* prm, const orc_cache* cache,
                     const int32_t* forced_iters) {
  orc_result* res = (orc_result*)xalloc(sizeof(orc_result));
  const int64_t N = sc->n_bodies;
  const int S = sc->n_scenes;
  const double h = prm->dt;
  double* stats = (double*)xalloc(9 * sizeof(double));
  put(res, ORC_STATS, stats, 9);

  /* ---- partitions: global ids, each scene owns a contiguous range ---- */
  int32_t* pbase = (int32_t*)xalloc((size_t)(S + 1) * sizeof(int32_t));
  for (int s = 0; s < S; ++s) {
    if (parts_per_scene[s] < 1 || parts_per_scene[s] > 64) {
      snprintf(res->err, sizeof res->err, "scene %d: parts %d out of [1,64]", s, parts_per_scene[s]);
      stats[6] = 1;
      free(pbase);
      return res;
    }
    pbase[s + 1] = pbase[s] + parts_per_scene[s];
  }
  const int32_t G = pbase[S];
  for (int64_t i = 0; i < N; ++i) {
    int s = sc->scene[i];
    int bad_shape = sc->shape[i] != 0 && !(sc->shape[i] == 1 && sc->halflen[i] > 0.0f);
    if (bad_shape || owner[i] < pbase[s] || owner[i] >= pbase[s + 1]) {
      snprintf(res->err, sizeof res->err, "body %lld: bad shape or owner", (long long)i);
      stats[6] = 1;
      free(pbase);
      return res;
    }
  }

  /* ---- contacts (Alg. 1 getContacts) ---- */
  pairset js;
  js.n = sc->n_joints;
  js.k = (int64_t*)xalloc((size_t)(js.n + 1) * sizeof(int64_t));
  for (int64_t j = 0; j < js.n; ++j) {
    int64_t a = sc->joint_ab[2 * j], b = sc->joint_ab[2 * j + 1];
    js.k[j] = ((a < b ? a : b) << 32) | (a < b ? b : a);
  }
  qsort(js.k, (size_t)js.n, sizeof(int64_t), cmp_i64);
  contact_list cl = {0};
  find_contacts(sc, state, &js, prm->brute_force_contacts, &cl);
  const int64_t C = cl.n;
  {
    uint64_t* key = (uint64_t*)xalloc((size_t)C * 8);
    double* nn = (double*)xalloc((size_t)C * 24);
    double* phi = (double*)xalloc((size_t)C * 8);
    double* ra = (double*)xalloc((size_t)C * 24);
    double* rb = (double*)xalloc((size_t)C * 24);
    for (int64_t i = 0; i < C; ++i) {
      key[i] = cl.c[i].key;
      phi[i] = cl.c[i].phi;
      for (int k = 0; k < 3; ++k) {
        nn[3 * i + k] = cl.c[i].n[k];
        ra[3 * i + k] = cl.c[i].ra[k];
        rb[3 * i + k] = cl.c[i].rb[k];
      }
    }
    put(res, ORC_CONTACT_KEY, key, C);
    put(res, ORC_CONTACT_N, nn, 3 * C);
    put(res, ORC_CONTACT_PHI, phi, C);
    put(res, ORC_CONTACT_RA, ra, 3 * C);
    put(res, ORC_CONTACT_RB, rb, 3 * C);
  }

  /* ---- constraint graph ---- */
  graph g;
  build_graph(sc, &cl, &g);
  put(res, ORC_ADJ_OFF, g.off, N + 1);
  put(res, ORC_ADJ, g.adj, g.off[N]);

  bfs_ws ws;
  ws.stamp = (int32_t*)xalloc((size_t)(N + 1) * 4);
  ws.dist = (int32_t*)xalloc((size_t)(N + 1) * 4);
  ws.queue = (int32_t*)xalloc((size_t)(N + 1) * 4);
  ws.cur = 0;

  /* ---- overlap sets (Eq. 9-10; Alg. 2-3 read as a k-hop halo): a body is
   * active in every partition that owns some body within k hops of it ---- */
  uint64_t* mask = (uint64_t*)xalloc((size_t)N * 8);
  int64_t n_overlap = 0;
  if (prm->lb_masks) {
    /* worker sets carried from the previous step, updated by Alg. 6 */
    for (int64_t v = 0; v < N; ++v) {
      mask[v] = prm->lb_masks[v];
      if (mask[v] == 0 || (mask[v] >> parts_per_scene[sc->scene[v]]) != 0) {
        snprintf(res->err, sizeof res->err, "body %lld: empty worker set or a bit beyond its scene's partitions",
                 (long long)v);
        stats[6] = 1;
        free(mask);
        return res;
      }
    }
    int64_t* load = (int64_t*)xalloc((size_t)(G + 1) * 8);
    for (int64_t v = 0; v < N; ++v)
      for (uint64_t t = mask[v]; t; t &= t - 1) load[pbase[sc->scene[v]] + lowest_bit(t)]++;
    lb_state st = {mask, load, pbase, sc->scene};
    load_balance(&st, &g, &cl, N, prm->lb_depth, &ws);
    free(load);
    for (int64_t v = 0; v < N; ++v)
      if (popcount64(mask[v]) >= 2) n_overlap++;
  } else {
    for (int64_t v = 0; v < N; ++v) {
      int64_t nv = bfs(&g, (int32_t)v, prm->halo_k, &ws);
      uint64_t m = 0;
      for (int64_t i = 0; i < nv; ++i) {
        int32_t u = ws.queue[i];
        m |= 1ull << (owner[u] - pbase[sc->scene[u]]);
      }
      mask[v] = m;
      if (popcount64(m) >= 2) n_overlap++;
    }
  }
  put(res, ORC_MASK, mask, N);

  /* ---- replica table: partition-major, bodies ascending ---- */
  int32_t* prep = (int32_t*)xalloc((size_t)(G + 1) * 4);
  for (int64_t v = 0; v < N; ++v) {
    int s = sc->scene[v];
    for (int b = 0; b < parts_per_scene[s]; ++b)
      if (mask[v] >> b & 1) prep[pbase[s] + b + 1]++;
  }
  for (int32_t p = 0; p < G; ++p) prep[p + 1] += prep[p];
  const int64_t R = prep[G];
  int32_t* rep_body = (int32_t*)xalloc((size_t)R * 4);
  {
    int32_t* fill = (int32_t*)xalloc((size_t)(G + 1) * 4);
    for (int64_t v = 0; v < N; ++v) {
      int s = sc->scene[v];
      for (int b = 0; b < parts_per_scene[s]; ++b)
        if (mask[v] >> b & 1) {
          int32_t p = pbase[s] + b;
          rep_body[prep[p] + fill[p]++] = (int32_t)v;
        }
    }
    free(fill);
  }
  put(res, ORC_PART_REP_OFF, prep, G + 1);
  put(res, ORC_REP_BODY, rep_body, R);

  /* ---- geodesic distances and weights (Eq. 15-16, Alg. 5) ----
   * D(o,i) = hops from o to the nearest body that is active in partition i
   * only; searched to depth beta; weight proportional to 1/D; partitions not
   * reached within beta get weight 0; if none is reached the weights are
   * uniform.  Bodies in a single partition have weight 1. */
  int32_t* repD = (int32_t*)xalloc((size_t)R * 4);
  double* repW = (double*)xalloc((size_t)R * 8);
  for (int64_t v = 0; v < N; ++v) {
    int s = sc->scene[v];
    int np = parts_per_scene[s];
    int nw = popcount64(mask[v]);
    int32_t D[64];
    for (int b = 0; b < 64; ++b) D[b] = 0;
    if (nw >= 2) {
      int64_t nv = bfs(&g, (int32_t)v, prm->beta, &ws);
      for (int64_t i = 0; i < nv; ++i) {
        int32_t u = ws.queue[i];
        if (popcount64(mask[u]) != 1 || !(mask[u] & mask[v])) continue;
        int b = lowest_bit(mask[u]);
        if (D[b] == 0 || ws.dist[u] < D[b]) D[b] = ws.dist[u];
      }
    }
    double dsum = 0.0;
    for (int b = 0; b < np; ++b)
      if ((mask[v] >> b & 1) && D[b] > 0) dsum += 1.0 / (double)D[b];
    for (int b = 0; b < np; ++b) {
      if (!(mask[v] >> b & 1)) continue;
      int32_t p = pbase[s] + b;
      int32_t li = local_rep(prep, rep_body, p, (int32_t)v);
      int64_t r = prep[p] + li;
      repD[r] = D[b];
      if (nw == 1)
        repW[r] = 1.0;
      else if (prm->equal_weights)
        repW[r] = 1.0 / (double)nw;
      else if (dsum > 0.0)
        repW[r] = (D[b] > 0 ? 1.0 / (double)D[b] : 0.0) / dsum;
      else
        repW[r] = 1.0 / (double)nw;
    }
  }
  put(res, ORC_REP_D, repD, R);
  put(res, ORC_REP_W, repW, R);

  /* ---- replica states at the start of the step: every replica is reset to
   * the blended state (Alg. 1 resetStateTo); external force = gravity ---- */
  replica* rep = (replica*)xalloc((size_t)(R ? R : 1) * sizeof(replica));
  for (int64_t r = 0; r < R; ++r) {
    int32_t v = rep_body[r];
    const float* s = state + 13 * (int64_t)v;
    replica* q = &rep[r];
    q->body = v;
    for (int k = 0; k < 3; ++k) {
      q->x[k] = s[k];
      q->v[k] = s[7 + k];
      q->w[k] = s[10 + k];
    }
    for (int k = 0; k < 4; ++k) q->q[k] = s[3 + k];
    /* mass splitting: the replica carries the share w of the body (inverse
     * mass and inverse inertia over w); weight 0 keeps the whole body */
    double share = 1.0;
    if (prm->coupling == 2 && repW[r] > 0.0) share = repW[r];
    q->invm = 1.0 / (double)sc->mass[v] / share;
    double Rm[9], Ib[3];
    quat_to_mat(q->q, Rm);
    for (int k = 0; k < 3; ++k) Ib[k] = 1.0 / (double)sc->inertia[3 * v + k];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += Rm[3 * i + k] * Ib[k] * Rm[3 * j + k];
        q->invi[3 * i + j] = acc / share;
      }
    /* Eq. 1 with f = m g: v~ = v + h g */
    q->v[0] += h * prm->gx;
    q->v[1] += h * prm->gy;
    q->v[2] += h * prm->gz;
    for (int k = 0; k < 3; ++k) {
      q->vt[k] = q->v[k];
      q->vt[3 + k] = q->w[k];
    }
  }

  /* ---- constraint copies: a partition solves every constraint whose
   * non-static bodies are all active in it; per partition the list is the
   * joints by index, then the contacts by key ---- */
  int32_t* pcop = (int32_t*)xalloc((size_t)(G + 1) * 4);
  int64_t M = 0, Mcap = 1024;
  copy_t* cp = (copy_t*)xalloc((size_t)Mcap * sizeof(copy_t));
  /* joints are sorted by scene, contacts by body a (so by scene): per-scene ranges */
  int64_t* jrng = (int64_t*)xalloc((size_t)(S + 1) * 8);
  int64_t* crng = (int64_t*)xalloc((size_t)(S + 1) * 8);
  for (int s = 0, j = 0, i = 0; s < S; ++s) {
    while (j < sc->n_joints && sc->scene[sc->joint_ab[2 * j]] < s) ++j;
    while (i < C && sc->scene[(int64_t)(cl.c[i].key >> 32)] < s) ++i;
    jrng[s] = j;
    crng[s] = i;
  }
  jrng[S] = sc->n_joints;
  crng[S] = C;
  for (int32_t p = 0; p < G; ++p) {
    pcop[p] = (int32_t)M;
    int s = 0;
    while (s < S && !(p >= pbase[s] && p < pbase[s + 1])) ++s;
    int b = p - pbase[s];
    for (int64_t j = jrng[s]; j < jrng[s + 1]; ++j) {
      int32_t a = sc->joint_ab[2 * j], bb = sc->joint_ab[2 * j + 1];
      if (sc->scene[a] != s || !(mask[a] >> b & 1) || !(mask[bb] >> b & 1)) continue;
      if (M == Mcap) {
        Mcap *= 2;
        cp = (copy_t*)xgrow(cp, (size_t)Mcap * sizeof(copy_t));
      }
      copy_t* c = &cp[M];
      memset(c, 0, sizeof *c);
      c->part = p;
      c->kind = 0;
      c->id = j;
      c->key = (uint64_t)j;
      c->uid = M;
      c->ia = local_rep(prep, rep_body, p, a);
      c->ib = local_rep(prep, rep_body, p, bb);
      ++M;
    }
    for (int64_t i = crng[s]; i < crng[s + 1]; ++i) {
      int32_t a = (int32_t)(cl.c[i].key >> 32);
      int64_t bc = (int64_t)((cl.c[i].key >> 1) & 0x7fffffff);
      if (sc->scene[a] != s || !(mask[a] >> b & 1)) continue;
      if (bc < N && !(mask[bc] >> b & 1)) continue;
      if (M == Mcap) {
        Mcap *= 2;
        cp = (copy_t*)xgrow(cp, (size_t)Mcap * sizeof(copy_t));
      }
      copy_t* c = &cp[M];
      memset(c, 0, sizeof *c);
      c->part = p;
      c->kind = 1;
      c->id = i;
      c->key = cl.c[i].key;
      c->uid = M;
      c->ia = local_rep(prep, rep_body, p, a);
      c->ib = bc < N ? local_rep(prep, rep_body, p, (int32_t)bc) : -1;
      ++M;
    }
  }
  pcop[G] = (int32_t)M;
  put(res, ORC_PART_COPY_OFF, pcop, G + 1);
  free(jrng);
  free(crng);

  /* ---- interface coupling (section 7's proposal, optional): the constraints
   * a partition leaves out because one of their two dynamic bodies is not
   * active in it still push on the body that is, with the impulse they
   * received in the previous step.  Per body the incident constraints are
   * taken in constraint-list order (joints by index, then contacts by key);
   * the impulse comes from the cache entry of the lowest partition active in
   * both bodies, converted as the warm start converts it; it acts on the body
   * inside the partition as F at its lever arm r: dv = F/m, dw = I^-1 (r x F),
   * with F = -sum_r lambda_r d_r on body a and +sum_r lambda_r d_r on body b
   * (the signs of the rows' impulses). ---- */
  for (int64_t r = 0; r < R; ++r)
    for (int k = 0; k < 6; ++k) rep[r].cpl[k] = 0.0;
  if (prm->coupling == 1 && cache && cache->n > 0) {
    /* incidence lists: body -> constraints (joints first, then contacts) */
    int64_t* ioff = (int64_t*)xalloc((size_t)(N + 1) * 8);
    for (int64_t v = 0; v <= N; ++v) ioff[v] = 0;
    for (int64_t j = 0; j < sc->n_joints; ++j) {
      ioff[sc->joint_ab[2 * j] + 1]++;
      ioff[sc->joint_ab[2 * j + 1] + 1]++;
    }
    for (int64_t i = 0; i < C; ++i) {
      int64_t bc = (int64_t)((cl.c[i].key >> 1) & 0x7fffffff);
      if (bc >= N) continue;
      ioff[(cl.c[i].key >> 32) + 1]++;
      ioff[bc + 1]++;
    }
    for (int64_t v = 0; v < N; ++v) ioff[v + 1] += ioff[v];
    int64_t* ifill = (int64_t*)xalloc((size_t)(N ? N : 1) * 8);
    int64_t* inc = (int64_t*)xalloc((size_t)(ioff[N] ? ioff[N] : 1) * 8);
    for (int64_t v = 0; v < N; ++v) ifill[v] = ioff[v];
    /* entries: joint j as j, contact i as n_joints + i */
    for (int64_t j = 0; j < sc->n_joints; ++j) {
      inc[ifill[sc->joint_ab[2 * j]]++] = j;
      inc[ifill[sc->joint_ab[2 * j + 1]]++] = j;
    }
    for (int64_t i = 0; i < C; ++i) {
      int64_t bc = (int64_t)((cl.c[i].key >> 1) & 0x7fffffff);
      if (bc >= N) continue;
      inc[ifill[cl.c[i].key >> 32]++] = sc->n_joints + i;
      inc[ifill[bc]++] = sc->n_joints + i;
    }
    for (int32_t p = 0; p < G; ++p) {
      int s = 0;
      while (s < S && !(p >= pbase[s] && p < pbase[s + 1])) ++s;
      int bit = p - pbase[s];
      for (int64_t r = prep[p]; r < prep[p + 1]; ++r) {
        replica* q = &rep[r];
        int32_t v = q->body;
        for (int64_t e = ioff[v]; e < ioff[v + 1]; ++e) {
          int64_t id = inc[e];
          int kind = id < sc->n_joints ? 0 : 1;
          int32_t a, b;
          uint64_t key;
          const contact* k = NULL;
          if (kind == 0) {
            a = sc->joint_ab[2 * id];
            b = sc->joint_ab[2 * id + 1];
            key = (uint64_t)id;
          } else {
            k = &cl.c[id - sc->n_joints];
            a = (int32_t)(k->key >> 32);
            b = (int32_t)((k->key >> 1) & 0x7fffffff);
            key = k->key;
          }
          int32_t o = v == a ? b : a;
          if (mask[o] >> bit & 1) continue; /* both bodies in P_p: solved here */
          uint64_t both = mask[v] & mask[o];
          if (!both) continue;
          int32_t src = pbase[s] + lowest_bit(both);
          int64_t f = cache_find(cache, src, kind, key);
          if (f < 0) continue;
          const float* val = cache->val + 4 * f;
          double lam[3], d[9], lever[3];
          if (kind == 0) {
            for (int i = 0; i < 3; ++i) lam[i] = val[i];
            for (int i = 0; i < 9; ++i) d[i] = 0.0;
            for (int i = 0; i < 3; ++i) d[3 * i + i] = -1.0;
            const float* an = sc->joint_anchor + 6 * id + (v == a ? 0 : 3);
            double Rm[9], anc[3] = {an[0], an[1], an[2]};
            quat_to_mat(q->q, Rm);
            mat3_vec(Rm, anc, lever);
          } else {
            double t1[3], t2[3];
            orc_tangents(k->n, t1, t2);
            for (int i = 0; i < 3; ++i) {
              d[i] = k->n[i];
              d[3 + i] = t1[i];
              d[6 + i] = t2[i];
              lever[i] = v == a ? k->ra[i] : k->rb[i];
            }
            double mu = sc->mu[s];
            double ln = val[0] > 0.0f ? (double)val[0] : 0.0;
            double fw[3] = {val[1], val[2], val[3]};
            lam[0] = ln;
            lam[1] = clampd(dot3(fw, t1), -mu * ln, mu * ln);
            lam[2] = clampd(dot3(fw, t2), -mu * ln, mu * ln);
          }
          double F[3], tq[3], dw[3];
          for (int i = 0; i < 3; ++i) F[i] = lam[0] * d[i] + lam[1] * d[3 + i] + lam[2] * d[6 + i];
          if (v == a)
            for (int i = 0; i < 3; ++i) F[i] = -F[i];
          cross3(lever, F, tq);
          mat3_vec(q->invi, tq, dw);
          for (int i = 0; i < 3; ++i) {
            q->cpl[i] += q->invm * F[i];
            q->cpl[3 + i] += dw[i];
          }
        }
        for (int i = 0; i < 3; ++i) {
          q->v[i] += q->cpl[i];
          q->w[i] += q->cpl[3 + i];
          q->vt[i] = q->v[i];
          q->vt[3 + i] = q->w[i];
        }
      }
    }
    free(ioff);
    free(ifill);
    free(inc);
  }
  {
    double* cpl = (double*)xalloc((size_t)(R ? R : 1) * 48);
    for (int64_t r = 0; r < R; ++r)
      for (int k = 0; k < 6; ++k) cpl[6 * r + k] = rep[r].cpl[k];
    put(res, ORC_REP_CPL, cpl, 6 * R);
  }

  /* ---- rows (Eq. 1-7): three rows per copy.
   * contact: directions n, t1, t2; the normal row has lower bound 0, the two
   *   friction rows the box [-mu lambda_n, mu lambda_n]; bias phi/h for a gap,
   *   erp*phi/h for a penetration (Eq. 2 stabilisation, scaled), none for
   *   friction.
   * ball joint: the three world axes with direction -e_k, unbounded, bias
   *   erp*C_k/h where C = (x_a + R_a a_a) - (x_b + R_b a_b).
   * A_rr = J_r M^-1 J_r^T + cfm (Eq. 4 diagonal). ---- */
  for (int64_t m = 0; m < M; ++m) {
    copy_t* c = &cp[m];
    replica* A = &rep[prep[c->part] + c->ia];
    replica* B = c->ib >= 0 ? &rep[prep[c->part] + c->ib] : NULL;
    if (c->kind == 1) {
      const contact* k = &cl.c[c->id];
      double t1[3], t2[3];
      orc_tangents(k->n, t1, t2);
      for (int i = 0; i < 3; ++i) {
        c->dir[i] = k->n[i];
        c->dir[3 + i] = t1[i];
        c->dir[6 + i] = t2[i];
        c->ra[i] = k->ra[i];
        c->rb[i] = k->rb[i];
      }
      c->mu = sc->mu[sc->scene[A->body]];
      c->bias[0] = k->phi > 0.0 ? k->phi / h : prm->erp * k->phi / h;
      c->bias[1] = c->bias[2] = 0.0;
    } else {
      int64_t j = c->id;
      const float* an = sc->joint_anchor + 6 * j;
      double Ra[9], Rb[9], aa[3] = {an[0], an[1], an[2]}, ab[3] = {an[3], an[4], an[5]};
      quat_to_mat(A->q, Ra);
      quat_to_mat(B->q, Rb);
      mat3_vec(Ra, aa, c->ra);
      mat3_vec(Rb, ab, c->rb);
      for (int i = 0; i < 9; ++i) c->dir[i] = 0.0;
      for (int r = 0; r < 3; ++r) {
        c->dir[3 * r + r] = -1.0;
        double Ck = (A->x[r] + c->ra[r]) - (B->x[r] + c->rb[r]);
        c->bias[r] = prm->erp * Ck / h;
      }
      c->mu = 0.0;
    }
    for (int r = 0; r < 3; ++r) {
      double* d = c->dir + 3 * r;
      cross3(c->ra, d, c->anga + 3 * r);
      mat3_vec(A->invi, c->anga + 3 * r, c->ka + 3 * r);
      double arr = A->invm * dot3(d, d) + dot3(c->anga + 3 * r, c->ka + 3 * r);
      if (B) {
        cross3(c->rb, d, c->angb + 3 * r);
        mat3_vec(B->invi, c->angb + 3 * r, c->kb + 3 * r);
        arr += B->invm * dot3(d, d) + dot3(c->angb + 3 * r, c->kb + 3 * r);
      }
      arr += prm->cfm;
      c->arr[r] = arr;
      c->invd[r] = 1.0 / arr;
    }
  }

  /* ---- colouring: within a partition two copies conflict when they share
   * a non-static body.  Greedy colouring in descending priority
   * (fmix32(uid ^ seed), uid): each copy takes the smallest colour not used
   * by a conflicting copy already coloured.  This fixes the Gauss-Seidel
   * order (colour, then uid) without changing the method. ---- */
  int max_colours = 0;
  int colour_overflow = 0;
  for (int32_t p = 0; p < G; ++p) {
    int64_t m0 = pcop[p], m1 = pcop[p + 1], nm = m1 - m0;
    int64_t nr = prep[p + 1] - prep[p];
    if (nm == 0) continue;
    int32_t* ioff = (int32_t*)xalloc((size_t)(nr + 1) * 4);
    int32_t* inc = (int32_t*)xalloc((size_t)(2 * nm) * 4);
    for (int64_t m = m0; m < m1; ++m) {
      ioff[cp[m].ia + 1]++;
      if (cp[m].ib >= 0) ioff[cp[m].ib + 1]++;
    }
    for (int64_t i = 0; i < nr; ++i) ioff[i + 1] += ioff[i];
    int32_t* fill = (int32_t*)xalloc((size_t)(nr + 1) * 4);
    for (int64_t m = m0; m < m1; ++m) {
      inc[ioff[cp[m].ia] + fill[cp[m].ia]++] = (int32_t)m;
      if (cp[m].ib >= 0) inc[ioff[cp[m].ib] + fill[cp[m].ib]++] = (int32_t)m;
    }
    prio_t* pr = (prio_t*)xalloc((size_t)nm * sizeof(prio_t));
    for (int64_t m = m0; m < m1; ++m) {
      /* conflict degree: other copies of the partition sharing a body */
      cp[m].deg = ioff[cp[m].ia + 1] - ioff[cp[m].ia] - 1;
      if (cp[m].ib >= 0) cp[m].deg += ioff[cp[m].ib + 1] - ioff[cp[m].ib] - 1;
      cp[m].colour = -1;
      pr[m - m0].h = orc_fmix32((uint32_t)cp[m].uid ^ prm->seed);
      pr[m - m0].uid = cp[m].uid;
      pr[m - m0].idx = m;
    }
    qsort(pr, (size_t)nm, sizeof(prio_t), cmp_prio_desc);
    for (int64_t t = 0; t < nm; ++t) {
      copy_t* c = &cp[pr[t].idx];
      uint64_t used = 0;
      int32_t ends[2] = {c->ia, c->ib};
      for (int e = 0; e < 2; ++e) {
        if (ends[e] < 0) continue;
        for (int32_t i = ioff[ends[e]]; i < ioff[ends[e] + 1]; ++i) {
          int32_t o = inc[i];
          if (cp[o].colour >= 0) used |= 1ull << cp[o].colour;
        }
      }
      if (used == ~0ull) {
        colour_overflow = 1;
        c->colour = 63;
      } else {
        int col = 0;
        while (used >> col & 1) ++col;
        c->colour = col;
      }
      if (c->colour + 1 > max_colours) max_colours = c->colour + 1;
    }
    free(pr);
    free(fill);
    free(inc);
    free(ioff);
  }

  /* ---- warm start: previous impulses of the same (partition, kind, key);
   * friction is carried as a world vector and projected on the new tangents,
   * then clipped to the new box ---- */
  for (int64_t m = 0; m < M; ++m) {
    copy_t* c = &cp[m];
    c->lam0[0] = c->lam0[1] = c->lam0[2] = 0.0;
    if (!prm->warmstart || !cache || cache->n == 0) continue;
    int64_t f = cache_find(cache, c->part, c->kind, c->key);
    if (f < 0) continue;
    const float* val = cache->val + 4 * f;
    if (c->kind == 0) {
      for (int r = 0; r < 3; ++r) c->lam0[r] = val[r];
    } else {
      double ln = val[0] > 0.0f ? (double)val[0] : 0.0;
      double fw[3] = {val[1], val[2], val[3]};
      double l1 = dot3(fw, c->dir + 3), l2 = dot3(fw, c->dir + 6);
      c->lam0[0] = ln;
      c->lam0[1] = clampd(l1, -c->mu * ln, c->mu * ln);
      c->lam0[2] = clampd(l2, -c->mu * ln, c->mu * ln);
    }
  }

  /* ---- learned warm start (not in the paper; an accelerator that leaves the
   * solve unchanged): per contact copy twelve features of the problem at the
   * start of the step, normalised by the velocity scale g h and the impulse
   * scale s = g h / (1/m_a + 1/m_b); the network predicts lambda / s, which is
   * projected on the contact's bounds.  Joints keep the plain start. ---- */
  {
    double g = sqrt(prm->gx * prm->gx + prm->gy * prm->gy + prm->gz * prm->gz);
    double vs = g * h > 0.0 ? g * h : 1.0;
    for (int64_t m = 0; m < M; ++m) {
      copy_t* c = &cp[m];
      for (int k = 0; k < 13; ++k) c->feat[k] = 0.0;
      for (int r = 0; r < 3; ++r) c->laml[r] = c->lam0[r];
      if (c->kind != 1) continue;
      const replica* A = &rep[prep[c->part] + c->ia];
      const replica* B = c->ib >= 0 ? &rep[prep[c->part] + c->ib] : NULL;
      const contact* k = &cl.c[c->id];
      double pa[3], pb[3] = {0, 0, 0}, t[3];
      cross3(A->vt + 3, c->ra, t);
      for (int i = 0; i < 3; ++i) pa[i] = A->vt[i] + t[i];
      double ima = A->invm, imb = 0.0;
      if (B) {
        cross3(B->vt + 3, c->rb, t);
        for (int i = 0; i < 3; ++i) pb[i] = B->vt[i] + t[i];
        imb = B->invm;
      }
      double vr[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
      double s_imp = vs / (ima + imb);
      double margin = sc->margin[sc->scene[A->body]];
      for (int i = 0; i < 3; ++i) c->feat[i] = c->dir[i];
      c->feat[3] = dot3(vr, c->dir) / vs;
      c->feat[4] = dot3(vr, c->dir + 3) / vs;
      c->feat[5] = dot3(vr, c->dir + 6) / vs;
      c->feat[6] = margin > 0.0 ? k->phi / margin : k->phi;
      c->feat[7] = ima / (ima + imb);
      c->feat[8] = imb / (ima + imb);
      c->feat[9] = c->lam0[0] / s_imp;
      c->feat[10] = sqrt(c->lam0[1] * c->lam0[1] + c->lam0[2] * c->lam0[2]) / s_imp;
      c->feat[11] = c->deg / 16.0;
      c->feat[12] = s_imp;
      if (prm->learned && prm->mlp) {
        double y[3];
        orc_mlp_infer(prm->mlp, c->feat, y);
        double ln = y[0] * s_imp > 0.0 ? y[0] * s_imp : 0.0;
        c->laml[0] = ln;
        c->laml[1] = clampd(y[1] * s_imp, -c->mu * ln, c->mu * ln);
        c->laml[2] = clampd(y[2] * s_imp, -c->mu * ln, c->mu * ln);
      }
    }
  }

  /* ---- projected Gauss-Seidel per partition, colours ascending then uid ---- */
  int32_t* pguard = (int32_t*)xalloc((size_t)(G ? G : 1) * 4);
  double* prho0 = (double*)xalloc((size_t)(G ? G : 1) * 16);
  int32_t* piters = (int32_t*)xalloc((size_t)(G ? G : 1) * 4);
  double* presid = (double*)xalloc((size_t)(G ? G : 1) * 8);
  int unconverged = 0;
  /* The partitions share no replica and no copy: each is solved on its own,
   * like the paper's workers, on up to prm->threads threads. */
  const int nthreads = prm->threads > 1 ? prm->threads : 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : unconverged) if (nthreads > 1)
  for (int32_t p = 0; p < G; ++p) {
    int64_t m0 = pcop[p], m1 = pcop[p + 1], nm = m1 - m0;
    replica* rp = rep + prep[p];
    order_t* od = (order_t*)xalloc((size_t)(nm ? nm : 1) * sizeof(order_t));
    for (int64_t m = m0; m < m1; ++m) {
      od[m - m0].colour = cp[m].colour;
      od[m - m0].uid = cp[m].uid;
      od[m - m0].idx = m;
    }
    qsort(od, (size_t)nm, sizeof(order_t), cmp_order);
    /* with the learned start, keep it only when its initial residual is
     * below the plain start's (the guard) */
    int use_learned = 0;
    if (prm->learned) {
      double rho_p = start_residual(rp, prep[p + 1] - prep[p], cp, od, nm, 0, prm->cfm);
      double rho_l = start_residual(rp, prep[p + 1] - prep[p], cp, od, nm, 1, prm->cfm);
      prho0[2 * p] = rho_p;
      prho0[2 * p + 1] = rho_l;
      use_learned = rho_l < rho_p;
      if (prm->forced_guard && prm->forced_guard[p] >= 0) use_learned = prm->forced_guard[p];
    }
    pguard[p] = use_learned;
    /* warm-start impulses enter the velocities in solve order */
    apply_start(rp, cp, od, nm, use_learned);
    int it = 0;
    double rho = 0.0;
    int cap = forced_iters ? forced_iters[p] : prm->max_iters;
    while (it < cap) {
      rho = 0.0;
      for (int64_t t = 0; t < nm; ++t) {
        copy_t* c = &cp[od[t].idx];
        replica* A = &rp[c->ia];
        replica* B = c->ib >= 0 ? &rp[c->ib] : NULL;
        for (int r = 0; r < 3; ++r) {
          double w = row_velocity(A, B, c, r) + c->bias[r] + prm->cfm * c->lam[r];
          double lo, hi;
          row_bounds(c, r, &lo, &hi);
          double ln = clampd(c->lam[r] - w * c->invd[r], lo, hi);
          double dl = ln - c->lam[r];
          c->lam[r] = ln;
          apply_row(A, B, c, r, dl);
          double e = fabs(dl) * c->arr[r];
          if (e > rho) rho = e;
        }
      }
      ++it;
      if (!forced_iters && prm->adaptive && rho <= prm->tol) break;
    }
    if (!forced_iters && prm->adaptive && nm > 0 && rho > prm->tol) unconverged++;
    piters[p] = it;
    presid[p] = rho;
    free(od);
  }
  put(res, ORC_PART_ITERS, piters, G);
  put(res, ORC_PART_RESID, presid, G);
  put(res, ORC_PART_GUARD, pguard, G);
  put(res, ORC_PART_RHO0, prho0, 2 * G);

  /* ---- exact natural-map residual of the final iterate ---- */
  double rho_exact = 0.0, rho_sum = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    copy_t* c = &cp[m];
    replica* rp = rep + prep[c->part];
    replica* A = &rp[c->ia];
    replica* B = c->ib >= 0 ? &rp[c->ib] : NULL;
    for (int r = 0; r < 3; ++r) {
      double w = row_velocity(A, B, c, r) + c->bias[r] + prm->cfm * c->lam[r];
      double lo, hi;
      row_bounds(c, r, &lo, &hi);
      double e = c->arr[r] * fabs(c->lam[r] - clampd(c->lam[r] - w * c->invd[r], lo, hi));
      if (e > rho_exact) rho_exact = e;
      rho_sum += e;
    }
  }

  /* ---- copy outputs ---- */
  {
    int32_t* kind = (int32_t*)xalloc((size_t)M * 4);
    uint64_t* key = (uint64_t*)xalloc((size_t)M * 8);
    int32_t* ia = (int32_t*)xalloc((size_t)M * 4);
    int32_t* ib = (int32_t*)xalloc((size_t)M * 4);
    int32_t* col = (int32_t*)xalloc((size_t)M * 4);
    double* dir = (double*)xalloc((size_t)M * 72);
    double* ra = (double*)xalloc((size_t)M * 24);
    double* rb = (double*)xalloc((size_t)M * 24);
    double* arr = (double*)xalloc((size_t)M * 24);
    double* bias = (double*)xalloc((size_t)M * 24);
    double* mu = (double*)xalloc((size_t)M * 8);
    double* l0 = (double*)xalloc((size_t)M * 24);
    double* l = (double*)xalloc((size_t)M * 24);
    int32_t* cpart = (int32_t*)xalloc((size_t)M * 4);
    int32_t* ckind = (int32_t*)xalloc((size_t)M * 4);
    uint64_t* ckey = (uint64_t*)xalloc((size_t)M * 8);
    float* cval = (float*)xalloc((size_t)M * 16);
    for (int64_t m = 0; m < M; ++m) {
      copy_t* c = &cp[m];
      kind[m] = c->kind;
      key[m] = c->key;
      ia[m] = c->ia;
      ib[m] = c->ib;
      col[m] = c->colour;
      mu[m] = c->mu;
      for (int i = 0; i < 9; ++i) dir[9 * m + i] = c->dir[i];
      for (int i = 0; i < 3; ++i) {
        ra[3 * m + i] = c->ra[i];
        rb[3 * m + i] = c->rb[i];
        arr[3 * m + i] = c->arr[i];
        bias[3 * m + i] = c->bias[i];
        l0[3 * m + i] = c->lam0[i];
        l[3 * m + i] = c->lam[i];
      }
      cpart[m] = c->part;
      ckind[m] = c->kind;
      ckey[m] = c->key;
      if (c->kind == 0) {
        for (int i = 0; i < 3; ++i) cval[4 * m + i] = (float)c->lam[i];
        cval[4 * m + 3] = 0.0f;
      } else {
        cval[4 * m] = (float)c->lam[0];
        for (int i = 0; i < 3; ++i) cval[4 * m + 1 + i] = (float)(c->lam[1] * c->dir[3 + i] + c->lam[2] * c->dir[6 + i]);
      }
    }
    put(res, ORC_COPY_KIND, kind, M);
    put(res, ORC_COPY_KEY, key, M);
    put(res, ORC_COPY_IA, ia, M);
    put(res, ORC_COPY_IB, ib, M);
    put(res, ORC_COPY_COLOUR, col, M);
    put(res, ORC_COPY_DIR, dir, 9 * M);
    put(res, ORC_COPY_RA, ra, 3 * M);
    put(res, ORC_COPY_RB, rb, 3 * M);
    put(res, ORC_COPY_ARR, arr, 3 * M);
    put(res, ORC_COPY_BIAS, bias, 3 * M);
    put(res, ORC_COPY_MU, mu, M);
    put(res, ORC_COPY_LAMBDA0, l0, 3 * M);
    put(res, ORC_COPY_LAMBDA, l, 3 * M);
    double* feat = (double*)xalloc((size_t)M * 13 * 8);
    double* laml = (double*)xalloc((size_t)M * 24);
    int32_t* deg = (int32_t*)xalloc((size_t)M * 4);
    for (int64_t m = 0; m < M; ++m) {
      for (int k = 0; k < 13; ++k) feat[13 * m + k] = cp[m].feat[k];
      for (int k = 0; k < 3; ++k) laml[3 * m + k] = cp[m].laml[k];
      deg[m] = cp[m].deg;
    }
    put(res, ORC_COPY_FEAT, feat, 13 * M);
    put(res, ORC_COPY_LAMBDAL, laml, 3 * M);
    put(res, ORC_COPY_DEG, deg, M);
    put(res, ORC_CACHE_PART, cpart, M);
    put(res, ORC_CACHE_KIND, ckind, M);
    put(res, ORC_CACHE_KEY, ckey, M);
    put(res, ORC_CACHE_VAL, cval, 4 * M);
  }

  /* ---- replica velocity snapshot and mass data ---- */
  {
    double* vt = (double*)xalloc((size_t)R * 48);
    double* im = (double*)xalloc((size_t)R * 8);
    double* ii = (double*)xalloc((size_t)R * 72);
    for (int64_t r = 0; r < R; ++r) {
      for (int k = 0; k < 6; ++k) vt[6 * r + k] = rep[r].vt[k];
      im[r] = rep[r].invm;
      for (int k = 0; k < 9; ++k) ii[9 * r + k] = rep[r].invi[k];
    }
    put(res, ORC_REP_VT, vt, 6 * R);
    put(res, ORC_REP_INVM, im, R);
    put(res, ORC_REP_INVI, ii, 9 * R);
  }

  /* ---- integration (semi-implicit Euler: positions from the new velocities;
   * q <- normalise(q + h/2 (0, w) q) with w in the world frame) ---- */
  double* rst = (double*)xalloc((size_t)R * 13 * 8);
  for (int64_t r = 0; r < R; ++r) {
    replica* q = &rep[r];
    for (int k = 0; k < 3; ++k) q->x[k] += h * q->v[k];
    double qw = q->q[0], qx = q->q[1], qy = q->q[2], qz = q->q[3];
    double wx = q->w[0], wy = q->w[1], wz = q->w[2];
    double dw = -(wx * qx + wy * qy + wz * qz);
    double dx = wx * qw + (wy * qz - wz * qy);
    double dy = wy * qw + (wz * qx - wx * qz);
    double dz = wz * qw + (wx * qy - wy * qx);
    qw += 0.5 * h * dw;
    qx += 0.5 * h * dx;
    qy += 0.5 * h * dy;
    qz += 0.5 * h * dz;
    double nn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    q->q[0] = qw / nn;
    q->q[1] = qx / nn;
    q->q[2] = qy / nn;
    q->q[3] = qz / nn;
    double* o = rst + 13 * r;
    for (int k = 0; k < 3; ++k) {
      o[k] = q->x[k];
      o[7 + k] = q->v[k];
      o[10 + k] = q->w[k];
    }
    for (int k = 0; k < 4; ++k) o[3 + k] = q->q[k];
  }
  put(res, ORC_REP_STATE, rst, 13 * R);

  /* ---- blending (Alg. 4, Eq. 11-14): replicas in ascending partition id;
   * a quaternion whose dot product with the first one is negative is
   * negated; the weighted quaternion is normalised.  A body active in one
   * partition keeps that partition's state unchanged. ---- */
  double* out = (double*)xalloc((size_t)N * 13 * 8);
  {
    double* sts = (double*)xalloc(64 * 13 * 8);
    double ws[64];
    for (int64_t v = 0; v < N; ++v) {
      int s = sc->scene[v];
      int nw = 0;
      for (int b = 0; b < parts_per_scene[s]; ++b) {
        if (!(mask[v] >> b & 1)) continue;
        int32_t p = pbase[s] + b;
        int64_t r = prep[p] + local_rep(prep, rep_body, p, (int32_t)v);
        memcpy(sts + 13 * nw, rst + 13 * r, 13 * sizeof(double));
        ws[nw++] = repW[r];
      }
      orc_blend(nw, sts, ws, out + 13 * v);
    }
    free(sts);
  }
  put(res, ORC_STATE, out, 13 * N);

  /* ---- joint violation of the blended state (largest and summed norm) ---- */
  double jviol = 0.0, jviol_sum = 0.0;
  for (int64_t j = 0; j < sc->n_joints; ++j) {
    int32_t a = sc->joint_ab[2 * j], b = sc->joint_ab[2 * j + 1];
    const float* an = sc->joint_anchor + 6 * j;
    double Ra[9], Rb[9], aa[3] = {an[0], an[1], an[2]}, ab[3] = {an[3], an[4], an[5]}, pa[3], pb[3];
    quat_to_mat(out + 13 * (int64_t)a + 3, Ra);
    quat_to_mat(out + 13 * (int64_t)b + 3, Rb);
    mat3_vec(Ra, aa, pa);
    mat3_vec(Rb, ab, pb);
    double e2 = 0;
    for (int k = 0; k < 3; ++k) {
      double d = (out[13 * (int64_t)a + k] + pa[k]) - (out[13 * (int64_t)b + k] + pb[k]);
      e2 += d * d;
    }
    if (sqrt(e2) > jviol) jviol = sqrt(e2);
    jviol_sum += sqrt(e2);
  }

  int max_it = 0;
  for (int32_t p = 0; p < G; ++p)
    if (piters[p] > max_it) max_it = piters[p];
  stats[0] = rho_exact;
  stats[1] = rho_sum;
  stats[2] = jviol;
  stats[3] = (double)n_overlap;
  stats[4] = (double)max_colours;
  stats[5] = (double)max_it;
  stats[6] = colour_overflow ? 2.0 : 0.0;
  stats[7] = (double)unconverged;
  stats[8] = jviol_sum;
  if (colour_overflow) snprintf(res->err, sizeof res->err, "more than 64 colours needed");

  free(rep);
  free(cp);
  free(cl.c);
  free(js.k);
  free(ws.stamp);
  free(ws.dist);
  free(ws.queue);
  free(pbase);
  return res;
}

void orc_free(orc_result* r) {
  if (!r) return;
  for (int f = 0; f < ORC_NFIELDS; ++f) free(r->ptr[f]);
  free(r);
}

int64_t orc_len(const orc_result* r, int32_t field) {
  if (!r || field < 0 || field >= ORC_NFIELDS) return -1;
  return r->len[field];
}

const void* orc_ptr(const orc_result* r, int32_t field) {
  if (!r || field < 0 || field >= ORC_NFIELDS) return NULL;
  return r->ptr[field];
}

const char* orc_error(const orc_result* r) { return r ? r->err : "null result"; }
