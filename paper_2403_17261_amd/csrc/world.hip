// C ABI of the library: world lifetime, device buffers, partitions, the step
// sequence with overflow recovery, state I/O and the debug export.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ovl.h"
#include "ovl_internal.h"

using namespace ovl;

namespace {

thread_local std::string g_create_error;

__global__ void k_cols_to_rows(const float* __restrict__ st, float* __restrict__ dst, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int k = 0; k < 13; ++k) dst[13 * (int64_t)i + k] = st[(int64_t)k * N + i];
}

}  // namespace

struct ovl_world {
  WP wp{};
  hipStream_t stream = nullptr;
  ovl_device_ctx ctx{};
  std::string err;
  ovl_params prm{};
  int32_t N = 0, S = 0, J = 0, P = 0, Q = 0, G = 0, T = 0;
  std::vector<int32_t> body_off, joint_off, pps, owner_local;
  std::vector<void*> static_allocs, cap_allocs, part_allocs;
  int32_t* scan_scratch = nullptr;
  bool forced_next = false;
  bool profiling = false;
  // launch configuration, captured step graph
  ovl_launch_cfg launch{1024, 4800, 0, 0};
  int n_cu = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  WP graph_wp{};
  bool graph_valid = false;
  int64_t graph_captures = 0;
  unsigned long long* digest = nullptr;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  double pgs_ms = 0.0;
  int64_t pgs_launches = 0;
  uint16_t* mlp_wb = nullptr;
  float* mlp_bias = nullptr;
  // dynamic load balancing: per-body buffers (allocated at the first enable)
  std::vector<void*> lb_allocs;

  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // fold finished event pairs into the totals (after a stream sync)
  void drain_events() {
    for (auto& pr : ev_pending) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        pgs_ms += ms;
        ++pgs_launches;
      }
      ev_pool.push_back(pr.first);
      ev_pool.push_back(pr.second);
    }
    ev_pending.clear();
  }

  ovl_status fail(ovl_status s, const std::string& msg) {
    err = msg;
    return s;
  }

  void* raw_alloc(size_t bytes) {
    bytes = std::max<size_t>(bytes, 16);
    if (ctx.alloc) return ctx.alloc(bytes, ctx.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
  }
  void raw_free(void* p) {
    if (!p) return;
    if (ctx.free)
      ctx.free(p, ctx.user);
    else
      (void)hipFree(p);
  }
  template <class T_>
  T_* alloc(std::vector<void*>& group, size_t n, bool& ok) {
    if (!ok) return nullptr;
    void* p = raw_alloc(n * sizeof(T_));
    if (!p) {
      ok = false;
      return nullptr;
    }
    group.push_back(p);
    return (T_*)p;
  }
  void free_group(std::vector<void*>& g) {
    for (void* p : g) raw_free(p);
    g.clear();
  }
  ~ovl_world() {
    (void)hipStreamSynchronize(stream);
    drain_events();
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    free_group(part_allocs);
    free_group(cap_allocs);
    free_group(lb_allocs);
    free_group(static_allocs);
  }

  bool upload(void* dst, const void* src, size_t bytes) {
    if (!bytes) return true;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream) == hipSuccess;
  }

  bool alloc_caps(int32_t Ccap, int32_t Mcap, int32_t Rcap, int32_t Acap) {
    bool ok = true;
    auto& g = cap_allocs;
    WP& w = wp;
    w.Ccap = Ccap;
    w.Mcap = Mcap;
    w.Rcap = Rcap;
    w.Acap = Acap;
    w.c_bkey = alloc<uint32_t>(g, Ccap, ok);
    w.c_a = alloc<int32_t>(g, Ccap, ok);
    w.c_geom = alloc<float>(g, (size_t)8 * Ccap, ok);
    w.adj = alloc<int32_t>(g, Acap, ok);
    w.rep_D_bm = alloc<int32_t>(g, Rcap, ok);
    w.rep_pm_of_bm = alloc<int32_t>(g, Rcap, ok);
    w.rep_body_pm = alloc<int32_t>(g, Rcap, ok);
    w.rst = alloc<float>(g, (size_t)13 * Rcap, ok);
    w.rep_w_bm = alloc<float>(g, Rcap, ok);
    w.inc_off = alloc<int32_t>(g, (size_t)2 * Rcap, ok);
    w.inc = alloc<int32_t>(g, (size_t)2 * Mcap, ok);
    w.cp_src = alloc<int32_t>(g, Mcap, ok);
    w.cp_part = alloc<int32_t>(g, Mcap, ok);
    w.cp_ia = alloc<int32_t>(g, Mcap, ok);
    w.cp_ib = alloc<int32_t>(g, Mcap, ok);
    w.cp_colour = alloc<int32_t>(g, Mcap, ok);
    w.cp_slot = alloc<int32_t>(g, Mcap, ok);
    w.cp_inv = alloc<int32_t>(g, Mcap, ok);
    w.r_rec = alloc<float4>(g, (size_t)3 * Mcap + kSlotPad, ok);
    w.r_gen = alloc<float4>(g, w.has_caps ? (size_t)2 * Mcap + kSlotPad : 1, ok);
    w.rep_ax = alloc<float4>(g, w.has_caps ? (size_t)Rcap : 1, ok);
    w.rep_cpl = alloc<float4>(g, (size_t)2 * Rcap, ok);
    w.r_ids = alloc<int2>(g, (size_t)Mcap + kSlotPad, ok);
    w.r_lam = alloc<float4>(g, (size_t)Mcap + kSlotPad, ok);
    w.r_lam0 = alloc<float4>(g, Mcap, ok);
    w.rep_v4 = alloc<float4>(g, (size_t)2 * Rcap, ok);
    w.r_feat = alloc<float>(g, (size_t)kFeatStride * Mcap, ok);
    w.r_lamL = alloc<float4>(g, Mcap, ok);
    w.wc_part = alloc<int32_t>(g, Mcap, ok);
    w.wc_kind = alloc<int32_t>(g, Mcap, ok);
    w.wc_key = alloc<uint64_t>(g, Mcap, ok);
    w.wc_val = alloc<float>(g, (size_t)4 * Mcap, ok);
    w.wc_k64 = alloc<uint64_t>(g, Mcap, ok);
    w.mc_blk[2] = alloc<int32_t>(g, (size_t)(nblocks(Ccap, 256) + 1) * 64, ok);
    w.rep_isc = alloc<float>(g, Rcap, ok);
    w.rep_im = alloc<float2>(g, Rcap, ok);
    return ok;
  }

  bool lb_alloc() {
    if (!lb_allocs.empty()) return true;
    bool ok = true;
    const size_t Np = std::max(N, 1);
    wp.lb_mask = alloc<uint64_t>(lb_allocs, Np, ok);
    wp.lb_queue = alloc<int32_t>(lb_allocs, Np, ok);
    wp.lb_visit = alloc<uint32_t>(lb_allocs, Np / 32 + 1, ok);
    wp.lb_bridge = alloc<uint32_t>(lb_allocs, Np / 32 + 1, ok);
    if (ok) ok = hipMemsetAsync(wp.lb_visit, 0, (Np / 32 + 1) * sizeof(uint32_t), stream) == hipSuccess &&
                 hipStreamSynchronize(stream) == hipSuccess;
    if (!ok) free_group(lb_allocs);
    return ok;
  }

  // carried sets = owners' singletons (the naive start of section 5.4)
  bool lb_reset_to_owners(const std::vector<int32_t>& local) {
    std::vector<uint64_t> m(std::max(N, 1), 0);
    for (int i = 0; i < N; ++i) m[i] = 1ull << local[i];
    return upload(wp.lb_mask, m.data(), (size_t)N * sizeof(uint64_t)) && hipStreamSynchronize(stream) == hipSuccess;
  }

  bool alloc_parts(int32_t G_) {
    bool ok = true;
    auto& g = part_allocs;
    WP& w = wp;
    w.G = G_;
    w.part_force_iters = alloc<int32_t>(g, G_ + 1, ok);
    w.s_part_base = alloc<int32_t>(g, S + 1, ok);
    w.part_scene = alloc<int32_t>(g, G_ + 1, ok);
    w.part_bit = alloc<int32_t>(g, G_ + 1, ok);
    w.g_tmp = alloc<int32_t>(g, G_ + 1, ok);
    for (int k = 0; k < 3; ++k) w.mc_psize[k] = alloc<int32_t>(g, G_ + 1, ok);
    w.part_rep_off = alloc<int32_t>(g, G_ + 1, ok);
    w.part_copy_off = alloc<int32_t>(g, G_ + 1, ok);
    w.part_col_off = alloc<int32_t>(g, (size_t)G_ * kColStride + 1, ok);
    w.part_ncol = alloc<int32_t>(g, G_ + 1, ok);
    w.part_iters = alloc<int32_t>(g, G_ + 1, ok);
    w.part_nstatic = alloc<int32_t>(g, G_ + 1, ok);
    w.part_guard = alloc<int32_t>(g, G_ + 1, ok);
    w.part_rho0 = alloc<float>(g, 2 * (size_t)G_ + 2, ok);
    w.part_force_guard = alloc<int32_t>(g, G_ + 1, ok);
    w.part_resid = alloc<float>(g, G_ + 1, ok);
    w.part_rsum = alloc<float>(g, G_ + 1, ok);
    w.part_order = alloc<int32_t>(g, G_ + 1, ok);
    w.wc_off = alloc<int32_t>(g, G_ + 1, ok);
    return ok;
  }

  void set_params(const ovl_params& p) {
    prm = p;
    wp.dt = p.dt;
    wp.gx = p.gravity[0];
    wp.gy = p.gravity[1];
    wp.gz = p.gravity[2];
    wp.cfm = p.cfm;
    wp.erp = p.erp;
    wp.tol = p.tol;
    wp.max_iters = p.max_iters;
    wp.adaptive = p.mode == OVL_MODE_ADAPTIVE;
    wp.warmstart = p.warmstart == OVL_WARM_PLAIN;
    wp.seed = p.seed;
    wp.equal_w = p.weights == OVL_WEIGHTS_EQUAL ? 1 : 0;
    wp.couple = p.coupling == OVL_COUPLING_PREV_IMPULSE ? 1 : 0;
    wp.msplit = p.coupling == OVL_COUPLING_MASS_SPLIT ? 1 : 0;
  }

  bool read_scal(int32_t* out) {
    if (hipMemcpyAsync(out, wp.scal, SC_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, stream) != hipSuccess)
      return false;
    return hipStreamSynchronize(stream) == hipSuccess;
  }

  bool write_scal(int idx, int32_t v) {
    return hipMemcpyAsync(wp.scal + idx, &v, sizeof(v), hipMemcpyHostToDevice, stream) == hipSuccess &&
           hipStreamSynchronize(stream) == hipSuccess;
  }

  hipError_t enqueue_step(hipStream_t s, bool exact, bool timed) {
    hipError_t e;
    if ((e = launch_collide(wp, scan_scratch, s))) return e;
    if ((e = launch_graph(wp, scan_scratch, s))) return e;
    if ((e = launch_solve_pre(wp, s))) return e;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      e0 = take_event();
      e1 = take_event();
      if (e0 && e1) ev_pending.emplace_back(e0, e1);
    }
    if ((e = launch_pgs(wp, s, e0, e1))) return e;
    return launch_solve_post(wp, s, exact);
  }

  // Capture one step (as the parameters stand) into a graph.  The parameter
  // block is baked into the kernel nodes, so the graph is captured again
  // whenever it changes (new buffers, parameters, partitions, modes).
  hipError_t capture() {
    hipError_t e;
    if (!cap_stream && (e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking))) return e;
    if (gexec) {
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
    graph_valid = false;
    if ((e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal))) return e;
    hipError_t le = enqueue_step(cap_stream, false, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap_stream, &g);
    if (le) e = le;
    if (e) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e) {
      gexec = nullptr;
      return e;
    }
    graph_wp = wp;
    graph_valid = true;
    ++graph_captures;
    return hipSuccess;
  }

  hipError_t run_one(bool exact) {
    if (launch.graph && !wp.forced && !exact && !profiling) {
      if (!graph_valid || memcmp(&graph_wp, &wp, sizeof(WP)) != 0) {
        hipError_t e = capture();
        if (e) return e;
      }
      return hipGraphLaunch(gexec, stream);
    }
    return enqueue_step(stream, exact, profiling);
  }

  // apply a launch configuration (validated by the caller)
  bool apply_launch(const ovl_launch_cfg& c, int cfg) {
    int per_lds = 0, per_glob = 0;
    if (pgs_occupancy(cfg, wp.has_caps != 0, wp.msplit != 0, &per_lds, &per_glob) != hipSuccess) return false;
    launch = c;
    wp.pgs_cfg = cfg;
    wp.pgs_persistent = c.persistent ? 1 : 0;
    wp.pgs_grid[0] = std::max(1, per_lds) * std::max(1, n_cu);
    wp.pgs_grid[1] = std::max(1, per_glob) * std::max(1, n_cu);
    return true;
  }

  // Grow every buffer whose count exceeded its capacity (device counts are exact).
  bool grow(const int32_t* sc) {
    int32_t C = std::max(wp.Ccap, (int32_t)std::ceil(1.5 * sc[SC_NCONTACT]) + 1024);
    int32_t A = std::max(wp.Acap, 2 * C + 2 * J);
    int32_t R = std::max(wp.Rcap, (int32_t)std::ceil(1.5 * sc[SC_NREP]) + 1024);
    int32_t M = std::max(wp.Mcap, (int32_t)std::ceil(1.5 * sc[SC_NCOPY]) + 1024);
    M = std::max(M, 2 * (C + J) + 1024);
    if (hipStreamSynchronize(stream) != hipSuccess) return false;
    // the warm-start cache of the last committed step moves to the new buffers
    const WP old = wp;
    const int64_t keep = std::min(sc[SC_PREV_NCOPY], old.Mcap);
    std::vector<void*> old_allocs;
    old_allocs.swap(cap_allocs);
    bool ok = alloc_caps(C, M, R, A);
    auto d2d = [&](void* dst, const void* src, size_t bytes) {
      ok = ok && (bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream) == hipSuccess);
    };
    d2d(wp.wc_part, old.wc_part, keep * sizeof(int32_t));
    d2d(wp.wc_kind, old.wc_kind, keep * sizeof(int32_t));
    d2d(wp.wc_key, old.wc_key, keep * sizeof(uint64_t));
    d2d(wp.wc_k64, old.wc_k64, keep * sizeof(uint64_t));
    for (int k = 0; k < 4; ++k) d2d(wp.wc_val + (size_t)k * wp.Mcap, old.wc_val + (size_t)k * old.Mcap, keep * sizeof(float));
    ok = ok && hipStreamSynchronize(stream) == hipSuccess;
    free_group(old_allocs);
    return ok;
  }
};

namespace {

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

ovl_status validate_params(const ovl_params* p, std::string& err) {
  if (!p) {
    err = "params is NULL";
    return OVL_ERR_INVALID_ARG;
  }
  if (!(p->dt > 0.0f) || !std::isfinite(p->dt)) err = "dt must be > 0";
  else if (!(p->cfm >= 0.0f)) err = "cfm must be >= 0";
  else if (!(p->erp >= 0.0f && p->erp <= 1.0f)) err = "erp must be in [0,1]";
  else if (p->max_iters < 1 || p->max_iters > 100000) err = "max_iters must be in [1,100000]";
  else if (p->mode != OVL_MODE_FIXED && p->mode != OVL_MODE_ADAPTIVE) err = "bad mode";
  else if (p->warmstart != OVL_WARM_NONE && p->warmstart != OVL_WARM_PLAIN) err = "bad warmstart mode";
  else if (!(p->tol >= 0.0f)) err = "tol must be >= 0";
  else if (p->weights != OVL_WEIGHTS_GEODESIC && p->weights != OVL_WEIGHTS_EQUAL) err = "bad weights mode";
  else if (p->coupling != OVL_COUPLING_NONE && p->coupling != OVL_COUPLING_PREV_IMPULSE &&
           p->coupling != OVL_COUPLING_MASS_SPLIT)
    err = "bad coupling mode";
  else if (!std::isfinite(p->gravity[0]) || !std::isfinite(p->gravity[1]) || !std::isfinite(p->gravity[2]))
    err = "gravity must be finite";
  else
    return OVL_OK;
  return OVL_ERR_INVALID_ARG;
}

ovl_status set_partitions_impl(ovl_world* w, const int32_t* owner, const int32_t* pps, int32_t halo_k,
                               int32_t beta) {
  const int S = w->S, N = w->N;
  std::vector<int32_t> base(S + 1, 0);
  for (int s = 0; s < S; ++s) {
    if (pps[s] < 1 || pps[s] > kMaxParts) return w->fail(OVL_ERR_INVALID_ARG, "parts_per_scene out of [1,64]");
    base[s + 1] = base[s] + pps[s];
  }
  if (halo_k < 1 || halo_k > 64) return w->fail(OVL_ERR_INVALID_ARG, "halo_k must be in [1,64]");
  if (beta < 1 || beta > 16) return w->fail(OVL_ERR_INVALID_ARG, "beta must be in [1,16]");
  std::vector<int32_t> local(N);
  for (int s = 0; s < S; ++s)
    for (int i = w->body_off[s]; i < w->body_off[s + 1]; ++i) {
      int o = owner[i] - base[s];
      if (o < 0 || o >= pps[s]) return w->fail(OVL_ERR_INVALID_ARG, "owner of body " + std::to_string(i) +
                                                                        " outside its scene's partitions");
      local[i] = o;
    }
  const int G = base[S];
  std::vector<int32_t> pscene(G), pbit(G);
  for (int s = 0; s < S; ++s)
    for (int b = 0; b < pps[s]; ++b) {
      pscene[base[s] + b] = s;
      pbit[base[s] + b] = b;
    }
  if (hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "stream sync failed");
  if (G != w->G) {
    w->free_group(w->part_allocs);
    if (!w->alloc_parts(G)) return w->fail(OVL_ERR_OOM, "partition buffers");
    w->forced_next = false;
    w->wp.force_guard = 0;
  }
  bool ok = w->upload((void*)w->wp.owner_local, local.data(), N * sizeof(int32_t)) &&
            w->upload((void*)w->wp.s_part_base, base.data(), (S + 1) * sizeof(int32_t)) &&
            w->upload((void*)w->wp.part_scene, pscene.data(), G * sizeof(int32_t)) &&
            w->upload((void*)w->wp.part_bit, pbit.data(), G * sizeof(int32_t));
  if (!ok || hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "upload failed");
  w->G = G;
  w->pps.assign(pps, pps + S);
  w->wp.halo_k = halo_k;
  w->wp.beta = beta;
  w->owner_local.assign(local.begin(), local.end());
  if (w->wp.lb_on && !w->lb_reset_to_owners(w->owner_local)) return w->fail(OVL_ERR_DEVICE, "upload failed");
  return OVL_OK;
}

}  // namespace

extern "C" {

const char* ovl_version(void) { return "ovl 0.1 (gfx950)"; }

const char* ovl_last_error(const ovl_world* w) { return w ? w->err.c_str() : g_create_error.c_str(); }

ovl_status ovl_create_world(const ovl_world_desc* d, const ovl_params* params, const ovl_device_ctx* ctx,
                            ovl_world** out) {
  g_create_error.clear();
  auto bad = [](const std::string& m) {
    g_create_error = m;
    return OVL_ERR_INVALID_ARG;
  };
  if (!out) return bad("out is NULL");
  *out = nullptr;
  if (!d) return bad("desc is NULL");
  std::string perr;
  if (validate_params(params, perr) != OVL_OK) return bad(perr);
  const int N = d->n_bodies, S = d->n_scenes, J = d->n_joints;
  if (N < 0 || S < 1 || J < 0) return bad("n_bodies >= 0, n_scenes >= 1, n_joints >= 0 required");
  if (N > (1 << 28)) return bad("too many bodies");
  if (N > 0 && (!d->scene || !d->shape || !d->radius || !d->mass || !d->inertia || !d->state))
    return bad("body arrays must not be NULL");
  if (!d->mu || !d->margin || !d->plane_off || !d->ssph_off) return bad("scene arrays must not be NULL");
  if (J > 0 && (!d->joint_ab || !d->joint_anchor)) return bad("joint arrays must not be NULL");
  std::vector<int32_t> body_off(S + 1, 0), joint_off(S + 1, 0);
  float rmax = 0.0f, mmax = 0.0f;
  bool has_caps = false;
  for (int i = 0; i < N; ++i) {
    int s = d->scene[i];
    if (s < 0 || s >= S || (i > 0 && s < d->scene[i - 1])) return bad("scene ids must be nondecreasing in [0,S)");
    if (d->shape[i] != 0 && d->shape[i] != 1) return bad("shape must be 0 (sphere) or 1 (capsule)");
    if (!(d->radius[i] > 0.0f) || !std::isfinite(d->radius[i])) return bad("radius must be > 0");
    if (!(d->mass[i] > 0.0f) || !std::isfinite(d->mass[i])) return bad("mass must be > 0");
    const float* I = d->inertia + 3 * (size_t)i;
    float bound = d->radius[i];
    if (d->shape[i] == 1) {
      if (!d->halflen || !(d->halflen[i] > 0.0f) || !std::isfinite(d->halflen[i]))
        return bad("a capsule needs a half-length > 0 (body " + std::to_string(i) + ")");
      if (!(I[0] > 0.0f) || !(I[2] > 0.0f) || !std::isfinite(I[0]) || !std::isfinite(I[2]) ||
          std::fabs(I[1] - I[0]) > 1e-6f * I[0])
        return bad("capsule inertia must be > 0 and symmetric about the body z axis (body " + std::to_string(i) +
                   ")");
      bound += d->halflen[i];
      has_caps = true;
    } else if (!(I[0] > 0.0f) || !std::isfinite(I[0]) || std::fabs(I[1] - I[0]) > 1e-6f * I[0] ||
               std::fabs(I[2] - I[0]) > 1e-6f * I[0]) {
      return bad("sphere inertia must be isotropic and > 0 (body " + std::to_string(i) + ")");
    }
    body_off[s + 1]++;
    rmax = std::max(rmax, bound);
  }
  if (N > 0 && !finite_all(d->state, (size_t)13 * N)) return bad("state has non-finite values");
  for (int s = 0; s < S; ++s) body_off[s + 1] += body_off[s];
  for (int s = 0; s < S; ++s) {
    if (!(d->mu[s] >= 0.0f) || !(d->margin[s] >= 0.0f)) return bad("mu and margin must be >= 0");
    if (d->plane_off[s + 1] < d->plane_off[s] || d->ssph_off[s + 1] < d->ssph_off[s])
      return bad("plane_off / ssph_off must be nondecreasing");
    mmax = std::max(mmax, d->margin[s]);
  }
  if (d->plane_off[0] != 0 || d->ssph_off[0] != 0) return bad("plane_off[0] and ssph_off[0] must be 0");
  const int P = d->plane_off[S], Q = d->ssph_off[S];
  if ((P > 0 && !d->planes) || (Q > 0 && !d->ssph)) return bad("static arrays must not be NULL");
  std::vector<std::vector<int32_t>> jad(N), jin(N);
  for (int j = 0; j < J; ++j) {
    int a = d->joint_ab[2 * j], b = d->joint_ab[2 * j + 1];
    if (a < 0 || a >= N || b < 0 || b >= N || a == b) return bad("joint body index out of range");
    if (d->scene[a] != d->scene[b]) return bad("joints must join bodies of one scene");
    if (j > 0 && d->scene[a] < d->scene[d->joint_ab[2 * j - 2]]) return bad("joints must be sorted by scene");
    joint_off[d->scene[a] + 1]++;
    jad[a].push_back(b);
    jad[b].push_back(a);
    jin[a].push_back(j);
    jin[b].push_back(j);
  }
  for (int s = 0; s < S; ++s) joint_off[s + 1] += joint_off[s];
  std::vector<int32_t> jadj_off(N + 1, 0), jadj;
  for (int i = 0; i < N; ++i) {
    std::sort(jad[i].begin(), jad[i].end());
    jadj_off[i + 1] = jadj_off[i] + (int32_t)jad[i].size();
    jadj.insert(jadj.end(), jad[i].begin(), jad[i].end());
  }
  std::vector<int32_t> jinc_off(N + 1, 0), jinc;
  for (int i = 0; i < N; ++i) {
    jinc_off[i + 1] = jinc_off[i] + (int32_t)jin[i].size();
    jinc.insert(jinc.end(), jin[i].begin(), jin[i].end());
  }

  ovl_world* w = new ovl_world();
  if (ctx) w->ctx = *ctx;
  w->stream = (hipStream_t)w->ctx.stream;
  w->N = N;
  w->S = S;
  w->J = J;
  w->P = P;
  w->Q = Q;
  w->body_off = body_off;
  w->joint_off = joint_off;
  int T = 64;
  while (T < 2 * N) T <<= 1;
  w->T = T;
  WP& wp = w->wp;
  wp.N = N;
  wp.S = S;
  wp.J = J;
  wp.P = P;
  wp.Q = Q;
  wp.T = T;
  wp.cs = std::max(1.02f * (2.0f * rmax + mmax), 1e-3f);
  wp.has_caps = has_caps ? 1 : 0;
  for (int s = 0; s < S; ++s) {
    const int ns = body_off[s + 1] - body_off[s];
    if (ns <= kLbLdsCap)
      wp.lb_lds_max = std::max(wp.lb_lds_max, ns);
    else
      wp.lb_big = 1;
  }
  w->set_params(*params);
  bool ok = true;
  auto& g = w->static_allocs;
  const int Np = std::max(N, 1);
  int32_t* b_scene = w->alloc<int32_t>(g, Np, ok);
  float* b_radius = w->alloc<float>(g, Np, ok);
  float* b_invm = w->alloc<float>(g, Np, ok);
  float* b_invI = w->alloc<float>(g, Np, ok);
  float* b_half = w->alloc<float>(g, Np, ok);
  float* b_dI = w->alloc<float>(g, Np, ok);
  float* s_mu = w->alloc<float>(g, S, ok);
  float* s_margin = w->alloc<float>(g, S, ok);
  int32_t* s_plane_off = w->alloc<int32_t>(g, S + 1, ok);
  float* planes = w->alloc<float>(g, 4 * (size_t)std::max(P, 1), ok);
  int32_t* s_ssph_off = w->alloc<int32_t>(g, S + 1, ok);
  float* ssph = w->alloc<float>(g, 4 * (size_t)std::max(Q, 1), ok);
  int32_t* s_body_off = w->alloc<int32_t>(g, S + 1, ok);
  int32_t* s_joint_off = w->alloc<int32_t>(g, S + 1, ok);
  int32_t* j_ab = w->alloc<int32_t>(g, 2 * (size_t)std::max(J, 1), ok);
  float* j_anchor = w->alloc<float>(g, 6 * (size_t)std::max(J, 1), ok);
  int32_t* jadj_off_d = w->alloc<int32_t>(g, N + 1, ok);
  int32_t* jadj_d = w->alloc<int32_t>(g, std::max<size_t>(jadj.size(), 1), ok);
  int32_t* jinc_off_d = w->alloc<int32_t>(g, N + 1, ok);
  int32_t* jinc_d = w->alloc<int32_t>(g, std::max<size_t>(jinc.size(), 1), ok);
  wp.joint_viol = w->alloc<float>(g, std::max(J, 1), ok);
  wp.owner_local = w->alloc<int32_t>(g, Np, ok);
  wp.st = w->alloc<float>(g, (size_t)13 * Np, ok);
  wp.cell = w->alloc<int32_t>(g, (size_t)3 * Np, ok);
  wp.bucket = w->alloc<uint32_t>(g, Np, ok);
  wp.bcount = w->alloc<int32_t>(g, T + 1, ok);
  wp.bstart = w->alloc<int32_t>(g, T + 1, ok);
  wp.bfill = w->alloc<int32_t>(g, T, ok);
  wp.bbody = w->alloc<int32_t>(g, Np, ok);
  wp.srt_cell = w->alloc<int4>(g, Np, ok);
  wp.srt_pos = w->alloc<float4>(g, Np, ok);
  wp.ccount = w->alloc<int32_t>(g, N + 1, ok);
  wp.c_keep = w->alloc<uint32_t>(g, (size_t)kKeep * Np, ok);
  wp.coff = w->alloc<int32_t>(g, N + 1, ok);
  wp.deg = w->alloc<int32_t>(g, N + 1, ok);
  wp.adj_off = w->alloc<int32_t>(g, N + 1, ok);
  wp.adj_fill = w->alloc<int32_t>(g, Np, ok);
  wp.mask = w->alloc<uint64_t>(g, Np, ok);
  wp.mask_tmp = w->alloc<uint64_t>(g, Np, ok);
  wp.reach = w->alloc<uint64_t>(g, Np, ok);
  wp.reach_tmp = w->alloc<uint64_t>(g, Np, ok);
  wp.rep_cnt = w->alloc<int32_t>(g, N + 1, ok);
  wp.rep_off_bm = w->alloc<int32_t>(g, N + 1, ok);
  wp.mc_blk[0] = w->alloc<int32_t>(g, (size_t)(nblocks(N, 256) + 1) * 64, ok);
  wp.mc_blk[1] = w->alloc<int32_t>(g, (size_t)(nblocks(J, 256) + 1) * 64, ok);
  for (int k = 0; k < 3; ++k) wp.mc_rank0[k] = w->alloc<int32_t>(g, (size_t)(S + 1) * 64, ok);
  wp.scal = w->alloc<int32_t>(g, SC_COUNT, ok);
  wp.stat_f = w->alloc<float>(g, 4, ok);
  wp.stat_i64 = w->alloc<int64_t>(g, 8, ok);
  wp.pgs_queue = w->alloc<int32_t>(g, 2, ok);
  w->digest = w->alloc<unsigned long long>(g, 1, ok);
  const size_t scan_n = std::max<size_t>({(size_t)T + 1, (size_t)N + 1, (size_t)64 * S + 1});
  w->scan_scratch = w->alloc<int32_t>(g, scan_scratch_ints((int64_t)scan_n) + 16, ok);
  const int32_t Ccap = std::max(1024, 8 * N);
  const int32_t Acap = 2 * Ccap + 2 * J;
  const int32_t Mcap = 2 * (Ccap + J) + 1024;
  const int32_t Rcap = 3 * N + 1024;
  if (!ok || !w->alloc_caps(Ccap, Mcap, Rcap, Acap)) {
    delete w;
    g_create_error = "device allocation failed";
    return OVL_ERR_OOM;
  }
  // host-side transforms of the inputs
  std::vector<float> invm(Np, 0.0f), invI(Np, 0.0f), half(Np, 0.0f), dI(Np, 0.0f), st_cols((size_t)13 * Np, 0.0f);
  for (int i = 0; i < N; ++i) {
    invm[i] = 1.0f / d->mass[i];
    invI[i] = 1.0f / d->inertia[3 * (size_t)i];
    if (d->shape[i] == 1) {
      half[i] = d->halflen[i];
      dI[i] = 1.0f / d->inertia[3 * (size_t)i + 2] - invI[i];
    }
    for (int k = 0; k < 13; ++k) st_cols[(size_t)k * N + i] = d->state[13 * (size_t)i + k];
  }
  wp.b_scene = b_scene;
  wp.b_radius = b_radius;
  wp.b_invm = b_invm;
  wp.b_invI = b_invI;
  wp.b_half = b_half;
  wp.b_dI = b_dI;
  wp.s_mu = s_mu;
  wp.s_margin = s_margin;
  wp.s_plane_off = s_plane_off;
  wp.planes = planes;
  wp.s_ssph_off = s_ssph_off;
  wp.ssph = ssph;
  wp.s_body_off = s_body_off;
  wp.s_joint_off = s_joint_off;
  wp.j_ab = j_ab;
  wp.j_anchor = j_anchor;
  wp.jadj_off = jadj_off_d;
  wp.jadj = jadj_d;
  wp.jinc_off = jinc_off_d;
  wp.jinc = jinc_d;
  std::vector<int32_t> zeros(SC_COUNT, 0);
  std::vector<int64_t> zeros64(8, 0);
  ok = w->upload(b_scene, d->scene, N * sizeof(int32_t)) && w->upload(b_radius, d->radius, N * sizeof(float)) &&
       w->upload(b_invm, invm.data(), N * sizeof(float)) && w->upload(b_invI, invI.data(), N * sizeof(float)) &&
       w->upload(b_half, half.data(), N * sizeof(float)) && w->upload(b_dI, dI.data(), N * sizeof(float)) &&
       w->upload(s_mu, d->mu, S * sizeof(float)) && w->upload(s_margin, d->margin, S * sizeof(float)) &&
       w->upload(s_plane_off, d->plane_off, (S + 1) * sizeof(int32_t)) &&
       w->upload(planes, d->planes, (size_t)4 * P * sizeof(float)) &&
       w->upload(s_ssph_off, d->ssph_off, (S + 1) * sizeof(int32_t)) &&
       w->upload(ssph, d->ssph, (size_t)4 * Q * sizeof(float)) &&
       w->upload(s_body_off, body_off.data(), (S + 1) * sizeof(int32_t)) &&
       w->upload(s_joint_off, joint_off.data(), (S + 1) * sizeof(int32_t)) &&
       w->upload(j_ab, d->joint_ab, (size_t)2 * J * sizeof(int32_t)) &&
       w->upload(j_anchor, d->joint_anchor, (size_t)6 * J * sizeof(float)) &&
       w->upload(jadj_off_d, jadj_off.data(), (N + 1) * sizeof(int32_t)) &&
       w->upload(jadj_d, jadj.data(), jadj.size() * sizeof(int32_t)) &&
       w->upload(jinc_off_d, jinc_off.data(), (N + 1) * sizeof(int32_t)) &&
       w->upload(jinc_d, jinc.data(), jinc.size() * sizeof(int32_t)) &&
       w->upload(wp.st, st_cols.data(), (size_t)13 * N * sizeof(float)) &&
       w->upload(wp.scal, zeros.data(), SC_COUNT * sizeof(int32_t)) &&
       w->upload(wp.stat_i64, zeros64.data(), 8 * sizeof(int64_t));
  if (!ok || hipStreamSynchronize(w->stream) != hipSuccess) {
    delete w;
    g_create_error = "upload failed";
    return OVL_ERR_DEVICE;
  }
  static bool attrs = false;
  if (!attrs) {
    if (pgs_set_attributes() != hipSuccess || lb_set_attributes() != hipSuccess) {
      delete w;
      g_create_error = "could not raise the LDS limit of the solver kernel";
      return OVL_ERR_DEVICE;
    }
    attrs = true;
  }
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      w->n_cu = prop.multiProcessorCount;
      w->wp.n_cu = prop.multiProcessorCount;
    }
    if (!w->apply_launch(w->launch, 0)) {
      delete w;
      g_create_error = "could not query the occupancy of the solver kernels";
      return OVL_ERR_DEVICE;
    }
  }
  // one partition per scene until ovl_set_partitions
  std::vector<int32_t> owner(Np, 0), pps(S, 1);
  for (int i = 0; i < N; ++i) owner[i] = d->scene[i];
  ovl_status st = set_partitions_impl(w, owner.data(), pps.data(), 1, 4);
  if (st != OVL_OK) {
    g_create_error = w->err;
    delete w;
    return st;
  }
  *out = w;
  return OVL_OK;
}

void ovl_destroy_world(ovl_world* w) { delete w; }

ovl_status ovl_set_params(ovl_world* w, const ovl_params* params) {
  if (!w) return OVL_ERR_INVALID_ARG;
  std::string e;
  if (validate_params(params, e) != OVL_OK) return w->fail(OVL_ERR_INVALID_ARG, e);
  w->set_params(*params);
  // mass splitting runs other solver variants: size the persistent grid for them
  if (!w->apply_launch(w->launch, w->wp.pgs_cfg)) return w->fail(OVL_ERR_DEVICE, "occupancy query failed");
  return OVL_OK;
}

ovl_status ovl_set_partitions(ovl_world* w, const int32_t* owner, int64_t n_bodies, const int32_t* parts_per_scene,
                              int32_t n_scenes, int32_t halo_k, int32_t beta) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (n_bodies != w->N || n_scenes != w->S) return w->fail(OVL_ERR_INVALID_ARG, "n_bodies/n_scenes mismatch");
  if ((w->N > 0 && !owner) || !parts_per_scene) return w->fail(OVL_ERR_INVALID_ARG, "NULL array");
  return set_partitions_impl(w, owner, parts_per_scene, halo_k, beta);
}

ovl_status ovl_set_load_balance(ovl_world* w, int32_t enable, int32_t depth, const uint64_t* sets,
                                int64_t n_sets) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (enable != 0 && enable != 1) return w->fail(OVL_ERR_INVALID_ARG, "enable must be 0 or 1");
  if (!enable) {
    w->wp.lb_on = 0;
    return OVL_OK;
  }
  if (depth < 0 || depth > 64) return w->fail(OVL_ERR_INVALID_ARG, "depth must be in [0,64]");
  if (sets && n_sets != w->N) return w->fail(OVL_ERR_INVALID_ARG, "sets must have n_bodies entries");
  if (sets)
    for (int s = 0; s < w->S; ++s)
      for (int i = w->body_off[s]; i < w->body_off[s + 1]; ++i)
        if (sets[i] == 0 || (w->pps[s] < 64 && (sets[i] >> w->pps[s]) != 0))
          return w->fail(OVL_ERR_INVALID_ARG, "set of body " + std::to_string(i) +
                                                  " is empty or names a partition outside its scene");
  if (hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "sync failed");
  if (!w->lb_alloc()) return w->fail(OVL_ERR_OOM, "load-balancing buffers");
  bool ok = sets ? w->upload(w->wp.lb_mask, sets, (size_t)w->N * sizeof(uint64_t))
                 : w->lb_reset_to_owners(w->owner_local);
  if (!ok || hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "upload failed");
  w->wp.lb_on = 1;
  w->wp.lb_depth = depth;
  return OVL_OK;
}

ovl_status ovl_force_iters(ovl_world* w, const int32_t* iters, int32_t n_parts) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (!iters) {
    w->forced_next = false;
    return OVL_OK;
  }
  if (n_parts != w->G) return w->fail(OVL_ERR_INVALID_ARG, "n_parts differs from the partition count");
  for (int g = 0; g < n_parts; ++g)
    if (iters[g] < 0 || iters[g] > 100000) return w->fail(OVL_ERR_INVALID_ARG, "iters out of [0,100000]");
  if (!w->upload((void*)w->wp.part_force_iters, iters, n_parts * sizeof(int32_t)) ||
      hipStreamSynchronize(w->stream) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "upload failed");
  w->forced_next = true;
  return OVL_OK;
}

static ovl_status run_steps(ovl_world* w, int32_t n, bool exact_last) {
  for (int i = 0; i < n; ++i) {
    w->wp.forced = w->forced_next ? 1 : 0;
    hipError_t e = w->run_one(exact_last && i == n - 1);
    w->wp.forced = 0;
    w->forced_next = false;
    if (e != hipSuccess) return w->fail(OVL_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  }
  return OVL_OK;
}

static ovl_status take_flags(ovl_world* w, int32_t flags) {
  if (!flags) return OVL_OK;
  w->write_scal(SC_FLAGS, 0);
  w->write_scal(SC_PREV_NCOPY, 0);
  if (flags & F_NONFINITE) return w->fail(OVL_ERR_NONFINITE, "a step produced non-finite values; state kept");
  if (flags & F_COLOUR_CAP) return w->fail(OVL_ERR_CAPACITY, "a partition needs more than 64 colours");
  return w->fail(OVL_ERR_CAPACITY, "per-step buffer overflow (flags " + std::to_string(flags) + ")");
}

ovl_status ovl_step(ovl_world* w, int32_t n_steps, ovl_step_stats* stats, int32_t compute_exact_residual) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (n_steps < 0) return w->fail(OVL_ERR_INVALID_ARG, "n_steps < 0");
  if (!stats) return run_steps(w, n_steps, false);
  int32_t sc[SC_COUNT];
  if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "sync failed");
  if (sc[SC_FLAGS]) {
    ovl_status s = take_flags(w, sc[SC_FLAGS]);
    if (s != OVL_OK) return s;
  }
  int64_t it0[4];
  if (hipMemcpy(it0, w->wp.stat_i64, sizeof(it0), hipMemcpyDeviceToHost) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "copy failed");
  const int32_t committed0 = sc[SC_COMMITTED];
  const bool forced = w->forced_next;
  std::vector<int32_t> saved_force;
  if (forced) {
    saved_force.resize(w->G);
    (void)hipMemcpy(saved_force.data(), w->wp.part_force_iters, w->G * sizeof(int32_t), hipMemcpyDeviceToHost);
  }
  ovl_status st = run_steps(w, n_steps, compute_exact_residual != 0);
  if (st != OVL_OK) return st;
  if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "step failed on the device");
  if (sc[SC_FLAGS] & (F_CONTACT_CAP | F_ADJ_CAP | F_REP_CAP | F_COPY_CAP)) {
    // grow, then run the steps that did not commit once more (the state is that of the last good step)
    int done = sc[SC_COMMITTED] - committed0;
    if (!w->grow(sc)) return w->fail(OVL_ERR_OOM, "could not grow the per-step buffers");
    w->write_scal(SC_FLAGS, 0);
    if (forced && done == 0) {
      (void)ovl_force_iters(w, saved_force.data(), w->G);
    }
    st = run_steps(w, n_steps - done, compute_exact_residual != 0);
    if (st != OVL_OK) return st;
    if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "step failed on the device");
  }
  if (sc[SC_FLAGS]) return take_flags(w, sc[SC_FLAGS]);
  std::vector<int32_t> iters(w->G), ncol(w->G);
  std::vector<float> resid(w->G);
  int64_t it1[4];
  float sf[4];
  bool ok = hipMemcpy(iters.data(), w->wp.part_iters, w->G * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(ncol.data(), w->wp.part_ncol, w->G * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(resid.data(), w->wp.part_resid, w->G * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(it1, w->wp.stat_i64, sizeof(it1), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(sf, w->wp.stat_f, sizeof(sf), hipMemcpyDeviceToHost) == hipSuccess;
  if (!ok) return w->fail(OVL_ERR_DEVICE, "copy failed");
  memset(stats, 0, sizeof(*stats));
  stats->n_contacts = sc[SC_NCONTACT];
  stats->n_copies = sc[SC_NCOPY];
  stats->n_replicas = sc[SC_NREP];
  stats->n_overlap = sc[SC_NOVERLAP];
  stats->n_lb_changes = sc[SC_LB_CHANGES];
  stats->steps = n_steps;
  stats->iters_total = it1[0] - it0[0];
  stats->n_unconverged = (int32_t)(it1[1] - it0[1]);
  for (int g = 0; g < w->G; ++g) {
    stats->max_iters = std::max(stats->max_iters, iters[g]);
    stats->max_colours = std::max(stats->max_colours, ncol[g]);
    stats->resid_sweep = std::max(stats->resid_sweep, resid[g]);
  }
  stats->resid_exact = compute_exact_residual ? sf[0] : -1.0f;
  stats->resid_exact_sum = -1.0;
  stats->joint_violation_max = stats->joint_violation_sum = -1.0;
  if (compute_exact_residual) {
    std::vector<float> rs(w->G), jv(w->J);
    if (hipMemcpy(rs.data(), w->wp.part_rsum, w->G * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        (w->J > 0 && hipMemcpy(jv.data(), w->wp.joint_viol, w->J * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess))
      return w->fail(OVL_ERR_DEVICE, "copy failed");
    stats->resid_exact_sum = 0.0;
    for (float x : rs) stats->resid_exact_sum += x;
    stats->joint_violation_max = stats->joint_violation_sum = 0.0;
    for (float x : jv) {
      stats->joint_violation_max = std::max(stats->joint_violation_max, (double)x);
      stats->joint_violation_sum += x;
    }
  }
  if (stats->n_unconverged > 0) return w->fail(OVL_NOT_CONVERGED, "some partitions hit the sweep cap");
  return OVL_OK;
}

ovl_status ovl_set_warmstart(ovl_world* w, int32_t mode, const float* params, int64_t n_params) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (mode == OVL_WARM_NONE || mode == OVL_WARM_PLAIN) {
    w->prm.warmstart = mode;
    w->wp.warmstart = mode == OVL_WARM_PLAIN;
    w->wp.learned = 0;
    return OVL_OK;
  }
  if (mode != OVL_WARM_LEARNED) return w->fail(OVL_ERR_INVALID_ARG, "unknown warm-start mode");
  if (!params || n_params != kMlpParams)
    return w->fail(OVL_ERR_INVALID_ARG, "learned mode needs OVL_MLP_PARAMS parameters");
  for (int64_t i = 0; i < n_params; ++i)
    if (!std::isfinite(params[i])) return w->fail(OVL_ERR_INVALID_ARG, "non-finite network parameter");
  std::vector<uint16_t> wb;
  std::vector<float> bias;
  mlp_pack(params, wb, bias);
  bool ok = true;
  if (!w->mlp_wb) {
    w->mlp_wb = w->alloc<uint16_t>(w->static_allocs, kMlpWb, ok);
    w->mlp_bias = w->alloc<float>(w->static_allocs, kMlpBias, ok);
    if (!ok) return w->fail(OVL_ERR_OOM, "network buffers");
  }
  if (hipStreamSynchronize(w->stream) != hipSuccess || !w->upload(w->mlp_wb, wb.data(), wb.size() * 2) ||
      !w->upload(w->mlp_bias, bias.data(), bias.size() * 4) || hipStreamSynchronize(w->stream) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "upload failed");
  w->wp.mlp_wb = w->mlp_wb;
  w->wp.mlp_bias = w->mlp_bias;
  w->prm.warmstart = OVL_WARM_PLAIN;
  w->wp.warmstart = 1;
  w->wp.learned = 1;
  w->wp.feat_on = 1;
  return OVL_OK;
}

ovl_status ovl_set_feature_export(ovl_world* w, int32_t enable) {
  if (!w) return OVL_ERR_INVALID_ARG;
  w->wp.feat_on = (enable != 0 || w->wp.learned) ? 1 : 0;
  return OVL_OK;
}

ovl_status ovl_force_guard(ovl_world* w, const int32_t* choice, int32_t n_parts) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (!choice) {
    w->wp.force_guard = 0;
    return OVL_OK;
  }
  if (n_parts != w->G) return w->fail(OVL_ERR_INVALID_ARG, "n_parts differs from the partition count");
  for (int g = 0; g < n_parts; ++g)
    if (choice[g] < -1 || choice[g] > 1) return w->fail(OVL_ERR_INVALID_ARG, "choice must be -1, 0 or 1");
  if (!w->upload((void*)w->wp.part_force_guard, choice, n_parts * sizeof(int32_t)) ||
      hipStreamSynchronize(w->stream) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "upload failed");
  w->wp.force_guard = 1;
  return OVL_OK;
}

ovl_status ovl_collect_training_rows(ovl_world* w, float* features, float* targets, int64_t capacity_rows,
                                     int64_t* n_rows) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (!w->wp.feat_on) return w->fail(OVL_ERR_INVALID_ARG, "feature export is off");
  if (hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "sync failed");
  const WP& p = w->wp;
  int32_t G = w->G, M = 0;
  if (hipMemcpy(&M, p.part_copy_off + G, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "copy failed");
  M = std::min(M, p.Mcap);
  std::vector<int32_t> src(M), slot(M);
  std::vector<float> feat((size_t)M * kFeatStride);
  std::vector<float4> lam(p.Mcap);
  if (M > 0 && (hipMemcpy(src.data(), p.cp_src, M * 4, hipMemcpyDeviceToHost) ||
                hipMemcpy(slot.data(), p.cp_slot, M * 4, hipMemcpyDeviceToHost) ||
                hipMemcpy(feat.data(), p.r_feat, feat.size() * 4, hipMemcpyDeviceToHost) ||
                hipMemcpy(lam.data(), p.r_lam, lam.size() * sizeof(float4), hipMemcpyDeviceToHost)))
    return w->fail(OVL_ERR_DEVICE, "copy failed");
  int64_t n = 0;
  for (int u = 0; u < M; ++u) {
    if (src[u] < w->J) continue;
    if (features && targets) {
      if (n >= capacity_rows) return w->fail(OVL_ERR_INVALID_ARG, "buffers too small");
      const float* f = &feat[(size_t)u * kFeatStride];
      for (int k = 0; k < kMlpIn; ++k) features[n * kMlpIn + k] = f[k];
      const float s_imp = f[12] > 0.0f ? f[12] : 1.0f;
      const float4 l = lam[slot[u]];
      targets[n * 3] = l.x / s_imp;
      targets[n * 3 + 1] = l.y / s_imp;
      targets[n * 3 + 2] = l.z / s_imp;
    }
    ++n;
  }
  if (n_rows) *n_rows = n;
  return OVL_OK;
}

static int find_pgs_cfg(int32_t block, int32_t reps) {
  for (int k = 0; k < kPgsCfgCount; ++k)
    if (kPgsCfgBlock[k] == block && kPgsCfgReps[k] == reps) return k;
  return -1;
}

ovl_status ovl_set_launch(ovl_world* w, const ovl_launch_cfg* cfg) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (!cfg) return w->fail(OVL_ERR_INVALID_ARG, "cfg is NULL");
  const int k = find_pgs_cfg(cfg->pgs_block, cfg->pgs_lds_reps);
  if (k < 0) return w->fail(OVL_ERR_INVALID_ARG, "unsupported (pgs_block, pgs_lds_reps) pair");
  if ((cfg->persistent != 0 && cfg->persistent != 1) || (cfg->graph != 0 && cfg->graph != 1))
    return w->fail(OVL_ERR_INVALID_ARG, "persistent and graph must be 0 or 1");
  if (hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "sync failed");
  if (!w->apply_launch(*cfg, k)) return w->fail(OVL_ERR_DEVICE, "occupancy query failed");
  return OVL_OK;
}

ovl_status ovl_get_launch(const ovl_world* w, ovl_launch_cfg* cfg) {
  if (!w || !cfg) return OVL_ERR_INVALID_ARG;
  *cfg = w->launch;
  return OVL_OK;
}

int32_t ovl_launch_candidates(ovl_launch_cfg* out, int32_t cap) {
  int n = 0;
  for (int k = 0; k < kPgsCfgCount; ++k)
    for (int pers = 0; pers < 2; ++pers) {
      if (out && n < cap) out[n] = ovl_launch_cfg{kPgsCfgBlock[k], kPgsCfgReps[k], pers, 0};
      ++n;
    }
  return n;
}

ovl_status ovl_autotune(ovl_world* w, int32_t trials, ovl_launch_cfg* chosen, float* ms, int32_t n_ms) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (trials < 1 || trials > 100) return w->fail(OVL_ERR_INVALID_ARG, "trials must be in [1,100]");
  if (w->forced_next) return w->fail(OVL_ERR_INVALID_ARG, "a forced sweep count is pending");
  const int n_cand = ovl_launch_candidates(nullptr, 0);
  if (ms && n_ms < n_cand) return w->fail(OVL_ERR_INVALID_ARG, "ms needs ovl_launch_candidates() entries");
  int32_t sc[SC_COUNT];
  if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "sync failed");
  if (sc[SC_FLAGS]) {
    ovl_status st = take_flags(w, sc[SC_FLAGS]);
    if (st != OVL_OK) return st;
  }
  w->wp.forced = 0;
  // contacts, graph, colours and rows of the step; grow once if a buffer overflowed
  for (int attempt = 0;; ++attempt) {
    hipError_t e = launch_collide(w->wp, w->scan_scratch, w->stream);
    if (!e) e = launch_graph(w->wp, w->scan_scratch, w->stream);
    if (!e) e = launch_solve_pre(w->wp, w->stream);
    if (e) return w->fail(OVL_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "step failed on the device");
    if (!(sc[SC_FLAGS] & (F_CONTACT_CAP | F_ADJ_CAP | F_REP_CAP | F_COPY_CAP))) break;
    if (attempt > 0 || !w->grow(sc)) return take_flags(w, sc[SC_FLAGS]);
    w->write_scal(SC_FLAGS, 0);
  }
  if (sc[SC_FLAGS]) return take_flags(w, sc[SC_FLAGS]);
  const ovl_launch_cfg keep = w->launch;
  const int keep_k = w->wp.pgs_cfg;
  hipEvent_t e0 = w->take_event(), e1 = w->take_event();
  if (!e0 || !e1) return w->fail(OVL_ERR_DEVICE, "event creation failed");
  std::vector<float> best_ms(n_cand, 0.0f);
  unsigned long long ref_digest = 0;
  int best = -1;
  ovl_status result = OVL_OK;
  for (int c = 0; c < n_cand && result == OVL_OK; ++c) {
    const int k = c / 2;
    const ovl_launch_cfg cand{kPgsCfgBlock[k], kPgsCfgReps[k], c % 2, keep.graph};
    if (!w->apply_launch(cand, k)) {
      result = w->fail(OVL_ERR_DEVICE, "occupancy query failed");
      break;
    }
    float tmin = 0.0f;
    for (int t = 0; t < trials; ++t) {
      hipError_t e = launch_reset_lambda(w->wp, w->stream);
      if (!e) e = hipEventRecord(e0, w->stream);
      if (!e) e = launch_pgs(w->wp, w->stream);
      if (!e) e = hipEventRecord(e1, w->stream);
      if (!e) e = hipStreamSynchronize(w->stream);
      float dt = 0.0f;
      if (!e) e = hipEventElapsedTime(&dt, e0, e1);
      if (e) {
        result = w->fail(OVL_ERR_DEVICE, std::string("autotune launch failed: ") + hipGetErrorString(e));
        break;
      }
      tmin = t == 0 ? dt : std::min(tmin, dt);
    }
    if (result != OVL_OK) break;
    unsigned long long dg = 0;
    if (launch_digest(w->wp, w->digest, w->stream) != hipSuccess ||
        hipMemcpyAsync(&dg, w->digest, sizeof(dg), hipMemcpyDeviceToHost, w->stream) != hipSuccess ||
        hipStreamSynchronize(w->stream) != hipSuccess) {
      result = w->fail(OVL_ERR_DEVICE, "digest failed");
      break;
    }
    if (c == 0) ref_digest = dg;
    else if (dg != ref_digest) result = w->fail(OVL_ERR_DEVICE, "launch configurations gave different results");
    best_ms[c] = tmin;
    if (best < 0 || tmin < best_ms[best]) best = c;
  }
  w->ev_pool.push_back(e0);
  w->ev_pool.push_back(e1);
  if (result != OVL_OK) {
    (void)w->apply_launch(keep, keep_k);
    return result;
  }
  // finish the step with the fastest configuration
  const int kb = best / 2;
  const ovl_launch_cfg win{kPgsCfgBlock[kb], kPgsCfgReps[kb], best % 2, keep.graph};
  (void)w->apply_launch(win, kb);
  hipError_t e = launch_reset_lambda(w->wp, w->stream);
  if (!e) e = launch_pgs(w->wp, w->stream);
  if (!e) e = launch_solve_post(w->wp, w->stream, false);
  if (e) return w->fail(OVL_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "step failed on the device");
  if (sc[SC_FLAGS]) return take_flags(w, sc[SC_FLAGS]);
  if (chosen) *chosen = win;
  if (ms)
    for (int c = 0; c < n_cand; ++c) ms[c] = best_ms[c];
  return OVL_OK;
}

ovl_status ovl_profile(ovl_world* w, int32_t enable) {
  if (!w) return OVL_ERR_INVALID_ARG;
  w->profiling = enable != 0;
  return OVL_OK;
}

ovl_status ovl_get_counters(ovl_world* w, ovl_counters* out) {
  if (!w || !out) return OVL_ERR_INVALID_ARG;
  if (hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "sync failed");
  w->drain_events();
  int64_t c[8];
  if (hipMemcpy(c, w->wp.stat_i64, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "copy failed");
  out->steps = c[4];
  out->sweeps_max_total = c[0];
  out->sweeps_part_total = c[3];
  out->unconverged_total = c[1];
  out->pgs_bytes = c[2];
  out->pgs_launches = w->pgs_launches;
  out->pgs_ms = w->pgs_ms;
  out->steps_capped = c[5];
  out->pgs_ops = c[6];
  return OVL_OK;
}

ovl_status ovl_synchronize(ovl_world* w) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "sync failed");
  return OVL_OK;
}

ovl_status ovl_read_state(ovl_world* w, float* dst, int64_t n_bodies, int32_t dst_is_device) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (n_bodies != w->N || (!dst && w->N > 0)) return w->fail(OVL_ERR_INVALID_ARG, "n_bodies mismatch or NULL dst");
  int32_t sc[SC_COUNT];
  if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "sync failed");
  ovl_status flag_status = take_flags(w, sc[SC_FLAGS]);
  const int N = w->N;
  if (N == 0) return flag_status;
  if (dst_is_device) {
    k_cols_to_rows<<<nblocks(N, 256), 256, 0, w->stream>>>(w->wp.st, dst, N);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(w->stream) != hipSuccess)
      return w->fail(OVL_ERR_DEVICE, "read_state kernel failed");
  } else {
    std::vector<float> cols((size_t)13 * N);
    if (hipMemcpyAsync(cols.data(), w->wp.st, cols.size() * sizeof(float), hipMemcpyDeviceToHost, w->stream) !=
            hipSuccess ||
        hipStreamSynchronize(w->stream) != hipSuccess)
      return w->fail(OVL_ERR_DEVICE, "copy failed");
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < 13; ++k) dst[13 * (size_t)i + k] = cols[(size_t)k * N + i];
  }
  return flag_status;
}

ovl_status ovl_write_state(ovl_world* w, const float* src, int64_t n_bodies, int32_t src_is_device,
                           int32_t keep_cache) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (n_bodies != w->N || (!src && w->N > 0)) return w->fail(OVL_ERR_INVALID_ARG, "n_bodies mismatch or NULL src");
  const int N = w->N;
  std::vector<float> rows((size_t)13 * N);
  if (src_is_device) {
    if (hipMemcpy(rows.data(), src, rows.size() * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
      return w->fail(OVL_ERR_DEVICE, "copy failed");
  } else {
    std::copy(src, src + rows.size(), rows.begin());
  }
  for (size_t i = 0; i < rows.size(); ++i)
    if (!std::isfinite(rows[i])) return w->fail(OVL_ERR_INVALID_ARG, "state has non-finite values");
  std::vector<float> cols(rows.size());
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 13; ++k) cols[(size_t)k * N + i] = rows[13 * (size_t)i + k];
  if (hipStreamSynchronize(w->stream) != hipSuccess || !w->upload(w->wp.st, cols.data(), cols.size() * sizeof(float)) ||
      hipStreamSynchronize(w->stream) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "upload failed");
  if (!keep_cache) w->write_scal(SC_PREV_NCOPY, 0);
  return OVL_OK;
}

ovl_status ovl_write_cache(ovl_world* w, const int32_t* part, const int32_t* kind, const uint64_t* key,
                           const float* val, int64_t n) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (n < 0 || (n > 0 && (!part || !kind || !key || !val))) return w->fail(OVL_ERR_INVALID_ARG, "bad cache arrays");
  if (n > w->wp.Mcap) return w->fail(OVL_ERR_CAPACITY, "cache larger than the copy capacity");
  for (int64_t i = 0; i < n; ++i) {
    if (part[i] < 0 || part[i] >= w->G || (kind[i] != 0 && kind[i] != 1))
      return w->fail(OVL_ERR_INVALID_ARG, "cache entry with a bad partition or kind");
    for (int k = 0; k < 4; ++k)
      if (!std::isfinite(val[4 * i + k])) return w->fail(OVL_ERR_INVALID_ARG, "non-finite cached impulse");
    if ((key[i] >> 63) != 0) return w->fail(OVL_ERR_INVALID_ARG, "cache key out of range");
    if (i > 0) {
      const bool less = part[i - 1] < part[i] ||
                        (part[i - 1] == part[i] && (kind[i - 1] < kind[i] || (kind[i - 1] == kind[i] && key[i - 1] < key[i])));
      if (!less) return w->fail(OVL_ERR_INVALID_ARG, "cache entries must be strictly increasing in (part, kind, key)");
    }
  }
  const int64_t MC = w->wp.Mcap;
  std::vector<float> cols((size_t)4 * MC, 0.0f);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 4; ++k) cols[(size_t)k * MC + i] = val[4 * i + k];
  // the search index: a 64-bit key per entry and each partition's range
  std::vector<uint64_t> k64((size_t)n);
  std::vector<int32_t> off((size_t)w->G + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    k64[i] = ((uint64_t)kind[i] << 63) | key[i];
    off[part[i] + 1]++;
  }
  for (int g = 0; g < w->G; ++g) off[g + 1] += off[g];
  if (hipStreamSynchronize(w->stream) != hipSuccess || !w->upload(w->wp.wc_part, part, n * sizeof(int32_t)) ||
      !w->upload(w->wp.wc_kind, kind, n * sizeof(int32_t)) || !w->upload(w->wp.wc_key, key, n * sizeof(uint64_t)) ||
      !w->upload(w->wp.wc_k64, k64.data(), n * sizeof(uint64_t)) ||
      !w->upload(w->wp.wc_off, off.data(), off.size() * sizeof(int32_t)) ||
      !w->upload(w->wp.wc_val, cols.data(), cols.size() * sizeof(float)) || hipStreamSynchronize(w->stream) != hipSuccess)
    return w->fail(OVL_ERR_DEVICE, "upload failed");
  w->write_scal(SC_PREV_NCOPY, (int32_t)n);
  return OVL_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ debug ----

namespace {

template <class T_>
bool dl(ovl_world* w, std::vector<T_>& v, const T_* src, size_t n) {
  v.resize(n);
  if (!n) return true;
  return hipMemcpy(v.data(), src, n * sizeof(T_), hipMemcpyDeviceToHost) == hipSuccess;
}

}  // namespace

extern "C" ovl_status ovl_read_debug(ovl_world* w, int32_t field, void* dst, int64_t capacity_bytes, int64_t* count) {
  if (!w) return OVL_ERR_INVALID_ARG;
  if (hipStreamSynchronize(w->stream) != hipSuccess) return w->fail(OVL_ERR_DEVICE, "sync failed");
  const WP& p = w->wp;
  const int N = w->N, G = w->G, J = w->J;
  int32_t sc[SC_COUNT];
  if (!w->read_scal(sc)) return w->fail(OVL_ERR_DEVICE, "sync failed");
  const int C = std::min(sc[SC_NCONTACT], p.Ccap);
  std::vector<int32_t> prep, pcop;
  if (!dl(w, prep, p.part_rep_off, G + 1) || !dl(w, pcop, p.part_copy_off, G + 1))
    return w->fail(OVL_ERR_DEVICE, "copy failed");
  const int R = std::min(prep[G], p.Rcap);
  const int M = std::min(pcop[G], p.Mcap);
  std::vector<uint8_t> out;
  int64_t n = 0;
  auto put = [&](const void* src, size_t elems, size_t es) {
    out.resize(elems * es);
    if (elems) memcpy(out.data(), src, elems * es);
    n = (int64_t)elems;
  };
  bool ok = true;
  switch (field) {
    case OVL_DBG_CONTACT_KEY: {
      std::vector<int32_t> a;
      std::vector<uint32_t> b;
      ok = dl(w, a, p.c_a, C) && dl(w, b, p.c_bkey, C);
      std::vector<uint64_t> k(C);
      for (int i = 0; i < C; ++i) k[i] = ((uint64_t)a[i] << 32) | b[i];
      put(k.data(), C, 8);
      break;
    }
    case OVL_DBG_CONTACT_GEOM: {
      std::vector<float> gcol;
      ok = dl(w, gcol, p.c_geom, (size_t)8 * p.Ccap);
      std::vector<float> g((size_t)8 * C);
      for (int i = 0; i < C && ok; ++i)
        for (int k = 0; k < 8; ++k) g[8 * (size_t)i + k] = gcol[(size_t)k * p.Ccap + i];
      put(g.data(), (size_t)8 * C, 4);
      break;
    }
    case OVL_DBG_ADJ_OFF: {
      std::vector<int32_t> v;
      ok = dl(w, v, p.adj_off, N + 1);
      put(v.data(), N + 1, 4);
      break;
    }
    case OVL_DBG_ADJ: {
      std::vector<int32_t> off, v;
      ok = dl(w, off, p.adj_off, N + 1);
      if (ok) ok = dl(w, v, p.adj, std::min(off[N], p.Acap));
      put(v.data(), v.size(), 4);
      break;
    }
    case OVL_DBG_MASK: {
      std::vector<uint64_t> v;
      ok = dl(w, v, p.mask, N);
      put(v.data(), N, 8);
      break;
    }
    case OVL_DBG_PART_REP_OFF:
      put(prep.data(), G + 1, 4);
      break;
    case OVL_DBG_REP_BODY: {
      std::vector<int32_t> v;
      ok = dl(w, v, p.rep_body_pm, R);
      put(v.data(), R, 4);
      break;
    }
    case OVL_DBG_REP_D:
    case OVL_DBG_REP_W: {
      std::vector<int32_t> pm, D;
      std::vector<float> W;
      ok = dl(w, pm, p.rep_pm_of_bm, R) && dl(w, D, p.rep_D_bm, R) && dl(w, W, p.rep_w_bm, R);
      if (field == OVL_DBG_REP_D) {
        std::vector<int32_t> o(R);
        for (int j = 0; j < R && ok; ++j)
          if (pm[j] >= 0 && pm[j] < R) o[pm[j]] = D[j];
        put(o.data(), R, 4);
      } else {
        std::vector<float> o(R);
        for (int j = 0; j < R && ok; ++j)
          if (pm[j] >= 0 && pm[j] < R) o[pm[j]] = W[j];
        put(o.data(), R, 4);
      }
      break;
    }
    case OVL_DBG_PART_COPY_OFF:
      put(pcop.data(), G + 1, 4);
      break;
    case OVL_DBG_COPY_KIND:
    case OVL_DBG_COPY_KEY: {
      std::vector<int32_t> src, a;
      std::vector<uint32_t> b;
      ok = dl(w, src, p.cp_src, M) && dl(w, a, p.c_a, C) && dl(w, b, p.c_bkey, C);
      if (field == OVL_DBG_COPY_KIND) {
        std::vector<int32_t> o(M);
        for (int u = 0; u < M; ++u) o[u] = src[u] < J ? 0 : 1;
        put(o.data(), M, 4);
      } else {
        std::vector<uint64_t> o(M);
        for (int u = 0; u < M && ok; ++u) {
          int s = src[u];
          o[u] = s < J ? (uint64_t)s : (s - J < C ? (((uint64_t)a[s - J] << 32) | b[s - J]) : ~0ull);
        }
        put(o.data(), M, 8);
      }
      break;
    }
    case OVL_DBG_COPY_IA:
    case OVL_DBG_COPY_IB:
    case OVL_DBG_COPY_COLOUR: {
      std::vector<int32_t> v;
      const int32_t* srcp = field == OVL_DBG_COPY_IA ? p.cp_ia : field == OVL_DBG_COPY_IB ? p.cp_ib : p.cp_colour;
      ok = dl(w, v, srcp, M);
      put(v.data(), M, 4);
      break;
    }
    case OVL_DBG_COPY_LAMBDA0:
    case OVL_DBG_COPY_LAMBDA: {
      std::vector<int32_t> slot;
      std::vector<float4> lc;
      ok = dl(w, slot, p.cp_slot, M) && dl(w, lc, field == OVL_DBG_COPY_LAMBDA ? (const float4*)p.r_lam
                                                                             : (const float4*)p.r_lam0, (size_t)p.Mcap);
      std::vector<float> o((size_t)3 * M);
      for (int u = 0; u < M && ok; ++u)
        if (slot[u] >= 0 && slot[u] < p.Mcap) {
          const float4 l = lc[slot[u]];
          o[3 * (size_t)u] = l.x;
          o[3 * (size_t)u + 1] = l.y;
          o[3 * (size_t)u + 2] = l.z;
        }
      put(o.data(), (size_t)3 * M, 4);
      break;
    }
    case OVL_DBG_REP_STATE: {
      std::vector<float> rc;
      ok = dl(w, rc, p.rst, (size_t)13 * p.Rcap);
      std::vector<float> o((size_t)13 * R);
      for (int r = 0; r < R && ok; ++r)
        for (int k = 0; k < 13; ++k) o[13 * (size_t)r + k] = rc[(size_t)k * p.Rcap + r];
      put(o.data(), (size_t)13 * R, 4);
      break;
    }
    case OVL_DBG_PART_ITERS: {
      std::vector<int32_t> v;
      ok = dl(w, v, p.part_iters, G);
      put(v.data(), G, 4);
      break;
    }
    case OVL_DBG_PART_RESID: {
      std::vector<float> v;
      ok = dl(w, v, p.part_resid, G);
      put(v.data(), G, 4);
      break;
    }
    case OVL_DBG_CACHE_PART:
    case OVL_DBG_CACHE_KIND:
    case OVL_DBG_CACHE_KEY:
    case OVL_DBG_CACHE_VAL: {
      const int Mc = std::min(sc[SC_PREV_NCOPY], p.Mcap);
      if (field == OVL_DBG_CACHE_PART || field == OVL_DBG_CACHE_KIND) {
        std::vector<int32_t> v;
        ok = dl(w, v, field == OVL_DBG_CACHE_PART ? p.wc_part : p.wc_kind, Mc);
        put(v.data(), Mc, 4);
      } else if (field == OVL_DBG_CACHE_KEY) {
        std::vector<uint64_t> v;
        ok = dl(w, v, p.wc_key, Mc);
        put(v.data(), Mc, 8);
      } else {
        std::vector<float> vc;
        ok = dl(w, vc, p.wc_val, (size_t)4 * p.Mcap);
        std::vector<float> o((size_t)4 * Mc);
        for (int u = 0; u < Mc && ok; ++u)
          for (int k = 0; k < 4; ++k) o[4 * (size_t)u + k] = vc[(size_t)k * p.Mcap + u];
        put(o.data(), (size_t)4 * Mc, 4);
      }
      break;
    }
    case OVL_DBG_PART_COL_OFF: {
      std::vector<int32_t> v;
      ok = dl(w, v, p.part_col_off, (size_t)G * kColStride);
      put(v.data(), (size_t)G * kColStride, 4);
      break;
    }
    case OVL_DBG_COPY_FEAT: {
      std::vector<float> f;
      ok = dl(w, f, p.r_feat, (size_t)M * kFeatStride);
      std::vector<float> o((size_t)13 * M);
      for (int u = 0; u < M && ok; ++u)
        for (int k = 0; k < 13; ++k) o[13 * (size_t)u + k] = f[(size_t)u * kFeatStride + k];
      put(o.data(), (size_t)13 * M, 4);
      break;
    }
    case OVL_DBG_COPY_LAMBDAL: {
      std::vector<int32_t> slot, src;
      std::vector<float4> lc, l0;
      ok = dl(w, slot, p.cp_slot, M) && dl(w, src, p.cp_src, M) && dl(w, lc, (const float4*)p.r_lamL, (size_t)p.Mcap) &&
           dl(w, l0, (const float4*)p.r_lam0, (size_t)p.Mcap);
      std::vector<float> o((size_t)3 * M);
      for (int u = 0; u < M && ok; ++u)
        if (slot[u] >= 0 && slot[u] < p.Mcap) {
          const float4 l = src[u] < J ? l0[slot[u]] : lc[slot[u]];
          o[3 * (size_t)u] = l.x;
          o[3 * (size_t)u + 1] = l.y;
          o[3 * (size_t)u + 2] = l.z;
        }
      put(o.data(), (size_t)3 * M, 4);
      break;
    }
    case OVL_DBG_PART_GUARD: {
      std::vector<int32_t> v;
      ok = dl(w, v, p.part_guard, G);
      put(v.data(), G, 4);
      break;
    }
    case OVL_DBG_REP_CPL: {
      std::vector<float4> rc;
      ok = dl(w, rc, p.rep_cpl, (size_t)2 * p.Rcap);
      std::vector<float> o((size_t)6 * R);
      for (int r = 0; r < R && ok; ++r) {
        const float4 a = rc[r], b = rc[(size_t)p.Rcap + r];
        const float v[6] = {a.x, a.y, a.z, b.x, b.y, b.z};
        for (int k = 0; k < 6; ++k) o[6 * (size_t)r + k] = v[k];
      }
      put(o.data(), (size_t)6 * R, 4);
      break;
    }
    case OVL_DBG_PART_RHO0: {
      std::vector<float> v;
      ok = dl(w, v, p.part_rho0, 2 * (size_t)G);
      put(v.data(), 2 * (size_t)G, 4);
      break;
    }
    default:
      return w->fail(OVL_ERR_INVALID_ARG, "unknown debug field");
  }
  if (!ok) return w->fail(OVL_ERR_DEVICE, "copy failed");
  if (count) *count = n;
  if (dst) {
    if ((int64_t)out.size() > capacity_bytes) return w->fail(OVL_ERR_INVALID_ARG, "dst too small");
    memcpy(dst, out.data(), out.size());
  }
  return OVL_OK;
}
