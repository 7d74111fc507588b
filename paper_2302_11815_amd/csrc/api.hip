// C-ABI of the walk-on-stars solver (declared in include/wost.h): scene
// upload, solves, probes, statistics and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/wost.h"
#include "scene_build.hpp"
#include "wost_internal.hpp"

static_assert(sizeof(wost_step_rec) == sizeof(wost::StepRec), "step record layouts differ");
static_assert(wost::kTopNodes == (1 << wost::kTopLevels) - 1, "LDS copies hold the promoted tree levels");
static_assert(wost::kStack<2> == wost::max_tree_depth(2) + 1 && wost::kStack<3> == wost::max_tree_depth(3) + 1,
              "traversal stacks must hold the deepest tree the builder makes");

namespace {

thread_local std::string g_err;

wost_status fail(wost_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

wost_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(WOST_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
  return fail(WOST_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, what)                   \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr float kOffsetRel = 1.0f / 262144.0f;   // 2^-18
constexpr int64_t kMaxSdf = 256;                  // analytic shapes per scene (each step tests all)
constexpr float kEscapeRel = 2.0f;
constexpr int kMaxSteps = 65536;
constexpr int kTrafficBase = 8;
constexpr int kEventBase = kTrafficBase + wost::kTrafficCounters;
constexpr int kCtrWords = kEventBase + 1 + 2 * wost::kEventCap;

}  // namespace

struct wost_scene_s {
  wost::HostScene host;
  wost::SceneDev dev{};
  std::vector<void*> allocs;
  int64_t device_bytes = 0;
  // per-solve scratch, grown on demand
  float* est = nullptr;
  size_t est_cap = 0;
  unsigned long long* ctr = nullptr;   // stats[4], cursor[1], pad, traffic[kTrafficCounters], events
  unsigned long long* ctr_view = nullptr;  // counters of the last solve: ctr, or the no-alloc array's
  bool counted = false;
  int last_mode = 0, last_grid = 0;
  int grid_lane = 0;   // resident capacity of the per-lane persistent kernel
  int64_t last_n = 0;
  int last_W = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool have_stats = false;
  int grid_default = 0;
  std::vector<int32_t> ninv;           // primitive id -> Neumann leaf slot, or -1
  int32_t* start = nullptr;            // boundary solves: start slot per point
  size_t start_cap = 0;
  ~wost_scene_s() {
    for (void* p : allocs) (void)hipFree(p);
    if (start) (void)hipFree(start);
    if (est) (void)hipFree(est);
    if (ctr) (void)hipFree(ctr);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

namespace {

template <typename T>
wost_status upload(wost_scene_s* s, const std::vector<T>& v, const T** out) {
  *out = nullptr;
  if (v.empty()) return WOST_OK;
  void* p = nullptr;
  HIP_TRY(hipMalloc(&p, v.size() * sizeof(T)), "hipMalloc");
  s->allocs.push_back(p);
  HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  s->device_bytes += (int64_t)(v.size() * sizeof(T));
  *out = static_cast<const T*>(p);
  return WOST_OK;
}

wost_status check_fn(const wost_fn& f, const char* name, bool allow_pc) {
  if (f.kind < WOST_FN_ZERO || f.kind > WOST_FN_EXPLIN)
    return fail(WOST_ERR_INVALID_ARG, std::string(name) + ": unknown kind");
  if (f.kind == WOST_FN_PER_CORNER && (!allow_pc || !f.per_corner))
    return fail(WOST_ERR_INVALID_ARG, std::string(name) + ": PER_CORNER needs data (g, h only)");
  if (f.kind == WOST_FN_PER_CORNER && f.as_normal_derivative)
    return fail(WOST_ERR_INVALID_ARG, std::string(name) + ": PER_CORNER cannot be a normal derivative");
  for (int i = 0; i < 10; ++i)
    if (!std::isfinite(f.coef[i])) return fail(WOST_ERR_INVALID_ARG, std::string(name) + ": non-finite coefficient");
  return WOST_OK;
}

wost::FnDev fn_dev(const wost_fn& f) {
  wost::FnDev d{};
  d.kind = f.kind;
  d.as_nd = f.as_normal_derivative ? 1 : 0;
  for (int i = 0; i < 10; ++i) d.c[i] = (float)f.coef[i];
  d.pc = nullptr;
  return d;
}

wost_status validate_desc(const wost_scene_desc* d) {
  if (!d) return fail(WOST_ERR_INVALID_ARG, "desc is NULL");
  wost_status st;
  if ((st = check_fn(d->g, "g", true)) != WOST_OK) return st;
  if ((st = check_fn(d->h, "h", true)) != WOST_OK) return st;
  if ((st = check_fn(d->f, "f", false)) != WOST_OK) return st;
  if ((st = check_fn(d->g_minus, "g_minus", true)) != WOST_OK) return st;
  if ((st = check_fn(d->h_minus, "h_minus", true)) != WOST_OK) return st;
  if (d->f.kind == WOST_FN_EXPCOS) return fail(WOST_ERR_INVALID_ARG, "f: EXPCOS is not supported for f");
  if (d->n_sdf < 0 || d->n_sdf > kMaxSdf || (d->n_sdf > 0 && !d->sdf))
    return fail(WOST_ERR_INVALID_ARG, "n_sdf must be 0.." + std::to_string(kMaxSdf) + " with a non-NULL sdf");
  if (d->n_sdf > 0 && d->g.kind == WOST_FN_PER_CORNER)
    return fail(WOST_ERR_INVALID_ARG, "g: PER_CORNER data cannot cover analytic shapes");
  for (int64_t i = 0; i < d->n_sdf; ++i) {
    const wost_sdf& f = d->sdf[i];
    const std::string at = "sdf[" + std::to_string(i) + "]: ";
    for (double x : f.p)
      if (!std::isfinite(x)) return fail(WOST_ERR_INVALID_ARG, at + "non-finite parameter");
    if (f.kind < WOST_SDF_BALL || f.kind > WOST_SDF_CAPSULE) return fail(WOST_ERR_INVALID_ARG, at + "unknown kind");
    if (f.inside != 0 && f.inside != 1) return fail(WOST_ERR_INVALID_ARG, at + "inside must be 0 or 1");
    if (f.kind != WOST_SDF_BOX && !(f.p[6] > 0)) return fail(WOST_ERR_INVALID_ARG, at + "radius must be > 0");
    if (f.kind == WOST_SDF_BOX) {
      for (int k = 0; k < d->dim && k < 3; ++k)
        if (!(f.p[3 + k] > 0)) return fail(WOST_ERR_INVALID_ARG, at + "half extents must be > 0");
      if (!(f.p[6] >= 0)) return fail(WOST_ERR_INVALID_ARG, at + "rounding must be >= 0");
    }
    if (f.inside && !(f.kind == WOST_SDF_BALL || (f.kind == WOST_SDF_BOX && f.p[6] == 0)))
      return fail(WOST_ERR_INVALID_ARG, at + "only a ball or a box without rounding can hold the domain inside");
  }
  if (d->f.as_normal_derivative) return fail(WOST_ERR_INVALID_ARG, "f cannot be a normal derivative");
  return WOST_OK;
}

void fill_info(const wost::HostScene& H, wost_scene_info* info) {
  std::memset(info, 0, sizeof(*info));
  info->dim = H.dim;
  info->n_prims = H.n_prims;
  info->n_dirichlet = (int64_t)H.d_prims.size();
  info->n_neumann = (int64_t)H.n_prims_list.size();
  info->n_silhouette_elements = (int64_t)H.elem_always.size();
  info->nodes_dirichlet = H.treeD.stats.n_nodes;
  info->nodes_neumann = H.treeN.stats.n_nodes;
  info->nodes_silhouette = H.treeS.stats.n_nodes;
  info->depth_dirichlet = H.treeD.stats.max_depth;
  info->depth_neumann = H.treeN.stats.max_depth;
  info->depth_silhouette = H.treeS.stats.max_depth;
  info->half_diagonal = H.L;
  for (int k = 0; k < 3; ++k) info->center[k] = H.center[k];
  const int dim = H.dim;
  const int64_t node_b = dim == 3 ? 64 : 48, prim_b = dim == 3 ? 48 : 16;
  const int64_t cone_b = dim == 3 ? 48 : 32, elem_b = dim == 3 ? 48 : 32;
  info->device_bytes = (info->nodes_dirichlet + info->nodes_neumann + info->nodes_silhouette) * node_b +
                       info->nodes_silhouette * cone_b + (info->n_dirichlet + info->n_neumann) * prim_b +
                       info->n_silhouette_elements * elem_b +
                       (info->n_dirichlet + 2 * info->n_neumann) * 4 + info->n_prims * 4;
}

wost_status preprocess_desc(const wost_scene_desc* d, wost::HostScene& H) {
  wost_status st = validate_desc(d);
  if (st != WOST_OK) return st;
  const int leaf = 4;
  // bounds of the analytic shapes, for the scene box
  std::vector<double> boxes;
  for (int64_t i = 0; i < d->n_sdf; ++i) {
    const wost_sdf& f = d->sdf[i];
    for (int side = 0; side < 2; ++side)
      for (int k = 0; k < 3; ++k) {
        double v = 0.0;
        if (k < d->dim) {
          const double sg = side ? 1.0 : -1.0;
          if (f.kind == WOST_SDF_BALL) v = f.p[k] + sg * f.p[6];
          else if (f.kind == WOST_SDF_BOX) v = f.p[k] + sg * (f.p[3 + k] + f.p[6]);
          else v = (side ? std::max(f.p[k], f.p[3 + k]) : std::min(f.p[k], f.p[3 + k])) + sg * f.p[6];
        }
        boxes.push_back(v);
      }
  }
  std::string err = wost::preprocess(d->dim, d->n_vertices, d->vertices, d->n_prims, d->prims,
                                     d->bc, H, leaf, leaf, leaf, &boxes);
  if (!err.empty()) return fail(WOST_ERR_INVALID_ARG, err);
  return WOST_OK;
}

// resolve options against defaults into the device scene copy and params
void apply_opts(const wost_scene_s* s, const wost_solve_opts* o, float eps, wost::SceneDev& S,
                wost::WalkParams& P, int& mode, int& grid) {
  S = s->dev;
  const double L = s->host.L;
  const float off_rel = (o && o->offset_rel > 0) ? o->offset_rel : kOffsetRel;
  const float esc_rel = (o && o->escape_rel > 0) ? o->escape_rel : kEscapeRel;
  S.offset = (float)(off_rel * L);
  const double er = esc_rel * L;
  S.escape2 = (float)(er * er);
  S.escape = (float)er;
  P.sigma = (o && o->sigma > 0) ? o->sigma : 0.0f;
  P.tik_sigma = (o && o->tikhonov_sigma > 0) ? o->tikhonov_sigma : 0.0f;
  P.tik_steps = (o && o->tikhonov_steps > 0) ? o->tikhonov_steps : 0;
  P.eps = eps;
  P.rmin = (o && o->r_min > 0) ? o->r_min : eps;
  P.max_steps = (o && o->max_steps > 0) ? o->max_steps : kMaxSteps;
  P.refill = (o && o->refill > 0) ? (o->refill > 64 ? 64 : o->refill) : 1;
  P.order = (o && o->walk_order == 1) ? 1 : 0;
  mode = (o && (o->mode == 1 || o->mode == 2)) ? o->mode : 0;
  grid = (o && o->grid > 0) ? o->grid : (mode == 2 ? s->grid_lane : s->grid_default);
}

wost_status ensure_scratch(wost_scene_s* s, size_t n_est) {
  if (!s->ctr)
    HIP_TRY(hipMalloc((void**)&s->ctr, kCtrWords * sizeof(unsigned long long)), "hipMalloc counters");
  if (n_est > s->est_cap) {
    if (s->est) {
      HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
      HIP_TRY(hipFree(s->est), "hipFree");
      s->est = nullptr;
      s->est_cap = 0;
    }
    HIP_TRY(hipMalloc((void**)&s->est, n_est * sizeof(float)), "hipMalloc walk estimates");
    s->est_cap = n_est;
  }
  return WOST_OK;
}

wost_status check_solve_args(wost_scene s, int64_t n, int32_t W, float eps,
                             const wost_solve_opts* o = nullptr) {
  if (!s) return fail(WOST_ERR_INVALID_ARG, "scene is NULL");
  if (o && (!std::isfinite(o->sigma) || !std::isfinite(o->tikhonov_sigma)))
    return fail(WOST_ERR_INVALID_ARG, "sigma and tikhonov_sigma must be finite");
  if (s->host.d_prims.empty() && s->dev.nS == 0 && !(o && (o->sigma > 0 || o->tikhonov_sigma > 0)))
    return fail(WOST_ERR_NOT_SUPPORTED,
                "scene has no Dirichlet primitives: a pure Neumann problem needs sigma > 0 or "
                "a Tikhonov switch (tikhonov_sigma > 0)");
  if (n < 0) return fail(WOST_ERR_INVALID_ARG, "n_points < 0");
  if (W < 1) return fail(WOST_ERR_INVALID_ARG, "walks_per_point < 1");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(WOST_ERR_INVALID_ARG, "eps must be finite and > 0");
  if (n > (int64_t(1) << 32)) return fail(WOST_ERR_INVALID_ARG, "n_points exceeds 2^32");
  return WOST_OK;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc((void**)&p, (n ? n : 1) * sizeof(T)); }
};

}  // namespace

extern "C" {

const char* wost_last_error(void) { return g_err.c_str(); }

wost_status wost_check_scene_host(const wost_scene_desc* desc, wost_scene_info* info) {
  g_err.clear();
  if (!info) return fail(WOST_ERR_INVALID_ARG, "info is NULL");
  try {
    wost::HostScene H;
    wost_status st = preprocess_desc(desc, H);
    if (st != WOST_OK) return st;
    fill_info(H, info);
    info->n_sdf = desc->n_sdf;
    return WOST_OK;
  } catch (const std::bad_alloc&) {
    return fail(WOST_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(WOST_ERR_INTERNAL, "unexpected exception");
  }
}

wost_status wost_build_scene(const wost_scene_desc* desc, wost_scene* out) {
  g_err.clear();
  if (!out) return fail(WOST_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  wost_scene_s* s = nullptr;
  try {
    s = new wost_scene_s();
    wost::HostScene& H = s->host;
    wost_status st = preprocess_desc(desc, H);
    if (st != WOST_OK) { delete s; return st; }
    const int dim = H.dim;
    auto vtx = [&](int32_t v, int k) { return H.V[3 * v + k]; };
    // primitive payloads in leaf order
    auto gather_prims = [&](const wost::FlatTree& T, const std::vector<int32_t>& ids,
                            std::vector<float>& pay, std::vector<int32_t>& orig, std::vector<float>* meas) {
      const size_t n = T.order.size();
      pay.assign(n * (dim == 3 ? 12 : 4), 0.0f);
      orig.resize(n);
      if (meas) meas->resize(n);
      for (size_t i = 0; i < n; ++i) {
        const int32_t p = ids[T.order[i]];
        orig[i] = p;
        if (meas) (*meas)[i] = (float)H.measure[p];
        if (dim == 3) {
          for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) pay[12 * i + 4 * c + k] = vtx(H.P[3 * p + c], k);
        } else {
          pay[4 * i + 0] = vtx(H.P[3 * p], 0);
          pay[4 * i + 1] = vtx(H.P[3 * p], 1);
          pay[4 * i + 2] = vtx(H.P[3 * p + 1], 0);
          pay[4 * i + 3] = vtx(H.P[3 * p + 1], 1);
        }
      }
    };
    // leaf blocks load kLeafMax slots unconditionally: pad every payload
    // array with copies of its last entry
    auto pad = [](std::vector<float>& v, size_t stride) {
      if (v.empty()) return;
      const std::vector<float> last(v.end() - stride, v.end());
      for (int k = 0; k < wost::kLeafMax - 1; ++k) v.insert(v.end(), last.begin(), last.end());
    };
    std::vector<float> dpay, npay, narea;
    std::vector<int32_t> did, nid;
    gather_prims(H.treeD, H.d_prims, dpay, did, nullptr);
    gather_prims(H.treeN, H.n_prims_list, npay, nid, &narea);
    pad(dpay, dim == 3 ? 12 : 4);
    pad(npay, dim == 3 ? 12 : 4);
    pad(narea, 1);
    std::vector<int32_t> ninv(H.n_prims, -1);
    for (size_t i = 0; i < nid.size(); ++i) ninv[nid[i]] = (int32_t)i;
    // silhouette elements in leaf order
    const size_t ne = H.treeS.order.size();
    std::vector<float> epay(ne * (dim == 3 ? 12 : 8), 0.0f);
    for (size_t i = 0; i < ne; ++i) {
      const int32_t e = H.treeS.order[i];
      const double* n0 = &H.elem_n[6 * e];
      const double* n1 = n0 + 3;
      const int32_t a = H.elem_v[2 * e], b = H.elem_v[2 * e + 1];
      if (dim == 3) {
        const float w[12] = {vtx(a, 0), vtx(a, 1), vtx(a, 2), (float)n0[0],
                             vtx(b, 0), vtx(b, 1), vtx(b, 2), (float)n0[1],
                             (float)n0[2], (float)n1[0], (float)n1[1], (float)n1[2]};
        std::memcpy(&epay[12 * i], w, sizeof w);
      } else {
        const float w[8] = {vtx(a, 0), vtx(a, 1), (float)n0[0], (float)n0[1],
                            (float)n1[0], (float)n1[1], 0.0f, 0.0f};
        std::memcpy(&epay[8 * i], w, sizeof w);
      }
    }
    pad(epay, dim == 3 ? 12 : 8);
    wost::SceneDev& D = s->dev;
    D.dim = dim;
    const float* fp;
    const int32_t* ip;
    if ((st = upload(s, H.treeD.nodes, &fp)) != WOST_OK) { delete s; return st; }
    D.dn = (const float4*)fp;
    if ((st = upload(s, dpay, &fp)) != WOST_OK) { delete s; return st; }
    D.dp = (const float4*)fp;
    if ((st = upload(s, did, &ip)) != WOST_OK) { delete s; return st; }
    D.did = ip;
    D.nD = (int)did.size();
    if ((st = upload(s, H.treeN.nodes, &fp)) != WOST_OK) { delete s; return st; }
    D.nn = (const float4*)fp;
    if ((st = upload(s, npay, &fp)) != WOST_OK) { delete s; return st; }
    D.np = (const float4*)fp;
    if ((st = upload(s, narea, &fp)) != WOST_OK) { delete s; return st; }
    D.narea = fp;
    if ((st = upload(s, nid, &ip)) != WOST_OK) { delete s; return st; }
    D.nid = ip;
    if ((st = upload(s, ninv, &ip)) != WOST_OK) { delete s; return st; }
    D.ninv = ip;
    s->ninv = ninv;
    D.nN = (int)nid.size();
    // silhouette tree, 3D: one 128-byte record per node (its node words, then
    // its two child cones), so that a visit reads one cache line: the trees
    // of a large mesh live beyond L2, and the record measured 35 % faster
    // than separate node and cone arrays on 1.31M triangles.  2D: separate
    // arrays, whose smaller footprint measured faster on the L2-resident
    // star polygon.
    if (dim == 2) {
      if ((st = upload(s, H.treeS.nodes, &fp)) != WOST_OK) { delete s; return st; }
      D.sn = (const float4*)fp;
      if ((st = upload(s, H.treeS.cones, &fp)) != WOST_OK) { delete s; return st; }
      D.sc = (const float4*)fp;
    } else {
      const size_t nf = dim == 3 ? 16 : 12, nc = dim == 3 ? 12 : 8;
      const size_t nn = H.treeS.nodes.size() / nf;
      std::vector<float> rec(nn * 4 * wost::kSRec, 0.0f);
      for (size_t i = 0; i < nn; ++i) {
        std::memcpy(&rec[i * 4 * wost::kSRec], &H.treeS.nodes[i * nf], nf * sizeof(float));
        std::memcpy(&rec[i * 4 * wost::kSRec + nf], &H.treeS.cones[i * nc], nc * sizeof(float));
      }
      if ((st = upload(s, rec, &fp)) != WOST_OK) { delete s; return st; }
      D.sn = (const float4*)fp;
      D.sc = nullptr;
    }
    if ((st = upload(s, epay, &fp)) != WOST_OK) { delete s; return st; }
    D.se = (const float4*)fp;
    D.nE = (int)ne;
    D.topD = H.topD;
    D.topN = H.topN;
    D.topS = H.topS;
    D.tdn = D.tnn = D.tsn = D.tsc = nullptr;
    D.ctD = D.ctN = D.ctS = 0;
    D.g = fn_dev(desc->g);
    D.h = fn_dev(desc->h);
    D.f = fn_dev(desc->f);
    // double-sided flags per leaf slot (only a scene that has such
    // primitives runs the double-sided kernels, which read them)
    D.ds = 0;
    for (uint8_t b : H.bc) D.ds |= b >= 2;
    D.dside = nullptr;
    D.nside = nullptr;
    D.gm = fn_dev(desc->g_minus);
    D.hm = fn_dev(desc->h_minus);
    if (D.ds) {
      std::vector<uint8_t> dside(std::max<size_t>(1, did.size()), 0), nside(std::max<size_t>(1, nid.size()), 0);
      for (size_t i = 0; i < did.size(); ++i) dside[i] = H.bc[did[i]] >= 2;
      for (size_t i = 0; i < nid.size(); ++i) nside[i] = H.bc[nid[i]] >= 2;
      const uint8_t* bp;
      if ((st = upload(s, dside, &bp)) != WOST_OK) { delete s; return st; }
      D.dside = bp;
      if ((st = upload(s, nside, &bp)) != WOST_OK) { delete s; return st; }
      D.nside = bp;
    }
    auto pc_upload = [&](const wost_fn& f, wost::FnDev& fd) -> wost_status {
      if (f.kind != WOST_FN_PER_CORNER) return WOST_OK;
      std::vector<float> pc(f.per_corner, f.per_corner + (size_t)H.n_prims * dim);
      for (float x : pc)
        if (!std::isfinite(x)) return fail(WOST_ERR_INVALID_ARG, "non-finite per-corner value");
      const float* q;
      wost_status r = upload(s, pc, &q);
      fd.pc = q;
      return r;
    };
    if ((st = pc_upload(desc->g, D.g)) != WOST_OK) { delete s; return st; }
    if ((st = pc_upload(desc->h, D.h)) != WOST_OK) { delete s; return st; }
    if ((st = pc_upload(desc->g_minus, D.gm)) != WOST_OK) { delete s; return st; }
    // analytic Dirichlet shapes: (p0, p1, p2, radius), (p3, p4, p5, kind | inside << 4)
    D.sdf = nullptr;
    D.nS = (int)desc->n_sdf;
    D.sdf_id0 = (int)H.n_prims;
    if (D.nS > 0) {
      std::vector<float> sp(8 * (size_t)D.nS, 0.0f);
      for (int i = 0; i < D.nS; ++i) {
        const wost_sdf& f = desc->sdf[i];
        const int32_t code = f.kind | (f.inside << 4);
        float cw;
        std::memcpy(&cw, &code, 4);
        const float w[8] = {(float)f.p[0], (float)f.p[1], (float)f.p[2], (float)f.p[6],
                            (float)f.p[3], (float)f.p[4], (float)f.p[5], cw};
        std::memcpy(&sp[8 * i], w, sizeof w);
      }
      if ((st = upload(s, sp, &fp)) != WOST_OK) { delete s; return st; }
      D.sdf = (const float4*)fp;
    }
    if ((st = pc_upload(desc->h_minus, D.hm)) != WOST_OK) { delete s; return st; }
    D.offset = (float)(kOffsetRel * H.L);
    D.escape2 = (float)((kEscapeRel * H.L) * (kEscapeRel * H.L));
    D.escape = (float)(kEscapeRel * H.L);
    D.cx = (float)H.center[0];
    D.cy = (float)H.center[1];
    D.cz = (float)H.center[2];
    s->grid_default = wost::max_resident_blocks(dim, true);
    s->grid_lane = wost::max_resident_blocks(dim, false);
    hipError_t ee = hipEventCreate(&s->ev0);
    if (ee == hipSuccess) ee = hipEventCreate(&s->ev1);
    if (ee != hipSuccess) {
      delete s;
      return hip_fail(ee, "hipEventCreate");
    }
    *out = s;
    return WOST_OK;
  } catch (const std::bad_alloc&) {
    delete s;
    return fail(WOST_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    delete s;
    return fail(WOST_ERR_INTERNAL, "unexpected exception");
  }
}

wost_status wost_destroy_scene(wost_scene s) {
  g_err.clear();
  if (!s) return WOST_OK;
  (void)hipDeviceSynchronize();
  delete s;
  return WOST_OK;
}

wost_status wost_get_scene_info(wost_scene s, wost_scene_info* info) {
  g_err.clear();
  if (!s || !info) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  fill_info(s->host, info);
  info->device_bytes = s->device_bytes;
  info->n_sdf = s->dev.nS;
  return WOST_OK;
}

}  // extern "C"

namespace {

// Boundary start codes of the device (WalkParams::start) from the caller's
// primitive ids: p >= 0 a Neumann primitive, its "+" side; -2 - p the "-"
// side of a double-sided Neumann primitive p; -1 an interior point.
wost_status start_codes(wost_scene s, const int32_t* prims, int64_t n, std::vector<int32_t>& slot) {
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = prims[i];
    if (c == -1) continue;
    const bool minus = c <= -2;
    const int64_t p = minus ? -2 - (int64_t)c : c;
    const bool ok = p >= 0 && p < (int64_t)s->ninv.size() && s->ninv[p] >= 0 &&
                    (!minus || s->host.bc[p] == 3);
    if (!ok)
      return fail(WOST_ERR_INVALID_ARG, "prims[" + std::to_string(i) + "] = " + std::to_string(c) +
                                            " is neither -1, a Neumann primitive, nor -2 - a "
                                            "double-sided Neumann primitive");
    slot[i] = minus ? -2 - s->ninv[p] : s->ninv[p];
  }
  return WOST_OK;
}

// d_start (device, [n] start codes, see start_codes) or NULL: boundary starts
wost_status solve_impl(wost_scene s, const float* d_points, const int32_t* d_start, int64_t n,
                       int32_t W, float eps, uint64_t seed, uint32_t point_base, uint32_t walk_base,
                       const wost_solve_opts* opts, double* d_mean, double* d_var, hipStream_t hs) {
  const bool count = opts && (opts->flags & WOST_SOLVE_COUNT_TRAFFIC);
  wost_status st;
  if ((st = ensure_scratch(s, (size_t)std::max<int64_t>(1, n * (int64_t)W))) != WOST_OK) return st;
  HIP_TRY(wost::launch_fill_u64(s->ctr, kCtrWords, hs), "fill counters");
  s->ctr_view = s->ctr;
  s->have_stats = true;
  s->counted = count;
  s->last_n = n;
  s->last_W = W;
  if (n == 0) {
    HIP_TRY(hipEventRecord(s->ev0, hs), "hipEventRecord");
    HIP_TRY(hipEventRecord(s->ev1, hs), "hipEventRecord");
    return WOST_OK;
  }
  wost::SceneDev S;
  wost::WalkParams P{};
  int mode, grid;
  apply_opts(s, opts, eps, S, P, mode, grid);
  P.points = d_points;
  P.start = d_start;
  P.n_points = n;
  P.W = W;
  P.point_base = point_base;
  P.walk_base = walk_base;
  P.seed_lo = (uint32_t)seed;
  P.seed_hi = (uint32_t)(seed >> 32);
  P.est = s->est;
  P.stats = s->ctr;
  P.counter = s->ctr + 4;
  P.traffic = s->ctr + kTrafficBase;
  P.events = s->ctr + kEventBase;
  s->last_mode = count ? 1 : (mode == 2 ? 3 : mode);
  s->last_grid = (count || mode == 1) ? (int)((n * (int64_t)W + wost::kBlock - 1) / wost::kBlock) : grid;
  HIP_TRY(hipEventRecord(s->ev0, hs), "hipEventRecord");
  HIP_TRY(wost::launch_walks(S, P, mode, grid, count, hs), "walk kernel launch");
  HIP_TRY(hipEventRecord(s->ev1, hs), "hipEventRecord");
  HIP_TRY(wost::launch_reduce(s->est, n, W, d_mean, d_var, hs), "reduce kernel launch");
  return WOST_OK;
}

wost_status check_ex_args(wost_scene s, const float* d_points, int64_t n, int32_t W, float eps,
                          const wost_solve_opts* opts, double* d_mean, double* d_var) {
  wost_status st = check_solve_args(s, n, W, eps, opts);
  if (st != WOST_OK) return st;
  if (n > 0 && (!d_points || !d_mean || !d_var)) return fail(WOST_ERR_INVALID_ARG, "NULL array");
  if (opts && (opts->flags & ~WOST_SOLVE_COUNT_TRAFFIC) != 0)
    return fail(WOST_ERR_INVALID_ARG, "unknown opts.flags bits");
  return WOST_OK;
}

}  // namespace

extern "C" {

wost_status wost_solve_ex(wost_scene s, const float* d_points, int64_t n, int32_t W, float eps,
                          uint64_t seed, uint32_t point_base, uint32_t walk_base,
                          const wost_solve_opts* opts, double* d_mean, double* d_var, void* stream) {
  g_err.clear();
  wost_status st = check_ex_args(s, d_points, n, W, eps, opts, d_mean, d_var);
  if (st != WOST_OK) return st;
  return solve_impl(s, d_points, nullptr, n, W, eps, seed, point_base, walk_base, opts, d_mean, d_var,
                    (hipStream_t)stream);
}

wost_status wost_solve_boundary_ex(wost_scene s, const float* d_points, const int32_t* prims,
                                   int64_t n, int32_t W, float eps, uint64_t seed, uint32_t point_base,
                                   uint32_t walk_base, const wost_solve_opts* opts, double* d_mean,
                                   double* d_var, void* stream) {
  g_err.clear();
  wost_status st = check_ex_args(s, d_points, n, W, eps, opts, d_mean, d_var);
  if (st != WOST_OK) return st;
  if (n > 0 && !prims) return fail(WOST_ERR_INVALID_ARG, "prims is NULL");
  std::vector<int32_t> slot((size_t)std::max<int64_t>(1, n), -1);
  if ((st = start_codes(s, prims, n, slot)) != WOST_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  // the staging buffer may still be read by this scene's previous boundary
  // solve on the stream: wait for it before overwriting
  HIP_TRY(hipStreamSynchronize(hs), "hipStreamSynchronize");
  if (slot.size() > s->start_cap) {
    if (s->start) HIP_TRY(hipFree(s->start), "hipFree");
    s->start = nullptr;
    s->start_cap = 0;
    HIP_TRY(hipMalloc((void**)&s->start, slot.size() * sizeof(int32_t)), "hipMalloc start slots");
    s->start_cap = slot.size();
  }
  HIP_TRY(hipMemcpy(s->start, slot.data(), slot.size() * sizeof(int32_t), hipMemcpyHostToDevice),
          "hipMemcpy start slots");
  return solve_impl(s, d_points, s->start, n, W, eps, seed, point_base, walk_base, opts, d_mean, d_var,
                    hs);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free solve
// ---------------------------------------------------------------------------
// The scratch of wost_solve_ex -- the solve's counters and the per-walk
// estimates -- in one fixed device array per GPU, so that the call makes no
// device allocation.  Host code never names the array in a device context:
// its address on the current device comes from hipGetSymbolAddress, looked
// up once per device on the first call there.
namespace {
constexpr int64_t kStaticWalks = int64_t(1) << 23;   // walk estimates per chunk (32 MiB)
constexpr int kStaticCtrWords = 512;                 // counter block (4 KiB)
static_assert(kCtrWords <= kStaticCtrWords, "the counters must fit the fixed array's counter block");
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned long long scratch[kStaticCtrWords + kStaticWalks / 2];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

wost_status static_scratch(unsigned long long** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(WOST_ERR_NOT_SUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned long long*>(g_scratch_ptr[dev]);
  return WOST_OK;
}
}  // namespace

extern "C" {

wost_status wost_solve_ex_noalloc(wost_scene s, const float* d_points, int64_t n, int32_t W, float eps,
                                  uint64_t seed, uint32_t point_base, uint32_t walk_base,
                                  const wost_solve_opts* opts, double* d_mean, double* d_var, void* stream) {
  g_err.clear();
  wost_status st = check_ex_args(s, d_points, n, W, eps, opts, d_mean, d_var);
  if (st != WOST_OK) return st;
  if (opts && opts->flags != 0)
    return fail(WOST_ERR_INVALID_ARG, "the no-alloc solve takes no opts.flags (no traffic accounting)");
  if ((int64_t)W > kStaticWalks)
    return fail(WOST_ERR_INVALID_ARG, "walks_per_point exceeds the no-alloc limit of 2^23 walks per point");
  unsigned long long* ctr = nullptr;
  if ((st = static_scratch(&ctr)) != WOST_OK) return st;
  float* est = reinterpret_cast<float*>(ctr + kStaticCtrWords);
  hipStream_t hs = (hipStream_t)stream;
  // a fill kernel, not a memset: the call may be captured into a graph
  HIP_TRY(wost::launch_fill_u64(ctr, kCtrWords, hs), "fill counters");
  s->ctr_view = ctr;
  s->have_stats = true;
  s->counted = false;
  s->last_n = n;
  s->last_W = W;
  HIP_TRY(hipEventRecord(s->ev0, hs), "hipEventRecord");
  if (n > 0) {
    wost::SceneDev S;
    wost::WalkParams P{};
    int mode, grid;
    apply_opts(s, opts, eps, S, P, mode, grid);
    P.W = W;
    P.walk_base = walk_base;
    P.seed_lo = (uint32_t)seed;
    P.seed_hi = (uint32_t)(seed >> 32);
    P.est = est;
    P.stats = ctr;
    P.counter = ctr + 4;
    P.traffic = ctr + kTrafficBase;
    P.events = ctr + kEventBase;
    s->last_mode = mode == 2 ? 3 : mode;
    // points in chunks whose walk estimates fit the array; every chunk keeps
    // its points' random-number ids, so the walks are those of one launch
    const int64_t chunk = kStaticWalks / W;
    for (int64_t p0 = 0; p0 < n; p0 += chunk) {
      const int64_t np = std::min(chunk, n - p0);
      P.points = d_points + p0 * s->host.dim;
      P.n_points = np;
      P.point_base = point_base + (uint32_t)p0;
      s->last_grid = mode == 1 ? (int)((np * (int64_t)W + wost::kBlock - 1) / wost::kBlock) : grid;
      if (p0 > 0) HIP_TRY(wost::launch_fill_u64(P.counter, 1, hs), "reset work cursor");
      HIP_TRY(wost::launch_walks(S, P, mode, grid, false, hs), "walk kernel launch");
      HIP_TRY(wost::launch_reduce(est, np, W, d_mean + p0, d_var + p0, hs), "reduce kernel launch");
    }
  }
  HIP_TRY(hipEventRecord(s->ev1, hs), "hipEventRecord");
  return WOST_OK;
}

wost_status wost_solve(wost_scene s, const float* points, int64_t n, int32_t W, float eps,
                       uint64_t seed, double* mean_out, double* var_out) {
  g_err.clear();
  wost_status st = check_solve_args(s, n, W, eps);
  if (st != WOST_OK) return st;
  if (n > 0 && (!points || !mean_out || !var_out)) return fail(WOST_ERR_INVALID_ARG, "NULL array");
  if (n == 0) return WOST_OK;
  const int dim = s->host.dim;
  DevBuf<float> dp;
  DevBuf<double> dm, dv;
  HIP_TRY(dp.alloc((size_t)n * dim), "hipMalloc points");
  HIP_TRY(dm.alloc((size_t)n), "hipMalloc mean");
  HIP_TRY(dv.alloc((size_t)n), "hipMalloc var");
  HIP_TRY(hipMemcpy(dp.p, points, (size_t)n * dim * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  st = wost_solve_ex(s, dp.p, n, W, eps, seed, 0, 0, nullptr, dm.p, dv.p, nullptr);
  if (st != WOST_OK) return st;
  HIP_TRY(hipMemcpy(mean_out, dm.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(var_out, dv.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  return WOST_OK;
}

wost_status wost_autotune(wost_scene s, const float* d_points, int64_t n, int32_t W, float eps,
                          uint64_t seed, int64_t sample_walks, wost_solve_opts* opts, void* stream) {
  g_err.clear();
  wost_status st = check_solve_args(s, n, W, eps, opts);
  if (st != WOST_OK) return st;
  if (!opts || (n > 0 && !d_points)) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  if (n == 0) return WOST_OK;
  if (sample_walks <= 0) sample_walks = int64_t(1) << 20;
  const int64_t ns = std::max<int64_t>(1, std::min<int64_t>(n, sample_walks / W));
  DevBuf<double> dm, dv;
  HIP_TRY(dm.alloc((size_t)ns), "hipMalloc");
  HIP_TRY(dv.alloc((size_t)ns), "hipMalloc");
  hipStream_t hs = (hipStream_t)stream;
  const int cap = s->grid_default;
  struct Cand { int refill, grid, order; };
  std::vector<Cand> cands;
  for (int order : {0, 1})
    for (int refill : {1, 8, 32})
      for (int grid : {cap, cap / 2 > 0 ? cap / 2 : 1}) cands.push_back({refill, grid, order});
  float best_ms = 3.0e38f;
  Cand best = cands[0];
  for (int rep = 0; rep < 2; ++rep) {        // the first pass also warms caches and code
    for (const Cand& c : cands) {
      wost_solve_opts o = *opts;
      o.mode = 0;
      o.flags = 0;
      o.refill = c.refill;
      o.grid = c.grid;
      o.walk_order = c.order;
      st = wost_solve_ex(s, d_points, ns, W, eps, seed, 0, 0, &o, dm.p, dv.p, stream);
      if (st != WOST_OK) return st;
      HIP_TRY(hipStreamSynchronize(hs), "hipStreamSynchronize");
      wost_stats ws;
      st = wost_get_stats(s, &ws);
      if (st != WOST_OK) return st;
      if (rep == 1 && ws.kernel_ms < best_ms) {
        best_ms = (float)ws.kernel_ms;
        best = c;
      }
    }
  }
  opts->mode = 0;
  opts->refill = best.refill;
  opts->grid = best.grid;
  opts->walk_order = best.order;
  return WOST_OK;
}

wost_status wost_get_stats(wost_scene s, wost_stats* out) {
  g_err.clear();
  if (!s || !out) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  if (!s->have_stats) return WOST_OK;
  HIP_TRY(hipEventSynchronize(s->ev1), "hipEventSynchronize");
  unsigned long long h[4];
  HIP_TRY(hipMemcpy(h, s->ctr_view, sizeof h, hipMemcpyDeviceToHost), "hipMemcpy stats");
  out->steps = h[0];
  out->walks = h[1];
  out->capped = h[2];
  out->escaped = h[3];
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, s->ev0, s->ev1), "hipEventElapsedTime");
  out->kernel_ms = ms;
  out->mode = s->last_mode;
  out->grid_blocks = s->last_grid;
  return WOST_OK;
}

wost_status wost_get_walk_events(wost_scene s, int32_t max, uint32_t* point_ids, uint32_t* walk_ids,
                                 int32_t* steps, int32_t* kinds, int32_t* n_out) {
  g_err.clear();
  if (!s || !n_out) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  *n_out = 0;
  if (max < 0 || (max > 0 && (!point_ids || !walk_ids || !steps || !kinds)))
    return fail(WOST_ERR_INVALID_ARG, "bad output arrays");
  if (!s->have_stats) return WOST_OK;
  HIP_TRY(hipEventSynchronize(s->ev1), "hipEventSynchronize");
  unsigned long long h[1 + 2 * wost::kEventCap];
  HIP_TRY(hipMemcpy(h, s->ctr_view + kEventBase, sizeof h, hipMemcpyDeviceToHost), "hipMemcpy events");
  const int n = (int)std::min<unsigned long long>(h[0], (unsigned long long)wost::kEventCap);
  const int m = std::min(n, (int)max);
  for (int i = 0; i < m; ++i) {
    point_ids[i] = (uint32_t)(h[1 + 2 * i] >> 32);
    walk_ids[i] = (uint32_t)h[1 + 2 * i];
    steps[i] = (int32_t)(h[2 + 2 * i] >> 8);
    kinds[i] = (int32_t)(h[2 + 2 * i] & 0xff);
  }
  *n_out = m;
  return WOST_OK;
}

wost_status wost_get_traffic(wost_scene s, wost_traffic* out) {
  g_err.clear();
  if (!s || !out) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  const int dim = s->host.dim;
  out->node_bytes = dim == 3 ? 64 : 48;
  out->cone_bytes = dim == 3 ? 48 : 32;
  out->prim_bytes = dim == 3 ? 48 : 16;
  out->elem_bytes = dim == 3 ? 48 : 32;
  if (!s->have_stats || !s->counted) return WOST_OK;
  HIP_TRY(hipEventSynchronize(s->ev1), "hipEventSynchronize");
  unsigned long long h[wost::kTrafficCounters];
  HIP_TRY(hipMemcpy(h, s->ctr_view + kTrafficBase, sizeof h, hipMemcpyDeviceToHost), "hipMemcpy traffic");
  out->q1_nodes = h[wost::kCntQ1Node];
  out->q1_prims = h[wost::kCntQ1Prim];
  out->q2_nodes = h[wost::kCntQ2Node];
  out->q2_cones = h[wost::kCntQ2Cone];
  out->q2_elems = h[wost::kCntQ2Elem];
  out->q3_nodes = h[wost::kCntQ3Node];
  out->q3_prims = h[wost::kCntQ3Prim];
  out->q4_nodes = h[wost::kCntQ4Node];
  out->q4_prims = h[wost::kCntQ4Prim];
  out->vis_nodes = h[wost::kCntVisNode];
  out->vis_prims = h[wost::kCntVisPrim];
  out->wave_q1 = h[wost::kWaveQ1Iter];
  out->wave_q1_leaf = h[wost::kWaveQ1Leaf];
  out->wave_q2 = h[wost::kWaveQ2Iter];
  out->wave_q2_leaf = h[wost::kWaveQ2Leaf];
  out->wave_q3 = h[wost::kWaveQ3Iter];
  out->wave_q3_leaf = h[wost::kWaveQ3Leaf];
  out->wave_q4 = h[wost::kWaveQ4Iter];
  out->wave_vis = h[wost::kWaveVisIter];
  out->wave_vis_leaf = h[wost::kWaveVisLeaf];
  out->wave_steps = h[wost::kWaveSteps];
  out->cyc_q1 = h[wost::kCycQ1];
  out->cyc_q2 = h[wost::kCycQ2];
  out->cyc_q3 = h[wost::kCycQ3];
  out->cyc_q4 = h[wost::kCycQ4];
  out->cyc_rest = h[wost::kCycRest];
  // per walk: its start point read, its estimate written and read back;
  // per point: mean and variance written
  out->io_bytes = (uint64_t)s->last_n * (uint64_t)s->last_W * (uint64_t)(4 * dim + 8) +
                  (uint64_t)s->last_n * 16ull;
  const uint64_t nodes = out->q1_nodes + out->q2_nodes + out->q3_nodes + out->q4_nodes + out->vis_nodes;
  const uint64_t prims = out->q1_prims + out->q3_prims + out->vis_prims;
  out->bytes = nodes * out->node_bytes + out->q2_cones * out->cone_bytes + prims * out->prim_bytes +
               out->q4_prims * (out->prim_bytes + 4) + out->q2_elems * out->elem_bytes + out->io_bytes;
  return WOST_OK;
}

wost_status wost_trace_walks(wost_scene s, const float* points, const uint32_t* pids,
                             const uint32_t* wids, const int32_t* prims, int64_t n, float eps,
                             uint64_t seed, const wost_solve_opts* opts, int32_t max_rec,
                             wost_step_rec* recs, int32_t* n_steps, float* values) {
  g_err.clear();
  wost_status st = check_solve_args(s, n, 1, eps, opts);
  if (st != WOST_OK) return st;
  if (max_rec < 1) return fail(WOST_ERR_INVALID_ARG, "max_rec < 1");
  if (n == 0) return WOST_OK;
  if (!points || !pids || !wids || !recs || !n_steps || !values) return fail(WOST_ERR_INVALID_ARG, "NULL array");
  const int dim = s->host.dim;
  DevBuf<float> dp, dval;
  DevBuf<uint32_t> dpi, dwi;
  DevBuf<wost::StepRec> drec;
  DevBuf<int> dns;
  HIP_TRY(dp.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dval.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dpi.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dwi.alloc((size_t)n), "hipMalloc");
  HIP_TRY(drec.alloc((size_t)n * max_rec), "hipMalloc");
  HIP_TRY(dns.alloc((size_t)n), "hipMalloc");
  HIP_TRY(hipMemcpy(dp.p, points, (size_t)n * dim * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemcpy(dpi.p, pids, (size_t)n * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemcpy(dwi.p, wids, (size_t)n * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemset(drec.p, 0, (size_t)n * max_rec * sizeof(wost::StepRec)), "hipMemset");
  DevBuf<int32_t> dst;
  if (prims) {
    std::vector<int32_t> slot((size_t)n, -1);
    wost_status st2 = start_codes(s, prims, n, slot);
    if (st2 != WOST_OK) return st2;
    HIP_TRY(dst.alloc((size_t)n), "hipMalloc");
    HIP_TRY(hipMemcpy(dst.p, slot.data(), (size_t)n * 4, hipMemcpyHostToDevice), "hipMemcpy");
  }
  wost::SceneDev S;
  wost::WalkParams P{};
  int mode, grid;
  apply_opts(s, opts, eps, S, P, mode, grid);
  P.points = dp.p;
  P.start = dst.p;
  P.n_points = n;
  P.W = 1;
  P.seed_lo = (uint32_t)seed;
  P.seed_hi = (uint32_t)(seed >> 32);
  HIP_TRY(wost::launch_trace(S, P, dpi.p, dwi.p, n, max_rec, drec.p, dns.p, dval.p, nullptr), "trace launch");
  HIP_TRY(hipDeviceSynchronize(), "trace kernel");
  HIP_TRY(hipMemcpy(recs, drec.p, (size_t)n * max_rec * sizeof(wost::StepRec), hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(n_steps, dns.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(values, dval.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  return WOST_OK;
}

wost_status wost_probe_closest_point(wost_scene s, const float* x, int64_t n, float* d, float* xbar,
                                     int32_t* prim) {
  g_err.clear();
  if (!s) return fail(WOST_ERR_INVALID_ARG, "scene is NULL");
  if (n <= 0) return n == 0 ? WOST_OK : fail(WOST_ERR_INVALID_ARG, "n < 0");
  if (!x || !d || !xbar || !prim) return fail(WOST_ERR_INVALID_ARG, "NULL array");
  const int dim = s->host.dim;
  DevBuf<float> dx, dd, dxb;
  DevBuf<int> dpr;
  HIP_TRY(dx.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dd.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dxb.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dpr.alloc((size_t)n), "hipMalloc");
  HIP_TRY(hipMemcpy(dx.p, x, (size_t)n * dim * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(wost::launch_probe_q1(s->dev, dx.p, n, dd.p, dxb.p, dpr.p, nullptr), "probe launch");
  HIP_TRY(hipDeviceSynchronize(), "probe kernel");
  HIP_TRY(hipMemcpy(d, dd.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(xbar, dxb.p, (size_t)n * dim * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(prim, dpr.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  return WOST_OK;
}

wost_status wost_probe_silhouette(wost_scene s, const float* x, const float* rmax, int64_t n, float* d) {
  g_err.clear();
  if (!s) return fail(WOST_ERR_INVALID_ARG, "scene is NULL");
  if (n <= 0) return n == 0 ? WOST_OK : fail(WOST_ERR_INVALID_ARG, "n < 0");
  if (!x || !rmax || !d) return fail(WOST_ERR_INVALID_ARG, "NULL array");
  const int dim = s->host.dim;
  DevBuf<float> dx, dr, dd;
  HIP_TRY(dx.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dr.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dd.alloc((size_t)n), "hipMalloc");
  HIP_TRY(hipMemcpy(dx.p, x, (size_t)n * dim * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemcpy(dr.p, rmax, (size_t)n * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(wost::launch_probe_q2(s->dev, dx.p, dr.p, n, dd.p, nullptr), "probe launch");
  HIP_TRY(hipDeviceSynchronize(), "probe kernel");
  HIP_TRY(hipMemcpy(d, dd.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  return WOST_OK;
}

wost_status wost_probe_ray(wost_scene s, const float* o, const float* v, const float* tmax,
                           const int32_t* skip, int64_t n, float* t, int32_t* prim) {
  g_err.clear();
  if (!s) return fail(WOST_ERR_INVALID_ARG, "scene is NULL");
  if (n <= 0) return n == 0 ? WOST_OK : fail(WOST_ERR_INVALID_ARG, "n < 0");
  if (!o || !v || !tmax || !skip || !t || !prim) return fail(WOST_ERR_INVALID_ARG, "NULL array");
  const int dim = s->host.dim;
  for (int64_t i = 0; i < n; ++i)
    if (skip[i] < -1 || skip[i] >= s->host.n_prims) return fail(WOST_ERR_INVALID_ARG, "skip id out of range");
  DevBuf<float> dO, dV, dT, dt;
  DevBuf<int> ds, dpr;
  HIP_TRY(dO.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dV.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dT.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dt.alloc((size_t)n), "hipMalloc");
  HIP_TRY(ds.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dpr.alloc((size_t)n), "hipMalloc");
  HIP_TRY(hipMemcpy(dO.p, o, (size_t)n * dim * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemcpy(dV.p, v, (size_t)n * dim * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemcpy(dT.p, tmax, (size_t)n * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemcpy(ds.p, skip, (size_t)n * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(wost::launch_probe_q3(s->dev, dO.p, dV.p, dT.p, ds.p, n, dt.p, dpr.p, nullptr), "probe launch");
  HIP_TRY(hipDeviceSynchronize(), "probe kernel");
  HIP_TRY(hipMemcpy(t, dt.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(prim, dpr.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  return WOST_OK;
}

wost_status wost_probe_neumann_sample(wost_scene s, const float* x, const float* r, int64_t n,
                                      uint64_t seed, float* z, float* pdf, int32_t* prim) {
  g_err.clear();
  if (!s) return fail(WOST_ERR_INVALID_ARG, "scene is NULL");
  if (n <= 0) return n == 0 ? WOST_OK : fail(WOST_ERR_INVALID_ARG, "n < 0");
  if (!x || !r || !z || !pdf || !prim) return fail(WOST_ERR_INVALID_ARG, "NULL array");
  const int dim = s->host.dim;
  DevBuf<float> dx, dr, dz, dpdf;
  DevBuf<int> dpr;
  HIP_TRY(dx.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dr.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dz.alloc((size_t)n * dim), "hipMalloc");
  HIP_TRY(dpdf.alloc((size_t)n), "hipMalloc");
  HIP_TRY(dpr.alloc((size_t)n), "hipMalloc");
  HIP_TRY(hipMemcpy(dx.p, x, (size_t)n * dim * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMemcpy(dr.p, r, (size_t)n * 4, hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(wost::launch_probe_q4(s->dev, dx.p, dr.p, n, (uint32_t)seed, (uint32_t)(seed >> 32), dz.p,
                                dpdf.p, dpr.p, nullptr), "probe launch");
  HIP_TRY(hipDeviceSynchronize(), "probe kernel");
  HIP_TRY(hipMemcpy(z, dz.p, (size_t)n * dim * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(pdf, dpdf.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemcpy(prim, dpr.p, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  return WOST_OK;
}

wost_status wost_measure_l2_read(int64_t bytes, int32_t reps, double* gbs) {
  g_err.clear();
  if (!gbs) return fail(WOST_ERR_INVALID_ARG, "gbs is NULL");
  if (bytes <= 0) bytes = 2 << 20;
  if (reps <= 0) reps = 16;
  if (bytes % 16 != 0 || bytes > (int64_t(64) << 20))
    return fail(WOST_ERR_INVALID_ARG, "bytes must be a multiple of 16 and at most 64 MiB");
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
  const int blocks = 4 * std::max(cus, 1);
  DevBuf<float> buf, sink;
  HIP_TRY(buf.alloc((size_t)(bytes / 4)), "hipMalloc");
  HIP_TRY(sink.alloc((size_t)blocks), "hipMalloc");
  HIP_TRY(hipMemset(buf.p, 0, (size_t)bytes), "hipMemset");
  const int n4 = (int)(bytes / 16);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
  hipError_t e = wost::launch_stream_read((const float4*)buf.p, n4, 1, blocks, sink.p, nullptr);   // warm the caches
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  if (e == hipSuccess) e = wost::launch_stream_read((const float4*)buf.p, n4, reps, blocks, sink.p, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "L2 read measurement");
  *gbs = (double)blocks * (double)bytes * reps / (ms * 1e-3) / 1e9;
  return WOST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
struct wost_batch_s {
  float* est = nullptr;
  size_t est_cap = 0;
  wost::BatchItem* d_items = nullptr;
  size_t items_cap = 0;
  unsigned long long* ctr = nullptr;   // stats[4], then one cursor per group
  int ctr_cap = 0;
  hipStream_t cap_stream = nullptr;    // capture stream (a graph cannot be captured on the null stream)
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> signature; // the items + options the cached graph was captured for
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool have_stats = false;
  int last_grid = 0;
  ~wost_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (est) (void)hipFree(est);
    if (d_items) (void)hipFree(d_items);
    if (ctr) (void)hipFree(ctr);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

namespace {

struct Group {
  int dim;
  bool hh, hf, ds;
  std::vector<int> idx;   // item indices
  size_t first = 0;       // offset of the group's entries in the device table
  int64_t n_chunks = 0;
};

}  // namespace

extern "C" {

wost_status wost_batch_create(wost_batch* out) {
  g_err.clear();
  if (!out) return fail(WOST_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  wost_batch_s* b = new (std::nothrow) wost_batch_s();
  if (!b) return fail(WOST_ERR_OUT_OF_MEMORY, "host allocation failed");
  hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "batch create");
  }
  *out = b;
  return WOST_OK;
}

wost_status wost_batch_destroy(wost_batch b) {
  g_err.clear();
  if (!b) return WOST_OK;
  (void)hipDeviceSynchronize();
  delete b;
  return WOST_OK;
}

wost_status wost_solve_batch(wost_batch b, const wost_batch_item* items, int32_t n_items,
                             const wost_solve_opts* opts, void* stream) {
  g_err.clear();
  if (!b) return fail(WOST_ERR_INVALID_ARG, "batch is NULL");
  if (n_items < 0 || (n_items > 0 && !items)) return fail(WOST_ERR_INVALID_ARG, "bad item array");
  if (opts && (opts->flags != 0 || opts->mode != 0))
    return fail(WOST_ERR_INVALID_ARG, "batched form: opts.mode and opts.flags must be 0");
  std::vector<Group> groups;
  int64_t est_total = 0;
  std::vector<int64_t> est_off(n_items, 0);
  for (int i = 0; i < n_items; ++i) {
    const wost_batch_item& it = items[i];
    wost_status st = check_solve_args(it.scene, it.n_points, it.walks_per_point, it.eps, opts);
    if (st != WOST_OK) return fail(st, "item " + std::to_string(i) + ": " + g_err);
    if (it.n_points > 0 && (!it.d_points || !it.d_mean || !it.d_var))
      return fail(WOST_ERR_INVALID_ARG, "item " + std::to_string(i) + ": NULL array");
    if (it.n_points == 0) continue;
    est_off[i] = est_total;
    est_total += it.n_points * (int64_t)it.walks_per_point;
    const wost::SceneDev& S = it.scene->dev;
    const bool hh = wost::has_neumann_data(S), hf = S.f.kind != 0, ds = S.ds != 0;
    Group* g = nullptr;
    for (Group& q : groups)
      if (q.dim == S.dim && q.hh == hh && q.hf == hf && q.ds == ds) g = &q;
    if (!g) {
      groups.push_back(Group{S.dim, hh, hf, ds, {}, 0, 0});
      g = &groups.back();
    }
    g->idx.push_back(i);
  }
  // chunk size: the caller's, else about four chunks per resident wave
  // (64 to 2048 walks, a multiple of 64), so that a small batch -- a serving
  // round -- still spreads over every wave while a large one keeps the
  // work-queue traffic low
  int chunk = (opts && opts->chunk_walks > 0) ? opts->chunk_walks : 0;
  if (chunk == 0) {
    const int64_t waves = (int64_t)wost::max_resident_blocks(3, true) * (wost::kBlock / 64);
    int64_t c = (est_total + 4 * waves - 1) / (4 * waves);
    c = ((c + 63) / 64) * 64;
    chunk = (int)std::min<int64_t>(2048, std::max<int64_t>(64, c));
  }
  // host table
  std::vector<wost::BatchItem> table;
  for (Group& g : groups) {
    g.first = table.size();
    int64_t chunks = 0;
    for (int i : g.idx) {
      const wost_batch_item& it = items[i];
      wost::BatchItem B{};
      int mode_unused, grid_unused;
      apply_opts(it.scene, opts, it.eps, B.S, B.P, mode_unused, grid_unused);
      B.P.points = it.d_points;
      B.P.n_points = it.n_points;
      B.P.W = it.walks_per_point;
      B.P.point_base = it.point_base;
      B.P.walk_base = it.walk_base;
      B.P.seed_lo = (uint32_t)it.seed;
      B.P.seed_hi = (uint32_t)(it.seed >> 32);
      B.P.est = nullptr;  // patched below once the buffer exists
      B.n_walks = it.n_points * (int64_t)it.walks_per_point;
      B.chunk_begin = chunks;
      chunks += (B.n_walks + chunk - 1) / chunk;
      table.push_back(B);
    }
    g.n_chunks = chunks;
  }
  // device buffers
  if ((size_t)std::max<int64_t>(1, est_total) > b->est_cap) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (b->est) HIP_TRY(hipFree(b->est), "hipFree");
    b->est = nullptr;
    b->est_cap = 0;
    HIP_TRY(hipMalloc((void**)&b->est, (size_t)std::max<int64_t>(1, est_total) * sizeof(float)), "hipMalloc batch estimates");
    b->est_cap = (size_t)std::max<int64_t>(1, est_total);
    b->signature.clear();
  }
  {
    size_t k = 0;
    for (Group& g : groups)
      for (int i : g.idx) table[k++].P.est = b->est + est_off[i];
  }
  if (table.size() > b->items_cap) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (b->d_items) HIP_TRY(hipFree(b->d_items), "hipFree");
    b->d_items = nullptr;
    HIP_TRY(hipMalloc((void**)&b->d_items, table.size() * sizeof(wost::BatchItem)), "hipMalloc batch table");
    b->items_cap = table.size();
    b->signature.clear();
  }
  const int ctr_words = 4 + (int)groups.size();
  if (ctr_words > b->ctr_cap) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (b->ctr) HIP_TRY(hipFree(b->ctr), "hipFree");
    b->ctr = nullptr;
    HIP_TRY(hipMalloc((void**)&b->ctr, ctr_words * sizeof(unsigned long long)), "hipMalloc batch counters");
    b->ctr_cap = ctr_words;
    b->signature.clear();
  }
  hipStream_t hs = (hipStream_t)stream;
  // the table must be in place before the graph runs: copy in stream order
  HIP_TRY(hipStreamSynchronize(hs), "hipStreamSynchronize");
  if (!table.empty())
    HIP_TRY(hipMemcpy(b->d_items, table.data(), table.size() * sizeof(wost::BatchItem), hipMemcpyHostToDevice),
            "hipMemcpy batch table");
  int grid = (opts && opts->grid > 0) ? opts->grid : 0;
  // signature of this batch: the table, the groups and the grid
  std::vector<unsigned char> sig(table.size() * sizeof(wost::BatchItem) + sizeof(int) * 2);
  if (!table.empty()) std::memcpy(sig.data(), table.data(), table.size() * sizeof(wost::BatchItem));
  std::memcpy(sig.data() + table.size() * sizeof(wost::BatchItem), &grid, sizeof(int));
  std::memcpy(sig.data() + table.size() * sizeof(wost::BatchItem) + sizeof(int), &chunk, sizeof(int));
  if (sig != b->signature || !b->exec) {
    if (b->exec) {
      HIP_TRY(hipGraphExecDestroy(b->exec), "hipGraphExecDestroy");
      b->exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = wost::launch_fill_u64(b->ctr, ctr_words, b->cap_stream);
    int used_grid = 0;
    for (size_t gi = 0; gi < groups.size() && e == hipSuccess; ++gi) {
      const Group& g = groups[gi];
      int gr = grid > 0 ? grid : wost::max_resident_blocks(g.dim, true);
      const int64_t cap = (g.n_chunks * (int64_t)chunk + wost::kBlock - 1) / wost::kBlock;
      if ((int64_t)gr > cap) gr = (int)std::max<int64_t>(1, cap);
      used_grid = std::max(used_grid, gr);
      e = wost::launch_batch(b->d_items + g.first, (int)g.idx.size(), g.dim, g.hh, g.hf, g.ds, g.n_chunks, chunk,
                             b->ctr + 4 + gi, b->ctr, gr, b->cap_stream);
    }
    for (int i = 0; i < n_items && e == hipSuccess; ++i) {
      const wost_batch_item& it = items[i];
      if (it.n_points == 0) continue;
      e = wost::launch_reduce(b->est + est_off[i], it.n_points, it.walks_per_point, it.d_mean, it.d_var,
                              b->cap_stream);
    }
    hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(e, "batch capture");
    }
    HIP_TRY(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(e, "hipGraphInstantiate");
    b->signature = sig;
    b->last_grid = used_grid;
  }
  HIP_TRY(hipEventRecord(b->ev0, hs), "hipEventRecord");
  HIP_TRY(hipGraphLaunch(b->exec, hs), "hipGraphLaunch");
  HIP_TRY(hipEventRecord(b->ev1, hs), "hipEventRecord");
  b->have_stats = true;
  return WOST_OK;
}

wost_status wost_batch_get_stats(wost_batch b, wost_stats* out) {
  g_err.clear();
  if (!b || !out) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  if (!b->have_stats) return WOST_OK;
  HIP_TRY(hipEventSynchronize(b->ev1), "hipEventSynchronize");
  unsigned long long h[4];
  HIP_TRY(hipMemcpy(h, b->ctr, sizeof h, hipMemcpyDeviceToHost), "hipMemcpy");
  out->steps = h[0];
  out->walks = h[1];
  out->capped = h[2];
  out->escaped = h[3];
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1), "hipEventElapsedTime");
  out->kernel_ms = ms;
  out->mode = 2;
  out->grid_blocks = b->last_grid;
  return WOST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving form
// ---------------------------------------------------------------------------
#include <chrono>
#include <deque>
#include <map>

namespace {

struct Request {
  int64_t id = 0;
  wost_scene scene = nullptr;
  std::vector<float> points;     // host copy
  int64_t n = 0;
  float eps = 0;
  uint64_t seed = 0;
  double target = 0;
  int32_t state = WOST_REQ_QUEUED;
  int32_t rounds = 0;
  int64_t walks = 0;
  int64_t next = 0;   // walks per point of the next round
  double max_se = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t bytes = 0;
  // device buffers while active
  float* d_points = nullptr;
  double *d_mean = nullptr, *d_m2 = nullptr, *d_rmean = nullptr, *d_rvar = nullptr;
  // results when done
  std::vector<double> mean, var;
  void free_device() {
    if (d_points) (void)hipFree(d_points);
    if (d_mean) (void)hipFree(d_mean);
    if (d_m2) (void)hipFree(d_m2);
    if (d_rmean) (void)hipFree(d_rmean);
    if (d_rvar) (void)hipFree(d_rvar);
    d_points = nullptr;
    d_mean = d_m2 = d_rmean = d_rvar = nullptr;
  }
};

}  // namespace

struct wost_server_s {
  wost_server_config cfg{};
  wost_batch batch = nullptr;
  hipStream_t stream = nullptr;
  std::map<int64_t, Request> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;
  int64_t next_id = 0;
  int64_t reserved = 0;
  unsigned int* d_maxse = nullptr;
  int maxse_cap = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  ~wost_server_s() {
    for (auto& kv : reqs) kv.second.free_device();
    if (batch) (void)wost_batch_destroy(batch);
    if (d_maxse) (void)hipFree(d_maxse);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

extern "C" {

wost_status wost_server_create(const wost_server_config* cfg, wost_server* out) {
  g_err.clear();
  if (!out) return fail(WOST_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (cfg && (cfg->solve.mode != 0 || cfg->solve.flags != 0))
    return fail(WOST_ERR_INVALID_ARG, "server: solve.mode and solve.flags must be 0");
  wost_server_s* s = new (std::nothrow) wost_server_s();
  if (!s) return fail(WOST_ERR_OUT_OF_MEMORY, "host allocation failed");
  if (cfg) s->cfg = *cfg;
  if (s->cfg.max_device_bytes <= 0) s->cfg.max_device_bytes = int64_t(4) << 30;
  if (s->cfg.round_walks <= 0) s->cfg.round_walks = 64;
  if (s->cfg.min_walks <= 0) s->cfg.min_walks = s->cfg.round_walks;
  if (s->cfg.max_walks <= 0) s->cfg.max_walks = 65536;
  if (s->cfg.max_active <= 0) s->cfg.max_active = 4096;
  if (s->cfg.max_round_walks <= 0) s->cfg.max_round_walks = 1024;
  if (s->cfg.max_round_walks < s->cfg.round_walks) s->cfg.max_round_walks = s->cfg.round_walks;
  s->cfg.adaptive = s->cfg.adaptive ? 1 : 0;
  wost_status st = wost_batch_create(&s->batch);
  if (st != WOST_OK) {
    delete s;
    return st;
  }
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipStreamCreate");
  }
  *out = s;
  return WOST_OK;
}

wost_status wost_server_destroy(wost_server s) {
  g_err.clear();
  if (!s) return WOST_OK;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  delete s;
  return WOST_OK;
}

wost_status wost_server_submit(wost_server s, wost_scene scene, const float* points, int64_t n,
                               float eps, uint64_t seed, double target_se, int64_t* request_id) {
  g_err.clear();
  if (!s || !scene || !points || !request_id) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  if (n < 1) return fail(WOST_ERR_INVALID_ARG, "n_points < 1");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(WOST_ERR_INVALID_ARG, "eps must be finite and > 0");
  if (!(target_se > 0)) return fail(WOST_ERR_INVALID_ARG, "target_se must be > 0");
  try {
    Request r;
    r.id = s->next_id++;
    r.scene = scene;
    const int dim = scene->host.dim;
    r.points.assign(points, points + n * dim);
    r.n = n;
    r.eps = eps;
    r.seed = seed;
    r.target = target_se;
    r.t_submit = s->now_ms();
    r.bytes = n * (int64_t)(dim * 4 + 4 * 8 +
                            4 * (s->cfg.adaptive ? s->cfg.max_round_walks : s->cfg.round_walks));
    r.next = std::min<int64_t>(s->cfg.round_walks, s->cfg.max_walks);
    *request_id = r.id;
    if (r.bytes > s->cfg.max_device_bytes) {
      r.state = WOST_REQ_REJECTED;
      r.t_done = r.t_submit;
    } else {
      s->queue.push_back(r.id);
    }
    s->reqs.emplace(r.id, std::move(r));
    return WOST_OK;
  } catch (const std::bad_alloc&) {
    return fail(WOST_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

wost_status wost_server_step(wost_server s, int32_t* n_open) {
  g_err.clear();
  if (!s) return fail(WOST_ERR_INVALID_ARG, "server is NULL");
  // admission (first come, first served, by device-memory budget)
  while (!s->queue.empty() && (int)s->active.size() < s->cfg.max_active) {
    Request& r = s->reqs[s->queue.front()];
    if (s->reserved + r.bytes > s->cfg.max_device_bytes) break;
    const int dim = r.scene->host.dim;
    hipError_t e = hipMalloc((void**)&r.d_points, r.n * dim * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&r.d_mean, r.n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&r.d_m2, r.n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&r.d_rmean, r.n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&r.d_rvar, r.n * sizeof(double));
    if (e == hipSuccess)
      e = hipMemcpy(r.d_points, r.points.data(), r.n * dim * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      r.free_device();
      if (s->active.empty()) return hip_fail(e, "server admission");
      break;   // retry once memory frees up
    }
    s->reserved += r.bytes;
    r.state = WOST_REQ_ACTIVE;
    r.t_admit = s->now_ms();
    s->active.push_back(r.id);
    s->queue.pop_front();
  }
  if (!s->active.empty()) {
    std::vector<wost_batch_item> items;
    for (int64_t id : s->active) {
      Request& r = s->reqs[id];
      wost_batch_item it{};
      it.scene = r.scene;
      it.d_points = r.d_points;
      it.n_points = r.n;
      it.walks_per_point = (int32_t)r.next;
      it.eps = r.eps;
      it.seed = r.seed;
      it.point_base = 0;
      it.walk_base = (uint32_t)r.walks;   // walk indices continue across rounds
      it.d_mean = r.d_rmean;
      it.d_var = r.d_rvar;
      items.push_back(it);
    }
    wost_solve_opts o = s->cfg.solve;
    wost_status st = wost_solve_batch(s->batch, items.data(), (int32_t)items.size(), &o, s->stream);
    if (st != WOST_OK) return st;
    const int na = (int)s->active.size();
    if (na > s->maxse_cap) {
      if (s->d_maxse) HIP_TRY(hipFree(s->d_maxse), "hipFree");
      s->d_maxse = nullptr;
      HIP_TRY(hipMalloc((void**)&s->d_maxse, na * sizeof(unsigned int)), "hipMalloc");
      s->maxse_cap = na;
    }
    HIP_TRY(wost::launch_fill_u32(s->d_maxse, na, s->stream), "fill");
    for (int k = 0; k < na; ++k) {
      Request& r = s->reqs[s->active[k]];
      HIP_TRY(wost::launch_merge(r.d_mean, r.d_m2, r.d_rmean, r.d_rvar, r.n, (double)r.walks,
                                 (double)r.next, s->d_maxse + k, s->stream), "merge");
    }
    std::vector<unsigned int> mse(na);
    HIP_TRY(hipMemcpyAsync(mse.data(), s->d_maxse, na * sizeof(unsigned int), hipMemcpyDeviceToHost, s->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    std::vector<int64_t> still;
    for (int k = 0; k < na; ++k) {
      Request& r = s->reqs[s->active[k]];
      r.rounds += 1;
      r.walks += r.next;
      float se;
      std::memcpy(&se, &mse[k], sizeof se);
      r.max_se = se;
      const bool conv = r.walks >= s->cfg.min_walks && r.max_se <= r.target;
      if (s->cfg.adaptive) {
        // walks for max SE <= target: (se / target)^2 * n, plus 15 %
        const double need = (r.max_se / r.target) * (r.max_se / r.target) * (double)r.walks * 1.15;
        int64_t more = need > 9e15 ? (int64_t)s->cfg.max_walks : (int64_t)std::ceil(need) - r.walks;
        more = std::max<int64_t>(more, s->cfg.min_walks - r.walks);
        more = ((more + 63) / 64) * 64;
        more = std::min<int64_t>(std::max<int64_t>(more, s->cfg.round_walks), s->cfg.max_round_walks);
        r.next = more;
      } else {
        r.next = s->cfg.round_walks;
      }
      r.next = std::min<int64_t>(r.next, s->cfg.max_walks - r.walks);
      if (conv || r.walks >= s->cfg.max_walks) {
        r.mean.resize(r.n);
        std::vector<double> m2(r.n);
        HIP_TRY(hipMemcpy(r.mean.data(), r.d_mean, r.n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
        HIP_TRY(hipMemcpy(m2.data(), r.d_m2, r.n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
        r.var.resize(r.n);
        for (int64_t i = 0; i < r.n; ++i) r.var[i] = r.walks > 1 ? m2[i] / (double)(r.walks - 1) : 0.0;
        r.free_device();
        s->reserved -= r.bytes;
        r.state = WOST_REQ_DONE;
        r.t_done = s->now_ms();
        r.points.clear();
        r.points.shrink_to_fit();
      } else {
        still.push_back(r.id);
      }
    }
    s->active.swap(still);
  }
  if (n_open) *n_open = (int32_t)(s->queue.size() + s->active.size());
  return WOST_OK;
}

wost_status wost_server_poll(wost_server s, int64_t id, wost_request_info* info, double* mean_out,
                             double* var_out) {
  g_err.clear();
  if (!s || !info) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(WOST_ERR_INVALID_ARG, "unknown request id");
  const Request& r = it->second;
  info->state = r.state;
  info->rounds = r.rounds;
  info->n_points = r.n;
  info->walks_per_point = r.walks;
  info->max_se = r.max_se;
  info->t_submit_ms = r.t_submit;
  info->t_admit_ms = r.t_admit;
  info->t_done_ms = r.t_done;
  if (r.state == WOST_REQ_DONE) {
    if (mean_out) std::memcpy(mean_out, r.mean.data(), r.n * sizeof(double));
    if (var_out) std::memcpy(var_out, r.var.data(), r.n * sizeof(double));
  }
  return WOST_OK;
}

}  // extern "C"
