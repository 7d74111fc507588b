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

static_assert(wost::kSil4Height == wost::kSil4Levels, "traversal stack bound and builder height bound");

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
  info->nodes_dirichlet = H.dim == 3 ? H.n_dir4 : H.treeD.stats.n_nodes;
  info->nodes_neumann = H.treeN.stats.n_nodes;
  // the 3D Dirichlet and silhouette trees are reported as searched: 4-wide
  // nodes and their height
  info->nodes_silhouette = H.dim == 3 ? H.n_sil4 : H.treeS.stats.n_nodes;
  info->depth_dirichlet = H.dim == 3 ? H.levels_dir4 : H.treeD.stats.max_depth;
  info->depth_neumann = H.treeN.stats.max_depth;
  info->depth_silhouette = H.dim == 3 ? H.levels_sil4 : H.treeS.stats.max_depth;
  info->half_diagonal = H.L;
  for (int k = 0; k < 3; ++k) info->center[k] = H.center[k];
  const int dim = H.dim;
  const int64_t node_b = dim == 3 ? 64 : 48, prim_b = dim == 3 ? 48 : 16;
  const int64_t cone_b = dim == 3 ? 64 : 32, elem_b = dim == 3 ? 48 : 32;
  // 3D: the Dirichlet, silhouette and ray records are 128 bytes (node_b +
  // cone_b); the Neumann tree is kept binary too (for the sample descent)
  info->device_bytes = (info->nodes_dirichlet + info->nodes_neumann + info->nodes_silhouette) * node_b +
                       (info->nodes_silhouette + (dim == 3 ? info->nodes_dirichlet : 0)) * cone_b +
                       H.n_ray4 * 128 +
                       (info->n_dirichlet + info->n_neumann) * prim_b +
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
  P.claim = (o && o->claim_walks > 0) ? o->claim_walks : (s->host.dim == 2 ? 128 : 1);
  P.steal = (o && o->steal_lanes > 0) ? (o->steal_lanes > 64 ? 64 : o->steal_lanes) : (s->host.dim == 2 ? 1 : 16);
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
    // Dirichlet tree: 3D 4-wide (one 128-byte record per node, exact child
    // boxes), 2D binary
    if (dim == 3) {
      const uint32_t* wp;
      if ((st = upload(s, H.dir4, &wp)) != WOST_OK) { delete s; return st; }
      D.dn = (const float4*)wp;
    } else {
      if ((st = upload(s, H.treeD.nodes, &fp)) != WOST_OK) { delete s; return st; }
      D.dn = (const float4*)fp;
    }
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
    // silhouette tree.  3D: four children per node, one 128-byte record per
    // node (a quantisation frame, the four child boxes as 8-bit lattice
    // coordinates, their codes, bounding radii and normal cones), so that a
    // visit reads one cache line and a search takes about half the dependent
    // node reads of a binary tree.  2D: binary, node and cone arrays
    // separate, whose smaller footprint measured faster on the L2-resident
    // star polygon.
    if (dim == 2) {
      if ((st = upload(s, H.treeS.nodes, &fp)) != WOST_OK) { delete s; return st; }
      D.sn = (const float4*)fp;
      if ((st = upload(s, H.treeS.cones, &fp)) != WOST_OK) { delete s; return st; }
      D.sc = (const float4*)fp;
    } else {
      const uint32_t* wp;
      if ((st = upload(s, H.sil4, &wp)) != WOST_OK) { delete s; return st; }
      D.sn = (const float4*)wp;
      D.sc = nullptr;
    }
    if ((st = upload(s, epay, &fp)) != WOST_OK) { delete s; return st; }
    D.se = (const float4*)fp;
    D.nE = (int)ne;
    D.topD = dim == 3 ? H.top_dir4 : H.topD;
    D.dn_root = dim == 3 ? H.root_dir4 : 0;
    D.topN = H.topN;
    D.topS = dim == 3 ? H.top_sil4 : H.topS;
    D.sil4_root = dim == 3 ? H.root_sil4 : 0;
    // the Neumann tree's 4-wide copy for the ray queries (3D)
    D.rn = nullptr;
    D.trn = nullptr;
    D.topR = D.ctR = 0;
    D.rn_root = 0;
    if (dim == 3 && !H.ray4.empty()) {
      const uint32_t* wp;
      if ((st = upload(s, H.ray4, &wp)) != WOST_OK) { delete s; return st; }
      D.rn = (const float4*)wp;
      D.topR = H.top_ray4;
      D.rn_root = H.root_ray4;
    }
    D.tdn = D.tnn = D.tsn = D.tsc = nullptr;
    D.ctD = D.ctN = D.ctS = 0;
    std::vector<wost::FnDev> fns(wost::kFnCount);
    fns[wost::kFnG] = fn_dev(desc->g);
    fns[wost::kFnH] = fn_dev(desc->h);
    fns[wost::kFnF] = fn_dev(desc->f);
    // double-sided flags per leaf slot (only a scene that has such
    // primitives runs the double-sided kernels, which read them)
    D.ds = 0;
    for (uint8_t b : H.bc) D.ds |= b >= 2;
    D.dside = nullptr;
    D.nside = nullptr;
    fns[wost::kFnGm] = fn_dev(desc->g_minus);
    fns[wost::kFnHm] = fn_dev(desc->h_minus);
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
    if ((st = pc_upload(desc->g, fns[wost::kFnG])) != WOST_OK) { delete s; return st; }
    if ((st = pc_upload(desc->h, fns[wost::kFnH])) != WOST_OK) { delete s; return st; }
    if ((st = pc_upload(desc->g_minus, fns[wost::kFnGm])) != WOST_OK) { delete s; return st; }
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
    if ((st = pc_upload(desc->h_minus, fns[wost::kFnHm])) != WOST_OK) { delete s; return st; }
    {
      const wost::FnDev* fnp;
      if ((st = upload(s, fns, &fnp)) != WOST_OK) { delete s; return st; }
      D.fn = fnp;
      for (int i = 0; i < wost::kFnCount; ++i) D.fn_kind[i] = fns[i].kind;
    }
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
  const bool d2 = s->host.dim == 2;
  // the knobs of the persistent cooperative kernel and their candidates; the
  // first candidate of each is the default.  Every candidate draws the same
  // random numbers, so tuning never changes results.
  const std::vector<std::vector<int>> cand = {
      {1, 8, 32},                                          // refill threshold
      {cap, std::max(1, cap / 2), std::max(1, 3 * cap / 4)},  // grid
      {0, 1},                                              // walk order (grouping of walks into waves)
      d2 ? std::vector<int>{128, 32, 512} : std::vector<int>{1},            // claim size (2D)
      d2 ? std::vector<int>{1} : std::vector<int>{16, 32, 8, 48},           // steal threshold (3D)
  };
  std::vector<int> best(cand.size());
  for (size_t k = 0; k < cand.size(); ++k) best[k] = cand[k][0];
  auto timed = [&](const std::vector<int>& v, float* ms) -> wost_status {
    wost_solve_opts o = *opts;
    o.mode = 0;
    o.flags = 0;
    o.refill = v[0];
    o.grid = v[1];
    o.walk_order = v[2];
    o.claim_walks = v[3];
    o.steal_lanes = v[4];
    wost_status r = wost_solve_ex(s, d_points, ns, W, eps, seed, 0, 0, &o, dm.p, dv.p, stream);
    if (r != WOST_OK) return r;
    HIP_TRY(hipStreamSynchronize(hs), "hipStreamSynchronize");
    wost_stats ws;
    if ((r = wost_get_stats(s, &ws)) != WOST_OK) return r;
    *ms = (float)ws.kernel_ms;
    return WOST_OK;
  };
  float best_ms;
  if ((st = timed(best, &best_ms)) != WOST_OK) return st;   // warms caches and code
  if ((st = timed(best, &best_ms)) != WOST_OK) return st;
  // coordinate search: each knob in turn over its candidates, the others
  // held at their best so far; two passes
  for (int pass = 0; pass < 2; ++pass)
    for (size_t k = 0; k < cand.size(); ++k)
      for (int c : cand[k]) {
        if (c == best[k]) continue;
        std::vector<int> v = best;
        v[k] = c;
        float ms;
        if ((st = timed(v, &ms)) != WOST_OK) return st;
        if (ms < best_ms) {
          best_ms = ms;
          best = v;
        }
      }
  opts->mode = 0;
  opts->refill = best[0];
  opts->grid = best[1];
  opts->walk_order = best[2];
  opts->claim_walks = best[3];
  opts->steal_lanes = best[4];
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
  // 3D: a Q.1, Q.2, Q.3 or visibility visit reads one 128-byte 4-wide
  // record (wide_node_bytes, a Q.2 record's cones included); a Q.4 visit
  // reads a 64-byte binary node
  out->node_bytes = dim == 3 ? 64 : 48;
  out->cone_bytes = dim == 3 ? 0 : 32;
  out->wide_node_bytes = dim == 3 ? 128 : 0;
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
  const uint64_t wide = dim == 3 ? out->q1_nodes + out->q2_nodes + out->q3_nodes + out->vis_nodes : 0;
  const uint64_t nodes = out->q1_nodes + out->q2_nodes + out->q3_nodes + out->q4_nodes + out->vis_nodes - wide;
  const uint64_t prims = out->q1_prims + out->q3_prims + out->vis_prims;
  out->bytes = wide * out->wide_node_bytes + nodes * out->node_bytes + out->q2_cones * out->cone_bytes +
               prims * out->prim_bytes +
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

wost_status wost_get_neumann_tree(wost_scene s, int64_t* n_nodes, float* nodes, int64_t* n_slots,
                                  int32_t* slot_prim, float* slot_measure) {
  g_err.clear();
  if (!s || !n_nodes || !n_slots) return fail(WOST_ERR_INVALID_ARG, "NULL argument");
  const wost::HostScene& H = s->host;
  const wost::FlatTree& T = H.treeN;
  const int words = H.dim == 3 ? 16 : 12;
  *n_nodes = (int64_t)(T.nodes.size() / words);
  *n_slots = (int64_t)T.order.size();
  if (nodes) std::memcpy(nodes, T.nodes.data(), T.nodes.size() * sizeof(float));
  for (size_t i = 0; i < T.order.size(); ++i) {
    const int32_t p = H.n_prims_list[T.order[i]];
    if (slot_prim) slot_prim[i] = p;
    if (slot_measure) slot_measure[i] = (float)H.measure[p];
  }
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

wost_status wost_measure_valu(int32_t kind, int32_t iters, double* glanes) {
  g_err.clear();
  if (!glanes) return fail(WOST_ERR_INVALID_ARG, "glanes is NULL");
  if (kind != 0 && kind != 1) return fail(WOST_ERR_INVALID_ARG, "kind must be 0 or 1");
  if (iters <= 0) iters = 1024;
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
  const int blocks = 8 * std::max(cus, 1);   // 8 waves per SIMD
  DevBuf<float> sink;
  HIP_TRY(sink.alloc((size_t)blocks), "hipMalloc");
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
  hipError_t e = wost::launch_valu_peak(kind, iters, blocks, sink.p, nullptr);   // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  if (e == hipSuccess) e = wost::launch_valu_peak(kind, iters, blocks, sink.p, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "VALU measurement");
  *glanes = (double)blocks * 256.0 * 8.0 * (kind == 1 ? 2.0 : 1.0) * iters / (ms * 1e-3) / 1e9;
  return WOST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
struct wost_batch_s {
  float* est = nullptr;
  size_t est_cap = 0;
  unsigned char* d_block = nullptr;     // device: head, groups, item table
  size_t block_cap = 0;
  unsigned char* h_block = nullptr;     // pinned host staging of the same bytes
  size_t h_block_cap = 0;
  unsigned long long* ctr = nullptr;   // stats[4], then one cursor per group
  int ctr_cap = 0;
  // graphs are captured on a stream made for the capture and destroyed after
  // it (a graph cannot be captured on the null stream, and a stream kept
  // idle would hold one of the process's few hardware queues)
  hipGraphExec_t exec = nullptr;
  std::vector<int> signature;          // group kinds, buffers and grid the cached graph was captured for
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t staged = nullptr;         // the last copy out of h_block has been made
  bool staging_busy = false;
  bool have_stats = false;
  int last_grid = 0;
  int64_t captures = 0;                // graphs captured so far (diagnostic)
  ~wost_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (est) (void)hipFree(est);
    if (d_block) (void)hipFree(d_block);
    if (h_block) (void)hipHostFree(h_block);
    if (ctr) (void)hipFree(ctr);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (staged) (void)hipEventDestroy(staged);
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

constexpr size_t align64(size_t x) { return (x + 63) & ~size_t(63); }

}  // namespace

extern "C" {

wost_status wost_batch_create(wost_batch* out) {
  g_err.clear();
  if (!out) return fail(WOST_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  wost_batch_s* b = new (std::nothrow) wost_batch_s();
  if (!b) return fail(WOST_ERR_OUT_OF_MEMORY, "host allocation failed");
  hipError_t e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
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
    const bool hh = wost::has_neumann_data(S), hf = S.fn_kind[wost::kFnF] != 0, ds = S.ds != 0;
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
  // device buffers, grown on demand; a buffer being replaced may still be
  // read by this context's last launch, so that launch is waited for (and
  // only that one: other work on the device keeps running)
  auto retire_old = [&](void* old) -> wost_status {
    if (!old) return WOST_OK;
    if (b->have_stats) HIP_TRY(hipEventSynchronize(b->ev1), "hipEventSynchronize");
    HIP_TRY(hipFree(old), "hipFree");
    return WOST_OK;
  };
  wost_status gst;
  if ((size_t)std::max<int64_t>(1, est_total) > b->est_cap) {
    if ((gst = retire_old(b->est)) != WOST_OK) return gst;
    b->est = nullptr;
    b->est_cap = 0;
    HIP_TRY(hipMalloc((void**)&b->est, (size_t)std::max<int64_t>(1, est_total) * sizeof(float)),
            "hipMalloc batch estimates");
    b->est_cap = (size_t)std::max<int64_t>(1, est_total);
  }
  size_t n_table = 0;
  for (const Group& g : groups) n_table += g.idx.size();
  const size_t off_groups = align64(sizeof(wost::BatchHeadDev));
  const size_t off_items = off_groups + align64(std::max<size_t>(1, groups.size()) * sizeof(wost::BatchGroupDev));
  const size_t bytes = off_items + std::max<size_t>(1, n_table) * sizeof(wost::BatchItem);
  if (bytes > b->block_cap) {
    const size_t cap = std::max<size_t>(bytes, 2 * b->block_cap);
    if ((gst = retire_old(b->d_block)) != WOST_OK) return gst;
    b->d_block = nullptr;
    b->block_cap = 0;
    HIP_TRY(hipMalloc((void**)&b->d_block, cap), "hipMalloc batch table");
    b->block_cap = cap;
  }
  const int ctr_words = 4 + (int)groups.size();
  if (ctr_words > b->ctr_cap) {
    if ((gst = retire_old(b->ctr)) != WOST_OK) return gst;
    b->ctr = nullptr;
    HIP_TRY(hipMalloc((void**)&b->ctr, ctr_words * sizeof(unsigned long long)), "hipMalloc batch counters");
    b->ctr_cap = ctr_words;
  }
  // the staging buffer is rewritten only once its previous copy has been made
  if (b->staging_busy) {
    HIP_TRY(hipEventSynchronize(b->staged), "hipEventSynchronize");
    b->staging_busy = false;
  }
  if (bytes > b->h_block_cap) {
    if (b->h_block) HIP_TRY(hipHostFree(b->h_block), "hipHostFree");
    b->h_block = nullptr;
    b->h_block_cap = 0;
    HIP_TRY(hipHostMalloc((void**)&b->h_block, b->block_cap, hipHostMallocDefault), "hipHostMalloc staging");
    b->h_block_cap = b->block_cap;
  }
  // host image of the head, the groups and the table, in group order
  std::memset(b->h_block, 0, bytes);
  auto* head = reinterpret_cast<wost::BatchHeadDev*>(b->h_block);
  auto* gdev = reinterpret_cast<wost::BatchGroupDev*>(b->h_block + off_groups);
  auto* table = reinterpret_cast<wost::BatchItem*>(b->h_block + off_items);
  size_t k = 0;
  int64_t points = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    g.first = k;
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
      B.P.est = b->est + est_off[i];
      B.n_walks = it.n_points * (int64_t)it.walks_per_point;
      B.chunk_begin = chunks;
      B.point_begin = points;
      B.mean = it.d_mean;
      B.var = it.d_var;
      chunks += (B.n_walks + chunk - 1) / chunk;
      points += it.n_points;
      table[k++] = B;
    }
    g.n_chunks = chunks;
    gdev[gi].first = (int)g.first;
    gdev[gi].n_items = (int)g.idx.size();
    gdev[gi].chunk = chunk;
    gdev[gi].n_chunks = chunks;
  }
  head->n_items_all = (int)n_table;
  head->points = points;
  hipStream_t hs = (hipStream_t)stream;
  // the table reaches the device in stream order, after the work already
  // enqueued there (which may still read the previous table)
  HIP_TRY(hipMemcpyAsync(b->d_block, b->h_block, bytes, hipMemcpyHostToDevice, hs), "hipMemcpyAsync batch table");
  HIP_TRY(hipEventRecord(b->staged, hs), "hipEventRecord");
  b->staging_busy = true;
  const int grid = (opts && opts->grid > 0) ? opts->grid : 0;
  // the graph depends only on the kinds of groups, the buffers and the grid;
  // sizes, RNG offsets and outputs are read from the table at run time
  std::vector<int> sig;
  for (const Group& g : groups) sig.insert(sig.end(), {g.dim, g.hh, g.hf, g.ds});
  const uintptr_t bufs[3] = {(uintptr_t)b->d_block, (uintptr_t)b->est, (uintptr_t)b->ctr};
  for (uintptr_t u : bufs) {
    sig.push_back((int)(u & 0xffffffffu));
    sig.push_back((int)(u >> 32));
  }
  sig.push_back(grid);
  sig.push_back((int)(off_items));
  if (sig != b->signature || !b->exec) {
    if (b->exec) {
      HIP_TRY(hipGraphExecDestroy(b->exec), "hipGraphExecDestroy");
      b->exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
    struct StreamGone {
      hipStream_t s;
      ~StreamGone() { (void)hipStreamDestroy(s); }
    } cap_gone{cap};
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = wost::launch_fill_u64(b->ctr, ctr_words, cap);
    int used_grid = 0;
    const auto* d_items = reinterpret_cast<const wost::BatchItem*>(b->d_block + off_items);
    const auto* d_groups = reinterpret_cast<const wost::BatchGroupDev*>(b->d_block + off_groups);
    for (size_t gi = 0; gi < groups.size() && e == hipSuccess; ++gi) {
      const Group& g = groups[gi];
      const int gr = grid > 0 ? grid : wost::max_resident_blocks(g.dim, true);
      used_grid = std::max(used_grid, gr);
      e = wost::launch_batch(d_items, d_groups + gi, g.dim, g.hh, g.hf, g.ds, b->ctr + 4 + gi, b->ctr, gr, cap);
    }
    if (e == hipSuccess && !groups.empty())
      e = wost::launch_reduce_batch(d_items, reinterpret_cast<const wost::BatchHeadDev*>(b->d_block), cap);
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
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
    b->captures += 1;
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
  out->graph_captures = (int32_t)b->captures;
  return WOST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving form
// ---------------------------------------------------------------------------
#include <chrono>
#include <deque>
#include <map>
#include <thread>

namespace {

// First-fit device arena for the request buffers: one allocation, made at
// the first admission, carved into 256-byte-aligned pieces; a freed piece
// merges with free neighbours.  Admission and retirement then make no
// device allocation.
struct DevArena {
  unsigned char* base = nullptr;
  int64_t cap = 0;
  std::map<int64_t, int64_t> free_;   // offset -> size
  static int64_t round_up(int64_t b) { return (b + 255) & ~int64_t(255); }
  hipError_t init(int64_t bytes) {
    cap = round_up(bytes);
    hipError_t e = hipMalloc((void**)&base, (size_t)cap);
    if (e == hipSuccess) free_[0] = cap;
    return e;
  }
  unsigned char* take(int64_t bytes) {
    bytes = round_up(std::max<int64_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const int64_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest > 0) free_[off + bytes] = rest;
      return base + off;
    }
    return nullptr;
  }
  void give(unsigned char* p, int64_t bytes) {
    bytes = round_up(std::max<int64_t>(bytes, 1));
    int64_t off = p - base;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        off = pv->first;
        bytes += pv->second;
        free_.erase(pv);
      }
    }
    free_[off] = bytes;
  }
  ~DevArena() {
    if (base) (void)hipFree(base);
  }
};

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
  int64_t bytes = 0;  // admission budget share
  bool in_flight = false;
  bool uploaded = false;   // the points are on the device
  // device buffers while active: one arena piece holding points, running
  // (mean, M2) and the round's (mean, variance)
  unsigned char* piece = nullptr;
  int64_t piece_bytes = 0;
  float* d_points = nullptr;
  double *d_mean = nullptr, *d_m2 = nullptr, *d_rmean = nullptr, *d_rvar = nullptr;
  // results when done
  std::vector<double> mean, var;
};

// One refinement round in flight: its own batch context (estimate buffer,
// table, graph) and stream, so that a new round can start while earlier
// ones drain; its requests' merges and largest standard errors follow the
// round's graph on the same stream.
struct RoundSlot {
  wost_batch batch = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<int64_t> ids;
  std::vector<int64_t> walks;
  wost::MergeItem* d_merge = nullptr;
  wost::MergeItem* h_merge = nullptr;   // pinned
  unsigned int* d_maxse = nullptr;
  unsigned int* h_maxse = nullptr;      // pinned
  int cap = 0;
  bool busy = false;
  ~RoundSlot() {
    if (batch) (void)wost_batch_destroy(batch);
    if (d_merge) (void)hipFree(d_merge);
    if (h_merge) (void)hipHostFree(h_merge);
    if (d_maxse) (void)hipFree(d_maxse);
    if (h_maxse) (void)hipHostFree(h_maxse);
    if (done) (void)hipEventDestroy(done);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

}  // namespace

struct wost_server_s {
  wost_server_config cfg{};
  std::vector<RoundSlot> slots;
  std::vector<int> in_flight;          // slots with a round running, in launch order
  DevArena arena;
  std::map<int64_t, Request> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;
  int64_t next_id = 0;
  int64_t reserved = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  ~wost_server_s() {
    for (RoundSlot& r : slots)
      if (r.stream) (void)hipStreamSynchronize(r.stream);
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
  if (s->cfg.max_rounds <= 0) s->cfg.max_rounds = 2;
  if (s->cfg.max_rounds > 4) s->cfg.max_rounds = 4;
  if (s->cfg.wait_us <= 0) s->cfg.wait_us = 2000;
  if (s->cfg.round_budget_walks <= 0) s->cfg.round_budget_walks = int64_t(1) << 24;
  s->cfg.adaptive = s->cfg.adaptive ? 1 : 0;
  s->slots.resize(s->cfg.max_rounds);
  for (RoundSlot& r : s->slots) {
    wost_status st = wost_batch_create(&r.batch);
    hipError_t e = st == WOST_OK ? hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) : hipSuccess;
    if (e == hipSuccess && st == WOST_OK) e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming);
    if (st != WOST_OK || e != hipSuccess) {
      delete s;
      return st != WOST_OK ? st : hip_fail(e, "server create");
    }
  }
  *out = s;
  return WOST_OK;
}

wost_status wost_server_destroy(wost_server s) {
  g_err.clear();
  if (!s) return WOST_OK;
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

}  // extern "C"

namespace {

// the walks a request takes in its next round, from its merged results
void plan_next(const wost_server_config& cfg, Request& r) {
  if (cfg.adaptive) {
    // walks for max SE <= target: (se / target)^2 * n, plus 15 %
    const double need = (r.max_se / r.target) * (r.max_se / r.target) * (double)r.walks * 1.15;
    int64_t more = need > 9e15 ? (int64_t)cfg.max_walks : (int64_t)std::ceil(need) - r.walks;
    more = std::max<int64_t>(more, cfg.min_walks - r.walks);
    more = ((more + 63) / 64) * 64;
    more = std::min<int64_t>(std::max<int64_t>(more, cfg.round_walks), cfg.max_round_walks);
    // a large request's round stays within the round budget (one round's
    // walks over all its requests), so that it cannot hold a round slot for
    // long; the cap depends on the request's own size only
    const int64_t fit = (cfg.round_budget_walks / std::max<int64_t>(r.n, 1)) / 64 * 64;
    more = std::min<int64_t>(more, std::max<int64_t>(fit, cfg.round_walks));
    r.next = more;
  } else {
    r.next = cfg.round_walks;
  }
  r.next = std::min<int64_t>(r.next, cfg.max_walks - r.walks);
}

// merges a finished round into its requests and retires the converged ones
wost_status retire_round(wost_server_s* s, RoundSlot& R) {
  for (size_t k = 0; k < R.ids.size(); ++k) {
    Request& r = s->reqs[R.ids[k]];
    r.in_flight = false;
    r.rounds += 1;
    r.walks += R.walks[k];
    float se;
    std::memcpy(&se, &R.h_maxse[k], sizeof se);
    r.max_se = se;
    const bool conv = r.walks >= s->cfg.min_walks && r.max_se <= r.target;
    plan_next(s->cfg, r);
    if (conv || r.walks >= s->cfg.max_walks) {
      r.mean.resize(r.n);
      std::vector<double> m2(r.n);
      HIP_TRY(hipMemcpyAsync(r.mean.data(), r.d_mean, r.n * sizeof(double), hipMemcpyDeviceToHost, R.stream),
              "hipMemcpyAsync");
      HIP_TRY(hipMemcpyAsync(m2.data(), r.d_m2, r.n * sizeof(double), hipMemcpyDeviceToHost, R.stream),
              "hipMemcpyAsync");
      HIP_TRY(hipStreamSynchronize(R.stream), "hipStreamSynchronize");
      r.var.resize(r.n);
      for (int64_t i = 0; i < r.n; ++i) r.var[i] = r.walks > 1 ? m2[i] / (double)(r.walks - 1) : 0.0;
      s->arena.give(r.piece, r.piece_bytes);
      r.piece = nullptr;
      r.d_points = nullptr;
      r.d_mean = r.d_m2 = r.d_rmean = r.d_rvar = nullptr;
      s->reserved -= r.bytes;
      r.state = WOST_REQ_DONE;
      r.t_done = s->now_ms();
      r.points.clear();
      r.points.shrink_to_fit();
      s->active.erase(std::find(s->active.begin(), s->active.end(), r.id));
    }
  }
  R.ids.clear();
  R.walks.clear();
  R.busy = false;
  return WOST_OK;
}

// retires every round that has finished, in any order (a request is in at
// most one round, so rounds are independent); when none has, waits up to
// wait_us for one to finish
wost_status poll_rounds(wost_server_s* s, int64_t wait_us, bool* retired) {
  *retired = false;
  if (s->in_flight.empty()) return WOST_OK;
  const auto t_end = std::chrono::steady_clock::now() + std::chrono::microseconds(wait_us);
  while (true) {
    for (size_t i = 0; i < s->in_flight.size();) {
      RoundSlot& R = s->slots[s->in_flight[i]];
      const hipError_t q = hipEventQuery(R.done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) return hip_fail(q, "round event");
      s->in_flight.erase(s->in_flight.begin() + i);
      wost_status st = retire_round(s, R);
      if (st != WOST_OK) return st;
      *retired = true;
    }
    if (*retired || s->in_flight.empty() || std::chrono::steady_clock::now() >= t_end) return WOST_OK;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

// launches one round for every admitted request without a round in flight
wost_status launch_round(wost_server_s* s, RoundSlot& R, const std::vector<int64_t>& ids) {
  std::vector<wost_batch_item> items;
  for (int64_t id : ids) {
    Request& r = s->reqs[id];
    if (!r.uploaded) {   // a new request: its points go first, on this round's stream
      HIP_TRY(hipMemcpyAsync(r.d_points, r.points.data(), r.n * r.scene->host.dim * sizeof(float),
                             hipMemcpyHostToDevice, R.stream), "hipMemcpyAsync points");
      r.uploaded = true;
    }
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
  // the merge tables grow before this round's work is enqueued (the slot's
  // earlier round, finished, is the only user of the old ones)
  const int na = (int)ids.size();
  if (na > R.cap) {
    if (R.d_merge) HIP_TRY(hipStreamSynchronize(R.stream), "hipStreamSynchronize");
    if (R.d_merge) HIP_TRY(hipFree(R.d_merge), "hipFree");
    if (R.h_merge) HIP_TRY(hipHostFree(R.h_merge), "hipHostFree");
    if (R.d_maxse) HIP_TRY(hipFree(R.d_maxse), "hipFree");
    if (R.h_maxse) HIP_TRY(hipHostFree(R.h_maxse), "hipHostFree");
    R.d_merge = nullptr;
    R.h_merge = nullptr;
    R.d_maxse = R.h_maxse = nullptr;
    R.cap = 0;
    const int cap = std::max(na, 64);
    HIP_TRY(hipMalloc((void**)&R.d_merge, cap * sizeof(wost::MergeItem)), "hipMalloc");
    HIP_TRY(hipHostMalloc((void**)&R.h_merge, cap * sizeof(wost::MergeItem), hipHostMallocDefault), "hipHostMalloc");
    HIP_TRY(hipMalloc((void**)&R.d_maxse, cap * sizeof(unsigned int)), "hipMalloc");
    HIP_TRY(hipHostMalloc((void**)&R.h_maxse, cap * sizeof(unsigned int), hipHostMallocDefault), "hipHostMalloc");
    R.cap = cap;
  }
  wost_solve_opts o = s->cfg.solve;
  wost_status st = wost_solve_batch(R.batch, items.data(), (int32_t)items.size(), &o, R.stream);
  if (st != WOST_OK) return st;
  int64_t points = 0;
  for (int k = 0; k < na; ++k) {
    Request& r = s->reqs[ids[k]];
    wost::MergeItem m{};
    m.mean = r.d_mean;
    m.m2 = r.d_m2;
    m.mb = r.d_rmean;
    m.vb = r.d_rvar;
    m.n = r.n;
    m.point_begin = points;
    m.na = (double)r.walks;
    m.nb = (double)r.next;
    m.max_se = R.d_maxse + k;
    points += r.n;
    R.h_merge[k] = m;
  }
  HIP_TRY(hipMemcpyAsync(R.d_merge, R.h_merge, na * sizeof(wost::MergeItem), hipMemcpyHostToDevice, R.stream),
          "hipMemcpyAsync merge table");
  HIP_TRY(wost::launch_fill_u32(R.d_maxse, na, R.stream), "fill");
  HIP_TRY(wost::launch_merge_batch(R.d_merge, na, points, R.stream), "merge");
  HIP_TRY(hipMemcpyAsync(R.h_maxse, R.d_maxse, na * sizeof(unsigned int), hipMemcpyDeviceToHost, R.stream),
          "hipMemcpyAsync");
  HIP_TRY(hipEventRecord(R.done, R.stream), "hipEventRecord");
  R.ids = ids;
  R.walks.clear();
  for (int64_t id : ids) {
    Request& r = s->reqs[id];
    R.walks.push_back(r.next);
    r.in_flight = true;
  }
  R.busy = true;
  return WOST_OK;
}

}  // namespace

extern "C" {

wost_status wost_server_step(wost_server s, int32_t* n_open) {
  g_err.clear();
  if (!s) return fail(WOST_ERR_INVALID_ARG, "server is NULL");
  wost_status st;
  // 1. rounds that have finished: merge, retire the converged requests
  bool retired = false;
  if ((st = poll_rounds(s, 0, &retired)) != WOST_OK) return st;
  // 2. admission (first come, first served, by the device-memory budget)
  while (!s->queue.empty() && (int)s->active.size() < s->cfg.max_active) {
    Request& r = s->reqs[s->queue.front()];
    if (s->reserved + r.bytes > s->cfg.max_device_bytes) break;
    if (!s->arena.base) HIP_TRY(s->arena.init(s->cfg.max_device_bytes), "hipMalloc request arena");
    const int dim = r.scene->host.dim;
    const int64_t pts_b = DevArena::round_up(r.n * dim * (int64_t)sizeof(float));
    const int64_t vec_b = DevArena::round_up(r.n * (int64_t)sizeof(double));
    r.piece_bytes = pts_b + 4 * vec_b;
    r.piece = s->arena.take(r.piece_bytes);
    if (!r.piece) break;   // fragmented: wait for retirements
    r.d_points = reinterpret_cast<float*>(r.piece);
    r.d_mean = reinterpret_cast<double*>(r.piece + pts_b);
    r.d_m2 = reinterpret_cast<double*>(r.piece + pts_b + vec_b);
    r.d_rmean = reinterpret_cast<double*>(r.piece + pts_b + 2 * vec_b);
    r.d_rvar = reinterpret_cast<double*>(r.piece + pts_b + 3 * vec_b);
    r.uploaded = false;   // copied by its first round, on that round's stream
    s->reserved += r.bytes;
    r.state = WOST_REQ_ACTIVE;
    r.t_admit = s->now_ms();
    s->active.push_back(r.id);
    s->queue.pop_front();
  }
  // 3. a round on a free slot for the admitted requests without one in
  // flight, in admission order, up to the round's walk budget (at least one
  // request); the others wait for the next round.  The budget only delays
  // requests: each request's round sizes depend on its own results alone.
  bool launched = false;
  int free_slot = -1;
  for (int i = 0; i < (int)s->slots.size(); ++i)
    if (!s->slots[i].busy) { free_slot = i; break; }
  if (free_slot >= 0) {
    std::vector<int64_t> ready;
    int64_t walks = 0;
    for (int64_t id : s->active) {
      const Request& r = s->reqs[id];
      if (r.in_flight) continue;
      const int64_t w = r.n * r.next;
      if (!ready.empty() && walks + w > s->cfg.round_budget_walks) continue;
      ready.push_back(id);
      walks += w;
    }
    if (!ready.empty()) {
      if ((st = launch_round(s, s->slots[free_slot], ready)) != WOST_OK) return st;
      s->in_flight.push_back(free_slot);
      launched = true;
    }
  }
  // 4. nothing started: wait a little (at most wait_us) for a round to end
  if (!launched && !s->in_flight.empty()) {
    if ((st = poll_rounds(s, s->cfg.wait_us, &retired)) != WOST_OK) return st;
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
  info->in_flight = r.in_flight ? 1 : 0;
  if (r.state == WOST_REQ_DONE) {
    if (mean_out) std::memcpy(mean_out, r.mean.data(), r.n * sizeof(double));
    if (var_out) std::memcpy(var_out, r.var.data(), r.n * sizeof(double));
  }
  return WOST_OK;
}

}  // extern "C"
