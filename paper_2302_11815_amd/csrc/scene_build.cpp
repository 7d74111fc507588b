// Host-side scene preprocessing and tree construction (see scene_build.hpp).
#include "scene_build.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace wost {

namespace {

struct BNode {
  float lo[3], hi[3];
  int32_t left = -1, right = -1;
  int32_t start = 0, count = 0;
  bool leaf = false;
};

float box_area(int dim, const float lo[3], const float hi[3]) {
  float d[3];
  for (int k = 0; k < 3; ++k) d[k] = std::max(0.0f, hi[k] - lo[k]);
  if (dim == 2) return d[0] + d[1];                       // half perimeter
  return d[0] * d[1] + d[1] * d[2] + d[2] * d[0];          // half surface area
}

void box_empty(float lo[3], float hi[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = std::numeric_limits<float>::max();
    hi[k] = -std::numeric_limits<float>::max();
  }
}

// radius of a box's bounding sphere about its centre, with the squared
// radius padded by 1e-4 and rounded up to FP32, so that a test which
// compares it with FP32 distances stays conservative; 0 for an empty box
float box_radius(int dim, const float lo[3], const float hi[3]) {
  double r2 = 0.0;
  for (int k = 0; k < dim; ++k) {
    if (!(lo[k] <= hi[k])) return 0.0f;
    const double e = 0.5 * ((double)hi[k] - (double)lo[k]);
    r2 += e * e;
  }
  const double r = std::sqrt(r2 * 1.0001);
  float f = (float)r;
  if ((double)f < r) f = std::nextafter(f, std::numeric_limits<float>::infinity());
  return f;
}

void box_grow(float lo[3], float hi[3], const float l2[3], const float h2[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = std::min(lo[k], l2[k]);
    hi[k] = std::max(hi[k], h2[k]);
  }
}

int ceil_log2(int64_t x) {
  int r = 0;
  while ((int64_t(1) << r) < x) ++r;
  return r;
}

// bounding cone of two cones (angle < 0: empty); conservative: the union
// cone's axis lies on the great circle through both axes
ItemCone cone_union(const ItemCone& a, const ItemCone& b) {
  if (a.angle < 0) return b;
  if (b.angle < 0) return a;
  if (a.angle >= M_PI || b.angle >= M_PI) return ItemCone{{a.axis[0], a.axis[1], a.axis[2]}, M_PI};
  const double c = std::max(-1.0, std::min(1.0, a.axis[0] * b.axis[0] + a.axis[1] * b.axis[1] +
                                                    a.axis[2] * b.axis[2]));
  const double phi = std::acos(c);
  if (a.angle >= phi + b.angle) return a;
  if (b.angle >= phi + a.angle) return b;
  const double th = 0.5 * (a.angle + phi + b.angle);
  if (th >= M_PI) return ItemCone{{a.axis[0], a.axis[1], a.axis[2]}, M_PI};
  const double sp = std::sin(phi);
  if (sp < 1e-12) return ItemCone{{a.axis[0], a.axis[1], a.axis[2]}, std::max(a.angle, b.angle)};
  const double d = th - a.angle;   // rotate a's axis toward b's by d
  const double wa = std::sin(phi - d) / sp, wb = std::sin(d) / sp;
  ItemCone r;
  double nn = 0;
  for (int k = 0; k < 3; ++k) {
    r.axis[k] = wa * a.axis[k] + wb * b.axis[k];
    nn += r.axis[k] * r.axis[k];
  }
  nn = std::sqrt(nn);
  for (int k = 0; k < 3; ++k) r.axis[k] /= nn;
  r.angle = th;
  return r;
}

double orientation_measure(const ItemCone& c) {
  if (c.angle < 0) return 0.0;
  return std::sin(std::min(c.angle, 0.5 * M_PI)) + kSaohViewTerm;
}

}  // namespace

FlatTree build_tree(int dim, const std::vector<ItemBox>& boxes, int leaf_size,
                    const std::vector<ItemCone>* cones) {
  FlatTree T;
  T.dim = dim;
  const int64_t n = (int64_t)boxes.size();
  if (leaf_size < 1) leaf_size = 1;
  if (leaf_size > kMaxLeaf) leaf_size = kMaxLeaf;
  T.stats.n_items = n;
  if (n == 0) return T;
  std::vector<float> cen(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) cen[3 * i + k] = 0.5f * (boxes[i].lo[k] + boxes[i].hi[k]);
  std::vector<int32_t> idx(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;

  std::vector<BNode> nodes;
  nodes.reserve(2 * n / std::max(1, leaf_size) + 2);
  struct Job { int32_t node; int32_t start, end; int depth; };
  std::vector<Job> stack;
  nodes.emplace_back();
  stack.push_back({0, 0, (int32_t)n, 0});
  constexpr int kBins = 16;
  int max_depth = 0;

  while (!stack.empty()) {
    Job J = stack.back();
    stack.pop_back();
    BNode& N = nodes[J.node];
    N.start = J.start;
    N.count = J.end - J.start;
    box_empty(N.lo, N.hi);
    float clo[3], chi[3];
    box_empty(clo, chi);
    for (int32_t i = J.start; i < J.end; ++i) {
      const ItemBox& b = boxes[idx[i]];
      box_grow(N.lo, N.hi, b.lo, b.hi);
      const float* c = &cen[3 * idx[i]];
      box_grow(clo, chi, c, c);
    }
    const int32_t cnt = N.count;
    max_depth = std::max(max_depth, J.depth);
    if (cnt <= leaf_size) {
      N.leaf = true;
      continue;
    }
    int axis = 0;
    float ext = -1;
    for (int k = 0; k < dim; ++k)
      if (chi[k] - clo[k] > ext) { ext = chi[k] - clo[k]; axis = k; }
    // keep the tree within the traversal stack: a median split halves the
    // items, so a subtree of cnt items needs ceil_log2(cnt / leaf_size) more
    // levels; fall back to median splits when the SAH would risk the bound
    const int need = ceil_log2((cnt + leaf_size - 1) / leaf_size);
    const bool force_median = J.depth + 1 + need + 2 >= max_tree_depth(dim);
    int32_t mid = -1;
    if (ext > 0 && !force_median) {
      int bcount[kBins] = {0};
      float blo[kBins][3], bhi[kBins][3];
      ItemCone bcone[kBins];
      for (int b = 0; b < kBins; ++b) {
        box_empty(blo[b], bhi[b]);
        bcone[b].angle = -1.0;
      }
      const float scale = kBins / ext;
      for (int32_t i = J.start; i < J.end; ++i) {
        int b = (int)((cen[3 * idx[i] + axis] - clo[axis]) * scale);
        b = std::min(std::max(b, 0), kBins - 1);
        bcount[b]++;
        box_grow(blo[b], bhi[b], boxes[idx[i]].lo, boxes[idx[i]].hi);
        if (cones) bcone[b] = cone_union(bcone[b], (*cones)[idx[i]]);
      }
      // each side's cost weight: area, times the orientation measure of its
      // normal cone when cones are given
      float lA[kBins], rA[kBins];
      int lN[kBins], rN[kBins];
      float lo[3], hi[3];
      box_empty(lo, hi);
      ItemCone cc;
      cc.angle = -1.0;
      int c = 0;
      for (int b = 0; b < kBins; ++b) {
        box_grow(lo, hi, blo[b], bhi[b]);
        c += bcount[b];
        lA[b] = box_area(dim, lo, hi);
        if (cones) {
          cc = cone_union(cc, bcone[b]);
          lA[b] *= (float)orientation_measure(cc);
        }
        lN[b] = c;
      }
      box_empty(lo, hi);
      cc.angle = -1.0;
      c = 0;
      for (int b = kBins - 1; b >= 0; --b) {
        box_grow(lo, hi, blo[b], bhi[b]);
        c += bcount[b];
        rA[b] = box_area(dim, lo, hi);
        if (cones) {
          cc = cone_union(cc, bcone[b]);
          rA[b] *= (float)orientation_measure(cc);
        }
        rN[b] = c;
      }
      float best = std::numeric_limits<float>::max();
      int best_b = -1;
      for (int b = 0; b < kBins - 1; ++b) {
        if (lN[b] == 0 || rN[b + 1] == 0) continue;
        float cost = lA[b] * lN[b] + rA[b + 1] * rN[b + 1];
        if (cost < best) { best = cost; best_b = b; }
      }
      if (best_b >= 0) {
        auto it = std::partition(idx.begin() + J.start, idx.begin() + J.end, [&](int32_t i) {
          int b = (int)((cen[3 * i + axis] - clo[axis]) * scale);
          b = std::min(std::max(b, 0), kBins - 1);
          return b <= best_b;
        });
        mid = (int32_t)(it - idx.begin());
        if (mid == J.start || mid == J.end) mid = -1;
      }
    }
    if (mid < 0) {
      mid = J.start + cnt / 2;
      std::nth_element(idx.begin() + J.start, idx.begin() + mid, idx.begin() + J.end,
                       [&](int32_t a, int32_t b) { return cen[3 * a + axis] < cen[3 * b + axis]; });
    }
    int32_t l = (int32_t)nodes.size();
    nodes.emplace_back();
    int32_t r = (int32_t)nodes.size();
    nodes.emplace_back();
    nodes[J.node].left = l;
    nodes[J.node].right = r;
    stack.push_back({r, mid, J.end, J.depth + 1});
    stack.push_back({l, J.start, mid, J.depth + 1});
  }

  // flatten: preorder over internal nodes; each emitted node carries both
  // children's boxes and codes
  const int nf = dim == 3 ? 16 : 12;
  std::vector<int32_t> dev_index(nodes.size(), -1);
  std::vector<int32_t> order_int;
  {
    std::vector<int32_t> st{0};
    while (!st.empty()) {
      int32_t b = st.back();
      st.pop_back();
      if (nodes[b].leaf && b != 0) continue;
      dev_index[b] = (int32_t)order_int.size();
      order_int.push_back(b);
      if (!nodes[b].leaf) {
        st.push_back(nodes[b].right);
        st.push_back(nodes[b].left);
      }
    }
  }
  T.nodes.assign(order_int.size() * nf, 0.0f);
  auto code_of = [&](int32_t b) -> int32_t {
    if (nodes[b].leaf) return leaf_code(nodes[b].start, nodes[b].count);
    return dev_index[b];
  };
  double sah = 0;
  const double root_area = std::max(1e-30f, box_area(dim, nodes[0].lo, nodes[0].hi));
  for (size_t d = 0; d < order_int.size(); ++d) {
    const BNode& B = nodes[order_int[d]];
    float* w = &T.nodes[d * nf];
    float llo[3], lhi[3], rlo[3], rhi[3];
    int32_t cl, cr;
    if (B.leaf) {  // the root is a single leaf
      std::memcpy(llo, B.lo, sizeof llo);
      std::memcpy(lhi, B.hi, sizeof lhi);
      box_empty(rlo, rhi);
      cl = leaf_code(B.start, B.count);
      cr = kEmpty;
    } else {
      const BNode& L = nodes[B.left];
      const BNode& R = nodes[B.right];
      std::memcpy(llo, L.lo, sizeof llo);
      std::memcpy(lhi, L.hi, sizeof lhi);
      std::memcpy(rlo, R.lo, sizeof rlo);
      std::memcpy(rhi, R.hi, sizeof rhi);
      cl = code_of(B.left);
      cr = code_of(B.right);
    }
    // the last two words: the children's bounding-sphere radii (read by the
    // silhouette-tree test, which would otherwise derive them per visit)
    if (dim == 3) {
      const float v[12] = {llo[0], llo[1], llo[2], lhi[0], lhi[1], lhi[2],
                           rlo[0], rlo[1], rlo[2], rhi[0], rhi[1], rhi[2]};
      std::memcpy(w, v, sizeof v);
      std::memcpy(w + 12, &cl, 4);
      std::memcpy(w + 13, &cr, 4);
      w[14] = box_radius(3, llo, lhi);
      w[15] = box_radius(3, rlo, rhi);
    } else {
      const float v[8] = {llo[0], llo[1], lhi[0], lhi[1], rlo[0], rlo[1], rhi[0], rhi[1]};
      std::memcpy(w, v, sizeof v);
      std::memcpy(w + 8, &cl, 4);
      std::memcpy(w + 9, &cr, 4);
      w[10] = box_radius(2, llo, lhi);
      w[11] = box_radius(2, rlo, rhi);
    }
    sah += box_area(dim, B.lo, B.hi) / root_area;
  }
  int64_t leaves = 0;
  for (const BNode& B : nodes)
    if (B.leaf) {
      ++leaves;
      sah += (double)B.count * box_area(dim, B.lo, B.hi) / root_area;
    }
  T.order = idx;
  T.stats.n_nodes = (int64_t)order_int.size();
  T.stats.n_leaves = leaves;
  T.stats.max_depth = max_depth;
  T.stats.sah_cost = sah;
  return T;
}

namespace {

// cone of the normals of items order[start, start + count)
Cone cone_of(const FlatTree& T, int32_t start, int32_t count,
             const std::vector<std::vector<double>>& normals, const std::vector<uint8_t>& always) {
  Cone c{{0, 0, 1}, -1.0f, 0.0f};   // full cone
  double s[3] = {0, 0, 0};
  int64_t m = 0;
  for (int32_t i = start; i < start + count; ++i) {
    const int32_t it = T.order[i];
    if (always[it]) return c;
    const std::vector<double>& nv = normals[it];
    for (size_t j = 0; j + 3 <= nv.size(); j += 3) {
      s[0] += nv[j]; s[1] += nv[j + 1]; s[2] += nv[j + 2];
      ++m;
    }
  }
  double len = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  if (m == 0 || len < 1e-6 * (double)m) return c;
  double ax[3] = {s[0] / len, s[1] / len, s[2] / len};
  double half = 0;
  for (int32_t i = start; i < start + count; ++i) {
    const std::vector<double>& nv = normals[T.order[i]];
    for (size_t j = 0; j + 3 <= nv.size(); j += 3) {
      double d = ax[0] * nv[j] + ax[1] * nv[j + 1] + ax[2] * nv[j + 2];
      d = std::min(1.0, std::max(-1.0, d));
      half = std::max(half, std::acos(d));
    }
  }
  half += 1e-4;   // padding: the device test runs in FP32
  if (half >= 0.5 * M_PI) return c;
  c.axis[0] = (float)ax[0];
  c.axis[1] = (float)ax[1];
  c.axis[2] = (float)ax[2];
  c.cos_a = (float)std::cos(half);
  c.sin_a = (float)std::sin(half);
  return c;
}

void decode(int32_t code, int32_t& start, int32_t& count) {
  int32_t v = -code - 1;
  start = v >> 3;
  count = v & 7;
}

// item range covered by a child code (internal children: walk to the
// leftmost and rightmost leaves)
void child_range(const FlatTree& T, int32_t code, int32_t& start, int32_t& count) {
  const int nf = T.dim == 3 ? 16 : 12;
  const int co = T.dim == 3 ? 12 : 8;
  if (code < 0) {
    decode(code, start, count);
    return;
  }
  int32_t lo_code = code, hi_code = code;
  while (lo_code >= 0) std::memcpy(&lo_code, &T.nodes[(size_t)lo_code * nf + co], 4);
  while (hi_code >= 0) {
    int32_t r;
    std::memcpy(&r, &T.nodes[(size_t)hi_code * nf + co + 1], 4);
    if (r == kEmpty) std::memcpy(&r, &T.nodes[(size_t)hi_code * nf + co], 4);
    hi_code = r;
  }
  int32_t s0, c0, s1, c1;
  decode(lo_code, s0, c0);
  decode(hi_code, s1, c1);
  start = s0;
  count = s1 + c1 - s0;
}

}  // namespace

void build_cones(FlatTree& T, const std::vector<std::vector<double>>& normals,
                 const std::vector<uint8_t>& always) {
  const int64_t nn = T.stats.n_nodes;
  const int nf = T.dim == 3 ? 16 : 12;
  const int co = T.dim == 3 ? 12 : 8;
  const int cw = T.dim == 3 ? 12 : 8;
  T.cones.assign((size_t)nn * cw, 0.0f);
  for (int64_t d = 0; d < nn; ++d) {
    Cone cc[2];
    for (int side = 0; side < 2; ++side) {
      int32_t code;
      std::memcpy(&code, &T.nodes[(size_t)d * nf + co + side], 4);
      if (code == kEmpty) {
        cc[side] = Cone{{0, 0, 1}, -1.0f, 0.0f};
        continue;
      }
      int32_t s, c;
      child_range(T, code, s, c);
      cc[side] = cone_of(T, s, c, normals, always);
    }
    float* w = &T.cones[(size_t)d * cw];
    if (T.dim == 3) {
      const float v[12] = {cc[0].axis[0], cc[0].axis[1], cc[0].axis[2], cc[0].cos_a,
                           cc[0].sin_a,   cc[1].axis[0], cc[1].axis[1], cc[1].axis[2],
                           cc[1].cos_a,   cc[1].sin_a,   0.0f,          0.0f};
      std::memcpy(w, v, sizeof v);
    } else {
      const float v[8] = {cc[0].axis[0], cc[0].axis[1], cc[0].cos_a, cc[0].sin_a,
                          cc[1].axis[0], cc[1].axis[1], cc[1].cos_a, cc[1].sin_a};
      std::memcpy(w, v, sizeof v);
    }
  }
}

std::string check_tree(const FlatTree& T, const std::vector<ItemBox>& boxes) {
  const int64_t n = (int64_t)boxes.size();
  if (n == 0) return T.stats.n_nodes == 0 ? "" : "nodes for an empty tree";
  if ((int64_t)T.order.size() != n) return "order size";
  std::vector<int> seen(n, 0);
  for (int32_t it : T.order) {
    if (it < 0 || it >= n) return "order index out of range";
    seen[it]++;
  }
  for (int64_t i = 0; i < n; ++i)
    if (seen[i] != 1) return "item not in exactly one slot";
  if (T.stats.max_depth > max_tree_depth(T.dim)) return "tree deeper than the traversal stack";
  const int nf = T.dim == 3 ? 16 : 12;
  const int co = T.dim == 3 ? 12 : 8;
  std::vector<int> leaf_hits(n, 0);
  struct E { int32_t node; int depth; };
  std::vector<E> st{{0, 0}};
  while (!st.empty()) {
    E e = st.back();
    st.pop_back();
    if (e.depth > max_tree_depth(T.dim)) return "stack bound exceeded";
    const float* w = &T.nodes[(size_t)e.node * nf];
    for (int side = 0; side < 2; ++side) {
      int32_t code;
      std::memcpy(&code, w + co + side, 4);
      if (code == kEmpty) continue;
      float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      if (T.dim == 3) {
        for (int k = 0; k < 3; ++k) { lo[k] = w[6 * side + k]; hi[k] = w[6 * side + 3 + k]; }
      } else {
        for (int k = 0; k < 2; ++k) { lo[k] = w[4 * side + k]; hi[k] = w[4 * side + 2 + k]; }
      }
      int32_t s, c;
      child_range(T, code, s, c);
      for (int32_t i = s; i < s + c; ++i) {
        const ItemBox& b = boxes[T.order[i]];
        for (int k = 0; k < T.dim; ++k)
          if (b.lo[k] < lo[k] || b.hi[k] > hi[k]) return "child box does not contain an item";
      }
      if (code < 0) {
        if (c < 1 || c > kMaxLeaf) return "leaf size";
        for (int32_t i = s; i < s + c; ++i) leaf_hits[T.order[i]]++;
      } else {
        if (code >= T.stats.n_nodes) return "child index out of range";
        st.push_back({code, e.depth + 1});
      }
    }
  }
  for (int64_t i = 0; i < n; ++i)
    if (leaf_hits[i] != 1) return "item reached by not exactly one leaf";
  return "";
}

int promote_top_levels(FlatTree& t, int levels) {
  const int nf = t.dim == 3 ? 16 : 12;
  const int co = t.dim == 3 ? 12 : 8;
  const int nc = t.dim == 3 ? 12 : 8;
  const int64_t n = t.stats.n_nodes;
  if (n <= 0 || levels <= 0) return 0;
  auto child = [&](int64_t node, int side) {
    int32_t c;
    std::memcpy(&c, &t.nodes[(size_t)node * nf + co + side], 4);
    return c;
  };
  // breadth-first over the top levels
  std::vector<int64_t> top{0};
  for (size_t h = 0, lvl_end = 1, depth = 0; h < top.size(); ++h) {
    if (h == lvl_end) {
      lvl_end = top.size();
      ++depth;
    }
    if ((int)depth + 1 >= levels) continue;
    for (int side = 0; side < 2; ++side) {
      const int32_t c = child(top[h], side);
      if (c >= 0) top.push_back(c);
    }
  }
  std::vector<int64_t> newid(n, -1);
  int64_t k = 0;
  for (int64_t o : top) newid[o] = k++;
  for (int64_t o = 0; o < n; ++o)
    if (newid[o] < 0) newid[o] = k++;
  std::vector<float> nodes(t.nodes.size());
  std::vector<float> cones(t.cones.size());
  for (int64_t o = 0; o < n; ++o) {
    const int64_t d = newid[o];
    std::memcpy(&nodes[(size_t)d * nf], &t.nodes[(size_t)o * nf], sizeof(float) * nf);
    for (int side = 0; side < 2; ++side) {
      int32_t c = child(o, side);
      if (c >= 0) c = (int32_t)newid[c];
      std::memcpy(&nodes[(size_t)d * nf + co + side], &c, 4);
    }
    if (!t.cones.empty())
      std::memcpy(&cones[(size_t)d * nc], &t.cones[(size_t)o * nc], sizeof(float) * nc);
  }
  t.nodes.swap(nodes);
  t.cones.swap(cones);
  return (int)top.size();
}

std::string preprocess(int dim, int64_t nv, const float* V, int64_t np, const int32_t* P,
                       const uint8_t* bc, HostScene& S, int leaf_d, int leaf_n, int leaf_s,
                       const std::vector<double>* extra_boxes) {
  if (dim != 2 && dim != 3) return "dim must be 2 or 3";
  const bool shapes = extra_boxes && !extra_boxes->empty();
  if (nv < 0 || np < 0) return "negative count";
  if (!shapes || np > 0) {
    if (nv <= 0 || !V) return "no vertices";
    if (np <= 0 || !P || !bc) return "no primitives";
  }
  if (np >= (int64_t(1) << 27)) return "too many primitives";
  S.dim = dim;
  S.n_vertices = nv;
  S.n_prims = np;
  S.V.assign(3 * nv, 0.0f);
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < dim; ++k) {
      float x = V[dim * i + k];
      if (!std::isfinite(x)) return "non-finite vertex coordinate";
      S.V[3 * i + k] = x;
    }
  S.P.assign(3 * np, 0);
  S.bc.assign(bc, bc + np);
  S.normal.assign(3 * np, 0.0);
  S.measure.assign(np, 0.0);
  S.d_prims.clear();
  S.n_prims_list.clear();
  for (int64_t i = 0; i < np; ++i) {
    if (bc[i] > 3) return "boundary flag must be 0 (Dirichlet), 1 (Neumann), 2 or 3 (double-sided)";
    for (int k = 0; k < dim; ++k) {
      int32_t v = P[dim * i + k];
      if (v < 0 || v >= nv) return "primitive vertex index out of range";
      S.P[3 * i + k] = v;
    }
    const float* a = &S.V[3 * S.P[3 * i]];
    const float* b = &S.V[3 * S.P[3 * i + 1]];
    double e1[3] = {(double)b[0] - a[0], (double)b[1] - a[1], (double)b[2] - a[2]};
    double n[3];
    if (dim == 2) {
      n[0] = e1[1]; n[1] = -e1[0]; n[2] = 0;
      S.measure[i] = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1]);
    } else {
      const float* c = &S.V[3 * S.P[3 * i + 2]];
      double e2[3] = {(double)c[0] - a[0], (double)c[1] - a[1], (double)c[2] - a[2]};
      n[0] = e1[1] * e2[2] - e1[2] * e2[1];
      n[1] = e1[2] * e2[0] - e1[0] * e2[2];
      n[2] = e1[0] * e2[1] - e1[1] * e2[0];
      S.measure[i] = 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    }
    double ln = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(ln > 0) || !(S.measure[i] > 0)) return "degenerate (zero-measure) primitive";
    for (int k = 0; k < 3; ++k) S.normal[3 * i + k] = n[k] / ln;
    ((bc[i] & 1) ? S.n_prims_list : S.d_prims).push_back((int32_t)i);
  }
  // scene box
  for (int k = 0; k < 3; ++k) { S.lo[k] = 1e300; S.hi[k] = -1e300; }
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) {
      S.lo[k] = std::min(S.lo[k], (double)S.V[3 * i + k]);
      S.hi[k] = std::max(S.hi[k], (double)S.V[3 * i + k]);
    }
  if (shapes)
    for (size_t i = 0; i + 6 <= extra_boxes->size(); i += 6)
      for (int k = 0; k < 3; ++k) {
        S.lo[k] = std::min(S.lo[k], (*extra_boxes)[i + k]);
        S.hi[k] = std::max(S.hi[k], (*extra_boxes)[i + 3 + k]);
      }
  double d2 = 0;
  for (int k = 0; k < 3; ++k) {
    S.center[k] = 0.5 * (S.lo[k] + S.hi[k]);
    d2 += (S.hi[k] - S.lo[k]) * (S.hi[k] - S.lo[k]);
  }
  S.L = 0.5 * std::sqrt(d2);

  // silhouette elements of the Neumann boundary
  struct K { int32_t a, b, prim; };
  std::vector<K> keys;
  keys.reserve(S.n_prims_list.size() * dim);
  for (int32_t p : S.n_prims_list) {
    if (dim == 2) {
      for (int k = 0; k < 2; ++k) keys.push_back({S.P[3 * p + k], S.P[3 * p + k], p});
    } else {
      for (int k = 0; k < 3; ++k) {
        int32_t a = S.P[3 * p + k], b = S.P[3 * p + (k + 1) % 3];
        keys.push_back({std::min(a, b), std::max(a, b), p});
      }
    }
  }
  std::sort(keys.begin(), keys.end(), [](const K& x, const K& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    return x.prim < y.prim;
  });
  S.elem_v.clear();
  S.elem_n.clear();
  S.elem_always.clear();
  for (size_t i = 0; i < keys.size();) {
    size_t j = i;
    while (j < keys.size() && keys[j].a == keys[i].a && keys[j].b == keys[i].b) ++j;
    const size_t m = j - i;
    auto emit = [&](int32_t p0, int32_t p1, bool single) {
      S.elem_v.push_back(keys[i].a);
      S.elem_v.push_back(keys[i].b);
      for (int k = 0; k < 3; ++k) S.elem_n.push_back(S.normal[3 * p0 + k]);
      for (int k = 0; k < 3; ++k) S.elem_n.push_back(single ? -S.normal[3 * p0 + k] : S.normal[3 * p1 + k]);
      S.elem_always.push_back(single ? 1 : 0);
    };
    if (m == 1) emit(keys[i].prim, keys[i].prim, true);
    else
      for (size_t u = i; u < j; ++u)
        for (size_t w = u + 1; w < j; ++w) emit(keys[u].prim, keys[w].prim, false);
    i = j;
  }

  // trees
  auto prim_box = [&](int32_t p) {
    ItemBox b;
    for (int k = 0; k < 3; ++k) { b.lo[k] = 3e38f; b.hi[k] = -3e38f; }
    for (int c = 0; c < dim; ++c)
      for (int k = 0; k < 3; ++k) {
        float x = S.V[3 * S.P[3 * p + c] + k];
        b.lo[k] = std::min(b.lo[k], x);
        b.hi[k] = std::max(b.hi[k], x);
      }
    return b;
  };
  std::vector<ItemBox> bd, bn, bs;
  for (int32_t p : S.d_prims) bd.push_back(prim_box(p));
  for (int32_t p : S.n_prims_list) bn.push_back(prim_box(p));
  const int64_t ne = (int64_t)S.elem_always.size();
  for (int64_t e = 0; e < ne; ++e) {
    ItemBox b;
    for (int k = 0; k < 3; ++k) {
      float x0 = S.V[3 * S.elem_v[2 * e] + k], x1 = S.V[3 * S.elem_v[2 * e + 1] + k];
      b.lo[k] = std::min(x0, x1);
      b.hi[k] = std::max(x0, x1);
    }
    bs.push_back(b);
  }
  S.treeD = build_tree(dim, bd, leaf_d);
  S.treeN = build_tree(dim, bn, leaf_n);
  // silhouette elements: normal cone of their two face normals (a full cone
  // for elements that are always silhouettes), for the orientation-aware
  // split cost
  std::vector<ItemCone> sc((size_t)ne);
  for (int64_t e = 0; e < ne; ++e) {
    const double* n0 = &S.elem_n[6 * e];
    const double* n1 = n0 + 3;
    double a[3], nn = 0;
    for (int k = 0; k < 3; ++k) {
      a[k] = n0[k] + n1[k];
      nn += a[k] * a[k];
    }
    nn = std::sqrt(nn);
    if (S.elem_always[e] || nn < 1e-9) {
      sc[e] = ItemCone{{n0[0], n0[1], n0[2]}, M_PI};
      continue;
    }
    for (int k = 0; k < 3; ++k) sc[e].axis[k] = a[k] / nn;
    const double d = sc[e].axis[0] * n0[0] + sc[e].axis[1] * n0[1] + sc[e].axis[2] * n0[2];
    sc[e].angle = std::acos(std::max(-1.0, std::min(1.0, d)));
  }
  S.treeS = build_tree(dim, bs, leaf_s, &sc);
  std::vector<std::vector<double>> en(ne);
  for (int64_t e = 0; e < ne; ++e) en[e].assign(S.elem_n.begin() + 6 * e, S.elem_n.begin() + 6 * e + 6);
  if (ne > 0) build_cones(S.treeS, en, S.elem_always);
  S.topD = promote_top_levels(S.treeD, kTopLevels);
  S.topN = promote_top_levels(S.treeN, kTopLevels);
  S.topS = promote_top_levels(S.treeS, kTopLevels);
  std::string err = check_tree(S.treeD, bd);
  if (err.empty()) err = check_tree(S.treeN, bn);
  if (err.empty()) err = check_tree(S.treeS, bs);
  if (!err.empty()) return "internal tree check failed: " + err;
  if (dim == 3 && ne > 0) {
    err = pack_tree4(S.treeS, true, S.sil4, S.n_sil4, S.levels_sil4, S.top_sil4, S.root_sil4);
    if (!err.empty()) return "4-wide silhouette tree: " + err;
  }
  if (dim == 3 && !S.d_prims.empty()) {
    err = pack_tree4(S.treeD, false, S.dir4, S.n_dir4, S.levels_dir4, S.top_dir4, S.root_dir4);
    if (!err.empty()) return "4-wide Dirichlet tree: " + err;
  }
  if (dim == 3 && !S.n_prims_list.empty()) {
    err = pack_tree4(S.treeN, false, S.ray4, S.n_ray4, S.levels_ray4, S.top_ray4, S.root_ray4);
    if (!err.empty()) return "4-wide Neumann ray tree: " + err;
  }
  return "";
}

namespace {

// octahedral map of a unit vector onto the square [-1, 1]^2, as two signed
// 16-bit lattice words, and its inverse with the steps the device takes
void oct_encode(const double n[3], int16_t q[2]) {
  const double l1 = std::fabs(n[0]) + std::fabs(n[1]) + std::fabs(n[2]);
  double p = n[0] / l1, r = n[1] / l1;
  if (n[2] < 0.0) {
    const double tp = (1.0 - std::fabs(r)) * (p >= 0.0 ? 1.0 : -1.0);
    const double tr = (1.0 - std::fabs(p)) * (r >= 0.0 ? 1.0 : -1.0);
    p = tp;
    r = tr;
  }
  q[0] = (int16_t)std::lround(std::max(-1.0, std::min(1.0, p)) * 32767.0);
  q[1] = (int16_t)std::lround(std::max(-1.0, std::min(1.0, r)) * 32767.0);
}

void oct_decode(const int16_t q[2], double n[3]) {
  double p = q[0] / 32767.0, r = q[1] / 32767.0;
  const double z = 1.0 - std::fabs(p) - std::fabs(r);
  if (z < 0.0) {
    const double tp = (1.0 - std::fabs(r)) * (p >= 0.0 ? 1.0 : -1.0);
    const double tr = (1.0 - std::fabs(p)) * (r >= 0.0 ? 1.0 : -1.0);
    p = tp;
    r = tr;
  }
  const double l = std::sqrt(p * p + r * r + z * z);
  n[0] = p / l;
  n[1] = r / l;
  n[2] = z / l;
}

struct Child4 {
  float lo[3], hi[3];
  int32_t code;       // binary code (leaf, or a binary node index), kEmpty if none
  Cone cone;
};

}  // namespace

std::string pack_tree4(const FlatTree& t, bool silhouette, std::vector<uint32_t>& words, int64_t& n_nodes,
                       int& levels, int& top, int32_t& root) {
  words.clear();
  n_nodes = 0;
  levels = 0;
  top = 0;
  root = 0;
  if (t.dim != 3) return "3D trees only";
  const int64_t nb = t.stats.n_nodes;
  if (nb <= 0) return "";
  const int nf = 16, co = 12, cw = 12;
  auto binary_child = [&](int64_t b, int side, Child4& c) {
    const float* w = &t.nodes[(size_t)b * nf];
    std::memcpy(&c.code, w + co + side, 4);
    for (int k = 0; k < 3; ++k) {
      c.lo[k] = w[6 * side + k];
      c.hi[k] = w[6 * side + 3 + k];
    }
    if (silhouette) {
      const float* q = &t.cones[(size_t)b * cw + 5 * side];
      c.cone = Cone{{q[0], q[1], q[2]}, q[3], q[4]};
    } else {
      c.cone = Cone{{0, 0, 1}, -1.0f, 0.0f};
    }
  };
  // the children of the 4-wide node made of binary node b: each binary
  // child that is a leaf, and the two children of each internal one
  auto children_of = [&](int64_t b, std::vector<Child4>& out) {
    out.clear();
    for (int side = 0; side < 2; ++side) {
      Child4 c;
      binary_child(b, side, c);
      if (c.code == kEmpty) continue;
      if (c.code < 0) {
        out.push_back(c);
        continue;
      }
      for (int s2 = 0; s2 < 2; ++s2) {
        Child4 g;
        binary_child(c.code, s2, g);
        if (g.code != kEmpty) out.push_back(g);
      }
    }
  };
  // breadth-first numbering of the 4-wide nodes (by their binary node)
  std::vector<int64_t> order{0};
  std::vector<int> level{0};
  std::vector<int64_t> id4(nb, -1);
  id4[0] = 0;
  std::vector<Child4> ch;
  for (size_t h = 0; h < order.size(); ++h) {
    children_of(order[h], ch);
    for (const Child4& c : ch)
      if (c.code >= 0) {
        if (c.code >= nb) return "child index out of range";
        if (id4[c.code] >= 0) return "node reached twice";
        id4[c.code] = (int64_t)order.size();
        order.push_back(c.code);
        level.push_back(level[h] + 1);
      }
  }
  n_nodes = (int64_t)order.size();
  if (n_nodes > (int64_t(1) << 22)) return "too many nodes for the traversal's entry codes";
  for (size_t h = 0; h < order.size(); ++h)
    if (level[h] < kSil4TopLevels) ++top;
  // subtree heights, children before parents (reverse breadth-first order)
  std::vector<int> height(order.size(), 1);
  for (size_t h = order.size(); h-- > 0;) {
    children_of(order[h], ch);
    for (const Child4& c : ch)
      if (c.code >= 0) height[h] = std::max(height[h], height[id4[c.code]] + 1);
  }
  levels = height[0];
  if (levels > kSil4Levels) return "taller than the traversal's stack bound";
  auto entry = [&](int64_t n4) { return (int32_t)(n4 | (int64_t)(height[n4] - 1) << 22); };
  root = entry(0);
  const int stride = silhouette ? kSil4Words : kDir4Words;
  words.assign((size_t)n_nodes * stride, 0u);
  for (int64_t n = 0; n < n_nodes; ++n) {
    children_of(order[n], ch);
    if (ch.empty() || ch.size() > 4) return "node without children or with more than four";
    uint32_t* w = &words[(size_t)n * stride];
    if (!silhouette) {
      // exact FP32 child boxes (lattice boxes measured 7 % slower here: the
      // closest-point search then reaches more leaves) and the child codes
      for (int i = 0; i < 4; ++i) {
        float b[6] = {0, 0, 0, 0, 0, 0};
        int32_t code = kEmpty;
        if (i < (int)ch.size()) {
          for (int k = 0; k < 3; ++k) {
            b[k] = ch[i].lo[k];
            b[3 + k] = ch[i].hi[k];
          }
          code = ch[i].code >= 0 ? entry(id4[ch[i].code]) : ch[i].code;
        }
        std::memcpy(w + 6 * i, b, sizeof b);
        std::memcpy(w + 24 + i, &code, 4);
      }
      continue;
    }
    float o[3], hi[3], s[3];
    for (int k = 0; k < 3; ++k) {
      o[k] = std::numeric_limits<float>::max();
      hi[k] = -std::numeric_limits<float>::max();
      for (const Child4& c : ch) {
        o[k] = std::min(o[k], c.lo[k]);
        hi[k] = std::max(hi[k], c.hi[k]);
      }
      if (!(o[k] <= hi[k])) return "empty child box";
      s[k] = (float)(((double)hi[k] - (double)o[k]) / 255.0);
      while (std::fmaf(255.0f, s[k], o[k]) < hi[k])
        s[k] = std::nextafter(s[k], std::numeric_limits<float>::infinity());
    }
    std::memcpy(w + 0, o, 12);
    std::memcpy(w + 3, s, 12);
    uint8_t qb[24] = {0};
    for (int i = 0; i < 4; ++i) {
      int32_t code = kEmpty;
      float R = 0.0f, cs = -1.0f, sn = 0.0f;
      int16_t oq[2] = {0, 0};
      if (i < (int)ch.size()) {
        const Child4& c = ch[i];
        float lo2[3], hi2[3];
        for (int k = 0; k < 3; ++k) {
          int ql = 0, qh = 0;
          if (s[k] > 0.0f) {
            ql = (int)std::floor(((double)c.lo[k] - (double)o[k]) / (double)s[k]);
            qh = (int)std::ceil(((double)c.hi[k] - (double)o[k]) / (double)s[k]);
          }
          ql = std::max(0, std::min(255, ql));
          qh = std::max(0, std::min(255, qh));
          while (ql > 0 && std::fmaf((float)ql, s[k], o[k]) > c.lo[k]) --ql;
          while (qh < 255 && std::fmaf((float)qh, s[k], o[k]) < c.hi[k]) ++qh;
          lo2[k] = std::fmaf((float)ql, s[k], o[k]);
          hi2[k] = std::fmaf((float)qh, s[k], o[k]);
          if (!(lo2[k] <= c.lo[k] && hi2[k] >= c.hi[k])) return "quantised box does not contain the child";
          qb[6 * i + k] = (uint8_t)ql;
          qb[6 * i + 3 + k] = (uint8_t)qh;
        }
        code = c.code >= 0 ? entry(id4[c.code]) : c.code;
        R = box_radius(3, lo2, hi2);
        if (c.cone.cos_a > 0.0f) {
          double a[3] = {c.cone.axis[0], c.cone.axis[1], c.cone.axis[2]};
          const double al = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
          for (double& v : a) v /= al;
          oct_encode(a, oq);
          double b[3];
          oct_decode(oq, b);
          const double dot = std::max(-1.0, std::min(1.0, a[0] * b[0] + a[1] * b[1] + a[2] * b[2]));
          // the stored half-angle, widened by the axis error and by a margin
          // for the device's FP32 decoding
          const double half = std::atan2((double)c.cone.sin_a, (double)c.cone.cos_a) + std::acos(dot) + 2e-6;
          if (half < 0.5 * M_PI) {
            cs = std::nextafter((float)std::cos(half), -std::numeric_limits<float>::infinity());
            sn = std::nextafter((float)std::sin(half), std::numeric_limits<float>::infinity());
            if (!(cs > 0.0f)) { cs = -1.0f; sn = 0.0f; oq[0] = oq[1] = 0; }
          } else {
            oq[0] = oq[1] = 0;
          }
        }
      }
      std::memcpy(w + 12 + i, &code, 4);
      std::memcpy(w + 16 + i, &R, 4);
      const uint32_t ow = (uint32_t)(uint16_t)oq[0] | ((uint32_t)(uint16_t)oq[1] << 16);
      w[20 + i] = ow;
      std::memcpy(w + 24 + i, &cs, 4);
      std::memcpy(w + 28 + i, &sn, 4);
    }
    std::memcpy(w + 6, qb, 24);
  }
  return "";
}

}  // namespace wost
