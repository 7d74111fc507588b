// Host-side scene preprocessing for the walk-on-stars solver: splitting the
// boundary into its Dirichlet and Neumann parts, the silhouette elements of
// the Neumann part (Sec. 5.1: mesh edges in 3D, polyline vertices in 2D, with
// the normals of their adjacent Neumann primitives), and the flattened trees
// the device traverses:
//   * a bounding volume hierarchy over the Dirichlet primitives (query Q.1),
//   * a bounding volume hierarchy over the Neumann primitives (Q.3 rays and
//     Q.4 sampling),
//   * a spatialized normal cone hierarchy over the silhouette elements (Q.2;
//     Sec. 5.1.1, after Johnson and Cohen), whose nodes carry normal cones
//     (axis = mean normal, half-angle = largest deviation from it).
// Trees are built with binned surface-area-heuristic splits (Sec. 5.1.1
// names SAH as the paper's choice) and stored in a "both children in the
// parent" layout: one node holds the bounds of its two children, so one
// node fetch decides both child tests.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace wost {

// Child codes stored in a node: >= 0 internal node index; < 0 leaf
// -(start * 8 + count) - 1 with 1 <= count <= kMaxLeaf; kEmpty for no child.
// The device unrolls leaf loops to kMaxLeaf primitives.
constexpr int32_t kEmpty = INT32_MIN;
constexpr int kMaxLeaf = 4;
// Deepest tree the device traversal accepts (its per-lane stacks hold one
// entry more).  2D trees are shallow, and their smaller stacks leave room in
// LDS for a fifth block per CU.
constexpr int max_tree_depth(int dim) { return dim == 2 ? 23 : 31; }

// Tree levels whose nodes are numbered first, breadth-first, so that the
// persistent walk kernels can keep them in LDS (at most 2^kTopLevels - 1
// nodes per tree).
constexpr int kTopLevels = 4;

inline int32_t leaf_code(int32_t start, int32_t count) { return -(start * 8 + count) - 1; }

struct TreeStats {
  int64_t n_nodes = 0, n_leaves = 0, n_items = 0;
  int max_depth = 0;
  double sah_cost = 0;
};

// One flattened tree: node words, the permutation of the input items in
// leaf order, and per-node cones (SNCH only).
struct FlatTree {
  int dim = 3;
  std::vector<float> nodes;      // 16 floats per node (3D) / 12 floats (2D)
  std::vector<int32_t> order;    // item index at each leaf slot
  std::vector<float> cones;      // 12 floats per node (3D) / 8 floats (2D)
  TreeStats stats;
};

struct ItemBox {
  float lo[3], hi[3];
};

// Normal cone of one item: unit axis and half-angle (radians; pi = all
// directions).
struct ItemCone {
  double axis[3];
  double angle;
};

// Builds a tree over `boxes` (centroids = box centres). leaf_size <= kMaxLeaf.
// With `cones` (one per item) the split cost is the surface area orientation
// heuristic: each side's area x item count is weighted by an orientation
// measure of the side's normal cone (the probability that a silhouette test
// from a random direction passes), so that splits also separate items by
// orientation and the cone culling of the silhouette query prunes more.
FlatTree build_tree(int dim, const std::vector<ItemBox>& boxes, int leaf_size,
                    const std::vector<ItemCone>* cones = nullptr);

// Half-angle-weighted orientation measure of the surface area orientation
// heuristic: sin(min(angle, pi/2)) + kSaohViewTerm, the pass probability of
// the cone test for a random view direction plus a term for the view cone
// of nearby queries.
constexpr double kSaohViewTerm = 0.1;

// Cone of a set of unit normals: axis and (cos, sin) of the half-angle,
// padded outward; `always` forces a half-angle of pi.
struct Cone {
  float axis[3];
  float cos_a, sin_a;
};

// Fills tree.cones given for each item the normals it carries
// (normals[item] is a list of unit vectors; an item flagged in `always`
// makes every cone containing it a full cone).
void build_cones(FlatTree& tree, const std::vector<std::vector<double>>& normals,
                 const std::vector<uint8_t>& always);

// Scene preprocessing on the host, shared by the device upload and the
// host-only checks.
// 3D trees with four children per node, one 128-byte record (32 words) per
// node, nodes numbered breadth-first from the root.  Dirichlet tree (and
// the Neumann tree's copy for the ray queries):
//   words 0-23  child boxes, FP32 (3 low then 3 high coordinates each)
//   words 24-27 child codes (as below), words 28-31 unused
// Silhouette tree:
//   words 0-2   quantisation origin o (FP32), the low corner of the node's box
//   words 3-5   lattice step s (FP32) per axis
//   words 6-11  child boxes, 6 bytes each (3 low then 3 high lattice indices q;
//               a coordinate is fmaf(q, s, o), never inside the child's box)
//   words 12-15 child codes: a leaf code, kEmpty, or a 4-wide node's index
//               (bits 0-21) with its subtree's height less one (bits 22-25;
//               a node whose children are all leaves has height 1)
//   words 16-19 radius of each dequantised child box's bounding sphere about
//               its centre, padded as box_radius does
//   words 20-23 child normal-cone axes, octahedral: two signed 16-bit words
//   words 24-27 cosines, words 28-31 sines of the cones' half-angles, widened
//               by the axis encoding's error (cosine <= 0: a full cone)
// (radii and sines derived on the device instead measured 7 % slower)
constexpr int kSil4Words = 32;
constexpr int kDir4Words = 32;
// the greatest height of a 4-wide tree (the traversal's stack bound)
constexpr int kSil4Levels = 16;
constexpr int kSil4TopLevels = 2;   // levels kept in LDS by the walk kernels

// Packs the binary tree t as 4-wide records, in the silhouette layout (t
// with its cones) or the Dirichlet layout; an empty string on success.
// levels receives the tree's height, top the number of nodes above level
// kSil4TopLevels (numbered first), root the root's traversal entry.
std::string pack_tree4(const FlatTree& t, bool silhouette, std::vector<uint32_t>& words, int64_t& n_nodes,
                       int& levels, int& top, int32_t& root);

struct HostScene {
  int dim = 3;
  int64_t n_vertices = 0, n_prims = 0;
  std::vector<float> V;            // [nv][3]
  std::vector<int32_t> P;          // [np][3]
  std::vector<uint8_t> bc;         // 0 / 1 Dirichlet / Neumann, 2 / 3 the same double-sided
  std::vector<double> normal;      // [np][3]
  std::vector<double> measure;     // [np]
  std::vector<int32_t> d_prims, n_prims_list;   // original ids
  // silhouette elements
  std::vector<int32_t> elem_v;     // [ne][2] vertex ids (2D: v, v)
  std::vector<double> elem_n;      // [ne][6] normals n0, n1 (n1 = -n0 for a single adjacent prim)
  std::vector<uint8_t> elem_always;
  FlatTree treeD, treeN, treeS;
  int topD = 0, topN = 0, topS = 0;   // nodes above depth kTopLevels, numbered first
  std::vector<uint32_t> sil4;        // 3D: the silhouette tree as 4-wide records
  int64_t n_sil4 = 0;
  int levels_sil4 = 0, top_sil4 = 0;
  int32_t root_sil4 = 0;
  std::vector<uint32_t> dir4;        // 3D: the Dirichlet tree as 4-wide records
  int64_t n_dir4 = 0;
  int levels_dir4 = 0, top_dir4 = 0;
  int32_t root_dir4 = 0;
  std::vector<uint32_t> ray4;        // 3D: the Neumann tree as 4-wide records (ray queries)
  int64_t n_ray4 = 0;
  int levels_ray4 = 0, top_ray4 = 0;
  int32_t root_ray4 = 0;
  double lo[3], hi[3], center[3], L = 0;
};

// Validates and preprocesses; returns an empty string or an error message.
// extra_boxes (optional, [n][6] lo[3] hi[3]): bounds of analytic shapes,
// folded into the scene box; with them the mesh may be empty.
std::string preprocess(int dim, int64_t nv, const float* V, int64_t np, const int32_t* P,
                       const uint8_t* bc, HostScene& out, int leaf_size_d, int leaf_size_n,
                       int leaf_size_s, const std::vector<double>* extra_boxes = nullptr);

// Renumbers a flattened tree so that its nodes above depth `levels` come
// first, in breadth-first order (the walk kernels copy them into LDS), and
// the others follow in their previous (depth-first) order; child codes and
// per-node cones move with their nodes.  Returns the number of promoted
// nodes (at most 2^levels - 1).
int promote_top_levels(FlatTree& t, int levels);

// Structural checks of a flattened tree (containment of every item in the
// boxes along its path, every item in exactly one leaf, depth bound).
std::string check_tree(const FlatTree& t, const std::vector<ItemBox>& boxes);

}  // namespace wost
