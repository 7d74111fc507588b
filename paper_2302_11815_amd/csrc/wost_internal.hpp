// Declarations shared by the C-ABI layer (api.hip) and the kernels
// (wost_kernels.hip).  Nothing here is part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wost {

constexpr int kBlock = 256;      // threads per block of the walk kernels
// traversal stack entries per lane: trees are at most kStack<D> - 1 deep
template <int D>
constexpr int kStack = D == 2 ? 24 : 32;
constexpr int kLeafMax = 4;      // primitives per tree leaf (the builder's leaf size bound)
constexpr int kTopNodes = 15;    // nodes per tree numbered first (top 4 levels), kept in LDS
constexpr int kSRec = 8;         // float4 per 3D silhouette-tree node record (128 B, one cache line)
constexpr int kEventCap = 64;

// 4-wide silhouette tree (3D).  A traversal entry that is not a leaf code
// holds a node index (bits 0-21) and the height h of the node's subtree
// (bits 22-25 hold h - 1; a node whose children are all leaves has h = 1);
// a revisit entry (kRevisitFlag) is such an entry plus, in bits 26-29, the
// mask of the node's children still to search.  A lane's search keeps at
// most K - h - 1 entries on its stack (K = kStack<3>) while it visits an
// entry of height h: it pushes a node's other admissible children (of
// height <= h - 1), farthest first, when the stack then holds at most K - h
// entries, and otherwise one revisit entry for them.  Both keep the bound
// for every entry visited next, so a stack never overflows; the builder
// keeps the root's height within kSil4Height.
constexpr int32_t kRevisitFlag = 1 << 30;
constexpr int kRevisitShift = 26;
constexpr int kHeightShift = 22;
constexpr int32_t kEntryNode = (1 << 22) - 1;
constexpr int kSil4Height = 16;
static_assert(kSil4Height <= kStack<3> - 1, "the root entry's stack bound");    // walks ended by the cap or the escape radius, recorded per solve

// traffic counters (node / primitive fetches per query kind)
// (lane-level fetch counts), then wave-level iteration counts of the
// traversal loops and their leaf loops (SIMT efficiency = lane iterations /
// (64 x wave iterations)), then walk steps counted per wave
enum {
  kCntQ1Node = 0, kCntQ1Prim, kCntQ2Node, kCntQ2Cone, kCntQ2Elem, kCntQ3Node, kCntQ3Prim,
  kCntQ4Node, kCntQ4Prim, kCntVisNode, kCntVisPrim,
  kWaveQ1Iter, kWaveQ1Leaf, kWaveQ2Iter, kWaveQ2Leaf, kWaveQ3Iter, kWaveQ3Leaf, kWaveQ4Iter,
  kWaveVisIter, kWaveVisLeaf, kWaveSteps,
  // wave-level shader-clock cycles per phase of the step (counting variant)
  kCycQ1, kCycQ2, kCycQ3, kCycQ4, kCycRest, kTrafficCounters
};

// boundary / source data on the device
struct FnDev {
  int kind;       // 0 zero, 1 const, 2 poly2, 3 expcos, 4 per-corner
  int as_nd;      // 1: value = grad(F) . n_prim
  float c[10];
  const float* pc;  // per-corner values [n_prims][dim], indexed by original primitive id
};

// entries of SceneDev::fn: Dirichlet g, Neumann h, source f, and the "-"
// side data of double-sided primitives
enum { kFnG = 0, kFnH, kFnF, kFnGm, kFnHm, kFnCount };

// Flattened, device-resident scene.  Node layout: 3D 4 float4 per node
// (both children's boxes, then their codes), 2D 3 float4 per node.
struct SceneDev {
  int dim;
  // Dirichlet tree and primitives (3D: 3 float4 per triangle, 2D: 1 float4 per segment);
  // the 3D tree is 4-wide, kSRec float4 per node (the builder's 32-word record)
  const float4* dn;
  const float4* dp;
  const int* did;          // original primitive id per slot
  const uint8_t* dside;    // per slot: 1 double-sided (read by the double-sided kernels only)
  int nD;
  // Neumann tree and primitives
  const float4* nn;
  const float4* np;
  const float* narea;      // length / area per slot
  const int* nid;          // original id per slot
  const int* ninv;         // original id -> slot (-1 for Dirichlet primitives)
  const uint8_t* nside;    // per slot: 1 double-sided
  int nN;
  // normal-cone hierarchy over silhouette elements
  const float4* sn;        // 3D: kSRec float4 per 4-wide node (the builder's 32-word
                           // record: frame, quantised child boxes, codes, radii, cones);
                           // 2D: binary nodes as above
  const float4* sc;        // 2D: child cones, 2 float4 per node (3D: in sn)
  const float4* se;        // elements: 3D 3 float4 (a, b, normals), 2D 2 float4 (p, normals)
  int nE;
  // top-level nodes: the first topD / topN / topS nodes of each tree (its
  // levels above depth 4); a kernel that copies them into LDS points
  // tdn / tnn / tsn / tsc there and sets ctD / ctN / ctS (0: read from HBM)
  int topD, topN, topS;
  int sil4_root;           // 3D: the 4-wide silhouette tree's root entry (with its height)
  int dn_root;             // 3D: the 4-wide Dirichlet tree's root entry
  // 3D: the Neumann tree again as 4-wide records (exact boxes, the Dirichlet
  // layout) for the two ray queries; the sample descent keeps the binary tree
  const float4* rn;
  int rn_root, topR;
  const float4* trn;
  int ctR;
  const float4* tdn;
  const float4* tnn;
  const float4* tsn;
  const float4* tsc;
  int ctD, ctN, ctS;
  // boundary and source data, in device memory (indexed by kFnG ... kFnHm):
  // read only where a value is taken, so the walk loop keeps no registers
  // for them; fn_kind copies the kinds for the host's launch choices
  const FnDev* fn;
  int fn_kind[5];
  const float4* sdf;       // analytic Dirichlet shapes, 2 float4 each (Q.1 slots nD + i)
  int nS;
  int sdf_id0;             // reported id of shape 0 (= number of mesh primitives)
  int ds;                  // 1: the scene has double-sided primitives
  float offset;            // inward offset of on-boundary query origins
  float escape2;           // squared escape radius
  float escape;            // escape radius (caps the star radius without a Dirichlet boundary)
  float cx, cy, cz;        // scene centre
};

struct WalkParams {
  const float* points;      // [n_points][dim]
  const int32_t* start;     // optional [n_points]: Neumann slot a point lies on ("+" side),
                            // -2 - slot ("-" side of a double-sided one), or -1
  int64_t n_points;
  int32_t W;               // walks per point
  uint32_t point_base;     // RNG point index of point 0
  uint32_t walk_base;      // RNG walk index of walk 0
  uint32_t seed_lo, seed_hi;
  float sigma;             // screening coefficient, Laplacian(u) - sigma u = f
  float tik_sigma;         // Tikhonov switch: added to sigma from step tik_steps on
  int32_t tik_steps;
  float eps, rmin;
  int32_t max_steps;
  int32_t refill;          // persistent kernel: refill when this many lanes idle
  int32_t claim;           // persistent kernel: most walks a wave claims at once (>= 1)
  int32_t steal;           // cooperative searches: a steal round once this many lanes are idle
  int32_t order;           // 0 point-major walk ids, 1 walk-major
  float* est;              // [n_points][W] per-walk estimates
  unsigned long long* stats;    // steps, walks, capped, escaped
  unsigned long long* counter;  // work-queue cursor (persistent kernel)
  unsigned long long* traffic;  // [kTrafficCounters] (traffic accounting variant only)
  unsigned long long* events;   // optional: [0] count, then kEventCap records of 2 words,
                                // (point << 32 | walk, step count << 8 | kind): walks that
                                // ended capped (kind 2) or escaped (kind 3)
};

// One entry of the batched form's device work queue: a scene and its solve.
// Walks of an item are handed out in chunks of `chunk` walks; chunk ids of
// item i are [chunk_begin, chunk_begin + ceil(n_walks / chunk)) within its
// group.  Its points are [point_begin, point_begin + P.n_points) of the
// batch's point numbering, which the reduction walks through.
struct BatchItem {
  SceneDev S;
  WalkParams P;        // P.est points at the item's slice of the batch buffer
  int64_t n_walks;
  int64_t chunk_begin;
  int64_t point_begin;
  double* mean;        // [P.n_points] FP64 outputs
  double* var;
};

// The per-call part of a batch, in device memory next to the item table, so
// that a captured graph of the batch's kernels serves every call with the
// same kinds of groups: group g runs items [first, first + n_items) in
// n_chunks chunks of `chunk` walks; the reduction covers `points` points of
// all `n_items_all` items.
struct BatchGroupDev {
  int first;
  int n_items;
  int chunk;
  int pad;
  int64_t n_chunks;
};
struct BatchHeadDev {
  int n_items_all;
  int pad;
  int64_t points;
};

// One request of a serving round: its running per-point (mean, M2) over na
// walks, the round's per-point (mean, variance) over nb walks, and the slot
// that receives its largest standard error; its points are
// [point_begin, point_begin + n) of the round's point numbering.
struct MergeItem {
  double* mean;
  double* m2;
  const double* mb;
  const double* vb;
  int64_t n;
  int64_t point_begin;
  double na, nb;
  unsigned int* max_se;
};

// FP32 record of one walk step (trace / parity probes)
struct StepRec {
  float x[3];
  float n[3];
  int onN, cur;            // cur: original id of the Neumann primitive the walk is on, -1 otherwise
  float dD;
  float xbar[3];
  int primD;               // original id
  int term;                // 0 continue, 1 eps-shell, 2 capped, 3 escaped
  float g_term;
  float dsil, r;
  float v[3];
  int hit, hit_prim;       // original id
  float t;
  float p[3];
  int n_prim, valid;       // original id of the sampled Neumann primitive
  float z[3];
  float pdf, Nhat;
  float s_frac, Shat;
  float acc;               // walk estimate after this step
  float q;                 // screened continuation factor Q (1 for Poisson)
  int roulette;            // 1: the walk ended here by Russian roulette
  int side_g, side_h;      // double-sided: +1 / -1 side of g at the end, of h for the sample; else 0
};

// whether the walk kernels need the Neumann term
__host__ __device__ inline bool has_neumann_data(const SceneDev& S) {
  return S.fn_kind[kFnH] != 0 || (S.ds && S.fn_kind[kFnHm] != 0);
}

// Walk-kernel launchers of one dimension and one boundary form (DS: the
// scene has double-sided primitives); each pair is compiled in a
// translation unit of its own (wost_walks.hip).
template <int D, bool DS>
struct WalkPart {
  static hipError_t walks(const SceneDev& S, const WalkParams& P, int mode, int grid, bool count,
                          hipStream_t s);
  static hipError_t batch(const BatchItem* items, const BatchGroupDev* group, bool hh, bool hf,
                          unsigned long long* cursor, unsigned long long* stats, int grid, hipStream_t s);
  static hipError_t trace(const SceneDev& S, const WalkParams& P, const uint32_t* point_ids,
                          const uint32_t* walk_ids, int64_t n, int max_rec, StepRec* recs, int* n_steps,
                          float* values, hipStream_t s);
  static int resident_blocks(bool coop);   // persistent kernel, per CU
};
extern template struct WalkPart<2, false>;
extern template struct WalkPart<2, true>;
extern template struct WalkPart<3, false>;
extern template struct WalkPart<3, true>;

// ---- launchers (wost_kernels.hip) -----------------------------------------
hipError_t launch_fill_u64(unsigned long long* p, int n, hipStream_t s);
// mode 0 persistent, 1 plain; count = traffic accounting variant (plain form)
hipError_t launch_walks(const SceneDev& S, const WalkParams& P, int mode, int grid_blocks,
                        bool count, hipStream_t s);
hipError_t launch_reduce(const float* est, int64_t n_points, int W, double* mean, double* var,
                         hipStream_t s);
hipError_t launch_trace(const SceneDev& S, const WalkParams& P, const uint32_t* point_ids,
                        const uint32_t* walk_ids, int64_t n, int max_rec, StepRec* recs,
                        int* n_steps, float* values, hipStream_t s);
hipError_t launch_probe_q1(const SceneDev& S, const float* x, int64_t n, float* d, float* xbar,
                           int* prim, hipStream_t s);
hipError_t launch_probe_q2(const SceneDev& S, const float* x, const float* rmax, int64_t n,
                           float* d, hipStream_t s);
hipError_t launch_probe_q3(const SceneDev& S, const float* o, const float* v, const float* tmax,
                           const int* skip, int64_t n, float* t, int* prim, hipStream_t s);
hipError_t launch_probe_q4(const SceneDev& S, const float* x, const float* r, int64_t n,
                           uint32_t seed_lo, uint32_t seed_hi, float* z, float* pdf, int* prim,
                           hipStream_t s);
int max_resident_blocks(int dim, bool coop);
// every block reads buf[0, n4) reps times (L2 read bandwidth measurement)
hipError_t launch_stream_read(const float4* buf, int n4, int reps, int blocks, float* sink, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, int n, hipStream_t s);
// VALU issue measurement: every lane of `blocks` x 256 runs 8 independent
// chains of iters FMAs (kind 0) or of iters xor + add pairs (kind 1)
hipError_t launch_valu_peak(int kind, int iters, int blocks, float* sink, hipStream_t s);
// the merges of a serving round: every point of every request (items in
// point order, `points` in all)
hipError_t launch_merge_batch(const MergeItem* d_items, int n_items, int64_t points, hipStream_t s);
// one persistent launch over the items of one group (all of the same dim and
// data kinds), read with the group's sizes from device memory; `cursor`
// counts claimed chunks, `stats` receives the counters
hipError_t launch_batch(const BatchItem* d_items, const BatchGroupDev* d_group, int dim, bool hh, bool hf,
                        bool ds, unsigned long long* cursor, unsigned long long* stats, int grid, hipStream_t s);
// the fixed-order FP64 per-point reduction of every item of a batch (sizes
// and outputs from the device table; a fixed grid strides over the points)
hipError_t launch_reduce_batch(const BatchItem* d_items, const BatchHeadDev* d_head, hipStream_t s);

}  // namespace wost
