// Walk-on-stars device code for gfx950 (CDNA4, wave64): the walk kernels and
// everything they call, included by wost_kernels.hip (probes, reductions,
// dispatch) and wost_walks.hip (the walk kernels of one dimension and
// boundary form per translation unit, compiled in parallel).
//
// One lane runs one random walk (Sawhney et al. 2023, Algorithm 1).  Each
// step makes the four geometric queries of Sec. 5 against flattened trees
// held in HBM: Q.1 closest Dirichlet point, Q.2 closest silhouette point
// (normal-cone culled, Sec. 5.1.2 / Algorithms 3-4), Q.3 first Neumann hit
// along a ray clipped to the star radius, Q.4 a Neumann point sample by one
// random root-to-leaf descent (Algorithms 5-6) plus a visibility ray.
// Traversal stacks live in LDS, one column per lane, so that a wave's
// pushes and pops hit 64 distinct banks.  All arithmetic is FP32; the walk
// estimate is a Kahan-compensated FP32 sum; the per-point mean and variance
// are reduced in FP64 in a fixed order, so results are bit-reproducible and
// independent of which lane or launch form ran a walk.  That also needs
// floating-point contraction limited to single expressions (contract(on)):
// with cross-statement fusion the backend may fuse a multiply-add in one
// kernel and not in another that inlines the same step code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wost_internal.hpp"

#pragma clang fp contract(on)

namespace wost {

constexpr float kInf = 3.0e38f;
// how far back along a ray (in units of the Neumann query offset) a crossing
// through a primitive the ray leaves is looked for: the origin may lie just
// outside the primitive by rounding, and at a grazing angle the crossing lies
// far behind it (the oracle's ray query takes the same bound)
constexpr float kBehindReach = 64.0f;
constexpr int32_t kEmptyCode = INT32_MIN;
constexpr float kPi = 3.14159265358979f;

// Fetch counters of one lane (traffic accounting variant of the kernels):
// node and primitive fetches per query; see wost_traffic in wost.h.
struct Cnt {
  uint32_t v[kTrafficCounters];
  uint64_t t_mark;
  __device__ void add(int i, uint32_t k = 1) { v[i] += k; }
  // wave-level cycles since the last mark, credited to phase i (in units of
  // 16 cycles so that a lane's 32-bit counter does not wrap)
  __device__ void phase(int i) {
    const uint64_t now = clock64();
    const unsigned long long m = __ballot(1);
    if (__lane_id() == __ffsll((long long)m) - 1) v[i] += (uint32_t)((now - t_mark) >> 4);
    t_mark = now;
  }
  // counted once per wave: by the first lane active at this point
  __device__ void wave(int i) {
    const unsigned long long m = __ballot(1);
    if (__lane_id() == __ffsll((long long)m) - 1) v[i] += 1;
  }
};

// ---------------------------------------------------------------------------
// small fixed-size vectors
// ---------------------------------------------------------------------------
template <int D>
struct Vec {
  float v[D];
  __device__ float& operator[](int i) { return v[i]; }
  __device__ float operator[](int i) const { return v[i]; }
};

template <int D>
__device__ inline float dot(const Vec<D>& a, const Vec<D>& b) {
  float s = a[0] * b[0];
#pragma unroll
  for (int k = 1; k < D; ++k) s += a[k] * b[k];
  return s;
}
template <int D>
__device__ inline Vec<D> sub(const Vec<D>& a, const Vec<D>& b) {
  Vec<D> o;
#pragma unroll
  for (int k = 0; k < D; ++k) o[k] = a[k] - b[k];
  return o;
}
template <int D>
__device__ inline Vec<D> axpy(const Vec<D>& x, float s, const Vec<D>& d) {
  Vec<D> o;
#pragma unroll
  for (int k = 0; k < D; ++k) o[k] = x[k] + s * d[k];
  return o;
}
template <int D>
__device__ inline Vec<D> vload(const float* p) {
  Vec<D> o;
#pragma unroll
  for (int k = 0; k < D; ++k) o[k] = p[k];
  return o;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (point, walk, step, slot),
// key = 64-bit seed.  A uniform is (u >> 8) * 2^-24, exact in FP32.
// ---------------------------------------------------------------------------
__device__ inline uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
  // Draws of one step differ only in the slot word, so the compiler would
  // share their first-round products and keep them live across the tree
  // searches between the draws (spilled to scratch); an empty asm makes each
  // draw's counter opaque, so every draw computes its own rounds.
  asm volatile("" : "+v"(c.x), "+v"(c.z));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}
__device__ inline float u01(uint32_t u) { return (float)(u >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------------------
// tree nodes
// ---------------------------------------------------------------------------
template <int D>
struct NodePair {
  float lo[2][D], hi[2][D];
  int32_t code[2];
  float rad[2];   // children's bounding-sphere radii, padded (used by Q.2)
};

template <int D>
__device__ inline NodePair<D> load_node(const float4* __restrict__ N, int i);

// node i from any address space (global, or a copy in LDS)
template <int D, class Ptr>
__device__ inline NodePair<D> load_node_from(Ptr N, int i);

template <>
__device__ inline NodePair<3> load_node<3>(const float4* __restrict__ N, int i) {
  return load_node_from<3>(N, i);
}

template <>
__device__ inline NodePair<2> load_node<2>(const float4* __restrict__ N, int i) {
  return load_node_from<2>(N, i);
}

template <int D, class Ptr>
__device__ inline NodePair<D> load_node_from(Ptr N, int i) {
  NodePair<D> n;
  if constexpr (D == 3) {
    const float4 a = N[4 * i], b = N[4 * i + 1], c = N[4 * i + 2], d = N[4 * i + 3];
    n.lo[0][0] = a.x; n.lo[0][1] = a.y; n.lo[0][D - 1] = a.z;
    n.hi[0][0] = a.w; n.hi[0][1] = b.x; n.hi[0][D - 1] = b.y;
    n.lo[1][0] = b.z; n.lo[1][1] = b.w; n.lo[1][D - 1] = c.x;
    n.hi[1][0] = c.y; n.hi[1][1] = c.z; n.hi[1][D - 1] = c.w;
    n.code[0] = __float_as_int(d.x);
    n.code[1] = __float_as_int(d.y);
    n.rad[0] = d.z;
    n.rad[1] = d.w;
  } else {
    const float4 a = N[3 * i], b = N[3 * i + 1], c = N[3 * i + 2];
    n.lo[0][0] = a.x; n.lo[0][1] = a.y; n.hi[0][0] = a.z; n.hi[0][1] = a.w;
    n.lo[1][0] = b.x; n.lo[1][1] = b.y; n.hi[1][0] = b.z; n.hi[1][1] = b.w;
    n.code[0] = __float_as_int(c.x);
    n.code[1] = __float_as_int(c.y);
    n.rad[0] = c.z;
    n.rad[1] = c.w;
  }
  return n;
}

// LDS copies are read through a pointer typed for LDS, so that the loads
// are LDS reads rather than flat loads (which a choice between an LDS and a
// global pointer would give); the words follow the layout above
typedef const __attribute__((address_space(3))) float* LdsF;

template <int D>
__device__ inline NodePair<D> load_node_lds(LdsF N, int i) {
  NodePair<D> n;
  const LdsF p = N + (D == 3 ? 16 : 12) * i;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    n.lo[0][k] = p[k];
    n.hi[0][k] = p[D + k];
    n.lo[1][k] = p[2 * D + k];
    n.hi[1][k] = p[3 * D + k];
  }
  n.code[0] = __float_as_int(p[4 * D]);
  n.code[1] = __float_as_int(p[4 * D + 1]);
  n.rad[0] = p[4 * D + 2];
  n.rad[1] = p[4 * D + 3];
  return n;
}

// Whether the persistent kernels keep the top tree levels in LDS: measured
// 2 % faster on the star polygon (2D) and 3 % on a 327,680-triangle mesh,
// once the LDS copies are read through LDS-typed pointers (reading them
// through generic pointers gave flat loads and cost 1 % in 2D).
template <int D>
constexpr bool kTopInLds = true;

// a node of a tree whose first nt nodes may also sit in LDS (T)
template <int D>
__device__ inline NodePair<D> load_node_c(const float4* __restrict__ N, const float4* T, int nt, int i) {
  if (!kTopInLds<D>) return load_node<D>(N, i);
  if (i < nt) return load_node_lds<D>((LdsF)(const float*)T, i);
  return load_node<D>(N, i);
}

__device__ inline void decode_leaf(int32_t code, int& start, int& count) {
  const int32_t v = -code - 1;
  start = v >> 3;
  count = v & 7;
}

template <int D>
__device__ inline float box_d2(const float* lo, const float* hi, const Vec<D>& x) {
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float d = fmaxf(fmaxf(lo[k] - x[k], x[k] - hi[k]), 0.0f);
    s += d * d;
  }
  return s;
}

// slab test against [tmin, tmax]; the far bound is widened (Ize, "Robust BVH
// ray traversal", JCGT 2013: 2 gamma_3 for a correctly rounded inverse
// direction; here 1 + 10 u, since the inverse comes from the 1-ulp hardware
// reciprocal) so that FP32 rounding never rejects a box the ray touches.
template <int D>
__device__ inline bool ray_box(const float* lo, const float* hi, const Vec<D>& o,
                               const Vec<D>& inv, float tmin, float tmax, float& tin) {
  float t0 = tmin, t1 = tmax;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float ta = (lo[k] - o[k]) * inv[k];
    const float tb = (hi[k] - o[k]) * inv[k];
    t0 = fmaxf(t0, fminf(ta, tb));
    t1 = fminf(t1, fmaxf(ta, tb) * 1.0000006f);
  }
  tin = t0;
  return t0 <= t1;
}

// ---------------------------------------------------------------------------
// primitives
// ---------------------------------------------------------------------------
template <int D>
struct Prim {
  Vec<D> a, b, c;  // c unused in 2D
};

template <int D>
__device__ inline Prim<D> load_prim(const float4* __restrict__ P, int i);

template <>
__device__ inline Prim<3> load_prim<3>(const float4* __restrict__ P, int i) {
  const float4 a = P[3 * i], b = P[3 * i + 1], c = P[3 * i + 2];
  Prim<3> p;
  p.a[0] = a.x; p.a[1] = a.y; p.a[2] = a.z;
  p.b[0] = b.x; p.b[1] = b.y; p.b[2] = b.z;
  p.c[0] = c.x; p.c[1] = c.y; p.c[2] = c.z;
  return p;
}

template <>
__device__ inline Prim<2> load_prim<2>(const float4* __restrict__ P, int i) {
  const float4 a = P[i];
  Prim<2> p;
  p.a[0] = a.x; p.a[1] = a.y;
  p.b[0] = a.z; p.b[1] = a.w;
  p.c[0] = 0.0f; p.c[1] = 0.0f;
  return p;
}

// hardware reciprocal (1 ulp): enough for the closest-point and ray
// parameters, whose results are compared at 1e-5 of the scene size
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// closest point on segment [a, b]; w = barycentric weight of b
template <int D>
__device__ inline Vec<D> closest_segment(const Vec<D>& x, const Vec<D>& a, const Vec<D>& b,
                                         float& w) {
  const Vec<D> e = sub(b, a);
  // a degenerate segment (e = 0) gives dot = 0 and t = 0 without a branch,
  // so the leaf loops stay straight-line code and their loads issue together
  const float ee = fmaxf(dot(e, e), 1e-30f);
  float t = dot(sub(x, a), e) * rcp(ee);
  t = fminf(fmaxf(t, 0.0f), 1.0f);
  w = t;
  return axpy(a, t, e);
}

// closest point on triangle (a, b, c) by Voronoi-region classification
// (Ericson, Real-Time Collision Detection, Sec. 5.1.5); (wb, wc) are the
// barycentric weights of b and c.
__device__ inline Vec<3> closest_triangle(const Vec<3>& p, const Vec<3>& a, const Vec<3>& b,
                                          const Vec<3>& c, float& wb, float& wc) {
  const Vec<3> ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
  const float d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.0f && d2 <= 0.0f) { wb = 0; wc = 0; return a; }
  const Vec<3> bp = sub(p, b);
  const float d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0f && d4 <= d3) { wb = 1; wc = 0; return b; }
  const float vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {
    const float v = d1 * rcp(d1 - d3);
    wb = v; wc = 0;
    return axpy(a, v, ab);
  }
  const Vec<3> cp = sub(p, c);
  const float d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0f && d5 <= d6) { wb = 0; wc = 1; return c; }
  const float vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {
    const float w = d2 * rcp(d2 - d6);
    wb = 0; wc = w;
    return axpy(a, w, ac);
  }
  const float va = d3 * d6 - d5 * d4;
  if (va <= 0.0f && (d4 - d3) >= 0.0f && (d5 - d6) >= 0.0f) {
    const float w = (d4 - d3) * rcp((d4 - d3) + (d5 - d6));
    wb = 1.0f - w; wc = w;
    return axpy(b, w, sub(c, b));
  }
  const float den = rcp(va + vb + vc);
  const float v = vb * den, w = vc * den;
  wb = v; wc = w;
  return axpy(axpy(a, v, ab), w, ac);
}

template <int D>
__device__ inline Vec<D> closest_prim(const Vec<D>& x, const Prim<D>& P, float& wb, float& wc);
template <>
__device__ inline Vec<3> closest_prim<3>(const Vec<3>& x, const Prim<3>& P, float& wb, float& wc) {
  return closest_triangle(x, P.a, P.b, P.c, wb, wc);
}
template <>
__device__ inline Vec<2> closest_prim<2>(const Vec<2>& x, const Prim<2>& P, float& wb, float& wc) {
  wc = 0.0f;
  return closest_segment(x, P.a, P.b, wb);
}

// Watertight ray/triangle test (Woop, Benthin and Wald, JCGT 2013): the
// vertices are sheared into a ray-aligned frame and the three 2D edge
// functions are evaluated without FMA contraction, so that an edge shared
// by two triangles yields exactly opposite values and no ray slips through.
// Returns t (in units of |dir|, negative for a crossing behind the origin) or
// -kInf for no crossing of the ray's line.  `leaving`: the ray crosses from
// the side the outward normal (b - a) x (c - a) points away from to the side
// it points into.  The sheared determinant U + V + W equals
// -((b - a) x (c - a)) . dir / |dir_kz| (the shear has determinant 1 and the
// axis order keeps the orientation, swapped exactly when dir_kz < 0), so
// leaving is det < 0.  `near`: the origin lies on the inner side of the
// primitive's plane, or outside it by less than `behind` (compared in
// squares, with the origin-relative corners already at hand).
// component k of a 3-vector without dynamic register indexing
__device__ inline float pick3(const Vec<3>& v, int k) {
  return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]);
}

#pragma clang fp contract(off)
__device__ inline float ray_triangle_wt(const Vec<3>& o, const Vec<3>& dir, int kx, int ky, int kz,
                                        float Sx, float Sy, float Sz, const Prim<3>& P, float behind,
                                        bool& leaving, bool& near) {
  const Vec<3> A = sub(P.a, o), B = sub(P.b, o), C = sub(P.c, o);
  {
    // (o - a) . N with N = (b - a) x (c - a): positive outside
    const Vec<3> e1 = sub(B, A), e2 = sub(C, A);
    Vec<3> N;
    N[0] = e1[1] * e2[2] - e1[2] * e2[1];
    N[1] = e1[2] * e2[0] - e1[0] * e2[2];
    N[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const float g = -dot(A, N);
    near = (g <= 0.0f) | (g * g < behind * behind * dot(N, N));
  }
  const float Az0 = pick3(A, kz), Bz0 = pick3(B, kz), Cz0 = pick3(C, kz);
  const float Ax = pick3(A, kx) - Sx * Az0, Ay = pick3(A, ky) - Sy * Az0;
  const float Bx = pick3(B, kx) - Sx * Bz0, By = pick3(B, ky) - Sy * Bz0;
  const float Cx = pick3(C, kx) - Sx * Cz0, Cy = pick3(C, ky) - Sy * Cz0;
  const float U = Cx * By - Cy * Bx;
  const float V = Ax * Cy - Ay * Cx;
  const float W = Bx * Ay - By * Ax;
  const float det = U + V + W;
  const float T = U * (Sz * Az0) + V * (Sz * Bz0) + W * (Sz * Cz0);
  // straight-line: mixed edge signs or a zero determinant reject (det = 0
  // makes the quotient inf or NaN, which the select discards)
  const bool miss = (((U < 0.0f) | (V < 0.0f) | (W < 0.0f)) & ((U > 0.0f) | (V > 0.0f) | (W > 0.0f))) |
                    (det == 0.0f);
  const float t = T * rcp(det);
  leaving = det < 0.0f;
  return miss ? -kInf : t;
}

// 2D counterpart: the segment is crossed when its endpoints lie on opposite
// sides of (or on) the ray's line, with each endpoint's side computed by the
// same expression wherever it appears.  den = sa - sb = -dir . n for the
// outward normal n = (b_y - a_y, a_x - b_x), so leaving is den < 0; `near`
// as in 3D.
__device__ inline float ray_segment_wt(const Vec<2>& o, const Vec<2>& dir, const Prim<2>& P, float behind,
                                       bool& leaving, bool& near) {
  const float ax = P.a[0] - o[0], ay = P.a[1] - o[1];
  const float bx = P.b[0] - o[0], by = P.b[1] - o[1];
  const float sa = dir[0] * ay - dir[1] * ax;
  const float sb = dir[0] * by - dir[1] * bx;
  const float den = sa - sb;
  // straight-line: both endpoints strictly on one side, or the segment on
  // the ray's line (den = 0: grazing, no crossing), reject
  const bool miss = ((sa > 0.0f) & (sb > 0.0f)) | ((sa < 0.0f) & (sb < 0.0f)) | (den == 0.0f);
  const float lam = sa * rcp(den);
  const float ex = bx - ax, ey = by - ay;
  const float qx = ax + lam * ex, qy = ay + lam * ey;
  const float t = (qx * dir[0] + qy * dir[1]) * rcp(dir[0] * dir[0] + dir[1] * dir[1]);
  leaving = den < 0.0f;
  // (o - a) . N = t den for N = (b_y - a_y, a_x - b_x) (o + t dir lies on
  // the segment's line); |N| is the segment's length
  const float g = t * den;
  near = (g <= 0.0f) | (g * g < behind * behind * (ex * ex + ey * ey));
  return miss ? -kInf : t;
}
#pragma clang fp contract(on)

template <int D>
struct RayCtx {
  Vec<D> o, d, inv;
  int kx, ky, kz;
  float Sx, Sy, Sz;
};

template <int D>
__device__ inline RayCtx<D> make_ray(const Vec<D>& o, const Vec<D>& d) {
  RayCtx<D> R;
  R.o = o;
  R.d = d;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float dk = fabsf(d[k]) < 1e-30f ? copysignf(1e-30f, d[k]) : d[k];
    R.inv[k] = rcp(dk);
  }
  R.kx = R.ky = R.kz = 0;
  R.Sx = R.Sy = R.Sz = 0.0f;
  if (D == 3) {
    int kz = 0;
    float m = fabsf(d[0]);
    if (fabsf(d[1]) > m) { kz = 1; m = fabsf(d[1]); }
    if (fabsf(d[2]) > m) kz = 2;
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    Vec<3> d3;
    d3[0] = d[0]; d3[1] = d[1]; d3[2] = d[D - 1];
    const float dz = pick3(d3, kz);
    if (dz < 0.0f) { const int t = kx; kx = ky; ky = t; }
    R.kx = kx; R.ky = ky; R.kz = kz;
    // one reciprocal for the shear: every triangle of the query sees the same
    // Sx, Sy, Sz, which is all the watertight test needs
    R.Sz = rcp(dz);
    R.Sx = pick3(d3, kx) * R.Sz;
    R.Sy = pick3(d3, ky) * R.Sz;
  }
  return R;
}

template <int D>
__device__ inline float ray_prim(const RayCtx<D>& R, const Prim<D>& P, float behind, bool& leaving, bool& near);
template <>
__device__ inline float ray_prim<3>(const RayCtx<3>& R, const Prim<3>& P, float behind, bool& leaving,
                                    bool& near) {
  return ray_triangle_wt(R.o, R.d, R.kx, R.ky, R.kz, R.Sx, R.Sy, R.Sz, P, behind, leaving, near);
}
template <>
__device__ inline float ray_prim<2>(const RayCtx<2>& R, const Prim<2>& P, float behind, bool& leaving,
                                    bool& near) {
  return ray_segment_wt(R.o, R.d, P, behind, leaving, near);
}

// ---------------------------------------------------------------------------
// boundary data (Sec. 3.2)
// ---------------------------------------------------------------------------
template <int D>
__device__ inline float fn_value(const FnDev& F, const Vec<D>& x) {
  const float* c = F.c;
  switch (F.kind) {
    case 1: return c[0];
    case 2:
      if (D == 2)
        return c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[0] * x[0] + c[4] * x[1] * x[1] +
               c[5] * x[0] * x[1];
      return c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[D - 1] + c[4] * x[0] * x[0] +
             c[5] * x[1] * x[1] + c[6] * x[D - 1] * x[D - 1] + c[7] * x[0] * x[1] +
             c[8] * x[1] * x[D - 1] + c[9] * x[D - 1] * x[0];
    case 3: return c[0] * expf(c[1] * x[0]) * cosf(c[1] * x[1]);
    case 5: return c[0] * expf(c[1] * x[0] + c[2] * x[1] + (D == 3 ? c[3] * x[D - 1] : 0.0f));
    default: return 0.0f;
  }
}

template <int D>
__device__ inline Vec<D> fn_grad(const FnDev& F, const Vec<D>& x) {
  const float* c = F.c;
  Vec<D> g;
#pragma unroll
  for (int k = 0; k < D; ++k) g[k] = 0.0f;
  if (F.kind == 2) {
    if (D == 2) {
      g[0] = c[1] + 2.0f * c[3] * x[0] + c[5] * x[1];
      g[1] = c[2] + 2.0f * c[4] * x[1] + c[5] * x[0];
    } else {
      g[0] = c[1] + 2.0f * c[4] * x[0] + c[7] * x[1] + c[9] * x[D - 1];
      g[1] = c[2] + 2.0f * c[5] * x[1] + c[7] * x[0] + c[8] * x[D - 1];
      g[D - 1] = c[3] + 2.0f * c[6] * x[D - 1] + c[8] * x[1] + c[9] * x[0];
    }
  } else if (F.kind == 3) {
    const float e = c[0] * c[1] * expf(c[1] * x[0]);
    float s, co;
    sincosf(c[1] * x[1], &s, &co);
    g[0] = e * co;
    g[1] = -e * s;
  } else if (F.kind == 5) {
    const float e = fn_value<D>(F, x);
#pragma unroll
    for (int k = 0; k < D; ++k) g[k] = c[1 + k] * e;
  }
  return g;
}

template <int D>
__device__ inline Vec<D> prim_normal(const Prim<D>& P);
template <>
__device__ inline Vec<3> prim_normal<3>(const Prim<3>& P) {
  const Vec<3> e1 = sub(P.b, P.a), e2 = sub(P.c, P.a);
  Vec<3> n;
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const float s = rsqrtf(dot(n, n));
  n[0] *= s; n[1] *= s; n[2] *= s;
  return n;
}
template <>
__device__ inline Vec<2> prim_normal<2>(const Prim<2>& P) {
  Vec<2> n;
  n[0] = P.b[1] - P.a[1];
  n[1] = -(P.b[0] - P.a[0]);
  const float s = rsqrtf(dot(n, n));
  n[0] *= s; n[1] *= s;
  return n;
}

// value of a boundary field on primitive `orig` (original id) at point q
// with barycentric weights (wb, wc) of corners b and c; a normal derivative
// is taken along sgn * (the primitive's normal): sgn = -1 on the "-" side
// of a double-sided primitive
template <int D>
__device__ inline float boundary_value(const FnDev& F, int orig, const Vec<D>& q, float wb,
                                       float wc, const Prim<D>& P, float sgn = 1.0f) {
  if (F.kind == 4) {
    const float* pc = F.pc + (int64_t)orig * D;
    if (D == 2) return (1.0f - wb) * pc[0] + wb * pc[1];
    return (1.0f - wb - wc) * pc[0] + wb * pc[1] + wc * pc[D - 1];
  }
  if (F.as_nd) return sgn * dot(fn_grad<D>(F, q), prim_normal<D>(P));
  return fn_value<D>(F, q);
}

// ---------------------------------------------------------------------------
// Q.2: closest silhouette point (Sec. 5.1; Algorithms 2-4)
// ---------------------------------------------------------------------------
struct ConeF {
  float ax[3];
  float cs, sn;
};

// the two child cones of node i, from any address space
template <int D, class Ptr>
__device__ inline void load_cones_from(Ptr C, int i, ConeF c[2]) {
  if constexpr (D == 3) {
    const float4 a = C[3 * i], b = C[3 * i + 1], d = C[3 * i + 2];
    c[0].ax[0] = a.x; c[0].ax[1] = a.y; c[0].ax[2] = a.z; c[0].cs = a.w; c[0].sn = b.x;
    c[1].ax[0] = b.y; c[1].ax[1] = b.z; c[1].ax[2] = b.w; c[1].cs = d.x; c[1].sn = d.y;
  } else {
    const float4 a = C[2 * i], b = C[2 * i + 1];
    c[0].ax[0] = a.x; c[0].ax[1] = a.y; c[0].ax[2] = 0.0f; c[0].cs = a.z; c[0].sn = a.w;
    c[1].ax[0] = b.x; c[1].ax[1] = b.y; c[1].ax[2] = 0.0f; c[1].cs = b.z; c[1].sn = b.w;
  }
}
// the same words from an LDS copy: 3D (axis0, cos0, sin0, axis1, cos1, sin1,
// 2 unused), 2D (axis0, cos0, sin0, axis1, cos1, sin1)
template <int D>
__device__ inline void load_cones_lds(LdsF C, int i, ConeF c[2]) {
  const LdsF p = C + (D == 3 ? 12 : 8) * i;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const LdsF q = p + j * (D + 2);
#pragma unroll
    for (int k = 0; k < 3; ++k) c[j].ax[k] = k < D ? q[k] : 0.0f;
    c[j].cs = q[D];
    c[j].sn = q[D + 1];
  }
}

// a cone axis from its octahedral words (two signed 16-bit lattice
// coordinates on [-1, 1]^2); the builder widens each cone by the encoding's
// error plus a margin for this FP32 decoding
__device__ inline void oct_axis(uint32_t w, float ax[3]) {
  float p = (float)(int16_t)(w & 0xffffu) * (1.0f / 32767.0f);
  float r = (float)(int16_t)(w >> 16) * (1.0f / 32767.0f);
  const float z = 1.0f - fabsf(p) - fabsf(r);
  if (z < 0.0f) {
    const float tp = (1.0f - fabsf(r)) * copysignf(1.0f, p);
    const float tr = (1.0f - fabsf(p)) * copysignf(1.0f, r);
    p = tp;
    r = tr;
  }
  const float il = rsqrtf(p * p + r * r + z * z);
  ax[0] = p * il;
  ax[1] = r * il;
  ax[2] = z * il;
}

// four (distance, code, slot) triples in ascending distance (a sorting
// network of five compare-exchanges, without branches)
__device__ inline void sort4(float d[4], int32_t c[4], int s[4]) {
  auto cx = [&](int a, int b) {
    const bool sw = d[b] < d[a];
    const float td = d[a];
    const int32_t tc = c[a];
    const int ts = s[a];
    d[a] = sw ? d[b] : td;
    d[b] = sw ? td : d[b];
    c[a] = sw ? c[b] : tc;
    c[b] = sw ? tc : c[b];
    s[a] = sw ? s[b] : ts;
    s[b] = sw ? ts : s[b];
  };
  cx(0, 1);
  cx(2, 3);
  cx(0, 2);
  cx(1, 3);
  cx(1, 2);
}

// child i's box from a 4-wide record: 8-bit lattice indices (bytes 6i to
// 6i + 5 of the words qb) on the node's lattice o + q s, with the fused
// multiply-add the builder checks its boxes with
__device__ inline void lattice_box(const uint32_t qb[6], const float s[3], const float o[3], int i,
                                   float lo[3], float hi[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int bl = 6 * i + k, bh = 6 * i + 3 + k;
    lo[k] = __builtin_fmaf((float)((qb[bl >> 2] >> (8 * (bl & 3))) & 255u), s[k], o[k]);
    hi[k] = __builtin_fmaf((float)((qb[bh >> 2] >> (8 * (bh & 3))) & 255u), s[k], o[k]);
  }
}

// The end of a 4-wide node visit: the admissible children (distance below
// kInf) sorted nearest first into ch, their count n, and the revisit entry
// of `item` for ch[1, n).
__device__ inline void finish4(float dk[4], int32_t cc[4], int sl[4], int32_t item, int32_t ch[4], int& n,
                               int32_t& rev) {
  n = (dk[0] < kInf) + (dk[1] < kInf) + (dk[2] < kInf) + (dk[3] < kInf);
  sort4(dk, cc, sl);
  int rest = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ch[j] = cc[j];
    if (j >= 1 && j < n) rest |= 1 << sl[j];
  }
  rev = kRevisitFlag | (rest << kRevisitShift) | (item & ((15 << kHeightShift) | kEntryNode));
}

// Conservative test whether a box may hold a silhouette as seen from x: do
// the normal cone and the view cone of the box's bounding sphere contain a
// pair of orthogonal directions?  Written with cosines and sines instead of
// arccos / arcsin: the cones (half-angles t_n, t_v, axes at angle phi) hold
// such a pair iff t_n + t_v >= pi/2 or |cos phi| <= sin(t_n + t_v).  R is the
// bounding sphere's radius about the box centre, stored with the node by the
// builder (padded: its square carries a 1e-4 margin, rounded up).
template <int D>
__device__ inline bool has_silhouette(const float* lo, const float* hi, float R, const ConeF& cn,
                                      const Vec<D>& x) {
  // straight-line form (every case evaluated, then combined): a full cone,
  // x inside the bounding sphere (where il may be inf and the rest NaN, which
  // the first two terms override), the summed half-angle reaching pi/2, or
  // the axes' angle within the summed half-angle of pi/2
  float l2 = 0.0f, cphi = 0.0f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float a = 0.5f * (lo[k] + hi[k]) - x[k];
    l2 += a * a;
    cphi += cn.ax[k] * a;
  }
  const float R2 = R * R;
  const float il = rsqrtf(l2);
  cphi *= il;
  const float sv = R * il;
  const float cv = sqrtf(fmaxf(0.0f, 1.0f - sv * sv));
  const float csum = cn.cs * cv - cn.sn * sv;
  const float ssum = cn.sn * cv + cn.cs * sv;
  return (cn.cs <= 0.0f) | (l2 <= R2) | (csum <= 0.0f) | (fabsf(cphi) <= ssum + 1e-5f);
}

// silhouette element (3D: an edge a-b, 2D: a vertex a) with the normals of
// its two adjacent Neumann primitives
template <int D>
struct Element {
  Vec<D> a, b, n0, n1;
};

template <int D>
__device__ inline Element<D> load_element(const SceneDev& S, int i) {
  Element<D> e;
  if (D == 3) {
    const float4 A = S.se[3 * i], B = S.se[3 * i + 1], N = S.se[3 * i + 2];
    e.a[0] = A.x; e.a[1] = A.y; e.a[D - 1] = A.z;
    e.b[0] = B.x; e.b[1] = B.y; e.b[D - 1] = B.z;
    e.n0[0] = A.w; e.n0[1] = B.w; e.n0[D - 1] = N.x;
    e.n1[0] = N.y; e.n1[1] = N.z; e.n1[D - 1] = N.w;
  } else {
    const float4 A = S.se[2 * i], B = S.se[2 * i + 1];
    e.a[0] = A.x; e.a[1] = A.y;
    e.b = e.a;
    e.n0[0] = A.z; e.n0[1] = A.w;
    e.n1[0] = B.x; e.n1[1] = B.y;
  }
  return e;
}

// silhouette test of an element from x (the normals face x from opposite
// sides, Eq. SilhouetteDefinition) and its squared distance
template <int D>
__device__ inline bool element_silhouette(const Element<D>& e, const Vec<D>& x, float& dd) {
  Vec<D> p = e.a;
  if (D == 3) {
    float w;
    p = closest_segment<D>(x, e.a, e.b, w);
  }
  const Vec<D> v = sub(p, x);
  dd = dot(v, v);
  return dot(v, e.n0) * dot(v, e.n1) <= 0.0f;
}

template <int D>
__device__ inline bool silhouette_element(const SceneDev& S, int i, const Vec<D>& x, float& dd) {
  return element_silhouette<D>(load_element<D>(S, i), x, dd);
}

// ---------------------------------------------------------------------------
// Query results as keys
// ---------------------------------------------------------------------------
// Q.1 (closest Dirichlet point), Q.2 (closest silhouette point) and Q.3
// (closest Neumann hit) each return the lexicographic minimum of
// (value, slot) over the primitives they accept, packed as
// value bits << 32 | slot; the values are non-negative floats, whose bits
// order like the values.  Trees are pruned against the running minimum
// widened by kPrune, so a primitive whose computed value ties or nearly ties
// the minimum is always examined.  The result therefore does not depend on
// the order in which nodes are visited: one query may be split over several
// lanes (the cooperative traversal below) and every launch form returns the
// same bits.
typedef unsigned long long Key;
constexpr Key kNoKey = ~0ull;
constexpr float kPrune = 1.0f + 1.0f / 4096.0f;

__device__ inline Key make_key(float v, int slot) {
  return ((Key)__float_as_uint(v) << 32) | (uint32_t)slot;
}
__device__ inline float key_value(Key k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ inline int key_slot(Key k) { return (uint32_t)k == 0xffffffffu ? -1 : (int)(uint32_t)k; }
__device__ inline Key key_min(Key a, Key b) { return b < a ? b : a; }

// children of a node in visiting order: the nearer (or earlier-entered)
// child first; a child is visited when its flag is set
__device__ inline void order_children(const int32_t code[2], bool a0, bool a1, bool swap, int32_t& cN,
                                      int32_t& cF, bool& vN, bool& vF) {
  cN = swap ? code[1] : code[0];
  cF = swap ? code[0] : code[1];
  vN = swap ? a1 : a0;
  vF = swap ? a0 : a1;
}

// Q.1: closest point on the Dirichlet boundary; value = squared distance.
template <int D, bool CNT>
struct Q1Query {
  static constexpr bool kAny = false;
  static constexpr int kDim = D;
  static constexpr int kWidth = D == 3 ? 4 : 2;   // children per tree node
  __device__ static int32_t root(const SceneDev& S) { return D == 3 ? S.dn_root : 0; }
  static constexpr int kWaveIter = kWaveQ1Iter, kWaveLeaf = kWaveQ1Leaf;
  Vec<D> x;
  // 3D: one 4-wide node (exact FP32 child boxes), or a revisit entry; as
  // Q2Query::node4
  __device__ void node4(const SceneDev& S, int32_t item, Key& key, const Key* shared, int32_t ch[4],
                        int& n, int32_t& rev, int& h, Cnt& cn) const {
    static_assert(D == 3, "4-wide Dirichlet nodes are 3D");
    const int node = item & kEntryNode;
    const int mask = (item & kRevisitFlag) ? (item >> kRevisitShift) & 15 : 15;
    h = ((item >> kHeightShift) & 15) + 1;
    float w[28];
    if (kTopInLds<D> && node < S.ctD) {
      const LdsF p = (LdsF)(const float*)S.tdn + 4 * kSRec * node;
#pragma unroll
      for (int j = 0; j < 28; ++j) w[j] = p[j];
    } else {
      const float4* __restrict__ p = S.dn + kSRec * node;
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const float4 v = p[j];
        w[4 * j] = v.x;
        w[4 * j + 1] = v.y;
        w[4 * j + 2] = v.z;
        w[4 * j + 3] = v.w;
      }
    }
    if (shared) key = key_min(key, *shared);   // after the loads are issued
    if (CNT) cn.add(kCntQ1Node);
    const float bound = key_value(key) * kPrune;
    float dk[4];
    int32_t cc[4];
    int sl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float d = box_d2<3>(w + 6 * i, w + 6 * i + 3, x);
      cc[i] = __float_as_int(w[24 + i]);
      const bool a = (((mask >> i) & 1) != 0) & (cc[i] != kEmptyCode) & (d <= bound);
      dk[i] = a ? d : kInf;
      sl[i] = i;
    }
    finish4(dk, cc, sl, item, ch, n, rev);
  }
  // 2D: binary nodes
  __device__ void node(const SceneDev& S, int item, Key& key, const Key* shared, int32_t& cN,
                       int32_t& cF, bool& vN, bool& vF, Cnt& cn) const {
    static_assert(D == 2, "the 3D Dirichlet tree is 4-wide (node4)");
    const NodePair<D> nd = load_node_c<D>(S.dn, S.tdn, S.ctD, item);
    if (shared) key = key_min(key, *shared);   // after the loads are issued
    if (CNT) cn.add(kCntQ1Node);
    // both boxes are tested unconditionally and empty children masked
    // afterwards: a conditional test would let the compiler sink the box
    // loads behind the code load, costing a second memory round trip
    const float d0 = box_d2<D>(nd.lo[0], nd.hi[0], x), d1 = box_d2<D>(nd.lo[1], nd.hi[1], x);
    const float bound = key_value(key) * kPrune;
    const bool a0 = (nd.code[0] != kEmptyCode) & (d0 <= bound);
    const bool a1 = (nd.code[1] != kEmptyCode) & (d1 <= bound);
    order_children(nd.code, a0, a1, d1 < d0, cN, cF, vN, vF);
  }
  // returns whether the leaf lowered the key (after the refresh)
  __device__ bool leaf(const SceneDev& S, int32_t item, Key& key, const Key* shared, Cnt& cn) const {
    int s0, cnt;
    decode_leaf(item, s0, cnt);
    if (CNT) cn.add(kCntQ1Prim, cnt);
    // primitive arrays carry kLeafMax - 1 padding slots, so all slots load
    // in bounds; all loads are issued before the first test
    Prim<D> Pk[kLeafMax];
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) Pk[k] = load_prim<D>(S.dp, s0 + k);
    if (shared) key = key_min(key, *shared);
    const Key k0 = key;
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) {
      float wb, wc;
      const Vec<D> dv = sub(closest_prim<D>(x, Pk[k], wb, wc), x);
      key = key_min(key, k < cnt ? make_key(dot(dv, dv), s0 + k) : kNoKey);
    }
    return key < k0;
  }
  __device__ void from(const Q1Query& own, int src) {
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = __shfl(own.x[k], src);
  }
};

// Q.2: closest point on the visibility silhouette of the Neumann boundary
// (Sec. 5.1, Algorithms 2-4); value = squared distance.  A node's two cones
// are read with it (one memory round trip per visit); a child that contains
// the query point skips the cone test.
template <int D, bool CNT>
struct Q2Query {
  static constexpr bool kAny = false;
  static constexpr int kDim = D;
  static constexpr int kWidth = D == 3 ? 4 : 2;   // children per tree node
  __device__ static int32_t root(const SceneDev& S) { return D == 3 ? S.sil4_root : 0; }
  static constexpr int kWaveIter = kWaveQ2Iter, kWaveLeaf = kWaveQ2Leaf;
  Vec<D> x;
  // 2D: binary nodes, node and cone words from separate arrays
  __device__ void node(const SceneDev& S, int item, Key& key, const Key* shared, int32_t& cN,
                       int32_t& cF, bool& vN, bool& vF, Cnt& cn) const {
    static_assert(D == 2, "the 3D silhouette tree is 4-wide (node4)");
    NodePair<D> nd;
    ConeF cones[2];
    if (kTopInLds<D> && item < S.ctS) {
      nd = load_node_lds<D>((LdsF)(const float*)S.tsn, item);
      load_cones_lds<D>((LdsF)(const float*)S.tsc, item, cones);
    } else {
      nd = load_node_from<D>(S.sn, item);
      load_cones_from<D>(S.sc, item, cones);
    }
    if (shared) key = key_min(key, *shared);
    if (CNT) { cn.add(kCntQ2Node); cn.add(kCntQ2Cone); }
    const float d0 = box_d2<D>(nd.lo[0], nd.hi[0], x), d1 = box_d2<D>(nd.lo[1], nd.hi[1], x);
    const bool c0 = has_silhouette<D>(nd.lo[0], nd.hi[0], nd.rad[0], cones[0], x);
    const bool c1 = has_silhouette<D>(nd.lo[1], nd.hi[1], nd.rad[1], cones[1], x);
    const float bound = key_value(key) * kPrune;
    // bitwise, not short-circuit: no branch, so the cone loads stay with
    // the node loads
    const bool a0 = (nd.code[0] != kEmptyCode) & (d0 <= bound) & ((d0 <= 0.0f) | c0);
    const bool a1 = (nd.code[1] != kEmptyCode) & (d1 <= bound) & ((d1 <= 0.0f) | c1);
    order_children(nd.code, a0, a1, d1 < d0, cN, cF, vN, vF);
  }
  // 3D: one 4-wide node, or a revisit entry (the node and the children
  // still to search); the admissible children nearest first in ch[0, n),
  // in rev an entry that revisits this node for ch[1, n), in h the height
  // of the node's subtree
  __device__ void node4(const SceneDev& S, int32_t item, Key& key, const Key* shared, int32_t ch[4],
                        int& n, int32_t& rev, int& h, Cnt& cn) const {
    static_assert(D == 3, "4-wide silhouette nodes are 3D");
    const int node = item & kEntryNode;
    const int mask = (item & kRevisitFlag) ? (item >> kRevisitShift) & 15 : 15;
    h = ((item >> kHeightShift) & 15) + 1;
    float4 r[kSRec];
    if (kTopInLds<D> && node < S.ctS) {
      const LdsF p = (LdsF)(const float*)S.tsn + 4 * kSRec * node;
#pragma unroll
      for (int j = 0; j < kSRec; ++j) r[j] = make_float4(p[4 * j], p[4 * j + 1], p[4 * j + 2], p[4 * j + 3]);
    } else {
      const float4* __restrict__ p = S.sn + kSRec * node;
#pragma unroll
      for (int j = 0; j < kSRec; ++j) r[j] = p[j];
    }
    if (shared) key = key_min(key, *shared);
    if (CNT) { cn.add(kCntQ2Node); cn.add(kCntQ2Cone); }
    const float bound = key_value(key) * kPrune;
    const float o[3] = {r[0].x, r[0].y, r[0].z}, s[3] = {r[0].w, r[1].x, r[1].y};
    const uint32_t qb[6] = {__float_as_uint(r[1].z), __float_as_uint(r[1].w), __float_as_uint(r[2].x),
                            __float_as_uint(r[2].y), __float_as_uint(r[2].z), __float_as_uint(r[2].w)};
    const int32_t code[4] = {__float_as_int(r[3].x), __float_as_int(r[3].y), __float_as_int(r[3].z),
                             __float_as_int(r[3].w)};
    const float rad[4] = {r[4].x, r[4].y, r[4].z, r[4].w};
    const uint32_t oc[4] = {__float_as_uint(r[5].x), __float_as_uint(r[5].y), __float_as_uint(r[5].z),
                            __float_as_uint(r[5].w)};
    const float cs[4] = {r[6].x, r[6].y, r[6].z, r[6].w};
    const float sn[4] = {r[7].x, r[7].y, r[7].z, r[7].w};
    float dk[4];
    int32_t cc[4];
    int sl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float lo[3], hi[3];
      lattice_box(qb, s, o, i, lo, hi);
      ConeF cone;
      oct_axis(oc[i], cone.ax);
      cone.cs = cs[i];
      cone.sn = sn[i];
      const float d = box_d2<3>(lo, hi, x);
      const bool c = has_silhouette<3>(lo, hi, rad[i], cone, x);
      const bool a = (((mask >> i) & 1) != 0) & (code[i] != kEmptyCode) & (d <= bound) & ((d <= 0.0f) | c);
      dk[i] = a ? d : kInf;
      cc[i] = code[i];
      sl[i] = i;
    }
    finish4(dk, cc, sl, item, ch, n, rev);
  }
  __device__ bool leaf(const SceneDev& S, int32_t item, Key& key, const Key* shared, Cnt& cn) const {
    int s0, cnt;
    decode_leaf(item, s0, cnt);
    if (CNT) cn.add(kCntQ2Elem, cnt);
    Element<D> E[kLeafMax];
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) E[k] = load_element<D>(S, s0 + k);
    if (shared) key = key_min(key, *shared);
    const Key k0 = key;
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) {
      float dd;
      const bool sil = element_silhouette<D>(E[k], x, dd);
      key = key_min(key, ((k < cnt) & sil) ? make_key(dd, s0 + k) : kNoKey);
    }
    return key < k0;
  }
  __device__ void from(const Q2Query& own, int src) {
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = __shfl(own.x[k], src);
  }
};

// Q.3: first Neumann crossing of o + t d with 0 < t <= tmax (closest hit;
// value = t, the key starts at (tmax, none)), or whether any crossing has
// 0 < t < tmax (ANY: occlusion; the key drops to 0 on a hit).  Slot `skip`
// is ignored.  The closest-hit query also takes a crossing at
// -kBehindReach * offset < t <= 0 through a one-sided primitive that the
// ray leaves, as a crossing at t = 0, when the origin lies outside the
// primitive's plane by less than behind = offset / 4: the origin then lies
// on that primitive up to FP32 rounding, possibly just outside it (a walk
// whose previous step ended within rounding of the boundary), and an
// outward ray from there must not pass through it.  The offset is the
// inward shift of on-boundary query origins; d is a unit vector for this
// query.
template <int D, bool ANY, bool CNT>
struct RayQuery {
  static constexpr bool kAny = ANY;
  static constexpr int kDim = D;
  static constexpr int kWidth = D == 3 ? 4 : 2;   // 3D: the Neumann tree's 4-wide copy
  __device__ static int32_t root(const SceneDev& S) { return D == 3 ? S.rn_root : 0; }
  static constexpr int kWaveIter = ANY ? kWaveVisIter : kWaveQ3Iter;
  static constexpr int kWaveLeaf = ANY ? kWaveVisLeaf : kWaveQ3Leaf;
  RayCtx<D> R;
  float tmax;
  int skip;
  // 3D: one 4-wide node (exact FP32 child boxes) or a revisit entry; the
  // children the ray meets, nearest entry first; as Q2Query::node4
  __device__ void node4(const SceneDev& S, int32_t item, Key& key, const Key* shared, int32_t ch[4],
                        int& n, int32_t& rev, int& h, Cnt& cn) const {
    static_assert(D == 3, "the 4-wide ray tree is 3D");
    const int node = item & kEntryNode;
    const int mask = (item & kRevisitFlag) ? (item >> kRevisitShift) & 15 : 15;
    h = ((item >> kHeightShift) & 15) + 1;
    float w[28];
    if (kTopInLds<D> && node < S.ctR) {
      const LdsF p = (LdsF)(const float*)S.trn + 4 * kSRec * node;
#pragma unroll
      for (int j = 0; j < 28; ++j) w[j] = p[j];
    } else {
      const float4* __restrict__ p = S.rn + kSRec * node;
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const float4 v = p[j];
        w[4 * j] = v.x;
        w[4 * j + 1] = v.y;
        w[4 * j + 2] = v.z;
        w[4 * j + 3] = v.w;
      }
    }
    if (shared) key = key_min(key, *shared);
    if (CNT) cn.add(ANY ? kCntVisNode : kCntQ3Node);
    const float tb = ANY ? tmax : key_value(key) * kPrune;
    const float ta = ANY ? 0.0f : -kBehindReach * S.offset;
    // an answered occlusion query visits nothing more
    const bool open = !ANY || key == kNoKey;
    float dk[4];
    int32_t cc[4];
    int sl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float t;
      const bool hit = ray_box<3>(w + 6 * i, w + 6 * i + 3, R.o, R.inv, ta, tb, t);
      cc[i] = __float_as_int(w[24 + i]);
      const bool a = (((mask >> i) & 1) != 0) & (cc[i] != kEmptyCode) & hit & open;
      dk[i] = a ? t : kInf;
      sl[i] = i;
    }
    finish4(dk, cc, sl, item, ch, n, rev);
  }
  // binary nodes (2D)
  __device__ void node(const SceneDev& S, int item, Key& key, const Key* shared, int32_t& cN,
                       int32_t& cF, bool& vN, bool& vF, Cnt& cn) const {
    static_assert(D == 2, "the 3D ray queries search the 4-wide tree (node4)");
    const NodePair<D> nd = load_node_c<D>(S.nn, S.tnn, S.ctN, item);
    if (shared) key = key_min(key, *shared);
    if (CNT) cn.add(ANY ? kCntVisNode : kCntQ3Node);
    const float tb = ANY ? tmax : key_value(key) * kPrune;
    const float ta = ANY ? 0.0f : -kBehindReach * S.offset;
    float t0, t1;
    const bool h0 = ray_box<D>(nd.lo[0], nd.hi[0], R.o, R.inv, ta, tb, t0);
    const bool h1 = ray_box<D>(nd.lo[1], nd.hi[1], R.o, R.inv, ta, tb, t1);
    // an answered occlusion query visits nothing more
    const bool open = !ANY || key == kNoKey;
    const bool a0 = (nd.code[0] != kEmptyCode) & h0 & open;
    const bool a1 = (nd.code[1] != kEmptyCode) & h1 & open;
    order_children(nd.code, a0, a1, a1 & (!a0 | (t1 < t0)), cN, cF, vN, vF);
  }
  __device__ bool leaf(const SceneDev& S, int32_t item, Key& key, const Key* shared, Cnt& cn) const {
    int s0, cnt;
    decode_leaf(item, s0, cnt);
    if (CNT) cn.add(ANY ? kCntVisPrim : kCntQ3Prim, cnt);
    Prim<D> Pk[kLeafMax];
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) Pk[k] = load_prim<D>(S.np, s0 + k);
    if (shared) key = key_min(key, *shared);
    const Key k0 = key;
    const float behind = 0.25f * S.offset, reach = -kBehindReach * S.offset;
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) {
      const int i = s0 + k;
      bool leaving, near;
      const float t = ray_prim<D>(R, Pk[k], behind, leaving, near);
      if (ANY) {
        const bool ok = (k < cnt) & (i != skip) & (t > 0.0f);
        key = (ok & (t < tmax)) ? 0ull : key;
      } else {
        // a crossing behind the origin counts (as t = 0) when the ray leaves
        // a one-sided primitive there and the origin lies beyond the
        // primitive's plane by less than `behind`, measured across the plane
        // (at grazing incidence a rounding-sized distance from the plane is
        // a long way back along the ray, hence the longer reach in t)
        const bool back = (t > reach) & near & leaving && (!S.ds || !S.nside[i]);
        const bool ok = (k < cnt) & (i != skip) & ((t > 0.0f) | back);
        key = key_min(key, ok ? make_key(fmaxf(t, 0.0f), i) : kNoKey);
      }
    }
    return key < k0;
  }
  __device__ void from(const RayQuery& own, int src) {
    Vec<D> o, d;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      o[k] = __shfl(own.R.o[k], src);
      d[k] = __shfl(own.R.d[k], src);
    }
    R = make_ray<D>(o, d);   // the owner's arithmetic, hence the owner's values
    tmax = __shfl(own.tmax, src);
    skip = __shfl(own.skip, src);
  }
};

// One lane, one query.  Flat traversal: each iteration holds one item -- a
// node (both children tested, the nearer taken next, the farther pushed) or
// a leaf (its primitives tested) -- and the next item comes from a select or
// a pop, so no lane waits on another lane's descent or pop.
template <class Qy, bool CNT>
__device__ Key traverse(const SceneDev& S, const Qy& q, Key key, int* stk, Cnt& cn) {
  int32_t item = Qy::root(S);
  int sp = 0;
  do {
    if (CNT) cn.wave(Qy::kWaveIter);
    int32_t next = kEmptyCode;
    if (item >= 0) {
      if constexpr (Qy::kWidth == 4) {
        int32_t ch[4], rev;
        int n, h;
        q.node4(S, item, key, nullptr, ch, n, rev, h, cn);
        if (n > 1) {
          if (sp + (n - 1) <= kStack<Qy::kDim> - h) {
#pragma unroll
            for (int j = 3; j >= 1; --j)
              if (j < n) stk[sp++ * kBlock] = ch[j];
          } else {
            stk[sp++ * kBlock] = rev;
          }
        }
        next = n > 0 ? ch[0] : kEmptyCode;
      } else {
        int32_t cN, cF;
        bool vN, vF;
        q.node(S, item, key, nullptr, cN, cF, vN, vF, cn);
        if (vN && vF) {
          stk[sp * kBlock] = cF;
          ++sp;
        }
        next = vN ? cN : (vF ? cF : kEmptyCode);
      }
    } else {
      if (CNT) cn.wave(Qy::kWaveLeaf);
      q.leaf(S, item, key, nullptr, cn);
      if (Qy::kAny && key != kNoKey) sp = 0;   // occluded: stop
    }
    if (next == kEmptyCode && sp > 0) {
      --sp;
      next = stk[sp * kBlock];
    }
    item = next;
  } while (item != kEmptyCode);
  return key;
}

// index into a ring of K stack entries for 0 <= i < 2K
template <int K>
__device__ inline int ring(int i) { return i >= K ? i - K : i; }

// Wave-cooperative traversal.  All lanes of the wave enter together; lanes
// with a query (`has`) start at the root, the others start idle.  A lane
// whose work is exhausted steals the bottom (shallowest, so largest) entry
// of another lane's stack together with that entry's query: the query's
// parameters come from its owner lane by cross-lane shuffles, and its running
// minimum lives in an LDS key that every lane working on the query lowers
// with atomicMin and re-reads before each item.  Stacks are rings of K
// entries: a lane's live entries [bot, sp) stay below K (a binary tree's
// search pushes at most one entry per level, and its depth is below K; see
// kRevisitFlag for the 4-wide tree); bot moves up as entries are stolen and
// both drop by K when bot reaches K, so indexes stay below 2K.  Because results
// do not depend on the visiting order (see Key), the result is the one-lane
// result, bit for bit; the gain is that no lane idles while another still
// has subtrees to search.
struct CoopLds {
  int* stk;    // the wave's 64 stack columns, stride kBlock
  Key* keys;   // 64 per wave: running result of each lane's own query
  int* vict;   // 64 per wave: lanes holding stack entries, by rank
  int steal;   // a steal round starts once at least this many lanes are idle
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class Qy, bool CNT>
__device__ Key coop_traverse(const SceneDev& S, const Qy& own, bool has, Key key0, const CoopLds& L,
                             Cnt& cn) {
  constexpr int K = kStack<Qy::kDim>;
  const int lane = __lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  int* const stk = L.stk + lane;
  L.keys[lane] = has ? key0 : kNoKey;
  wave_sync();
  const unsigned long long all = __ballot(true);
  Qy wk = own;            // parameters of the query this lane works on
  int wq = has ? lane : -1;
  int32_t item = has ? Qy::root(S) : kEmptyCode;
  int sp = 0, bot = 0;        // LDS ring entries [bot, sp)
  Key cur = has ? key0 : kNoKey;
  while (true) {
    if (CNT) cn.wave(Qy::kWaveIter);
    if (item != kEmptyCode) {
      // the node and leaf tests re-read the shared key once their own loads
      // are in flight
      const Key* shared = L.keys + wq;
      int32_t next = kEmptyCode;
      if (item >= 0) {
        if constexpr (Qy::kWidth == 4) {
          int32_t ch[4], rev;
          int n, h;
          wk.node4(S, item, cur, shared, ch, n, rev, h, cn);
          if (n > 1) {
            if (sp - bot + (n - 1) <= K - h) {
#pragma unroll
              for (int j = 3; j >= 1; --j)
                if (j < n) stk[ring<K>(sp++) * kBlock] = ch[j];
            } else {
              stk[ring<K>(sp++) * kBlock] = rev;
            }
          }
          next = n > 0 ? ch[0] : kEmptyCode;
        } else {
          int32_t cN, cF;
          bool vN, vF;
          wk.node(S, item, cur, shared, cN, cF, vN, vF, cn);
          if (vN && vF) {
            stk[ring<K>(sp) * kBlock] = cF;
            ++sp;
          }
          next = vN ? cN : (vF ? cF : kEmptyCode);
        }
      } else {
        if (CNT) cn.wave(Qy::kWaveLeaf);
        if (wk.leaf(S, item, cur, shared, cn)) atomicMin(L.keys + wq, cur);
      }
      if (Qy::kAny && cur != kNoKey) {   // the query is answered: drop the rest
        next = kEmptyCode;
        sp = bot;
      }
      if (next == kEmptyCode && sp != bot) {
        --sp;
        next = stk[ring<K>(sp) * kBlock];
      }
      item = next;
      if (item == kEmptyCode) {
        sp = 0;
        bot = 0;
        wq = -1;
      }
    }
    const unsigned long long idle = __ballot(item == kEmptyCode);
    if (idle == 0ull) continue;
    const unsigned long long rich = __ballot(sp != bot);
    if (rich == 0ull) {
      if (idle == all) break;
      continue;
    }
    // a steal round costs ~70 instructions and three LDS round trips: in 3D,
    // where node and leaf tests are heavier, it pays only once a quarter of
    // the wave is idle (measured: 16 idle lanes best in 3D with the 4-wide
    // trees, 32 with binary ones; 1 in 2D).  The 3D threshold is a solve
    // option for the autotuner; in 2D a run-time threshold measured 11 more
    // spilled registers, so 2D keeps 1.
    if (__popcll(idle) < (Qy::kDim == 2 ? 1 : L.steal)) continue;
    // the k-th idle lane takes the bottom entry of the k-th lane with entries
    const bool am_rich = (rich >> lane) & 1ull, am_idle = (idle >> lane) & 1ull;
    const int nr = __popcll(rich), ni = __popcll(idle);
    const int rr = __popcll(rich & below), ri = __popcll(idle & below);
    if (am_rich) L.vict[rr] = lane;
    wave_sync();
    const int v = (am_idle && ri < nr) ? L.vict[ri] : -1;
    const int src = v >= 0 ? v : lane;
    const int vbot = __shfl(bot, src);
    const int vwq = __shfl(wq, src);
    Qy got;
    got.from(own, v >= 0 ? vwq : lane);
    if (v >= 0) {
      item = L.stk[v + ring<K>(vbot) * kBlock];
      wq = vwq;
      wk = got;
      cur = kNoKey;
      sp = 0;
      bot = 0;
    }
    if (am_rich && rr < ni && ++bot == K) {
      bot = 0;
      sp -= K;
    }
    wave_sync();
  }
  wave_sync();
  return has ? L.keys[lane] : kNoKey;
}

template <class Qy, bool CNT, bool COOP>
__device__ inline Key run_query(const SceneDev& S, const Qy& q, bool has, Key key0, int* stk,
                                const CoopLds& L, Cnt& cn) {
  if (COOP) return coop_traverse<Qy, CNT>(S, q, has, key0, L, cn);
  return has ? traverse<Qy, CNT>(S, q, key0, stk, cn) : key0;
}

// ---------------------------------------------------------------------------
// Q.4: Neumann point sample (Algorithms 5-6): one random descent from the
// root, choosing among the children whose box meets B(x, r) with weights
// proportional to the free-space Green's function at the box centre
// (1 / distance, clamped below by the offset), then a primitive of the leaf
// that meets the ball in proportion to its measure, then a point uniformly
// on it.  pdf = (product of branch probabilities) / (leaf measure in ball).
// Uniforms come from Philox slots 1, 2, ... of the step.
// ---------------------------------------------------------------------------
template <int D, bool CNT>
__device__ int q4_sample(const SceneDev& S, const Vec<D>& x, float r, uint4 ctr, uint32_t k0,
                         uint32_t k1, Vec<D>& z, float& pdf, float& wb, float& wc, Cnt& cn) {
  pdf = 0.0f;
  if (S.nN == 0) return -1;
  const float r2 = r * r;
  ctr.w = 1;
  uint4 u = philox(ctr, k0, k1);
  const float u_leaf = u01(u.x), u_p0 = u01(u.y), u_p1 = u01(u.z);
  uint32_t pool[4] = {u.w, 0u, 0u, 0u};
  int avail = 1, used = 0;
  float pT = 1.0f;
  int node = 0;
  int32_t leaf = kEmptyCode;
  for (int level = 0; level < 64; ++level) {
    const NodePair<D> nd = load_node_c<D>(S.nn, S.tnn, S.ctN, node);
    if (CNT) { cn.add(kCntQ4Node); cn.wave(kWaveQ4Iter); }
    float w[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float c2 = 0.0f;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float a = 0.5f * (nd.lo[j][k] + nd.hi[j][k]) - x[k];
        c2 += a * a;
      }
      const bool meets = nd.code[j] != kEmptyCode && box_d2<D>(nd.lo[j], nd.hi[j], x) <= r2;
      w[j] = meets ? rsqrtf(fmaxf(c2, S.offset * S.offset)) : 0.0f;
    }
    const float tot = w[0] + w[1];
    if (!(tot > 0.0f)) return -1;
    if (used == avail) {
      ctr.w += 1;
      const uint4 q = philox(ctr, k0, k1);
      pool[0] = q.x; pool[1] = q.y; pool[2] = q.z; pool[3] = q.w;
      avail = 4;
      used = 0;
    }
    const float uu = u01(pool[used]);
    ++used;
    const float pl = w[0] * rcp(tot);
    int32_t c;
    if (uu < pl) { c = nd.code[0]; pT *= pl; }
    else { c = nd.code[1]; pT *= (1.0f - pl); }
    if (c < 0) { leaf = c; break; }
    node = c;
  }
  if (leaf == kEmptyCode) return -1;
  int s0, cnt;
  decode_leaf(leaf, s0, cnt);
  if (CNT) cn.add(kCntQ4Prim, cnt);
  // one pass over the leaf's slots (padded, so all load in bounds): the
  // measure of each primitive meeting the ball, then the pick by the
  // cumulative measure in slot order
  float m[kLeafMax];
  float total = 0.0f;
#pragma unroll
  for (int k = 0; k < kLeafMax; ++k) {
    const Prim<D> Q = load_prim<D>(S.np, s0 + k);
    const float ar = S.narea[s0 + k];
    float a, b;
    const Vec<D> p = closest_prim<D>(x, Q, a, b);
    const Vec<D> dv = sub(p, x);
    m[k] = (k < cnt && dot(dv, dv) <= r2) ? ar : 0.0f;
    total += m[k];
  }
  if (!(total > 0.0f)) return -1;
  const float target = u_leaf * total;
  float cum = 0.0f;
  int pick = -1;
  bool done = false;
#pragma unroll
  for (int k = 0; k < kLeafMax; ++k) {
    const bool in = m[k] > 0.0f && !done;
    pick = in ? s0 + k : pick;
    cum += in ? m[k] : 0.0f;
    done = done || (in && cum > target);
  }
  const Prim<D> P = load_prim<D>(S.np, pick);
  if (D == 2) {
    wb = u_p0;
    wc = 0.0f;
    z = axpy(P.a, u_p0, sub(P.b, P.a));
  } else {
    const float s = sqrtf(u_p0);
    wb = s * (1.0f - u_p1);
    wc = s * u_p1;
#pragma unroll
    for (int k = 0; k < D; ++k) z[k] = (1.0f - s) * P.a[k] + wb * P.b[k] + wc * P.c[k];
  }
  pdf = pT * rcp(total);
  return pick;
}

// ---------------------------------------------------------------------------
// ball kernels (App. A.1) and samplers (Sec. 4.4, 4.6)
// ---------------------------------------------------------------------------
template <int D>
__device__ inline float green_ball(float rho, float R) {
  if (D == 2) return logf(R * rcp(rho)) * (1.0f / (2.0f * kPi));
  return (rcp(rho) - rcp(R)) * (1.0f / (4.0f * kPi));
}
template <int D>
__device__ inline float green_ball_norm(float R) {
  return D == 2 ? R * R * 0.25f : R * R * (1.0f / 6.0f);
}

// ---- screened Poisson (App. A.2) ------------------------------------------
// Modified Bessel functions for the 2D kernels, exponentially scaled
// (ie_n = e^-x I_n(x), ke_n = e^x K_n(x)), by the polynomial approximations
// of Abramowitz and Stegun, Handbook of Mathematical Functions, 9.8.1-9.8.8
// (relative error below 1e-6).
__device__ inline float bessel_ie0(float x) {
  if (x <= 3.75f) {
    const float t = x * (1.0f / 3.75f), y = t * t;
    return (1.0f + y * (3.5156229f + y * (3.0899424f + y * (1.2067492f + y * (0.2659732f +
            y * (0.0360768f + y * 0.0045813f)))))) * expf(-x);
  }
  const float y = 3.75f / x;
  return (0.39894228f + y * (0.01328592f + y * (0.00225319f + y * (-0.00157565f + y * (0.00916281f +
          y * (-0.02057706f + y * (0.02635537f + y * (-0.01647633f + y * 0.00392377f)))))))) * rsqrtf(x);
}
__device__ inline float bessel_ie1(float x) {
  if (x <= 3.75f) {
    const float t = x * (1.0f / 3.75f), y = t * t;
    return x * (0.5f + y * (0.87890594f + y * (0.51498869f + y * (0.15084934f + y * (0.02658733f +
            y * (0.00301532f + y * 0.00032411f)))))) * expf(-x);
  }
  const float y = 3.75f / x;
  return (0.39894228f + y * (-0.03988024f + y * (-0.00362018f + y * (0.00163801f + y * (-0.01031555f +
          y * (0.02282967f + y * (-0.02895312f + y * (0.01787654f - y * 0.00420059f)))))))) * rsqrtf(x);
}
__device__ inline float bessel_ke0(float x) {
  if (x <= 2.0f) {
    const float y = 0.25f * x * x;
    const float k0 = -logf(0.5f * x) * bessel_ie0(x) * expf(x) +
                     (-0.57721566f + y * (0.42278420f + y * (0.23069756f + y * (0.03488590f +
                      y * (0.00262698f + y * (0.00010750f + y * 0.0000074f))))));
    return k0 * expf(x);
  }
  const float y = 2.0f / x;
  return (1.25331414f + y * (-0.07832358f + y * (0.02189568f + y * (-0.01062446f + y * (0.00587872f +
          y * (-0.00251540f + y * 0.00053208f)))))) * rsqrtf(x);
}
__device__ inline float bessel_ke1(float x) {
  if (x <= 2.0f) {
    const float y = 0.25f * x * x;
    const float xk1 = x * logf(0.5f * x) * bessel_ie1(x) * expf(x) + 1.0f +
                      y * (0.15443144f + y * (-0.67278579f + y * (-0.18156897f + y * (-0.01919402f +
                      y * (-0.00110404f - y * 0.00004686f)))));
    return xk1 / x * expf(x);
  }
  const float y = 2.0f / x;
  return (1.25331414f + y * (0.23498619f + y * (-0.03655620f + y * (0.01504268f + y * (-0.00780353f +
          y * (0.00325614f - y * 0.00068245f)))))) * rsqrtf(x);
}

// Q^{sigma,B}(r; R) (Eq. ScreenedPoissonKernelsSphere), a = sqrt(sigma) > 0
template <int D>
__device__ inline float screened_q(float a, float r, float R) {
  const float zr = r * a, zR = R * a;
  if (D == 2) {
    if (zr < 1e-12f) return 1.0f;
    // (K1(zr) + I1(zr) K0(zR) / I0(zR)) zr with the exponentials combined
    return (bessel_ke1(zr) * expf(-zr) +
            bessel_ie1(zr) * bessel_ke0(zR) / bessel_ie0(zR) * expf(zr - 2.0f * zR)) * zr;
  }
  // e^-zr (zr + 1) + (zr cosh zr - sinh zr) e^-zR / sinh zR, with
  // e^-zR / sinh zR = 2 e^-2zR / (1 - e^-2zR) and a series for the
  // cancelling numerator at small zr
  const float num = zr < 0.1f ? zr * zr * zr * (1.0f / 3.0f + zr * zr * (1.0f / 30.0f))
                              : zr * coshf(zr) - sinhf(zr);
  return expf(-zr) * (zr + 1.0f) + num * 2.0f * expf(-2.0f * zR) / -expm1f(-2.0f * zR);
}

// G^{sigma,B} at distance rho in a ball of radius R
template <int D>
__device__ inline float green_ball_screened(float a, float rho, float R) {
  const float zr = rho * a, zR = R * a;
  if (D == 2)
    return (bessel_ke0(zr) * expf(-zr) -
            bessel_ie0(zr) * bessel_ke0(zR) / bessel_ie0(zR) * expf(zr - 2.0f * zR)) * (1.0f / (2.0f * kPi));
  // sinh((R - rho) a) / (4 pi rho sinh(R a)) = e^-zr (1 - e^-2(zR - zr)) /
  // (1 - e^-2zR) / (4 pi rho), the differences by expm1
  return expf(-zr) * expm1f(-2.0f * (zR - zr)) / expm1f(-2.0f * zR) * (1.0f / (4.0f * kPi)) * rcp(rho);
}

// |G^{sigma,B}| = integral over the ball; series near zR = 0, where the
// closed forms cancel
template <int D>
__device__ inline float green_ball_norm_screened(float sigma, float a, float R) {
  const float z = R * a, z2 = z * z;
  if (D == 2) {
    // (1 - 1 / I0(z)) / sigma = (I0(z) - 1) / (I0(z) sigma)
    const float i0 = bessel_ie0(z) * expf(z);
    const float i0m1 = z < 0.5f ? z2 * (0.25f + z2 * (1.0f / 64.0f + z2 * (1.0f / 2304.0f))) : i0 - 1.0f;
    return i0m1 / (i0 * sigma);
  }
  // (1 - z / sinh z) / sigma = (sinh z - z) / (sinh z sigma)
  const float sh = sinhf(z);
  const float shm = z < 0.5f ? z * z2 * (1.0f / 6.0f + z2 * (1.0f / 120.0f + z2 * (1.0f / 5040.0f))) : sh - z;
  return shm / (sh * sigma);
}

template <int D>
__device__ inline Vec<D> sample_direction(float U0, float U1) {
  Vec<D> v;
  if (D == 2) {
    // the hardware sine and cosine take their argument in turns
    // (sin(2 pi a)), so the angle 2 pi U0 needs no range reduction
    v[0] = __builtin_amdgcn_cosf(U0);
    v[1] = __builtin_amdgcn_sinf(U0);
  } else {
    const float zz = 1.0f - 2.0f * U0;
    const float rr = sqrtf(fmaxf(0.0f, 1.0f - zz * zz));
    v[0] = rr * __builtin_amdgcn_cosf(U1);
    v[1] = rr * __builtin_amdgcn_sinf(U1);
    v[D - 1] = zz;
  }
  return v;
}

template <int D>
__device__ inline float source_fraction(float U2, float U3) {
  if (D == 2) return sqrtf(U2 * U3);
  return 0.5f + cosf((acosf(1.0f - 2.0f * U2) - 2.0f * kPi) * (1.0f / 3.0f));
}

// ---------------------------------------------------------------------------
// one step of Algorithm 1
// ---------------------------------------------------------------------------
template <int D>
struct WalkState {
  Vec<D> x, n;      // on the Neumann boundary, n is the normal of the walk's side
  Vec<D> q;         // x_k - x_{k-1} (double-sided forms); the start side's normal at a boundary start
  int cur;          // Neumann slot the walk sits on, -1 otherwise
  int lastD;        // Dirichlet slot closest at the previous step, -1 at the start
  int lastS;        // silhouette element closest at the previous step, or -1
  int onN;
  uint32_t k;       // step index
  uint32_t point, walk;
  float acc, comp;  // Kahan sum
};

__device__ inline void kahan_add(float& acc, float& comp, float v) {
  const float y = v - comp;
  const float t = acc + y;
  comp = (t - acc) - y;
  acc = t;
}

template <int D>
__device__ inline float g_at(const SceneDev& S, const FnDev& F, const Vec<D>& x, int slot) {
  if (slot < 0) return 0.0f;
  if (F.kind != 4 || slot >= S.nD) return fn_value<D>(F, x);   // analytic data, or a shape
  const Prim<D> P = load_prim<D>(S.dp, slot);
  float wb, wc;
  closest_prim<D>(x, P, wb, wc);
  return boundary_value<D>(F, S.did[slot], x, wb, wc, P);
}

// Analytic Dirichlet shapes (mixed representations, Sec. 6): two float4
// each, (p0, p1, p2, radius or rounding) and (p3, p4, p5, code), code = kind
// | inside << 4; kind 0 ball (centre p0..2), 1 box (centre p0..2, half
// extents p3..5, rounded by the radius), 2 capsule (segment p0..2 - p3..5).
// Returns the distance to the surface (0 for a point on the wrong side) and
// its closest point o.
template <int D>
__device__ inline float sdf_closest(const float4 a, const float4 b, const Vec<D>& x, Vec<D>& o) {
  const int code = __float_as_int(b.w);
  const int kind = code & 15;
  const bool inside = (code >> 4) & 1;
  const float c3[3] = {a.x, a.y, a.z}, e3[3] = {b.x, b.y, b.z};
  if (kind == 1 && inside) {   // sharp box seen from inside: the nearest face
    int km = 0;
    float gm = kInf;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const float g = e3[k] - fabsf(x[k] - c3[k]);
      if (g < gm) { gm = g; km = k; }
    }
    o = x;
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (k == km) o[k] = c3[k] + (x[k] >= c3[k] ? e3[k] : -e3[k]);
    return fmaxf(gm, 0.0f);
  }
  // closest point of the core: the centre, the sharp box or the segment
  Vec<D> core;
  if (kind == 0) {
#pragma unroll
    for (int k = 0; k < D; ++k) core[k] = c3[k];
  } else if (kind == 1) {
#pragma unroll
    for (int k = 0; k < D; ++k) core[k] = fminf(fmaxf(x[k], c3[k] - e3[k]), c3[k] + e3[k]);
  } else {
    float ab2 = 0.0f, axab = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      ab2 += (e3[k] - c3[k]) * (e3[k] - c3[k]);
      axab += (x[k] - c3[k]) * (e3[k] - c3[k]);
    }
    const float t = ab2 > 0.0f ? fminf(fmaxf(axab / ab2, 0.0f), 1.0f) : 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) core[k] = c3[k] + t * (e3[k] - c3[k]);
  }
  const Vec<D> v = sub(x, core);
  const float l = sqrtf(dot(v, v));
  if (l > 0.0f) {
    o = axpy(core, a.w / l, v);
  } else {   // on the core (the ball's centre): any surface point is closest
    o = core;
    o[0] += a.w;
  }
  return fmaxf(inside ? a.w - l : l - a.w, 0.0f);
}

// Q.1 over the analytic shapes: lowers key k (squared distance, slot nD + i)
// and keeps the closest point of the winning shape in xs
template <int D>
__device__ inline Key sdf_query(const SceneDev& S, const Vec<D>& x, Key k, Vec<D>& xs) {
  for (int i = 0; i < S.nS; ++i) {
    Vec<D> o;
    const float d = sdf_closest<D>(S.sdf[2 * i], S.sdf[2 * i + 1], x, o);
    const Key ks = make_key(d * d, S.nD + i);
    if (ks < k) {
      k = ks;
      xs = o;
    }
  }
  return k;
}

// Double-sided primitives (appendix on open domains and double-sided
// boundaries): "+" is the side a primitive's normal points away from, "-"
// the side it points into.  The g of a walk's end is taken from the side
// the walk approached from: q . n+ > 0 means "+", with q = x_k - x_{k-1},
// or, at the first step of an interior start, the direction from the start
// point to its closest point (the side the start lies on).
template <int D>
__device__ inline float g_end(const SceneDev& S, const WalkState<D>& w, const Vec<D>& xb, int slot,
                              int& side) {
  side = 0;
  if (slot < 0 || slot >= S.nD || !S.dside[slot]) return g_at<D>(S, S.fn[kFnG], xb, slot);
  const Vec<D> qd = (w.k == 0 && !w.onN) ? sub(xb, w.x) : w.q;
  const bool minus = !(dot(qd, prim_normal<D>(load_prim<D>(S.dp, slot))) > 0.0f);
  side = minus ? -1 : 1;
  return g_at<D>(S, S.fn[minus ? kFnGm : kFnG], xb, slot);
}

// One step of the walk held by this lane when `live`.  Returns 0 to
// continue (or when not live), 1 eps-shell, 2 capped, 3 escaped, 4 ended
// by Russian roulette (screened problems).  With COOP
// the four tree queries are wave-cooperative: every lane of the wave must
// call this together (lanes without a live walk help the others); without
// COOP each lane runs its own queries and may call it alone.
template <int D, bool HH, bool HF, bool TRACE, bool CNT, bool COOP, bool DS>
__device__ int walk_step(const SceneDev& S, const WalkParams& P, WalkState<D>& w, bool live, int* stk,
                         const CoopLds& L, StepRec* rec, Cnt& cn) {
  if (TRACE && live) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { rec->x[k] = k < D ? w.x[k] : 0.0f; rec->n[k] = k < D ? w.n[k] : 0.0f; }
    rec->onN = w.onN;
    rec->cur = w.cur >= 0 ? S.nid[w.cur] : -1;
  }
  if (CNT && live) {
    cn.wave(kWaveSteps);
    cn.phase(kCycRest);
  }
  // Q.1, warm-started from the previous step's closest primitive
  Q1Query<D, CNT> q1;
  q1.x = w.x;
  const bool has1 = live && S.nD > 0;
  Key k1 = make_key(kInf, -1);
  if (has1 && w.lastD >= 0 && w.lastD < S.nD) {
    if (CNT) cn.add(kCntQ1Prim);
    float wb, wc;
    const Vec<D> dv = sub(closest_prim<D>(w.x, load_prim<D>(S.dp, w.lastD), wb, wc), w.x);
    k1 = make_key(dot(dv, dv), w.lastD);
  }
  k1 = run_query<Q1Query<D, CNT>, CNT, COOP>(S, q1, has1, k1, stk, L, cn);
  Vec<D> xb = w.x;
  if (live) k1 = sdf_query<D>(S, w.x, k1, xb);   // analytic shapes, slots nD + i
  const int pD = live ? key_slot(k1) : -1;
  float dD = kInf;
  if (pD >= 0) {   // the closest point itself, once
    if (pD < S.nD) {
      float wb, wc;
      xb = closest_prim<D>(w.x, load_prim<D>(S.dp, pD), wb, wc);
    }
    dD = sqrtf(key_value(k1));
  }
  if (CNT && live) cn.phase(kCycQ1);
  int term = 0;
  if (live) {
    w.lastD = pD;
    float dc2 = 0.0f;
    const float c3[3] = {S.cx, S.cy, S.cz};
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const float a = w.x[k] - c3[k];
      dc2 += a * a;
    }
    if (dD < P.eps) term = 1;
    else if ((int)w.k >= P.max_steps) term = 2;
    else if (dc2 > S.escape2) term = 3;
    if (TRACE) {
      rec->dD = dD;
#pragma unroll
      for (int k = 0; k < 3; ++k) rec->xbar[k] = k < D ? xb[k] : 0.0f;
      rec->primD = pD < 0 ? -1 : (pD < S.nD ? S.did[pD] : S.sdf_id0 + (pD - S.nD));
      rec->term = term;
    }
    if (term) {
      int side = 0;
      const float g = DS ? g_end<D>(S, w, xb, pD, side) : g_at<D>(S, S.fn[kFnG], xb, pD);
      kahan_add(w.acc, w.comp, g);
      if (TRACE) { rec->g_term = g; rec->acc = w.acc; rec->side_g = side; }
    }
  }
  const bool go = live && term == 0;
  Vec<D> xq = w.x;
  if (w.onN) xq = axpy(w.x, -S.offset, w.n);

  // Q.2, r_max = d_D, warm-started from the previous closest silhouette element
  Q2Query<D, CNT> q2;
  q2.x = xq;
  const bool has2 = go && S.nE > 0;
  Key k2 = make_key(dD * dD, -1);
  if (has2 && w.lastS >= 0) {
    if (CNT) cn.add(kCntQ2Elem);
    float dd;
    const bool sil = silhouette_element<D>(S, w.lastS, xq, dd);
    k2 = key_min(k2, sil ? make_key(dd, w.lastS) : kNoKey);
  }
  k2 = run_query<Q2Query<D, CNT>, CNT, COOP>(S, q2, has2, k2, stk, L, cn);
  const int sarg = has2 ? key_slot(k2) : -1;
  const float dsil = sarg >= 0 ? sqrtf(key_value(k2)) : dD;
  if (go) w.lastS = sarg;
  if (CNT && live) cn.phase(kCycQ2);
  // star radius; without a Dirichlet boundary (screened problems only) it is
  // capped at the escape radius
  const float r = fminf(fminf(dD, fmaxf(P.rmin, dsil)), S.escape);
  // screening of this step: sigma, plus the Tikhonov sigma_T from step
  // tik_steps on (Sec. 3.4)
  const float sig = P.sigma + ((P.tik_sigma > 0.0f && (int)w.k >= P.tik_steps) ? P.tik_sigma : 0.0f);
  const float sa = sqrtf(sig);

  uint4 ctr = make_uint4(w.point, w.walk, w.k, 0u);
  const uint4 u0 = philox(ctr, P.seed_lo, P.seed_hi);
  Vec<D> v = sample_direction<D>(u01(u0.x), u01(u0.y));
  if (w.onN && dot(w.n, v) > 0.0f) {
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = -v[k];
  }
  // Q.3: first Neumann crossing within the star radius
  RayQuery<D, false, CNT> q3;
  q3.R = make_ray<D>(xq, v);
  q3.tmax = r;
  q3.skip = w.onN ? w.cur : -1;
  const bool has3 = go && S.nN > 0;
  const Key k3 = run_query<RayQuery<D, false, CNT>, CNT, COOP>(S, q3, has3, make_key(r, -1), stk, L, cn);
  const int hp = has3 ? key_slot(k3) : -1;
  // the next point lies on the ray that was tested, from the (offset)
  // query origin: its first Neumann crossing, else the end of the ray
  const float t = hp >= 0 ? key_value(k3) : r;
  if (CNT && live) cn.phase(kCycQ3);
  const Vec<D> p = axpy(xq, t, v);

  float Nhat = 0.0f;
  if (HH) {
    Vec<D> z = xq;
    float pdf = 0.0f, wb = 0.0f, wc = 0.0f, rho = 0.0f;
    int zp = -1;
    bool cand = false;
    if (go) {
      zp = q4_sample<D, CNT>(S, w.x, r, ctr, P.seed_lo, P.seed_hi, z, pdf, wb, wc, cn);
      if (zp >= 0) {
        const Vec<D> dz = sub(z, w.x);
        rho = sqrtf(dot(dz, dz));
        cand = pdf > 0.0f && rho > 0.0f && rho < r;
      }
    }
    // visibility of the sample from the (offset) query origin
    RayQuery<D, true, CNT> qv;
    qv.R = make_ray<D>(xq, sub(z, xq));
    qv.tmax = 1.0f - 1e-6f;
    qv.skip = zp;
    const Key kv = run_query<RayQuery<D, true, CNT>, CNT, COOP>(S, qv, cand, kNoKey, stk, L, cn);
    const bool valid = cand && kv == kNoKey;
    int hside = 0;
    if (valid) {
      const float alpha = w.onN ? 0.5f : 1.0f;
      const Prim<D> Pz = load_prim<D>(S.np, zp);
      // double-sided: the data of the side of zp that the query origin sees
      bool minus = false;
      if (DS && S.nside[zp]) {
        minus = !(dot(sub(z, xq), prim_normal<D>(Pz)) > 0.0f);
        hside = minus ? -1 : 1;
      }
      const float hz = boundary_value<D>(S.fn[minus ? kFnHm : kFnH], S.nid[zp], z, wb, wc, Pz, minus ? -1.0f : 1.0f);
      const float G = sig > 0.0f ? green_ball_screened<D>(sa, rho, r) : green_ball<D>(rho, r);
      Nhat = G * hz * rcp(alpha * pdf);
      if (!isfinite(Nhat)) Nhat = 0.0f;   // an overflowing 1/pdf: drop the sample
    }
    if (TRACE && go) {
      rec->n_prim = zp >= 0 ? S.nid[zp] : -1;
      rec->valid = valid;
      rec->side_h = hside;
#pragma unroll
      for (int k = 0; k < 3; ++k) rec->z[k] = (zp >= 0 && k < D) ? z[k] : 0.0f;
      rec->pdf = pdf;
    }
  }
  if (CNT && live) cn.phase(kCycQ4);
  if (!go) return term;
  float Shat = 0.0f;
  float sf = 0.0f;
  if (HF) {
    sf = source_fraction<D>(u01(u0.z), u01(u0.w));
    const float ts = r * sf;
    if (ts < t) {
      Shat = green_ball_norm<D>(r) * fn_value<D>(S.fn[kFnF], axpy(w.x, ts, v));
      // screened: the Poisson-density sample reweighted by G^{sigma,B} / G^B
      if (sig > 0.0f && ts > 0.0f) Shat *= green_ball_screened<D>(sa, ts, r) / green_ball<D>(ts, r);
    }
  }
  kahan_add(w.acc, w.comp, Nhat - Shat);
  // the screened continuation factor Q^{sigma,B}(t; r) as Russian roulette:
  // the walk goes on, unweighted, with probability Q (its own Philox slot)
  float q = 1.0f;
  int roulette = 0;
  if (sig > 0.0f) {
    q = screened_q<D>(sa, t, r);
    const uint4 ur = philox(make_uint4(w.point, w.walk, w.k, 0xffffffffu), P.seed_lo, P.seed_hi);
    roulette = u01(ur.x) >= q;
  }
  if (TRACE) {
    rec->dsil = dsil;
    rec->r = r;
#pragma unroll
    for (int k = 0; k < 3; ++k) { rec->v[k] = k < D ? v[k] : 0.0f; rec->p[k] = k < D ? p[k] : 0.0f; }
    rec->hit = hp >= 0;
    rec->hit_prim = hp >= 0 ? S.nid[hp] : -1;
    rec->t = t;
    rec->Nhat = Nhat;
    rec->s_frac = sf;
    rec->Shat = Shat;
    rec->acc = w.acc;
    rec->q = q;
    rec->roulette = roulette;
    if (roulette) rec->term = 4;
  }
  if (roulette) return 4;
  if (DS) w.q = sub(p, w.x);
  w.x = p;
  w.onN = hp >= 0;
  w.cur = hp;
  if (hp >= 0) {
    w.n = prim_normal<D>(load_prim<D>(S.np, hp));
    // double-sided: the normal of the side the walk arrives on
    if (DS && S.nside[hp] && dot(w.q, w.n) < 0.0f) {
#pragma unroll
      for (int k = 0; k < D; ++k) w.n[k] = -w.n[k];
    }
  }
  w.k += 1;
  return 0;
}

// An evaluation point on the Neumann boundary starts on its primitive
// (Algorithm 1 with the on-boundary flag set at the start).  code: the
// Neumann slot for the "+" side, -2 - slot for the "-" side of a
// double-sided primitive, -1 for an interior point.
template <int D>
__device__ inline void start_on_boundary(const SceneDev& S, int code, WalkState<D>& w) {
  if (code == -1) return;
  const bool minus = code <= -2;
  const int slot = minus ? -2 - code : code;
  w.onN = 1;
  w.cur = slot;
  w.n = prim_normal<D>(load_prim<D>(S.np, slot));
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (minus) w.n[k] = -w.n[k];
    w.q[k] = w.n[k];
  }
}

// walk id -> (point, walk): point-major keeps a point's walks in adjacent
// lanes, walk-major spreads consecutive points over a wave; the estimate
// slot is point * W + walk either way
template <int D>
__device__ inline void init_walk(const SceneDev& S, const WalkParams& P, int64_t id, WalkState<D>& w) {
  int64_t pt, wk;
  if (P.order == 1) {
    wk = id / P.n_points;
    pt = id - wk * P.n_points;
  } else {
    pt = id / P.W;
    wk = id - pt * P.W;
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    w.x[k] = P.points[pt * D + k];
    w.n[k] = 0.0f;
    w.q[k] = 0.0f;
  }
  w.cur = -1;
  w.lastD = -1;
  w.lastS = -1;
  w.onN = 0;
  w.k = 0;
  w.point = P.point_base + (uint32_t)pt;
  w.walk = P.walk_base + (uint32_t)wk;
  w.acc = 0.0f;
  w.comp = 0.0f;
  if (P.start) start_on_boundary<D>(S, P.start[pt], w);
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ inline void flush_stats(const WalkParams& P, unsigned long long steps,
                                   unsigned long long walks, unsigned long long capped,
                                   unsigned long long escaped) {
  steps = wave_sum_u64(steps);
  walks = wave_sum_u64(walks);
  capped = wave_sum_u64(capped);
  escaped = wave_sum_u64(escaped);
  if (__lane_id() == 0) {
    atomicAdd(P.stats + 0, steps);
    atomicAdd(P.stats + 1, walks);
    if (capped) atomicAdd(P.stats + 2, capped);
    if (escaped) atomicAdd(P.stats + 3, escaped);
  }
}

// the same for counters already summed over the wave (wave-uniform values,
// which the compiler keeps in scalar registers instead of four 64-bit
// vector registers per lane)
__device__ inline void flush_wave_stats(const WalkParams& P, unsigned long long steps,
                                        unsigned long long walks, unsigned long long capped,
                                        unsigned long long escaped) {
  if (__lane_id() == 0) {
    atomicAdd(P.stats + 0, steps);
    atomicAdd(P.stats + 1, walks);
    if (capped) atomicAdd(P.stats + 2, capped);
    if (escaped) atomicAdd(P.stats + 3, escaped);
  }
}

// a walk that ended capped or escaped: its RNG ids, its length and how it
// ended, into the first kEventCap slots of the solve's event list (rare:
// these ends are counted and should not occur on a closed domain)
template <int D>
__device__ inline void record_event(const WalkParams& P, const WalkState<D>& w, int term) {
  if (!P.events || (term != 2 && term != 3)) return;
  const unsigned long long slot = atomicAdd(P.events, 1ull);
  if (slot < (unsigned long long)kEventCap) {
    P.events[1 + 2 * slot] = ((unsigned long long)w.point << 32) | w.walk;
    P.events[2 + 2 * slot] = ((unsigned long long)(w.k + 1) << 8) | (unsigned)term;
  }
}

// counts one wave iteration of a persistent loop: lanes that stepped, and
// walks that ended (all, capped, escaped), by ballot on converged lanes
__device__ inline void count_wave(bool stepped, int ended, unsigned long long& steps,
                                  unsigned long long& walks, unsigned long long& capped,
                                  unsigned long long& escaped) {
  steps += __popcll(__ballot(stepped));
  walks += __popcll(__ballot(ended != 0));
  capped += __popcll(__ballot(ended == 2));
  escaped += __popcll(__ballot(ended == 3));
}

__device__ inline void flush_traffic(const WalkParams& P, const Cnt& cn) {
#pragma unroll
  for (int i = 0; i < kTrafficCounters; ++i) {
    const unsigned long long v = wave_sum_u64((unsigned long long)cn.v[i]);
    if (__lane_id() == 0 && v) atomicAdd(P.traffic + i, v);
  }
}

__device__ inline void zero(Cnt& cn) {
#pragma unroll
  for (int i = 0; i < kTrafficCounters; ++i) cn.v[i] = 0;
  cn.t_mark = clock64();
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Top tree levels in LDS: the first nodes of each tree (numbered first by
// the builder: a binary tree's top four levels, at most 15 nodes; a 4-wide
// tree's top two, at most 5 records) and, in 2D, the silhouette tree's
// cones, copied once per block; queries then read them from LDS instead of
// through the caches.  Regions (float4): Dirichlet, binary Neumann,
// silhouette, then the 2D cones or the 3D ray tree.
template <int D>
constexpr int kTopD = D == 3 ? kSRec * 5 : 3 * kTopNodes;
template <int D>
constexpr int kTopN = (D == 3 ? 4 : 3) * kTopNodes;
template <int D>
constexpr int kTopS = D == 3 ? kSRec * 5 : 3 * kTopNodes;
template <int D>
constexpr int kTopX = D == 3 ? kSRec * 5 : 2 * kTopNodes;
template <int D>
constexpr int kTopCache = kTopInLds<D> ? kTopD<D> + kTopN<D> + kTopS<D> + kTopX<D> : 1;

template <int D>
__device__ inline void install_top(SceneDev& S, float4* cache) {
  constexpr int nf = D == 3 ? 4 : 3;           // float4 per binary node
  constexpr int rd = D == 3 ? kSRec : nf;      // float4 per Dirichlet-tree node in dn
  constexpr int rs = D == 3 ? kSRec : nf;      // float4 per silhouette-tree node in sn
  float4* cd = cache;
  float4* cn = cd + kTopD<D>;
  float4* cs = cn + kTopN<D>;
  float4* cx = cs + kTopS<D>;                  // 2D cones, 3D ray tree
  for (int i = threadIdx.x; i < rd * S.topD; i += kBlock) cd[i] = S.dn[i];
  for (int i = threadIdx.x; i < nf * S.topN; i += kBlock) cn[i] = S.nn[i];
  for (int i = threadIdx.x; i < rs * S.topS; i += kBlock) cs[i] = S.sn[i];
  if (D == 2)
    for (int i = threadIdx.x; i < 2 * S.topS; i += kBlock) cx[i] = S.sc[i];
  else
    for (int i = threadIdx.x; i < kSRec * S.topR; i += kBlock) cx[i] = S.rn[i];
  __syncthreads();
  S.tdn = cd;
  S.tnn = cn;
  S.tsn = cs;
  S.tsc = D == 2 ? cx : nullptr;
  S.trn = D == 3 ? cx : nullptr;
  S.ctD = S.topD;
  S.ctN = S.topN;
  S.ctS = S.topS;
  S.ctR = D == 3 ? S.topR : 0;
}

// Plain form: one lane per walk, fixed assignment; the wave runs as long as
// its longest walk.
// The walk kernels hold their traversal stacks in LDS (kStack<D> entries x
// 256 lanes x 4 B per block, plus 3 KiB for the cooperative keys and victim
// lists): 27 KiB in 2D, so a 160 KiB CU holds 5 blocks, 5 waves per SIMD,
// and 35 KiB in 3D, 4 blocks.  Registers are budgeted to match: 2D to 5 waves
// (<= 96 VGPRs, a few spilled to scratch; measured 6 % faster than 4 waves
// with 32-entry stacks, and 4 % faster than 6 waves with 22-entry stacks),
// 3D to 4 waves (<= 128 VGPRs, a few spills; the triangle tests take ~130
// unconstrained, which leaves 3 waves; 5 waves measured 8 % slower).
#define kWalkOccupancy __attribute__((amdgpu_waves_per_eu(D == 2 ? 5 : 4)))

template <int D, bool HH, bool HF, bool CNT, bool DS>
__global__ __launch_bounds__(kBlock) kWalkOccupancy void k_walk_plain(SceneDev S, WalkParams P) {
  __shared__ int stack[kStack<D> * kBlock];
  int* stk = stack + threadIdx.x;
  const int64_t total = P.n_points * (int64_t)P.W;
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long steps = 0, walks = 0, capped = 0, escaped = 0;
  Cnt cn;
  zero(cn);
  if (id < total) {
    WalkState<D> w{};
    init_walk<D>(S, P, id, w);
    while (true) {
      const int term = walk_step<D, HH, HF, false, CNT, false, DS>(S, P, w, true, stk, CoopLds{}, nullptr, cn);
      ++steps;
      if (term) {
        P.est[(int64_t)(w.point - P.point_base) * P.W + (w.walk - P.walk_base)] = w.acc;
        record_event<D>(P, w, term);
        walks = 1;
        capped = term == 2;
        escaped = term == 3;
        break;
      }
    }
  }
  flush_stats(P, steps, walks, capped, escaped);
  if (CNT) flush_traffic(P, cn);
}

// Persistent form: a grid sized to the resident capacity; a lane whose walk
// ends takes the next walk index from its wave's pool.  A wave claims walks
// from the device-wide cursor up to P.claim at a time with one atomic, so
// the cursor sees about one atomic per P.claim walks (not one per refill)
// and the estimates a wave writes are contiguous.  Claims shrink as the work
// runs out (a quarter of the remaining walks per wave of the grid), so that
// no wave is left with a long private tail when the others have finished,
// and always cover the idle lanes.  In 3D a step costs far more than the
// refill atomic and the pool's tail cost outweighs its gain: 3D claims
// exactly the idle lanes' share (a run-time claim size measured 11 more
// spilled registers there); in 2D the claim is a solve option, 128 by
// default.  Idle lanes of a wave are refilled together:
// each takes its rank among the idle lanes (ballot + mbcnt) past the pool's
// front, and ranks beyond the pool's end take the front of a new claim.
// Every wave exits once the cursor has passed the last walk, its pool is
// empty and its own lanes are done.  With COOP the wave steps all its walks
// together and shares the tree searches among its lanes (coop_traverse).
template <int D, bool HH, bool HF, bool COOP, bool DS>
__global__ __launch_bounds__(kBlock) kWalkOccupancy void k_walk_persistent(SceneDev S0, WalkParams P) {
  __shared__ int stack[kStack<D> * kBlock];
  __shared__ float4 top[kTopCache<D>];
  SceneDev S = S0;
  if (kTopInLds<D>) install_top<D>(S, top);
  __shared__ Key keys[COOP ? kBlock : 1];
  __shared__ int vict[COOP ? kBlock : 1];
  int* stk = stack + threadIdx.x;
  const int wbase = threadIdx.x & ~63;
  const CoopLds L{stack + wbase, keys + (COOP ? wbase : 0), vict + (COOP ? wbase : 0), P.steal};
  const int64_t total = P.n_points * (int64_t)P.W;
  unsigned long long steps = 0, walks = 0, capped = 0, escaped = 0;
  WalkState<D> w{};
  int64_t id = -1;
  bool active = false;
  bool drained = false;            // the cursor has passed the last walk
  int64_t pool = 0, pool_end = 0;  // wave-uniform: unassigned claimed walks [pool, pool_end)
  int64_t seen = 0;                // wave-uniform: the cursor at this wave's last claim
  const int64_t n_waves = (int64_t)gridDim.x * (kBlock / 64);
  Cnt cn;
  const int lane = __lane_id();
  while (true) {
    if (!drained || pool < pool_end) {
      const unsigned long long idle = __ballot(!active);
      const int n_idle = __popcll(idle);
      if (n_idle >= P.refill || (n_idle > 0 && idle == ~0ull)) {
        const int64_t avail = pool_end - pool;
        int64_t fresh = 0, fresh_end = 0;   // a new claim, taken when the pool runs short
        if (avail < n_idle && !drained) {
          const int64_t want = max(min((total - seen) / (4 * n_waves), (int64_t)(D == 2 ? P.claim : 1)), (int64_t)n_idle - avail);
          const int leader = __ffsll((long long)idle) - 1;
          unsigned long long base = 0;
          if (lane == leader) base = atomicAdd(P.counter, (unsigned long long)want);
          // readlane keeps the claim (and the pool) in scalar registers
          const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(base & 0xffffffffull), leader);
          const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), leader);
          base = ((unsigned long long)hi << 32) | lo;
          if (base + (unsigned long long)want >= (unsigned long long)total) drained = true;
          fresh = base < (unsigned long long)total ? (int64_t)base : total;
          fresh_end = min(fresh + want, total);
          seen = fresh;
        }
        if (!active) {
          const int rank = __popcll(idle & ((1ull << lane) - 1ull));
          int64_t cand = -1;
          if (rank < avail) cand = pool + rank;
          else if (rank - avail < fresh_end - fresh) cand = fresh + (rank - avail);
          if (cand >= 0) {
            id = cand;
            init_walk<D>(S, P, id, w);
            active = true;
          }
        }
        if (avail >= n_idle) {
          pool += n_idle;
        } else if (fresh_end > fresh) {
          pool = min(fresh + (n_idle - avail), fresh_end);
          pool_end = fresh_end;
        } else {
          pool = pool_end;
        }
      }
    }
    if (!__any(active)) {
      if (drained && pool >= pool_end) break;
      continue;
    }
    bool stepped = false;
    int ended = 0;
    if (COOP || active) {
      const int term = walk_step<D, HH, HF, false, false, COOP, DS>(S, P, w, active, stk, L, nullptr, cn);
      if (active) {
        stepped = true;
        if (term) {
          P.est[(int64_t)(w.point - P.point_base) * P.W + (w.walk - P.walk_base)] = w.acc;
          if (term >= 2) record_event<D>(P, w, term);
          ended = term;
          active = false;
        }
      }
    }
    count_wave(stepped, ended, steps, walks, capped, escaped);
  }
  flush_wave_stats(P, steps, walks, capped, escaped);
}

// Batched form: one persistent grid over the chunks of many (scene, point
// set) items.  A wave claims one chunk at a time with a single atomic, so its
// scene and solve parameters stay wave-uniform (scalar registers); inside the
// chunk idle lanes are refilled from a wave-local cursor (ballot + mbcnt), so
// no further atomics are needed.
__device__ inline int64_t uniform_i64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v & 0xffffffffull));
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int D, bool HH, bool HF, bool COOP, bool DS>
__global__ __launch_bounds__(kBlock) kWalkOccupancy void k_walk_batch(const BatchItem* __restrict__ table,
                                                       const BatchGroupDev* __restrict__ group,
                                                       unsigned long long* cursor,
                                                       unsigned long long* stats) {
  // the group's sizes come from device memory, written for each call
  const BatchItem* __restrict__ items = table + group->first;
  const int n_items = group->n_items;
  const int64_t n_chunks = group->n_chunks;
  const int chunk = group->chunk;
  __shared__ int stack[kStack<D> * kBlock];
  __shared__ Key keys[COOP ? kBlock : 1];
  __shared__ int vict[COOP ? kBlock : 1];
  int* stk = stack + threadIdx.x;
  const int wbase = threadIdx.x & ~63;
  CoopLds L{stack + wbase, keys + (COOP ? wbase : 0), vict + (COOP ? wbase : 0), 1};
  const int lane = __lane_id();
  unsigned long long steps = 0, walks = 0, capped = 0, escaped = 0;
  Cnt cn;
  while (true) {
    unsigned long long g0 = 0;
    if (lane == 0) g0 = atomicAdd(cursor, 1ull);
    const int64_t g = uniform_i64((int64_t)__shfl(g0, 0));
    if (g >= n_chunks) break;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].chunk_begin <= g) lo = mid;
      else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const SceneDev S = items[lo].S;
    const WalkParams P = items[lo].P;
    L.steal = P.steal;
    const int64_t w0 = (g - items[lo].chunk_begin) * (int64_t)chunk;
    const int64_t w1 = min(w0 + (int64_t)chunk, items[lo].n_walks);
    int64_t lc = w0;
    WalkState<D> w{};
    int64_t id = -1;
    bool active = false;
    while (true) {
      const unsigned long long idle = __ballot(!active);
      if (idle != 0ull && lc < w1) {
        if (!active) {
          const int64_t cand = lc + __popcll(idle & ((1ull << lane) - 1ull));
          if (cand < w1) {
            id = cand;
            init_walk<D>(S, P, id, w);
            active = true;
          }
        }
        lc = min(lc + (int64_t)__popcll(idle), w1);
      }
      if (!__any(active)) break;
      bool stepped = false;
      int ended = 0;
      if (COOP || active) {
        const int term = walk_step<D, HH, HF, false, false, COOP, DS>(S, P, w, active, stk, L, nullptr, cn);
        if (active) {
          stepped = true;
          if (term) {
            P.est[(int64_t)(w.point - P.point_base) * P.W + (w.walk - P.walk_base)] = w.acc;
            if (term >= 2) record_event<D>(P, w, term);
            ended = term;
            active = false;
          }
        }
      }
      count_wave(stepped, ended, steps, walks, capped, escaped);
    }
  }
  WalkParams Q{};
  Q.stats = stats;
  flush_wave_stats(Q, steps, walks, capped, escaped);
}

template <int D, bool HH, bool HF, bool DS>
__global__ __launch_bounds__(kBlock) void k_trace(SceneDev S, WalkParams P, const uint32_t* pids,
                                                  const uint32_t* wids, int64_t n, int max_rec,
                                                  StepRec* recs, int* n_steps, float* values) {
  __shared__ int stack[kStack<D> * kBlock];
  int* stk = stack + threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  WalkState<D> w{};
#pragma unroll
  for (int k = 0; k < D; ++k) {
    w.x[k] = P.points[i * D + k];
    w.n[k] = 0.0f;
    w.q[k] = 0.0f;
  }
  w.cur = -1;
  w.lastD = -1;
  w.lastS = -1;
  w.onN = 0;
  w.k = 0;
  w.point = pids[i];
  w.walk = wids[i];
  w.acc = 0.0f;
  w.comp = 0.0f;
  if (P.start) start_on_boundary<D>(S, P.start[i], w);
  StepRec dummy;
  Cnt cn;
  int ns = 0;
  while (true) {
    StepRec* rec = ns < max_rec ? recs + i * (int64_t)max_rec + ns : &dummy;
    const int term = walk_step<D, HH, HF, true, false, false, DS>(S, P, w, true, stk, CoopLds{}, rec, cn);
    ++ns;
    if (term) break;
  }
  n_steps[i] = ns;
  values[i] = w.acc;
}

// ---------------------------------------------------------------------------
// walk launchers, one WalkPart<D, DS> per translation unit
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int D, bool HH, bool HF, bool DS>
static hipError_t launch_walks_t(const SceneDev& S, const WalkParams& P, int mode, int grid,
                                 bool count, hipStream_t s) {
  const int64_t total = P.n_points * (int64_t)P.W;
  if (count) {
    hipLaunchKernelGGL((k_walk_plain<D, HH, HF, true, DS>), dim3(blocks_for(total)), dim3(kBlock), 0, s, S, P);
  } else if (mode == 1) {
    hipLaunchKernelGGL((k_walk_plain<D, HH, HF, false, DS>), dim3(blocks_for(total)), dim3(kBlock), 0, s, S, P);
  } else if (mode == 2) {
    hipLaunchKernelGGL((k_walk_persistent<D, HH, HF, false, DS>), dim3(grid), dim3(kBlock), 0, s, S, P);
  } else {
    hipLaunchKernelGGL((k_walk_persistent<D, HH, HF, true, DS>), dim3(grid), dim3(kBlock), 0, s, S, P);
  }
  return hipGetLastError();
}

template <int D, bool DS>
hipError_t WalkPart<D, DS>::walks(const SceneDev& S, const WalkParams& P, int mode, int grid, bool count,
                                  hipStream_t s) {
  const bool hh = has_neumann_data(S), hf = S.fn_kind[kFnF] != 0;
  if (hh && hf) return launch_walks_t<D, true, true, DS>(S, P, mode, grid, count, s);
  if (hh) return launch_walks_t<D, true, false, DS>(S, P, mode, grid, count, s);
  if (hf) return launch_walks_t<D, false, true, DS>(S, P, mode, grid, count, s);
  return launch_walks_t<D, false, false, DS>(S, P, mode, grid, count, s);
}

template <int D, bool DS>
hipError_t WalkPart<D, DS>::batch(const BatchItem* it, const BatchGroupDev* g, bool hh, bool hf,
                                  unsigned long long* cur, unsigned long long* st, int grid, hipStream_t s) {
  if (hh && hf)
    hipLaunchKernelGGL((k_walk_batch<D, true, true, true, DS>), dim3(grid), dim3(kBlock), 0, s, it, g, cur, st);
  else if (hh)
    hipLaunchKernelGGL((k_walk_batch<D, true, false, true, DS>), dim3(grid), dim3(kBlock), 0, s, it, g, cur, st);
  else if (hf)
    hipLaunchKernelGGL((k_walk_batch<D, false, true, true, DS>), dim3(grid), dim3(kBlock), 0, s, it, g, cur, st);
  else
    hipLaunchKernelGGL((k_walk_batch<D, false, false, true, DS>), dim3(grid), dim3(kBlock), 0, s, it, g, cur, st);
  return hipGetLastError();
}

template <int D, bool DS>
hipError_t WalkPart<D, DS>::trace(const SceneDev& S, const WalkParams& P, const uint32_t* pids,
                                  const uint32_t* wids, int64_t n, int max_rec, StepRec* recs, int* ns,
                                  float* vals, hipStream_t s) {
  const bool hh = has_neumann_data(S), hf = S.fn_kind[kFnF] != 0;
  const dim3 g(blocks_for(n)), b(kBlock);
  if (hh && hf)
    hipLaunchKernelGGL((k_trace<D, true, true, DS>), g, b, 0, s, S, P, pids, wids, n, max_rec, recs, ns, vals);
  else if (hh)
    hipLaunchKernelGGL((k_trace<D, true, false, DS>), g, b, 0, s, S, P, pids, wids, n, max_rec, recs, ns, vals);
  else if (hf)
    hipLaunchKernelGGL((k_trace<D, false, true, DS>), g, b, 0, s, S, P, pids, wids, n, max_rec, recs, ns, vals);
  else
    hipLaunchKernelGGL((k_trace<D, false, false, DS>), g, b, 0, s, S, P, pids, wids, n, max_rec, recs, ns, vals);
  return hipGetLastError();
}

// blocks per CU of the persistent kernel (the form with a Neumann term; the
// occupancy attributes give every variant of one dimension the same bound)
template <int D, bool DS>
int WalkPart<D, DS>::resident_blocks(bool coop) {
  int nb = 0;
  const hipError_t e =
      coop ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_persistent<D, true, D == 3, true, DS>, kBlock, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_persistent<D, true, D == 3, false, DS>, kBlock, 0);
  return (e != hipSuccess || nb < 1) ? 1 : nb;
}

}  // namespace wost
