// Walk-on-stars kernels outside the walk loop (FP64 reductions, serving
// merges, fills and per-query probes) and the dispatch of the walk launchers
// to the WalkPart<dim, double-sided> translation units.
#include <algorithm>

#include "wost_device.hpp"

namespace wost {

// fixed-order FP64 per-point reduction: one wave per point, lane l takes
// walks l, l + 64, ...; butterfly sums; two passes (mean, then squares)
__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ est, int64_t n, int W,
                                                double* mean, double* var) {
  const int64_t pt = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (pt >= n) return;
  const float* e = est + pt * (int64_t)W;
  double s = 0.0;
  for (int j = lane; j < W; j += 64) s += (double)e[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  const double m = s / (double)W;
  double q = 0.0;
  for (int j = lane; j < W; j += 64) {
    const double d = (double)e[j] - m;
    q += d * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
  if (lane == 0) {
    mean[pt] = m;
    var[pt] = W > 1 ? q / (double)(W - 1) : 0.0;
  }
}

// Chan et al.'s pairwise update, for every point of a serving round: the
// round's nb walks (per-point mean mb and unbiased variance vb) merge into
// (mean, M2) over na walks.  Point gp
// belongs to the item whose [point_begin, point_begin + n) holds it; the
// largest standard error goes to the item's slot (float bits of a
// non-negative value order like integers)
__global__ __launch_bounds__(256) void k_merge_batch(const MergeItem* __restrict__ items, int n_items,
                                                     int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t gp = (int64_t)blockIdx.x * 256 + threadIdx.x; gp < total; gp += stride) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].point_begin <= gp) lo = mid;
      else hi = mid - 1;
    }
    const MergeItem& it = items[lo];
    const int64_t i = gp - it.point_begin;
    const double na = it.na, nb = it.nb;
    const double m2b = it.vb[i] * (nb - 1.0);
    double m, q;
    if (na == 0.0) {
      m = it.mb[i];
      q = m2b;
    } else {
      const double tot = na + nb;
      const double d = it.mb[i] - it.mean[i];
      m = it.mean[i] + d * (nb / tot);
      q = it.m2[i] + m2b + d * d * (na * nb / tot);
    }
    it.mean[i] = m;
    it.m2[i] = q;
    const double nt = na + nb;
    const float se = nt > 1.0 ? (float)sqrt(q / (nt - 1.0) / nt) : 0.0f;
    if (se > 0.0f) atomicMax(it.max_se, __float_as_uint(se));
  }
}

hipError_t launch_merge_batch(const MergeItem* d_items, int n_items, int64_t points, hipStream_t s) {
  if (n_items <= 0 || points <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(4096, (points + 255) / 256);
  hipLaunchKernelGGL(k_merge_batch, dim3((unsigned)blocks), dim3(256), 0, s, d_items, n_items, points);
  return hipGetLastError();
}

__global__ void k_fill_u32(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}


hipError_t launch_fill_u32(unsigned int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ---- probes -----------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kBlock) void k_probe_q1(SceneDev S, const float* x, int64_t n,
                                                     float* d, float* xbar, int* prim) {
  __shared__ int stack[kStack<D> * kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  Cnt cn;
  Q1Query<D, false> q;
  q.x = vload<D>(x + i * D);
  Key k = make_key(kInf, -1);
  if (S.nD > 0) k = traverse<Q1Query<D, false>, false>(S, q, k, stack + threadIdx.x, cn);
  Vec<D> xb = q.x;
  k = sdf_query<D>(S, q.x, k, xb);
  const int p = key_slot(k);
  float dd = kInf;
  if (p >= 0) {
    if (p < S.nD) {
      float wb, wc;
      xb = closest_prim<D>(q.x, load_prim<D>(S.dp, p), wb, wc);
    }
    dd = sqrtf(key_value(k));
  }
  d[i] = dd;
  for (int k = 0; k < D; ++k) xbar[i * D + k] = xb[k];
  prim[i] = p < 0 ? -1 : (p < S.nD ? S.did[p] : S.sdf_id0 + (p - S.nD));
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_probe_q2(SceneDev S, const float* x, const float* rmax,
                                                     int64_t n, float* d) {
  __shared__ int stack[kStack<D> * kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  Cnt cn;
  Q2Query<D, false> q;
  q.x = vload<D>(x + i * D);
  Key k = make_key(rmax[i] * rmax[i], -1);
  if (S.nE > 0) k = traverse<Q2Query<D, false>, false>(S, q, k, stack + threadIdx.x, cn);
  d[i] = key_slot(k) >= 0 ? sqrtf(key_value(k)) : rmax[i];
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_probe_q3(SceneDev S, const float* o, const float* v,
                                                     const float* tmax, const int* skip, int64_t n,
                                                     float* t, int* prim) {
  __shared__ int stack[kStack<D> * kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  RayQuery<D, false, false> q;
  q.R = make_ray<D>(vload<D>(o + i * D), vload<D>(v + i * D));
  q.tmax = tmax[i];
  q.skip = skip[i] >= 0 ? S.ninv[skip[i]] : -1;
  Cnt cn;
  Key k = make_key(tmax[i], -1);
  if (S.nN > 0) k = traverse<RayQuery<D, false, false>, false>(S, q, k, stack + threadIdx.x, cn);
  const int p = key_slot(k);
  t[i] = p >= 0 ? key_value(k) : tmax[i];
  prim[i] = p >= 0 ? S.nid[p] : -1;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_probe_q4(SceneDev S, const float* x, const float* r,
                                                     int64_t n, uint32_t k0, uint32_t k1, float* z,
                                                     float* pdf, int* prim) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  Vec<D> zz;
  float pp, wb, wc;
  const uint4 ctr = make_uint4((uint32_t)i, 0u, 0u, 0u);
  Cnt cn;
  const int p = q4_sample<D, false>(S, vload<D>(x + i * D), r[i], ctr, k0, k1, zz, pp, wb, wc, cn);
  for (int k = 0; k < D; ++k) z[i * D + k] = p >= 0 ? zz[k] : 0.0f;
  pdf[i] = p >= 0 ? pp : 0.0f;
  prim[i] = p >= 0 ? S.nid[p] : -1;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_walks(const SceneDev& S, const WalkParams& P, int mode, int grid, bool count,
                        hipStream_t s) {
  if (S.dim == 2)
    return S.ds ? WalkPart<2, true>::walks(S, P, mode, grid, count, s)
                : WalkPart<2, false>::walks(S, P, mode, grid, count, s);
  return S.ds ? WalkPart<3, true>::walks(S, P, mode, grid, count, s)
              : WalkPart<3, false>::walks(S, P, mode, grid, count, s);
}

hipError_t launch_batch(const BatchItem* it, const BatchGroupDev* g, int dim, bool hh, bool hf, bool ds,
                        unsigned long long* cur, unsigned long long* st, int grid, hipStream_t s) {
  if (dim == 2)
    return ds ? WalkPart<2, true>::batch(it, g, hh, hf, cur, st, grid, s)
              : WalkPart<2, false>::batch(it, g, hh, hf, cur, st, grid, s);
  return ds ? WalkPart<3, true>::batch(it, g, hh, hf, cur, st, grid, s)
            : WalkPart<3, false>::batch(it, g, hh, hf, cur, st, grid, s);
}

// batched reduction: global point gp of the batch belongs to the item whose
// [point_begin, point_begin + n_points) holds it; one wave per point, the
// same fixed order and arithmetic as k_reduce
__global__ __launch_bounds__(256) void k_reduce_batch(const BatchItem* __restrict__ items,
                                                      const BatchHeadDev* __restrict__ head) {
  const int n_items = head->n_items_all;
  const int64_t total = head->points;
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t gp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); gp < total; gp += waves) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].point_begin <= gp) lo = mid;
      else hi = mid - 1;
    }
    const BatchItem& it = items[lo];
    const int64_t pt = gp - it.point_begin;
    const int W = it.P.W;
    const float* e = it.P.est + pt * (int64_t)W;
    double s = 0.0;
    for (int j = lane; j < W; j += 64) s += (double)e[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const double m = s / (double)W;
    double q = 0.0;
    for (int j = lane; j < W; j += 64) {
      const double d = (double)e[j] - m;
      q += d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
    if (lane == 0) {
      it.mean[pt] = m;
      it.var[pt] = W > 1 ? q / (double)(W - 1) : 0.0;
    }
  }
}

hipError_t launch_reduce_batch(const BatchItem* d_items, const BatchHeadDev* d_head, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_batch, dim3(2048), dim3(256), 0, s, d_items, d_head);
  return hipGetLastError();
}

hipError_t launch_trace(const SceneDev& S, const WalkParams& P, const uint32_t* pids,
                        const uint32_t* wids, int64_t n, int max_rec, StepRec* recs, int* ns,
                        float* vals, hipStream_t s) {
  if (S.dim == 2)
    return S.ds ? WalkPart<2, true>::trace(S, P, pids, wids, n, max_rec, recs, ns, vals, s)
                : WalkPart<2, false>::trace(S, P, pids, wids, n, max_rec, recs, ns, vals, s);
  return S.ds ? WalkPart<3, true>::trace(S, P, pids, wids, n, max_rec, recs, ns, vals, s)
              : WalkPart<3, false>::trace(S, P, pids, wids, n, max_rec, recs, ns, vals, s);
}

int max_resident_blocks(int dim, bool coop) {
  const int nb = dim == 2 ? WalkPart<2, false>::resident_blocks(coop) : WalkPart<3, false>::resident_blocks(coop);
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus < 1) cus = 1;
  return nb * cus;
}

hipError_t launch_reduce(const float* est, int64_t n, int W, double* mean, double* var,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, est, n, W, mean, var);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

// ---- L2 read bandwidth ----------------------------------------------------
// Every block reads the whole buffer `reps` times in float4s, starting at a
// block-dependent offset so that the blocks of one CU are at different
// places (the 32 KiB L1 cannot serve them); a buffer of a few MiB stays in
// each XCD's 4 MiB L2 after the first pass.  The sum is written only if it
// takes an impossible value, which keeps the loads alive.
__global__ __launch_bounds__(256) void k_stream_read(const float4* __restrict__ buf, int n4, int reps,
                                                     float* sink) {
  float acc = 0.0f;
  const int start = (int)(((int64_t)blockIdx.x * 7919 * 256) % n4);
  for (int r = 0; r < reps; ++r)
    for (int i = threadIdx.x; i < n4; i += 256) {
      int j = start + i;
      if (j >= n4) j -= n4;
      const float4 v = buf[j];
      acc += (v.x + v.y) + (v.z + v.w);
    }
  if (acc == -1.0f) sink[blockIdx.x] = acc;
}

hipError_t launch_stream_read(const float4* buf, int n4, int reps, int blocks, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, s, buf, n4, reps, sink);
  return hipGetLastError();
}

// VALU issue calibration: every lane runs 8 independent chains of `iters`
// fused multiply-adds (8 * iters v_fma_f32 per lane, no memory traffic in
// the loop; unpacked, as the walk kernels are built)
__global__ __launch_bounds__(256) void k_valu_peak(int iters, float a, float* sink) {
  const float b = (float)(threadIdx.x & 7) * 1e-3f;
  float x0 = b, x1 = b + 1.0f, x2 = b + 2.0f, x3 = b + 3.0f, x4 = b + 4.0f, x5 = b + 5.0f, x6 = b + 6.0f,
        x7 = b + 7.0f;
  for (int i = 0; i < iters; ++i) {
    x0 = fmaf(x0, a, 0.5f);
    x1 = fmaf(x1, a, 0.5f);
    x2 = fmaf(x2, a, 0.5f);
    x3 = fmaf(x3, a, 0.5f);
    x4 = fmaf(x4, a, 0.5f);
    x5 = fmaf(x5, a, 0.5f);
    x6 = fmaf(x6, a, 0.5f);
    x7 = fmaf(x7, a, 0.5f);
  }
  const float t = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
  if (t == -1.0f) sink[blockIdx.x] = t;
}

// the same with integer work: 8 independent chains of an xor and an add
// (2 * 8 * iters VALU instructions per lane)
__global__ __launch_bounds__(256) void k_valu_peak_int(int iters, uint32_t a, float* sink) {
  uint32_t x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = threadIdx.x + (uint32_t)j;
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (x[j] ^ a) + 0x9E3779B9u;
  uint32_t t = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) t ^= x[j];
  if (t == 12345u) sink[blockIdx.x] = (float)t;
}

hipError_t launch_valu_peak(int kind, int iters, int blocks, float* sink, hipStream_t s) {
  if (kind == 1)
    hipLaunchKernelGGL(k_valu_peak_int, dim3(blocks), dim3(256), 0, s, iters, 12345u, sink);
  else
    hipLaunchKernelGGL(k_valu_peak, dim3(blocks), dim3(256), 0, s, iters, 0.9999f, sink);
  return hipGetLastError();
}

hipError_t launch_probe_q1(const SceneDev& S, const float* x, int64_t n, float* d, float* xbar,
                           int* prim, hipStream_t s) {
  if (S.dim == 2)
    hipLaunchKernelGGL(k_probe_q1<2>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, x, n, d, xbar, prim);
  else
    hipLaunchKernelGGL(k_probe_q1<3>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, x, n, d, xbar, prim);
  return hipGetLastError();
}

hipError_t launch_probe_q2(const SceneDev& S, const float* x, const float* rmax, int64_t n,
                           float* d, hipStream_t s) {
  if (S.dim == 2)
    hipLaunchKernelGGL(k_probe_q2<2>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, x, rmax, n, d);
  else
    hipLaunchKernelGGL(k_probe_q2<3>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, x, rmax, n, d);
  return hipGetLastError();
}

hipError_t launch_probe_q3(const SceneDev& S, const float* o, const float* v, const float* tmax,
                           const int* skip, int64_t n, float* t, int* prim, hipStream_t s) {
  if (S.dim == 2)
    hipLaunchKernelGGL(k_probe_q3<2>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, o, v, tmax, skip, n,
                       t, prim);
  else
    hipLaunchKernelGGL(k_probe_q3<3>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, o, v, tmax, skip, n,
                       t, prim);
  return hipGetLastError();
}

hipError_t launch_probe_q4(const SceneDev& S, const float* x, const float* r, int64_t n,
                           uint32_t k0, uint32_t k1, float* z, float* pdf, int* prim,
                           hipStream_t s) {
  if (S.dim == 2)
    hipLaunchKernelGGL(k_probe_q4<2>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, x, r, n, k0, k1, z,
                       pdf, prim);
  else
    hipLaunchKernelGGL(k_probe_q4<3>, dim3(blocks_for(n)), dim3(kBlock), 0, s, S, x, r, n, k0, k1, z,
                       pdf, prim);
  return hipGetLastError();
}

}  // namespace wost
