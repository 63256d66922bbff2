// Device-side building blocks: wave reductions, deterministic grid
// reductions (per-block partial + last-block finish), XCD-aware work ranges.
#pragma once

#include "common.hpp"

namespace mgpbd {

// Fixed-tree sum over a group of G lanes (G a power of two <= 64) inside a
// wavefront; every lane of the group receives the total. Deterministic.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(G >= 1 && G <= 64, "group size");
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

template <int G>
__device__ __forceinline__ uint64_t group_max_u64(uint64_t v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(v, off, G);
    v = o > v ? o : v;
  }
  return v;
}

// Logical block index that keeps consecutive chunks of work on the same XCD:
// hardware block b runs on XCD b % 8; the 8 XCDs get contiguous ranges.
__device__ __forceinline__ int xcd_block() {
  int g = gridDim.x, b = blockIdx.x;
  if (g < kNumXcd) return b;
  int per = g / kNumXcd;
  int rem = g % kNumXcd;          // XCDs x < rem own one extra block
  int x = b % kNumXcd, k = b / kNumXcd;
  int base = x * per + (x < rem ? x : rem);
  return base + k;
}

// Contiguous range of `items` handled by this block (XCD-aware order).
__device__ __forceinline__ void block_range(int64_t items, int64_t &lo, int64_t &hi) {
  int64_t g = gridDim.x;
  int64_t per = (items + g - 1) / g;
  int64_t lb = xcd_block();
  lo = lb * per;
  hi = lo + per;
  if (hi > items) hi = items;
  if (lo > items) lo = items;
}

// The items of this block's XCD (the union of block_range over the XCD's
// blocks) visited in lockstep: the XCD's bpx blocks take consecutive chunks
// of `chunk` items, block j the j-th chunk of every window of bpx chunks, so
// the whole XCD sweeps one window at a time. Data shared by nearby items
// (the vertex records of a row pass, the gathered entries of a vertex gather)
// is then reused within a short time and stays in the XCD's L2, where
// contiguous per-block ranges revisit it only after the XCD has streamed many
// megabytes. Every item is visited exactly once: loop
// for (c0 = first; c0 < hi; c0 += step) over items [c0, min(c0 + chunk, hi)).
struct XcdStride {
  int64_t hi, first, step;
};
__device__ __forceinline__ XcdStride xcd_stride(int64_t items, int64_t chunk) {
  const int g = gridDim.x, b = blockIdx.x;
  const int per = g / kNumXcd, rem = g % kNumXcd;
  const int x = b % kNumXcd, j = b / kNumXcd;
  const int bpx = per + (x < rem ? 1 : 0);
  const int base = x * per + (x < rem ? x : rem);
  const int64_t perb = (items + g - 1) / g;
  int64_t lo = (int64_t)base * perb, hi = (int64_t)(base + bpx) * perb;
  if (lo > items) lo = items;
  if (hi > items) hi = items;
  return {hi, lo + (int64_t)j * chunk, (int64_t)bpx * chunk};
}

// Deterministic grid-wide reductions in two kernels. The producing kernel
// calls block_partials (fixed-tree sum per block, one partial per block); a
// one-block finisher kernel calls sum_partials, which adds the partials in a
// fixed order. No device-scope fence is needed inside a kernel: the kernel
// boundary makes the partials visible (a device-scope fence inside the kernel
// would write back the XCD's L2 from every block).
template <int NV>
__device__ void block_partials(const double (&v)[NV], double *partials) {
  static_assert(NV <= kMaxBlockSums, "the partials buffer holds kMaxBlockSums sums per block");
  __shared__ double sh[NV][kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = group_sum<kWave>(v[k]);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = sh[k][0];
      for (int q = 1; q < nw; ++q) s += sh[k][q];
      partials[(size_t)k * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Called by every thread of a single block of kBlock threads; out[k] holds
// the total of the nparts partials of value k in every thread.
template <int NV>
__device__ void sum_partials(const double *partials, int nparts, double (&out)[NV]) {
  __shared__ double sh[NV][kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int q = threadIdx.x; q < nparts; q += blockDim.x) s += partials[(size_t)k * nparts + q];
    s = group_sum<kWave>(s);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double tot = sh[k][0];
    for (int q = 1; q < nw; ++q) tot += sh[k][q];
    out[k] = tot;
  }
}

// PCG control block in device memory (one per solve context).
struct PcgCtl {
  int done;        // 0 running, 1 converged, 2 breakdown, 3 forced count reached, 4 cap
  int iters;       // completed iterations
  int force;       // >0: stop after exactly this many iterations
  int max_iters;
  double bnorm;    // |b|
  double tol;
  double rho;      // r^T z
  double pq;       // p^T A p
  double alpha;
  double rr;       // r^T r
  double beta;
  double ratio;    // |r| / |b|
};

}  // namespace mgpbd
