// Device-side building blocks: wave reductions, deterministic grid
// reductions (per-block partial + last-block finish), XCD-aware work ranges.
#pragma once

#include "common.hpp"

namespace mgpbd {

// Fixed-tree sum over a group of G lanes (G a power of two <= 64) inside a
// wavefront; every lane of the group receives the total. Deterministic.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
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

// Coherent (L1-bypassing) load of a value written by another block of the
// same kernel before its __threadfence().
__device__ __forceinline__ double load_agent(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Deterministic grid-wide reduction of NV doubles. Every block calls
// grid_reduce with its threads' values; it returns true in exactly one block
// (the last to finish) with out[k] holding the grand totals in every thread.
// The per-block sum and the final sum follow fixed trees, so the result does
// not depend on scheduling. partials must hold NV * gridDim.x doubles; ticket
// starts at 0 and is reset by the last block.
template <int NV>
__device__ bool grid_reduce(const double (&v)[NV], double *partials, unsigned *ticket,
                            double (&out)[NV]) {
  __shared__ double sh[NV][kBlock / kWave];
  __shared__ bool last;
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
    __threadfence();
    unsigned t = atomicAdd(ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x)
      s += load_agent(partials + (size_t)k * gridDim.x + q);
    s = group_sum<kWave>(s);
    __syncthreads();
    if (lane == 0) sh[k][w] = s;
    __syncthreads();
    double tot = sh[k][0];
    for (int q = 1; q < nw; ++q) tot += sh[k][q];
    out[k] = tot;
  }
  if (threadIdx.x == 0) *ticket = 0u;
  return true;
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
