// Fused coarse end of the V-cycle (Sec. 4.4-4.5): from a start level down to
// each body's dense coarsest solve and back up, in one launch with one
// workgroup per body. Below a few thousand rows a level's passes are too
// small to fill the GPU and each separate launch costs about as much as its
// work; bodies are independent on every level (block-diagonal system), so
// one workgroup can run a body's whole coarse recursion with barriers in
// between passes. Every pass sums in the same lane order and fixed tree as
// the per-level kernels (k_rows, k_restrict, k_prolong, k_dense_apply_batch),
// so the fused form computes the same bits.
#pragma once

#include "kernels.hpp"

namespace mgpbd {

constexpr int kTailBlock = 512;     // threads of the workgroup that runs one body
constexpr int kTailMaxDepth = 16;   // levels a body may have inside the tail

// One level of the tail (device pointers of that level's arrays).
template <class T>
struct TailLevel {
  const int64_t *rp = nullptr;
  const int32_t *col = nullptr;
  const T *val = nullptr;
  const T *wdinv = nullptr;      // omega(body) / a_ii
  const T *dinv = nullptr;       // 1 / a_ii (Chebyshev)
  const T *cheb = nullptr;       // Chebyshev coefficients [segment][steps][2]
  const int32_t *rowseg = nullptr;
  int G = 8;                     // lanes per row of the level's row passes
  int rlanes = 8;                // lanes per aggregate of its restriction
  // transfer to the next level (unused on a body's last level)
  const T *p = nullptr;
  const int32_t *agg = nullptr;
  const int64_t *agg_ptr = nullptr;
  const int32_t *agg_mem = nullptr;
  // V-cycle vectors: right-hand side, iterate, scratch iterate, residual,
  // Chebyshev direction
  T *r = nullptr, *z = nullptr, *t = nullptr, *res = nullptr, *dir = nullptr;
};

// One body inside the tail: its rows on each tail level (the last one is
// solved with its dense inverse) and that inverse's offset and size.
struct TailBody {
  int32_t depth = 0;                 // tail levels of the body (>= 1)
  int64_t row0[kTailMaxDepth] = {};  // first row on each tail level
  int64_t n[kTailMaxDepth] = {};     // rows on each tail level
  int64_t ainv = 0;                  // offset of its dense inverse (n[depth-1]^2 values)
};

// Smoothing schedule of the tail (the one vcycle() uses).
struct TailPlan {
  int pre = 2, post = 2;
  int smoother = 0;      // 0 = omega-Jacobi, 1 = Chebyshev
  int steps = 2;         // Chebyshev steps per smoothing pass
  bool fuse_first = true;  // Jacobi: the first two sweeps from zero as one pass
};

template <class T>
void launch_vcycle_tail(int nbodies, const TailLevel<T> *levels, const TailBody *bodies,
                        const TailPlan &plan, const double *ainv, const int *done,
                        hipStream_t s);

}  // namespace mgpbd
