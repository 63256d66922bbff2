// Sparse kernels of the solving phase (Sec. 4.4-4.5): CSR products with G
// lanes per row and fixed-tree group sums, the omega-Jacobi smoother, the
// residual, restriction / prolongation through the aggregate lists, the
// dense coarsest solve, and the FP64 PCG loop with deterministic grid
// reductions and a device-resident control block (no host round trip per
// iteration; every kernel returns at once when the solve is finished).
#include <algorithm>

#include "kernels.hpp"
#include "rowops.hpp"

namespace mgpbd {

int lanes_for_rowlen(double mean) {
  if (mean >= 96.0) return 32;
  if (mean >= 24.0) return 16;
  if (mean >= 10.0) return 8;
  return 4;
}

#define MG_DISPATCH_G(lanes, LAUNCH) \
  switch (lanes) {                   \
    case 4: LAUNCH(4); break;        \
    case 8: LAUNCH(8); break;        \
    case 16: LAUNCH(16); break;      \
    case 32: LAUNCH(32); break;      \
    default: LAUNCH(64); break;      \
  }

// Row-group kernel: G lanes per row, strided loads, fixed-tree lane sum.
template <int G, class T, class In, class Op>
__global__ __launch_bounds__(kBlock) void k_rows(const int *done, int64_t n,
                                                 const int64_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col,
                                                 const T *__restrict__ val, In x, Op op,
                                                 double *partials) {
  if (done && *done) return;
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(n, lo, hi);
  double acc = 0.0;
  for (int64_t base = lo; base < hi; base += R) {
    int64_t i = base + grp;
    bool ok = i < hi;
    int64_t a = ok ? rp[i] : 0, b = ok ? rp[i + 1] : 0;
    T s = 0;
#pragma unroll 4
    for (int64_t e = a + sub; e < b; e += G) s += val[e] * x(col[e]);
    s = group_sum<G, T>(s);
    if (ok && sub == 0) op(i, s, acc);
  }
  if (partials) {
    double v[1] = {acc};
    block_partials<1>(v, partials);
  }
}

// Stream kernel: a block walks a contiguous range of row tiles; for each tile
// all threads first load the tile's entries with independent coalesced loads
// (TILE / kBlock per thread) and stage the products in LDS, then 8 lanes per
// row add the row's segment and apply the epilogue.
template <bool NT, class V>
__device__ __forceinline__ V stream_load(const V *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <int TILE, bool NT, class T, class In, class Op>
__global__ __launch_bounds__(kBlock) void k_stream(const int *done, int64_t ntiles,
                                                   const int64_t *__restrict__ tiles,
                                                   const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const T *__restrict__ val, In x, Op op,
                                                   double *partials) {
  if (done && *done) return;
  constexpr int PER = TILE / kBlock;
  constexpr int LR = 8;                 // lanes per row in the reduction
  __shared__ T prod[TILE];
  int64_t t_lo, t_hi;
  block_range(ntiles, t_lo, t_hi);
  double acc = 0.0;
  for (int64_t t = t_lo; t < t_hi; ++t) {
    const int64_t r0 = tiles[t], r1 = tiles[t + 1];
    const int64_t e0 = rp[r0], e1 = rp[r1];
    int32_t c[PER];
    T v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int64_t e = e0 + threadIdx.x + (int64_t)j * kBlock;
      bool in = e < e1;
      // matrix entries are read once per pass: non-temporal loads keep the
      // L2 for the gathered vector
      c[j] = in ? stream_load<NT>(col + e) : 0;
      v[j] = in ? stream_load<NT>(val + e) : (T)0;
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) prod[threadIdx.x + j * kBlock] = v[j] * x(c[j]);
    __syncthreads();
    const int sub = threadIdx.x % LR;
    for (int64_t base = r0; base < r1; base += kBlock / LR) {
      int64_t i = base + threadIdx.x / LR;
      bool ok = i < r1;
      T s = 0;
      if (ok) {
        int a = (int)(rp[i] - e0), b = (int)(rp[i + 1] - e0);
        for (int k = a + sub; k < b; k += LR) s += prod[k];
      }
      s = group_sum<LR, T>(s);
      if (ok && sub == 0) op(i, s, acc);
    }
    __syncthreads();
  }
  if (partials) {
    double vv[1] = {acc};
    block_partials<1>(vv, partials);
  }
}

// SELL-C-sigma kernel: one wavefront per chunk of 64 rows, lane t owns slot
// t of the chunk and adds its row's entries in column order (padding adds
// exact zeros), then applies the epilogue to the row it holds.
template <class T, class In, class Op>
__global__ __launch_bounds__(kBlock) void k_sell(const int *done, SellView<T> S, In x, Op op,
                                                 double *partials) {
  if (done && *done) return;
  constexpr int WPB = kBlock / kWave;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  int64_t lo, hi;
  block_range(S.nchunks, lo, hi);
  double acc = 0.0;
  for (int64_t c = lo + wv; c < hi; c += WPB) {
    const int64_t b = S.ptr[c], len = (S.ptr[c + 1] - b) / kSellC;
    const int32_t row = S.perm[c * kSellC + lane];
    T s = 0;
    for (int64_t k = 0; k < len; ++k) {
      const int64_t e = b + k * kSellC + lane;
      s += S.val[e] * x(S.col[e]);
    }
    if (row >= 0) op(row, s, acc);
  }
  if (partials) {
    double v[1] = {acc};
    block_partials<1>(v, partials);
  }
}

void build_sell(const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                std::vector<int32_t> &perm, std::vector<int64_t> &ptr,
                std::vector<int32_t> &scol, std::vector<int64_t> &slot) {
  const int64_t n = (int64_t)rp.size() - 1;
  const int64_t nchunks = (n + kSellC - 1) / kSellC;
  perm.assign(nchunks * kSellC, -1);
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  for (int64_t w0 = 0; w0 < n; w0 += kSellSigma) {
    const int64_t w1 = std::min<int64_t>(n, w0 + kSellSigma);
    std::stable_sort(order.begin() + w0, order.begin() + w1, [&](int32_t a, int32_t b) {
      return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
    });
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = order[i];
  ptr.assign(nchunks + 1, 0);
  for (int64_t c = 0; c < nchunks; ++c) {
    int64_t len = 0;
    for (int t = 0; t < kSellC; ++t) {
      const int32_t r = perm[c * kSellC + t];
      if (r >= 0) len = std::max<int64_t>(len, rp[r + 1] - rp[r]);
    }
    ptr[c + 1] = ptr[c] + len * kSellC;
  }
  scol.assign(ptr[nchunks], 0);
  slot.assign(rp[n], 0);
  for (int64_t c = 0; c < nchunks; ++c)
    for (int t = 0; t < kSellC; ++t) {
      const int32_t r = perm[c * kSellC + t];
      if (r < 0) continue;
      for (int64_t k = 0; k < rp[r + 1] - rp[r]; ++k) {
        const int64_t pos = ptr[c] + k * kSellC + t;
        scol[pos] = col[rp[r] + k];
        slot[rp[r] + k] = pos;
      }
    }
}

template <class S, class T>
__global__ void k_sell_values(int64_t nnz, const int64_t *__restrict__ slot,
                              const S *__restrict__ val, T *__restrict__ sval) {
  int64_t lo, hi;
  block_range(nnz, lo, hi);
  for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) sval[slot[e]] = (T)val[e];
}
template <class S, class T>
void launch_sell_values(int64_t nnz, const int64_t *slot, const S *val, T *sval, hipStream_t s) {
  if (nnz) k_sell_values<S, T><<<grid_for(nnz, kBlock), kBlock, 0, s>>>(nnz, slot, val, sval);
}
template void launch_sell_values<double, double>(int64_t, const int64_t *, const double *,
                                                 double *, hipStream_t);
template void launch_sell_values<double, float>(int64_t, const int64_t *, const double *,
                                                float *, hipStream_t);
template void launch_sell_values<float, float>(int64_t, const int64_t *, const float *, float *,
                                               hipStream_t);

#define MG_DISPATCH_TILE(tile, LAUNCH) \
  switch (tile) {                      \
    case 1024: LAUNCH(1024); break;    \
    case 4096: LAUNCH(4096); break;    \
    default: LAUNCH(2048); break;      \
  }

template <class T, class In, class Op>
static int launch_pass(const CsrView<T> &A, In x, Op op, const int *done, double *partials,
                       hipStream_t s) {
  if (A.n == 0) return 0;
  if (A.sell.val) {
    const int grid = grid_for(A.sell.nchunks * kWave, kBlock);
    k_sell<T, In, Op><<<grid, kBlock, 0, s>>>(done, A.sell, x, op, partials);
    return grid;
  }
  if (A.tile > 0) {
    int grid = grid_for(A.ntiles, 1);
    if (A.nt) {
#define L_(TL) k_stream<TL, true, T, In, Op><<<grid, kBlock, 0, s>>>(done, A.ntiles, A.tiles, A.rowptr, A.col, A.val, x, op, partials)
      MG_DISPATCH_TILE(A.tile, L_);
#undef L_
    } else {
#define L_(TL) k_stream<TL, false, T, In, Op><<<grid, kBlock, 0, s>>>(done, A.ntiles, A.tiles, A.rowptr, A.col, A.val, x, op, partials)
      MG_DISPATCH_TILE(A.tile, L_);
#undef L_
    }
    return grid;
  }
  int grid = grid_for(A.n * A.lanes, kBlock);
#define L_(G) k_rows<G, T, In, Op><<<grid, kBlock, 0, s>>>(done, A.n, A.rowptr, A.col, A.val, x, op, partials)
  MG_DISPATCH_G(A.lanes, L_);
#undef L_
  return grid;
}

bool build_row_tiles(const std::vector<int64_t> &rp, int tile, std::vector<int64_t> &tiles) {
  tiles.clear();
  const int64_t n = (int64_t)rp.size() - 1;
  int64_t r = 0;
  tiles.push_back(0);
  while (r < n) {
    int64_t start = rp[r];
    if (rp[r + 1] - start > tile) return false;
    int64_t q = r + 1;
    while (q < n && rp[q + 1] - start <= tile) ++q;
    tiles.push_back(q);
    r = q;
  }
  return true;
}

// ------------------------------------------------------------------ SpMV
template <class T>
void launch_spmv(const CsrView<T> &A, const T *x, T *y, hipStream_t s) {
  launch_pass<T>(A, InVec<T>{x}, OpSpmv<T>{y}, nullptr, nullptr, s);
}

int launch_spmv_dot_partials(const CsrView<double> &A, const double *p, double *q,
                             const int *done, double *partials, hipStream_t s) {
  return launch_pass<double>(A, InVec<double>{p}, OpPcgDot{p, q}, done, partials, s);
}

// ------------------------------------------------------------ smoother
template <class T>
__global__ __launch_bounds__(kBlock) void k_jacobi_first(int64_t n, const T *__restrict__ wdinv,
                                                         const T *__restrict__ r,
                                                         T *__restrict__ z, const int *done) {
  if (done && *done) return;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) z[i] = r[i] * wdinv[i];
}

template <class T>
void launch_jacobi_first(int64_t n, const T *wdinv, const T *r, T *z, const int *done,
                         hipStream_t s) {
  if (n == 0) return;
  k_jacobi_first<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, wdinv, r, z, done);
}
template <class T>
void launch_jacobi(const CsrView<T> &A, const T *wdinv, const T *r, const T *zi, T *zo,
                   const int *done, hipStream_t s) {
  launch_pass<T>(A, InVec<T>{zi}, OpJacobi<T, InVec<T>>{wdinv, r, InVec<T>{zi}, zo}, done,
                 nullptr, s);
}
template <class T>
void launch_jacobi_scaled(const CsrView<T> &A, const T *wdinv, const T *r, T *zo,
                          const int *done, hipStream_t s) {
  const InScaled<T> in{r, wdinv};
  launch_pass<T>(A, in, OpJacobi<T, InScaled<T>>{wdinv, r, in, zo}, done, nullptr, s);
}
// first Chebyshev step from z = 0: d = c2 D^-1 r, z = d
template <class T>
__global__ __launch_bounds__(kBlock) void k_cheb_first(int64_t n, const T *__restrict__ r,
                                                       const T *__restrict__ dinv,
                                                       const T *__restrict__ coef,
                                                       const int32_t *__restrict__ rowseg,
                                                       int steps, T *__restrict__ d,
                                                       T *__restrict__ z, const int *done) {
  if (done && *done) return;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const T c2 = coef[2 * (int64_t)(rowseg ? rowseg[i] : 0) * steps + 1];
    const T dn = c2 * (r[i] * dinv[i]);
    d[i] = dn;
    z[i] = dn;
  }
}
template <class T>
void launch_cheb_first(int64_t n, const T *r, const T *dinv, const T *coef,
                       const int32_t *rowseg, int steps, T *d, T *z, const int *done,
                       hipStream_t s) {
  if (n == 0) return;
  k_cheb_first<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, r, dinv, coef, rowseg, steps, d, z,
                                                         done);
}
template <class T>
void launch_cheb(const CsrView<T> &A, const T *r, const T *dinv, const T *coef,
                 const int32_t *rowseg, int steps, int k, const T *zi, T *d, T *zo,
                 const int *done, hipStream_t s) {
  const InVec<T> in{zi};
  launch_pass<T>(A, in, OpCheb<T, InVec<T>>{r, dinv, d, zo, coef, rowseg, steps, k, in}, done,
                 nullptr, s);
}

template <class T>
void launch_jacobi_prolong(const CsrView<T> &A, const T *wdinv, const T *r, const T *zi,
                           const T *p, const int32_t *agg, const T *e, T *zo, const int *done,
                           hipStream_t s) {
  const InProlong<T> in{zi, p, e, agg};
  launch_pass<T>(A, in, OpJacobi<T, InProlong<T>>{wdinv, r, in, zo}, done, nullptr, s);
}
template <class T>
void launch_cheb_prolong(const CsrView<T> &A, const T *r, const T *dinv, const T *coef,
                         const int32_t *rowseg, int steps, int k, const T *zi, const T *p,
                         const int32_t *agg, const T *e, T *d, T *zo, const int *done,
                         hipStream_t s) {
  const InProlong<T> in{zi, p, e, agg};
  launch_pass<T>(A, in, OpCheb<T, InProlong<T>>{r, dinv, d, zo, coef, rowseg, steps, k, in},
                 done, nullptr, s);
}

// Residual and restriction in one pass: G lanes per aggregate walk its member
// rows in ascending order; each row's product sums with the fixed lane tree of
// k_rows, and the aggregate's sum adds p_i (r_i - (A z)_i) member by member.
template <int G, class T>
__global__ __launch_bounds__(kBlock) void k_residual_restrict(
    const int *done, int64_t na, const int64_t *__restrict__ ap, const int32_t *__restrict__ mem,
    const int64_t *__restrict__ rp, const int32_t *__restrict__ col, const T *__restrict__ val,
    const T *__restrict__ r, const T *__restrict__ z, const T *__restrict__ p,
    T *__restrict__ rc) {
  if (done && *done) return;
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(na, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    const int64_t a = base + grp;
    const bool ok = a < hi;
    const int64_t m0 = ok ? ap[a] : 0, m1 = ok ? ap[a + 1] : 0;
    T acc = 0;
    for (int64_t t = m0; t < m1; ++t) {
      const int32_t i = mem[t];
      const int64_t e0 = rp[i], e1 = rp[i + 1];
      T s = 0;
#pragma unroll 4
      for (int64_t e = e0 + sub; e < e1; e += G) s += val[e] * z[col[e]];
      s = group_sum<G, T>(s);
      acc += p[i] * (r[i] - s);
    }
    if (ok && sub == 0) rc[a] = acc;
  }
}
template <class T>
void launch_residual_restrict(const CsrView<T> &A, const T *r, const T *z, int64_t na,
                              const int64_t *ap, const int32_t *mem, const T *p, T *rc,
                              const int *done, hipStream_t s) {
  if (na == 0) return;
  const int G = A.lanes;
  const int grid = grid_for(na * G, kBlock);
#define L_(GG) k_residual_restrict<GG, T><<<grid, kBlock, 0, s>>>(done, na, ap, mem, A.rowptr, \
                                                                 A.col, A.val, r, z, p, rc)
  MG_DISPATCH_G(G, L_);
#undef L_
}

template <class T>
void launch_residual(const CsrView<T> &A, const T *r, const T *z, T *res, const int *done,
                     hipStream_t s) {
  launch_pass<T>(A, InVec<T>{z}, OpResidual<T>{r, res}, done, nullptr, s);
}

// ------------------------------------------------------------ transfers
template <int G, class T>
__global__ __launch_bounds__(kBlock) void k_restrict(int64_t na, const int64_t *__restrict__ ap,
                                                     const int32_t *__restrict__ mem,
                                                     const T *__restrict__ p,
                                                     const T *__restrict__ res,
                                                     T *__restrict__ rc, const int *done,
                                                     CoarseFirst<T> first) {
  if (done && *done) return;
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(na, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t a = base + grp;
    bool ok = a < hi;
    int64_t b0 = ok ? ap[a] : 0, b1 = ok ? ap[a + 1] : 0;
    T s = 0;
    for (int64_t k = b0 + sub; k < b1; k += G) {
      int32_t i = mem[k];
      s += p[i] * res[i];
    }
    s = group_sum<G>(s);
    if (ok && sub == 0) {
      rc[a] = s;
      if (first.z) first.z[a] = s * first.wd[a];
    }
  }
}

// the restriction's member sums when the terms p_i res_i are already stored
// (same lanes, order and tree as k_restrict, so the same bits)
template <int G, class T>
__global__ __launch_bounds__(kBlock) void k_restrict_sum(int64_t na,
                                                         const int64_t *__restrict__ ap,
                                                         const int32_t *__restrict__ mem,
                                                         const T *__restrict__ w,
                                                         T *__restrict__ rc, const int *done,
                                                         CoarseFirst<T> first) {
  if (done && *done) return;
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(na, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t a = base + grp;
    bool ok = a < hi;
    int64_t b0 = ok ? ap[a] : 0, b1 = ok ? ap[a + 1] : 0;
    T s = 0;
    for (int64_t k = b0 + sub; k < b1; k += G) s += w[mem[k]];
    s = group_sum<G>(s);
    if (ok && sub == 0) {
      rc[a] = s;
      if (first.z) first.z[a] = s * first.wd[a];
    }
  }
}
template <class T>
void launch_restrict_sum(int64_t na, const int64_t *ap, const int32_t *mem, const T *w, T *rc,
                         int lanes, const int *done, hipStream_t s, CoarseFirst<T> first) {
  if (na == 0) return;
  const int grid = grid_for(na * lanes, kBlock);
  switch (lanes) {
    case 64:
      k_restrict_sum<64, T><<<grid, kBlock, 0, s>>>(na, ap, mem, w, rc, done, first);
      break;
    case 32:
      k_restrict_sum<32, T><<<grid, kBlock, 0, s>>>(na, ap, mem, w, rc, done, first);
      break;
    case 16:
      k_restrict_sum<16, T><<<grid, kBlock, 0, s>>>(na, ap, mem, w, rc, done, first);
      break;
    default:
      k_restrict_sum<8, T><<<grid, kBlock, 0, s>>>(na, ap, mem, w, rc, done, first);
      break;
  }
}

template <class T>
void launch_restrict(int64_t na, const int64_t *ap, const int32_t *mem, const T *p, const T *res,
                     T *rc, int lanes, const int *done, hipStream_t s, CoarseFirst<T> first) {
  if (na == 0) return;
  const int grid = grid_for(na * lanes, kBlock);
  switch (lanes) {
    case 64:
      k_restrict<64, T><<<grid, kBlock, 0, s>>>(na, ap, mem, p, res, rc, done, first);
      break;
    case 32:
      k_restrict<32, T><<<grid, kBlock, 0, s>>>(na, ap, mem, p, res, rc, done, first);
      break;
    case 16:
      k_restrict<16, T><<<grid, kBlock, 0, s>>>(na, ap, mem, p, res, rc, done, first);
      break;
    default:
      k_restrict<8, T><<<grid, kBlock, 0, s>>>(na, ap, mem, p, res, rc, done, first);
      break;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_prolong(int64_t n, const int32_t *__restrict__ agg,
                                                    const T *__restrict__ p,
                                                    const T *__restrict__ ec,
                                                    T *__restrict__ z, const int *done) {
  if (done && *done) return;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    int32_t a = agg[i];
    if (a >= 0) z[i] = z[i] + p[i] * ec[a];
  }
}

template <class T>
void launch_prolong(int64_t n, const int32_t *agg, const T *p, const T *ec, T *z, const int *done,
                    hipStream_t s) {
  if (n == 0) return;
  k_prolong<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, agg, p, ec, z, done);
}

// ------------------------------------------------------------ utilities
__global__ void k_d2f(int64_t n, const double *__restrict__ in, float *__restrict__ out,
                      const int *done) {
  if (done && *done) return;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) out[i] = (float)in[i];
}
void launch_d2f(int64_t n, const double *in, float *out, const int *done, hipStream_t s) {
  if (n) k_d2f<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, in, out, done);
}
template <class T>
__global__ void k_copy_t(int64_t n, const T *__restrict__ in, T *__restrict__ out, const int *done) {
  if (done && *done) return;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) out[i] = in[i];
}
template <class T>
void launch_copy_t(int64_t n, const T *in, T *out, const int *done, hipStream_t s) {
  if (n) k_copy_t<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, in, out, done);
}
template <class T>
__global__ void k_zero_t(int64_t n, T *__restrict__ out, const int *done) {
  if (done && *done) return;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) out[i] = (T)0;
}
template <class T>
void launch_zero_t(int64_t n, T *out, const int *done, hipStream_t s) {
  if (n) k_zero_t<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, out, done);
}
__global__ void k_copy(int64_t n, const double *__restrict__ in, double *__restrict__ out,
                       const int *done) {
  if (done && *done) return;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) out[i] = in[i];
}
void launch_copy(int64_t n, const double *in, double *out, const int *done, hipStream_t s) {
  if (n) k_copy<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, in, out, done);
}
template <class V>
__global__ void k_fill(int64_t n, V v, V *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = v;
}
void launch_fill(int64_t n, double v, double *out, hipStream_t s) {
  if (n) k_fill<double><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, v, out);
}
void launch_fill_i32(int64_t n, int32_t v, int32_t *out, hipStream_t s) {
  if (n) k_fill<int32_t><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, v, out);
}
void launch_fill_u8(int64_t n, uint8_t v, uint8_t *out, hipStream_t s) {
  if (n) k_fill<uint8_t><<<grid_for(n, kBlock), kBlock, 0, s>>>(n, v, out);
}

// ------------------------------------------------------------------ PCG
// Finisher of the fused product + dot of one solve (the other PCG kernels,
// for one body or several, are the segmented ones).
__global__ __launch_bounds__(kBlock) void k_fin_pq(PcgCtl *ctl, const double *partials,
                                                   int nparts) {
  if (ctl->done) return;
  double tot[1];
  sum_partials<1>(partials, nparts, tot);
  if (threadIdx.x == 0) {
    ctl->pq = tot[0];
    if (!(tot[0] > 0.0) || !(ctl->rho > 0.0)) ctl->done = 2;
    else ctl->alpha = ctl->rho / tot[0];
  }
}
void launch_fin_pq(PcgCtl *ctl, const double *partials, int nparts, hipStream_t s) {
  k_fin_pq<<<1, kBlock, 0, s>>>(ctl, partials, nparts);
}

// ------------------------------------------------------------------ scan
// Three-phase exclusive scan: block sums of 1024-element tiles, a scan of
// the tile sums (recursive), then the tile-local scan plus tile offset.
constexpr int kScanTile = 1024;

template <class In>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const In *in, int64_t n, int64_t *sums) {
  __shared__ int64_t sh[kBlock / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
    int64_t i = base + k;
    if (i < n) s += (int64_t)in[i];
  }
  s = group_sum<kWave>(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w];
    sums[blockIdx.x] = t;
  }
}

template <class In>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const In *in, int64_t n, const int64_t *offs,
                                                      int64_t *out) {
  // each thread owns 4 consecutive elements of the tile
  __shared__ int64_t sh[kBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 4;
  int64_t v[4];
  int64_t loc = 0;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + k;
    v[k] = (i < n) ? (int64_t)in[i] : 0;
    loc += v[k];
  }
  sh[threadIdx.x] = loc;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 256 thread sums
  for (int off = 1; off < kBlock; off <<= 1) {
    int64_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = offs[blockIdx.x] + sh[threadIdx.x] - loc;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (blockIdx.x == ntiles - 1 && threadIdx.x == kBlock - 1) out[n] = run;
}

template <class In>
static void scan_impl(const In *in, int64_t *out, int64_t n, DevBuf<int64_t> &tmp, size_t tmp_off,
                      hipStream_t s) {
  if (n == 0) {
    MG_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    return;
  }
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  // tmp layout from tmp_off: tile sums [ntiles], their exclusive scan [ntiles + 1]
  size_t need = tmp_off + 2 * (size_t)ntiles + 1;
  if (tmp.n < need) throw Error(MGPBD_E_SETUP, "scan scratch too small");
  int64_t *sums = tmp.p + tmp_off;
  int64_t *offs = sums + ntiles;
  k_tile_sums<In><<<(unsigned)ntiles, kBlock, 0, s>>>(in, n, sums);
  if (ntiles == 1) {
    MG_HIP(hipMemsetAsync(offs, 0, sizeof(int64_t), s));
  } else {
    scan_impl<int64_t>(sums, offs, ntiles, tmp, tmp_off + 2 * (size_t)ntiles + 1, s);
  }
  k_tile_scan<In><<<(unsigned)ntiles, kBlock, 0, s>>>(in, n, offs, out);
}

static size_t scan_scratch(int64_t n) {
  size_t tot = 0;
  while (true) {
    int64_t nt = (n + kScanTile - 1) / kScanTile;
    tot += 2 * (size_t)nt + 1;
    if (nt <= 1) break;
    n = nt;
  }
  return tot + 8;
}

void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, DevBuf<int64_t> &tmp,
                        hipStream_t s) {
  tmp.reserve(scan_scratch(n));
  scan_impl<int64_t>(in, out, n, tmp, 0, s);
}
void scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, DevBuf<int64_t> &tmp,
                               hipStream_t s) {
  tmp.reserve(scan_scratch(n));
  scan_impl<int32_t>(in, out, n, tmp, 0, s);
}

// explicit instantiations
#define MG_INST(T)                                                                                  \
  template void launch_spmv<T>(const CsrView<T> &, const T *, T *, hipStream_t);                    \
  template void launch_jacobi_first<T>(int64_t, const T *, const T *, T *, const int *,             \
                                       hipStream_t);                                                \
  template void launch_jacobi<T>(const CsrView<T> &, const T *, const T *, const T *, T *,          \
                                 const int *, hipStream_t);                                         \
  template void launch_residual<T>(const CsrView<T> &, const T *, const T *, T *, const int *,      \
                                   hipStream_t);                                                    \
  template void launch_jacobi_scaled<T>(const CsrView<T> &, const T *, const T *, T *, const int *, \
                                        hipStream_t);                                               \
  template void launch_cheb_first<T>(int64_t, const T *, const T *, const T *, const int32_t *, int, \
                                     T *, T *, const int *, hipStream_t);                           \
  template void launch_cheb<T>(const CsrView<T> &, const T *, const T *, const T *, const int32_t *, \
                               int, int, const T *, T *, T *, const int *, hipStream_t);            \
  template void launch_restrict<T>(int64_t, const int64_t *, const int32_t *, const T *, const T *, \
                                   T *, int, const int *, hipStream_t, CoarseFirst<T>);             \
  template void launch_restrict_sum<T>(int64_t, const int64_t *, const int32_t *, const T *, T *,  \
                                       int, const int *, hipStream_t, CoarseFirst<T>);             \
  template void launch_jacobi_prolong<T>(const CsrView<T> &, const T *, const T *, const T *,     \
                                         const T *, const int32_t *, const T *, T *, const int *, \
                                         hipStream_t);                                            \
  template void launch_cheb_prolong<T>(const CsrView<T> &, const T *, const T *, const T *,       \
                                       const int32_t *, int, int, const T *, const T *,           \
                                       const int32_t *, const T *, T *, T *, const int *,         \
                                       hipStream_t);                                              \
  template void launch_residual_restrict<T>(const CsrView<T> &, const T *, const T *, int64_t,    \
                                            const int64_t *, const int32_t *, const T *, T *,     \
                                            const int *, hipStream_t);                            \
  template void launch_prolong<T>(int64_t, const int32_t *, const T *, const T *, T *, const int *, \
                                  hipStream_t);                                                     \
  template void launch_copy_t<T>(int64_t, const T *, T *, const int *, hipStream_t);                \
  template void launch_zero_t<T>(int64_t, T *, const int *, hipStream_t);
MG_INST(double)
MG_INST(float)
#undef MG_INST

}  // namespace mgpbd
