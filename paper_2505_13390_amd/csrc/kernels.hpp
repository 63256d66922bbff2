// Host-callable launchers of the library's HIP kernels. Every launcher
// enqueues on the given stream and returns immediately.
#pragma once

#include "common.hpp"
#include "devutil.hpp"

namespace mgpbd {

// Lanes per row used by the row-group CSR kernels for a given mean row length.
int lanes_for_rowlen(double mean_nnz_per_row);

// SELL-C-sigma copy of a level's matrix (Kreutzer et al., SIAM J. Sci.
// Comput. 2014): within windows of kSellSigma rows the rows are ordered by
// decreasing length, consecutive groups of kSellC = 64 rows form chunks, and
// a chunk stores its rows' entries column-major, padded with zeros to its
// longest row, so lane t of a wavefront reads entry k of its row at
// val[ptr[c] + 64 k + t]: one coalesced load per step for 64 rows.
constexpr int kSellC = 64;
constexpr int kSellSigma = 1024;
template <class T>
struct SellView {
  int64_t nchunks = 0;
  const int32_t *perm = nullptr;   // [nchunks * 64] row of each slot (-1 = padding)
  const int64_t *ptr = nullptr;    // [nchunks + 1] first entry of each chunk
  const int32_t *col = nullptr;    // [ptr[nchunks]] column of each entry (padding: 0)
  const T *val = nullptr;          // [ptr[nchunks]] value of each entry (padding: 0)
};

// CSR view of one level (device pointers) and the product variant chosen
// for it: sell.val != nullptr -> SELL-C-sigma kernels over the level's SELL
// copy; else tile == 0 -> row-group kernels with `lanes` lanes per row;
// tile > 0 -> LDS-staged stream kernels over row tiles of at most `tile`
// entries (tiles[0..ntiles] are the first rows of the tiles).
template <class T>
struct CsrView {
  int64_t n = 0, nnz = 0;
  const int64_t *rowptr = nullptr;
  const int32_t *col = nullptr;
  const T *val = nullptr;
  int lanes = 16;
  int tile = 0;
  bool nt = false;   // non-temporal loads of the matrix entries (stream kernels)
  int64_t ntiles = 0;
  const int64_t *tiles = nullptr;
  SellView<T> sell;
};

// Host build of the SELL-C-sigma layout of a CSR pattern: perm, chunk
// pointers, columns, and for every CSR entry its slot in the SELL arrays.
void build_sell(const std::vector<int64_t> &rowptr, const std::vector<int32_t> &col,
                std::vector<int32_t> &perm, std::vector<int64_t> &ptr,
                std::vector<int32_t> &scol, std::vector<int64_t> &slot);
// sval[slot[e]] = val[e] for every CSR entry e (the values after each
// assembly or Galerkin product; padding stays zero)
template <class S, class T>
void launch_sell_values(int64_t nnz, const int64_t *slot, const S *val, T *sval, hipStream_t s);

// Row tiles of at most `tile` entries (host, from the row pointers); returns
// false when some row alone is longer than a tile.
bool build_row_tiles(const std::vector<int64_t> &rowptr, int tile, std::vector<int64_t> &tiles);

// ---------------- sparse kernels of the V-cycle (T = double or float) ----
template <class T> void launch_spmv(const CsrView<T> &A, const T *x, T *y, hipStream_t s);
// q = A p and the partial sums of p^T q (one per block of `grid`); returns grid
int launch_spmv_dot_partials(const CsrView<double> &A, const double *p, double *q,
                             const int *done, double *partials, hipStream_t s);
// z = omega D^-1 r (first sweep from z = 0); wdinv = omega D^-1 per row
template <class T> void launch_jacobi_first(int64_t n, const T *wdinv, const T *r, T *z,
                                            const int *done, hipStream_t s);
// zo = zi + omega D^-1 (r - A zi)
template <class T> void launch_jacobi(const CsrView<T> &A, const T *wdinv, const T *r,
                                      const T *zi, T *zo, const int *done, hipStream_t s);
// The first post-smoothing step with the coarse correction folded in: its
// input is z + P e formed on the fly (p the one-column prolongator values,
// agg the aggregate of each row, e the coarse correction), the same values
// k_prolong would have stored, so the pass and the separate prolongation
// followed by the pass compute the same bits.
template <class T> void launch_jacobi_prolong(const CsrView<T> &A, const T *wdinv, const T *r,
                                              const T *zi, const T *p, const int32_t *agg,
                                              const T *e, T *zo, const int *done,
                                              hipStream_t s);
template <class T> void launch_cheb_prolong(const CsrView<T> &A, const T *r, const T *dinv,
                                            const T *coef, const int32_t *rowseg, int steps,
                                            int k, const T *zi, const T *p, const int32_t *agg,
                                            const T *e, T *d, T *zo, const int *done,
                                            hipStream_t s);
// With z set, a restriction also writes z[a] = rc[a] wd[a], the coarse level's
// first Jacobi sweep from zero (the values k_jacobi_first would write there).
template <class T>
struct CoarseFirst {
  const T *wd = nullptr;
  T *z = nullptr;
};
// rc[a] = sum of w_i over the members i of aggregate a (ascending, RL lanes
// with the fixed tree of the restriction): the restriction when the residual
// pass already stored w = p (r - A z)
template <class T> void launch_restrict_sum(int64_t na, const int64_t *ap, const int32_t *mem,
                                            const T *w, T *rc, int lanes, const int *done,
                                            hipStream_t s, CoarseFirst<T> first = {});
// rc = P^T (r - A z) in one pass over the aggregates [0, na): G lanes per
// aggregate form each member row's residual (ascending members) and add
// p_i res_i in that order; the fine residual is not stored
template <class T> void launch_residual_restrict(const CsrView<T> &A, const T *r, const T *z,
                                                 int64_t na, const int64_t *ap,
                                                 const int32_t *mem, const T *p, T *rc,
                                                 const int *done, hipStream_t s);
// res = r - A z
template <class T> void launch_residual(const CsrView<T> &A, const T *r, const T *z, T *res,
                                        const int *done, hipStream_t s);
// the first two sweeps from z = 0 in one pass: zo = z1 + omega D^-1 (r - A z1)
// with z1 = omega D^-1 r formed on the fly
template <class T> void launch_jacobi_scaled(const CsrView<T> &A, const T *wdinv, const T *r,
                                             T *zo, const int *done, hipStream_t s);
// Chebyshev smoothing steps (coefficient table [segment][steps][2], rowseg
// the segment of each row or nullptr): the first step from z = 0
// (d = c2 D^-1 r, z = d), and step k after the product A zi
// (d = c1 d + c2 D^-1 (r - A zi), zo = zi + d; c1 unused at k = 0)
template <class T> void launch_cheb_first(int64_t n, const T *r, const T *dinv, const T *coef,
                                          const int32_t *rowseg, int steps, T *d, T *z,
                                          const int *done, hipStream_t s);
template <class T> void launch_cheb(const CsrView<T> &A, const T *r, const T *dinv,
                                    const T *coef, const int32_t *rowseg, int steps, int k,
                                    const T *zi, T *d, T *zo, const int *done, hipStream_t s);
// rc[a] = sum over members i of a of p_i res_i; `lanes` (8, 16, 32 or 64) lanes per
// aggregate, each summing a strided share, then a fixed-tree lane sum
template <class T> void launch_restrict(int64_t n_agg, const int64_t *agg_ptr,
                                        const int32_t *agg_mem, const T *p, const T *res, T *rc,
                                        int lanes, const int *done, hipStream_t s,
                                        CoarseFirst<T> first = {});
// z_i += p_i ec[agg_i]
template <class T> void launch_prolong(int64_t n, const int32_t *agg, const T *p, const T *ec,
                                       T *z, const int *done, hipStream_t s);


void launch_d2f(int64_t n, const double *in, float *out, const int *done, hipStream_t s);
template <class T> void launch_copy_t(int64_t n, const T *in, T *out, const int *done, hipStream_t s);
template <class T> void launch_zero_t(int64_t n, T *out, const int *done, hipStream_t s);
void launch_copy(int64_t n, const double *in, double *out, const int *done, hipStream_t s);
void launch_fill(int64_t n, double v, double *out, hipStream_t s);
void launch_fill_i32(int64_t n, int32_t v, int32_t *out, hipStream_t s);
void launch_fill_u8(int64_t n, uint8_t v, uint8_t *out, hipStream_t s);

// ---------------- PCG (FP64 outer loop), control block in device memory ----
// finisher of p^T A p: pq, alpha (or breakdown) from nparts block partials
void launch_fin_pq(PcgCtl *ctl, const double *partials, int nparts, hipStream_t s);

// ---------------- scans (deterministic) ----------------
// out[i] = sum_{k<i} in[k], out[n] = total (out has n+1 entries)
void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, DevBuf<int64_t> &tmp,
                        hipStream_t s);
void scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n,
                               DevBuf<int64_t> &tmp, hipStream_t s);

}  // namespace mgpbd
