// Host-callable launchers of the library's HIP kernels. Every launcher
// enqueues on the given stream and returns immediately.
#pragma once

#include "common.hpp"
#include "devutil.hpp"

namespace mgpbd {

// Lanes per row used by the row-group CSR kernels for a given mean row length.
int lanes_for_rowlen(double mean_nnz_per_row);

// CSR view of one level (device pointers).
// CSR view of one level (device pointers) and the product variant chosen
// for it: tile == 0 -> row-group kernels with `lanes` lanes per row;
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
};

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
                                        int lanes, const int *done, hipStream_t s);
// z_i += p_i ec[agg_i]
template <class T> void launch_prolong(int64_t n, const int32_t *agg, const T *p, const T *ec,
                                       T *z, const int *done, hipStream_t s);


void launch_d2f(int64_t n, const double *in, float *out, const int *done, hipStream_t s);
void launch_f2d(int64_t n, const float *in, double *out, const int *done, hipStream_t s);
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
