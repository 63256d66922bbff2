// Launchers of the AMG setup kernels (Sec. 4.1, 4.3, 4.5) and of the
// Galerkin product (Sec. 4.4, Eq. 6).
#pragma once

#include "kernels.hpp"

namespace mgpbd {

// *bad = 1 unless rp[0..n] / col[0..nnz) form a valid CSR (bounds monotone
// within [0, nnz], rp[0] = 0, columns in [0, n) strictly ascending per row)
void launch_validate_csr(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *col, int *bad,
                         hipStream_t s);
void launch_diagpos(int64_t n, const int64_t *rp, const int32_t *col, int64_t *dpos, int *bad,
                    hipStream_t s);
// diag[i] = A_ii, dinv = 1 / A_ii (FP64, optional FP32 copy); bad = 1 if some A_ii <= 0
void launch_extract_diag(int64_t n, const int64_t *dpos, const double *val, double *diag,
                         double *dinv, float *dinv32, int *bad, hipStream_t s);

// strength of connection, kept iff a_ij^2 >= theta2 (|a_ii| |a_jj|), j != i
void launch_strong(const CsrView<double> &A, const double *diag, double theta2, uint8_t *strong,
                   uint8_t *conn, hipStream_t s);
void launch_mis_round(const CsrView<double> &A, const uint8_t *strong, uint64_t *key,
                      uint64_t *m1, int *undecided, hipStream_t s);
void launch_root_flags(int64_t n, const uint64_t *key, int32_t *flag, hipStream_t s);
void launch_pass1(const CsrView<double> &A, const uint8_t *strong, const uint64_t *key,
                  const int64_t *rid, int32_t *agg1, hipStream_t s);
void launch_pass2(const CsrView<double> &A, const uint8_t *strong, const uint8_t *conn,
                  const int32_t *agg1, int32_t *agg, hipStream_t s);
void launch_count_members(int64_t n, const int32_t *agg, int32_t *cnt, hipStream_t s);
void launch_scatter_members(int64_t n, const int32_t *agg, const int64_t *ptr, int32_t *cursor,
                            int32_t *mem, hipStream_t s);
void launch_sort_segments(int64_t nseg, const int64_t *ptr, int32_t *mem, hipStream_t s);

// Jones-Plassmann by counters: higher-key neighbour counts and the first
// frontier (rows with none), then one launch per frontier
void launch_color_count(const CsrView<double> &A, const uint64_t *key, int32_t *cnt,
                        int32_t *front, int *nfront, hipStream_t s);
void launch_color_front(const CsrView<double> &A, int64_t nf, const int32_t *front,
                        const uint64_t *key, int32_t *color, int32_t *cnt, int32_t *next,
                        int *nnext, int *overflow, hipStream_t s);
void launch_count_colors(int64_t n, const int32_t *color, int32_t *cnt, hipStream_t s);
void launch_scatter_colors(int64_t n, const int32_t *color, const int64_t *off, int32_t *cursor,
                           int32_t *rows, hipStream_t s);
// one colour of a Gauss-Seidel sweep on A x = 0
void launch_gs_color(int64_t cnt, const int32_t *rows, const CsrView<double> &A,
                     const double *diag, double *x, hipStream_t s);
// one colour of a Gauss-Seidel smoothing sweep for A x = r
template <class T>
void launch_gs_rhs(int64_t cnt, const int32_t *rows, const CsrView<T> &A, const T *dinv,
                   const T *r, T *x, const int *done, hipStream_t s);
// one-column QR per aggregate: p = B / |B|_aggregate, Bn = |B|_aggregate
void launch_normalize(int64_t na, const int64_t *ap, const int32_t *mem, const double *B,
                      double *p, float *p32, double *Bn, hipStream_t s);

// Galerkin symbolic: per coarse row a, distinct coarse columns and the fine
// entries that feed each coarse entry in ascending fine order
// rowcnt[a] = distinct coarse columns of aggregate row a (-1 when they do not
// fit the LDS table: *overflow is raised and launch_gal_count_big redoes it),
// elen[a] = fine entries connecting it to other aggregates
void launch_gal_count(int64_t na, const int64_t *ap, const int32_t *mem, const CsrView<double> &A,
                      const int32_t *agg, int64_t *rowcnt, int64_t *elen, int *overflow,
                      hipStream_t s);
// rows[q] (q < nbig) with a table of tcap[q] slots (a power of two) at
// 5 toff[q] int32 of scratch
void launch_gal_count_big(int nbig, const int32_t *rows, const int64_t *toff, const int32_t *tcap,
                          int32_t *scratch, const int64_t *ap, const int32_t *mem,
                          const CsrView<double> &A, const int32_t *agg, int64_t *rowcnt,
                          int *overflow, hipStream_t s);
// sorted columns and Galerkin lists of the rows with at most 1024 distinct
// columns; the others are left to launch_gal_fill_big
void launch_gal_fill(int64_t na, const int64_t *ap, const int32_t *mem, const CsrView<double> &A,
                     const int32_t *agg, const int64_t *crp, const int64_t *eoff, int32_t *ccol,
                     int32_t *crow, int64_t *gl_ptr, int32_t *gl_idx, int32_t *gl_row,
                     hipStream_t s);
void launch_gal_fill_big(int nbig, const int32_t *rows, const int64_t *toff, const int32_t *tcap,
                         int32_t *scratch, const int64_t *ap, const int32_t *mem,
                         const CsrView<double> &A, const int32_t *agg, const int64_t *crp,
                         const int64_t *eoff, int32_t *ccol, int32_t *crow, int64_t *gl_ptr,
                         int32_t *gl_idx, int32_t *gl_row, hipStream_t s);
void launch_gal_mirror(int64_t nnzc, const int32_t *crow, const int32_t *ccol, const int64_t *crp,
                       int32_t *mirror, int *bad, hipStream_t s);
void launch_gal_numeric(int64_t nnzc, const int32_t *crow, const int32_t *ccol,
                        const int32_t *mirror, const int64_t *gl_ptr, const int32_t *gl_idx,
                        const int32_t *gl_row, const int32_t *fcol, const double *fval,
                        const double *p, double *cval, float *cval32, hipStream_t s);

// K > 1 candidates (k_cand.hip)
void launch_put_column(int64_t n, int K, int k, const double *x, double *B, hipStream_t s);
void launch_qr_agg(int64_t na, int K, const int64_t *ap, const int32_t *mem, const double *B,
                   double *Q, double *R, int32_t *kq, hipStream_t s);
void launch_scatter_r(int64_t na, int K, const int32_t *kq, const int64_t *coff, const double *R,
                      double *Bn, hipStream_t s);
void launch_member_slots(int64_t nmem, const int32_t *mem, int32_t *slot, hipStream_t s);
void launch_galk_rowlen(int64_t na, const int64_t *arp, const int32_t *acol, const int32_t *kq,
                        int64_t *cstart, int64_t *rowlen, int64_t *blocksz, hipStream_t s);
void launch_galk_pattern(int64_t na, const int32_t *kq, const int64_t *coff, const int64_t *arp,
                         const int32_t *acol, const int64_t *base, const int64_t *rowlen,
                         int64_t *rowptr, int32_t *col, hipStream_t s);
void launch_galk_numeric(int K, int64_t annz, const int32_t *acrow, const int32_t *acol,
                         const int32_t *amirror, const int64_t *gl_ptr, const int32_t *gl_idx,
                         const int32_t *gl_row, const int32_t *fcol, const double *fval,
                         const int32_t *slot, const double *Q, const int32_t *kq,
                         const int64_t *coff, const int64_t *crp, const int64_t *cstart,
                         double *cval, float *cval32, hipStream_t s);
template <class T>
void launch_restrict_k(int64_t na, int K, const int32_t *kq, const int64_t *coff,
                       const int64_t *ap, const int32_t *mem, const T *Q, const T *res, T *rc,
                       const int *done, hipStream_t s);
template <class T>
void launch_prolong_k(int64_t n, int K, const int32_t *agg, const int32_t *slot,
                      const int32_t *kq, const int64_t *coff, const T *Q, const T *zc, T *z,
                      const int *done, hipStream_t s);

}  // namespace mgpbd
