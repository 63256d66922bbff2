// Matrix-free application of the fine-level operator of Eq. 3,
//   A x = J W J^T x + alpha~ x,
// from the constraint gradients instead of the assembled CSR values (the
// direction the Conclusion and Limitations section names for future work).
// Two kernels per product: a vertex gather u_v = w_v sum_{c contains v}
// g_{c,v} x_c over the vertex -> row incidence (ascending rows), reading the
// gradient of each incidence from a vertex-major copy; then a row pass
// (A x)_c = sum_k g_{c,k} . u_{v_k} + alpha~_c x_c that recomputes the row's
// gradients from the positions with the constraint kernel's own formulas
// (grad.hpp), so it reads only the row's vertex ids from HBM (ARAP rows read
// their stored gradients instead). Both use
// exactly the gradients the assembly used. The assembled A is still built
// every global iteration: the setup, the Galerkin products and the Jacobi
// diagonal read it.
#pragma once

#include "kernels.hpp"

namespace mgpbd {

template <class T>
struct MfView {
  int64_t m = 0, nv = 0;
  const int32_t *rv = nullptr;    // [m][4] vertex ids of each row, -1 padded (edge rows)
  const T *pos = nullptr;         // [nv][4] positions (x, y, z, unused) of this iteration
  const T *alpha = nullptr;       // [m] alpha~ = alpha / dt^2
  const int64_t *vptr = nullptr;  // [nv + 1] incidence range of each vertex
  const int32_t *vrow = nullptr;  // [E] row of each incidence, ascending per vertex
  // gradient of each incidence: FP64 [E][3]; FP32 [E][4], the gradient and the
  // incidence's row (its int32 bits in the fourth lane), one 16-byte load each
  const T *gT = nullptr;
  const T *w = nullptr;           // [nv] inverse masses
  T *u = nullptr;                 // [nv][4] scratch of the vertex gather
  // rows whose gradients are read instead of recomputed (ARAP rows, whose
  // nearest rotation is too costly to repeat per product): kind[c] != 0 marks
  // them, gst[c][4][3] holds their gradients; both null without such rows
  const int8_t *kind = nullptr;
  const T *gst = nullptr;
  bool ok() const { return m > 0 && rv && pos && alpha && vptr && vrow && gT && w && u; }
};

// Per global iteration, after the constraint kernel: positions as T
// (pos[v] = (x, y, z)) and the per-incidence gradients gT[e] = the gradient
// of slot vslot[e] of row vrow[e], converted to T (FP32: with vrow[e] beside it).
template <class T>
void launch_mf_prepare(int64_t nv, const double *x, const double *y, const double *z,
                       int64_t n_inc, const int32_t *vrow, const int8_t *vslot,
                       const double *grad, T *pos, T *gT, hipStream_t s);

template <class T>
void launch_mf_jacobi(const MfView<T> &A, const T *wdinv, const T *r, const T *zi, T *zo,
                      const int *done, hipStream_t s);
template <class T>
void launch_mf_cheb(const MfView<T> &A, const T *r, const T *dinv, const T *coef,
                    const int32_t *rowseg, int steps, int k, const T *zi, T *d, T *zo,
                    const int *done, hipStream_t s);
// the first post-smoothing step with the coarse correction z + P e formed
// on the fly (see launch_jacobi_prolong)
template <class T>
void launch_mf_jacobi_prolong(const MfView<T> &A, const T *wdinv, const T *r, const T *zi,
                              const T *p, const int32_t *agg, const T *e, T *zo,
                              const int *done, hipStream_t s);
template <class T>
void launch_mf_cheb_prolong(const MfView<T> &A, const T *r, const T *dinv, const T *coef,
                            const int32_t *rowseg, int steps, int k, const T *zi, const T *p,
                            const int32_t *agg, const T *e, T *d, T *zo, const int *done,
                            hipStream_t s);
template <class T>
void launch_mf_residual(const MfView<T> &A, const T *r, const T *z, T *res, const int *done,
                        hipStream_t s);
// w = p (r - A z), the terms of the restriction P^T (r - A z) in row order
template <class T>
void launch_mf_residual_scaled(const MfView<T> &A, const T *r, const T *z, const T *p, T *w,
                               const int *done, hipStream_t s);
// the PCG product q = A p as its two kernels (timed one by one when
// profiling): the vertex gather, then the row pass writing q and the partial
// sums of p^T q (returns the number of partials; launch_fin_pq finishes)
void launch_mf_gather(const MfView<double> &A, const double *x, const int *done, hipStream_t s);
int launch_mf_rows_dot(const MfView<double> &A, const double *p, double *q, const int *done,
                       double *partials, hipStream_t s);

}  // namespace mgpbd
