// Row epilogues shared by the CSR passes and the matrix-free passes of the
// fine level: what a pass does with the row sum s = (A x)_i.
#pragma once

#include "devutil.hpp"

namespace mgpbd {

// Every pass of the solving phase (product, smoother sweep, residual, PCG
// product + dot) is one of these epilogues on a product kernel.
template <class T>
struct OpSpmv {
  T *y;
  __device__ void operator()(int64_t i, T s, double &) const { y[i] = s; }
};
// Input vectors of a pass, read through a functor so that an elementwise
// step before the product (the first Jacobi sweep from zero) is applied on
// the fly instead of in a kernel of its own.
template <class T>
struct InVec {  // x_j
  const T *x;
  __device__ __forceinline__ T operator()(int64_t j) const { return x[j]; }
};
template <class T>
struct InScaled {  // the first sweep from z = 0: z_j = omega D^-1 r, as r_j * wdinv_j
  const T *r, *wdinv;
  __device__ __forceinline__ T operator()(int64_t j) const { return r[j] * wdinv[j]; }
};
template <class T>
struct InProlong {  // the iterate after the coarse correction: z_j + p_j e_agg(j)
  const T *z, *p, *e;
  const int32_t *agg;   // -1: row not aggregated (isolated), no correction
  __device__ __forceinline__ T operator()(int64_t j) const {
    const int32_t a = agg[j];
    return a >= 0 ? z[j] + p[j] * e[a] : z[j];
  }
};
template <class T, class In>
struct OpJacobi {  // zo = zi + omega D^-1 (r - A zi), wdinv = omega D^-1 per row
  const T *wdinv, *r;
  In zi;
  T *zo;
  __device__ void operator()(int64_t i, T s, double &) const {
    zo[i] = zi(i) + (r[i] - s) * wdinv[i];
  }
};
// One Chebyshev step (Saad, Alg. 12.1, M = D) after the product s = (A z_k)_i:
// d_k = c1 d_{k-1} + c2 D^-1 (r - A z_k), z_{k+1} = z_k + d_k, with (c1, c2) of
// step k from the coefficient table of the row's body (c1 unused at k = 0).
template <class T, class In>
struct OpCheb {
  const T *r, *dinv;
  T *d, *zo;
  const T *coef;          // [segment][steps][2]
  const int32_t *rowseg;  // segment of each row (nullptr: one segment)
  int steps, k;
  In zi;
  __device__ void operator()(int64_t i, T s, double &) const {
    const int64_t c = 2 * ((int64_t)(rowseg ? rowseg[i] : 0) * steps + k);
    const T rr = (r[i] - s) * dinv[i];
    const T dn = k == 0 ? coef[c + 1] * rr : coef[c] * d[i] + coef[c + 1] * rr;
    d[i] = dn;
    zo[i] = zi(i) + dn;
  }
};

template <class T>
struct OpResidualScaled {  // w = p (r - A z): the restriction's terms, stored in row order
  const T *r, *p;
  T *w;
  __device__ void operator()(int64_t i, T s, double &) const { w[i] = p[i] * (r[i] - s); }
};
template <class T>
struct OpResidual {  // res = r - A z
  const T *r;
  T *res;
  __device__ void operator()(int64_t i, T s, double &) const { res[i] = r[i] - s; }
};
struct OpPcgDot {  // q = A p, accumulate p^T q
  const double *p;
  double *q;
  __device__ void operator()(int64_t i, double s, double &acc) const {
    q[i] = s;
    acc += p[i] * s;
  }
};

}  // namespace mgpbd
