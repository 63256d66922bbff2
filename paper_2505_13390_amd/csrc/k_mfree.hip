// Matrix-free fine-level passes (see mfree.hpp): A x = J W J^T x + alpha~ x
// (Eq. 3) from per-row gradient planes and per-incidence gradients. Each pass
// is a vertex gather followed by a row pass that ends in the same epilogues
// as the CSR passes (product, Jacobi sweep, residual, PCG product + dot).
#include "mfree.hpp"
#include "rowops.hpp"

namespace mgpbd {

constexpr int kMfLanes = 8;   // lanes per vertex in the gather (about 36 rows per vertex)

// ---------------------------------------------------------------- prepare
template <class T>
__global__ void k_mf_planes(int64_t m, const int32_t *__restrict__ rv,
                            const double *__restrict__ grad, T *__restrict__ gp) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const double *g = grad + 12 * c;
  if (rv[4 * c + 2] < 0) {   // edge row: slot 1 is the negated slot 0
#pragma unroll
    for (int d = 0; d < 3; ++d) gp[d * m + c] = (T)g[d];
  } else {                   // volume row: slot 0 is minus the sum of slots 1-3
#pragma unroll
    for (int q = 3; q < 12; ++q) gp[q * m + c] = (T)g[q];
  }
}

template <class T>
__global__ void k_mf_incidence(int64_t n_inc, const int32_t *__restrict__ vrow,
                               const int8_t *__restrict__ vslot, const double *__restrict__ grad,
                               T *__restrict__ gT) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_inc) return;
  const double *g = grad + 12 * (int64_t)vrow[e] + 3 * vslot[e];
  T *o = gT + 3 * e;
  o[0] = (T)g[0];
  o[1] = (T)g[1];
  o[2] = (T)g[2];
}

template <class T>
void launch_mf_prepare(int64_t m, int64_t n_inc, const int32_t *rv, const double *grad,
                       const int32_t *vrow, const int8_t *vslot, T *gp, T *gT, hipStream_t s) {
  if (m) k_mf_planes<T><<<blocks_for(m, kBlock), kBlock, 0, s>>>(m, rv, grad, gp);
  if (n_inc)
    k_mf_incidence<T><<<blocks_for(n_inc, kBlock), kBlock, 0, s>>>(n_inc, vrow, vslot, grad, gT);
}

// ----------------------------------------------------------------- passes
// u_v = w_v sum_{e in incidence(v)} gT_e x_{row(e)}; G lanes per vertex with
// a fixed lane assignment and a fixed-tree sum.
template <int G, class T>
__global__ __launch_bounds__(kBlock) void k_mf_gather(const int *done, MfView<T> A,
                                                      const T *__restrict__ x) {
  if (done && *done) return;
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(A.nv, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    const int64_t v = base + grp;
    const bool ok = v < hi;
    T sx = 0, sy = 0, sz = 0;
    if (ok) {
      const int64_t a = A.vptr[v], b = A.vptr[v + 1];
      for (int64_t e = a + sub; e < b; e += G) {
        const T xc = x[A.vrow[e]];
        const T *g = A.gT + 3 * e;
        sx += g[0] * xc;
        sy += g[1] * xc;
        sz += g[2] * xc;
      }
    }
    sx = group_sum<G, T>(sx);
    sy = group_sum<G, T>(sy);
    sz = group_sum<G, T>(sz);
    if (ok && sub == 0) {
      const T wv = A.w[v];
      T *u = A.u + 4 * v;
      u[0] = wv * sx;
      u[1] = wv * sy;
      u[2] = wv * sz;
    }
  }
}

// (A x)_c = sum_k g_{c,k} . u_{v_k} + alpha~_c x_c, one thread per row.
template <class T, class Op>
__global__ __launch_bounds__(kBlock) void k_mf_rows(const int *done, MfView<T> A,
                                                    const T *__restrict__ x, Op op,
                                                    double *partials) {
  if (done && *done) return;
  const int64_t m = A.m;
  int64_t lo, hi;
  block_range(m, lo, hi);
  double acc = 0.0;
  for (int64_t c = lo + threadIdx.x; c < hi; c += blockDim.x) {
    const int4 r = *reinterpret_cast<const int4 *>(A.rv + 4 * c);
    T s;
    if (r.z < 0) {
      const T gx = A.gp[c], gy = A.gp[m + c], gz = A.gp[2 * m + c];
      const T *ui = A.u + 4 * (int64_t)r.x, *uj = A.u + 4 * (int64_t)r.y;
      s = (gx * (ui[0] - uj[0]) + gy * (ui[1] - uj[1])) + gz * (ui[2] - uj[2]);
    } else {
      T g[4][3];
#pragma unroll
      for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[k][d] = A.gp[(3 * k + d) * m + c];
#pragma unroll
      for (int d = 0; d < 3; ++d) g[0][d] = -((g[1][d] + g[2][d]) + g[3][d]);
      const int32_t vs[4] = {r.x, r.y, r.z, r.w};
      s = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T *uk = A.u + 4 * (int64_t)vs[k];
        s += (g[k][0] * uk[0] + g[k][1] * uk[1]) + g[k][2] * uk[2];
      }
    }
    s = s + A.alpha[c] * x[c];
    op(c, s, acc);
  }
  if (partials) {
    double v[1] = {acc};
    block_partials<1>(v, partials);
  }
}

template <class T, class Op>
static int launch_mf_pass(const MfView<T> &A, const T *x, Op op, const int *done,
                          double *partials, hipStream_t s) {
  if (!A.m) return 0;
  if (A.nv)
    k_mf_gather<kMfLanes, T><<<grid_for(A.nv * kMfLanes, kBlock), kBlock, 0, s>>>(done, A, x);
  const int grid = grid_for(A.m, kBlock);
  k_mf_rows<T, Op><<<grid, kBlock, 0, s>>>(done, A, x, op, partials);
  return grid;
}

template <class T>
void launch_mf_spmv(const MfView<T> &A, const T *x, T *y, const int *done, hipStream_t s) {
  launch_mf_pass<T>(A, x, OpSpmv<T>{y}, done, nullptr, s);
}
template <class T>
void launch_mf_jacobi(const MfView<T> &A, const T *wdinv, const T *r, const T *zi, T *zo,
                      const int *done, hipStream_t s) {
  launch_mf_pass<T>(A, zi, OpJacobi<T>{wdinv, r, zi, zo}, done, nullptr, s);
}
template <class T>
void launch_mf_residual(const MfView<T> &A, const T *r, const T *z, T *res, const int *done,
                        hipStream_t s) {
  launch_mf_pass<T>(A, z, OpResidual<T>{r, res}, done, nullptr, s);
}

void launch_mf_gather(const MfView<double> &A, const double *x, const int *done, hipStream_t s) {
  if (A.m && A.nv)
    k_mf_gather<kMfLanes, double>
        <<<grid_for(A.nv * kMfLanes, kBlock), kBlock, 0, s>>>(done, A, x);
}
int launch_mf_rows_dot(const MfView<double> &A, const double *p, double *q, const int *done,
                       double *partials, hipStream_t s) {
  if (!A.m) return 0;
  const int grid = grid_for(A.m, kBlock);
  k_mf_rows<double, OpPcgDot><<<grid, kBlock, 0, s>>>(done, A, p, OpPcgDot{p, q}, partials);
  return grid;
}

void launch_mf_pcg_spmv_dot(PcgCtl *ctl, const MfView<double> &A, const double *p, double *q,
                            double *partials, hipStream_t s) {
  const int *done = reinterpret_cast<const int *>(ctl);   // PcgCtl::done is the first field
  const int grid = launch_mf_pass<double>(A, p, OpPcgDot{p, q}, done, partials, s);
  launch_fin_pq(ctl, partials, grid, s);
}

#define MG_INST(T)                                                                              \
  template void launch_mf_prepare<T>(int64_t, int64_t, const int32_t *, const double *,        \
                                     const int32_t *, const int8_t *, T *, T *, hipStream_t);   \
  template void launch_mf_spmv<T>(const MfView<T> &, const T *, T *, const int *, hipStream_t); \
  template void launch_mf_jacobi<T>(const MfView<T> &, const T *, const T *, const T *, T *,    \
                                    const int *, hipStream_t);                                  \
  template void launch_mf_residual<T>(const MfView<T> &, const T *, const T *, T *,             \
                                      const int *, hipStream_t);
MG_INST(double)
MG_INST(float)
#undef MG_INST

}  // namespace mgpbd
