// Matrix-free fine-level passes (see mfree.hpp): A x = J W J^T x + alpha~ x
// (Eq. 3) with the gradients recomputed from the positions. Each pass is a
// vertex gather followed by a row pass that ends in the same epilogues as the
// CSR passes (product, Jacobi sweep, residual, PCG product + dot).
#include "grad.hpp"
#include "mfree.hpp"
#include "rowops.hpp"


namespace mgpbd {

// lanes per vertex in the gather (about 36 rows per vertex; 16 measured fastest of
// 4 to 64 on the 32x32x128 beam)
constexpr int kMfLanes = 16;

// ---------------------------------------------------------------- prepare
template <class T>
__global__ void k_mf_pos(int64_t nv, const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, T *__restrict__ pos) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  T *p = pos + 4 * v;
  p[0] = (T)x[v];
  p[1] = (T)y[v];
  p[2] = (T)z[v];
  p[3] = (T)0;
}

template <class T>
__global__ void k_mf_incidence(int64_t n_inc, const int32_t *__restrict__ vrow,
                               const int8_t *__restrict__ vslot, const double *__restrict__ grad,
                               T *__restrict__ gT) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_inc) return;
  const double *g = grad + 12 * (int64_t)vrow[e] + 3 * vslot[e];
  if constexpr (sizeof(T) == 4) {
    reinterpret_cast<float4 *>(gT)[e] =
        make_float4((float)g[0], (float)g[1], (float)g[2], __int_as_float(vrow[e]));
  } else {
    T *o = gT + 3 * e;
    o[0] = (T)g[0];
    o[1] = (T)g[1];
    o[2] = (T)g[2];
  }
}

template <class T>
void launch_mf_prepare(int64_t nv, const double *x, const double *y, const double *z,
                       int64_t n_inc, const int32_t *vrow, const int8_t *vslot,
                       const double *grad, T *pos, T *gT, hipStream_t s) {
  if (nv) k_mf_pos<T><<<blocks_for(nv, kBlock), kBlock, 0, s>>>(nv, x, y, z, pos);
  if (n_inc)
    k_mf_incidence<T><<<blocks_for(n_inc, kBlock), kBlock, 0, s>>>(n_inc, vrow, vslot, grad, gT);
}

// ----------------------------------------------------------------- passes
// u_v = w_v sum_{e in incidence(v)} gT_e x_{row(e)}; G lanes per vertex with a
// fixed lane assignment and a fixed-tree sum.
template <int G, class T, class In>
__global__ __launch_bounds__(kBlock) void k_mf_gather(const int *done, MfView<T> A, In x) {
  if (done && *done) return;
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  const XcdStride S = xcd_stride(A.nv, R);
  for (int64_t base = S.first; base < S.hi; base += S.step) {
    const int64_t v = base + grp;
    const bool ok = v < S.hi;
    T sx = 0, sy = 0, sz = 0;
    if (ok) {
      const int64_t a = A.vptr[v], b = A.vptr[v + 1];
      for (int64_t e = a + sub; e < b; e += G) {
        if constexpr (sizeof(T) == 4) {
          const float4 r = reinterpret_cast<const float4 *>(A.gT)[e];
          const T xc = x(__float_as_int(r.w));
          sx += r.x * xc;
          sy += r.y * xc;
          sz += r.z * xc;
        } else {
          const T xc = x(A.vrow[e]);
          const T *g = A.gT + 3 * e;
          sx += g[0] * xc;
          sy += g[1] * xc;
          sz += g[2] * xc;
        }
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

template <class T>
__device__ __forceinline__ T dot_u(const T (&g)[3], const T *__restrict__ u) {
  return (g[0] * u[0] + g[1] * u[1]) + g[2] * u[2];
}

// (J u)_c = sum_k g_{c,k} . u_{v_k} for row c. The slot gradients are formed
// one at a time (the same expressions as tet_grads) and consumed at once,
// which keeps the register count low enough for full occupancy.
template <class T>
__device__ __forceinline__ T mf_row(const MfView<T> &A, const int64_t c, const int4 r) {
  const T *__restrict__ pos = A.pos;
  const T *__restrict__ u = A.u;
  const int64_t va = r.x, vb = r.y;
  T s;
  if (A.kind && A.kind[c]) {   // stored gradients (same values the assembly read)
    const T *g = A.gst + 12 * c;
    T g0[3] = {g[0], g[1], g[2]}, g1[3] = {g[3], g[4], g[5]};
    T g2[3] = {g[6], g[7], g[8]}, g3[3] = {g[9], g[10], g[11]};
    s = dot_u(g0, u + 4 * va);
    s += dot_u(g1, u + 4 * vb);
    s += dot_u(g2, u + 4 * (int64_t)r.z);
    s += dot_u(g3, u + 4 * (int64_t)r.w);
  } else if (r.z < 0) {
    T g0[3], g1[3];
    edge_grads(pos + 4 * va, pos + 4 * vb, g0, g1);
    s = dot_u(g0, u + 4 * va);
    s += dot_u(g1, u + 4 * vb);
  } else {
    const int64_t vc = r.z, vd = r.w;
    T e1[3], e2[3], e3[3], cr[3], g1[3], g2[3], g3[3], g0[3];
    tet_edges(pos + 4 * va, pos + 4 * vb, pos + 4 * vc, pos + 4 * vd, e1, e2, e3);
    cross(e2, e3, cr);
#pragma unroll
    for (int d = 0; d < 3; ++d) g1[d] = cr[d] / (T)6;
    cross(e3, e1, cr);
#pragma unroll
    for (int d = 0; d < 3; ++d) g2[d] = cr[d] / (T)6;
    cross(e1, e2, cr);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g3[d] = cr[d] / (T)6;
      g0[d] = -((g1[d] + g2[d]) + g3[d]);
    }
    s = dot_u(g0, u + 4 * va);
    s += dot_u(g1, u + 4 * vb);
    s += dot_u(g2, u + 4 * vc);
    s += dot_u(g3, u + 4 * vd);
  }
  return s;
}

// (A x)_c = (J u)_c + alpha~_c x_c, one thread per row, then the epilogue.
template <class T, class In, class Op>
__global__ __launch_bounds__(kBlock, 8) void k_mf_rows(const int *done, MfView<T> A, In x, Op op,
                                                       double *partials) {
  if (done && *done) return;
  const XcdStride S = xcd_stride(A.m, blockDim.x);
  const int64_t hi = S.hi;
  double acc = 0.0;
  const int4 *rv4 = reinterpret_cast<const int4 *>(A.rv);
  // the vertex ids of the next row are loaded while this row is computed
  int64_t c = S.first + threadIdx.x;
  int4 rn = c < hi ? rv4[c] : make_int4(0, 0, -1, -1);
  for (; c < hi; c += S.step) {
    const int4 r = rn;
    const int64_t cn = c + S.step;
    if (cn < hi) rn = rv4[cn];
    const T s = mf_row(A, c, r) + A.alpha[c] * x(c);
    op(c, s, acc);
  }
  if (partials) {
    double v[1] = {acc};
    block_partials<1>(v, partials);
  }
}

template <class T, class In>
static void launch_mf_gather_in(const MfView<T> &A, In x, const int *done, hipStream_t s) {
  if (A.m && A.nv)
    k_mf_gather<kMfLanes, T, In><<<grid_for(A.nv * kMfLanes, kBlock), kBlock, 0, s>>>(done, A, x);
}

template <class T, class In, class Op>
static int launch_mf_pass(const MfView<T> &A, In x, Op op, const int *done, double *partials,
                          hipStream_t s) {
  if (!A.m) return 0;
  launch_mf_gather_in<T>(A, x, done, s);
  const int grid = grid_for(A.m, kBlock);
  k_mf_rows<T, In, Op><<<grid, kBlock, 0, s>>>(done, A, x, op, partials);
  return grid;
}

template <class T>
void launch_mf_jacobi(const MfView<T> &A, const T *wdinv, const T *r, const T *zi, T *zo,
                      const int *done, hipStream_t s) {
  const InVec<T> in{zi};
  launch_mf_pass<T>(A, in, OpJacobi<T, InVec<T>>{wdinv, r, in, zo}, done, nullptr, s);
}
template <class T>
void launch_mf_cheb(const MfView<T> &A, const T *r, const T *dinv, const T *coef,
                    const int32_t *rowseg, int steps, int k, const T *zi, T *d, T *zo,
                    const int *done, hipStream_t s) {
  const InVec<T> in{zi};
  launch_mf_pass<T>(A, in, OpCheb<T, InVec<T>>{r, dinv, d, zo, coef, rowseg, steps, k, in}, done,
                    nullptr, s);
}
template <class T>
void launch_mf_jacobi_prolong(const MfView<T> &A, const T *wdinv, const T *r, const T *zi,
                              const T *p, const int32_t *agg, const T *e, T *zo,
                              const int *done, hipStream_t s) {
  const InProlong<T> in{zi, p, e, agg};
  launch_mf_pass<T>(A, in, OpJacobi<T, InProlong<T>>{wdinv, r, in, zo}, done, nullptr, s);
}
template <class T>
void launch_mf_cheb_prolong(const MfView<T> &A, const T *r, const T *dinv, const T *coef,
                            const int32_t *rowseg, int steps, int k, const T *zi, const T *p,
                            const int32_t *agg, const T *e, T *d, T *zo, const int *done,
                            hipStream_t s) {
  const InProlong<T> in{zi, p, e, agg};
  launch_mf_pass<T>(A, in, OpCheb<T, InProlong<T>>{r, dinv, d, zo, coef, rowseg, steps, k, in},
                    done, nullptr, s);
}
template <class T>
void launch_mf_residual_scaled(const MfView<T> &A, const T *r, const T *z, const T *p, T *w,
                               const int *done, hipStream_t s) {
  launch_mf_pass<T>(A, InVec<T>{z}, OpResidualScaled<T>{r, p, w}, done, nullptr, s);
}
template <class T>
void launch_mf_residual(const MfView<T> &A, const T *r, const T *z, T *res, const int *done,
                        hipStream_t s) {
  launch_mf_pass<T>(A, InVec<T>{z}, OpResidual<T>{r, res}, done, nullptr, s);
}
void launch_mf_gather(const MfView<double> &A, const double *x, const int *done, hipStream_t s) {
  launch_mf_gather_in<double>(A, InVec<double>{x}, done, s);
}
int launch_mf_rows_dot(const MfView<double> &A, const double *p, double *q, const int *done,
                       double *partials, hipStream_t s) {
  if (!A.m) return 0;
  const int grid = grid_for(A.m, kBlock);
  k_mf_rows<double, InVec<double>, OpPcgDot>
      <<<grid, kBlock, 0, s>>>(done, A, InVec<double>{p}, OpPcgDot{p, q}, partials);
  return grid;
}

#define MG_INST(T)                                                                              \
  template void launch_mf_prepare<T>(int64_t, const double *, const double *, const double *,  \
                                     int64_t, const int32_t *, const int8_t *, const double *,  \
                                     T *, T *, hipStream_t);                                    \
  template void launch_mf_jacobi_prolong<T>(const MfView<T> &, const T *, const T *, const T *, \
                                            const T *, const int32_t *, const T *, T *,         \
                                            const int *, hipStream_t);                          \
  template void launch_mf_cheb_prolong<T>(const MfView<T> &, const T *, const T *, const T *,   \
                                          const int32_t *, int, int, const T *, const T *,      \
                                          const int32_t *, const T *, T *, T *, const int *,    \
                                          hipStream_t);                                         \
  template void launch_mf_residual_scaled<T>(const MfView<T> &, const T *, const T *, const T *, \
                                             T *, const int *, hipStream_t);                     \
  template void launch_mf_jacobi<T>(const MfView<T> &, const T *, const T *, const T *, T *,    \
                                    const int *, hipStream_t);                                  \
  template void launch_mf_residual<T>(const MfView<T> &, const T *, const T *, T *,             \
                                      const int *, hipStream_t);                                \
  template void launch_mf_cheb<T>(const MfView<T> &, const T *, const T *, const T *,           \
                                  const int32_t *, int, int, const T *, T *, T *, const int *,  \
                                  hipStream_t);
MG_INST(double)
MG_INST(float)
#undef MG_INST

}  // namespace mgpbd
