// Constraint gradients of the rows of A (Eq. 3 inputs), shared by the
// constraint kernel and the matrix-free operator so that both evaluate the
// same IEEE sequence and the operator sees exactly the assembled gradients.
//   edge (i, j):        n = (x_i - x_j) / |x_i - x_j| (0 for a zero-length
//                       edge); slot 0 gets n, slot 1 gets -n
//   volume (a, b, c, d): e1 = x_b - x_a, e2 = x_c - x_a, e3 = x_d - x_a;
//                       slot 1 (e2 x e3)/6, slot 2 (e3 x e1)/6,
//                       slot 3 (e1 x e2)/6, slot 0 -((g1 + g2) + g3)
#pragma once

#include <hip/hip_runtime.h>

namespace mgpbd {

// Both slot gradients of an edge row; returns |x_i - x_j|. A zero-length edge
// has zero gradients (+0 in both slots). Written with selects rather than
// branches so that the arrays stay in registers.
template <class T>
__device__ __forceinline__ T edge_grads(const T *pi, const T *pj, T (&g0)[3], T (&g1)[3]) {
  const T dx = pi[0] - pj[0], dy = pi[1] - pj[1], dz = pi[2] - pj[2];
  const T len = sqrt((dx * dx + dy * dy) + dz * dz);
  const bool ok = len > (T)0;
  const T n0 = dx / len, n1 = dy / len, n2 = dz / len;
  g0[0] = ok ? n0 : (T)0;
  g0[1] = ok ? n1 : (T)0;
  g0[2] = ok ? n2 : (T)0;
  g1[0] = ok ? -n0 : (T)0;
  g1[1] = ok ? -n1 : (T)0;
  g1[2] = ok ? -n2 : (T)0;
  return len;
}

template <class T>
__device__ __forceinline__ void cross(const T (&a)[3], const T (&b)[3], T (&o)[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

template <class T>
__device__ __forceinline__ void tet_edges(const T *pa, const T *pb, const T *pc, const T *pd,
                                          T (&e1)[3], T (&e2)[3], T (&e3)[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    e1[d] = pb[d] - pa[d];
    e2[d] = pc[d] - pa[d];
    e3[d] = pd[d] - pa[d];
  }
}

// All four slot gradients; returns e1 . (e2 x e3) (six times the volume).
template <class T>
__device__ __forceinline__ T tet_grads(const T *pa, const T *pb, const T *pc, const T *pd,
                                       T (&g)[4][3]) {
  T e1[3], e2[3], e3[3], c23[3], c31[3], c12[3];
  tet_edges(pa, pb, pc, pd, e1, e2, e3);
  cross(e2, e3, c23);
  cross(e3, e1, c31);
  cross(e1, e2, c12);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g[1][d] = c23[d] / (T)6;
    g[2][d] = c31[d] / (T)6;
    g[3][d] = c12[d] / (T)6;
    g[0][d] = -((g[1][d] + g[2][d]) + g[3][d]);
  }
  return (e1[0] * c23[0] + e1[1] * c23[1]) + e1[2] * c23[2];
}

// The gradient of one slot (bitwise equal to that slot of tet_grads).
template <class T>
__device__ __forceinline__ void tet_grad_slot(const T *pa, const T *pb, const T *pc, const T *pd,
                                              int k, T (&g)[3]) {
  T e1[3], e2[3], e3[3];
  tet_edges(pa, pb, pc, pd, e1, e2, e3);
  if (k == 0) {
    T c23[3], c31[3], c12[3];
    cross(e2, e3, c23);
    cross(e3, e1, c31);
    cross(e1, e2, c12);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      g[d] = -((c23[d] / (T)6 + c31[d] / (T)6) + c12[d] / (T)6);
  } else {
    T c[3];
    if (k == 1) cross(e2, e3, c);
    else if (k == 2) cross(e3, e1, c);
    else cross(e1, e2, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = c[d] / (T)6;
  }
}

}  // namespace mgpbd
