// ARAP constraint rows (Sec. 5.3, Eq. 8, As-Rigid-As-Possible constraints): per tet
// (x0, x1, x2, x3), F = Ds Dm^-1 with Ds = [x1 - x0, x2 - x0, x3 - x0] and
// Dm the same matrix at rest, C = |F - R|_F^2 with R the rotation nearest
// to F (det R = +1; an inverted tet keeps C > 0), and the gradient
// dC/dDs = 2 (F - R) Dm^-T: column k - 1 is the gradient of slot k, slot 0
// takes the negated sum. One thread per row.
//
// R = U V^T from the eigen-decomposition F^T F = V S^2 V^T, computed by the
// cyclic Jacobi method (Golub and Van Loan, Matrix Computations, Sec. 8.5):
// sweeps of plane rotations a <- J^T a J over the pairs (0,1), (0,2), (1,2)
// until the off-diagonal mass is below 1e-30 of the whole; eigenvectors in
// descending eigenvalue order with det V = +1; u1, u2 = F v1, F v2
// normalised (u2 first made orthogonal to u1), u3 = u1 x u2; R = I when
// rank(F) <= 1 (no unique nearest rotation). Every product is formed as
// (a0 b0 + a1 b1) + a2 b2 with IEEE double operations (no contraction), so
// the result is a fixed function of the inputs. Dm^-1 comes from Gauss-Jordan
// elimination with partial pivoting, once at creation.
#include "xpbd.hpp"

namespace mgpbd {

namespace {

// o = a b for row-major 3x3 matrices
__device__ __forceinline__ void mul3(const double (&a)[9], const double (&b)[9], double (&o)[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      o[3 * i + j] = (a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j]) + a[3 * i + 2] * b[6 + j];
}

// one Jacobi rotation in the plane (P, Q): a <- J^T a J, v <- v J
template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(double (&a)[9], double (&v)[9]) {
  const double apq = a[3 * P + Q];
  if (apq == 0.0) return;
  const double tau = (a[3 * Q + Q] - a[3 * P + P]) / (2.0 * apq);
  const double t = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                              : -1.0 / (-tau + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
  double J[9], Jt[9], tmp[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) J[i] = (i % 4 == 0) ? 1.0 : 0.0;
  J[3 * P + P] = c;
  J[3 * P + Q] = s;
  J[3 * Q + P] = -s;
  J[3 * Q + Q] = c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Jt[3 * j + i] = J[3 * i + j];
  mul3(Jt, a, tmp);
  mul3(tmp, J, a);
  mul3(v, J, tmp);
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = tmp[i];
}

// columns I and J of V (eigenvectors) swap when eigenvalue J exceeds I's
template <int I, int J>
__device__ __forceinline__ void order_pair(double (&lam)[3], double (&V)[9]) {
  if (lam[J] > lam[I]) {
    const double t = lam[I];
    lam[I] = lam[J];
    lam[J] = t;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = V[3 * d + I];
      V[3 * d + I] = V[3 * d + J];
      V[3 * d + J] = x;
    }
  }
}

// R (row-major) nearest to F (row-major)
__device__ void nearest_rotation(const double (&F)[9], double (&R)[9]) {
  double Ft[9], S[9], V[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Ft[3 * j + i] = F[3 * i + j];
  mul3(Ft, F, S);
#pragma unroll
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, all = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      all += S[i] * S[i];
      if (i % 4 != 0) off += S[i] * S[i];
    }
    if (off <= 1e-30 * all) break;
    jacobi_rotate<0, 1>(S, V);
    jacobi_rotate<0, 2>(S, V);
    jacobi_rotate<1, 2>(S, V);
  }
  double lam[3] = {S[0], S[4], S[8]};
  order_pair<0, 1>(lam, V);
  order_pair<0, 2>(lam, V);
  order_pair<1, 2>(lam, V);
  double v0[3], v1[3], v2[3];   // eigenvectors, descending eigenvalue
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    v0[d] = V[3 * d];
    v1[d] = V[3 * d + 1];
    v2[d] = V[3 * d + 2];
  }
  const double det = v0[0] * (v1[1] * v2[2] - v1[2] * v2[1]) -
                     v0[1] * (v1[0] * v2[2] - v1[2] * v2[0]) +
                     v0[2] * (v1[0] * v2[1] - v1[1] * v2[0]);
  if (det < 0.0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) v2[d] = -v2[d];
  }
  double u0[3], u1[3], u2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u0[d] = (F[3 * d] * v0[0] + F[3 * d + 1] * v0[1]) + F[3 * d + 2] * v0[2];
    u1[d] = (F[3 * d] * v1[0] + F[3 * d + 1] * v1[1]) + F[3 * d + 2] * v1[2];
  }
  const double n0 = sqrt((u0[0] * u0[0] + u0[1] * u0[1]) + u0[2] * u0[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) u0[d] /= n0;
  const double pr = (u0[0] * u1[0] + u0[1] * u1[1]) + u0[2] * u1[2];
#pragma unroll
  for (int d = 0; d < 3; ++d) u1[d] -= pr * u0[d];
  const double n1 = sqrt((u1[0] * u1[0] + u1[1] * u1[1]) + u1[2] * u1[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) u1[d] /= n1;
  u2[0] = u0[1] * u1[2] - u0[2] * u1[1];
  u2[1] = u0[2] * u1[0] - u0[0] * u1[2];
  u2[2] = u0[0] * u1[1] - u0[1] * u1[0];
  const bool ok = n0 > 0.0 && n1 > 0.0;   // rank(F) <= 1: not unique, R = I
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double r = (u0[i] * v0[j] + u1[i] * v1[j]) + u2[i] * v2[j];
      R[3 * i + j] = ok ? r : (i == j ? 1.0 : 0.0);
    }
}

}  // namespace

// Gauss-Jordan with partial pivoting on [Dm | I] (runs once per body; the
// pivot rows are chosen at run time, so the matrix may live in scratch)
__global__ __launch_bounds__(kBlock) void k_arap_rest(int64_t m, const int32_t *__restrict__ rv,
                                                      const int8_t *__restrict__ kind,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z,
                                                      double *__restrict__ dm_inv,
                                                      double *__restrict__ det6) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m || !kind[r]) return;
  const int32_t *v = rv + 4 * r;
  double M[3][6];   // M[d][k] = (x_{k+1} - x_0)_d, then the identity
  for (int k = 0; k < 3; ++k) {
    const int32_t q = v[k + 1], o = v[0];
    M[0][k] = x[q] - x[o];
    M[1][k] = y[q] - y[o];
    M[2][k] = z[q] - z[o];
  }
  // det Dm (six times the rest volume), checked by the host to be > 0
  det6[r] = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
            M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
            M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i][3 + j] = (i == j) ? 1.0 : 0.0;
  bool singular = false;
  for (int c = 0; c < 3 && !singular; ++c) {
    int p = c;
    for (int q = c + 1; q < 3; ++q)
      if (fabs(M[q][c]) > fabs(M[p][c])) p = q;
    if (M[p][c] == 0.0) {
      singular = true;
      break;
    }
    if (p != c)
      for (int j = 0; j < 6; ++j) {
        const double t = M[c][j];
        M[c][j] = M[p][j];
        M[p][j] = t;
      }
    const double piv = M[c][c];
    for (int j = 0; j < 6; ++j) M[c][j] /= piv;
    for (int q = 0; q < 3; ++q) {
      if (q == c) continue;
      const double f = M[q][c];
      for (int j = 0; j < 6; ++j) M[q][j] -= f * M[c][j];
    }
  }
  double *o = dm_inv + 9 * r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o[3 * i + j] = singular ? 0.0 : M[i][3 + j];
}

__global__ __launch_bounds__(kBlock) void k_arap(int64_t m, const int32_t *__restrict__ rv,
                                                 const int8_t *__restrict__ kind,
                                                 const double *__restrict__ dm_inv,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 const double *__restrict__ z,
                                                 double *__restrict__ C,
                                                 double *__restrict__ grad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m || !kind[r]) return;
  const int32_t *v = rv + 4 * r;
  double Ds[9], Dm[9];   // Ds[3 d + k] = (x_{k+1} - x_0)_d
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t q = v[k + 1], o = v[0];
    Ds[k] = x[q] - x[o];
    Ds[3 + k] = y[q] - y[o];
    Ds[6 + k] = z[q] - z[o];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) Dm[i] = dm_inv[9 * r + i];
  double F[9], R[9];
  mul3(Ds, Dm, F);
  nearest_rotation(F, R);
  double c = 0.0, P[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double e = F[i] - R[i];
    c += e * e;
    P[i] = 2.0 * e;
  }
  C[r] = c;
  // H = P Dm^-T; slot k (1..3) is column k - 1 of H
  double DmT[9], H[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) DmT[3 * j + i] = Dm[3 * i + j];
  mul3(P, DmT, H);
  double *go = grad + 12 * r;
#pragma unroll
  for (int k = 1; k <= 3; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) go[3 * k + d] = H[3 * d + (k - 1)];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    go[d] = -((H[3 * d] + H[3 * d + 1]) + H[3 * d + 2]);
}

void launch_arap_rest(int64_t m, const int32_t *rv, const int8_t *kind,
                      const double *const *rest, double *dm_inv, double *det6, hipStream_t s) {
  if (m && kind)
    k_arap_rest<<<blocks_for(m, kBlock), kBlock, 0, s>>>(m, rv, kind, rest[0], rest[1], rest[2],
                                                         dm_inv, det6);
}

void launch_arap_constraints(int64_t m, const int32_t *rv, const int8_t *kind,
                             const double *dm_inv, const double *const *xyz, double *C,
                             double *grad, hipStream_t s) {
  if (m && kind)
    k_arap<<<blocks_for(m, kBlock), kBlock, 0, s>>>(m, rv, kind, dm_inv, xyz[0], xyz[1], xyz[2],
                                                    C, grad);
}

}  // namespace mgpbd
