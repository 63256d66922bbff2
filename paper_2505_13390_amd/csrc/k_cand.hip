// Several near-kernel candidates per level (Sec. 4.3 generates six; Sec. 4.1
// forms each next level from a QR factorisation of them). Level l holds K
// candidates B [n][K]. Every aggregate's block of B is factorised by modified
// Gram-Schmidt: column k loses its projections on the columns kept so far,
// one after another, and is kept (normalised) unless what remains is at most
// 1e-8 of its norm (numerically dependent; always so past the aggregate's
// size). The kept columns are the aggregate's columns of P (Q [members][K],
// zeros beyond them), their coefficients R the next level's candidates, and
// the coarse unknowns are the (aggregate, kept column) pairs, numbered
// coff[a] + s. A block of zeros keeps one normalised all-ones column.
//
// The coarse matrix A_c = P^T A P has one dense kq[a] x kq[b] block per pair
// of aggregates that a fine entry connects: entry ((a,s),(b,t)) on or above
// the diagonal is the sum over those fine entries (i, j) in ascending fine
// order of (Q_i,s a_ij) Q_j,t, and the entries below the diagonal take their
// mirrors' values. Its rows list the blocks in ascending aggregate order, so
// row (a, s) = base[a] + s * rowlen[a] and block (a, b) starts cstart[e]
// entries into the row of every (a, s).
#include "setup.hpp"

namespace mgpbd {

constexpr double kQrDrop = 1e-8;

// column k of B [n][K] = x
__global__ void k_put_column(int64_t n, int K, int k, const double *__restrict__ x,
                             double *__restrict__ B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) B[i * K + k] = x[i];
}
void launch_put_column(int64_t n, int K, int k, const double *x, double *B, hipStream_t s) {
  if (n) k_put_column<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, K, k, x, B);
}

// One thread per aggregate (the blocks are small and this runs at setup
// only); the column being orthogonalised lives in its own slot of Q.
__global__ void k_qr_agg(int64_t na, int K, const int64_t *__restrict__ ap,
                         const int32_t *__restrict__ mem, const double *__restrict__ B,
                         double *__restrict__ Q, double *__restrict__ R, int32_t *__restrict__ kq) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  const int64_t b0 = ap[a], s = ap[a + 1] - b0;
  double *Qa = Q + b0 * K;
  double *Ra = R + a * K * K;
  for (int i = 0; i < K * K; ++i) Ra[i] = 0.0;
  for (int64_t i = 0; i < s * K; ++i) Qa[i] = 0.0;
  int kept = 0;
  for (int k = 0; k < K; ++k) {
    double n0 = 0.0;
    for (int64_t t = 0; t < s; ++t) {
      const double v = B[(int64_t)mem[b0 + t] * K + k];
      Qa[t * K + kept] = v;
      n0 = n0 + v * v;
    }
    n0 = sqrt(n0);
    for (int j = 0; j < kept; ++j) {
      double r = 0.0;
      for (int64_t t = 0; t < s; ++t) r = r + Qa[t * K + j] * Qa[t * K + kept];
      Ra[j * K + k] = r;
      for (int64_t t = 0; t < s; ++t) Qa[t * K + kept] = Qa[t * K + kept] - r * Qa[t * K + j];
    }
    double nr = 0.0;
    for (int64_t t = 0; t < s; ++t) nr = nr + Qa[t * K + kept] * Qa[t * K + kept];
    nr = sqrt(nr);
    if (nr > 0.0 && nr > kQrDrop * n0) {
      for (int64_t t = 0; t < s; ++t) Qa[t * K + kept] = Qa[t * K + kept] / nr;
      Ra[kept * K + k] = nr;
      ++kept;
    } else {
      for (int64_t t = 0; t < s; ++t) Qa[t * K + kept] = 0.0;
    }
  }
  if (kept == 0) {
    const double sa = sqrt((double)s);
    for (int64_t t = 0; t < s; ++t) Qa[t * K] = 1.0 / sa;
    Ra[0] = sa;
    kept = 1;
  }
  kq[a] = kept;
}
void launch_qr_agg(int64_t na, int K, const int64_t *ap, const int32_t *mem, const double *B,
                   double *Q, double *R, int32_t *kq, hipStream_t s) {
  if (na) k_qr_agg<<<blocks_for(na, 64), 64, 0, s>>>(na, K, ap, mem, B, Q, R, kq);
}

// next level's candidates: row coff[a] + j = R[a][j][*]
__global__ void k_scatter_r(int64_t na, int K, const int32_t *__restrict__ kq,
                            const int64_t *__restrict__ coff, const double *__restrict__ R,
                            double *__restrict__ Bn) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  for (int j = 0; j < kq[a]; ++j)
    for (int k = 0; k < K; ++k) Bn[(coff[a] + j) * K + k] = R[(a * K + j) * K + k];
}
void launch_scatter_r(int64_t na, int K, const int32_t *kq, const int64_t *coff, const double *R,
                      double *Bn, hipStream_t s) {
  if (na) k_scatter_r<<<blocks_for(na, kBlock), kBlock, 0, s>>>(na, K, kq, coff, R, Bn);
}

// slot[mem[m]] = m (rows outside every aggregate keep their -1)
__global__ void k_member_slots(int64_t nmem, const int32_t *__restrict__ mem,
                               int32_t *__restrict__ slot) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m < nmem) slot[mem[m]] = (int32_t)m;
}
void launch_member_slots(int64_t nmem, const int32_t *mem, int32_t *slot, hipStream_t s) {
  if (nmem) k_member_slots<<<blocks_for(nmem, kBlock), kBlock, 0, s>>>(nmem, mem, slot);
}

// ------------------------------------------------------------ Galerkin
// per aggregate row: where each block starts in the row, the row length and
// the block row's size (kq[a] rows)
__global__ void k_galk_rowlen(int64_t na, const int64_t *__restrict__ arp,
                              const int32_t *__restrict__ acol, const int32_t *__restrict__ kq,
                              int64_t *__restrict__ cstart, int64_t *__restrict__ rowlen,
                              int64_t *__restrict__ blocksz) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  int64_t len = 0;
  for (int64_t e = arp[a]; e < arp[a + 1]; ++e) {
    cstart[e] = len;
    len += kq[acol[e]];
  }
  rowlen[a] = len;
  blocksz[a] = len * kq[a];
}
void launch_galk_rowlen(int64_t na, const int64_t *arp, const int32_t *acol, const int32_t *kq,
                        int64_t *cstart, int64_t *rowlen, int64_t *blocksz, hipStream_t s) {
  if (na)
    k_galk_rowlen<<<blocks_for(na, kBlock), kBlock, 0, s>>>(na, arp, acol, kq, cstart, rowlen,
                                                            blocksz);
}

__global__ void k_galk_pattern(int64_t na, const int32_t *__restrict__ kq,
                               const int64_t *__restrict__ coff, const int64_t *__restrict__ arp,
                               const int32_t *__restrict__ acol, const int64_t *__restrict__ base,
                               const int64_t *__restrict__ rowlen, int64_t *__restrict__ rowptr,
                               int32_t *__restrict__ col) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  for (int s = 0; s < kq[a]; ++s) {
    int64_t k = base[a] + s * rowlen[a];
    rowptr[coff[a] + s] = k;
    for (int64_t e = arp[a]; e < arp[a + 1]; ++e) {
      const int32_t b = acol[e];
      for (int t = 0; t < kq[b]; ++t) col[k++] = (int32_t)(coff[b] + t);
    }
  }
}
void launch_galk_pattern(int64_t na, const int32_t *kq, const int64_t *coff, const int64_t *arp,
                         const int32_t *acol, const int64_t *base, const int64_t *rowlen,
                         int64_t *rowptr, int32_t *col, hipStream_t s) {
  if (na)
    k_galk_pattern<<<blocks_for(na, 64), 64, 0, s>>>(na, kq, coff, arp, acol, base, rowlen,
                                                     rowptr, col);
}

// One thread per aggregate block on or above the diagonal; the K x K sums
// stay in registers.
template <int K>
__global__ __launch_bounds__(kBlock) void k_galk_numeric(
    int64_t annz, const int32_t *__restrict__ acrow, const int32_t *__restrict__ acol,
    const int32_t *__restrict__ amirror, const int64_t *__restrict__ gl_ptr,
    const int32_t *__restrict__ gl_idx, const int32_t *__restrict__ gl_row,
    const int32_t *__restrict__ fcol, const double *__restrict__ fval,
    const int32_t *__restrict__ slot, const double *__restrict__ Q,
    const int32_t *__restrict__ kq, const int64_t *__restrict__ coff,
    const int64_t *__restrict__ crp, const int64_t *__restrict__ cstart,
    double *__restrict__ cval, float *__restrict__ cval32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= annz) return;
  const int32_t a = acrow[e], b = acol[e];
  if (b < a) return;
  double acc[K][K];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int t = 0; t < K; ++t) acc[s][t] = 0.0;
  for (int64_t g = gl_ptr[e]; g < gl_ptr[e + 1]; ++g) {
    const int32_t f = gl_idx[g];
    const double v = fval[f];
    const double *qi = Q + (int64_t)slot[gl_row[g]] * K;
    const double *qj = Q + (int64_t)slot[fcol[f]] * K;
    double qjv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) qjv[t] = qj[t];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const double w = qi[s] * v;
#pragma unroll
      for (int t = 0; t < K; ++t) acc[s][t] = acc[s][t] + w * qjv[t];
    }
  }
  const int ka = kq[a], kb = kq[b];
  const int64_t ca = coff[a], cb = coff[b];
  const int64_t ea = cstart[e];
  const int64_t eb = cstart[amirror[e]];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if (s >= ka || t >= kb) continue;
      if (a == b && t < s) continue;   // the lower half of a diagonal block mirrors the upper
      const double v = acc[s][t];
      const int64_t up = crp[ca + s] + ea + t;    // ((a,s),(b,t))
      const int64_t lo = crp[cb + t] + eb + s;    // ((b,t),(a,s))
      cval[up] = v;
      cval[lo] = v;
      if (cval32) {
        cval32[up] = (float)v;
        cval32[lo] = (float)v;
      }
    }
}
void launch_galk_numeric(int K, int64_t annz, const int32_t *acrow, const int32_t *acol,
                         const int32_t *amirror, const int64_t *gl_ptr, const int32_t *gl_idx,
                         const int32_t *gl_row, const int32_t *fcol, const double *fval,
                         const int32_t *slot, const double *Q, const int32_t *kq,
                         const int64_t *coff, const int64_t *crp, const int64_t *cstart,
                         double *cval, float *cval32, hipStream_t s) {
  if (!annz) return;
  const int grid = blocks_for(annz, kBlock);
#define G_(KK)                                                                                 \
  k_galk_numeric<KK><<<grid, kBlock, 0, s>>>(annz, acrow, acol, amirror, gl_ptr, gl_idx,        \
                                             gl_row, fcol, fval, slot, Q, kq, coff, crp,       \
                                             cstart, cval, cval32)
  switch (K) {
    case 2: G_(2); break;
    case 3: G_(3); break;
    case 4: G_(4); break;
    case 5: G_(5); break;
    case 6: G_(6); break;
    case 7: G_(7); break;
    default: G_(8); break;
  }
#undef G_
}

// ------------------------------------------------------------ transfers
// rc[(a, s)] = sum over the aggregate's rows in ascending order of Q_i,s res_i
template <class T>
__global__ void k_restrict_k(const int *done, int64_t na, int K, const int32_t *__restrict__ kq,
                             const int64_t *__restrict__ coff, const int64_t *__restrict__ ap,
                             const int32_t *__restrict__ mem, const T *__restrict__ Q,
                             const T *__restrict__ res, T *__restrict__ rc) {
  if (done && *done) return;
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  for (int s = 0; s < kq[a]; ++s) {
    T acc = 0;
    for (int64_t m = ap[a]; m < ap[a + 1]; ++m) acc = acc + Q[m * K + s] * res[mem[m]];
    rc[coff[a] + s] = acc;
  }
}
template <class T>
void launch_restrict_k(int64_t na, int K, const int32_t *kq, const int64_t *coff,
                       const int64_t *ap, const int32_t *mem, const T *Q, const T *res, T *rc,
                       const int *done, hipStream_t s) {
  if (na)
    k_restrict_k<T><<<blocks_for(na, kBlock), kBlock, 0, s>>>(done, na, K, kq, coff, ap, mem, Q,
                                                              res, rc);
}

// z_i += sum_s Q_i,s zc[(agg(i), s)]
template <class T>
__global__ void k_prolong_k(const int *done, int64_t n, int K, const int32_t *__restrict__ agg,
                            const int32_t *__restrict__ slot, const int32_t *__restrict__ kq,
                            const int64_t *__restrict__ coff, const T *__restrict__ Q,
                            const T *__restrict__ zc, T *__restrict__ z) {
  if (done && *done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t a = agg[i];
  if (a < 0) return;
  const T *qi = Q + (int64_t)slot[i] * K;
  const T *zca = zc + coff[a];
  T acc = 0;
  for (int s = 0; s < kq[a]; ++s) acc = acc + qi[s] * zca[s];
  z[i] = z[i] + acc;
}
template <class T>
void launch_prolong_k(int64_t n, int K, const int32_t *agg, const int32_t *slot,
                      const int32_t *kq, const int64_t *coff, const T *Q, const T *zc, T *z,
                      const int *done, hipStream_t s) {
  if (n)
    k_prolong_k<T><<<blocks_for(n, kBlock), kBlock, 0, s>>>(done, n, K, agg, slot, kq, coff, Q,
                                                            zc, z);
}

#define MG_INST(T)                                                                              \
  template void launch_restrict_k<T>(int64_t, int, const int32_t *, const int64_t *,           \
                                     const int64_t *, const int32_t *, const T *, const T *,    \
                                     T *, const int *, hipStream_t);                            \
  template void launch_prolong_k<T>(int64_t, int, const int32_t *, const int32_t *,            \
                                    const int32_t *, const int64_t *, const T *, const T *, T *, \
                                    const int *, hipStream_t);
MG_INST(double)
MG_INST(float)
#undef MG_INST

}  // namespace mgpbd
