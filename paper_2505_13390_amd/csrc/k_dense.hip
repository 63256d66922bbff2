// Coarsest level: dense FP64 Cholesky factorisation and explicit inverse.
// The last level has at most dense_max rows; it is factorised once per global
// iteration (its Galerkin values change) and every V-cycle then applies the
// inverse as a dense product. The trailing updates of the factorisation and
// the product Y^T Y that forms the inverse run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64) in 16 x 16 tiles.
#include "seg.hpp"
#include "setup.hpp"

namespace mgpbd {

typedef double v4d __attribute__((ext_vector_type(4)));

// C(16x16 tile at r0, c0) -= A(r0.., k0..k0+kk) * B(c0.., k0..k0+kk)^T with
// A and B row-major n x n; one wavefront, kk a multiple of 4.
// MFMA f64 16x16x4 operand layout (wave64): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; lane l holds D[l / 16 + 4 q][l % 16], q = 0..3.
__device__ __forceinline__ v4d mfma_tile_nt(const double *__restrict__ M, int64_t n, int64_t r0,
                                            int64_t c0, int64_t k0, int64_t kk, v4d acc) {
  const int lane = threadIdx.x & 63;
  const int64_t ar = r0 + (lane & 15), bc = c0 + (lane & 15);
  const int kq = lane >> 4;
  for (int64_t k = k0; k < k0 + kk; k += 4) {
    double a = M[ar * n + k + kq];
    double b = M[bc * n + k + kq];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// rows of a 16-column panel that the factorisation keeps in LDS (60 KB)
constexpr int kPanelRows = 480;
// threads of the workgroup that factorises and inverts one matrix: the
// trailing updates and the product Z Z^T spread their 16 x 16 tiles over its
// sixteen wavefronts
constexpr int kDenseThreads = 1024;
static_assert(kDenseThreads / kWave <= 16,
              "the triangular inverse gives each wavefront a kPanelRows slice of the panel buffer");

// Factorisation + inverse of one matrix by one workgroup of kDenseThreads
// threads; returns nonzero (in every thread) when a pivot is not positive.
// n is padded by the caller to a multiple of 16 with an identity block (the
// padding does not change the inverse of the leading n x n part).
__device__ int chol_inverse_block(int64_t n, int64_t np, double *__restrict__ D,
                                  double *__restrict__ Y, double *__restrict__ Ainv) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, nw = nthr >> 6, lane = tid & 63;
  __shared__ int bad;
  if (tid == 0) bad = 0;
  __syncthreads();
  // ---- blocked right-looking Cholesky, 16-column panels ----
  // The panel (rows j0..np-1 of columns j0..j0+15) is factorised in LDS when
  // it fits (its sixteen column steps are chains of barriers and dependent
  // loads, which global memory makes slow), then written back for the
  // trailing update; the arithmetic is the same either way.
  __shared__ double panel[kPanelRows * 16];
  const bool in_lds = np <= kPanelRows;
  for (int64_t j0 = 0; j0 < np; j0 += 16) {
    double *Pb = in_lds ? panel : D + j0 * np + j0;   // element (i, k) at
    const int64_t ps = in_lds ? 16 : np;               // Pb[(i - j0) ps + k - j0]
    if (in_lds) {
      __syncthreads();
      for (int64_t idx = tid; idx < (np - j0) * 16; idx += nthr)
        panel[idx] = D[(j0 + idx / 16) * np + j0 + idx % 16];
    }
    // panel factorisation (columns j0..j0+15), scalar
    for (int64_t j = j0; j < j0 + 16; ++j) {
      __syncthreads();
      double *pj = Pb + (j - j0) * ps + (j - j0);
      if (tid == 0) {
        double d = *pj;
        if (!(d > 0.0)) bad = 1;
        *pj = sqrt(d > 0.0 ? d : 1.0);
      }
      __syncthreads();
      if (bad) break;
      double ljj = *pj;
      for (int64_t i = j + 1 + tid; i < np; i += nthr) {
        double *e = Pb + (i - j0) * ps + (j - j0);
        *e = *e / ljj;
      }
      __syncthreads();
      // update the rest of the panel columns j+1..j0+15 for all rows below
      for (int64_t idx = tid; idx < (np - j - 1) * (j0 + 15 - j); idx += nthr) {
        int64_t w = j0 + 15 - j;
        int64_t i = j + 1 + idx / w, k = j + 1 + idx % w;
        if (k <= i) {
          double *e = Pb + (i - j0) * ps + (k - j0);
          *e = *e - Pb[(i - j0) * ps + (j - j0)] * Pb[(k - j0) * ps + (j - j0)];
        }
      }
    }
    __syncthreads();
    if (in_lds) {
      for (int64_t idx = tid; idx < (np - j0) * 16; idx += nthr)
        D[(j0 + idx / 16) * np + j0 + idx % 16] = panel[idx];
      __syncthreads();
    }
    if (bad) break;
    // trailing update with the FP64 matrix cores: tiles (ti, tk) below the
    // panel, tk <= ti, D[ti,tk] -= L[ti, panel] L[tk, panel]^T
    int64_t t0 = j0 + 16;
    int64_t nt = (np - t0) / 16;
    for (int64_t t = wave; t < nt * (nt + 1) / 2; t += nw) {
      // map t -> (ti, tk) with tk <= ti
      int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      while (ti * (ti + 1) / 2 > t) --ti;
      int64_t tk = t - ti * (ti + 1) / 2;
      int64_t r0 = t0 + ti * 16, c0 = t0 + tk * 16;
      v4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mfma_tile_nt(D, np, r0, c0, j0, 16, acc);
      const int cc = lane & 15, rb = lane >> 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int64_t rr = r0 + rb + 4 * q, cl = c0 + cc;
        if (cl <= rr) D[rr * np + cl] = D[rr * np + cl] - acc[q];
      }
    }
  }
  __syncthreads();
  if (bad) return 1;
  // ---- Z = (L^-1)^T: column c of L^-1 is stored as row c of Z ----
  if (in_lds) {
    // One wavefront per column: each substitution step's dot product is split
    // over the 64 lanes (lane l owns the entries k = c + l mod 64, which it
    // also keeps in this wave's slice of the now free panel buffer) and summed
    // by a butterfly, so a column costs np - c short steps instead of one
    // thread's (np - c)^2 / 2 dependent multiply-adds.
    double *own = panel + wave * kPanelRows;
    __syncthreads();
    for (int64_t c = wave; c < np; c += nw) {
      double *zc = Y + c * np;
      for (int64_t i = lane; i < c; i += kWave) zc[i] = 0.0;
      for (int64_t i = c; i < np; ++i) {
        double s = 0.0;
        for (int64_t k = c + lane; k < i; k += kWave) s += D[i * np + k] * own[k];
        s = group_sum<kWave>(s);
        const double zi = (((i == c) ? 1.0 : 0.0) - s) / D[i * np + i];
        if (((i - c) & (kWave - 1)) == lane) {
          own[i] = zi;
          zc[i] = zi;
        }
      }
    }
  } else {
    // thread c solves column c, walking its row of Z and row i of L
    for (int64_t c = tid; c < np; c += nthr) {
      double *zc = Y + c * np;
      for (int64_t i = 0; i < c; ++i) zc[i] = 0.0;
      for (int64_t i = c; i < np; ++i) {
        double s = (i == c) ? 1.0 : 0.0;
        for (int64_t k = c; k < i; ++k) s -= D[i * np + k] * zc[k];
        zc[i] = s / D[i * np + i];
      }
    }
  }
  __syncthreads();
  // ---- Ainv = Z Z^T on the matrix cores: Ainv[r][c] = sum_k Z[r][k] Z[c][k],
  // both operands read along rows of Z ----
  int64_t nt = np / 16;
  for (int64_t t = wave; t < nt * nt; t += nw) {
    int64_t ti = t / nt, tk = t % nt;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    int64_t kstart = (ti > tk ? ti : tk) * 16;   // Z[r][k] = 0 for k < r
    acc = mfma_tile_nt(Y, np, ti * 16, tk * 16, kstart, np - kstart, acc);
    const int cc = lane & 15, rb = lane >> 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int64_t rr = ti * 16 + rb + 4 * q, cl = tk * 16 + cc;
      if (rr < n && cl < n) Ainv[rr * n + cl] = acc[q];
    }
  }
  return 0;
}

// ------------------------------------------------------------ dense batch
__global__ void k_dense_init_batch(const DenseJob *jobs, const int64_t *__restrict__ rp,
                                     const int32_t *__restrict__ col,
                                     const double *__restrict__ val, double *scratch) {
  const DenseJob j = jobs[blockIdx.y];
  const int64_t np = (j.n + 15) / 16 * 16;
  double *P = scratch + j.scratch + np * np;   // padded matrix
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < np * np;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = idx / np, k = idx % np;
    P[idx] = (i == k && i >= j.n) ? 1.0 : 0.0;
  }
}
__global__ void k_dense_scatter_batch(const DenseJob *jobs, const int64_t *__restrict__ rp,
                                      const int32_t *__restrict__ col,
                                      const double *__restrict__ val, double *scratch) {
  const DenseJob j = jobs[blockIdx.y];
  const int64_t np = (j.n + 15) / 16 * 16;
  double *P = scratch + j.scratch + np * np;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < j.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gi = j.row0 + i;
    for (int64_t e = rp[gi]; e < rp[gi + 1]; ++e) P[i * np + (col[e] - j.row0)] = val[e];
  }
}

__global__ __launch_bounds__(kDenseThreads) void k_chol_inverse_batch(const DenseJob *jobs, double *scratch,
                                                            double *ainv, int *status) {
  const DenseJob j = jobs[blockIdx.x];
  const int64_t np = (j.n + 15) / 16 * 16;
  double *Y = scratch + j.scratch;
  double *P = Y + np * np;
  int bad = chol_inverse_block(j.n, np, P, Y, ainv + j.ainv);
  if (threadIdx.x == 0 && bad) atomicExch(status, 1);
}

void launch_dense_factor_batch(int njobs, const DenseJob *jobs, const int64_t *rp,
                               const int32_t *col, const double *val, double *scratch,
                               double *ainv, int *status, hipStream_t s) {
  if (njobs <= 0) return;
  dim3 g(64, njobs);
  k_dense_init_batch<<<g, kBlock, 0, s>>>(jobs, rp, col, val, scratch);
  k_dense_scatter_batch<<<g, kBlock, 0, s>>>(jobs, rp, col, val, scratch);
  k_chol_inverse_batch<<<njobs, kDenseThreads, 0, s>>>(jobs, scratch, ainv, status);
}


}  // namespace mgpbd
