// AMG setup kernels. Every value that feeds an aggregation decision is
// computed as a fixed-order sequence of IEEE operations (no contraction), so
// the setup is a pure function of the bits of A:
//  - strength of connection (Sec. 4.1) as a squared comparison;
//  - aggregation pass 1 as the greedy distance-2 independent set in
//    descending priority, computed by rounds: a node becomes a root when it
//    holds the largest key among undecided nodes within distance 2 and no
//    root is that close; nodes within distance 2 of a root drop out. This
//    selects the same set as the sequential greedy visit;
//  - pass 2: the strongest pass-1 neighbour, ties to the smallest index;
//  - greedy colouring by Jones-Plassmann rounds (same result as the greedy
//    visit in priority order) for the multicolour Gauss-Seidel sweeps of the
//    near-kernel (Sec. 4.3), one lane per row summing in ascending column;
//  - injection of the candidate into P with a one-column QR per aggregate;
//  - Galerkin A_{l+1} = P^T A_l P (Eq. 6): each coarse entry sums its fine
//    contributions in ascending fine order; the lower triangle mirrors the
//    upper one.
#include "setup.hpp"

namespace mgpbd {

#define MG_DISPATCH_G(lanes, LAUNCH) \
  switch (lanes) {                   \
    case 4: LAUNCH(4); break;        \
    case 8: LAUNCH(8); break;        \
    case 16: LAUNCH(16); break;      \
    case 32: LAUNCH(32); break;      \
    default: LAUNCH(64); break;      \
  }

// ------------------------------------------------------------ diagonal
// Structure check of a caller CSR before any kernel indexes through it: each
// row's bounds must satisfy 0 = rp[0] <= rp[i] <= rp[i+1] <= nnz and its
// columns must lie in [0, n) and ascend strictly. A row whose bounds are bad
// is flagged without reading its columns, so the check itself reads only
// rp[0..n] and col[0..nnz).
__global__ void k_validate_csr(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                               const int32_t *__restrict__ col, int *bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t lo = rp[i], hi = rp[i + 1];
  bool ok = lo >= 0 && lo <= hi && hi <= nnz && (i > 0 || lo == 0);
  if (ok) {
    int64_t prev = -1;
    for (int64_t e = lo; e < hi; ++e) {
      const int64_t c = col[e];
      if (c <= prev || c >= n) { ok = false; break; }
      prev = c;
    }
  }
  if (!ok) atomicExch(bad, 1);
}
void launch_validate_csr(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *col, int *bad,
                         hipStream_t s) {
  if (n) k_validate_csr<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, nnz, rp, col, bad);
}

__global__ void k_diagpos(int64_t n, const int64_t *__restrict__ rp,
                          const int32_t *__restrict__ col, int64_t *__restrict__ dpos, int *bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t lo = rp[i], hi = rp[i + 1] - 1, found = -1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    int32_t c = col[mid];
    if (c == (int32_t)i) { found = mid; break; }
    if (c < (int32_t)i) lo = mid + 1; else hi = mid - 1;
  }
  dpos[i] = found;
  if (found < 0) atomicExch(bad, 1);
}
void launch_diagpos(int64_t n, const int64_t *rp, const int32_t *col, int64_t *dpos, int *bad,
                    hipStream_t s) {
  if (n) k_diagpos<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, rp, col, dpos, bad);
}

__global__ void k_extract_diag(int64_t n, const int64_t *__restrict__ dpos,
                               const double *__restrict__ val, double *__restrict__ diag,
                               double *__restrict__ dinv, float *__restrict__ dinv32, int *bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = val[dpos[i]];
  if (!(d > 0.0) || d > 1.7976931348623157e308) atomicExch(bad, 1);
  diag[i] = d;
  double di = 1.0 / d;
  dinv[i] = di;
  if (dinv32) dinv32[i] = (float)di;
}
void launch_extract_diag(int64_t n, const int64_t *dpos, const double *val, double *diag,
                         double *dinv, float *dinv32, int *bad, hipStream_t s) {
  if (n) k_extract_diag<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, dpos, val, diag, dinv, dinv32, bad);
}

// ------------------------------------------------------------ strength
template <int G>
__global__ __launch_bounds__(kBlock) void k_strong(int64_t n, const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const double *__restrict__ val,
                                                   const double *__restrict__ diag, double theta2,
                                                   uint8_t *__restrict__ strong,
                                                   uint8_t *__restrict__ conn) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t i = base + grp;
    bool ok = i < hi;
    int any = 0;
    if (ok) {
      double di = fabs(diag[i]);
      for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G) {
        int32_t j = col[e];
        double a = val[e];
        uint8_t st = (j != (int32_t)i) && (a * a >= theta2 * (di * fabs(diag[j])));
        strong[e] = st;
        any |= st;
      }
    }
    any = group_sum<G>(any);
    if (ok && sub == 0) conn[i] = any > 0;
  }
}
void launch_strong(const CsrView<double> &A, const double *diag, double theta2, uint8_t *strong,
                   uint8_t *conn, hipStream_t s) {
  if (!A.n) return;
  int grid = grid_for(A.n * A.lanes, kBlock);
#define L_(G) k_strong<G><<<grid, kBlock, 0, s>>>(A.n, A.rowptr, A.col, A.val, diag, theta2, strong, conn)
  MG_DISPATCH_G(A.lanes, L_);
#undef L_
}

// ------------------------------------------------------------ MIS-2
constexpr uint64_t kRootKey = ~0ULL;

// m1[i] = max of key over i and its strong neighbours
template <int G>
__global__ __launch_bounds__(kBlock) void k_mis_max1(int64_t n, const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const uint8_t *__restrict__ strong,
                                                     const uint64_t *__restrict__ key,
                                                     uint64_t *__restrict__ m1) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t i = base + grp;
    bool ok = i < hi;
    uint64_t m = 0;
    if (ok) {
      m = key[i];
      for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G)
        if (strong[e]) {
          uint64_t k = key[col[e]];
          m = k > m ? k : m;
        }
    }
    m = group_max_u64<G>(m);
    if (ok && sub == 0) m1[i] = m;
  }
}

// decide undecided nodes from the distance-2 maximum
template <int G>
__global__ __launch_bounds__(kBlock) void k_mis_max2(int64_t n, const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const uint8_t *__restrict__ strong,
                                                     const uint64_t *__restrict__ m1,
                                                     uint64_t *__restrict__ key, int *undecided) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t i = base + grp;
    bool ok = i < hi;
    uint64_t ki = ok ? key[i] : 0;
    bool und = ok && ki != 0 && ki != kRootKey;
    uint64_t m = 0;
    if (und) {
      m = m1[i];
      for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G)
        if (strong[e]) {
          uint64_t k = m1[col[e]];
          m = k > m ? k : m;
        }
    }
    m = group_max_u64<G>(m);
    if (und && sub == 0) {
      if (m == kRootKey) key[i] = 0;
      else if (m == ki) key[i] = kRootKey;
      else atomicAdd(undecided, 1);
    }
  }
}
void launch_mis_round(const CsrView<double> &A, const uint8_t *strong, uint64_t *key,
                      uint64_t *m1, int *undecided, hipStream_t s) {
  int grid = grid_for(A.n * A.lanes, kBlock);
#define L1_(G) k_mis_max1<G><<<grid, kBlock, 0, s>>>(A.n, A.rowptr, A.col, strong, key, m1)
#define L2_(G) k_mis_max2<G><<<grid, kBlock, 0, s>>>(A.n, A.rowptr, A.col, strong, m1, key, undecided)
  MG_DISPATCH_G(A.lanes, L1_);
  MG_DISPATCH_G(A.lanes, L2_);
#undef L1_
#undef L2_
}

__global__ void k_root_flags(int64_t n, const uint64_t *__restrict__ key, int32_t *__restrict__ f) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = key[i] == kRootKey;
}
void launch_root_flags(int64_t n, const uint64_t *key, int32_t *flag, hipStream_t s) {
  if (n) k_root_flags<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, key, flag);
}

// pass 1: roots and their strong neighbours (a node has at most one root
// among its strong neighbours since roots are >= 3 apart)
template <int G>
__global__ __launch_bounds__(kBlock) void k_pass1(int64_t n, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const uint8_t *__restrict__ strong,
                                                  const uint64_t *__restrict__ key,
                                                  const int64_t *__restrict__ rid,
                                                  int32_t *__restrict__ agg1) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t i = base + grp;
    bool ok = i < hi;
    int64_t found = -1;
    if (ok) {
      if (key[i] == kRootKey) {
        found = rid[i];
      } else {
        for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G)
          if (strong[e] && key[col[e]] == kRootKey) found = rid[col[e]];
      }
    }
    // at most one distinct value >= 0 in the group
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      int64_t o = __shfl_xor(found, off, G);
      found = o > found ? o : found;
    }
    if (ok && sub == 0) agg1[i] = (int32_t)found;
  }
}
void launch_pass1(const CsrView<double> &A, const uint8_t *strong, const uint64_t *key,
                  const int64_t *rid, int32_t *agg1, hipStream_t s) {
  if (!A.n) return;
  int grid = grid_for(A.n * A.lanes, kBlock);
#define L_(G) k_pass1<G><<<grid, kBlock, 0, s>>>(A.n, A.rowptr, A.col, strong, key, rid, agg1)
  MG_DISPATCH_G(A.lanes, L_);
#undef L_
}

// pass 2: remaining connected nodes join the pass-1 aggregate of their
// strongest strong neighbour; ties go to the smallest neighbour index
template <int G>
__global__ __launch_bounds__(kBlock) void k_pass2(int64_t n, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  const uint8_t *__restrict__ strong,
                                                  const uint8_t *__restrict__ conn,
                                                  const int32_t *__restrict__ agg1,
                                                  int32_t *__restrict__ agg) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t i = base + grp;
    bool ok = i < hi;
    bool need = ok && agg1[i] < 0 && conn[i];
    double best = -1.0;
    int32_t bj = 0x7fffffff;
    if (need) {
      for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G) {
        int32_t j = col[e];
        if (!strong[e] || agg1[j] < 0) continue;
        double a = fabs(val[e]);
        if (a > best) { best = a; bj = j; }   // ascending j within the lane
      }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      double ob = __shfl_xor(best, off, G);
      int32_t oj = __shfl_xor(bj, off, G);
      if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
    }
    if (ok && sub == 0) agg[i] = need ? (best >= 0.0 ? agg1[bj] : -1) : agg1[i];
  }
}
void launch_pass2(const CsrView<double> &A, const uint8_t *strong, const uint8_t *conn,
                  const int32_t *agg1, int32_t *agg, hipStream_t s) {
  if (!A.n) return;
  int grid = grid_for(A.n * A.lanes, kBlock);
#define L_(G) k_pass2<G><<<grid, kBlock, 0, s>>>(A.n, A.rowptr, A.col, A.val, strong, conn, agg1, agg)
  MG_DISPATCH_G(A.lanes, L_);
#undef L_
}

// ------------------------------------------------------------ members
__global__ void k_count_members(int64_t n, const int32_t *__restrict__ agg, int32_t *cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && agg[i] >= 0) atomicAdd(&cnt[agg[i]], 1);
}
void launch_count_members(int64_t n, const int32_t *agg, int32_t *cnt, hipStream_t s) {
  if (n) k_count_members<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, agg, cnt);
}
__global__ void k_scatter_members(int64_t n, const int32_t *__restrict__ agg,
                                  const int64_t *__restrict__ ptr, int32_t *cursor,
                                  int32_t *__restrict__ mem) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t a = agg[i];
  if (a < 0) return;
  int32_t k = atomicAdd(&cursor[a], 1);
  mem[ptr[a] + k] = (int32_t)i;
}
void launch_scatter_members(int64_t n, const int32_t *agg, const int64_t *ptr, int32_t *cursor,
                            int32_t *mem, hipStream_t s) {
  if (n) k_scatter_members<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, agg, ptr, cursor, mem);
}
// each segment sorted ascending (insertion sort; segments are aggregates)
__global__ void k_sort_segments(int64_t nseg, const int64_t *__restrict__ ptr, int32_t *mem) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nseg) return;
  int64_t b0 = ptr[a], b1 = ptr[a + 1];
  for (int64_t k = b0 + 1; k < b1; ++k) {
    int32_t v = mem[k];
    int64_t q = k - 1;
    while (q >= b0 && mem[q] > v) { mem[q + 1] = mem[q]; --q; }
    mem[q + 1] = v;
  }
}
void launch_sort_segments(int64_t nseg, const int64_t *ptr, int32_t *mem, hipStream_t s) {
  if (nseg) k_sort_segments<<<blocks_for(nseg, 64), 64, 0, s>>>(nseg, ptr, mem);
}

// ------------------------------------------------------------ colouring
constexpr int kMaxColors = 256;

// Jones-Plassmann colouring driven by counters: cnt[i] = number of
// neighbours with a higher key; a row is coloured once that count reaches
// zero (all higher-priority neighbours coloured), with the smallest colour
// none of them uses, which is exactly the greedy colouring in descending key
// order. Each round colours one frontier and decrements the counters of the
// lower-priority neighbours; rows reaching zero form the next frontier.
template <int G>
__global__ __launch_bounds__(kBlock) void k_color_count(int64_t n, const int64_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const uint64_t *__restrict__ key,
                                                        int32_t *__restrict__ cnt,
                                                        int32_t *__restrict__ front, int *nfront) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(n, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    const int64_t i = base + grp;
    const bool ok = i < hi;
    int c = 0;
    if (ok) {
      const uint64_t ki = key[i];
      for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G) {
        const int32_t j = col[e];
        if (j != (int32_t)i && key[j] > ki) ++c;
      }
    }
    c = group_sum<G, int>(c);
    if (ok && sub == 0) {
      cnt[i] = c;
      if (c == 0) front[atomicAdd(nfront, 1)] = (int32_t)i;
    }
  }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_color_front(
    int64_t nf, const int32_t *__restrict__ front, const int64_t *__restrict__ rp,
    const int32_t *__restrict__ col, const uint64_t *__restrict__ key, int32_t *color,
    int32_t *cnt, int32_t *__restrict__ next, int *nnext, int *overflow) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(nf, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    const int64_t f = base + grp;
    const bool ok = f < hi;
    const int32_t i = ok ? front[f] : 0;
    uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
    int over = 0;
    if (ok) {
      const uint64_t ki = key[i];
      for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G) {
        const int32_t j = col[e];
        if (j == i || key[j] < ki) continue;
        const int32_t cj = color[j];
        if (cj < 0 || cj >= kMaxColors) { over = 1; continue; }
        const uint64_t bit = 1ULL << (cj & 63);
        if (cj < 64) m0 |= bit; else if (cj < 128) m1 |= bit; else if (cj < 192) m2 |= bit; else m3 |= bit;
      }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      m0 |= __shfl_xor(m0, off, G);
      m1 |= __shfl_xor(m1, off, G);
      m2 |= __shfl_xor(m2, off, G);
      m3 |= __shfl_xor(m3, off, G);
      over |= __shfl_xor(over, off, G);
    }
    if (!ok) continue;
    if (sub == 0) {
      int c = -1;
      if (~m0) c = __ffsll((long long)~m0) - 1;
      else if (~m1) c = 64 + __ffsll((long long)~m1) - 1;
      else if (~m2) c = 128 + __ffsll((long long)~m2) - 1;
      else if (~m3) c = 192 + __ffsll((long long)~m3) - 1;
      if (over || c < 0) atomicExch(overflow, 1);
      color[i] = c < 0 ? kMaxColors : c;
    }
    // release the lower-priority neighbours (the colour is read in a later launch)
    const uint64_t ki = key[i];
    for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G) {
      const int32_t j = col[e];
      if (j == i || key[j] > ki) continue;
      if (atomicSub(&cnt[j], 1) == 1) next[atomicAdd(nnext, 1)] = j;
    }
  }
}

void launch_color_count(const CsrView<double> &A, const uint64_t *key, int32_t *cnt,
                        int32_t *front, int *nfront, hipStream_t s) {
  if (!A.n) return;
  const int grid = grid_for(A.n * A.lanes, kBlock);
#define L_(G) k_color_count<G><<<grid, kBlock, 0, s>>>(A.n, A.rowptr, A.col, key, cnt, front, nfront)
  MG_DISPATCH_G(A.lanes, L_);
#undef L_
}
void launch_color_front(const CsrView<double> &A, int64_t nf, const int32_t *front,
                        const uint64_t *key, int32_t *color, int32_t *cnt, int32_t *next,
                        int *nnext, int *overflow, hipStream_t s) {
  if (!nf) return;
  const int grid = grid_for(nf * A.lanes, kBlock);
#define L_(G) k_color_front<G><<<grid, kBlock, 0, s>>>(nf, front, A.rowptr, A.col, key, color, cnt, next, nnext, overflow)
  MG_DISPATCH_G(A.lanes, L_);
#undef L_
}

__global__ void k_count_colors(int64_t n, const int32_t *__restrict__ color, int32_t *cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[color[i]], 1);
}
void launch_count_colors(int64_t n, const int32_t *color, int32_t *cnt, hipStream_t s) {
  if (n) k_count_colors<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, color, cnt);
}
__global__ void k_scatter_colors(int64_t n, const int32_t *__restrict__ color,
                                 const int64_t *__restrict__ off, int32_t *cursor,
                                 int32_t *__restrict__ rows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = color[i];
  int32_t k = atomicAdd(&cursor[c], 1);
  rows[off[c] + k] = (int32_t)i;
}
void launch_scatter_colors(int64_t n, const int32_t *color, const int64_t *off, int32_t *cursor,
                           int32_t *rows, hipStream_t s) {
  if (n) k_scatter_colors<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, color, off, cursor, rows);
}

// x_i <- -(sum_{j != i, ascending j} a_ij x_j) / a_ii for the rows of one colour
__global__ __launch_bounds__(kBlock) void k_gs_color(int64_t cnt, const int32_t *__restrict__ rows,
                                                     const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ diag,
                                                     double *__restrict__ x) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  int32_t i = rows[k];
  double s = 0.0;
  int64_t e = rp[i];
  const int64_t e1 = rp[i + 1];
  // four entries' loads in flight at a time; the sum still runs in entry order
  for (; e + 4 <= e1; e += 4) {
    const int32_t j0 = col[e], j1 = col[e + 1], j2 = col[e + 2], j3 = col[e + 3];
    const double a0 = val[e], a1 = val[e + 1], a2 = val[e + 2], a3 = val[e + 3];
    const double x0 = x[j0], x1 = x[j1], x2 = x[j2], x3 = x[j3];
    if (j0 != i) s = s + a0 * x0;
    if (j1 != i) s = s + a1 * x1;
    if (j2 != i) s = s + a2 * x2;
    if (j3 != i) s = s + a3 * x3;
  }
  for (; e < e1; ++e) {
    int32_t j = col[e];
    if (j != i) s = s + val[e] * x[j];
  }
  x[i] = (-s) / diag[i];
}
void launch_gs_color(int64_t cnt, const int32_t *rows, const CsrView<double> &A,
                     const double *diag, double *x, hipStream_t s) {
  if (cnt) k_gs_color<<<blocks_for(cnt, kBlock), kBlock, 0, s>>>(cnt, rows, A.rowptr, A.col, A.val, diag, x);
}

// one colour of a Gauss-Seidel sweep for A x = r (smoother):
// x_i <- (r_i - sum_{j != i} a_ij x_j) * dinv_i, G lanes per row
template <int G, class T>
__global__ __launch_bounds__(kBlock) void k_gs_rhs(int64_t cnt, const int32_t *__restrict__ rows,
                                                   const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const T *__restrict__ val,
                                                   const T *__restrict__ dinv,
                                                   const T *__restrict__ r, T *x,
                                                   const int *done) {
  if (done && *done) return;
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(cnt, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    const int64_t k = base + grp;
    const bool ok = k < hi;
    const int32_t i = ok ? rows[k] : 0;
    T s = 0;
    if (ok)
      for (int64_t e = rp[i] + sub; e < rp[i + 1]; e += G) {
        const int32_t j = col[e];
        if (j != i) s += val[e] * x[j];
      }
    s = group_sum<G, T>(s);
    if (ok && sub == 0) x[i] = (r[i] - s) * dinv[i];
  }
}
template <class T>
void launch_gs_rhs(int64_t cnt, const int32_t *rows, const CsrView<T> &A, const T *dinv,
                   const T *r, T *x, const int *done, hipStream_t s) {
  if (!cnt) return;
  const int grid = grid_for(cnt * A.lanes, kBlock);
#define L_(G) k_gs_rhs<G, T><<<grid, kBlock, 0, s>>>(cnt, rows, A.rowptr, A.col, A.val, dinv, r, x, done)
  MG_DISPATCH_G(A.lanes, L_);
#undef L_
}
template void launch_gs_rhs<double>(int64_t, const int32_t *, const CsrView<double> &,
                                    const double *, const double *, double *, const int *,
                                    hipStream_t);
template void launch_gs_rhs<float>(int64_t, const int32_t *, const CsrView<float> &,
                                   const float *, const float *, float *, const int *,
                                   hipStream_t);

__global__ void k_normalize(int64_t na, const int64_t *__restrict__ ap,
                            const int32_t *__restrict__ mem, const double *__restrict__ B,
                            double *__restrict__ p, float *__restrict__ p32,
                            double *__restrict__ Bn) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  int64_t b0 = ap[a], b1 = ap[a + 1];
  double s = 0.0;
  for (int64_t k = b0; k < b1; ++k) {
    double bi = B[mem[k]];
    s = s + bi * bi;
  }
  double sa = sqrt(s);
  if (sa == 0.0) {
    sa = sqrt((double)(b1 - b0));
    for (int64_t k = b0; k < b1; ++k) {
      double v = 1.0 / sa;
      p[mem[k]] = v;
      if (p32) p32[mem[k]] = (float)v;
    }
  } else {
    for (int64_t k = b0; k < b1; ++k) {
      double v = B[mem[k]] / sa;
      p[mem[k]] = v;
      if (p32) p32[mem[k]] = (float)v;
    }
  }
  Bn[a] = sa;
}
void launch_normalize(int64_t na, const int64_t *ap, const int32_t *mem, const double *B,
                      double *p, float *p32, double *Bn, hipStream_t s) {
  if (na) k_normalize<<<blocks_for(na, 64), 64, 0, s>>>(na, ap, mem, B, p, p32, Bn);
}

// ------------------------------------------------------------ Galerkin
// One wavefront per coarse row a. An open-addressing table holds the
// distinct coarse columns b = agg(j) met in the rows of a's members. The
// table lives in LDS (kHashCap slots) for every row that fits; a row with
// more distinct columns is redone with a table in global memory sized for
// its entries (the *_big kernels), so no row is ever refused.
constexpr int kHashCap = 1024;
constexpr int kHashShift = 22;   // 32 - log2(kHashCap)

// the table of one row: cap slots (a power of two), shift = 32 - log2(cap)
struct GalTab {
  int32_t *keys;    // coarse column per slot (-1 = empty)
  int32_t *rank;    // sorted position of the slot's column
  int32_t *list;    // distinct columns, then sorted
  int32_t *start;   // list offset of each rank (within the row)
  int32_t *cursor;  // per-rank counts, then placement cursors
  int cap, shift;
};

__device__ __forceinline__ int hash_slot(int32_t b, int shift, int cap) {
  return (int)(((uint32_t)b * 2654435761u) >> shift) & (cap - 1);
}
// insert b; returns 1 if it was new, 0 if present, -1 if the table is full
__device__ __forceinline__ int hash_insert(int32_t *keys, int shift, int cap, int32_t b) {
  int s = hash_slot(b, shift, cap);
  for (int probe = 0; probe < cap; ++probe) {
    int32_t old = atomicCAS(&keys[s], -1, b);
    if (old == -1) return 1;
    if (old == b) return 0;
    s = (s + 1) & (cap - 1);
  }
  return -1;
}
__device__ __forceinline__ int hash_find(const int32_t *keys, int shift, int cap, int32_t b) {
  int s = hash_slot(b, shift, cap);
  for (int probe = 0; probe < cap; ++probe) {
    int32_t k = keys[s];
    if (k == b) return s;
    if (k == -1) return -1;
    s = (s + 1) & (cap - 1);
  }
  return -1;
}

// distinct coarse columns (*nd) and connecting entries (*tot) of row a; full
// when the table could not hold them
__device__ void gal_count_row(int64_t a, const int64_t *__restrict__ ap,
                              const int32_t *__restrict__ mem, const int64_t *__restrict__ rp,
                              const int32_t *__restrict__ col, const int32_t *__restrict__ agg,
                              const GalTab &T, int64_t *nd, int64_t *tot, int *full) {
  const int lane = threadIdx.x;
  for (int s = lane; s < T.cap; s += kWave) T.keys[s] = -1;
  __syncthreads();
  int64_t mytot = 0, mynew = 0;
  int myfull = 0;
  for (int64_t t = ap[a]; t < ap[a + 1]; ++t) {
    int32_t i = mem[t];
    for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += kWave) {
      int32_t b = agg[col[e]];
      if (b < 0) continue;
      ++mytot;
      int r = hash_insert(T.keys, T.shift, T.cap, b);
      if (r == 1) ++mynew;
      else if (r < 0) myfull = 1;
    }
  }
  *tot = group_sum<kWave>(mytot);
  *nd = group_sum<kWave>(mynew);
  *full = group_sum<kWave>(myfull);
  __syncthreads();
}

// the sorted columns of row a, its Galerkin lists (fine entries per coarse
// entry, ascending fine order); the table must hold the row
__device__ void gal_fill_row(int64_t a, const int64_t *__restrict__ ap,
                             const int32_t *__restrict__ mem, const int64_t *__restrict__ rp,
                             const int32_t *__restrict__ col, const int32_t *__restrict__ agg,
                             const int64_t *__restrict__ crp, const int64_t *__restrict__ eoff,
                             int32_t *__restrict__ ccol, int32_t *__restrict__ crow,
                             int64_t *__restrict__ gl_ptr, int32_t *__restrict__ gl_idx,
                             int32_t *__restrict__ gl_row, const GalTab &T) {
  const int lane = threadIdx.x;
  for (int s = lane; s < T.cap; s += kWave) { T.keys[s] = -1; T.cursor[s] = 0; T.start[s] = 0; }
  __syncthreads();
  for (int64_t t = ap[a]; t < ap[a + 1]; ++t) {
    int32_t i = mem[t];
    for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += kWave) {
      int32_t b = agg[col[e]];
      if (b < 0) continue;
      (void)hash_insert(T.keys, T.shift, T.cap, b);
    }
  }
  __syncthreads();
  // compact the occupied slots into list (order irrelevant: sorted next)
  int n_d = 0;
  for (int s0 = 0; s0 < T.cap; s0 += kWave) {
    const int s = s0 + lane;
    const bool occ = s < T.cap && T.keys[s] >= 0;
    const uint64_t m = __ballot(occ);
    if (occ) T.list[n_d + __popcll(m & ((1ULL << lane) - 1ULL))] = T.keys[s];
    n_d += __popcll(m);
  }
  __syncthreads();
  int pw = 1;
  while (pw < n_d) pw <<= 1;
  for (int s = n_d + lane; s < pw; s += kWave) T.list[s] = 0x7fffffff;
  __syncthreads();
  // bitonic sort of list[0, pw)
  for (int k = 2; k <= pw; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int x = lane; x < pw; x += kWave) {
        int y = x ^ j;
        if (y > x) {
          int32_t u = T.list[x], v = T.list[y];
          bool up = (x & k) == 0;
          if ((u > v) == up) { T.list[x] = v; T.list[y] = u; }
        }
      }
      __syncthreads();
    }
  for (int r = lane; r < n_d; r += kWave) T.rank[hash_find(T.keys, T.shift, T.cap, T.list[r])] = r;
  __syncthreads();
  // entries per rank
  for (int64_t t = ap[a]; t < ap[a + 1]; ++t) {
    int32_t i = mem[t];
    for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += kWave) {
      int32_t b = agg[col[e]];
      if (b < 0) continue;
      atomicAdd(&T.cursor[T.rank[hash_find(T.keys, T.shift, T.cap, b)]], 1);
    }
  }
  __syncthreads();
  // exclusive scan of the counts into start[], reset cursor
  if (lane == 0) {
    int run = 0;
    for (int r = 0; r < n_d; ++r) { T.start[r] = run; run += T.cursor[r]; T.cursor[r] = 0; }
  }
  __syncthreads();
  const int64_t row0 = crp[a];
  const int64_t e0 = eoff[a];
  for (int r = lane; r < n_d; r += kWave) {
    ccol[row0 + r] = T.list[r];
    crow[row0 + r] = (int32_t)a;
    gl_ptr[row0 + r] = e0 + T.start[r];
  }
  // stable placement: entries in ascending fine order, 64 at a time
  for (int64_t t = ap[a]; t < ap[a + 1]; ++t) {
    int32_t i = mem[t];
    for (int64_t eb = rp[i]; eb < rp[i + 1]; eb += kWave) {
      int64_t e = eb + lane;
      int myr = -1;
      if (e < rp[i + 1]) {
        int32_t b = agg[col[e]];
        if (b >= 0) myr = T.rank[hash_find(T.keys, T.shift, T.cap, b)];
      }
      bool pending = myr >= 0;
      uint64_t pend = __ballot(pending);
      while (pend) {
        int leader = __ffsll((long long)pend) - 1;
        int R = __shfl(myr, leader, kWave);
        uint64_t mask = __ballot(pending && myr == R);
        if (pending && myr == R) {
          int before = __popcll(mask & ((1ULL << lane) - 1ULL));
          int64_t pos = e0 + T.start[R] + T.cursor[R] + before;
          gl_idx[pos] = (int32_t)e;
          gl_row[pos] = i;
          pending = false;
        }
        __syncthreads();
        if (lane == leader) T.cursor[R] += __popcll(mask);
        __syncthreads();
        pend &= ~mask;
      }
    }
  }
  __syncthreads();
}

// rowcnt[a] = distinct columns, elen[a] = connecting entries; a row that does
// not fit the LDS table gets rowcnt[a] = -1 and raises *overflow (the host
// then redoes it with k_gal_count_big)
__global__ __launch_bounds__(kWave) void k_gal_count(int64_t na, const int64_t *__restrict__ ap,
                                                     const int32_t *__restrict__ mem,
                                                     const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ agg,
                                                     int64_t *__restrict__ rowcnt,
                                                     int64_t *__restrict__ elen, int *overflow) {
  __shared__ int32_t keys[kHashCap];
  const GalTab T{keys, nullptr, nullptr, nullptr, nullptr, kHashCap, kHashShift};
  for (int64_t a = blockIdx.x; a < na; a += gridDim.x) {
    int64_t nd, tot;
    int full;
    gal_count_row(a, ap, mem, rp, col, agg, T, &nd, &tot, &full);
    if (threadIdx.x == 0) {
      rowcnt[a] = full ? -1 : nd;
      elen[a] = tot;
      if (full) atomicExch(overflow, 1);
    }
  }
}
void launch_gal_count(int64_t na, const int64_t *ap, const int32_t *mem, const CsrView<double> &A,
                      const int32_t *agg, int64_t *rowcnt, int64_t *elen, int *overflow,
                      hipStream_t s) {
  if (!na) return;
  unsigned grid = (unsigned)(na < 65536 ? na : 65536);
  k_gal_count<<<grid, kWave, 0, s>>>(na, ap, mem, A.rowptr, A.col, agg, rowcnt, elen, overflow);
}

// table of big row q: 5 cap int32 at 5 toff[q] of the scratch, cap = tcap[q]
__device__ __forceinline__ GalTab big_tab(int32_t *scratch, const int64_t *toff,
                                          const int32_t *tcap, int q) {
  const int cap = tcap[q];
  int32_t *base = scratch + 5 * toff[q];
  return GalTab{base, base + cap, base + 2 * cap, base + 3 * cap, base + 4 * cap, cap,
                32 - (31 - __clz(cap))};
}

__global__ __launch_bounds__(kWave) void k_gal_count_big(
    int nbig, const int32_t *__restrict__ rows, const int64_t *__restrict__ toff,
    const int32_t *__restrict__ tcap, int32_t *scratch, const int64_t *__restrict__ ap,
    const int32_t *__restrict__ mem, const int64_t *__restrict__ rp,
    const int32_t *__restrict__ col, const int32_t *__restrict__ agg,
    int64_t *__restrict__ rowcnt, int *overflow) {
  for (int q = blockIdx.x; q < nbig; q += gridDim.x) {
    const GalTab T = big_tab(scratch, toff, tcap, q);
    int64_t nd, tot;
    int full;
    gal_count_row(rows[q], ap, mem, rp, col, agg, T, &nd, &tot, &full);
    if (threadIdx.x == 0) {
      rowcnt[rows[q]] = nd;
      if (full) atomicExch(overflow, 1);   // cannot happen: cap >= 2 entries
    }
  }
}
void launch_gal_count_big(int nbig, const int32_t *rows, const int64_t *toff, const int32_t *tcap,
                          int32_t *scratch, const int64_t *ap, const int32_t *mem,
                          const CsrView<double> &A, const int32_t *agg, int64_t *rowcnt,
                          int *overflow, hipStream_t s) {
  if (!nbig) return;
  unsigned grid = (unsigned)(nbig < 65536 ? nbig : 65536);
  k_gal_count_big<<<grid, kWave, 0, s>>>(nbig, rows, toff, tcap, scratch, ap, mem, A.rowptr,
                                         A.col, agg, rowcnt, overflow);
}

// rows with more than kHashCap distinct columns are left to k_gal_fill_big
__global__ __launch_bounds__(kWave) void k_gal_fill(
    int64_t na, const int64_t *__restrict__ ap, const int32_t *__restrict__ mem,
    const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
    const int32_t *__restrict__ agg, const int64_t *__restrict__ crp,
    const int64_t *__restrict__ eoff, int32_t *__restrict__ ccol, int32_t *__restrict__ crow,
    int64_t *__restrict__ gl_ptr, int32_t *__restrict__ gl_idx, int32_t *__restrict__ gl_row) {
  __shared__ int32_t keys[kHashCap], rank[kHashCap], list[kHashCap], start[kHashCap],
      cursor[kHashCap];
  const GalTab T{keys, rank, list, start, cursor, kHashCap, kHashShift};
  for (int64_t a = blockIdx.x; a < na; a += gridDim.x) {
    if (crp[a + 1] - crp[a] > kHashCap) continue;
    gal_fill_row(a, ap, mem, rp, col, agg, crp, eoff, ccol, crow, gl_ptr, gl_idx, gl_row, T);
  }
}
void launch_gal_fill(int64_t na, const int64_t *ap, const int32_t *mem, const CsrView<double> &A,
                     const int32_t *agg, const int64_t *crp, const int64_t *eoff, int32_t *ccol,
                     int32_t *crow, int64_t *gl_ptr, int32_t *gl_idx, int32_t *gl_row,
                     hipStream_t s) {
  if (!na) return;
  unsigned grid = (unsigned)(na < 65536 ? na : 65536);
  k_gal_fill<<<grid, kWave, 0, s>>>(na, ap, mem, A.rowptr, A.col, agg, crp, eoff, ccol, crow,
                                    gl_ptr, gl_idx, gl_row);
}

__global__ __launch_bounds__(kWave) void k_gal_fill_big(
    int nbig, const int32_t *__restrict__ rows, const int64_t *__restrict__ toff,
    const int32_t *__restrict__ tcap, int32_t *scratch, const int64_t *__restrict__ ap,
    const int32_t *__restrict__ mem, const int64_t *__restrict__ rp,
    const int32_t *__restrict__ col, const int32_t *__restrict__ agg,
    const int64_t *__restrict__ crp, const int64_t *__restrict__ eoff, int32_t *__restrict__ ccol,
    int32_t *__restrict__ crow, int64_t *__restrict__ gl_ptr, int32_t *__restrict__ gl_idx,
    int32_t *__restrict__ gl_row) {
  for (int q = blockIdx.x; q < nbig; q += gridDim.x) {
    const GalTab T = big_tab(scratch, toff, tcap, q);
    gal_fill_row(rows[q], ap, mem, rp, col, agg, crp, eoff, ccol, crow, gl_ptr, gl_idx, gl_row,
                 T);
  }
}
void launch_gal_fill_big(int nbig, const int32_t *rows, const int64_t *toff, const int32_t *tcap,
                         int32_t *scratch, const int64_t *ap, const int32_t *mem,
                         const CsrView<double> &A, const int32_t *agg, const int64_t *crp,
                         const int64_t *eoff, int32_t *ccol, int32_t *crow, int64_t *gl_ptr,
                         int32_t *gl_idx, int32_t *gl_row, hipStream_t s) {
  if (!nbig) return;
  unsigned grid = (unsigned)(nbig < 65536 ? nbig : 65536);
  k_gal_fill_big<<<grid, kWave, 0, s>>>(nbig, rows, toff, tcap, scratch, ap, mem, A.rowptr, A.col,
                                        agg, crp, eoff, ccol, crow, gl_ptr, gl_idx, gl_row);
}

__global__ void k_gal_mirror(int64_t nnzc, const int32_t *__restrict__ crow,
                             const int32_t *__restrict__ ccol, const int64_t *__restrict__ crp,
                             int32_t *__restrict__ mirror, int *bad) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnzc) return;
  int32_t a = crow[k], b = ccol[k];
  int64_t lo = crp[b], hi = crp[b + 1] - 1, found = -1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    int32_t c = ccol[mid];
    if (c == a) { found = mid; break; }
    if (c < a) lo = mid + 1; else hi = mid - 1;
  }
  mirror[k] = (int32_t)found;
  if (found < 0) atomicExch(bad, 1);
}
void launch_gal_mirror(int64_t nnzc, const int32_t *crow, const int32_t *ccol, const int64_t *crp,
                       int32_t *mirror, int *bad, hipStream_t s) {
  if (nnzc) k_gal_mirror<<<blocks_for(nnzc, kBlock), kBlock, 0, s>>>(nnzc, crow, ccol, crp, mirror, bad);
}

// entry (a, b), a <= b: sum in ascending fine order of (p_i a_ij) p_j; the
// mirror entry (b, a) receives the same value
__global__ __launch_bounds__(kBlock) void k_gal_numeric(
    int64_t nnzc, const int32_t *__restrict__ crow, const int32_t *__restrict__ ccol,
    const int32_t *__restrict__ mirror, const int64_t *__restrict__ gl_ptr,
    const int32_t *__restrict__ gl_idx, const int32_t *__restrict__ gl_row,
    const int32_t *__restrict__ fcol, const double *__restrict__ fval,
    const double *__restrict__ p, double *__restrict__ cval, float *__restrict__ cval32) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnzc) return;
  if (ccol[k] < crow[k]) return;
  double acc = 0.0;
  for (int64_t t = gl_ptr[k]; t < gl_ptr[k + 1]; ++t) {
    int32_t e = gl_idx[t];
    int32_t i = gl_row[t];
    acc = acc + (p[i] * fval[e]) * p[fcol[e]];
  }
  cval[k] = acc;
  int32_t m = mirror[k];
  cval[m] = acc;
  if (cval32) {
    cval32[k] = (float)acc;
    cval32[m] = (float)acc;
  }
}
void launch_gal_numeric(int64_t nnzc, const int32_t *crow, const int32_t *ccol,
                        const int32_t *mirror, const int64_t *gl_ptr, const int32_t *gl_idx,
                        const int32_t *gl_row, const int32_t *fcol, const double *fval,
                        const double *p, double *cval, float *cval32, hipStream_t s) {
  if (nnzc)
    k_gal_numeric<<<blocks_for(nnzc, kBlock), kBlock, 0, s>>>(nnzc, crow, ccol, mirror, gl_ptr, gl_idx,
                                                              gl_row, fcol, fval, p, cval, cval32);
}

}  // namespace mgpbd
