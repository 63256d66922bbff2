// Per-body (segmented) kernels: PCG vector updates with one control block per
// body, per-body reductions, per-body power method, keys from body-local
// indices, and batched dense coarsest solves. Every block of a segmented
// kernel works on rows of exactly one body (see SegTable), so a body's sums
// are the fixed-order sum of its own block partials.
#include <algorithm>

#include "seg.hpp"

namespace mgpbd {

void SegTable::build(const std::vector<int64_t> &offsets, hipStream_t s) {
  off = offsets;
  const int nseg = (int)off.size() - 1;
  const int64_t total = off.back() - off.front();
  int64_t rpb = std::max<int64_t>(kBlock, (total + kMaxGrid - 1) / kMaxGrid);
  bseg.clear(); blo.clear(); bhi.clear(); first.clear();
  for (int sidx = 0; sidx < nseg; ++sidx) {
    first.push_back((int32_t)bseg.size());
    int64_t a = off[sidx], b = off[sidx + 1];
    if (a == b) continue;
    for (int64_t q = a; q < b; q += rpb) {
      bseg.push_back(sidx);
      blo.push_back(q);
      bhi.push_back(std::min(b, q + rpb));
    }
  }
  first.push_back((int32_t)bseg.size());
  if (bseg.empty()) {   // keep the table non-empty (one idle block)
    bseg.push_back(0); blo.push_back(0); bhi.push_back(0);
    first.back() = 1;
  }
  d_bseg.upload(bseg.data(), bseg.size(), s);
  d_blo.upload(blo.data(), blo.size(), s);
  d_bhi.upload(bhi.data(), bhi.size(), s);
  d_first.upload(first.data(), first.size(), s);
  d_off.upload(off.data(), off.size(), s);
}

#define SEG_BLOCK(t)                       \
  const int bb_ = xcd_block();             \
  const int seg = (t).bseg[bb_];           \
  const int64_t lo = (t).blo[bb_];         \
  const int64_t hi = (t).bhi[bb_];         \
  (void)seg;

// block partials in block-table order: partials[k * nblk + table index]
template <int NV>
__device__ void seg_partials(const double (&v)[NV], double *partials) {
  static_assert(NV <= kMaxBlockSums, "the partials buffer holds kMaxBlockSums sums per block");
  __shared__ double sh[NV][kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = group_sum<kWave>(v[k]);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int bb = xcd_block();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = sh[k][0];
      for (int q = 1; q < nw; ++q) s += sh[k][q];
      partials[(size_t)k * gridDim.x + bb] = s;
    }
  }
}

// finisher side: block `seg` adds its segment's partials in a fixed order
template <int NV>
__device__ void seg_total(const SegTab &t, const double *partials, int seg, double (&out)[NV]) {
  __shared__ double sh[NV][kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int b0 = t.first[seg], b1 = t.first[seg + 1];
  const int bd = blockDim.x;
  // eight independent loads per value and round, summed in a fixed order
  double acc[NV][8];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[k][u] = 0.0;
  int q = b0 + threadIdx.x;
  for (; q + 7 * bd < b1; q += 8 * bd) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[k][u] += partials[(size_t)k * t.nblk + q + u * bd];
  }
  for (; q < b1; q += bd) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k][0] += partials[(size_t)k * t.nblk + q];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = ((acc[k][0] + acc[k][1]) + (acc[k][2] + acc[k][3])) +
               ((acc[k][4] + acc[k][5]) + (acc[k][6] + acc[k][7]));
    s = group_sum<kWave>(s);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double tot = sh[k][0];
    for (int q = 1; q < nw; ++q) tot += sh[k][q];
    out[k] = tot;
  }
}

__global__ void k_all_done(const PcgCtl *ctl, int nseg, int *all_done) {
  __shared__ int any_running;
  if (threadIdx.x == 0) any_running = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nseg; k += blockDim.x)
    if (ctl[k].done == 0) any_running = 1;
  __syncthreads();
  if (threadIdx.x == 0) *all_done = any_running ? 0 : 1;
}
// with one body the V-cycle kernels read that body's done flag directly
static void all_done_update(const SegTab &t, const PcgCtl *ctl, int *all_done, hipStream_t s) {
  if (t.nseg > 1) k_all_done<<<1, kBlock, 0, s>>>(ctl, t.nseg, all_done);
}

// ------------------------------------------------------------------ PCG
__global__ __launch_bounds__(kBlock) void k_s_pcg_init(SegTab t, const double *__restrict__ b,
                                                       double *__restrict__ x,
                                                       double *__restrict__ r, double *partials) {
  SEG_BLOCK(t);
  double v[1] = {0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    double bi = b[i];
    x[i] = 0.0;
    r[i] = bi;
    v[0] += bi * bi;
  }
  seg_partials<1>(v, partials);
}
__global__ __launch_bounds__(kBlock) void k_s_fin_init(SegTab t, PcgCtl *ctl,
                                                       const double *partials) {
  const int seg = blockIdx.x;
  double tot[1];
  seg_total<1>(t, partials, seg, tot);
  if (threadIdx.x == 0) {
    PcgCtl &c = ctl[seg];
    c.bnorm = sqrt(tot[0]);
    c.iters = 0;
    c.ratio = 0.0;
    c.rr = tot[0];
    c.done = (c.bnorm == 0.0) ? 1 : 0;
    if (!(tot[0] == tot[0]) || tot[0] > 1.7976931348623157e308) c.done = 2;
  }
}
void launch_s_pcg_init(const SegTab &t, PcgCtl *ctl, const double *b, double *x, double *r,
                       double *partials, int *all_done, hipStream_t s) {
  k_s_pcg_init<<<t.nblk, kBlock, 0, s>>>(t, b, x, r, partials);
  k_s_fin_init<<<t.nseg, kBlock, 0, s>>>(t, ctl, partials);
  all_done_update(t, ctl, all_done, s);
}

__global__ __launch_bounds__(kBlock) void k_s_pcg_init_p(SegTab t, const PcgCtl *ctl,
                                                         const double *__restrict__ r,
                                                         const double *__restrict__ z,
                                                         const float *__restrict__ z32,
                                                         double *__restrict__ p,
                                                         float *__restrict__ zold32,
                                                         double *partials) {
  SEG_BLOCK(t);
  double v[1] = {0.0};
  if (!ctl[seg].done) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      double zi;
      if (z32) {
        const float zf = z32[i];
        zi = (double)zf;
        zold32[i] = zf;
      } else {
        zi = z[i];
      }
      p[i] = zi;
      v[0] += r[i] * zi;
    }
  }
  seg_partials<1>(v, partials);
}
__global__ __launch_bounds__(kBlock) void k_s_fin_init_p(SegTab t, PcgCtl *ctl,
                                                         const double *partials) {
  const int seg = blockIdx.x;
  if (ctl[seg].done) return;
  double tot[1];
  seg_total<1>(t, partials, seg, tot);
  if (threadIdx.x == 0) {
    ctl[seg].rho = tot[0];
    if (!(tot[0] > 0.0)) ctl[seg].done = 2;
  }
}
void launch_s_pcg_init_p(const SegTab &t, PcgCtl *ctl, const double *r, const double *z,
                         const float *z32, double *p, float *zold32, double *partials,
                         int *all_done, hipStream_t s) {
  k_s_pcg_init_p<<<t.nblk, kBlock, 0, s>>>(t, ctl, r, z, z32, p, zold32, partials);
  k_s_fin_init_p<<<t.nseg, kBlock, 0, s>>>(t, ctl, partials);
  all_done_update(t, ctl, all_done, s);
}

__global__ __launch_bounds__(kBlock) void k_s_dot_pq(SegTab t, const PcgCtl *ctl,
                                                     const double *__restrict__ p,
                                                     const double *__restrict__ q,
                                                     double *partials) {
  SEG_BLOCK(t);
  double v[1] = {0.0};
  if (!ctl[seg].done)
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) v[0] += p[i] * q[i];
  seg_partials<1>(v, partials);
}
__global__ __launch_bounds__(kBlock) void k_s_fin_pq(SegTab t, PcgCtl *ctl,
                                                     const double *partials) {
  const int seg = blockIdx.x;
  if (ctl[seg].done) return;
  double tot[1];
  seg_total<1>(t, partials, seg, tot);
  if (threadIdx.x == 0) {
    PcgCtl &c = ctl[seg];
    c.pq = tot[0];
    if (!(tot[0] > 0.0) || !(c.rho > 0.0)) c.done = 2;
    else c.alpha = c.rho / tot[0];
  }
}
void launch_s_pcg_dot_pq(const SegTab &t, PcgCtl *ctl, const double *p, const double *q,
                         double *partials, hipStream_t s) {
  k_s_dot_pq<<<t.nblk, kBlock, 0, s>>>(t, ctl, p, q, partials);
  k_s_fin_pq<<<t.nseg, kBlock, 0, s>>>(t, ctl, partials);
}

// x += alpha p, r -= alpha q and the partial sums of |r|^2; with `first` the
// new r also feeds the V-cycle's first fine-level step: its FP32 copy and the
// first Jacobi iterate omega D^-1 r (k_d2f and k_jacobi_first's values). The
// V-cycle runs over every row while any body is still iterating, so a
// finished body's rows get the same values from its unchanged r.
__global__ __launch_bounds__(kBlock) void k_s_pcg_update(SegTab t, const PcgCtl *ctl,
                                                         const double *__restrict__ p,
                                                         const double *__restrict__ q,
                                                         double *__restrict__ x,
                                                         double *__restrict__ r,
                                                         double *partials, FirstSweep first) {
  SEG_BLOCK(t);
  double v[1] = {0.0};
  const bool live = !ctl[seg].done;
  const bool feed = (first.z64 || first.r32) && !*first.cycle_done;
  if (live || feed) {
    const double alpha = ctl[seg].alpha;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      double ri;
      if (live) {
        x[i] = x[i] + alpha * p[i];
        ri = r[i] - alpha * q[i];
        r[i] = ri;
        v[0] += ri * ri;
      } else {
        ri = r[i];
      }
      if (first.z64) first.z64[i] = ri * first.wd64[i];
      if (first.r32) {
        const float rf = (float)ri;
        first.r32[i] = rf;
        if (first.z32) first.z32[i] = rf * first.wd32[i];
      }
    }
  }
  seg_partials<1>(v, partials);
}
__global__ __launch_bounds__(kBlock) void k_s_fin_update(SegTab t, PcgCtl *ctl,
                                                         const double *partials) {
  const int seg = blockIdx.x;
  if (ctl[seg].done) return;
  double tot[1];
  seg_total<1>(t, partials, seg, tot);
  if (threadIdx.x == 0) {
    PcgCtl &c = ctl[seg];
    int it = c.iters + 1;
    c.iters = it;
    c.rr = tot[0];
    double ratio = sqrt(tot[0]) / c.bnorm;
    c.ratio = ratio;
    if (!(ratio == ratio)) c.done = 2;
    else if (c.force > 0) { if (it >= c.force) c.done = 3; }
    else if (ratio <= c.tol) c.done = 1;
    else if (it >= c.max_iters) c.done = 4;
  }
}
void launch_s_pcg_update(const SegTab &t, PcgCtl *ctl, const double *p, const double *q,
                         double *x, double *r, double *partials, int *all_done, hipStream_t s,
                         const FirstSweep &first) {
  k_s_pcg_update<<<t.nblk, kBlock, 0, s>>>(t, ctl, p, q, x, r, partials, first);
  k_s_fin_update<<<t.nseg, kBlock, 0, s>>>(t, ctl, partials);
  all_done_update(t, ctl, all_done, s);
}

// r^T z and, with the FP32 V-cycle, the flexible numerator r^T (z - zold)
// (zold = the previous z, kept as the FP32 values it equals)
__global__ __launch_bounds__(kBlock) void k_s_pcg_rz(SegTab t, const PcgCtl *ctl,
                                                     const double *__restrict__ r,
                                                     const double *__restrict__ z,
                                                     const float *__restrict__ z32,
                                                     float *__restrict__ zold32,
                                                     double *partials) {
  SEG_BLOCK(t);
  double v[2] = {0.0, 0.0};
  if (!ctl[seg].done) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const double ri = r[i];
      if (z32) {
        const float zf = z32[i];
        const double zi = (double)zf;
        v[0] += ri * zi;
        v[1] += ri * (zi - (double)zold32[i]);
        zold32[i] = zf;
      } else {
        v[0] += ri * z[i];
      }
    }
  }
  seg_partials<2>(v, partials);
}
__global__ __launch_bounds__(kBlock) void k_s_fin_rz(SegTab t, PcgCtl *ctl,
                                                     const double *partials, int flexible) {
  const int seg = blockIdx.x;
  if (ctl[seg].done) return;
  double tot[2];
  seg_total<2>(t, partials, seg, tot);
  if (threadIdx.x == 0) {
    PcgCtl &c = ctl[seg];
    double rho_new = tot[0];
    double num = flexible ? tot[1] : rho_new;
    c.beta = num / c.rho;
    c.rho = rho_new;
    if (!(rho_new > 0.0)) c.done = 2;
  }
}
void launch_s_pcg_rz(const SegTab &t, PcgCtl *ctl, const double *r, const double *z,
                     const float *z32, float *zold32, double *partials, hipStream_t s) {
  k_s_pcg_rz<<<t.nblk, kBlock, 0, s>>>(t, ctl, r, z, z32, zold32, partials);
  k_s_fin_rz<<<t.nseg, kBlock, 0, s>>>(t, ctl, partials, z32 ? 1 : 0);
}

__global__ __launch_bounds__(kBlock) void k_s_pcg_pupdate(SegTab t, const PcgCtl *ctl,
                                                          const double *__restrict__ z,
                                                          const float *__restrict__ z32,
                                                          double *__restrict__ p) {
  SEG_BLOCK(t);
  if (ctl[seg].done) return;
  const double beta = ctl[seg].beta;
  if (z32) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
      p[i] = (double)z32[i] + beta * p[i];
  } else {
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) p[i] = z[i] + beta * p[i];
  }
}
void launch_s_pcg_pupdate(const SegTab &t, const PcgCtl *ctl, const double *z, const float *z32,
                          double *p, hipStream_t s) {
  k_s_pcg_pupdate<<<t.nblk, kBlock, 0, s>>>(t, ctl, z, z32, p);
}

// ------------------------------------------------------------ reductions
__global__ __launch_bounds__(kBlock) void k_s_dot(SegTab t, const double *__restrict__ a,
                                                  const double *__restrict__ b,
                                                  double *partials) {
  SEG_BLOCK(t);
  double v[1] = {0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) v[0] += a[i] * b[i];
  seg_partials<1>(v, partials);
}
__global__ __launch_bounds__(kBlock) void k_s_fin_store1(SegTab t, const double *partials,
                                                         double *out) {
  double tot[1];
  seg_total<1>(t, partials, blockIdx.x, tot);
  if (threadIdx.x == 0) out[blockIdx.x] = tot[0];
}
__global__ __launch_bounds__(kBlock) void k_s_fin_store2(SegTab t, const double *partials,
                                                         double *out) {
  double tot[2];
  seg_total<2>(t, partials, blockIdx.x, tot);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = tot[0];
    out[2 * blockIdx.x + 1] = tot[1];
  }
}
void launch_s_dot(const SegTab &t, const double *a, const double *b, double *out,
                  double *partials, hipStream_t s) {
  k_s_dot<<<t.nblk, kBlock, 0, s>>>(t, a, b, partials);
  k_s_fin_store1<<<t.nseg, kBlock, 0, s>>>(t, partials, out);
}

__global__ __launch_bounds__(kBlock) void k_s_pow_scale(SegTab t, double *__restrict__ w,
                                                        const double *__restrict__ diag,
                                                        double *partials) {
  SEG_BLOCK(t);
  double v[1] = {0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    double wi = w[i] / diag[i];
    w[i] = wi;
    v[0] += wi * wi;
  }
  seg_partials<1>(v, partials);
}
void launch_s_pow_scale(const SegTab &t, double *w, const double *diag, double *out,
                        double *partials, hipStream_t s) {
  k_s_pow_scale<<<t.nblk, kBlock, 0, s>>>(t, w, diag, partials);
  k_s_fin_store1<<<t.nseg, kBlock, 0, s>>>(t, partials, out);
}
__global__ __launch_bounds__(kBlock) void k_s_pow_normalize(SegTab t, const double *__restrict__ w,
                                                            const double *__restrict__ nrm2,
                                                            double *__restrict__ v) {
  SEG_BLOCK(t);
  double nr = sqrt(nrm2[seg]);
  if (!(nr > 0.0)) return;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) v[i] = w[i] / nr;
}
void launch_s_pow_normalize(const SegTab &t, const double *w, const double *nrm2, double *v,
                            hipStream_t s) {
  k_s_pow_normalize<<<t.nblk, kBlock, 0, s>>>(t, w, nrm2, v);
}
__global__ __launch_bounds__(kBlock) void k_s_rayleigh(SegTab t, const double *__restrict__ v,
                                                       const double *__restrict__ Av,
                                                       const double *__restrict__ diag,
                                                       double *partials) {
  SEG_BLOCK(t);
  double s3[3] = {0.0, 0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double vi = v[i], ai = Av[i], di = diag[i];
    s3[0] += vi * ai;
    s3[1] += vi * di * vi;
    s3[2] += ai * (ai / di);
  }
  seg_partials<3>(s3, partials);
}
__global__ __launch_bounds__(kBlock) void k_s_fin_store3(SegTab t, const double *partials,
                                                         double *out) {
  double tot[3];
  seg_total<3>(t, partials, blockIdx.x, tot);
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x] = tot[0];
    out[3 * blockIdx.x + 1] = tot[1];
    out[3 * blockIdx.x + 2] = tot[2];
  }
}
void launch_s_rayleigh(const SegTab &t, const double *v, const double *Av, const double *diag,
                       double *out, double *partials, hipStream_t s) {
  k_s_rayleigh<<<t.nblk, kBlock, 0, s>>>(t, v, Av, diag, partials);
  k_s_fin_store3<<<t.nseg, kBlock, 0, s>>>(t, partials, out);
}
__global__ void k_s_pow_init(SegTab t, uint64_t salt, int level, double *__restrict__ v) {
  SEG_BLOCK(t);
  const int64_t base = t.segoff[seg];
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
    v[i] = uniform_open(mix64_salted(salt, ((uint64_t)level << 40) + (uint64_t)(i - base)));
}
void launch_s_pow_init(const SegTab &t, uint64_t salt, int level, double *v, hipStream_t s) {
  k_s_pow_init<<<t.nblk, kBlock, 0, s>>>(t, salt, level, v);
}
__global__ void k_s_rowseg(SegTab t, int32_t *__restrict__ rowseg) {
  SEG_BLOCK(t);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) rowseg[i] = seg;
}
void launch_s_rowseg(const SegTab &t, int32_t *rowseg, hipStream_t s) {
  k_s_rowseg<<<t.nblk, kBlock, 0, s>>>(t, rowseg);
}
__global__ void k_s_wdinv(SegTab t, const double *__restrict__ omega,
                          const double *__restrict__ dinv, double *__restrict__ wdinv,
                          float *__restrict__ wdinv32) {
  SEG_BLOCK(t);
  const double om = omega[seg];
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    double v = om * dinv[i];
    wdinv[i] = v;
    if (wdinv32) wdinv32[i] = (float)v;
  }
}
void launch_s_wdinv(const SegTab &t, const double *omega, const double *dinv, double *wdinv,
                    float *wdinv32, hipStream_t s) {
  k_s_wdinv<<<t.nblk, kBlock, 0, s>>>(t, omega, dinv, wdinv, wdinv32);
}

__global__ __launch_bounds__(kBlock) void k_s_absmax(SegTab t, const int64_t *__restrict__ rp,
                                                     const double *__restrict__ val,
                                                     unsigned long long *amax) {
  SEG_BLOCK(t);
  unsigned long long m = 0;
  for (int64_t e = rp[lo] + threadIdx.x; e < rp[hi]; e += blockDim.x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(fabs(val[e]));
    m = b > m ? b : m;
  }
  m = group_max_u64<kWave>(m);
  if ((threadIdx.x & 63) == 0) atomicMax(&amax[seg], m);
}
void launch_s_absmax(const SegTab &t, const int64_t *rp, const double *val,
                     unsigned long long *amax, hipStream_t s) {
  k_s_absmax<<<t.nblk, kBlock, 0, s>>>(t, rp, val, amax);
}
// random start of a near-kernel candidate: index idx_off + body-local row
__global__ void k_s_candidate_init(SegTab t, uint64_t salt, const unsigned long long *amax,
                                   uint64_t idx_off, double *__restrict__ B) {
  SEG_BLOCK(t);
  const int64_t base = t.segoff[seg];
  const double am = __longlong_as_double((long long)amax[seg]);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
    B[i] = uniform_open(mix64_salted(salt, idx_off + (uint64_t)(i - base))) * am;
}
void launch_s_candidate_init(const SegTab &t, uint64_t salt, const unsigned long long *amax,
                             uint64_t idx_off, double *B, hipStream_t s) {
  k_s_candidate_init<<<t.nblk, kBlock, 0, s>>>(t, salt, amax, idx_off, B);
}
__global__ void k_s_mis_init(SegTab t, const uint8_t *__restrict__ conn, uint64_t salt, int level,
                             uint64_t *__restrict__ key) {
  SEG_BLOCK(t);
  const int64_t base = t.segoff[seg];
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
    key[i] = conn[i] ? prio_key(salt, level, i - base) + 1ULL : 0ULL;
}
void launch_s_mis_init(const SegTab &t, const uint8_t *conn, uint64_t salt, int level,
                       uint64_t *key, hipStream_t s) {
  k_s_mis_init<<<t.nblk, kBlock, 0, s>>>(t, conn, salt, level, key);
}
__global__ void k_s_color_keys(SegTab t, uint64_t salt, int level, uint64_t *__restrict__ key) {
  SEG_BLOCK(t);
  const int64_t base = t.segoff[seg];
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
    key[i] = prio_key(salt, level, i - base);
}
void launch_s_color_keys(const SegTab &t, uint64_t salt, int level, uint64_t *key,
                         hipStream_t s) {
  k_s_color_keys<<<t.nblk, kBlock, 0, s>>>(t, salt, level, key);
}

// one wavefront per row over all jobs; rowstart[j] = first global wave row of
// job j (prefix of the jobs' row counts)
template <class T>
__global__ __launch_bounds__(kBlock) void k_dense_apply_batch(int njobs, const DenseJob *jobs,
                                                              int64_t total,
                                                              const int64_t *__restrict__ rowstart,
                                                              const double *__restrict__ ainv,
                                                              const T *__restrict__ r,
                                                              T *__restrict__ z, const int *done) {
  if (done && *done) return;
  const int lane = threadIdx.x % kWave;
  const int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (w >= total) return;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {   // last job with rowstart <= w
    int mid = (lo + hi + 1) / 2;
    if (rowstart[mid] <= w) lo = mid; else hi = mid - 1;
  }
  const DenseJob j = jobs[lo];
  const int64_t i = w - rowstart[lo];
  const double *Ai = ainv + j.ainv + i * j.n;
  double s = 0.0;
  for (int64_t k = lane; k < j.n; k += kWave) s += Ai[k] * (double)r[j.row0 + k];
  s = group_sum<kWave>(s);
  if (lane == 0) z[j.row0 + i] = (T)s;
}
template <class T>
void launch_dense_apply_batch(int njobs, const DenseJob *jobs, int64_t total_rows,
                              const int64_t *rowstart, const double *ainv, const T *r, T *z,
                              const int *done, hipStream_t s) {
  if (njobs <= 0 || total_rows <= 0) return;
  k_dense_apply_batch<T><<<blocks_for(total_rows, kBlock / kWave), kBlock, 0, s>>>(
      njobs, jobs, total_rows, rowstart, ainv, r, z, done);
}
template void launch_dense_apply_batch<double>(int, const DenseJob *, int64_t, const int64_t *,
                                               const double *, const double *, double *,
                                               const int *, hipStream_t);
template void launch_dense_apply_batch<float>(int, const DenseJob *, int64_t, const int64_t *,
                                              const double *, const float *, float *,
                                              const int *, hipStream_t);

}  // namespace mgpbd
