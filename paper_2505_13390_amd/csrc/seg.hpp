// Segmented (per-body) row operations. A level holds the rows of several
// bodies back to back; a block table assigns each block a row range inside
// one body, so per-body reductions are sums of that body's block partials.
#pragma once

#include "kernels.hpp"

namespace mgpbd {

// Device view of a block table.
struct SegTab {
  int nblk = 0;
  int nseg = 0;
  const int32_t *bseg = nullptr;    // [nblk] segment of each block
  const int64_t *blo = nullptr;     // [nblk] first row
  const int64_t *bhi = nullptr;     // [nblk] one past the last row
  const int32_t *first = nullptr;   // [nseg + 1] first block of each segment
  const int64_t *segoff = nullptr;  // [nseg + 1] first row of each segment
};

// Host-built block table for segment row offsets `off` (size nseg + 1).
struct SegTable {
  std::vector<int32_t> bseg, first;
  std::vector<int64_t> blo, bhi, off;
  DevBuf<int32_t> d_bseg, d_first;
  DevBuf<int64_t> d_blo, d_bhi, d_off;
  void build(const std::vector<int64_t> &offsets, hipStream_t s);
  SegTab view() const {
    SegTab t;
    t.nblk = (int)bseg.size();
    t.nseg = (int)off.size() - 1;
    t.bseg = d_bseg.p; t.blo = d_blo.p; t.bhi = d_bhi.p; t.first = d_first.p; t.segoff = d_off.p;
    return t;
  }
};

// ---- per-body PCG (ctl is an array of nseg control blocks; all_done is set
// when every body's solve has ended) ----
void launch_s_pcg_init(const SegTab &t, PcgCtl *ctl, const double *b, double *x, double *r,
                       double *partials, int *all_done, hipStream_t s);
// The preconditioned residual z comes either as FP64 (z, FP64 V-cycle:
// Fletcher-Reeves beta) or as the FP32 V-cycle's output z32 (z = (double) z32
// exactly: flexible beta, with zold32 = the previous z32; z is then not used)
void launch_s_pcg_init_p(const SegTab &t, PcgCtl *ctl, const double *r, const double *z,
                         const float *z32, double *p, float *zold32, double *partials,
                         int *all_done, hipStream_t s);
void launch_s_pcg_dot_pq(const SegTab &t, PcgCtl *ctl, const double *p, const double *q,
                         double *partials, hipStream_t s);
// What the V-cycle's first fine-level step needs from the new residual,
// written by the PCG update (all null: nothing): z64 = r wd64 (FP64 cycle), or
// r32 = (float) r and z32 = r32 wd32 (FP32 cycle); cycle_done is the flag that
// skips the V-cycle (required when anything is written)
struct FirstSweep {
  const int *cycle_done = nullptr;
  const double *wd64 = nullptr;
  double *z64 = nullptr;
  const float *wd32 = nullptr;
  float *r32 = nullptr, *z32 = nullptr;
};
void launch_s_pcg_update(const SegTab &t, PcgCtl *ctl, const double *p, const double *q,
                         double *x, double *r, double *partials, int *all_done, hipStream_t s,
                         const FirstSweep &first = FirstSweep());
void launch_s_pcg_rz(const SegTab &t, PcgCtl *ctl, const double *r, const double *z,
                     const float *z32, float *zold32, double *partials, hipStream_t s);
void launch_s_pcg_pupdate(const SegTab &t, const PcgCtl *ctl, const double *z, const float *z32,
                          double *p, hipStream_t s);

// ---- per-body reductions into out[seg] ----
void launch_s_dot(const SegTab &t, const double *a, const double *b, double *out,
                  double *partials, hipStream_t s);
void launch_s_pow_scale(const SegTab &t, double *w, const double *diag, double *out,
                        double *partials, hipStream_t s);
void launch_s_pow_normalize(const SegTab &t, const double *w, const double *nrm2, double *v,
                            hipStream_t s);
// out[3 seg] = v^T Av, out[3 seg + 1] = sum (v_i diag_i) v_i,
// out[3 seg + 2] = sum Av_i (Av_i / diag_i)
void launch_s_rayleigh(const SegTab &t, const double *v, const double *Av, const double *diag,
                       double *out, double *partials, hipStream_t s);
void launch_s_pow_init(const SegTab &t, uint64_t salt, int level, double *v, hipStream_t s);
// segment index of every row
void launch_s_rowseg(const SegTab &t, int32_t *rowseg, hipStream_t s);
// omega D^-1 per row (omega per segment)
void launch_s_wdinv(const SegTab &t, const double *omega, const double *dinv, double *wdinv,
                    float *wdinv32, hipStream_t s);
// per-segment max |a| over the entries of the segment's rows
void launch_s_absmax(const SegTab &t, const int64_t *rp, const double *val,
                     unsigned long long *amax, hipStream_t s);
void launch_s_candidate_init(const SegTab &t, uint64_t salt, const unsigned long long *amax,
                             uint64_t idx_off, double *B, hipStream_t s);
// aggregation / colouring keys from body-local row indices
void launch_s_mis_init(const SegTab &t, const uint8_t *conn, uint64_t salt, int level,
                       uint64_t *key, hipStream_t s);
void launch_s_color_keys(const SegTab &t, uint64_t salt, int level, uint64_t *key,
                         hipStream_t s);

// ---- dense coarsest blocks of several bodies ----
struct DenseJob {        // one body's last level
  int64_t row0;          // first row in its level
  int64_t n;             // rows
  int64_t ainv;          // offset of its inverse in the packed inverse buffer
  int64_t scratch;       // offset of its scratch (2 np^2 doubles, np = n rounded up to 16)
  int64_t nnz0;          // first entry of its rows in the level's CSR
};
void launch_dense_factor_batch(int njobs, const DenseJob *jobs, const int64_t *rp,
                               const int32_t *col, const double *val, double *scratch,
                               double *ainv, int *status, hipStream_t s);
// z[row0 + i] = sum_k Ainv[i][k] r[row0 + k] for every job (wave per row)
template <class T>
void launch_dense_apply_batch(int njobs, const DenseJob *jobs, int64_t total_rows,
                              const int64_t *rowstart, const double *ainv, const T *r, T *z,
                              const int *done, hipStream_t s);

}  // namespace mgpbd
