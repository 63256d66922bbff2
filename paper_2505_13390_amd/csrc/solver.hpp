// AMG hierarchy (setup phase, Sec. 4.1-4.3, 4.5) and MGPCG solve (Sec. 4.4)
// on one GPU, for one body or for several bodies at once. Several bodies form
// a block-diagonal system: every level stores the rows of the bodies that
// reach it back to back (segments), each body keeps its own Jacobi weights,
// coarsening depth, coarsest factor and PCG scalars, and every kernel of an
// iteration covers all bodies in one launch. The host sequences kernels; all
// data stays in device memory.
#pragma once

#include <memory>

#include "mfree.hpp"
#include "seg.hpp"
#include "setup.hpp"
#include "tail.hpp"

namespace mgpbd {

struct Level {
  int64_t n = 0, nnz = 0;
  int lanes = 16;    // lanes per row of the FP64 row-group kernels (autotuned)
  int lanes32 = 16;  // same for the FP32 copy
  int tile = 0, tile32 = 0;  // > 0: LDS stream kernels with row tiles of this many entries
  bool nt = false, nt32 = false;  // non-temporal matrix loads in the stream kernels
  DevBuf<int64_t> tiles, tiles32;
  int64_t ntiles = 0, ntiles32 = 0;
  // SELL-C-sigma copy when the autotuner picks it (sell / sell32): layout,
  // and the slot of every CSR entry for refreshing its values
  bool sell = false, sell32 = false;
  int64_t sell_chunks = 0;
  DevBuf<int32_t> sell_perm, sell_col;
  DevBuf<int64_t> sell_ptr, sell_slot;
  DevBuf<double> sell_val;
  DevBuf<float> sell_val32;
  DevBuf<int64_t> rowptr;
  DevBuf<int32_t> col;
  DevBuf<double> val;
  DevBuf<float> val32;
  DevBuf<int64_t> diagpos;
  DevBuf<double> diag, dinv, wdinv;   // wdinv = omega(body) / a_ii
  DevBuf<float> wdinv32, dinv32;
  // Chebyshev smoother: coefficient table [segment][step][2], row -> segment
  // (several segments only), search direction
  DevBuf<double> cheb, dir;
  DevBuf<float> cheb32, dir32;
  DevBuf<int32_t> rowseg;
  // bodies present on this level
  std::vector<int64_t> seg;           // row offsets, one segment per body
  std::vector<int32_t> body;          // body id of each segment
  std::vector<double> omega;          // Jacobi weight of each segment
  std::vector<double> lmax;           // lmax_scale * lambda_max estimate of each segment
  std::vector<char> terminal;         // the body has no coarser level
  SegTable tab;
  DevBuf<double> d_omega;
  // dense coarsest solves of the bodies that end here
  std::vector<DenseJob> jobs;
  DevBuf<DenseJob> d_jobs;
  DevBuf<int64_t> d_jobstart;
  int64_t job_rows = 0;
  bool smooth_here = true;            // false when every body ending here is solved densely
  // entries of this (coarse) level: row of each entry and its transpose position
  DevBuf<int32_t> crow, mirror;
  // transfer to the next level
  bool has_next = false;
  int64_t n_agg = 0;
  int rlanes = 8;   // lanes per aggregate in the restriction (from the mean aggregate size)
  DevBuf<int32_t> agg;
  DevBuf<int64_t> agg_ptr;
  DevBuf<int32_t> agg_mem;
  DevBuf<double> p, B;
  DevBuf<float> p32;
  // fine entries feeding each entry of the next level (of each aggregate block
  // when K > 1), ascending fine order
  DevBuf<int64_t> gl_ptr;
  DevBuf<int32_t> gl_idx, gl_row;
  // K > 1 candidates: B is [n][K]; P row of member slot m is Q[m][0..kq-1];
  // the next level's aggregate-level pattern (entries, their rows and
  // mirrors, each block's start within the expanded rows)
  int K = 1;
  int64_t nmem = 0, annz = 0;
  DevBuf<int32_t> kq, slot, acol, acrow, amirror;
  DevBuf<int64_t> coff, arp, cstart;
  DevBuf<double> Q;
  DevBuf<float> Q32;
  // multicolour order (level 0 near-kernel sweeps)
  int n_colors = 0;
  std::vector<int64_t> color_off;
  DevBuf<int32_t> color, color_rows;
  // V-cycle vectors
  DevBuf<double> r, z, t, res;
  DevBuf<float> r32, z32, t32, res32;

  CsrView<double> view() const {
    CsrView<double> v;
    v.n = n; v.nnz = nnz; v.rowptr = rowptr.p; v.col = col.p; v.val = val.p; v.lanes = lanes;
    v.tile = tile; v.nt = nt; v.ntiles = ntiles; v.tiles = tiles.p;
    if (sell) v.sell = {sell_chunks, sell_perm.p, sell_ptr.p, sell_col.p, sell_val.p};
    return v;
  }
  CsrView<float> view32() const {
    CsrView<float> v;
    v.n = n; v.nnz = nnz; v.rowptr = rowptr.p; v.col = col.p; v.val = val32.p; v.lanes = lanes32;
    v.tile = tile32; v.nt = nt32; v.ntiles = ntiles32; v.tiles = tiles32.p;
    if (sell32) v.sell = {sell_chunks, sell_perm.p, sell_ptr.p, sell_col.p, sell_val32.p};
    return v;
  }
};

struct PcgResult {
  int status = 0;  // PcgCtl::done code
  int iters = 0;
  double ratio = 0.0;
  double bnorm = 0.0;
};

class Solver {
 public:
  explicit Solver(const mgpbd_options &o);
  ~Solver();

  mgpbd_options opt;
  hipStream_t st = nullptr;
  std::vector<std::unique_ptr<Level>> lev;
  int nlev = 0;
  int nb = 1;                   // bodies (segments of level 0)
  bool built = false;
  bool val32_external = false;  // level-0 FP32 values written by the assembler
  bool pattern_dirty = true;    // level-0 pattern changed: recompute diagpos / tuning

  // matrix-free level-0 operator, set by a simulation context (unset: the
  // level-0 passes read the assembled CSR); mf32 serves the FP32 V-cycle
  MfView<double> mf;
  MfView<float> mf32;

  // per-iteration profiling of the fine-level A p product
  int64_t spmv_calls = 0;
  double spmv_ms = 0.0;        // whole product (both kernels when matrix-free)
  double spmv_first_ms = 0.0;  // its first kernel (the matrix-free gather; 0 for CSR)
  // profiling of the V-cycle level by level: each level's own passes (entry to
  // descent plus return to exit) summed over the timed V-cycles
  static constexpr int kProfLevels = 16;
  // fused coarse end of the V-cycle (tail.hpp): start level (0 = not used),
  // bodies present there, per-level views in both precisions, per-body rows
  int tail_l0 = 0;
  int tail_nb = 0;
  TailPlan tail_plan;
  DevBuf<TailLevel<double>> tail_lv;
  DevBuf<TailLevel<float>> tail_lv32;
  DevBuf<TailBody> tail_bodies;
  void plan_tail();
  void choose_fine_operator();   // matrix_free = 2: keep the faster fine-level product
  void sync_sell();   // SELL copies take the levels' current values
  void sync_sell_level(int l);
  void build_sell_level(int l, const std::vector<int64_t> &hrp);
  double level_ms[kProfLevels] = {};
  int64_t vcycles = 0;
  void reset_profile();

  Level &L0() { return *lev[0]; }
  bool mixed() const { return opt.precision == MGPBD_PREC_MIXED; }
  void set_stream(hipStream_t s);
  void invalidate_graph();
  // row offsets of the bodies on level 0 (default: one body covering all rows)
  void set_bodies(const std::vector<int64_t> &offsets);
  // levels of body k in the current hierarchy
  int body_levels(int k) const;

  // Full setup on the current level-0 values (aggregation, candidates, P,
  // Galerkin pattern and values, omega, coarsest inverses).
  void setup();
  // Solving-phase refresh for new level-0 values with the kept P and omega.
  void refresh();
  // MGPCG on A_0 for every body at once: x_out <- A_0^-1 b; force (nullable,
  // [nb]) fixes iteration counts. One result per body.
  // y = A x on the fine level with the PCG loop's own kernels (no sync)
  void apply_fine(const double *x, double *y);
  // the same product with the matrix-free gather vector in the caller's u
  // ([nv][4]) and no partial sums: allocates nothing
  void apply_fine_into(const double *x, double *y, double *u);
  std::vector<PcgResult> pcg(const double *b, double *x_out, double tol, int max_iters,
                             const int32_t *force);
  double *dl() { return x.p; }   // internal PCG iterate
  // per-body sum of squares of a level-0 vector (synchronous)
  std::vector<double> norm2(const double *v);

 private:
  DevBuf<PcgCtl> ctl;
  DevBuf<int> all_done;
  DevBuf<double> red_partials;
  DevBuf<double> x, r, z, p, q;
  DevBuf<float> zold32;   // FP32 V-cycle: the previous z (flexible beta)
  DevBuf<double> dscal;
  DevBuf<int> flags;
  DevBuf<unsigned long long> amax;
  DevBuf<int64_t> scan_tmp;
  DevBuf<uint8_t> strong, conn;
  DevBuf<uint64_t> key, m1;
  DevBuf<int32_t> itmp, itmp2;
  DevBuf<int64_t> ltmp, ltmp2;
  DevBuf<double> dscratch, Ainv;
  std::vector<char> force_last, stalled;
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_ok = false;
  std::vector<hipEvent_t> ev;
  // level events of the profiled V-cycles: [chunk slot][level][4] (entry,
  // descent, return, exit); prof_k = slot of the V-cycle being recorded
  std::vector<hipEvent_t> lev_ev;
  int prof_k = -1;
  // the PCG update already wrote the fine level's first Jacobi iterate (and
  // the FP32 residual): the next vcycle(0) skips that step
  bool first_ready = false;
  FirstSweep first_sweep_targets();
  // level l >= 1 takes its first Jacobi iterate from the restriction into it
  bool first_from_restriction(int l) const;
  void pmark(int l, int j);

  double *partials() { return red_partials.p; }
  const int *done_ptr() const;
  int read_flag(int k);
  void reset_flags();
  void ensure_vectors();
  void ensure_pinned(size_t bytes);
  void ensure_partials(int nblk);
  void finish_level(int l);
  std::vector<int64_t> aggregate(int l);
  void candidate0();
  void colour_level(int l);
  void build_members(int l);
  // aggregate rows whose symbolic Galerkin tables live in global memory
  struct BigRows {
    int n = 0;
    DevBuf<int32_t> rows, tcap, scratch;
    DevBuf<int64_t> toff;
  };
  void gal_count_rows(int l, BigRows &big);
  void gal_fill_rows(int l, const BigRows &big, const int64_t *crp, const int64_t *eoff,
                     int32_t *ccol, int32_t *crow);
  void galerkin_symbolic(int l);
  void galerkin_numeric(int l);
  int64_t qr_level(int l);
  void galerkin_symbolic_k(int l);
  template <class T> void restrict_to(int l, const T *res, T *rc, CoarseFirst<T> first = {});
  template <class T> void prolong_from(int l, const T *ec, T *z);
  void power_omega(int l);
  void tune_lanes(int l);
  void chebyshev_table(int l);
  void plan_dense();
  void factor_dense();
  void iterate_once(int k);
  template <class T> void vcycle(int l, const T *r, T *z);
  template <class T> void gs_vcycle(int l, const T *r, T *z);
  template <class T> const MfView<T> *level_mf(int l) const;
};

}  // namespace mgpbd
