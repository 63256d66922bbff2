// AMG setup and MGPCG orchestration (host side). See solver.hpp.
#include "solver.hpp"

#include <algorithm>
#include <cmath>
#include <cstddef>

namespace mgpbd {

template <class V>
static V read_dev(const V *d, hipStream_t st, void *pinned) {
  V *h = static_cast<V *>(pinned);
  MG_HIP(hipMemcpyAsync(h, d, sizeof(V), hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  return *h;
}

enum Flag { kFBadDiag = 0, kFOverflow, kFUndecided, kFRemaining, kFColorOver, kFChol, kFMirror,
            kFDiagMissing, kNumFlags };

Solver::Solver(const mgpbd_options &o) : opt(o) {
  lev.emplace_back(new Level());
  nlev = 1;
  ctl.alloc(1);
  all_done.alloc(1);
  red_partials.alloc(kMaxBlockSums * (size_t)kMaxGrid + 64);
  dscal.alloc(16);
  flags.alloc(kNumFlags);
  amax.alloc(1);
  ensure_pinned(4096);
}

Solver::~Solver() {
  invalidate_graph();
  for (auto e : ev) (void)hipEventDestroy(e);
  for (auto e : lev_ev) (void)hipEventDestroy(e);
  if (pinned) (void)hipHostFree(pinned);
}

void Solver::ensure_pinned(size_t bytes) {
  if (bytes <= pinned_bytes) return;
  if (pinned) (void)hipHostFree(pinned);
  pinned = nullptr;
  pinned_bytes = 0;
  MG_HIP(hipHostMalloc(&pinned, bytes, hipHostMallocDefault));
  pinned_bytes = bytes;
}

void Solver::ensure_partials(int nblk) {
  red_partials.reserve(kMaxBlockSums * (size_t)std::max(nblk, kMaxGrid) + 64);
}

void Solver::reset_profile() {
  spmv_calls = 0;
  spmv_ms = 0.0;
  spmv_first_ms = 0.0;
  vcycles = 0;
  for (double &v : level_ms) v = 0.0;
}

void Solver::pmark(int l, int j) {
  if (prof_k < 0 || l >= kProfLevels) return;
  MG_HIP(hipEventRecord(lev_ev[((size_t)prof_k * kProfLevels + l) * 4 + j], st));
}

void Solver::set_stream(hipStream_t s) {
  if (s != st) invalidate_graph();
  st = s;
}

void Solver::invalidate_graph() {
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  gexec = nullptr;
  graph = nullptr;
  graph_ok = false;
}

void Solver::set_bodies(const std::vector<int64_t> &offsets) {
  MG_REQUIRE(offsets.size() >= 2 && offsets.front() == 0, MGPBD_E_INVALID_ARG, "body offsets");
  for (size_t k = 1; k < offsets.size(); ++k)
    MG_REQUIRE(offsets[k] >= offsets[k - 1], MGPBD_E_INVALID_ARG, "body offsets must ascend");
  nb = (int)offsets.size() - 1;
  Level &F = L0();
  F.seg = offsets;
  F.body.resize(nb);
  for (int k = 0; k < nb; ++k) F.body[k] = k;
  built = false;
  invalidate_graph();
}

int Solver::body_levels(int k) const {
  int d = 0;
  for (int l = 0; l < nlev; ++l)
    if (std::find(lev[l]->body.begin(), lev[l]->body.end(), k) != lev[l]->body.end()) d = l + 1;
  return d;
}

// with one body the V-cycle kernels read that body's control block directly
const int *Solver::done_ptr() const {
  if (nb == 1)
    return reinterpret_cast<const int *>(reinterpret_cast<const char *>(ctl.p) +
                                         offsetof(PcgCtl, done));
  return all_done.p;
}

void Solver::reset_flags() { MG_HIP(hipMemsetAsync(flags.p, 0, sizeof(int) * kNumFlags, st)); }

int Solver::read_flag(int k) { return read_dev(flags.p + k, st, pinned); }

std::vector<double> Solver::norm2(const double *v) {
  Level &F = L0();
  if (F.seg.empty() || F.seg.back() != F.n) set_bodies({0, F.n});
  if (F.tab.off != F.seg) F.tab.build(F.seg, st);
  SegTab t = F.tab.view();
  ensure_partials(t.nblk);
  dscal.reserve(std::max<size_t>(16, 3 * (size_t)nb + 8));
  launch_s_dot(t, v, v, dscal.p, partials(), st);
  std::vector<double> out(nb);
  MG_HIP(hipMemcpyAsync(out.data(), dscal.p, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  return out;
}

// ------------------------------------------------------------------ setup
void Solver::finish_level(int l) {
  Level &L = *lev[l];
  L.tab.build(L.seg, st);
  ensure_partials(L.tab.view().nblk);
  if (l > 0 || pattern_dirty) {
    L.diagpos.alloc(L.n);
    reset_flags();
    launch_diagpos(L.n, L.rowptr.p, L.col.p, L.diagpos.p, flags.p + kFDiagMissing, st);
    MG_REQUIRE(read_flag(kFDiagMissing) == 0, MGPBD_E_INVALID_ARG,
               "level " + std::to_string(l) + " has a row without a diagonal entry");
    L.lanes = L.lanes32 = lanes_for_rowlen(L.n ? (double)L.nnz / (double)L.n : 1.0);
    if (l == 0) pattern_dirty = false;
    L.r.alloc(L.n); L.t.alloc(L.n);
    if (mixed()) { L.r32.alloc(L.n); L.t32.alloc(L.n); }
    tune_lanes(l);
    if (l == 0 && opt.matrix_free == 2 && mf.ok()) choose_fine_operator();
  }
  L.diag.alloc(L.n);
  L.dinv.alloc(L.n);
  L.wdinv.alloc(L.n);
  if (mixed()) L.wdinv32.alloc(L.n);
  if (mixed() && opt.smoother != 0) L.dinv32.alloc(L.n);
  reset_flags();
  launch_extract_diag(L.n, L.diagpos.p, L.val.p, L.diag.p, L.dinv.p, L.dinv32.p,
                      flags.p + kFBadDiag, st);
  MG_REQUIRE(read_flag(kFBadDiag) == 0, MGPBD_E_BREAKDOWN,
             "level " + std::to_string(l) + " has a non-positive diagonal entry");
  // vectors of the V-cycle
  L.r.alloc(L.n); L.z.alloc(L.n); L.t.alloc(L.n);
  if (mixed()) { L.r32.alloc(L.n); L.z32.alloc(L.n); L.t32.alloc(L.n); }
  L.res.alloc(L.n);
  if (mixed()) L.res32.alloc(L.n);
  sync_sell_level(l);   // the products below read the level's SELL copy when it has one
  power_omega(l);
  if (opt.smoother == 1) chebyshev_table(l);
  if (opt.smoother == 2) colour_level(l);
  L.d_omega.upload(L.omega.data(), L.omega.size(), st);
  launch_s_wdinv(L.tab.view(), L.d_omega.p, L.dinv.p, L.wdinv.p, mixed() ? L.wdinv32.p : nullptr,
                 st);
}

// Autotuner of the CSR passes: on large levels, time one product for each
// variant (lanes per row of the row-group kernel; tile size and load kind of
// the LDS stream kernel) and keep the fastest, separately for FP64 and FP32.
void Solver::tune_lanes(int l) {
  Level &L = *lev[l];
  L.tile = L.tile32 = 0;
  L.nt = L.nt32 = false;
  L.sell = L.sell32 = false;
  if (opt.spmv_lanes > 0) L.lanes = L.lanes32 = opt.spmv_lanes;
  if (opt.spmv_tile > 0 && L.n > 0) {
    std::vector<int64_t> hrp(L.n + 1), part;
    L.rowptr.download(hrp.data(), L.n + 1, st);
    MG_HIP(hipStreamSynchronize(st));
    if (build_row_tiles(hrp, opt.spmv_tile, part)) {
      L.tile = L.tile32 = opt.spmv_tile;
      L.tiles.upload(part.data(), part.size(), st);
      L.tiles32.upload(part.data(), part.size(), st);
      L.ntiles = L.ntiles32 = (int64_t)part.size() - 1;
      MG_HIP(hipStreamSynchronize(st));
    }
    return;
  }
  if (opt.spmv_tile == -2 && L.n > 0) {   // SELL-C-sigma on every level
    std::vector<int64_t> hrp(L.n + 1);
    L.rowptr.download(hrp.data(), L.n + 1, st);
    MG_HIP(hipStreamSynchronize(st));
    build_sell_level(l, hrp);
    L.sell = true;
    L.sell32 = mixed() && L.sell_val32.p;
    MG_HIP(hipStreamSynchronize(st));
    return;
  }
  if (opt.spmv_tile < 0 || opt.spmv_lanes > 0 || L.n < 20000) return;
  std::vector<int64_t> hrp(L.n + 1);
  L.rowptr.download(hrp.data(), L.n + 1, st);
  MG_HIP(hipStreamSynchronize(st));
  struct Cand { int lanes, tile; bool nt; std::vector<int64_t> part; bool sell; };
  std::vector<Cand> cands;
  for (int g : {8, 16, 32, 64}) cands.push_back({g, 0, false, {}, false});
  for (int t : {1024, 2048, 4096})
    for (bool ntl : {false, true}) {
      Cand c{16, t, ntl, {}, false};
      if (build_row_tiles(hrp, t, c.part)) cands.push_back(std::move(c));
    }
  // the SELL-C-sigma copy of this level, timed like the CSR variants
  build_sell_level(l, hrp);
  cands.push_back({0, 0, false, {}, true});
  hipEvent_t a, b;
  MG_HIP(hipEventCreate(&a));
  MG_HIP(hipEventCreate(&b));
  launch_fill(L.n, 1.0, L.r.p, st);
  const bool do32 = mixed() && L.val32.p;
  if (do32) launch_d2f(L.n, L.r.p, L.r32.p, nullptr, st);
  DevBuf<int64_t> tmp;
  float best = 1e30f, best32 = 1e30f;
  size_t pick = 0, pick32 = 0;
  auto timeit = [&](auto &&fn) {
    fn();  // warm
    MG_HIP(hipEventRecord(a, st));
    for (int rep = 0; rep < 3; ++rep) fn();
    MG_HIP(hipEventRecord(b, st));
    MG_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    MG_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  };
  for (size_t k = 0; k < cands.size(); ++k) {
    Cand &c = cands[k];
    if (c.tile) tmp.upload(c.part.data(), c.part.size(), st);
    CsrView<double> A = L.view();
    A.lanes = c.lanes; A.tile = c.tile; A.nt = c.nt;
    A.ntiles = c.tile ? (int64_t)c.part.size() - 1 : 0;
    A.tiles = c.tile ? tmp.p : nullptr;
    if (c.sell) A.sell = {L.sell_chunks, L.sell_perm.p, L.sell_ptr.p, L.sell_col.p, L.sell_val.p};
    float ms = timeit([&] { launch_spmv<double>(A, L.r.p, L.t.p, st); });
    if (ms < best) { best = ms; pick = k; }
    if (do32) {
      CsrView<float> F = L.view32();
      F.lanes = c.lanes; F.tile = c.tile; F.nt = c.nt; F.ntiles = A.ntiles; F.tiles = A.tiles;
      if (c.sell)
        F.sell = {L.sell_chunks, L.sell_perm.p, L.sell_ptr.p, L.sell_col.p, L.sell_val32.p};
      float ms32 = timeit([&] { launch_spmv<float>(F, L.r32.p, L.t32.p, st); });
      if (ms32 < best32) { best32 = ms32; pick32 = k; }
    }
  }
  MG_HIP(hipStreamSynchronize(st));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  const Cand &c = cands[pick];
  L.sell = c.sell;
  L.sell32 = do32 && cands[pick32].sell;
  if (c.sell) L.lanes = lanes_for_rowlen(L.n ? (double)L.nnz / (double)L.n : 1.0);
  else L.lanes = c.lanes;
  L.tile = c.tile;
  L.nt = c.nt;
  if (c.tile) {
    L.tiles.upload(c.part.data(), c.part.size(), st);
    L.ntiles = (int64_t)c.part.size() - 1;
  }
  if (do32) {
    const Cand &c32 = cands[pick32];
    L.lanes32 = c32.sell ? lanes_for_rowlen(L.n ? (double)L.nnz / (double)L.n : 1.0) : c32.lanes;
    L.tile32 = c32.tile;
    L.nt32 = c32.nt;
    if (c32.tile) {
      L.tiles32.upload(c32.part.data(), c32.part.size(), st);
      L.ntiles32 = (int64_t)c32.part.size() - 1;
    }
  }
  if (!L.sell) L.sell_val.release();
  if (!L.sell32) L.sell_val32.release();
  if (!L.sell && !L.sell32) {
    L.sell_perm.release();
    L.sell_ptr.release();
    L.sell_col.release();
    L.sell_slot.release();
    L.sell_chunks = 0;
  }
  MG_HIP(hipStreamSynchronize(st));
}

// SELL-C-sigma layout of level l (host build from its pattern) with the
// level's current values (FP32 as well in the mixed path)
void Solver::build_sell_level(int l, const std::vector<int64_t> &hrp) {
  Level &L = *lev[l];
  std::vector<int32_t> hcol(L.nnz), perm, scol;
  std::vector<int64_t> ptr, slot;
  L.col.download(hcol.data(), L.nnz, st);
  MG_HIP(hipStreamSynchronize(st));
  build_sell(hrp, hcol, perm, ptr, scol, slot);
  L.sell_chunks = (int64_t)ptr.size() - 1;
  L.sell_perm.upload(perm.data(), perm.size(), st);
  L.sell_ptr.upload(ptr.data(), ptr.size(), st);
  L.sell_col.upload(scol.data(), scol.size(), st);   // non-empty: every row has its diagonal
  L.sell_slot.upload(slot.data(), slot.size(), st);
  L.sell_val.alloc(std::max<size_t>(scol.size(), 1));
  MG_HIP(hipMemsetAsync(L.sell_val.p, 0, sizeof(double) * L.sell_val.n, st));
  launch_sell_values<double, double>(L.nnz, L.sell_slot.p, L.val.p, L.sell_val.p, st);
  if (mixed() && L.val32.p) {
    L.sell_val32.alloc(std::max<size_t>(scol.size(), 1));
    MG_HIP(hipMemsetAsync(L.sell_val32.p, 0, sizeof(float) * L.sell_val32.n, st));
    launch_sell_values<float, float>(L.nnz, L.sell_slot.p, L.val32.p, L.sell_val32.p, st);
  }
  MG_HIP(hipStreamSynchronize(st));
}

void Solver::sync_sell_level(int l) {
  Level &L = *lev[l];
  if (L.sell) launch_sell_values<double, double>(L.nnz, L.sell_slot.p, L.val.p, L.sell_val.p, st);
  if (L.sell32) {
    if (L.val32.p)
      launch_sell_values<float, float>(L.nnz, L.sell_slot.p, L.val32.p, L.sell_val32.p, st);
    else
      launch_sell_values<double, float>(L.nnz, L.sell_slot.p, L.val.p, L.sell_val32.p, st);
  }
}

void Solver::sync_sell() {
  for (int l = 0; l < nlev; ++l) sync_sell_level(l);
}

// omega = 2 / (lmax_scale lambda_max(D^-1 A) + lambda_min) for each body,
// lambda_max from the power method (Sec. 4.5): v <- D^-1 A v / |D^-1 A v|
// from a positive pseudo-random start. At step power_iters and then every
// kPowerCheck steps the Rayleigh quotient theta = v^T A v / v^T D v and the
// eigen-residual |D^-1 A v - theta v|_D are formed from the step's own
// product A v; a body stops once the residual is at most power_tol theta
// |v|_D (or at step power_max) and keeps that theta. With w = A v,
// |D^-1 w - theta v|_D^2 = sum w_i^2 / d_i - theta v^T w. Bodies are
// independent (block-diagonal A, per-body normalisation), so iterating a body
// past its stop does not change the others.
static constexpr int kPowerCheck = 10;
void Solver::power_omega(int l) {
  Level &L = *lev[l];
  const int ns = (int)L.seg.size() - 1;
  L.omega.assign(ns, 0.0);
  L.lmax.assign(ns, 0.0);
  if (L.n == 0) return;
  SegTab t = L.tab.view();
  dscal.reserve(std::max<size_t>(16, 4 * (size_t)ns + 8));
  double *nrm2 = dscal.p, *ray = dscal.p + ns;
  double *v = L.r.p, *w = L.t.p;
  launch_s_pow_init(t, stream_salt(opt.seed, kStreamPowerStart), l, v, st);
  CsrView<double> A = L.view();
  std::vector<double> theta(ns, 0.0), h(3 * (size_t)ns);
  std::vector<char> stopped(ns, 0);
  // a body without rows has no estimate to make
  int left = 0;
  for (int k = 0; k < ns; ++k) {
    if (L.seg[k + 1] == L.seg[k]) stopped[k] = 1;
    else ++left;
  }
  for (int it = 0; left > 0; ++it) {
    launch_spmv<double>(A, v, w, st);
    const bool last = it >= opt.power_max;
    if (last || (it >= opt.power_iters && (it - opt.power_iters) % kPowerCheck == 0)) {
      launch_s_rayleigh(t, v, w, L.diag.p, ray, partials(), st);
      MG_HIP(hipMemcpyAsync(h.data(), ray, sizeof(double) * 3 * ns, hipMemcpyDeviceToHost, st));
      MG_HIP(hipStreamSynchronize(st));
      for (int k = 0; k < ns; ++k) {
        if (stopped[k]) continue;
        const double s1 = h[3 * k], s2 = h[3 * k + 1], s3 = h[3 * k + 2];
        const double th = s1 / s2;
        const double res2 = s3 - th * s1;
        const double res = res2 > 0.0 ? std::sqrt(res2) : 0.0;
        theta[k] = th;
        if (last || res <= opt.power_tol * th * std::sqrt(s2)) {
          stopped[k] = 1;
          --left;
        }
      }
      if (left == 0) break;
    }
    launch_s_pow_scale(t, w, L.diag.p, nrm2, partials(), st);
    launch_s_pow_normalize(t, w, nrm2, v, st);
  }
  for (int k = 0; k < ns; ++k) {
    L.lmax[k] = opt.lmax_scale * theta[k];
    L.omega[k] = 2.0 / (L.lmax[k] + opt.lambda_min);
  }
}

// Chebyshev smoother coefficients of every body on level l (Sec. 4.5, the
// recurrence of Saad, Alg. 12.1, with M = D) on [lambda_min, lmax]:
// theta = (b + a)/2, delta = (b - a)/2, sigma = theta/delta; step 0 uses
// c2 = 1/theta; step k >= 1 uses rho_k = 1/(2 sigma - rho_{k-1}) (rho_0 =
// 1/sigma), c1 = rho_k rho_{k-1}, c2 = 2 rho_k / delta.
void Solver::chebyshev_table(int l) {
  Level &L = *lev[l];
  const int ns = (int)L.seg.size() - 1;
  const int steps = std::max(1, std::max(opt.pre_sweeps, opt.post_sweeps));
  std::vector<double> c((size_t)2 * steps * ns, 0.0);
  for (int g = 0; g < ns; ++g) {
    const double a = opt.lambda_min, b = L.lmax[g];
    const double theta = (b + a) / 2.0, delta = (b - a) / 2.0, sigma = theta / delta;
    double rho = 1.0 / sigma;
    for (int k = 0; k < steps; ++k) {
      double c1 = 0.0, c2 = 1.0 / theta;
      if (k > 0) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        c1 = rn * rho;
        c2 = 2.0 * rn / delta;
        rho = rn;
      }
      c[2 * ((size_t)g * steps + k)] = c1;
      c[2 * ((size_t)g * steps + k) + 1] = c2;
    }
  }
  L.cheb.upload(c.data(), c.size(), st);
  if (mixed()) {
    std::vector<float> f(c.begin(), c.end());
    L.cheb32.upload(f.data(), f.size(), st);
  }
  if (ns > 1) {
    L.rowseg.alloc(std::max<int64_t>(L.n, 1));
    launch_s_rowseg(L.tab.view(), L.rowseg.p, st);
  } else {
    L.rowseg.release();
  }
  L.dir.alloc(std::max<int64_t>(L.n, 1));
  if (mixed()) L.dir32.alloc(std::max<int64_t>(L.n, 1));
  MG_HIP(hipStreamSynchronize(st));
}

// Aggregation of every body that coarsens further (Sec. 4.1); rows of bodies
// that end on this level count as isolated and join no aggregate. Returns the
// first aggregate of each body (size nseg + 1).
std::vector<int64_t> Solver::aggregate(int l) {
  Level &L = *lev[l];
  const int64_t n = L.n;
  const int ns = (int)L.seg.size() - 1;
  CsrView<double> A = L.view();
  strong.reserve(L.nnz);
  conn.reserve(n);
  key.reserve(n);
  m1.reserve(n);
  const double theta2 = opt.theta * opt.theta;
  launch_strong(A, L.diag.p, theta2, strong.p, conn.p, st);
  for (int k = 0; k < ns; ++k)
    if (L.terminal[k] && L.seg[k + 1] > L.seg[k])
      launch_fill_u8(L.seg[k + 1] - L.seg[k], 0, conn.p + L.seg[k], st);
  launch_s_mis_init(L.tab.view(), conn.p, stream_salt(opt.seed, kStreamAggPrio), l, key.p, st);
  for (int round = 0;; ++round) {
    MG_REQUIRE(round < 100000, MGPBD_E_SETUP, "aggregation did not terminate");
    reset_flags();
    launch_mis_round(A, strong.p, key.p, m1.p, flags.p + kFUndecided, st);
    if (read_flag(kFUndecided) == 0) break;
  }
  itmp.reserve(n);
  ltmp.reserve(n + 1);
  launch_root_flags(n, key.p, itmp.p, st);
  scan_exclusive_i32_to_i64(itmp.p, ltmp.p, n, scan_tmp, st);
  // aggregates are numbered by ascending root row, so each body's aggregates
  // are the roots ranked inside its row range
  std::vector<int64_t> first(ns + 1);
  if (ns == 1) {
    first[0] = 0;
    first[1] = read_dev(ltmp.p + n, st, pinned);
  } else {
    std::vector<int64_t> rank(n + 1);
    ltmp.download(rank.data(), n + 1, st);
    MG_HIP(hipStreamSynchronize(st));
    for (int k = 0; k <= ns; ++k) first[k] = rank[L.seg[k]];
  }
  L.n_agg = first[ns];
  L.agg.alloc(n);
  itmp2.reserve(n);
  launch_pass1(A, strong.p, key.p, ltmp.p, itmp2.p, st);
  launch_pass2(A, strong.p, conn.p, itmp2.p, L.agg.p, st);
  return first;
}

// Greedy colouring of level l in descending priority (Jones-Plassmann by
// counters; keys from body-local indices, so each body is coloured as if it
// were alone) and the rows of each colour: the order of the near-kernel
// sweeps (level 0) and of the Gauss-Seidel smoother (every level).
void Solver::colour_level(int l) {
  Level &L = *lev[l];
  const int64_t n = L.n;
  CsrView<double> A = L.view();
  SegTab t = L.tab.view();
  key.reserve(n);
  L.color.alloc(n);
  launch_s_color_keys(t, stream_salt(opt.seed, kStreamColorPrio), l, key.p, st);
  launch_fill_i32(n, -1, L.color.p, st);
  {
    itmp.reserve(n);             // higher-priority neighbour counts
    DevBuf<int32_t> fr[2];
    fr[0].alloc(std::max<int64_t>(n, 1));
    fr[1].alloc(std::max<int64_t>(n, 1));
    reset_flags();
    launch_color_count(A, key.p, itmp.p, fr[0].p, flags.p + kFRemaining, st);
    int64_t nf = read_flag(kFRemaining), done_rows = 0;
    for (int round = 0; nf > 0; ++round) {
      MG_REQUIRE(round < 1000000, MGPBD_E_SETUP, "colouring did not terminate");
      done_rows += nf;
      MG_REQUIRE(done_rows <= n, MGPBD_E_SETUP, "colouring frontier overflow");
      const int cur = round & 1;
      MG_HIP(hipMemsetAsync(flags.p + kFRemaining, 0, sizeof(int), st));
      launch_color_front(A, nf, fr[cur].p, key.p, L.color.p, itmp.p, fr[cur ^ 1].p,
                         flags.p + kFRemaining, flags.p + kFColorOver, st);
      nf = read_flag(kFRemaining);
    }
    MG_REQUIRE(read_flag(kFColorOver) == 0, MGPBD_E_SETUP, "more than 256 colours needed");
    MG_REQUIRE(done_rows == n, MGPBD_E_SETUP, "colouring left rows uncoloured");
  }
  // rows grouped by colour
  itmp.reserve(256);
  MG_HIP(hipMemsetAsync(itmp.p, 0, 256 * sizeof(int32_t), st));
  launch_count_colors(n, L.color.p, itmp.p, st);
  std::vector<int32_t> cnt(256);
  MG_HIP(hipMemcpyAsync(cnt.data(), itmp.p, 256 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  L.n_colors = 0;
  for (int c = 0; c < 256; ++c) if (cnt[c]) L.n_colors = c + 1;
  L.color_off.assign(L.n_colors + 1, 0);
  for (int c = 0; c < L.n_colors; ++c) L.color_off[c + 1] = L.color_off[c] + cnt[c];
  ltmp2.reserve(257);
  MG_HIP(hipMemcpyAsync(ltmp2.p, L.color_off.data(), sizeof(int64_t) * (L.n_colors + 1),
                        hipMemcpyHostToDevice, st));
  MG_HIP(hipMemsetAsync(itmp.p, 0, 256 * sizeof(int32_t), st));
  L.color_rows.alloc(n);
  launch_scatter_colors(n, L.color.p, ltmp2.p, itmp.p, L.color_rows.p, st);
  MG_HIP(hipStreamSynchronize(st));
}

// Near-kernel candidates of level 0 (Sec. 4.3): each starts uniform in
// (0, max |A_ij| of its body), drawn with indices k 2^40 + row for candidate
// k, then takes gs_sweeps multicolour Gauss-Seidel sweeps on A x = 0; B is
// [n][K].
void Solver::candidate0() {
  Level &L = *lev[0];
  const int64_t n = L.n;
  const int ns = (int)L.seg.size() - 1;
  const int K = opt.n_cand;
  L.B.alloc(n * K);
  if (opt.b_mode == 1) {
    launch_fill(n * K, 1.0, L.B.p, st);
    return;
  }
  CsrView<double> A = L.view();
  SegTab t = L.tab.view();
  amax.reserve(ns);
  MG_HIP(hipMemsetAsync(amax.p, 0, sizeof(unsigned long long) * ns, st));
  launch_s_absmax(t, L.rowptr.p, L.val.p, amax.p, st);
  if (opt.smoother != 2) colour_level(0);   // (the Gauss-Seidel smoother coloured it already)
  DevBuf<double> x;
  if (K > 1) x.alloc(n);
  for (int k = 0; k < K; ++k) {
    double *v = K > 1 ? x.p : L.B.p;
    launch_s_candidate_init(t, stream_salt(opt.seed, kStreamNearKernel), amax.p,
                            (uint64_t)k << 40, v, st);
    for (int s = 0; s < opt.gs_sweeps; ++s)
      for (int c = 0; c < L.n_colors; ++c)
        launch_gs_color(L.color_off[c + 1] - L.color_off[c], L.color_rows.p + L.color_off[c], A,
                        L.diag.p, v, st);
    if (K > 1) launch_put_column(n, K, k, x.p, L.B.p, st);
  }
  MG_HIP(hipStreamSynchronize(st));
}

void Solver::build_members(int l) {
  Level &L = *lev[l];
  const int64_t na = L.n_agg;
  itmp.reserve(std::max<int64_t>(na, 1));
  MG_HIP(hipMemsetAsync(itmp.p, 0, sizeof(int32_t) * na, st));
  launch_count_members(L.n, L.agg.p, itmp.p, st);
  L.agg_ptr.alloc(na + 1);
  scan_exclusive_i32_to_i64(itmp.p, L.agg_ptr.p, na, scan_tmp, st);
  MG_HIP(hipMemsetAsync(itmp.p, 0, sizeof(int32_t) * na, st));
  int64_t nmem = read_dev(L.agg_ptr.p + na, st, pinned);
  L.nmem = nmem;
  // enough lanes per aggregate that each sums a handful of members: the
  // member loads are scattered, so fewer and longer chains leave the loads
  // waiting one after another
  const double mean = na ? (double)nmem / (double)na : 1.0;
  L.rlanes = mean <= 16.0 ? 8 : mean <= 48.0 ? 16 : mean <= 160.0 ? 32 : 64;
  L.agg_mem.alloc(std::max<int64_t>(nmem, 1));
  launch_scatter_members(L.n, L.agg.p, L.agg_ptr.p, itmp.p, L.agg_mem.p, st);
  launch_sort_segments(na, L.agg_ptr.p, L.agg_mem.p, st);
}

// Aggregate-level symbolic Galerkin counts of level l into ltmp (distinct
// coarse columns per aggregate row) and ltmp2 (connecting fine entries). Rows
// whose columns do not fit the LDS table of k_gal_count are counted again
// with a table in global memory of at least twice their entries; big keeps
// those rows and tables for the fill.
void Solver::gal_count_rows(int l, BigRows &big) {
  Level &L = *lev[l];
  const int64_t na = L.n_agg;
  CsrView<double> A = L.view();
  ltmp.reserve(na + 1);
  ltmp2.reserve(na + 1);
  reset_flags();
  launch_gal_count(na, L.agg_ptr.p, L.agg_mem.p, A, L.agg.p, ltmp.p, ltmp2.p,
                   flags.p + kFOverflow, st);
  big.n = 0;
  if (read_flag(kFOverflow) == 0) return;
  std::vector<int64_t> cnt(na), el(na);
  ltmp.download(cnt.data(), na, st);
  ltmp2.download(el.data(), na, st);
  MG_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> rows, caps;
  std::vector<int64_t> offs;
  int64_t tot = 0;
  for (int64_t a = 0; a < na; ++a) {
    if (cnt[a] >= 0) continue;
    int64_t cap = 2048;
    while (cap < 2 * el[a]) cap <<= 1;
    MG_REQUIRE(cap <= ((int64_t)1 << 30), MGPBD_E_SETUP, "aggregate row too long");
    rows.push_back((int32_t)a);
    caps.push_back((int32_t)cap);
    offs.push_back(tot);
    tot += cap;
  }
  big.n = (int)rows.size();
  big.rows.upload(rows.data(), rows.size(), st);
  big.tcap.upload(caps.data(), caps.size(), st);
  big.toff.upload(offs.data(), offs.size(), st);
  big.scratch.alloc(5 * (size_t)tot);
  reset_flags();
  launch_gal_count_big(big.n, big.rows.p, big.toff.p, big.tcap.p, big.scratch.p, L.agg_ptr.p,
                       L.agg_mem.p, A, L.agg.p, ltmp.p, flags.p + kFOverflow, st);
  MG_REQUIRE(read_flag(kFOverflow) == 0, MGPBD_E_SETUP, "symbolic Galerkin table overflow");
}

void Solver::gal_fill_rows(int l, const BigRows &big, const int64_t *crp, const int64_t *eoff,
                           int32_t *ccol, int32_t *crow) {
  Level &L = *lev[l];
  CsrView<double> A = L.view();
  launch_gal_fill(L.n_agg, L.agg_ptr.p, L.agg_mem.p, A, L.agg.p, crp, eoff, ccol, crow,
                  L.gl_ptr.p, L.gl_idx.p, L.gl_row.p, st);
  launch_gal_fill_big(big.n, big.rows.p, big.toff.p, big.tcap.p, big.scratch.p, L.agg_ptr.p,
                      L.agg_mem.p, A, L.agg.p, crp, eoff, ccol, crow, L.gl_ptr.p, L.gl_idx.p,
                      L.gl_row.p, st);
}

void Solver::galerkin_symbolic(int l) {
  Level &L = *lev[l];
  Level &C = *lev[l + 1];
  const int64_t na = L.n_agg;
  BigRows big;
  gal_count_rows(l, big);
  C.n = na;
  C.rowptr.alloc(na + 1);
  scan_exclusive_i64(ltmp.p, C.rowptr.p, na, scan_tmp, st);
  DevBuf<int64_t> eoff;
  eoff.alloc(na + 1);
  scan_exclusive_i64(ltmp2.p, eoff.p, na, scan_tmp, st);
  C.nnz = read_dev(C.rowptr.p + na, st, pinned);
  int64_t nlist = read_dev(eoff.p + na, st, pinned);
  MG_REQUIRE(nlist < (int64_t)INT32_MAX * 2, MGPBD_E_SETUP, "Galerkin list too long");
  C.col.alloc(C.nnz);
  C.crow.alloc(C.nnz);
  C.mirror.alloc(C.nnz);
  L.gl_ptr.alloc(C.nnz + 1);
  L.gl_idx.alloc(std::max<int64_t>(nlist, 1));
  L.gl_row.alloc(std::max<int64_t>(nlist, 1));
  reset_flags();
  gal_fill_rows(l, big, C.rowptr.p, eoff.p, C.col.p, C.crow.p);
  MG_HIP(hipMemcpyAsync(L.gl_ptr.p + C.nnz, eoff.p + na, sizeof(int64_t),
                        hipMemcpyDeviceToDevice, st));
  launch_gal_mirror(C.nnz, C.crow.p, C.col.p, C.rowptr.p, C.mirror.p, flags.p + kFMirror, st);
  int *h = static_cast<int *>(pinned);
  MG_HIP(hipMemcpyAsync(h, flags.p, sizeof(int) * kNumFlags, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  MG_REQUIRE(h[kFMirror] == 0, MGPBD_E_SETUP, "coarse pattern is not symmetric");
  C.val.alloc(C.nnz);
  if (mixed()) C.val32.alloc(C.nnz);
}

// K > 1: modified Gram-Schmidt QR of every aggregate's candidates (member
// slots, Q, kq, coff) and the next level's candidates from R. Returns the
// number of coarse unknowns.
int64_t Solver::qr_level(int l) {
  Level &L = *lev[l];
  Level &C = *lev[l + 1];
  const int K = opt.n_cand;
  const int64_t na = L.n_agg;
  L.K = K;
  L.slot.alloc(std::max<int64_t>(L.n, 1));
  launch_fill_i32(L.n, -1, L.slot.p, st);
  launch_member_slots(L.nmem, L.agg_mem.p, L.slot.p, st);
  L.Q.alloc(std::max<int64_t>(L.nmem * K, 1));
  L.kq.alloc(std::max<int64_t>(na, 1));
  DevBuf<double> R;
  R.alloc(std::max<int64_t>(na * K * K, 1));
  launch_qr_agg(na, K, L.agg_ptr.p, L.agg_mem.p, L.B.p, L.Q.p, R.p, L.kq.p, st);
  L.coff.alloc(na + 1);
  scan_exclusive_i32_to_i64(L.kq.p, L.coff.p, na, scan_tmp, st);
  const int64_t nc = read_dev(L.coff.p + na, st, pinned);
  C.B.alloc(std::max<int64_t>(nc * K, 1));
  launch_scatter_r(na, K, L.kq.p, L.coff.p, R.p, C.B.p, st);
  if (mixed()) {
    L.Q32.alloc(std::max<int64_t>(L.nmem * K, 1));
    launch_d2f(L.nmem * K, L.Q.p, L.Q32.p, nullptr, st);
  }
  MG_HIP(hipStreamSynchronize(st));
  return nc;
}

// K > 1: the aggregate-level pattern of the next level (the K = 1 symbolic
// kernels), then each aggregate entry expanded into its block of unknowns.
void Solver::galerkin_symbolic_k(int l) {
  Level &L = *lev[l];
  Level &C = *lev[l + 1];
  const int64_t na = L.n_agg;
  BigRows big;
  gal_count_rows(l, big);
  L.arp.alloc(na + 1);
  scan_exclusive_i64(ltmp.p, L.arp.p, na, scan_tmp, st);
  DevBuf<int64_t> eoff;
  eoff.alloc(na + 1);
  scan_exclusive_i64(ltmp2.p, eoff.p, na, scan_tmp, st);
  L.annz = read_dev(L.arp.p + na, st, pinned);
  const int64_t nlist = read_dev(eoff.p + na, st, pinned);
  MG_REQUIRE(nlist < (int64_t)INT32_MAX * 2, MGPBD_E_SETUP, "Galerkin list too long");
  const int64_t an = std::max<int64_t>(L.annz, 1);
  L.acol.alloc(an);
  L.acrow.alloc(an);
  L.amirror.alloc(an);
  L.gl_ptr.alloc(L.annz + 1);
  L.gl_idx.alloc(std::max<int64_t>(nlist, 1));
  L.gl_row.alloc(std::max<int64_t>(nlist, 1));
  reset_flags();
  gal_fill_rows(l, big, L.arp.p, eoff.p, L.acol.p, L.acrow.p);
  MG_HIP(hipMemcpyAsync(L.gl_ptr.p + L.annz, eoff.p + na, sizeof(int64_t),
                        hipMemcpyDeviceToDevice, st));
  launch_gal_mirror(L.annz, L.acrow.p, L.acol.p, L.arp.p, L.amirror.p, flags.p + kFMirror, st);
  int *h = static_cast<int *>(pinned);
  MG_HIP(hipMemcpyAsync(h, flags.p, sizeof(int) * kNumFlags, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  MG_REQUIRE(h[kFMirror] == 0, MGPBD_E_SETUP, "coarse pattern is not symmetric");
  // expansion into unknowns
  L.cstart.alloc(an);
  DevBuf<int64_t> rowlen, blocksz, base;
  rowlen.alloc(std::max<int64_t>(na, 1));
  blocksz.alloc(std::max<int64_t>(na, 1));
  base.alloc(na + 1);
  launch_galk_rowlen(na, L.arp.p, L.acol.p, L.kq.p, L.cstart.p, rowlen.p, blocksz.p, st);
  scan_exclusive_i64(blocksz.p, base.p, na, scan_tmp, st);
  C.n = read_dev(L.coff.p + na, st, pinned);
  C.nnz = read_dev(base.p + na, st, pinned);
  MG_REQUIRE(C.nnz < (int64_t)INT32_MAX * 4, MGPBD_E_SETUP, "coarse level too large");
  C.rowptr.alloc(C.n + 1);
  C.col.alloc(std::max<int64_t>(C.nnz, 1));
  launch_galk_pattern(na, L.kq.p, L.coff.p, L.arp.p, L.acol.p, base.p, rowlen.p, C.rowptr.p,
                      C.col.p, st);
  MG_HIP(hipMemcpyAsync(C.rowptr.p + C.n, base.p + na, sizeof(int64_t), hipMemcpyDeviceToDevice,
                        st));
  C.val.alloc(std::max<int64_t>(C.nnz, 1));
  if (mixed()) C.val32.alloc(std::max<int64_t>(C.nnz, 1));
  MG_HIP(hipStreamSynchronize(st));
}

void Solver::galerkin_numeric(int l) {
  Level &L = *lev[l];
  Level &C = *lev[l + 1];
  if (L.K > 1) {
    launch_galk_numeric(L.K, L.annz, L.acrow.p, L.acol.p, L.amirror.p, L.gl_ptr.p, L.gl_idx.p,
                        L.gl_row.p, L.col.p, L.val.p, L.slot.p, L.Q.p, L.kq.p, L.coff.p,
                        C.rowptr.p, L.cstart.p, C.val.p, mixed() ? C.val32.p : nullptr, st);
    return;
  }
  launch_gal_numeric(C.nnz, C.crow.p, C.col.p, C.mirror.p, L.gl_ptr.p, L.gl_idx.p, L.gl_row.p,
                     L.col.p, L.val.p, L.p.p, C.val.p, mixed() ? C.val32.p : nullptr, st);
}

// Every body's last level is solved by an explicit inverse when it has at
// most dense_max rows; otherwise (all rows isolated, or the level cap) the
// smoother is that body's last-level solver. A stalled coarsening that ends
// above dense_max is a setup failure.
void Solver::plan_dense() {
  int64_t ainv_off = 0, scratch_off = 0;
  for (int l = 0; l < nlev; ++l) {
    Level &L = *lev[l];
    L.jobs.clear();
    const int ns = (int)L.seg.size() - 1;
    bool any_smooth = false;
    for (int k = 0; k < ns; ++k) {
      const bool last = (l == nlev - 1) || L.terminal[k];
      if (!last) { any_smooth = true; continue; }
      const int64_t nk = L.seg[k + 1] - L.seg[k];
      if (nk == 0) continue;
      if (nk <= opt.dense_max) {
        DenseJob j;
        j.row0 = L.seg[k];
        j.n = nk;
        j.ainv = ainv_off;
        j.scratch = scratch_off;
        j.nnz0 = 0;
        const int64_t np = (nk + 15) / 16 * 16;
        ainv_off += nk * nk;
        scratch_off += 2 * np * np;
        L.jobs.push_back(j);
      } else {
        MG_REQUIRE(!stalled[L.body[k]], MGPBD_E_SETUP,
                   "coarsening stalled with " + std::to_string(nk) + " rows above dense_max");
        any_smooth = true;
      }
    }
    L.smooth_here = any_smooth;
    L.job_rows = 0;
    std::vector<int64_t> start;
    for (auto &j : L.jobs) { start.push_back(L.job_rows); L.job_rows += j.n; }
    start.push_back(L.job_rows);
    if (!L.jobs.empty()) {
      L.d_jobs.upload(L.jobs.data(), L.jobs.size(), st);
      L.d_jobstart.upload(start.data(), start.size(), st);
    }
  }
  Ainv.reserve(std::max<int64_t>(ainv_off, 1));
  dscratch.reserve(std::max<int64_t>(scratch_off, 1));
  MG_HIP(hipStreamSynchronize(st));
}

void Solver::factor_dense() {
  reset_flags();
  for (int l = 0; l < nlev; ++l) {
    Level &L = *lev[l];
    if (L.jobs.empty()) continue;
    launch_dense_factor_batch((int)L.jobs.size(), L.d_jobs.p, L.rowptr.p, L.col.p, L.val.p,
                              dscratch.p, Ainv.p, flags.p + kFChol, st);
  }
  MG_REQUIRE(read_flag(kFChol) == 0, MGPBD_E_BREAKDOWN,
             "a coarsest level is not positive definite");
}

void Solver::setup() {
  invalidate_graph();
  built = false;
  tail_l0 = 0;
  tail_nb = 0;
  while (lev.size() > 1) lev.pop_back();
  Level &F = *lev[0];
  if (F.seg.empty() || F.seg.back() != F.n) set_bodies({0, F.n});
  F.has_next = false;
  F.n_agg = 0;
  MG_REQUIRE(opt.max_levels >= 1 && opt.max_levels <= 32, MGPBD_E_INVALID_ARG,
             "max_levels must be in 1..32");
  if (mixed() && !val32_external) {
    F.val32.alloc(F.nnz);
    launch_d2f(F.nnz, F.val.p, F.val32.p, nullptr, st);
  }
  force_last.assign(nb, 0);
  stalled.assign(nb, 0);
  nlev = 1;
  for (int l = 0;; ++l) {
    Level &L = *lev[l];
    nlev = l + 1;
    const int ns = (int)L.seg.size() - 1;
    finish_level(l);
    L.has_next = false;
    L.terminal.assign(ns, 0);
    bool any = false;
    for (int k = 0; k < ns; ++k) {
      const int64_t nk = L.seg[k + 1] - L.seg[k];
      L.terminal[k] = force_last[L.body[k]] || nk <= opt.coarse_max || nlev >= opt.max_levels;
      any = any || !L.terminal[k];
    }
    if (!any) break;
    std::vector<int64_t> first = aggregate(l);
    bool cont = false;
    for (int k = 0; k < ns; ++k) {
      if (!L.terminal[k] && first[k + 1] == first[k]) L.terminal[k] = 1;  // all rows isolated
      cont = cont || !L.terminal[k];
    }
    if (!cont) break;
    if (l == 0) candidate0();
    build_members(l);
    lev.emplace_back(new Level());
    Level &C = *lev[l + 1];
    // first coarse unknown of each segment's aggregates
    std::vector<int64_t> cfirst = first;
    if (opt.n_cand > 1) {
      qr_level(l);
      std::vector<int64_t> coffh(L.n_agg + 1);
      L.coff.download(coffh.data(), L.n_agg + 1, st);
      MG_HIP(hipStreamSynchronize(st));
      for (int k = 0; k <= ns; ++k) cfirst[k] = coffh[first[k]];
      galerkin_symbolic_k(l);
    } else {
      L.p.alloc(L.n);
      if (mixed()) L.p32.alloc(L.n);
      launch_fill(L.n, 0.0, L.p.p, st);
      C.B.alloc(L.n_agg);
      launch_normalize(L.n_agg, L.agg_ptr.p, L.agg_mem.p, L.B.p, L.p.p, nullptr, C.B.p, st);
      if (mixed()) launch_d2f(L.n, L.p.p, L.p32.p, nullptr, st);
      galerkin_symbolic(l);
    }
    galerkin_numeric(l);
    L.has_next = true;
    C.seg.assign(1, 0);
    C.body.clear();
    for (int k = 0; k < ns; ++k) {
      if (L.terminal[k]) continue;
      const int64_t na_k = cfirst[k + 1] - cfirst[k];
      const int64_t nk = L.seg[k + 1] - L.seg[k];
      C.seg.push_back(C.seg.back() + na_k);
      C.body.push_back(L.body[k]);
      if ((double)na_k > 0.95 * (double)nk) force_last[L.body[k]] = stalled[L.body[k]] = 1;
    }
  }
  Level &last = *lev[nlev - 1];
  last.terminal.assign(last.seg.size() - 1, 1);
  plan_dense();
  factor_dense();
  ensure_vectors();
  plan_tail();
  sync_sell();
  built = true;
}

// matrix_free = 2: one FP64 fine-level product timed both ways on the first
// setup (the constraint-gradient operator, and the assembled values in the
// format the autotuner picked for level 0); when the assembled form is faster
// the matrix-free views are dropped, so every fine-level pass of this context
// (PCG product, smoothing, residual, in both precisions) reads the assembled
// values from then on. For a batch the choice covers the whole system.
void Solver::choose_fine_operator() {
  Level &F = *lev[0];
  launch_fill(F.n, 1.0, F.r.p, st);
  hipEvent_t a, b;
  MG_HIP(hipEventCreate(&a));
  MG_HIP(hipEventCreate(&b));
  auto timeit = [&](auto &&fn) {
    fn();   // warm
    MG_HIP(hipEventRecord(a, st));
    for (int rep = 0; rep < 3; ++rep) fn();
    MG_HIP(hipEventRecord(b, st));
    MG_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    MG_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  };
  const float t_mf = timeit([&] {
    launch_mf_gather(mf, F.r.p, nullptr, st);
    launch_mf_rows_dot(mf, F.r.p, F.t.p, nullptr, nullptr, st);
  });
  const float t_csr = timeit([&] { launch_spmv<double>(F.view(), F.r.p, F.t.p, st); });
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (t_csr < t_mf) {
    mf = MfView<double>();
    mf32 = MfView<float>();
  }
}

// The fused coarse V-cycle starts at the first level l >= 1 from which on
// every body has at most opt.vcycle_tail rows per level, provided each body
// there ends in a dense solve, the transfers are one-column (K = 1), the
// smoother is Jacobi or Chebyshev and the bodies' depth below fits the table.
void Solver::plan_tail() {
  tail_l0 = 0;
  tail_nb = 0;
  if (opt.vcycle_tail <= 0 || opt.smoother == 2 || nlev < 2) return;
  int l0 = nlev;
  for (int l = nlev - 1; l >= 1; --l) {
    const Level &L = *lev[l];
    bool small = L.K == 1 || l == nlev - 1;
    for (size_t k = 0; small && k + 1 < L.seg.size(); ++k)
      small = L.seg[k + 1] - L.seg[k] <= (int64_t)opt.vcycle_tail;
    if (!small) break;
    l0 = l;
  }
  if (l0 >= nlev || nlev - l0 > kTailMaxDepth) return;
  const Level &S = *lev[l0];
  std::vector<TailBody> tb;
  for (int s0 = 0; s0 + 1 < (int)S.seg.size(); ++s0) {
    if (S.seg[s0 + 1] == S.seg[s0]) continue;   // no rows: nothing to do
    TailBody b;
    const int body = S.body[s0];
    int seg = s0;
    for (int l = l0;; ++l) {
      const Level &L = *lev[l];
      b.row0[l - l0] = L.seg[seg];
      b.n[l - l0] = L.seg[seg + 1] - L.seg[seg];
      b.depth = l - l0 + 1;
      if (l == nlev - 1 || L.terminal[seg]) {
        const DenseJob *job = nullptr;
        for (const DenseJob &j : L.jobs)
          if (j.row0 == L.seg[seg] && j.n == b.n[l - l0]) job = &j;
        if (!job) return;   // a last level without a dense solve: keep the per-level path
        b.ainv = job->ainv;
        break;
      }
      const Level &C = *lev[l + 1];
      int next = -1;
      for (size_t k = 0; k < C.body.size(); ++k)
        if (C.body[k] == body) next = (int)k;
      if (next < 0) return;
      seg = next;
    }
    tb.push_back(b);
  }
  if (tb.empty()) return;
  std::vector<TailLevel<double>> v64;
  std::vector<TailLevel<float>> v32;
  for (int l = l0; l < nlev; ++l) {
    Level &L = *lev[l];
    TailLevel<double> d;
    d.rp = L.rowptr.p; d.col = L.col.p; d.val = L.val.p;
    d.wdinv = L.wdinv.p; d.dinv = L.dinv.p; d.cheb = L.cheb.p; d.rowseg = L.rowseg.p;
    d.G = L.tile > 0 ? 8 : L.lanes;   // the stream kernels sum rows with 8 lanes
    d.rlanes = L.rlanes;
    d.p = L.p.p; d.agg = L.agg.p; d.agg_ptr = L.agg_ptr.p; d.agg_mem = L.agg_mem.p;
    d.r = L.r.p; d.z = L.z.p; d.t = L.t.p; d.res = L.res.p; d.dir = L.dir.p;
    v64.push_back(d);
    if (mixed()) {
      TailLevel<float> f;
      f.rp = L.rowptr.p; f.col = L.col.p; f.val = L.val32.p;
      f.wdinv = L.wdinv32.p; f.dinv = L.dinv32.p; f.cheb = L.cheb32.p; f.rowseg = L.rowseg.p;
      f.G = L.tile32 > 0 ? 8 : L.lanes32;
      f.rlanes = L.rlanes;
      f.p = L.p32.p; f.agg = L.agg.p; f.agg_ptr = L.agg_ptr.p; f.agg_mem = L.agg_mem.p;
      f.r = L.r32.p; f.z = L.z32.p; f.t = L.t32.p; f.res = L.res32.p; f.dir = L.dir32.p;
      v32.push_back(f);
    }
  }
  tail_lv.upload(v64.data(), v64.size(), st);
  if (mixed()) tail_lv32.upload(v32.data(), v32.size(), st);
  tail_bodies.upload(tb.data(), tb.size(), st);
  tail_plan.pre = opt.pre_sweeps;
  tail_plan.post = opt.post_sweeps;
  tail_plan.smoother = opt.smoother;
  tail_plan.steps = std::max(1, std::max(opt.pre_sweeps, opt.post_sweeps));
  tail_plan.fuse_first = opt.smoother == 0;
  MG_HIP(hipStreamSynchronize(st));
  tail_nb = (int)tb.size();
  tail_l0 = l0;
}

void Solver::refresh() {
  MG_REQUIRE(built, MGPBD_E_STATE, "refresh without a hierarchy");
  Level &F = *lev[0];
  if (mixed() && !val32_external) launch_d2f(F.nnz, F.val.p, F.val32.p, nullptr, st);
  for (int l = 0; l + 1 < nlev; ++l) galerkin_numeric(l);
  reset_flags();
  for (int l = 0; l < nlev; ++l) {
    Level &L = *lev[l];
    launch_extract_diag(L.n, L.diagpos.p, L.val.p, L.diag.p, L.dinv.p, L.dinv32.p,
                        flags.p + kFBadDiag, st);
    launch_s_wdinv(L.tab.view(), L.d_omega.p, L.dinv.p, L.wdinv.p,
                   mixed() ? L.wdinv32.p : nullptr, st);
  }
  MG_REQUIRE(read_flag(kFBadDiag) == 0, MGPBD_E_BREAKDOWN, "non-positive diagonal entry");
  factor_dense();
  sync_sell();
}

void Solver::ensure_vectors() {
  const int64_t n = lev[0]->n;
  x.reserve(n); r.reserve(n); z.reserve(n); p.reserve(n); q.reserve(n);
  if (mixed()) zold32.reserve(n);
  ctl.reserve(nb);
  ensure_pinned(std::max<size_t>(4096, sizeof(PcgCtl) * (size_t)nb + 64));
}

// ------------------------------------------------------------ V-cycle
template <class T> struct Buf;
template <> struct Buf<double> {
  static const TailLevel<double> *tail(const Solver &S) { return S.tail_lv.p; }
  static DevBuf<double> &z(Level &L) { return L.z; }
  static DevBuf<double> &t(Level &L) { return L.t; }
  static DevBuf<double> &r(Level &L) { return L.r; }
  static DevBuf<double> &res(Level &L) { return L.res; }
  static CsrView<double> A(const Level &L) { return L.view(); }
  static const double *wdinv(const Level &L) { return L.wdinv.p; }
  static const double *dinv(const Level &L) { return L.dinv.p; }
  static const double *cheb(const Level &L) { return L.cheb.p; }
  static double *dir(Level &L) { return L.dir.p; }
  static const double *p(const Level &L) { return L.p.p; }
  static const double *Q(const Level &L) { return L.Q.p; }
};
template <> struct Buf<float> {
  static const TailLevel<float> *tail(const Solver &S) { return S.tail_lv32.p; }
  static DevBuf<float> &z(Level &L) { return L.z32; }
  static DevBuf<float> &t(Level &L) { return L.t32; }
  static DevBuf<float> &r(Level &L) { return L.r32; }
  static DevBuf<float> &res(Level &L) { return L.res32; }
  static CsrView<float> A(const Level &L) { return L.view32(); }
  static const float *wdinv(const Level &L) { return L.wdinv32.p; }
  static const float *dinv(const Level &L) { return L.dinv32.p; }
  static const float *cheb(const Level &L) { return L.cheb32.p; }
  static float *dir(Level &L) { return L.dir32.p; }
  static const float *p(const Level &L) { return L.p32.p; }
  static const float *Q(const Level &L) { return L.Q32.p; }
};

template <>
const MfView<double> *Solver::level_mf<double>(int l) const {
  return (l == 0 && mf.ok()) ? &mf : nullptr;
}
template <>
const MfView<float> *Solver::level_mf<float>(int l) const {
  return (l == 0 && mf32.ok()) ? &mf32 : nullptr;
}

// V-cycle on level l with the multicolour Gauss-Seidel smoother (Sec. 4.5):
// from z = 0, pre_sweeps forward sweeps over the colours, coarse
// correction, post_sweeps sweeps in reversed colour order. The sweeps read
// the assembled values on every level (also where the products are
// matrix-free): each colour needs the latest values of its neighbours.
template <class T>
void Solver::gs_vcycle(int l, const T *r, T *z) {
  Level &L = *lev[l];
  const int *done = done_ptr();
  const CsrView<T> A = Buf<T>::A(L);
  const T *dv = Buf<T>::dinv(L);
  auto sweep = [&](bool backward) {
    for (int q = 0; q < L.n_colors; ++q) {
      const int c = backward ? L.n_colors - 1 - q : q;
      launch_gs_rhs<T>(L.color_off[c + 1] - L.color_off[c], L.color_rows.p + L.color_off[c], A,
                       dv, r, z, done, st);
    }
  };
  pmark(l, 0);
  launch_zero_t<T>(L.n, z, done, st);
  for (int k = 0; k < opt.pre_sweeps; ++k) sweep(false);
  if (l + 1 < nlev) {
    Level &C = *lev[l + 1];
    T *rc = Buf<T>::r(C).p, *ec = Buf<T>::z(C).p;
    const T *pl = Buf<T>::p(L);
    T *res = Buf<T>::res(L).p;
    if (const MfView<T> *M = level_mf<T>(l)) launch_mf_residual<T>(*M, r, z, res, done, st);
    else launch_residual<T>(A, r, z, res, done, st);
    (void)pl;
    restrict_to<T>(l, res, rc);
    pmark(l, 1);
    vcycle<T>(l + 1, rc, ec);
    pmark(l, 2);
    prolong_from<T>(l, ec, z);
  } else {
    pmark(l, 1);
    pmark(l, 2);
  }
  for (int k = 0; k < opt.post_sweeps; ++k) sweep(true);
  if (!L.jobs.empty())
    launch_dense_apply_batch<T>((int)L.jobs.size(), L.d_jobs.p, L.job_rows, L.d_jobstart.p,
                                Ainv.p, r, z, done, st);
  pmark(l, 3);
}

// transfers between level l and l + 1: P^T (restriction) and P (prolongation
// added to z); one value per row, or the Q blocks when K > 1
template <class T>
void Solver::restrict_to(int l, const T *res, T *rc, CoarseFirst<T> first) {
  Level &L = *lev[l];
  Level &C = *lev[l + 1];
  if (L.K > 1)
    launch_restrict_k<T>(L.n_agg, L.K, L.kq.p, L.coff.p, L.agg_ptr.p, L.agg_mem.p, Buf<T>::Q(L),
                         res, rc, done_ptr(), st);
  else
    launch_restrict<T>(C.n, L.agg_ptr.p, L.agg_mem.p, Buf<T>::p(L), res, rc, L.rlanes,
                       done_ptr(), st, first);
}

// The restriction into level l (one candidate) also writes that level's first
// Jacobi sweep from zero, omega D^-1 r, when vcycle(l) would start with it:
// Jacobi smoother, at least one pre-sweep, a level that smooths, outside the
// fused tail and the fused residual-restriction pass. On an assembled level
// this replaces the pass that forms the first two sweeps together (whose
// gather reads r and omega D^-1 for every entry): the second sweep then
// gathers the stored iterate like every later one. Same values either way.
bool Solver::first_from_restriction(int l) const {
  if (l < 1 || l >= nlev) return false;
  if (tail_l0 > 0 && l >= tail_l0) return false;
  return lev[l]->smooth_here && lev[l - 1]->K == 1 && opt.smoother == 0 &&
         opt.pre_sweeps >= 1 && !opt.fuse_transfers;
}
template <class T>
void Solver::prolong_from(int l, const T *ec, T *z) {
  Level &L = *lev[l];
  if (L.K > 1)
    launch_prolong_k<T>(L.n, L.K, L.agg.p, L.slot.p, L.kq.p, L.coff.p, Buf<T>::Q(L), ec, z,
                        done_ptr(), st);
  else
    launch_prolong<T>(L.n, L.agg.p, Buf<T>::p(L), ec, z, done_ptr(), st);
}

template <class T>
void Solver::vcycle(int l, const T *r, T *z) {
  Level &L = *lev[l];
  const int *done = done_ptr();
  if (tail_l0 > 0 && l == tail_l0) {   // every coarser level in one launch
    pmark(l, 0);
    launch_vcycle_tail<T>(tail_nb, Buf<T>::tail(*this), tail_bodies.p, tail_plan, Ainv.p, done,
                          st);
    pmark(l, 1);
    pmark(l, 2);
    pmark(l, 3);
    return;
  }
  if (!L.smooth_here) {   // every body on this level ends with a dense solve
    pmark(l, 0);
    launch_dense_apply_batch<T>((int)L.jobs.size(), L.d_jobs.p, L.job_rows, L.d_jobstart.p,
                                Ainv.p, r, z, done, st);
    pmark(l, 1);
    pmark(l, 2);
    pmark(l, 3);
    return;
  }
  const int pre = opt.pre_sweeps, post = opt.post_sweeps;
  const bool coarse = l + 1 < nlev;
  const MfView<T> *M = level_mf<T>(l);
  const CsrView<T> A = Buf<T>::A(L);
  const T *wd = Buf<T>::wdinv(L);
  // The first Jacobi sweep from zero, z1 = omega D^-1 r, comes from the pass
  // that produced r where it can: the restriction into a coarse level, the
  // PCG update on a matrix-free fine level (first_ready). An assembled fine
  // level forms the first two sweeps in one pass with z1 computed on the fly;
  // otherwise z1 is an elementwise pass of its own.
  const bool from_restriction = first_from_restriction(l);
  const bool fuse = (M == nullptr) && opt.smoother == 0 && !from_restriction;
  const bool cheb = opt.smoother == 1;
  const int steps = std::max(1, std::max(pre, post));
  // The iterate ping-pongs between z and the level's scratch vector; the
  // first target is chosen so that the last write lands in z.
  const int pre_writes = pre == 0 ? 1 : (fuse && pre >= 2) ? pre - 1 : pre;
  const int writes = pre_writes + post;
  T *bufs[2] = {z, Buf<T>::t(L).p};
  int w = (writes % 2) ? 0 : 1;
  auto next = [&]() { return bufs[(w++) % 2]; };
  // sweep k of a smoothing pass: a Jacobi sweep or Chebyshev step k
  auto sweep = [&](int k, const T *zi, T *zo) {
    if (cheb) {
      const T *dv = Buf<T>::dinv(L), *cf = Buf<T>::cheb(L);
      T *d = Buf<T>::dir(L);
      if (M) launch_mf_cheb<T>(*M, r, dv, cf, L.rowseg.p, steps, k, zi, d, zo, done, st);
      else launch_cheb<T>(A, r, dv, cf, L.rowseg.p, steps, k, zi, d, zo, done, st);
    } else if (M) {
      launch_mf_jacobi<T>(*M, wd, r, zi, zo, done, st);
    } else {
      launch_jacobi<T>(A, wd, r, zi, zo, done, st);
    }
  };
  if (opt.smoother == 2) {   // Gauss-Seidel: in place on z
    gs_vcycle<T>(l, r, z);
    return;
  }
  pmark(l, 0);
  T *cur = next();
  int k0 = 1;
  if (pre == 0) {
    launch_zero_t<T>(L.n, cur, done, st);
  } else if (cheb) {
    launch_cheb_first<T>(L.n, r, Buf<T>::dinv(L), Buf<T>::cheb(L), L.rowseg.p, steps,
                         Buf<T>::dir(L), cur, done, st);
  } else if (from_restriction) {
    // the restriction into this level wrote omega D^-1 r into cur
  } else if (fuse && pre >= 2) {
    launch_jacobi_scaled<T>(A, wd, r, cur, done, st);
    k0 = 2;
  } else if (l == 0 && first_ready) {
    first_ready = false;   // the PCG update wrote omega D^-1 r into cur
  } else {
    launch_jacobi_first<T>(L.n, wd, r, cur, done, st);
  }
  for (int k = k0; k < pre; ++k) {
    T *o = next();
    sweep(k, cur, o);
    cur = o;
  }
  // With fuse_transfers (off by default: measured slower) and a one-column
  // transfer (K = 1): on assembled levels the residual and the restriction
  // are one pass, and on every level the prolongation is folded into the
  // first post-sweep, which reads z + P e through its input functor instead
  // of a stored z.
  const bool fold = coarse && opt.fuse_transfers && L.K == 1 && post > 0;
  const T *ec_fold = nullptr;
  if (coarse) {
    Level &C = *lev[l + 1];
    T *rc = Buf<T>::r(C).p, *ec = Buf<T>::z(C).p;
    const T *pl = Buf<T>::p(L);
    T *res = Buf<T>::res(L).p;
    // the coarse level's first iterate goes where its vcycle() starts writing
    // (the buffer whose parity leaves the last write in ec)
    CoarseFirst<T> cf;
    if (first_from_restriction(l + 1)) {
      cf.wd = Buf<T>::wdinv(C);
      cf.z = ((pre + post) % 2) ? ec : Buf<T>::t(C).p;
    }
    if (!M && opt.fuse_transfers && L.K == 1) {
      launch_residual_restrict<T>(A, r, cur, C.n, L.agg_ptr.p, L.agg_mem.p, pl, rc, done, st);
    } else if (M && L.K == 1) {
      // the matrix-free residual stores the restriction's terms p_i res_i in
      // row order (coalesced), so the restriction gathers one scattered value
      // per member instead of two; the terms and their order are unchanged
      launch_mf_residual_scaled<T>(*M, r, cur, pl, res, done, st);
      launch_restrict_sum<T>(C.n, L.agg_ptr.p, L.agg_mem.p, res, rc, L.rlanes, done, st, cf);
    } else {
      if (M) launch_mf_residual<T>(*M, r, cur, res, done, st);
      else launch_residual<T>(A, r, cur, res, done, st);
      restrict_to<T>(l, res, rc, cf);
    }
    pmark(l, 1);
    vcycle<T>(l + 1, rc, ec);
    pmark(l, 2);
    if (fold) ec_fold = ec;
    else prolong_from<T>(l, ec, cur);
  } else {
    pmark(l, 1);
    pmark(l, 2);
  }
  for (int k = 0; k < post; ++k) {
    T *o = next();
    if (k == 0 && fold) {
      const T *pl = Buf<T>::p(L);
      if (cheb) {
        const T *dv = Buf<T>::dinv(L), *cf = Buf<T>::cheb(L);
        T *d = Buf<T>::dir(L);
        if (M)
          launch_mf_cheb_prolong<T>(*M, r, dv, cf, L.rowseg.p, steps, 0, cur, pl, L.agg.p,
                                    ec_fold, d, o, done, st);
        else
          launch_cheb_prolong<T>(A, r, dv, cf, L.rowseg.p, steps, 0, cur, pl, L.agg.p, ec_fold,
                                 d, o, done, st);
      } else if (M) {
        launch_mf_jacobi_prolong<T>(*M, wd, r, cur, pl, L.agg.p, ec_fold, o, done, st);
      } else {
        launch_jacobi_prolong<T>(A, wd, r, cur, pl, L.agg.p, ec_fold, o, done, st);
      }
    } else {
      sweep(k, cur, o);
    }
    cur = o;
  }
  if (cur != z) launch_copy_t<T>(L.n, cur, z, done, st);   // not reached: w makes cur == z
  // bodies that end here with a dense solve: their rows are that solve's
  if (!L.jobs.empty())
    launch_dense_apply_batch<T>((int)L.jobs.size(), L.d_jobs.p, L.job_rows, L.d_jobstart.p,
                                Ainv.p, r, z, done, st);
  pmark(l, 3);
}

// ------------------------------------------------------------ PCG
// Where the PCG update can write the V-cycle's first fine-level step: the
// FP32 residual of the mixed cycle always, and the first Jacobi iterate
// omega D^-1 r when vcycle(0) would form it elementwise (Jacobi smoother,
// matrix-free fine level, at least one pre-sweep), into the buffer vcycle's
// ping-pong picks for it (the last write of the level lands in z).
FirstSweep Solver::first_sweep_targets() {
  FirstSweep f;
  Level &F = *lev[0];
  const bool flex = mixed();
  f.cycle_done = done_ptr();
  if (flex) f.r32 = F.r32.p;
  const bool mf0 = flex ? mf32.ok() : mf.ok();
  if (!(F.smooth_here && opt.smoother == 0 && opt.pre_sweeps >= 1 && mf0)) return f;
  const int writes = opt.pre_sweeps + opt.post_sweeps;
  const bool into_z = (writes % 2) != 0;
  if (flex) {
    f.wd32 = F.wdinv32.p;
    f.z32 = into_z ? F.z32.p : F.t32.p;
  } else {
    f.wd64 = F.wdinv.p;
    f.z64 = into_z ? z.p : F.t.p;
  }
  return f;
}

void Solver::iterate_once(int k) {
  Level &F = *lev[0];
  const int64_t n = F.n;
  const bool flex = mixed();
  SegTab t = F.tab.view();
  // profiling: events before the product, after its first kernel (the
  // matrix-free gather) and after its last kernel (before the dot finisher)
  auto mark = [&](int j) {
    if (opt.profile_spmv) MG_HIP(hipEventRecord(ev[3 * k + j], st));
  };
  mark(0);
  if (nb == 1) {   // q = A p fused with the partial sums of p^T q
    int grid;
    if (mf.ok()) {
      launch_mf_gather(mf, p.p, done_ptr(), st);
      mark(1);
      grid = launch_mf_rows_dot(mf, p.p, q.p, done_ptr(), partials(), st);
    } else {
      mark(1);
      grid = launch_spmv_dot_partials(F.view(), p.p, q.p, done_ptr(), partials(), st);
    }
    mark(2);
    launch_fin_pq(ctl.p, partials(), grid, st);
  } else {
    if (mf.ok()) {
      launch_mf_gather(mf, p.p, done_ptr(), st);
      mark(1);
      launch_mf_rows_dot(mf, p.p, q.p, done_ptr(), nullptr, st);
    } else {
      mark(1);
      launch_spmv<double>(F.view(), p.p, q.p, st);
    }
    mark(2);
  }
  if (nb > 1) launch_s_pcg_dot_pq(t, ctl.p, p.p, q.p, partials(), st);
  const FirstSweep fs = first_sweep_targets();
  launch_s_pcg_update(t, ctl.p, p.p, q.p, x.p, r.p, partials(), all_done.p, st, fs);
  first_ready = fs.z32 != nullptr || fs.z64 != nullptr;
  prof_k = opt.profile_spmv ? k : -1;
  if (flex) {
    if (!fs.r32) launch_d2f(n, r.p, F.r32.p, done_ptr(), st);
    vcycle<float>(0, F.r32.p, F.z32.p);
    launch_s_pcg_rz(t, ctl.p, r.p, nullptr, F.z32.p, zold32.p, partials(), st);
  } else {
    vcycle<double>(0, r.p, z.p);
    launch_s_pcg_rz(t, ctl.p, r.p, z.p, nullptr, nullptr, partials(), st);
  }
  prof_k = -1;
  first_ready = false;
  launch_s_pcg_pupdate(t, ctl.p, z.p, flex ? F.z32.p : nullptr, p.p, st);
}

void Solver::apply_fine(const double *x, double *y) {
  Level &F = *lev[0];
  MG_REQUIRE(F.n > 0 && F.val.p, MGPBD_E_STATE, "no assembled matrix");
  ensure_partials(F.tab.view().nblk);
  if (mf.ok()) {
    launch_mf_gather(mf, x, nullptr, st);
    launch_mf_rows_dot(mf, x, y, nullptr, partials(), st);
  } else {
    launch_spmv_dot_partials(F.view(), x, y, nullptr, partials(), st);
  }
}

void Solver::apply_fine_into(const double *x, double *y, double *u) {
  Level &F = *lev[0];
  MG_REQUIRE(F.n > 0 && F.val.p, MGPBD_E_STATE, "no assembled matrix");
  if (mf.ok()) {
    MfView<double> v = mf;
    v.u = u;
    launch_mf_gather(v, x, nullptr, st);
    launch_mf_rows_dot(v, x, y, nullptr, nullptr, st);
  } else {
    launch_spmv_dot_partials(F.view(), x, y, nullptr, nullptr, st);
  }
}

std::vector<PcgResult> Solver::pcg(const double *b, double *x_out, double tol, int max_iters,
                                   const int32_t *force) {
  MG_REQUIRE(built, MGPBD_E_STATE, "solve without a hierarchy");
  Level &F = *lev[0];
  const int64_t n = F.n;
  ensure_vectors();
  SegTab t = F.tab.view();
  ensure_partials(t.nblk);
  PcgCtl *hp = static_cast<PcgCtl *>(pinned);
  for (int k = 0; k < nb; ++k) {
    PcgCtl h{};
    h.done = 0;
    h.iters = 0;
    h.force = force ? force[k] : 0;
    h.max_iters = max_iters;
    h.tol = tol;
    hp[k] = h;
  }
  MG_HIP(hipMemcpyAsync(ctl.p, hp, sizeof(PcgCtl) * nb, hipMemcpyHostToDevice, st));
  launch_s_pcg_init(t, ctl.p, b, x.p, r.p, partials(), all_done.p, st);
  if (mixed()) {
    launch_d2f(n, r.p, F.r32.p, done_ptr(), st);
    vcycle<float>(0, F.r32.p, F.z32.p);
    launch_s_pcg_init_p(t, ctl.p, r.p, nullptr, F.z32.p, p.p, zold32.p, partials(), all_done.p,
                        st);
  } else {
    vcycle<double>(0, r.p, z.p);
    launch_s_pcg_init_p(t, ctl.p, r.p, z.p, nullptr, p.p, nullptr, partials(), all_done.p, st);
  }
  const int chunk = std::max(1, opt.check_every);
  // events around the fine-level product are recorded on the stream, so the
  // profiled solve launches kernels directly instead of replaying the graph
  const bool use_graph = opt.use_graph && !opt.profile_spmv && st != nullptr;
  if (opt.profile_spmv && (int)ev.size() < 3 * chunk) {
    invalidate_graph();
    for (auto e : ev) (void)hipEventDestroy(e);
    ev.assign(3 * chunk, nullptr);
    for (auto &e : ev) MG_HIP(hipEventCreate(&e));
    for (auto e : lev_ev) (void)hipEventDestroy(e);
    lev_ev.assign((size_t)chunk * kProfLevels * 4, nullptr);
    for (auto &e : lev_ev) MG_HIP(hipEventCreate(&e));
  }
  if (use_graph && !graph_ok) {
    invalidate_graph();
    MG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      for (int k = 0; k < chunk; ++k) iterate_once(k);
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(st, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    MG_HIP(hipStreamEndCapture(st, &graph));
    MG_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    graph_ok = true;
  }
  auto max_iters_done = [&]() {
    int m = 0;
    for (int k = 0; k < nb; ++k) m = std::max(m, hp[k].iters + (hp[k].done == 2 ? 1 : 0));
    return m;
  };
  int launched = 0;
  while (true) {
    // the control blocks tell whether every solve already ended
    MG_HIP(hipMemcpyAsync(hp, ctl.p, sizeof(PcgCtl) * nb, hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    bool ended = true;
    for (int k = 0; k < nb; ++k) ended = ended && hp[k].done != 0;
    if (ended || launched >= max_iters) break;
    const int before = max_iters_done();
    if (use_graph) {
      MG_HIP(hipGraphLaunch(gexec, st));
    } else {
      for (int k = 0; k < chunk; ++k) iterate_once(k);
    }
    launched += chunk;
    if (opt.profile_spmv) {
      MG_HIP(hipMemcpyAsync(hp, ctl.p, sizeof(PcgCtl) * nb, hipMemcpyDeviceToHost, st));
      MG_HIP(hipStreamSynchronize(st));
      const int ran = std::min(chunk, max_iters_done() - before);
      for (int k = 0; k < ran; ++k) {
        float ms = 0.f, ms1 = 0.f;
        MG_HIP(hipEventElapsedTime(&ms, ev[3 * k], ev[3 * k + 2]));
        MG_HIP(hipEventElapsedTime(&ms1, ev[3 * k], ev[3 * k + 1]));
        spmv_ms += ms;
        spmv_first_ms += ms1;
        ++spmv_calls;
        // levels below the start of the fused tail record no events of their own
        const int visited = tail_l0 > 0 ? tail_l0 + 1 : nlev;
        for (int l = 0; l < std::min(visited, (int)kProfLevels); ++l) {
          hipEvent_t *e = &lev_ev[((size_t)k * kProfLevels + l) * 4];
          float a = 0.f, b = 0.f;
          MG_HIP(hipEventElapsedTime(&a, e[0], e[1]));
          MG_HIP(hipEventElapsedTime(&b, e[2], e[3]));
          level_ms[l] += a + b;
        }
        ++vcycles;
      }
    }
  }
  if (x_out != x.p) launch_copy(n, x.p, x_out, nullptr, st);
  std::vector<PcgResult> res(nb);
  for (int k = 0; k < nb; ++k) {
    res[k].status = hp[k].done ? hp[k].done : 4;
    res[k].iters = hp[k].iters;
    res[k].ratio = hp[k].ratio;
    res[k].bnorm = hp[k].bnorm;
  }
  return res;
}

template void Solver::vcycle<double>(int, const double *, double *);
template void Solver::vcycle<float>(int, const float *, float *);

}  // namespace mgpbd
