// C ABI (include/mgpbd.h): simulation contexts running Algorithm 1 on one
// GPU, the standalone solver entry, inspection hooks, and batching.
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>

#include "solver.hpp"
#include "xpbd.hpp"

using namespace mgpbd;

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() { MG_HIP(hipEventCreate(&a)); MG_HIP(hipEventCreate(&b)); }
  ~Timer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  void start(hipStream_t s) { MG_HIP(hipEventRecord(a, s)); }
  double stop(hipStream_t s) {
    MG_HIP(hipEventRecord(b, s));
    MG_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    MG_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
};

// Events recorded around the phases of a frame and read once after the
// frame's last synchronisation (no extra host round trip per phase); the
// pool grows to the largest frame and is reused.
struct PhaseEvents {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  ~PhaseEvents() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  void reset() { used = 0; }
  size_t mark(hipStream_t s) {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      MG_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    MG_HIP(hipEventRecord(pool[used], s));
    return used++;
  }
  double ms(size_t a, size_t b) const {
    float v = 0.f;
    MG_HIP(hipEventElapsedTime(&v, pool[a], pool[b]));
    return v;
  }
};

struct mgpbd_ctx {
  std::string err;
  mgpbd_options opt;
  int device = -1;                 // the HIP device current at creation
  PhaseEvents phase;               // assembly and update timers of the frame
  hipStream_t own = nullptr;
  hipStream_t st = nullptr;
  std::unique_ptr<Solver> solver;
  // bodies (none for solver-only contexts; several for the system of a batch)
  bool has_body = false;
  int nb = 1;
  int64_t nv = 0, m = 0, nnz = 0;
  std::vector<int64_t> voff{0, 0}, roff{0, 0};   // first vertex / row of each body
  double dt = 0.0, g[3] = {0, 0, 0};
  int64_t frame = 0;
  bool stale = true;
  DevBuf<int32_t> rv;
  DevBuf<uint32_t> meta;
  DevBuf<int64_t> vptr;
  DevBuf<int32_t> vrow;
  DevBuf<int8_t> vslot;
  DevBuf<double> w, alpha_t, rest_c, C, grad, lambda, b, old[3], vold[3];
  DevBuf<int> bad;
  // ARAP rows (absent without them): kind[r] = 1 marks one, dm_inv[r] holds
  // the inverse rest shape matrix of its tet
  bool has_arap = false;
  DevBuf<int8_t> kind;
  DevBuf<double> dm_inv;
  // matrix-free fine operator: positions of the current iteration, the
  // per-incidence gradients and the gather scratch (FP64; FP32 copies for the
  // mixed V-cycle)
  DevBuf<double> mf_pos, mf_gT, mf_u;
  DevBuf<float> mf_pos32, mf_gT32, mf_u32, mf_alpha32, mf_w32, mf_g32;
  std::vector<int32_t> force;
  bool have_rhs = false;
  bool batch_owned = false;   // the system context of a batch (freed with it)
};

// A batch owns a system context whose arrays are its bodies' arrays back to
// back (vertex, row and entry indices shifted by each body's offsets).
struct mgpbd_batch {
  std::vector<mgpbd_ctx *> ctxs;
  mgpbd_ctx sys;
  DevBuf<double> pos[3], vel[3];
};

// Scratch of mgpbd_apply_noalloc: the matrix-free vertex gather's u[nv][4]
// (FP64) for callers that cannot allocate. Each GPU holds one copy until the
// process ends, shared by every call on that GPU. In host code `scratch` is
// only a stand-in for the device array: its device address on each GPU comes
// from hipGetSymbolAddress (scratch_addr) and only that address is handed to
// kernels.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Look up this device's copy of `scratch` once (the device must be current).
void scratch_setup(int dev) {
  MG_REQUIRE(dev >= 0 && dev < kMaxDevices, MGPBD_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[dev]) return;
  void *p = nullptr;
  MG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  MG_REQUIRE(p != nullptr, MGPBD_E_DEVICE, "no device address for the scratch array");
  g_scratch_addr[dev] = p;
}

void *scratch_addr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return dev >= 0 && dev < kMaxDevices ? g_scratch_addr[dev] : nullptr;
}

mgpbd_status fail(mgpbd_ctx *c, const Error &e) {
  if (c) c->err = e.what();
  return (mgpbd_status)e.status;
}

// Runs f and turns its exceptions into a status. A failed HIP call also
// leaves the runtime's per-thread last error set; it is cleared here so that
// it cannot surface later in the caller's own, unrelated HIP calls.
template <class F>
mgpbd_status guard(mgpbd_ctx *c, F f) {
  try {
    f();
    if (c) c->err.clear();
    return MGPBD_OK;
  } catch (const Error &e) {
    (void)hipGetLastError();
    return fail(c, e);
  } catch (const std::bad_alloc &) {
    (void)hipGetLastError();
    if (c) c->err = "host allocation failed";
    return MGPBD_E_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
    (void)hipGetLastError();
    if (c) c->err = e.what();
    return MGPBD_E_DEVICE;
  }
}

void check_options(const mgpbd_options &o) {
  MG_REQUIRE(o.theta >= 0.0 && std::isfinite(o.theta), MGPBD_E_INVALID_ARG, "theta");
  MG_REQUIRE(o.gs_sweeps >= 0 && o.pre_sweeps >= 0 && o.post_sweeps >= 0, MGPBD_E_INVALID_ARG,
             "sweep counts must be >= 0");
  MG_REQUIRE(o.pre_sweeps == o.post_sweeps, MGPBD_E_INVALID_ARG,
             "pre and post sweeps must match (symmetric V-cycle)");
  MG_REQUIRE(o.coarse_max >= 0 && o.dense_max >= 0 && o.dense_max <= 8192, MGPBD_E_INVALID_ARG,
             "coarse_max / dense_max");
  MG_REQUIRE(o.max_levels >= 1 && o.max_levels <= 32, MGPBD_E_INVALID_ARG, "max_levels");
  MG_REQUIRE(o.power_iters >= 0 && o.power_max >= 0 && o.max_pcg >= 1 && o.check_every >= 1,
             MGPBD_E_INVALID_ARG, "iteration counts");
  MG_REQUIRE(o.power_tol >= 0.0 && std::isfinite(o.power_tol), MGPBD_E_INVALID_ARG, "power_tol");
  MG_REQUIRE(o.vcycle_tail >= 0, MGPBD_E_INVALID_ARG, "vcycle_tail");
  MG_REQUIRE(o.fuse_transfers == 0 || o.fuse_transfers == 1, MGPBD_E_INVALID_ARG,
             "fuse_transfers must be 0 or 1");
  MG_REQUIRE(o.resetup_on_breakdown == 0 || o.resetup_on_breakdown == 1, MGPBD_E_INVALID_ARG,
             "resetup_on_breakdown must be 0 or 1");
  MG_REQUIRE(o.tol >= 0.0 && o.lmax_scale > 0.0, MGPBD_E_INVALID_ARG, "tol / lmax_scale");
  MG_REQUIRE(o.precision == MGPBD_PREC_FP64 || o.precision == MGPBD_PREC_MIXED,
             MGPBD_E_INVALID_ARG, "precision");
  MG_REQUIRE(o.reuse_interval >= 0, MGPBD_E_INVALID_ARG, "reuse_interval");
  MG_REQUIRE(o.spmv_tile == 0 || o.spmv_tile == -1 || o.spmv_tile == -2 ||
                 o.spmv_tile == 1024 || o.spmv_tile == 2048 || o.spmv_tile == 4096,
             MGPBD_E_INVALID_ARG, "spmv_tile must be 0, -1, -2, 1024, 2048 or 4096");
  MG_REQUIRE(o.spmv_lanes == 0 || o.spmv_lanes == 4 || o.spmv_lanes == 8 || o.spmv_lanes == 16 ||
                 o.spmv_lanes == 32 || o.spmv_lanes == 64,
             MGPBD_E_INVALID_ARG, "spmv_lanes must be 0, 4, 8, 16, 32 or 64");
  MG_REQUIRE(o.matrix_free >= 0 && o.matrix_free <= 2, MGPBD_E_INVALID_ARG,
             "matrix_free must be 0, 1 or 2");
  MG_REQUIRE(o.smoother >= 0 && o.smoother <= 2, MGPBD_E_INVALID_ARG,
             "smoother must be 0 (omega-Jacobi), 1 (Chebyshev) or 2 (Gauss-Seidel)");
  MG_REQUIRE(o.n_cand >= 1 && o.n_cand <= 8, MGPBD_E_INVALID_ARG, "n_cand must be in 1..8");
}

void init_ctx(mgpbd_ctx *c, const mgpbd_options *opt) {
  if (opt) c->opt = *opt; else mgpbd_default_options(&c->opt);
  check_options(c->opt);
  MG_HIP(hipGetDevice(&c->device));
  scratch_setup(c->device);
  MG_HIP(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
  c->st = c->own;
  c->solver.reset(new Solver(c->opt));
  c->solver->set_stream(c->st);
}

// per-iteration arrays of a context whose pattern (F.rowptr/col, rv, ...) is set
void alloc_state(mgpbd_ctx *c) {
  Solver &S = *c->solver;
  Level &F = S.L0();
  F.n = c->m;
  F.nnz = c->nnz;
  F.val.alloc(c->nnz);
  if (c->opt.precision == MGPBD_PREC_MIXED) {
    F.val32.alloc(c->nnz);
    S.val32_external = true;
  }
  S.pattern_dirty = true;
  S.set_bodies(c->roff);
  c->C.alloc(c->m);
  c->grad.alloc(12 * (size_t)c->m);
  c->lambda.alloc(c->m);
  c->b.alloc(c->m);
  c->bad.alloc(1);
  for (int k = 0; k < 3; ++k) {
    c->old[k].alloc(c->nv);
    c->vold[k].alloc(c->nv);
  }
  S.mf = MfView<double>();
  S.mf32 = MfView<float>();
  if (c->opt.matrix_free && c->m > 0) {
    const size_t nv4 = 4 * (size_t)std::max<int64_t>(c->nv, 1);
    const size_t ninc3 = 3 * (size_t)std::max<int64_t>((int64_t)c->vrow.n, 1);
    c->mf_pos.alloc(nv4);
    c->mf_gT.alloc(ninc3);
    c->mf_u.alloc(nv4);
    MfView<double> v;
    v.m = c->m; v.nv = c->nv; v.rv = c->rv.p; v.pos = c->mf_pos.p; v.alpha = c->alpha_t.p;
    v.vptr = c->vptr.p; v.vrow = c->vrow.p; v.gT = c->mf_gT.p; v.w = c->w.p;
    v.u = c->mf_u.p;
    if (c->has_arap) {
      v.kind = c->kind.p;
      v.gst = c->grad.p;
    }
    S.mf = v;
    if (S.mixed()) {
      c->mf_pos32.alloc(nv4);
      c->mf_gT32.alloc(4 * (size_t)std::max<int64_t>((int64_t)c->vrow.n, 1));
      c->mf_u32.alloc(nv4);
      c->mf_alpha32.alloc(c->m);
      c->mf_w32.alloc(std::max<int64_t>(c->nv, 1));
      launch_d2f(c->m, c->alpha_t.p, c->mf_alpha32.p, nullptr, c->st);
      launch_d2f(c->nv, c->w.p, c->mf_w32.p, nullptr, c->st);
      MfView<float> f;
      f.m = c->m; f.nv = c->nv; f.rv = c->rv.p; f.pos = c->mf_pos32.p;
      f.alpha = c->mf_alpha32.p; f.vptr = c->vptr.p; f.vrow = c->vrow.p; f.gT = c->mf_gT32.p;
      f.w = c->mf_w32.p; f.u = c->mf_u32.p;
      if (c->has_arap) {
        c->mf_g32.alloc(12 * (size_t)c->m);
        f.kind = c->kind.p;
        f.gst = c->mf_g32.p;
      }
      S.mf32 = f;
    }
  }
}

void run_frame(mgpbd_ctx *c, double *const xyz[3], double *const vxyz[3], int n_iters,
               const std::vector<const std::vector<int32_t> *> &force,
               mgpbd_step_stats *stats);

// One frame of Algorithm 1 for every body of c. force[k] (nullable) fixes
// body k's PCG iteration counts; stats (nullable) holds one struct per body.
// A body whose |b| falls below eps_b stops: later iterations solve a zero
// right-hand side for it, which leaves its x and lambda unchanged.
void run_step(mgpbd_ctx *c, double *const xyz[3], double *const vxyz[3], int n_iters,
              const std::vector<const std::vector<int32_t> *> &force, mgpbd_step_stats *stats) {
  hipStream_t st = c->st;
  const int64_t nv = c->nv;
  MG_HIP(hipMemsetAsync(c->bad.p, 0, sizeof(int), st));
  for (int k = 0; k < 3; ++k) {
    launch_check_finite(nv, xyz[k], c->bad.p, st);
    launch_check_finite(nv, vxyz[k], c->bad.p, st);
  }
  int hbad = 0;
  MG_HIP(hipMemcpyAsync(&hbad, c->bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  MG_REQUIRE(hbad == 0, MGPBD_E_INVALID_ARG, "non-finite positions or velocities");
  // the velocities entering the frame, so that a failed frame can hand the
  // caller back its own state (the positions are kept by the predict)
  for (int k = 0; k < 3; ++k)
    if (nv)
      MG_HIP(hipMemcpyAsync(c->vold[k].p, vxyz[k], sizeof(double) * nv, hipMemcpyDeviceToDevice,
                            st));
  try {
    run_frame(c, xyz, vxyz, n_iters, force, stats);
  } catch (...) {
    // an error inside the frame (breakdown, failed setup, device error):
    // restore x and v as they entered, drop the partial frame and make the
    // next step rebuild the hierarchy
    for (int k = 0; k < 3; ++k)
      if (nv) {
        (void)hipMemcpyAsync(xyz[k], c->old[k].p, sizeof(double) * nv, hipMemcpyDeviceToDevice,
                             st);
        (void)hipMemcpyAsync(vxyz[k], c->vold[k].p, sizeof(double) * nv,
                             hipMemcpyDeviceToDevice, st);
      }
    (void)hipStreamSynchronize(st);
    c->stale = true;
    throw;
  }
}

// The frame itself (after the finiteness check): predict, global iterations,
// velocity. Throws on breakdown or setup failure with x and v part-updated;
// run_step restores them.
void run_frame(mgpbd_ctx *c, double *const xyz[3], double *const vxyz[3], int n_iters,
               const std::vector<const std::vector<int32_t> *> &force,
               mgpbd_step_stats *stats) {
  hipStream_t st = c->st;
  Solver &S = *c->solver;
  const int nb = c->nb;
  const int64_t nv = c->nv, m = c->m;
  double *oxyz[3] = {c->old[0].p, c->old[1].p, c->old[2].p};
  Timer total, part;
  total.start(st);
  double ms_setup = 0.0, ms_pcg = 0.0, ms_galerkin = 0.0;
  S.reset_profile();
  c->phase.reset();
  std::vector<std::pair<size_t, size_t>> asm_ev, upd_ev;
  launch_predict(nv, c->w.p, c->g, c->dt, xyz, vxyz, oxyz, st);
  if (m == 0) {
    // no constraint rows: every global iteration is empty, the frame is the
    // semi-implicit Euler step alone
    launch_velocity(nv, c->dt, xyz, oxyz, vxyz, st);
    c->frame++;
    const double ms = total.stop(st);
    if (stats)
      for (int k = 0; k < nb; ++k) {
        stats[k].iters_done = 0;
        stats[k].ms_setup = 0.0;
        stats[k].ms_pcg = 0.0;
        stats[k].ms_total = ms;
        stats[k].spmv_calls = 0;
        stats[k].spmv_ms = 0.0;
        stats[k].spmv_first_ms = 0.0;
        stats[k].ms_assembly = 0.0;
        stats[k].ms_galerkin = 0.0;
        stats[k].ms_update = 0.0;
        stats[k].vcycles = 0;
        for (double &v : stats[k].ms_level) v = 0.0;
      }
    return;
  }
  launch_fill(m, 0.0, c->lambda.p, st);
  Level &F = S.L0();
  std::vector<char> stopped(nb, 0);
  std::vector<int> iters_done(nb, 0);
  std::vector<int32_t> fv(nb, 0);
  int n_stopped = 0;
  for (int ite = 0; ite < n_iters && n_stopped < nb; ++ite) {
    const size_t a0 = c->phase.mark(st);
    const int8_t *kind = c->has_arap ? c->kind.p : nullptr;
    launch_constraints(m, c->rv.p, kind, c->rest_c.p, xyz, c->C.p, c->grad.p, st);
    if (kind) launch_arap_constraints(m, c->rv.p, kind, c->dm_inv.p, xyz, c->C.p, c->grad.p, st);
    const int64_t n_inc = (int64_t)c->vrow.n;
    if (S.mf.ok())
      launch_mf_prepare<double>(nv, xyz[0], xyz[1], xyz[2], n_inc, c->vrow.p, c->vslot.p,
                                c->grad.p, c->mf_pos.p, c->mf_gT.p, st);
    if (S.mf32.ok()) {
      launch_mf_prepare<float>(nv, xyz[0], xyz[1], xyz[2], n_inc, c->vrow.p, c->vslot.p,
                               c->grad.p, c->mf_pos32.p, c->mf_gT32.p, st);
      if (kind) launch_d2f(12 * m, c->grad.p, c->mf_g32.p, nullptr, st);
    }
    launch_assemble(m, 16, F.rowptr.p, F.col.p, c->meta.p, c->rv.p, c->w.p, c->grad.p,
                    c->alpha_t.p, c->C.p, c->lambda.p, F.val.p, S.mixed() ? F.val32.p : nullptr,
                    c->b.p, st);
    for (int k = 0; k < nb; ++k)
      if (stopped[k] && c->roff[k + 1] > c->roff[k])
        MG_HIP(hipMemsetAsync(c->b.p + c->roff[k], 0,
                              sizeof(double) * (c->roff[k + 1] - c->roff[k]), st));
    c->have_rhs = true;
    asm_ev.emplace_back(a0, c->phase.mark(st));
    std::vector<double> bn = S.norm2(c->b.p);
    for (auto &v : bn) v = std::sqrt(v);
    const int R = c->opt.reuse_interval;
    const bool due = c->stale || !S.built || R <= 0 || (ite == 0 && (c->frame % R) == 0);
    for (int k = 0; k < nb; ++k) {
      if (stopped[k] || !stats) continue;
      if (stats[k].bnorm) stats[k].bnorm[ite] = bn[k];
      if (stats[k].setup_ran) stats[k].setup_ran[ite] = due ? 1 : 0;
    }
    part.start(st);
    if (due) {
      S.setup();
      c->stale = false;
    } else {
      S.refresh();
    }
    const double ms_s = part.stop(st);
    ms_setup += ms_s;
    if (!due) ms_galerkin += ms_s;
    for (int k = 0; k < nb; ++k) {
      const std::vector<int32_t> *f = k < (int)force.size() ? force[k] : nullptr;
      fv[k] = (!stopped[k] && f && ite < (int)f->size()) ? (*f)[ite] : 0;
    }
    part.start(st);
    std::vector<PcgResult> pr = S.pcg(c->b.p, S.dl(), c->opt.tol, c->opt.max_pcg, fv.data());
    ms_pcg += part.stop(st);
    bool broke = false;
    for (int k = 0; k < nb; ++k) broke = broke || (!stopped[k] && pr[k].status == 2);
    if (broke && !due && c->opt.resetup_on_breakdown) {
      // the lazy setup keeps the hierarchy and its smoother weights while they
      // still precondition A; this A they no longer do (the V-cycle is not
      // positive definite for it): set up afresh and solve the iteration again
      for (int k = 0; k < nb; ++k)
        if (!stopped[k] && stats && stats[k].setup_ran) stats[k].setup_ran[ite] = 2;
      part.start(st);
      S.setup();
      ms_setup += part.stop(st);
      part.start(st);
      pr = S.pcg(c->b.p, S.dl(), c->opt.tol, c->opt.max_pcg, fv.data());
      ms_pcg += part.stop(st);
    }
    for (int k = 0; k < nb; ++k) {
      if (stopped[k]) continue;
      if (stats && stats[k].pcg_iters) stats[k].pcg_iters[ite] = pr[k].iters;
      if (stats && stats[k].pcg_ratio) stats[k].pcg_ratio[ite] = pr[k].ratio;
      MG_REQUIRE(pr[k].status != 2, MGPBD_E_BREAKDOWN,
                 "PCG breakdown (p^T A p <= 0 or r^T z <= 0)" +
                     (nb > 1 ? " in body " + std::to_string(k) : std::string()));
    }
    const size_t u0 = c->phase.mark(st);
    launch_dx_update(nv, c->vptr.p, c->vrow.p, c->vslot.p, c->grad.p, S.dl(), c->w.p,
                     c->opt.omega_relax, xyz, st);
    launch_lambda_add(m, c->lambda.p, S.dl(), st);
    upd_ev.emplace_back(u0, c->phase.mark(st));
    for (int k = 0; k < nb; ++k) {
      if (stopped[k]) continue;
      iters_done[k] = ite + 1;
      if (bn[k] < c->opt.eps_b) { stopped[k] = 1; ++n_stopped; }
    }
  }
  launch_velocity(nv, c->dt, xyz, oxyz, vxyz, st);
  c->frame++;
  double ms_total = total.stop(st);   // synchronises: every phase event has completed
  double ms_asm = 0.0, ms_upd = 0.0;
  for (auto &e : asm_ev) ms_asm += c->phase.ms(e.first, e.second);
  for (auto &e : upd_ev) ms_upd += c->phase.ms(e.first, e.second);
  if (stats)
    for (int k = 0; k < nb; ++k) {
      stats[k].iters_done = iters_done[k];
      stats[k].ms_setup = ms_setup;
      stats[k].ms_pcg = ms_pcg;
      stats[k].ms_total = ms_total;
      stats[k].spmv_calls = S.spmv_calls;
      stats[k].spmv_ms = S.spmv_ms;
      stats[k].spmv_first_ms = S.spmv_first_ms;
      stats[k].ms_assembly = ms_asm;
      stats[k].ms_galerkin = ms_galerkin;
      stats[k].ms_update = ms_upd;
      stats[k].vcycles = S.vcycles;
      for (int l = 0; l < 16; ++l)
        stats[k].ms_level[l] = l < Solver::kProfLevels ? S.level_ms[l] : 0.0;
    }
}

}  // namespace

extern "C" {

void mgpbd_default_options(mgpbd_options *o) {
  o->theta = 0.1;
  o->gs_sweeps = 20;
  o->pre_sweeps = 2;
  o->post_sweeps = 2;
  o->lambda_min = 0.1;
  o->coarse_max = 400;
  o->dense_max = 4096;
  o->max_levels = 16;
  o->power_iters = 30;
  o->omega_relax = 0.1;
  o->tol = 1e-6;
  o->max_pcg = 5000;
  o->seed = 20250513ULL;
  o->reuse_interval = 20;
  o->b_mode = 0;
  o->eps_b = 0.0;
  o->precision = MGPBD_PREC_FP64;
  o->lmax_scale = 1.05;
  o->check_every = 8;
  o->use_graph = 1;
  o->profile_spmv = 0;
  o->spmv_tile = 0;
  o->spmv_lanes = 0;
  o->matrix_free = 1;
  o->smoother = 0;
  o->n_cand = 1;
  o->power_max = 500;
  o->power_tol = 1e-2;
  o->vcycle_tail = 0;
  o->fuse_transfers = 0;
  o->resetup_on_breakdown = 1;
}

mgpbd_status mgpbd_solver_create(const mgpbd_options *opt, mgpbd_ctx **out) {
  if (!out) return MGPBD_E_INVALID_ARG;
  *out = nullptr;
  auto *c = new (std::nothrow) mgpbd_ctx();
  if (!c) return MGPBD_E_OUT_OF_MEMORY;
  mgpbd_status s = guard(c, [&] { init_ctx(c, opt); });
  if (s != MGPBD_OK) { delete c; return s; }
  *out = c;
  return MGPBD_OK;
}

mgpbd_status mgpbd_create(const mgpbd_mesh *mesh, const mgpbd_constraints *cons,
                          const double *compliance, double dt, const double *gravity,
                          const mgpbd_options *opt, mgpbd_ctx **out) {
  if (!out) return MGPBD_E_INVALID_ARG;
  *out = nullptr;
  if (!mesh || !cons || !compliance || !gravity || !mesh->rest || !mesh->inv_mass)
    return MGPBD_E_INVALID_ARG;
  if ((mesh->n_tets && !mesh->tets) || (cons->n_edges && !cons->edges) ||
      (cons->n_vols && !cons->vol_tet) || (cons->n_arap && !cons->arap_tet))
    return MGPBD_E_INVALID_ARG;
  auto *c = new (std::nothrow) mgpbd_ctx();
  if (!c) return MGPBD_E_OUT_OF_MEMORY;
  mgpbd_status s = guard(c, [&] {
    MG_REQUIRE(dt > 0.0 && std::isfinite(dt), MGPBD_E_INVALID_ARG, "dt must be > 0");
    init_ctx(c, opt);
    for (int k = 0; k < 3; ++k)
      MG_REQUIRE(std::isfinite(gravity[k]), MGPBD_E_INVALID_ARG, "gravity not finite");
    const int64_t nv = mesh->n_verts;
    for (int64_t v = 0; v < nv; ++v) {
      MG_REQUIRE(mesh->inv_mass[v] >= 0.0 && std::isfinite(mesh->inv_mass[v]),
                 MGPBD_E_INVALID_ARG, "inverse mass must be finite and >= 0");
      for (int k = 0; k < 3; ++k)
        MG_REQUIRE(std::isfinite(mesh->rest[3 * v + k]), MGPBD_E_INVALID_ARG, "rest not finite");
    }
    Topology t;
    build_topology(nv, mesh->n_tets, mesh->tets, cons->n_edges, cons->edges, cons->n_vols,
                   cons->vol_tet, cons->n_arap, cons->arap_tet, t);
    MG_REQUIRE(t.nnz < (int64_t)INT32_MAX, MGPBD_E_INVALID_ARG,
               "A has more than 2^31 entries; split the body into a batch");
    c->has_body = true;
    c->nv = nv; c->m = t.m; c->nnz = t.nnz;
    c->voff = {0, nv};
    c->roff = {0, t.m};
    c->dt = dt;
    for (int k = 0; k < 3; ++k) c->g[k] = gravity[k];
    const double dt2 = dt * dt;
    std::vector<double> at(t.m);
    for (int64_t r = 0; r < t.m; ++r) {
      MG_REQUIRE(compliance[r] >= 0.0 && std::isfinite(compliance[r]), MGPBD_E_INVALID_ARG,
                 "compliance must be finite and >= 0");
      at[r] = compliance[r] / dt2;
    }
    hipStream_t st = c->st;
    c->rv.upload(t.rv.data(), t.rv.size(), st);
    c->meta.upload(t.meta.data(), t.meta.size(), st);
    c->vptr.upload(t.vptr.data(), t.vptr.size(), st);
    c->vrow.upload(t.vrow.data(), t.vrow.size(), st);
    c->vslot.upload(t.vslot.data(), t.vslot.size(), st);
    std::vector<double> w(mesh->inv_mass, mesh->inv_mass + nv);
    c->w.upload(w.data(), nv, st);
    c->alpha_t.upload(at.data(), t.m, st);
    Level &F = c->solver->L0();
    F.rowptr.upload(t.rowptr.data(), t.rowptr.size(), st);
    F.col.upload(t.col.data(), t.col.size(), st);
    const int64_t arap_lo = t.n_edges + t.n_vols;
    if (t.n_arap > 0) {
      c->has_arap = true;
      std::vector<int8_t> kind(t.m, 0);
      for (int64_t r = arap_lo; r < t.m; ++r) kind[r] = 1;
      c->kind.upload(kind.data(), t.m, st);
      c->dm_inv.alloc(9 * (size_t)t.m);
    }
    alloc_state(c);
    c->rest_c.alloc(t.m);
    // rest lengths and volumes: the constraint kernel itself at the rest
    // positions, so that C is exactly zero at rest
    DevBuf<double> rx[3];
    std::vector<double> comp(nv);
    for (int k = 0; k < 3; ++k) {
      for (int64_t v = 0; v < nv; ++v) comp[v] = mesh->rest[3 * v + k];
      rx[k].upload(comp.data(), nv, st);
    }
    // (ARAP rows keep rest_c = 0: their target is C = 0)
    launch_fill(t.m, 0.0, c->rest_c.p, st);
    launch_fill(t.m, 0.0, c->C.p, st);
    double *xyz[3] = {rx[0].p, rx[1].p, rx[2].p};
    const int8_t *kind = c->has_arap ? c->kind.p : nullptr;
    launch_constraints(t.m, c->rv.p, kind, c->rest_c.p, xyz, c->C.p, c->grad.p, st);
    MG_HIP(hipMemcpyAsync(c->rest_c.p, c->C.p, sizeof(double) * t.m, hipMemcpyDeviceToDevice, st));
    std::vector<double> rc(t.m);
    c->rest_c.download(rc.data(), t.m, st);
    std::vector<double> det6;
    if (kind) {
      launch_arap_rest(t.m, c->rv.p, kind, xyz, c->dm_inv.p, c->C.p, st);
      det6.resize(t.m);
      c->C.download(det6.data(), t.m, st);
    }
    MG_HIP(hipStreamSynchronize(st));
    for (int64_t r = 0; r < t.m; ++r) {
      const bool ok = r < arap_lo ? rc[r] > 0.0 : det6[r] > 0.0;
      MG_REQUIRE(ok, MGPBD_E_INVALID_ARG,
                 (r < t.n_edges ? "zero-length rest edge at row "
                                : "non-positive rest volume at row ") +
                     std::to_string(r));
    }
  });
  if (s != MGPBD_OK) {
    if (c->own) (void)hipStreamDestroy(c->own);
    c->solver.reset();
    delete c;
    return s;
  }
  *out = c;
  return MGPBD_OK;
}

mgpbd_status mgpbd_setup(mgpbd_ctx *c, int32_t max_levels, int32_t reuse_interval) {
  if (!c) return MGPBD_E_INVALID_ARG;
  return guard(c, [&] {
    MG_REQUIRE(max_levels >= 1 && max_levels <= 32, MGPBD_E_INVALID_ARG, "max_levels in 1..32");
    MG_REQUIRE(reuse_interval >= 0, MGPBD_E_INVALID_ARG, "reuse_interval >= 0");
    c->opt.max_levels = max_levels;
    c->opt.reuse_interval = reuse_interval;
    c->solver->opt.max_levels = max_levels;
    c->solver->opt.reuse_interval = reuse_interval;
    c->stale = true;
  });
}

mgpbd_status mgpbd_set_stream(mgpbd_ctx *c, void *s) {
  if (!c) return MGPBD_E_INVALID_ARG;
  return guard(c, [&] {
    c->st = s ? (hipStream_t)s : c->own;
    c->solver->set_stream(c->st);
  });
}

mgpbd_status mgpbd_force_pcg_iters(mgpbd_ctx *c, const int32_t *iters, int32_t n) {
  if (!c || n < 0) return MGPBD_E_INVALID_ARG;
  c->force.clear();
  if (iters) c->force.assign(iters, iters + n);
  return MGPBD_OK;
}

mgpbd_status mgpbd_step(mgpbd_ctx *c, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, int32_t n_iters, mgpbd_step_stats *stats) {
  if (!c) return MGPBD_E_INVALID_ARG;
  if (!c->has_body) { c->err = "context has no body"; return MGPBD_E_STATE; }
  if (!x || !y || !z || !vx || !vy || !vz || n_iters < 0) return MGPBD_E_INVALID_ARG;
  if (c->nb != 1) { c->err = "context belongs to a batch"; return MGPBD_E_STATE; }
  return guard(c, [&] {
    double *xyz[3] = {x, y, z};
    double *vxyz[3] = {vx, vy, vz};
    std::vector<const std::vector<int32_t> *> force{&c->force};
    try {
      run_step(c, xyz, vxyz, n_iters, force, stats);
    } catch (...) {
      c->force.clear();
      throw;
    }
    c->force.clear();
  });
}

mgpbd_status mgpbd_solve(mgpbd_ctx *c, const mgpbd_csr *A, const double *b, double tol,
                         double *x_out, mgpbd_solve_stats *stats) {
  if (!c || !A || !b || !x_out || !A->rowptr || !A->col || !A->val) return MGPBD_E_INVALID_ARG;
  if (c->has_body) { c->err = "mgpbd_solve needs a solver context"; return MGPBD_E_STATE; }
  int status = MGPBD_OK;
  mgpbd_status s = guard(c, [&] {
    MG_REQUIRE(A->n >= 0 && A->n < (int64_t)INT32_MAX && A->nnz >= A->n && A->nnz < (int64_t)INT32_MAX,
               MGPBD_E_INVALID_ARG, "matrix size out of range");
    MG_REQUIRE(tol >= 0.0, MGPBD_E_INVALID_ARG, "tol must be >= 0");
    hipStream_t st = c->st;
    Solver &S = *c->solver;
    int64_t last = -1;
    MG_HIP(hipMemcpyAsync(&last, A->rowptr + A->n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    MG_REQUIRE(last == A->nnz, MGPBD_E_INVALID_ARG, "rowptr[n] != nnz");
    // every row's bounds and columns, before any kernel indexes through them
    c->bad.alloc(1);
    MG_HIP(hipMemsetAsync(c->bad.p, 0, sizeof(int), st));
    launch_validate_csr(A->n, A->nnz, A->rowptr, A->col, c->bad.p, st);
    int hbad = 0;
    MG_HIP(hipMemcpyAsync(&hbad, c->bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    MG_REQUIRE(hbad == 0, MGPBD_E_INVALID_ARG,
               "malformed CSR: row bounds not monotone in [0, nnz] or a column outside [0, n) "
               "or not strictly ascending");
    Level &F = S.L0();
    F.n = A->n;
    F.nnz = A->nnz;
    F.rowptr.alloc(A->n + 1);
    F.col.alloc(A->nnz);
    F.val.alloc(A->nnz);
    MG_HIP(hipMemcpyAsync(F.rowptr.p, A->rowptr, sizeof(int64_t) * (A->n + 1), hipMemcpyDeviceToDevice, st));
    MG_HIP(hipMemcpyAsync(F.col.p, A->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToDevice, st));
    MG_HIP(hipMemcpyAsync(F.val.p, A->val, sizeof(double) * A->nnz, hipMemcpyDeviceToDevice, st));
    S.pattern_dirty = true;
    S.val32_external = false;
    Timer t;
    t.start(st);
    S.setup();
    double ms_setup = t.stop(st);
    t.start(st);
    PcgResult pr = S.pcg(b, x_out, tol, c->opt.max_pcg, nullptr)[0];
    double ms_solve = t.stop(st);
    if (stats) {
      stats->iters = pr.iters;
      stats->ratio = pr.ratio;
      stats->ms_setup = ms_setup;
      stats->ms_solve = ms_solve;
    }
    if (pr.status == 2) status = MGPBD_E_BREAKDOWN;
    else if (pr.status == 4) status = MGPBD_E_NOT_CONVERGED;
  });
  if (s != MGPBD_OK) return s;
  if (status == MGPBD_E_NOT_CONVERGED) c->err = "PCG reached max_pcg";
  if (status == MGPBD_E_BREAKDOWN) c->err = "PCG breakdown";
  return (mgpbd_status)status;
}

void mgpbd_destroy(mgpbd_ctx *c) {
  if (!c || c->batch_owned) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  c->solver.reset();
  hipStream_t own = c->own;
  delete c;
  if (own) (void)hipStreamDestroy(own);
}

const char *mgpbd_last_error(const mgpbd_ctx *c) { return c ? c->err.c_str() : "null context"; }

mgpbd_status mgpbd_num_rows(const mgpbd_ctx *c, int64_t *m, int64_t *nnz) {
  if (!c || !m || !nnz) return MGPBD_E_INVALID_ARG;
  *m = c->solver->lev[0]->n;
  *nnz = c->solver->lev[0]->nnz;
  return MGPBD_OK;
}

mgpbd_status mgpbd_num_levels(const mgpbd_ctx *c, int32_t *levels) {
  if (!c || !levels) return MGPBD_E_INVALID_ARG;
  *levels = c->solver->built ? c->solver->nlev : 0;
  return MGPBD_OK;
}

static mgpbd_status level_ok(const mgpbd_ctx *c, int32_t l) {
  if (!c) return MGPBD_E_INVALID_ARG;
  if (!c->solver->built) return MGPBD_E_STATE;
  if (l < 0 || l >= c->solver->nlev) return MGPBD_E_INVALID_ARG;
  return MGPBD_OK;
}

mgpbd_status mgpbd_get_level(const mgpbd_ctx *c, int32_t l, int64_t *n, int64_t *nnz,
                             double *omega, int64_t *n_agg) {
  mgpbd_status s = level_ok(c, l);
  if (s != MGPBD_OK) return s;
  const Level &L = *c->solver->lev[l];
  if (n) *n = L.n;
  if (nnz) *nnz = L.nnz;
  if (omega) *omega = L.omega.empty() ? 0.0 : L.omega[0];
  if (n_agg) *n_agg = L.has_next ? L.n_agg : -1;
  return MGPBD_OK;
}

mgpbd_status mgpbd_get_aggregates(const mgpbd_ctx *c, int32_t l, int32_t *agg) {
  mgpbd_status s = level_ok(c, l);
  if (s != MGPBD_OK) return s;
  const Level &L = *c->solver->lev[l];
  if (!L.has_next || !agg) return MGPBD_E_INVALID_ARG;
  return guard(const_cast<mgpbd_ctx *>(c), [&] {
    L.agg.download(agg, L.n, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
  });
}

mgpbd_status mgpbd_get_qr(const mgpbd_ctx *c, int32_t l, int32_t *kq, int64_t *coff, double *Q,
                          double *B) {
  mgpbd_status s = level_ok(c, l);
  if (s != MGPBD_OK) return s;
  const Level &L = *c->solver->lev[l];
  if (!L.has_next) return MGPBD_E_INVALID_ARG;
  if (L.K < 2) return MGPBD_E_STATE;
  return guard(const_cast<mgpbd_ctx *>(c), [&] {
    if (kq) L.kq.download(kq, L.n_agg, c->st);
    if (coff) L.coff.download(coff, L.n_agg + 1, c->st);
    if (Q) L.Q.download(Q, L.nmem * L.K, c->st);
    if (B) L.B.download(B, L.n * L.K, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
  });
}

mgpbd_status mgpbd_get_transfer(const mgpbd_ctx *c, int32_t l, double *p, double *B) {
  mgpbd_status s = level_ok(c, l);
  if (s != MGPBD_OK) return s;
  const Level &L = *c->solver->lev[l];
  if (!L.has_next) return MGPBD_E_INVALID_ARG;
  if (L.K > 1) return MGPBD_E_STATE;   // mgpbd_get_qr
  return guard(const_cast<mgpbd_ctx *>(c), [&] {
    if (p) L.p.download(p, L.n, c->st);
    if (B) L.B.download(B, L.n, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
  });
}

mgpbd_status mgpbd_get_matrix(const mgpbd_ctx *c, int32_t l, int64_t *rowptr, int32_t *col,
                              double *val) {
  mgpbd_status s = level_ok(c, l);
  if (s != MGPBD_OK) return s;
  const Level &L = *c->solver->lev[l];
  return guard(const_cast<mgpbd_ctx *>(c), [&] {
    if (rowptr) L.rowptr.download(rowptr, L.n + 1, c->st);
    if (col) L.col.download(col, L.nnz, c->st);
    if (val) L.val.download(val, L.nnz, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
  });
}

mgpbd_status mgpbd_apply(mgpbd_ctx *c, const double *x, double *y) {
  if (!c || !x || !y || x == y) return MGPBD_E_INVALID_ARG;
  if (!c->has_body || !c->have_rhs) {
    c->err = "no assembled system: run a step first";
    return MGPBD_E_STATE;
  }
  return guard(c, [&] { c->solver->apply_fine(x, y); });
}

mgpbd_status mgpbd_apply_noalloc(mgpbd_ctx *c, const double *x, double *y) {
  if (!c || !x || !y || x == y) return MGPBD_E_INVALID_ARG;
  if (!c->has_body || !c->have_rhs) {
    c->err = "no assembled system: run a step first";
    return MGPBD_E_STATE;
  }
  return guard(c, [&] {
    int dev = -1;
    MG_HIP(hipGetDevice(&dev));
    MG_REQUIRE(dev == c->device, MGPBD_E_INVALID_ARG,
               "the context's device must be current");
    const size_t need = sizeof(double) * 4 * (size_t)c->nv;
    MG_REQUIRE(need <= kNoAllocScratchBytes, MGPBD_E_INVALID_ARG,
               "mgpbd_apply_noalloc: " + std::to_string(c->nv) + " vertices need " +
                   std::to_string(need) + " bytes of scratch, more than the " +
                   std::to_string(kNoAllocScratchBytes) + " it holds");
    void *u = scratch_addr(c->device);
    MG_REQUIRE(u != nullptr, MGPBD_E_STATE, "scratch address not set up for this device");
    c->solver->apply_fine_into(x, y, static_cast<double *>(u));
  });
}

mgpbd_status mgpbd_get_fine_operator(const mgpbd_ctx *c, int32_t *matrix_free) {
  if (!c || !matrix_free) return MGPBD_E_INVALID_ARG;
  if (!c->has_body || !c->solver->built) return MGPBD_E_STATE;
  *matrix_free = c->solver->mf.ok() ? 1 : 0;
  return MGPBD_OK;
}

mgpbd_status mgpbd_get_rhs(const mgpbd_ctx *c, double *b) {
  if (!c || !b) return MGPBD_E_INVALID_ARG;
  if (!c->has_body || !c->have_rhs) return MGPBD_E_STATE;
  return guard(const_cast<mgpbd_ctx *>(c), [&] {
    c->b.download(b, c->m, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
  });
}

mgpbd_status mgpbd_get_lambda(const mgpbd_ctx *c, double *lambda) {
  if (!c || !lambda) return MGPBD_E_INVALID_ARG;
  if (!c->has_body) return MGPBD_E_STATE;
  return guard(const_cast<mgpbd_ctx *>(c), [&] {
    c->lambda.download(lambda, c->m, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
  });
}

mgpbd_status mgpbd_get_colors(const mgpbd_ctx *c, int32_t *color, int32_t *n_colors) {
  mgpbd_status s = level_ok(c, 0);
  if (s != MGPBD_OK) return s;
  const Level &L = *c->solver->lev[0];
  if (!L.n_colors) return MGPBD_E_STATE;
  if (n_colors) *n_colors = L.n_colors;
  if (!color) return MGPBD_OK;
  return guard(const_cast<mgpbd_ctx *>(c), [&] {
    L.color.download(color, L.n, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
  });
}

// Test hook: device FP64 sqrt and division of n values (device arrays).
mgpbd_status mgpbd_selftest_sqrt_div(int64_t n, const double *a, const double *b, double *s,
                                     double *q) {
  if (n < 0 || (n && (!a || !b || !s || !q))) return MGPBD_E_INVALID_ARG;
  launch_sqrt_div(n, a, b, s, q, nullptr);
  return hipDeviceSynchronize() == hipSuccess ? MGPBD_OK : MGPBD_E_DEVICE;
}

// ------------------------------------------------------------------ batch
mgpbd_status mgpbd_batch_create(mgpbd_ctx *const *ctxs, int32_t n, mgpbd_batch **out) {
  if (!ctxs || n <= 0 || !out) return MGPBD_E_INVALID_ARG;
  *out = nullptr;
  for (int32_t k = 0; k < n; ++k)
    if (!ctxs[k] || !ctxs[k]->has_body || ctxs[k]->nb != 1) return MGPBD_E_INVALID_ARG;
  for (int32_t k = 1; k < n; ++k) {
    const mgpbd_ctx &a = *ctxs[0], &b = *ctxs[k];
    if (a.dt != b.dt || a.g[0] != b.g[0] || a.g[1] != b.g[1] || a.g[2] != b.g[2] ||
        a.opt.precision != b.opt.precision)
      return MGPBD_E_INVALID_ARG;
  }
  auto *bt = new (std::nothrow) mgpbd_batch();
  if (!bt) return MGPBD_E_OUT_OF_MEMORY;
  mgpbd_ctx *c = &bt->sys;
  mgpbd_status s = guard(c, [&] {
    bt->ctxs.assign(ctxs, ctxs + n);
    init_ctx(c, &ctxs[0]->opt);
    hipStream_t st = c->st;
    c->has_body = true;
    c->batch_owned = true;
    c->nb = n;
    c->dt = ctxs[0]->dt;
    for (int k = 0; k < 3; ++k) c->g[k] = ctxs[0]->g[k];
    std::vector<int64_t> eoff(n + 1, 0), toff(n + 1, 0);
    c->voff.assign(n + 1, 0);
    c->roff.assign(n + 1, 0);
    for (int k = 0; k < n; ++k) {
      const mgpbd_ctx &b = *ctxs[k];
      c->voff[k + 1] = c->voff[k] + b.nv;
      c->roff[k + 1] = c->roff[k] + b.m;
      eoff[k + 1] = eoff[k] + b.nnz;
      toff[k + 1] = toff[k] + (int64_t)b.vrow.n;
    }
    c->nv = c->voff[n];
    c->m = c->roff[n];
    c->nnz = eoff[n];
    MG_REQUIRE(c->nnz < (int64_t)INT32_MAX && c->m < (int64_t)INT32_MAX &&
                   c->nv < (int64_t)INT32_MAX,
               MGPBD_E_INVALID_ARG, "the batch has more than 2^31 entries");
    Level &F = c->solver->L0();
    c->rv.alloc(4 * (size_t)c->m);
    c->meta.alloc(c->nnz);
    c->vptr.alloc(c->nv + 1);
    c->vrow.alloc(std::max<int64_t>(toff[n], 1));
    c->vslot.alloc(std::max<int64_t>(toff[n], 1));
    c->w.alloc(c->nv);
    c->alpha_t.alloc(c->m);
    c->rest_c.alloc(c->m);
    F.rowptr.alloc(c->m + 1);
    F.col.alloc(c->nnz);
    for (int k = 0; k < n; ++k) c->has_arap = c->has_arap || ctxs[k]->has_arap;
    if (c->has_arap) {
      c->kind.alloc(c->m);
      c->dm_inv.alloc(9 * (size_t)c->m);
    }
    auto d2d = [&](void *dst, const void *src, size_t bytes) {
      if (bytes) MG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    };
    for (int k = 0; k < n; ++k) {
      const mgpbd_ctx &b = *ctxs[k];
      const Level &Fb = b.solver->L0();
      const int64_t v0 = c->voff[k], r0 = c->roff[k], e0 = eoff[k], t0 = toff[k];
      launch_offset_copy(4 * b.m, b.rv.p, (int32_t)v0, c->rv.p + 4 * r0, st);
      d2d(c->meta.p + e0, b.meta.p, sizeof(uint32_t) * b.nnz);
      launch_offset_copy(b.m, Fb.rowptr.p, e0, F.rowptr.p + r0, st);
      launch_offset_copy(b.nnz, Fb.col.p, (int32_t)r0, F.col.p + e0, st);
      launch_offset_copy(b.nv, b.vptr.p, t0, c->vptr.p + v0, st);
      launch_offset_copy((int64_t)b.vrow.n, b.vrow.p, (int32_t)r0, c->vrow.p + t0, st);
      d2d(c->vslot.p + t0, b.vslot.p, b.vslot.n);
      d2d(c->w.p + v0, b.w.p, sizeof(double) * b.nv);
      d2d(c->alpha_t.p + r0, b.alpha_t.p, sizeof(double) * b.m);
      d2d(c->rest_c.p + r0, b.rest_c.p, sizeof(double) * b.m);
      if (c->has_arap && b.m) {
        if (b.has_arap) {
          d2d(c->kind.p + r0, b.kind.p, b.m);
          d2d(c->dm_inv.p + 9 * r0, b.dm_inv.p, sizeof(double) * 9 * b.m);
        } else {
          MG_HIP(hipMemsetAsync(c->kind.p + r0, 0, b.m, st));
        }
      }
    }
    MG_HIP(hipMemcpyAsync(F.rowptr.p + c->m, &eoff[n], sizeof(int64_t), hipMemcpyHostToDevice, st));
    MG_HIP(hipMemcpyAsync(c->vptr.p + c->nv, &toff[n], sizeof(int64_t), hipMemcpyHostToDevice, st));
    alloc_state(c);
    for (int k = 0; k < 3; ++k) {
      bt->pos[k].alloc(c->nv);
      bt->vel[k].alloc(c->nv);
    }
    MG_HIP(hipStreamSynchronize(st));
  });
  if (s != MGPBD_OK) {
    const std::string msg = c->err;
    delete bt;
    if (n > 0 && ctxs[0]) ctxs[0]->err = msg;
    return s;
  }
  *out = bt;
  return MGPBD_OK;
}

mgpbd_status mgpbd_batch_step(mgpbd_batch *bt, double *const *xyz, double *const *vxyz,
                              int32_t n_iters, mgpbd_step_stats *stats) {
  if (!bt || !xyz || !vxyz || n_iters < 0) return MGPBD_E_INVALID_ARG;
  const int n = (int)bt->ctxs.size();
  for (int k = 0; k < 3 * n; ++k)
    if (!xyz[k] || !vxyz[k]) return MGPBD_E_INVALID_ARG;
  mgpbd_ctx *c = &bt->sys;
  return guard(c, [&] {
    hipStream_t st = c->st;
    // every body's state is copied in, stepped in one system, and copied out
    for (int k = 0; k < n; ++k) {
      const int64_t v0 = c->voff[k], nvk = c->voff[k + 1] - v0;
      if (!nvk) continue;
      for (int d = 0; d < 3; ++d) {
        MG_HIP(hipMemcpyAsync(bt->pos[d].p + v0, xyz[3 * k + d], sizeof(double) * nvk,
                              hipMemcpyDeviceToDevice, st));
        MG_HIP(hipMemcpyAsync(bt->vel[d].p + v0, vxyz[3 * k + d], sizeof(double) * nvk,
                              hipMemcpyDeviceToDevice, st));
      }
    }
    double *pos[3] = {bt->pos[0].p, bt->pos[1].p, bt->pos[2].p};
    double *vel[3] = {bt->vel[0].p, bt->vel[1].p, bt->vel[2].p};
    std::vector<const std::vector<int32_t> *> force(n);
    for (int k = 0; k < n; ++k) force[k] = &bt->ctxs[k]->force;
    try {
      run_step(c, pos, vel, n_iters, force, stats);
    } catch (...) {
      for (auto *b : bt->ctxs) b->force.clear();
      throw;
    }
    for (auto *b : bt->ctxs) b->force.clear();
    for (int k = 0; k < n; ++k) {
      const int64_t v0 = c->voff[k], nvk = c->voff[k + 1] - v0;
      if (!nvk) continue;
      for (int d = 0; d < 3; ++d) {
        MG_HIP(hipMemcpyAsync(xyz[3 * k + d], bt->pos[d].p + v0, sizeof(double) * nvk,
                              hipMemcpyDeviceToDevice, st));
        MG_HIP(hipMemcpyAsync(vxyz[3 * k + d], bt->vel[d].p + v0, sizeof(double) * nvk,
                              hipMemcpyDeviceToDevice, st));
      }
    }
    MG_HIP(hipStreamSynchronize(st));
  });
}

mgpbd_ctx *mgpbd_batch_context(mgpbd_batch *bt) { return bt ? &bt->sys : nullptr; }

void mgpbd_batch_destroy(mgpbd_batch *bt) {
  if (!bt) return;
  mgpbd_ctx *c = &bt->sys;
  if (c->st) (void)hipStreamSynchronize(c->st);
  c->solver.reset();
  hipStream_t own = c->own;
  delete bt;
  if (own) (void)hipStreamDestroy(own);
}

}  // extern "C"
