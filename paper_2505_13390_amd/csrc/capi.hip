// C ABI (include/mgpbd.h): simulation contexts running Algorithm 1 on one
// GPU, the standalone solver entry, inspection hooks, and batching.
#include <chrono>
#include <cmath>
#include <memory>

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

struct mgpbd_ctx {
  std::string err;
  mgpbd_options opt;
  hipStream_t own = nullptr;
  hipStream_t st = nullptr;
  std::unique_ptr<Solver> solver;
  // body (absent for solver-only contexts)
  bool has_body = false;
  int64_t nv = 0, n_edges = 0, n_vols = 0, m = 0, nnz = 0;
  double dt = 0.0, g[3] = {0, 0, 0};
  int64_t frame = 0;
  bool stale = true;
  DevBuf<int32_t> rv;
  DevBuf<uint32_t> meta;
  DevBuf<int64_t> vptr;
  DevBuf<int32_t> vrow;
  DevBuf<int8_t> vslot;
  DevBuf<double> w, alpha_t, rest_c, C, grad, lambda, b, old[3];
  DevBuf<int> bad;
  std::vector<int32_t> force;
  bool have_rhs = false;
};

struct mgpbd_batch {
  std::vector<mgpbd_ctx *> ctxs;
};

namespace {

mgpbd_status fail(mgpbd_ctx *c, const Error &e) {
  if (c) c->err = e.what();
  return (mgpbd_status)e.status;
}

template <class F>
mgpbd_status guard(mgpbd_ctx *c, F f) {
  try {
    f();
    if (c) c->err.clear();
    return MGPBD_OK;
  } catch (const Error &e) {
    return fail(c, e);
  } catch (const std::bad_alloc &) {
    if (c) c->err = "host allocation failed";
    return MGPBD_E_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
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
  MG_REQUIRE(o.power_iters >= 0 && o.max_pcg >= 1 && o.check_every >= 1, MGPBD_E_INVALID_ARG,
             "iteration counts");
  MG_REQUIRE(o.tol >= 0.0 && o.lmax_scale > 0.0, MGPBD_E_INVALID_ARG, "tol / lmax_scale");
  MG_REQUIRE(o.precision == MGPBD_PREC_FP64 || o.precision == MGPBD_PREC_MIXED,
             MGPBD_E_INVALID_ARG, "precision");
  MG_REQUIRE(o.reuse_interval >= 0, MGPBD_E_INVALID_ARG, "reuse_interval");
  MG_REQUIRE(o.spmv_tile == 0 || o.spmv_tile == -1 || o.spmv_tile == 1024 ||
                 o.spmv_tile == 2048 || o.spmv_tile == 4096,
             MGPBD_E_INVALID_ARG, "spmv_tile must be 0, -1, 1024, 2048 or 4096");
  MG_REQUIRE(o.spmv_lanes == 0 || o.spmv_lanes == 4 || o.spmv_lanes == 8 || o.spmv_lanes == 16 ||
                 o.spmv_lanes == 32 || o.spmv_lanes == 64,
             MGPBD_E_INVALID_ARG, "spmv_lanes must be 0, 4, 8, 16, 32 or 64");
}

void init_ctx(mgpbd_ctx *c, const mgpbd_options *opt) {
  if (opt) c->opt = *opt; else mgpbd_default_options(&c->opt);
  check_options(c->opt);
  MG_HIP(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
  c->st = c->own;
  c->solver.reset(new Solver(c->opt));
  c->solver->set_stream(c->st);
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
      (cons->n_vols && !cons->vol_tet))
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
                   cons->vol_tet, t);
    MG_REQUIRE(t.nnz < (int64_t)INT32_MAX, MGPBD_E_INVALID_ARG,
               "A has more than 2^31 entries; split the body into a batch");
    c->has_body = true;
    c->nv = nv; c->n_edges = t.n_edges; c->n_vols = t.n_vols; c->m = t.m; c->nnz = t.nnz;
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
    F.n = t.m;
    F.nnz = t.nnz;
    F.rowptr.upload(t.rowptr.data(), t.rowptr.size(), st);
    F.col.upload(t.col.data(), t.col.size(), st);
    F.val.alloc(t.nnz);
    if (c->opt.precision == MGPBD_PREC_MIXED) {
      F.val32.alloc(t.nnz);
      c->solver->val32_external = true;
    }
    c->solver->pattern_dirty = true;
    c->C.alloc(t.m);
    c->grad.alloc(12 * (size_t)t.m);
    c->lambda.alloc(t.m);
    c->b.alloc(t.m);
    c->rest_c.alloc(t.m);
    c->bad.alloc(1);
    for (int k = 0; k < 3; ++k) c->old[k].alloc(nv);
    // rest lengths and volumes: the constraint kernel itself at the rest
    // positions, so that C is exactly zero at rest
    DevBuf<double> rx[3];
    std::vector<double> comp(nv);
    for (int k = 0; k < 3; ++k) {
      for (int64_t v = 0; v < nv; ++v) comp[v] = mesh->rest[3 * v + k];
      rx[k].upload(comp.data(), nv, st);
    }
    launch_fill(t.m, 0.0, c->rest_c.p, st);
    double *xyz[3] = {rx[0].p, rx[1].p, rx[2].p};
    launch_constraints(t.m, t.n_edges, c->rv.p, c->rest_c.p, xyz, c->C.p, c->grad.p, st);
    MG_HIP(hipMemcpyAsync(c->rest_c.p, c->C.p, sizeof(double) * t.m, hipMemcpyDeviceToDevice, st));
    std::vector<double> rc(t.m);
    c->rest_c.download(rc.data(), t.m, st);
    MG_HIP(hipStreamSynchronize(st));
    for (int64_t r = 0; r < t.m; ++r)
      MG_REQUIRE(rc[r] > 0.0, MGPBD_E_INVALID_ARG,
                 (r < t.n_edges ? "zero-length rest edge at row " : "non-positive rest volume at row ") +
                     std::to_string(r));
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
  return guard(c, [&] {
    hipStream_t st = c->st;
    Solver &S = *c->solver;
    const int64_t nv = c->nv, m = c->m;
    double *xyz[3] = {x, y, z};
    double *vxyz[3] = {vx, vy, vz};
    double *oxyz[3] = {c->old[0].p, c->old[1].p, c->old[2].p};
    MG_HIP(hipMemsetAsync(c->bad.p, 0, sizeof(int), st));
    for (int k = 0; k < 3; ++k) {
      launch_check_finite(nv, xyz[k], c->bad.p, st);
      launch_check_finite(nv, vxyz[k], c->bad.p, st);
    }
    int hbad = 0;
    MG_HIP(hipMemcpyAsync(&hbad, c->bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    MG_REQUIRE(hbad == 0, MGPBD_E_INVALID_ARG, "non-finite positions or velocities");
    Timer total, part;
    total.start(st);
    double ms_setup = 0.0, ms_pcg = 0.0;
    S.spmv_calls = 0;
    S.spmv_ms = 0.0;
    launch_predict(nv, c->w.p, c->g, c->dt, xyz, vxyz, oxyz, st);
    launch_fill(m, 0.0, c->lambda.p, st);
    Level &F = S.L0();
    int done_iters = 0;
    for (int ite = 0; ite < n_iters; ++ite) {
      launch_constraints(m, c->n_edges, c->rv.p, c->rest_c.p, xyz, c->C.p, c->grad.p, st);
      launch_assemble(m, c->n_edges, 16, F.rowptr.p, F.col.p, c->meta.p, c->rv.p, c->w.p,
                      c->grad.p, c->alpha_t.p, c->C.p, c->lambda.p, F.val.p,
                      S.mixed() ? F.val32.p : nullptr, c->b.p, st);
      c->have_rhs = true;
      double bn = std::sqrt(S.norm2(c->b.p, m));
      if (stats && stats->bnorm) stats->bnorm[ite] = bn;
      const int R = c->opt.reuse_interval;
      bool due = c->stale || !S.built || R <= 0 || (ite == 0 && (c->frame % R) == 0);
      if (stats && stats->setup_ran) stats->setup_ran[ite] = due ? 1 : 0;
      part.start(st);
      if (due) {
        S.setup();
        c->stale = false;
      } else {
        S.refresh();
      }
      ms_setup += part.stop(st);
      int force = (ite < (int)c->force.size()) ? c->force[ite] : 0;
      part.start(st);
      PcgResult pr = S.pcg(c->b.p, S.dl(), c->opt.tol, c->opt.max_pcg, force);
      ms_pcg += part.stop(st);
      if (stats && stats->pcg_iters) stats->pcg_iters[ite] = pr.iters;
      if (stats && stats->pcg_ratio) stats->pcg_ratio[ite] = pr.ratio;
      MG_REQUIRE(pr.status != 2, MGPBD_E_BREAKDOWN, "PCG breakdown (p^T A p <= 0 or r^T z <= 0)");
      launch_dx_update(nv, c->vptr.p, c->vrow.p, c->vslot.p, c->grad.p, S.dl(), c->w.p,
                       c->opt.omega_relax, xyz, st);
      launch_lambda_add(m, c->lambda.p, S.dl(), st);
      done_iters = ite + 1;
      if (bn < c->opt.eps_b) break;
    }
    launch_velocity(nv, c->dt, xyz, oxyz, vxyz, st);
    c->frame++;
    double ms_total = total.stop(st);
    c->force.clear();
    if (stats) {
      stats->iters_done = done_iters;
      stats->ms_setup = ms_setup;
      stats->ms_pcg = ms_pcg;
      stats->ms_total = ms_total;
      stats->spmv_calls = S.spmv_calls;
      stats->spmv_ms = S.spmv_ms;
    }
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
    PcgResult pr = S.pcg(b, x_out, tol, c->opt.max_pcg, 0);
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
  if (!c) return;
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
  if (omega) *omega = L.omega;
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

mgpbd_status mgpbd_get_transfer(const mgpbd_ctx *c, int32_t l, double *p, double *B) {
  mgpbd_status s = level_ok(c, l);
  if (s != MGPBD_OK) return s;
  const Level &L = *c->solver->lev[l];
  if (!L.has_next) return MGPBD_E_INVALID_ARG;
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
  for (int32_t k = 0; k < n; ++k)
    if (!ctxs[k] || !ctxs[k]->has_body) return MGPBD_E_INVALID_ARG;
  auto *b = new (std::nothrow) mgpbd_batch();
  if (!b) return MGPBD_E_OUT_OF_MEMORY;
  b->ctxs.assign(ctxs, ctxs + n);
  *out = b;
  return MGPBD_OK;
}

mgpbd_status mgpbd_batch_step(mgpbd_batch *b, double *const *xyz, double *const *vxyz,
                              int32_t n_iters, mgpbd_step_stats *st) {
  if (!b || !xyz || !vxyz) return MGPBD_E_INVALID_ARG;
  for (size_t k = 0; k < b->ctxs.size(); ++k) {
    mgpbd_status s = mgpbd_step(b->ctxs[k], xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2],
                                vxyz[3 * k], vxyz[3 * k + 1], vxyz[3 * k + 2], n_iters,
                                st ? &st[k] : nullptr);
    if (s != MGPBD_OK) return s;
  }
  return MGPBD_OK;
}

void mgpbd_batch_destroy(mgpbd_batch *b) { delete b; }

}  // extern "C"
