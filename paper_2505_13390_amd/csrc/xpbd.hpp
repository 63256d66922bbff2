// Launchers of the simulation-loop kernels (Algorithm 1) and host-side
// construction of the fixed pattern of A.
#pragma once

#include "kernels.hpp"

namespace mgpbd {

void launch_predict(int64_t nv, const double *w, const double *g, double dt, double *const *xyz,
                    double *const *vxyz, double *const *oxyz, hipStream_t s);
// rows with kind[r] != 0 (ARAP) are skipped; kind may be null (no ARAP rows)
void launch_constraints(int64_t m, const int32_t *rv, const int8_t *kind, const double *rest_c,
                        const double *const *xyz, double *C, double *grad, hipStream_t s);
// ARAP rows (Sec. 5.3, Eq. 8): C = |F - R|_F^2 with F = Ds Dm^-1 and R the nearest
// rotation (det +1) of F; grad slot k = column k - 1 of 2 (F - R) Dm^-T
// (k = 1..3), slot 0 the negated sum. Only rows with kind[r] != 0.
void launch_arap_constraints(int64_t m, const int32_t *rv, const int8_t *kind,
                             const double *dm_inv, const double *const *xyz, double *C,
                             double *grad, hipStream_t s);
// Rest shape of the ARAP rows: dm_inv[9 r ..] = Dm^-1 (row-major) and
// det6[r] = det Dm (six times the rest volume; must be > 0).
void launch_arap_rest(int64_t m, const int32_t *rv, const int8_t *kind,
                      const double *const *rest, double *dm_inv, double *det6, hipStream_t s);
void launch_assemble(int64_t m, int lanes, const int64_t *rp, const int32_t *col,
                     const uint32_t *meta, const int32_t *rv, const double *w, const double *grad,
                     const double *alpha_t, const double *C, const double *lambda, double *val,
                     float *val32, double *b, hipStream_t s);
void launch_dx_update(int64_t nv, const int64_t *vptr, const int32_t *vrow, const int8_t *vslot,
                      const double *grad, const double *dl, const double *w, double omega,
                      double *const *xyz, hipStream_t s);
void launch_lambda_add(int64_t m, double *lambda, const double *dl, hipStream_t s);
void launch_velocity(int64_t nv, double dt, double *const *xyz, double *const *oxyz,
                     double *const *vxyz, hipStream_t s);
// out = in + add (int32: negative entries kept as they are)
void launch_offset_copy(int64_t n, const int32_t *in, int32_t add, int32_t *out, hipStream_t s);
void launch_offset_copy(int64_t n, const int64_t *in, int64_t add, int64_t *out, hipStream_t s);
void launch_check_finite(int64_t n, const double *a, int *bad, hipStream_t s);
void launch_sqrt_div(int64_t n, const double *a, const double *b, double *s, double *q,
                     hipStream_t st);

// Host-built topology: rows (edges, volumes, ARAP), the pattern of A (pairs of
// rows sharing a vertex, sorted columns) with per-entry shared-vertex codes,
// and the vertex -> (row, slot) incidence used by the dx gather.
struct Topology {
  int64_t n_verts = 0, n_edges = 0, n_vols = 0, n_arap = 0, m = 0, nnz = 0;
  std::vector<int32_t> rv;       // [m][4], -1 padded
  std::vector<int64_t> rowptr;   // [m + 1]
  std::vector<int32_t> col;      // [nnz]
  std::vector<uint32_t> meta;    // [nnz]
  std::vector<int64_t> vptr;     // [n_verts + 1]
  std::vector<int32_t> vrow;     // rows containing each vertex, ascending
  std::vector<int8_t> vslot;     // local slot of the vertex in that row
};

// Validates indices and ordering (throws Error(MGPBD_E_INVALID_ARG)).
void build_topology(int64_t n_verts, int64_t n_tets, const int32_t *tets, int64_t n_edges,
                    const int32_t *edges, int64_t n_vols, const int32_t *vol_tet,
                    int64_t n_arap, const int32_t *arap_tet, Topology &t);

}  // namespace mgpbd
