/*
 * FP64 CPU oracle for the MGPBD global XPBD iteration (Li et al., "MGPBD: A
 * Multigrid Accelerated Global XPBD Solver", SIGGRAPH 2025).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do. It shares no code, header, table or helper with the HIP
 * library; it is written from the paper, plain, single threaded and slow.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle_mgpbd.so mgpbd_oracle.c -lm
 * (no -ffast-math; every floating-point expression below is evaluated exactly
 * in the order it is written).
 *
 * What it computes (section and equation references are to the paper):
 *  - Algorithm 1 (the MGPBD simulation loop): semi-implicit Euler predict,
 *    lambda reset, then per global iteration: C and grad C, A, b, lazy AMG
 *    setup, MGPCG solve, dx = M^-1 gradC^T dlambda (Eq. 5), lambda += dlambda,
 *    x += omega dx, and v = (x - x_old)/dt at the end of the frame.
 *  - Eq. 3: A = gradC M^-1 gradC^T + alpha~, b = -C - alpha~ lambda,
 *    alpha~ = alpha / dt^2 (Sec. 3). Values follow the per-entry form of
 *    Sec. 4.2 (diagonal: sum over the element's vertices of m^-1 |g|^2 plus
 *    alpha~; off-diagonal: sum over shared vertices of m^-1 g_i . g_j).
 *  - Sec. 4.1 setup: strength filter |A_ij| >= theta sqrt(|A_ii||A_jj|),
 *    aggregation (roots with their strong neighbours, leftovers to the
 *    strongest neighbouring aggregate), injection of the near-kernel vector
 *    into P, next-level candidate from the QR factor (one candidate: the
 *    aggregate norm), recursion until the matrix has at most coarse_max rows.
 *  - Sec. 4.3 near-kernel: Gauss-Seidel sweeps on A x = 0 from x0 drawn
 *    uniformly in (0, max|A_ij|).
 *  - Sec. 4.4 (Eq. 6): A_{l+1} = P_l^T A_l P_l, rebuilt in the solving phase;
 *    PCG with one V-cycle as preconditioner.
 *  - Sec. 4.5: omega-Jacobi smoother, 2 pre + 2 post sweeps,
 *    omega = 2 / (lambda_max(D^-1 A) + lambda_min), lambda_max by the power
 *    method (run until its eigen-residual is small, power_lmax), lambda_min a
 *    user estimate (0.1); computed at setup only.
 *    Optionally the Chebyshev smoother of the same subsection: s steps of
 *    Chebyshev acceleration of Jacobi on the interval [lambda_min, lambda_max]
 *    (the recurrence of Saad, Iterative Methods for Sparse Linear Systems,
 *    2nd ed., Alg. 12.1, with M = D), coefficients fixed at setup; or the
 *    parallel (multicolour) Gauss-Seidel smoother: colours of every level from
 *    a greedy colouring in descending priority, forward colour order before
 *    the coarse correction and reversed order after it (the adjoint, so the
 *    V-cycle stays symmetric).
 *  - Sec. 5.3, Eq. 8 (As-Rigid-As-Possible constraints): a tet row with
 *    C = |F - R|_F^2, F the deformation gradient and R its nearest rotation
 *    (arap_eval, with the readings listed there).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - by default one near-kernel candidate per aggregate (K = 1): P column =
 *    candidate restricted to the aggregate and normalised; next-level
 *    candidate = norm. Option n_cand = K > 1 (Sec. 4.3 generates six):
 *    K candidates from K random starts, modified Gram-Schmidt QR per
 *    aggregate with dependent columns dropped (qr_aggregate), so an
 *    aggregate gives 1..K coarse unknowns;
 *  - aggregation pass 1 is the greedy distance-2 independent set taken in
 *    descending pseudo-random priority; pass 2 joins the neighbour with the
 *    largest |a_ij| (ties: smallest j); aggregates numbered by root index;
 *  - Gauss-Seidel uses a greedy multicolour order (descending priority);
 *  - coarsest level solved by dense Cholesky; PCG from x0 = 0, stop when the
 *    recurrence residual satisfies |r| <= tol |b|, Fletcher-Reeves beta;
 *  - volume constraint C = V - V0 with V = e1.(e2 x e3)/6 (not in the paper).
 * Random numbers: SplitMix64 (Steele, Lea, Flood 2014) through
 * mix64(seed, stream, i) = splitmix64(splitmix64(seed<<8 | stream) + i).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID 1
#define ORC_E_NOMEM 2
#define ORC_E_NOT_CONVERGED 4
#define ORC_E_BREAKDOWN 5
#define ORC_E_SETUP 6

typedef struct orc_opts {
  double theta;        /* strength threshold (Sec. 4.1): 0.1 */
  int gs_sweeps;       /* near-kernel GS sweeps (Sec. 4.3): 20 */
  int pre_sweeps;      /* Jacobi pre-sweeps (Sec. 4.5): 2 */
  int post_sweeps;     /* Jacobi post-sweeps: 2 */
  double lambda_min;   /* user estimate of lambda_min(D^-1 A) (Sec. 4.5): 0.1 */
  int coarse_max;      /* stop coarsening at <= this many rows (Sec. 4.1): 400 */
  int dense_max;       /* largest coarsest level accepted for dense Cholesky: 4096 */
  int max_levels;      /* cap on the number of levels: 16 */
  int power_iters;     /* power-method steps before the first stopping test: 30 */
  double omega_relax;  /* x += omega dx (Algorithm 1): 0.1 */
  double tol;          /* PCG relative residual: 1e-6 */
  int max_pcg;         /* PCG iteration cap: 5000 */
  uint64_t seed;       /* solver's own random streams */
  int reuse_interval;  /* setup at iteration 0 of frames f % R == 0; 0 = every iteration */
  int b_mode;          /* 0 = smoothed near-kernel, 1 = all-ones candidate */
  double eps_b;        /* stop the frame loop when |b| < eps_b (0 = never) */
  int flexible;        /* 0 = Fletcher-Reeves beta, 1 = Polak-Ribiere beta */
  double lmax_scale;   /* omega = 2 / (lmax_scale * lambda_max + lambda_min): 1.05 */
  int smoother;        /* 0 = omega-Jacobi, 1 = Chebyshev, 2 = multicolour GS (Sec. 4.5): 0 */
  int n_cand;          /* near-kernel candidates per level K (Sec. 4.3 uses six): 1 */
  int power_max;       /* power-method step cap: 500 */
  double power_tol;    /* power-method stop: eigen-residual <= power_tol * estimate: 1e-2 */
  int resetup_on_breakdown; /* 1: a PCG breakdown under a hierarchy kept from an earlier
                               iteration sets up afresh for the current A and solves
                               again (once): 1 */
} orc_opts;

void orc_default_opts(orc_opts *o) {
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
  o->flexible = 0;
  o->lmax_scale = 1.05;
  o->smoother = 0;
  o->n_cand = 1;
  o->power_max = 500;
  o->power_tol = 1e-2;
  o->resetup_on_breakdown = 1;
}

/* ------------------------------------------------------------------ */
/* random numbers                                                      */
/* ------------------------------------------------------------------ */
static uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t z) { return splitmix64(z); }

uint64_t orc_mix64(uint64_t seed, uint64_t stream, uint64_t i) {
  uint64_t salt = splitmix64((seed << 8) | stream);
  return splitmix64(salt + i);
}

static double uniform01(uint64_t seed, uint64_t stream, uint64_t i) {
  return ((double)(orc_mix64(seed, stream, i) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* priority key: high 32 bits pseudo-random, low 32 bits the node index, so
   keys are distinct; larger key = visited earlier. */
static uint64_t prio_key(uint64_t seed, uint64_t stream, int level, int64_t i) {
  uint64_t h = orc_mix64(seed, stream, ((uint64_t)level << 40) + (uint64_t)i);
  return (h & 0xFFFFFFFF00000000ULL) | (uint64_t)(uint32_t)i;
}

/* ------------------------------------------------------------------ */
/* CSR matrix                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t n, nnz;
  int64_t *rowptr;
  int32_t *col; /* ascending within each row */
  double *val;
} csr;

static void csr_free(csr *a) {
  free(a->rowptr);
  free(a->col);
  free(a->val);
  memset(a, 0, sizeof *a);
}

static double csr_get_diag(const csr *a, int64_t i) {
  for (int64_t e = a->rowptr[i]; e < a->rowptr[i + 1]; ++e)
    if (a->col[e] == i) return a->val[e];
  return 0.0;
}

/* y = A x, each row summed in ascending column order */
static void spmv(const csr *a, const double *x, double *y) {
  for (int64_t i = 0; i < a->n; ++i) {
    double s = 0.0;
    for (int64_t e = a->rowptr[i]; e < a->rowptr[i + 1]; ++e) s += a->val[e] * x[a->col[e]];
    y[i] = s;
  }
}

static double dot(int64_t n, const double *x, const double *y) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
  return s;
}

/* ------------------------------------------------------------------ */
/* The simulated body: vertices, constraint rows, fixed pattern of A   */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t n_verts, n_tets, n_edges, n_vols, n_arap, m;
  double *rest, *w;      /* rest[N][3], inverse masses */
  int32_t *tets;         /* [T][4] */
  int32_t *rv;           /* vertices of each row: [m][4], -1 padding */
  int *rk;               /* arity of each row: 2 (edge) or 4 (volume, ARAP) */
  int *arap;             /* 1 for an ARAP row, else 0 */
  double *dm_inv;        /* [m][9] inverse rest shape matrix of ARAP rows, row-major */
  double *rest_c;        /* L0 or V0 per row (0 for ARAP rows) */
  double *alpha_t;       /* alpha / dt^2 per row */
  double dt, g[3];
  orc_opts o;
  csr A;                 /* pattern + current values */
  /* vertex -> (row, slot) incidence, rows ascending */
  int64_t *vc_ptr;
  int32_t *vc_row, *vc_slot;
  /* state */
  double *lambda, *C, *grad; /* grad[m][4][3] */
  double *b_last;            /* right-hand side of the last global iteration */
  int64_t frame;
  void *hier;
} orc_sim;

/* ------------------------------------------------------------------ */
/* ARAP constraint (Sec. 5.3, Eq. 8, As-Rigid-As-Possible Constraints)          */
/* ------------------------------------------------------------------ */
/* Per tet (x0, x1, x2, x3): Ds = [x1 - x0, x2 - x0, x3 - x0] (columns),
   Dm the same matrix at rest, F = Ds Dm^-1 the deformation gradient and
   C = |F - R|_F^2 with R the rotation of F.
   Readings (the paper defers the details to Kim and Eberle's 2020 course
   notes on deformables):
    - R is the rotation (det R = +1) nearest to F in the Frobenius norm, i.e.
      U V^T from the signed SVD F = U S V^T with U, V rotations and the sign of
      det F carried by the smallest singular value; an inverted tet therefore
      has C > 0 and is pushed back. When it is not unique (rank(F) <= 1),
      R = I.
    - C(F) = min over rotations Q of |F - Q|^2, so by the envelope theorem
      dC/dF = 2 (F - R) wherever R is unique. With F = Ds Dm^-1,
      dC/dDs = 2 (F - R) Dm^-T, whose column i - 1 is dC/dx_i (i = 1, 2, 3),
      and dC/dx_0 = -(dC/dx_1 + dC/dx_2 + dC/dx_3).
    - The row's target is C = 0 (rest_c = 0); its compliance alpha is an
      input (the paper takes alpha = 1 / (mu V_rest)).
   Matrices are row-major 3x3: M[3 * i + j]. */

static void mat3_mul(const double *a, const double *b, double *o) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      o[3 * i + j] = (a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j]) + a[3 * i + 2] * b[6 + j];
}

static void mat3_transpose(const double *a, double *o) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o[3 * j + i] = a[3 * i + j];
}

/* Inverse by Gauss-Jordan elimination with partial pivoting; returns 0 if
   the matrix is singular. */
static int mat3_inverse(const double *a, double *inv) {
  double m[3][6];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      m[i][j] = a[3 * i + j];
      m[i][3 + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int c = 0; c < 3; ++c) {
    int p = c;
    for (int r = c + 1; r < 3; ++r)
      if (fabs(m[r][c]) > fabs(m[p][c])) p = r;
    if (m[p][c] == 0.0) return 0;
    if (p != c)
      for (int j = 0; j < 6; ++j) { double t = m[c][j]; m[c][j] = m[p][j]; m[p][j] = t; }
    double piv = m[c][c];
    for (int j = 0; j < 6; ++j) m[c][j] /= piv;
    for (int r = 0; r < 3; ++r) {
      if (r == c) continue;
      double f = m[r][c];
      for (int j = 0; j < 6; ++j) m[r][j] -= f * m[c][j];
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) inv[3 * i + j] = m[i][3 + j];
  return 1;
}

/* Eigen-decomposition of a symmetric 3x3 matrix by the cyclic Jacobi method
   (Golub and Van Loan, Matrix Computations, Sec. 8.5): rotations in the
   planes (0,1), (0,2), (1,2) until the off-diagonal part is negligible.
   On return a is diagonal (the eigenvalues) and the columns of v are the
   eigenvectors. */
static void sym3_jacobi(double *a, double *v) {
  for (int i = 0; i < 9; ++i) v[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, all = 0.0;
    for (int i = 0; i < 9; ++i) {
      all += a[i] * a[i];
      if (i % 4 != 0) off += a[i] * a[i];
    }
    if (off <= 1e-30 * all) break; /* off-diagonal norm below ~1e-15 of the whole */
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        double apq = a[3 * p + q];
        if (apq == 0.0) continue;
        /* the symmetric 2x2 Schur decomposition of rows/columns p, q */
        double tau = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
        double t = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                              : -1.0 / (-tau + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        double J[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Jt[9], tmp[9];
        J[3 * p + p] = c; J[3 * p + q] = s;
        J[3 * q + p] = -s; J[3 * q + q] = c;
        mat3_transpose(J, Jt);
        mat3_mul(Jt, a, tmp);
        mat3_mul(tmp, J, a);
        mat3_mul(v, J, tmp);
        memcpy(v, tmp, sizeof tmp);
      }
  }
}

/* The rotation nearest to F (see the readings above): eigenvectors V of
   F^T F ordered by descending eigenvalue with det V = +1, u_1 and u_2 the
   normalised (and orthogonalised) F v_1 and F v_2, u_3 = u_1 x u_2,
   R = U V^T. Exported for the tests. */
void orc_closest_rotation(const double *F, double *R) {
  double Ft[9], S[9], V[9];
  mat3_transpose(F, Ft);
  mat3_mul(Ft, F, S);
  sym3_jacobi(S, V);
  double lam[3] = {S[0], S[4], S[8]};
  int ord[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (lam[ord[j]] > lam[ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
  double v[3][3]; /* v[k] = k-th eigenvector, descending eigenvalue */
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) v[k][d] = V[3 * d + ord[k]];
  double det = v[0][0] * (v[1][1] * v[2][2] - v[1][2] * v[2][1]) -
               v[0][1] * (v[1][0] * v[2][2] - v[1][2] * v[2][0]) +
               v[0][2] * (v[1][0] * v[2][1] - v[1][1] * v[2][0]);
  if (det < 0.0)
    for (int d = 0; d < 3; ++d) v[2][d] = -v[2][d];
  double u[3][3];
  for (int k = 0; k < 2; ++k)
    for (int d = 0; d < 3; ++d)
      u[k][d] = (F[3 * d] * v[k][0] + F[3 * d + 1] * v[k][1]) + F[3 * d + 2] * v[k][2];
  double n0 = sqrt((u[0][0] * u[0][0] + u[0][1] * u[0][1]) + u[0][2] * u[0][2]);
  if (!(n0 > 0.0)) { for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0; return; }
  for (int d = 0; d < 3; ++d) u[0][d] /= n0;
  double pr = (u[0][0] * u[1][0] + u[0][1] * u[1][1]) + u[0][2] * u[1][2];
  for (int d = 0; d < 3; ++d) u[1][d] -= pr * u[0][d];
  double n1 = sqrt((u[1][0] * u[1][0] + u[1][1] * u[1][1]) + u[1][2] * u[1][2]);
  if (!(n1 > 0.0)) { for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0; return; }
  for (int d = 0; d < 3; ++d) u[1][d] /= n1;
  u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
  u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
  u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      R[3 * i + j] = (u[0][i] * v[0][j] + u[1][i] * v[1][j]) + u[2][i] * v[2][j];
}

/* Dm^-1 of a tet from its rest positions p[4][3]; 0 if Dm is singular. */
static int arap_rest(const double *p0, const double *p1, const double *p2, const double *p3,
                     double *dm_inv) {
  double Dm[9];
  for (int d = 0; d < 3; ++d) {
    Dm[3 * d + 0] = p1[d] - p0[d];
    Dm[3 * d + 1] = p2[d] - p0[d];
    Dm[3 * d + 2] = p3[d] - p0[d];
  }
  return mat3_inverse(Dm, dm_inv);
}

/* C = |F - R|_F^2 and the four slot gradients g[4][3] of one ARAP row. */
static double arap_eval(const double *dm_inv, const double *x0, const double *x1,
                        const double *x2, const double *x3, double *g) {
  double Ds[9], F[9], R[9], P[9], DmT[9], H[9];
  for (int d = 0; d < 3; ++d) {
    Ds[3 * d + 0] = x1[d] - x0[d];
    Ds[3 * d + 1] = x2[d] - x0[d];
    Ds[3 * d + 2] = x3[d] - x0[d];
  }
  mat3_mul(Ds, dm_inv, F);
  orc_closest_rotation(F, R);
  double c = 0.0;
  for (int i = 0; i < 9; ++i) {
    double e = F[i] - R[i];
    c += e * e;
    P[i] = 2.0 * e;
  }
  mat3_transpose(dm_inv, DmT);
  mat3_mul(P, DmT, H);
  for (int k = 1; k <= 3; ++k)
    for (int d = 0; d < 3; ++d) g[3 * k + d] = H[3 * d + (k - 1)];
  for (int d = 0; d < 3; ++d) g[d] = -((g[3 + d] + g[6 + d]) + g[9 + d]);
  return c;
}

/* test hook: C and gradient of one ARAP tet from rest[4][3] and x[4][3];
   returns 0 for a singular rest shape */
int orc_arap_eval(const double *rest, const double *x, double *C, double *g) {
  double dm_inv[9];
  if (!arap_rest(rest, rest + 3, rest + 6, rest + 9, dm_inv)) return 0;
  *C = arap_eval(dm_inv, x, x + 3, x + 6, x + 9, g);
  return 1;
}

/* Constraint value and gradient of one row (Eq. 3 inputs).
   Edge (i, j): C = |x_i - x_j| - L0, g_i = n, g_j = -n.
   Volume (a, b, c, d): V = e1.(e2 x e3)/6, C = V - V0,
   g_b = (e2 x e3)/6, g_c = (e3 x e1)/6, g_d = (e1 x e2)/6, g_a = -(g_b + g_c + g_d).
   ARAP (a, b, c, d): C = |F - R|_F^2 (arap_eval). */
static double eval_row(const orc_sim *s, int64_t r, const double *pos, double *g /* [4][3] */) {
  const int32_t *v = s->rv + 4 * r;
  for (int k = 0; k < 12; ++k) g[k] = 0.0;
  if (s->arap[r])
    return arap_eval(s->dm_inv + 9 * r, pos + 3 * (int64_t)v[0], pos + 3 * (int64_t)v[1],
                     pos + 3 * (int64_t)v[2], pos + 3 * (int64_t)v[3], g);
  if (s->rk[r] == 2) {
    const double *xi = pos + 3 * (int64_t)v[0], *xj = pos + 3 * (int64_t)v[1];
    double dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
    double len = sqrt((dx * dx + dy * dy) + dz * dz);
    if (len > 0.0) {
      double nx = dx / len, ny = dy / len, nz = dz / len;
      g[0] = nx; g[1] = ny; g[2] = nz;
      g[3] = -nx; g[4] = -ny; g[5] = -nz;
    }
    return len;
  } else {
    const double *xa = pos + 3 * (int64_t)v[0], *xb = pos + 3 * (int64_t)v[1];
    const double *xc = pos + 3 * (int64_t)v[2], *xd = pos + 3 * (int64_t)v[3];
    double e1[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
    double e2[3] = {xc[0] - xa[0], xc[1] - xa[1], xc[2] - xa[2]};
    double e3[3] = {xd[0] - xa[0], xd[1] - xa[1], xd[2] - xa[2]};
    double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2],
                     e2[0] * e3[1] - e2[1] * e3[0]};
    double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2],
                     e3[0] * e1[1] - e3[1] * e1[0]};
    double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                     e1[0] * e2[1] - e1[1] * e2[0]};
    double vol = ((e1[0] * c23[0] + e1[1] * c23[1]) + e1[2] * c23[2]) / 6.0;
    for (int k = 0; k < 3; ++k) {
      g[3 + k] = c23[k] / 6.0;
      g[6 + k] = c31[k] / 6.0;
      g[9 + k] = c12[k] / 6.0;
      g[k] = -((g[3 + k] + g[6 + k]) + g[9 + k]);
    }
    return vol;
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Fixed pattern of A: (c, d) is stored iff rows c and d share a vertex
   (Sec. 4.2: precomputed once per topology), explicit zeros included. */
static int build_pattern(orc_sim *s) {
  int64_t m = s->m, N = s->n_verts;
  s->vc_ptr = calloc(N + 1, sizeof(int64_t));
  if (!s->vc_ptr) return ORC_E_NOMEM;
  for (int64_t r = 0; r < m; ++r)
    for (int k = 0; k < s->rk[r]; ++k) s->vc_ptr[s->rv[4 * r + k] + 1]++;
  for (int64_t v = 0; v < N; ++v) s->vc_ptr[v + 1] += s->vc_ptr[v];
  int64_t tot = s->vc_ptr[N];
  s->vc_row = malloc(sizeof(int32_t) * (tot ? tot : 1));
  s->vc_slot = malloc(sizeof(int32_t) * (tot ? tot : 1));
  int64_t *cur = malloc(sizeof(int64_t) * (N ? N : 1));
  if (!s->vc_row || !s->vc_slot || !cur) return ORC_E_NOMEM;
  memcpy(cur, s->vc_ptr, sizeof(int64_t) * N);
  for (int64_t r = 0; r < m; ++r)
    for (int k = 0; k < s->rk[r]; ++k) {
      int32_t v = s->rv[4 * r + k];
      s->vc_row[cur[v]] = (int32_t)r;
      s->vc_slot[cur[v]] = k;
      cur[v]++;
    }
  free(cur);
  /* rows */
  int32_t *mark = malloc(sizeof(int32_t) * (m ? m : 1));
  int32_t *buf = malloc(sizeof(int32_t) * 4096);
  s->A.n = m;
  s->A.rowptr = calloc(m + 1, sizeof(int64_t));
  if (!mark || !buf || !s->A.rowptr) return ORC_E_NOMEM;
  for (int64_t r = 0; r < m; ++r) mark[r] = -1;
  /* pass 1: counts */
  for (int64_t r = 0; r < m; ++r) {
    int64_t cnt = 0;
    for (int k = 0; k < s->rk[r]; ++k) {
      int32_t v = s->rv[4 * r + k];
      for (int64_t e = s->vc_ptr[v]; e < s->vc_ptr[v + 1]; ++e) {
        int32_t d = s->vc_row[e];
        if (mark[d] != (int32_t)r) { mark[d] = (int32_t)r; cnt++; }
      }
    }
    s->A.rowptr[r + 1] = s->A.rowptr[r] + cnt;
  }
  s->A.nnz = s->A.rowptr[m];
  s->A.col = malloc(sizeof(int32_t) * (s->A.nnz ? s->A.nnz : 1));
  s->A.val = calloc(s->A.nnz ? s->A.nnz : 1, sizeof(double));
  if (!s->A.col || !s->A.val) return ORC_E_NOMEM;
  for (int64_t r = 0; r < m; ++r) mark[r] = -1;
  for (int64_t r = 0; r < m; ++r) {
    int64_t cnt = s->A.rowptr[r];
    for (int k = 0; k < s->rk[r]; ++k) {
      int32_t v = s->rv[4 * r + k];
      for (int64_t e = s->vc_ptr[v]; e < s->vc_ptr[v + 1]; ++e) {
        int32_t d = s->vc_row[e];
        if (mark[d] != (int32_t)r) { mark[d] = (int32_t)r; s->A.col[cnt++] = d; }
      }
    }
    qsort(s->A.col + s->A.rowptr[r], (size_t)(s->A.rowptr[r + 1] - s->A.rowptr[r]),
          sizeof(int32_t), cmp_i32);
  }
  free(mark);
  free(buf);
  return ORC_OK;
}

void orc_sim_free(orc_sim *s);

orc_sim *orc_sim_create(int64_t n_verts, const double *rest, const double *inv_mass,
                        int64_t n_tets, const int32_t *tets, int64_t n_edges,
                        const int32_t *edges, int64_t n_vols, const int32_t *vol_tet,
                        int64_t n_arap, const int32_t *arap_tet,
                        const double *alpha, double dt, double gx, double gy, double gz,
                        const orc_opts *opts, int *status) {
  *status = ORC_E_INVALID;
  if (dt <= 0.0 || n_verts <= 0 || n_edges < 0 || n_vols < 0 || n_arap < 0 || n_tets < 0)
    return NULL;
  orc_sim *s = calloc(1, sizeof *s);
  if (!s) { *status = ORC_E_NOMEM; return NULL; }
  if (opts) s->o = *opts; else orc_default_opts(&s->o);
  s->n_verts = n_verts; s->n_tets = n_tets; s->n_edges = n_edges; s->n_vols = n_vols;
  s->n_arap = n_arap;
  s->m = n_edges + n_vols + n_arap;
  s->dt = dt; s->g[0] = gx; s->g[1] = gy; s->g[2] = gz;
  int64_t m = s->m;
  s->rest = malloc(sizeof(double) * 3 * n_verts);
  s->w = malloc(sizeof(double) * n_verts);
  s->tets = malloc(sizeof(int32_t) * 4 * (n_tets ? n_tets : 1));
  s->rv = malloc(sizeof(int32_t) * 4 * (m ? m : 1));
  s->rk = malloc(sizeof(int) * (m ? m : 1));
  s->arap = calloc(m ? m : 1, sizeof(int));
  s->dm_inv = calloc(9 * (m ? m : 1), sizeof(double));
  s->rest_c = malloc(sizeof(double) * (m ? m : 1));
  s->alpha_t = malloc(sizeof(double) * (m ? m : 1));
  s->lambda = calloc(m ? m : 1, sizeof(double));
  s->C = calloc(m ? m : 1, sizeof(double));
  s->grad = calloc(12 * (m ? m : 1), sizeof(double));
  s->b_last = calloc(m ? m : 1, sizeof(double));
  if (!s->rest || !s->w || !s->tets || !s->rv || !s->rk || !s->arap || !s->dm_inv ||
      !s->rest_c || !s->alpha_t ||
      !s->lambda || !s->C || !s->grad || !s->b_last) { orc_sim_free(s); *status = ORC_E_NOMEM; return NULL; }
  memcpy(s->rest, rest, sizeof(double) * 3 * n_verts);
  memcpy(s->w, inv_mass, sizeof(double) * n_verts);
  if (n_tets) memcpy(s->tets, tets, sizeof(int32_t) * 4 * n_tets);
  for (int64_t v = 0; v < n_verts; ++v)
    if (!(inv_mass[v] >= 0.0) || !isfinite(inv_mass[v]) || !isfinite(rest[3 * v]) ||
        !isfinite(rest[3 * v + 1]) || !isfinite(rest[3 * v + 2])) { orc_sim_free(s); return NULL; }
  double dt2 = dt * dt;
  for (int64_t e = 0; e < n_edges; ++e) {
    int32_t i = edges[2 * e], j = edges[2 * e + 1];
    if (i < 0 || j >= n_verts || i >= j) { orc_sim_free(s); return NULL; }
    if (e > 0) {
      int32_t pi = edges[2 * e - 2], pj = edges[2 * e - 1];
      if (pi > i || (pi == i && pj >= j)) { orc_sim_free(s); return NULL; }
    }
    s->rv[4 * e] = i; s->rv[4 * e + 1] = j; s->rv[4 * e + 2] = -1; s->rv[4 * e + 3] = -1;
    s->rk[e] = 2;
  }
  for (int64_t q = 0; q < n_vols; ++q) {
    int32_t t = vol_tet[q];
    if (t < 0 || t >= n_tets) { orc_sim_free(s); return NULL; }
    int64_t r = n_edges + q;
    for (int k = 0; k < 4; ++k) {
      int32_t v = tets[4 * (int64_t)t + k];
      if (v < 0 || v >= n_verts) { orc_sim_free(s); return NULL; }
      s->rv[4 * r + k] = v;
    }
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (s->rv[4 * r + a] == s->rv[4 * r + b]) { orc_sim_free(s); return NULL; }
    s->rk[r] = 4;
  }
  for (int64_t q = 0; q < n_arap; ++q) {
    int32_t t = arap_tet[q];
    if (t < 0 || t >= n_tets) { orc_sim_free(s); return NULL; }
    int64_t r = n_edges + n_vols + q;
    for (int k = 0; k < 4; ++k) {
      int32_t v = tets[4 * (int64_t)t + k];
      if (v < 0 || v >= n_verts) { orc_sim_free(s); return NULL; }
      s->rv[4 * r + k] = v;
    }
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (s->rv[4 * r + a] == s->rv[4 * r + b]) { orc_sim_free(s); return NULL; }
    s->rk[r] = 4;
    s->arap[r] = 1;
  }
  for (int64_t r = 0; r < m; ++r) {
    if (!(alpha[r] >= 0.0) || !isfinite(alpha[r])) { orc_sim_free(s); return NULL; }
    s->alpha_t[r] = alpha[r] / dt2;
    double g[12];
    if (s->arap[r]) {
      /* rest shape: Dm^-1, and a positive rest volume (positively oriented tet) */
      const int32_t *v = s->rv + 4 * r;
      const double *p0 = rest + 3 * (int64_t)v[0], *p1 = rest + 3 * (int64_t)v[1];
      const double *p2 = rest + 3 * (int64_t)v[2], *p3 = rest + 3 * (int64_t)v[3];
      double e1[3], e2[3], e3[3];
      for (int d = 0; d < 3; ++d) { e1[d] = p1[d] - p0[d]; e2[d] = p2[d] - p0[d]; e3[d] = p3[d] - p0[d]; }
      double vol6 = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                    e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
      if (!(vol6 > 0.0) || !arap_rest(p0, p1, p2, p3, s->dm_inv + 9 * r)) {
        orc_sim_free(s); return NULL;
      }
      s->rest_c[r] = 0.0;
      continue;
    }
    s->rest_c[r] = eval_row(s, r, rest, g);
    if (!(s->rest_c[r] > 0.0)) { orc_sim_free(s); return NULL; } /* zero edge / inverted tet */
  }
  int st = build_pattern(s);
  if (st != ORC_OK) { orc_sim_free(s); *status = st; return NULL; }
  *status = ORC_OK;
  return s;
}

int64_t orc_sim_rows(const orc_sim *s) { return s->m; }
int64_t orc_sim_nnz(const orc_sim *s) { return s->A.nnz; }

void orc_sim_pattern(const orc_sim *s, int64_t *rowptr, int32_t *col) {
  memcpy(rowptr, s->A.rowptr, sizeof(int64_t) * (s->m + 1));
  memcpy(col, s->A.col, sizeof(int32_t) * s->A.nnz);
}

/* C and grad C for all rows (Algorithm 1: constraint values and gradients) */
void orc_sim_constraints(orc_sim *s, const double *pos, double *C, double *grad) {
  for (int64_t r = 0; r < s->m; ++r) {
    double g[12];
    double v = eval_row(s, r, pos, g);
    C[r] = v - s->rest_c[r];
    if (grad) memcpy(grad + 12 * r, g, sizeof g);
  }
}

/* A and b (Eq. 3; per-entry form of Sec. 4.2). grad and C must be current.
   Diagonal: (sum over slots in local order of w_k (g_k . g_k)) + alpha~.
   Off-diagonal: sum over shared vertices in ascending vertex id of
   w_v (g_{c,v} . g_{d,v}). Dot products as (x x' + y y') + z z'. */
static void assemble(orc_sim *s, double *val, double *b) {
  for (int64_t c = 0; c < s->m; ++c) {
    const int32_t *vc = s->rv + 4 * c;
    const double *gc = s->grad + 12 * c;
    int kc = s->rk[c];
    /* slots of c sorted by vertex id */
    int ord[4] = {0, 1, 2, 3};
    for (int a = 1; a < kc; ++a)
      for (int q = a; q > 0 && vc[ord[q - 1]] > vc[ord[q]]; --q) {
        int t = ord[q]; ord[q] = ord[q - 1]; ord[q - 1] = t;
      }
    for (int64_t e = s->A.rowptr[c]; e < s->A.rowptr[c + 1]; ++e) {
      int64_t d = s->A.col[e];
      double acc;
      if (d == c) {
        acc = 0.0;
        for (int k = 0; k < kc; ++k) {
          const double *gk = gc + 3 * k;
          double gg = (gk[0] * gk[0] + gk[1] * gk[1]) + gk[2] * gk[2];
          double t = s->w[vc[k]] * gg;
          acc = (k == 0) ? t : acc + t;
        }
        acc = acc + s->alpha_t[c];
      } else {
        const int32_t *vd = s->rv + 4 * d;
        const double *gd = s->grad + 12 * d;
        int kd = s->rk[d];
        int first = 1;
        acc = 0.0;
        for (int a = 0; a < kc; ++a) {
          int sc = ord[a];
          int32_t v = vc[sc];
          for (int sd = 0; sd < kd; ++sd)
            if (vd[sd] == v) {
              const double *g1 = gc + 3 * sc, *g2 = gd + 3 * sd;
              double gg = (g1[0] * g2[0] + g1[1] * g2[1]) + g1[2] * g2[2];
              double t = s->w[v] * gg;
              acc = first ? t : acc + t;
              first = 0;
            }
        }
      }
      val[e] = acc;
    }
    b[c] = -s->C[c] - s->alpha_t[c] * s->lambda[c];
  }
}

/* test hook: A and b at the given positions and multipliers */
void orc_sim_assemble(orc_sim *s, const double *pos, const double *lambda, double *val,
                      double *b) {
  orc_sim_constraints(s, pos, s->C, s->grad);
  if (lambda) memcpy(s->lambda, lambda, sizeof(double) * s->m);
  else memset(s->lambda, 0, sizeof(double) * s->m);
  assemble(s, val, b);
}

/* ------------------------------------------------------------------ */
/* AMG setup (Sec. 4.1, 4.3, 4.5) and solve (Sec. 4.4)                 */
/* ------------------------------------------------------------------ */
typedef struct {
  csr A;
  double *diag;       /* A_ii */
  double omega;       /* Jacobi weight */
  double lmax;        /* lmax_scale * power-method estimate of lambda_max(D^-1 A) */
  /* transfer to level l+1 (absent on the last level) */
  int32_t *agg;       /* aggregate of each row, -1 = isolated */
  int64_t n_agg;
  int64_t *agg_ptr;   /* members of each aggregate, ascending */
  int32_t *agg_mem;
  /* P: the columns of aggregate q are the coarse unknowns coff[q] ..
     coff[q] + kq[q] - 1; member slot m (position in agg_mem) holds its row
     of P in Q[m K .. m K + kq - 1] (zeros beyond kq); slot[i] = slot of row i */
  int32_t *kq;
  int64_t *coff;
  int32_t *slot;
  double *Q;
  double *B;          /* near-kernel candidates on this level, [n][K] */
  int32_t *color;     /* level 0: multicolour GS order */
  int n_colors;
  /* Gauss-Seidel smoother: rows grouped by colour */
  int sm_colors;
  int64_t *sm_ptr;
  int32_t *sm_rows;
} level_t;

typedef struct {
  int L;              /* number of levels */
  level_t lev[32];
  int last_dense;     /* 1 if the last level is solved by dense Cholesky */
  double *chol;       /* dense lower factor of the last level, row major */
  int64_t nd;
  orc_opts o;
  /* scratch per level */
  double *tmp[32], *res[32], *rc[32], *zc[32], *dir[32];
} hier_t;

static void level_free(level_t *lv) {
  csr_free(&lv->A);
  free(lv->diag); free(lv->agg); free(lv->agg_ptr); free(lv->agg_mem);
  free(lv->kq); free(lv->coff); free(lv->slot); free(lv->Q);
  free(lv->B); free(lv->color); free(lv->sm_ptr); free(lv->sm_rows);
  memset(lv, 0, sizeof *lv);
}

void orc_hier_free(hier_t *h) {
  if (!h) return;
  for (int l = 0; l < h->L; ++l) {
    level_free(&h->lev[l]);
    free(h->tmp[l]); free(h->res[l]); free(h->rc[l]); free(h->zc[l]); free(h->dir[l]);
  }
  free(h->chol);
  free(h);
}

/* strength of connection: keep j != i iff a_ij^2 >= theta^2 |a_ii| |a_jj|
   (the filter of Sec. 4.1 squared; kept on equality) */
static int strong(double aij, double aii, double ajj, double theta2) {
  return aij * aij >= theta2 * (fabs(aii) * fabs(ajj));
}

typedef struct { uint64_t key; int32_t i; } kv_t;
static int cmp_kv_desc(const void *a, const void *b) {
  uint64_t x = ((const kv_t *)a)->key, y = ((const kv_t *)b)->key;
  return (x < y) - (x > y);
}

/* Aggregation (Sec. 4.1). prio[i] gives the visiting order (descending).
   Pass 1: greedy distance-2 independent set of roots over the strength graph;
   aggregate = root + its strong neighbours. Pass 2: each remaining connected
   node joins the pass-1 aggregate of its strongest strong neighbour. Nodes
   with no strong neighbour stay alone (agg = -1). Returns the count. */
int64_t orc_aggregate(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                      double theta, const uint64_t *prio, int32_t *agg, int32_t *is_root_out) {
  double theta2 = theta * theta;
  double *diag = malloc(sizeof(double) * (n ? n : 1));
  char *sflag = malloc(rowptr[n] ? rowptr[n] : 1);
  char *conn = calloc(n ? n : 1, 1);
  int32_t *root_of = malloc(sizeof(int32_t) * (n ? n : 1)); /* pass-1 aggregate root */
  char *blocked = calloc(n ? n : 1, 1);
  kv_t *ord = malloc(sizeof(kv_t) * (n ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    diag[i] = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      if (col[e] == i) diag[i] = val[e];
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = col[e];
      sflag[e] = (j != i) && strong(val[e], diag[i], diag[j], theta2);
      if (sflag[e]) conn[i] = 1;
    }
  int64_t no = 0;
  for (int64_t i = 0; i < n; ++i) {
    root_of[i] = -1;
    if (conn[i]) { ord[no].key = prio[i]; ord[no].i = (int32_t)i; no++; }
  }
  qsort(ord, (size_t)no, sizeof(kv_t), cmp_kv_desc);
  /* pass 1 */
  char *is_root = calloc(n ? n : 1, 1);
  for (int64_t q = 0; q < no; ++q) {
    int32_t i = ord[q].i;
    if (blocked[i]) continue;
    is_root[i] = 1;
    blocked[i] = 1;
    root_of[i] = i;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      if (!sflag[e]) continue;
      int32_t j = col[e];
      blocked[j] = 1;
      root_of[j] = i;
      for (int64_t f = rowptr[j]; f < rowptr[j + 1]; ++f)
        if (sflag[f]) blocked[col[f]] = 1;
    }
  }
  /* number aggregates by ascending root index */
  int32_t *num = malloc(sizeof(int32_t) * (n ? n : 1));
  int64_t na = 0;
  for (int64_t i = 0; i < n; ++i) num[i] = is_root[i] ? (int32_t)na++ : -1;
  if (is_root_out)
    for (int64_t i = 0; i < n; ++i) is_root_out[i] = is_root[i];
  int32_t *agg1 = malloc(sizeof(int32_t) * (n ? n : 1));
  for (int64_t i = 0; i < n; ++i) agg1[i] = root_of[i] >= 0 ? num[root_of[i]] : -1;
  /* pass 2 */
  for (int64_t i = 0; i < n; ++i) {
    agg[i] = agg1[i];
    if (agg1[i] >= 0 || !conn[i]) continue;
    double best = -1.0;
    int32_t bj = -1;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = col[e];
      if (!sflag[e] || agg1[j] < 0) continue;
      double a = fabs(val[e]);
      if (a > best) { best = a; bj = j; } /* ascending j: ties keep the smallest */
    }
    agg[i] = bj >= 0 ? agg1[bj] : -1;
  }
  free(diag); free(sflag); free(conn); free(root_of); free(blocked); free(ord);
  free(is_root); free(num); free(agg1);
  return na;
}

/* greedy colouring in descending priority over the structural graph:
   each node takes the smallest colour unused by its higher-priority neighbours */
int orc_color(int64_t n, const int64_t *rowptr, const int32_t *col, const uint64_t *prio,
              int32_t *color) {
  kv_t *ord = malloc(sizeof(kv_t) * (n ? n : 1));
  for (int64_t i = 0; i < n; ++i) { ord[i].key = prio[i]; ord[i].i = (int32_t)i; color[i] = -1; }
  qsort(ord, (size_t)n, sizeof(kv_t), cmp_kv_desc);
  int maxc = 0;
  int cap = 64;
  char *used = calloc(cap, 1);
  for (int64_t q = 0; q < n; ++q) {
    int32_t i = ord[q].i;
    int64_t deg = rowptr[i + 1] - rowptr[i];
    if (deg + 1 > cap) { cap = (int)deg + 1; free(used); used = calloc(cap, 1); }
    memset(used, 0, cap);
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t c = color[col[e]];
      if (col[e] != i && c >= 0 && c < cap) used[c] = 1;
    }
    int c = 0;
    while (used[c]) ++c;
    color[i] = c;
    if (c + 1 > maxc) maxc = c + 1;
  }
  free(used); free(ord);
  return maxc;
}

/* one multicolour Gauss-Seidel sweep on A x = 0: colours ascending, within a
   colour rows ascending, x_i <- -(sum_{j != i, ascending} a_ij x_j) / a_ii */
static void gs_sweep_homog(const csr *a, const double *diag, const int32_t *color, int nc,
                           const int64_t *cptr, const int32_t *crow, double *x) {
  (void)color;
  for (int c = 0; c < nc; ++c)
    for (int64_t q = cptr[c]; q < cptr[c + 1]; ++q) {
      int32_t i = crow[q];
      double s = 0.0;
      for (int64_t e = a->rowptr[i]; e < a->rowptr[i + 1]; ++e)
        if (a->col[e] != i) s = s + a->val[e] * x[a->col[e]];
      x[i] = (-s) / diag[i];
    }
}

/* Galerkin product A_c = P^T A P (Eq. 6). Coarse unknowns are the
   (aggregate, column) pairs (a, s), numbered coff[a] + s. The pattern of
   A_c: row (a, s) holds (b, t) for every aggregate b that some fine entry
   (i, j), agg(i) = a, agg(j) = b, reaches, and every t < kq[b]; columns
   ascending. Entry ((a, s), (b, t)) above or on the diagonal = sum over those
   fine entries, taken in ascending i then ascending j, of
   (Q_i,s a_ij) Q_j,t; an entry below the diagonal takes the value of its
   mirror above it (A_c is symmetric). With one candidate this is the sum
   of (p_i a_ij) p_j. */
static int galerkin_pattern(const csr *a, const int32_t *agg, int64_t na, const int32_t *kq,
                            const int64_t *coff, csr *c) {
  /* aggregate-level pattern first */
  int64_t *arp = calloc(na + 1, sizeof(int64_t));
  int32_t *mark = malloc(sizeof(int32_t) * (na ? na : 1));
  int64_t *mptr = calloc(na + 1, sizeof(int64_t));
  if (!arp || !mark || !mptr) { free(arp); free(mark); free(mptr); return ORC_E_NOMEM; }
  for (int64_t q = 0; q < na; ++q) mark[q] = -1;
  /* members of each aggregate, ascending: count then fill */
  for (int64_t i = 0; i < a->n; ++i) if (agg[i] >= 0) mptr[agg[i] + 1]++;
  for (int64_t q = 0; q < na; ++q) mptr[q + 1] += mptr[q];
  int32_t *mem = malloc(sizeof(int32_t) * (mptr[na] ? mptr[na] : 1));
  int64_t *cur = malloc(sizeof(int64_t) * (na ? na : 1));
  memcpy(cur, mptr, sizeof(int64_t) * na);
  for (int64_t i = 0; i < a->n; ++i) if (agg[i] >= 0) mem[cur[agg[i]]++] = (int32_t)i;
  for (int64_t q = 0; q < na; ++q) {
    int64_t cnt = 0;
    for (int64_t t = mptr[q]; t < mptr[q + 1]; ++t) {
      int32_t i = mem[t];
      for (int64_t e = a->rowptr[i]; e < a->rowptr[i + 1]; ++e) {
        int32_t b = agg[a->col[e]];
        if (b >= 0 && mark[b] != (int32_t)q) { mark[b] = (int32_t)q; cnt++; }
      }
    }
    arp[q + 1] = arp[q] + cnt;
  }
  int32_t *acol = malloc(sizeof(int32_t) * (arp[na] ? arp[na] : 1));
  for (int64_t q = 0; q < na; ++q) mark[q] = -1;
  for (int64_t q = 0; q < na; ++q) {
    int64_t k = arp[q];
    for (int64_t t = mptr[q]; t < mptr[q + 1]; ++t) {
      int32_t i = mem[t];
      for (int64_t e = a->rowptr[i]; e < a->rowptr[i + 1]; ++e) {
        int32_t b = agg[a->col[e]];
        if (b >= 0 && mark[b] != (int32_t)q) { mark[b] = (int32_t)q; acol[k++] = b; }
      }
    }
    qsort(acol + arp[q], (size_t)(arp[q + 1] - arp[q]), sizeof(int32_t), cmp_i32);
  }
  /* expand every aggregate entry (a, b) into the block of (a, s) x (b, t) */
  int64_t nc = coff[na];
  c->n = nc;
  c->rowptr = calloc(nc + 1, sizeof(int64_t));
  if (!c->rowptr) { free(arp); free(mark); free(mptr); free(mem); free(cur); free(acol); return ORC_E_NOMEM; }
  for (int64_t q = 0; q < na; ++q) {
    int64_t len = 0;
    for (int64_t e = arp[q]; e < arp[q + 1]; ++e) len += kq[acol[e]];
    for (int s = 0; s < kq[q]; ++s) c->rowptr[coff[q] + s + 1] = len;
  }
  for (int64_t r = 0; r < nc; ++r) c->rowptr[r + 1] += c->rowptr[r];
  c->nnz = c->rowptr[nc];
  c->col = malloc(sizeof(int32_t) * (c->nnz ? c->nnz : 1));
  c->val = calloc(c->nnz ? c->nnz : 1, sizeof(double));
  for (int64_t q = 0; q < na; ++q)
    for (int s = 0; s < kq[q]; ++s) {
      int64_t k = c->rowptr[coff[q] + s];
      for (int64_t e = arp[q]; e < arp[q + 1]; ++e)
        for (int t = 0; t < kq[acol[e]]; ++t) c->col[k++] = (int32_t)(coff[acol[e]] + t);
    }
  free(arp); free(mark); free(mptr); free(mem); free(cur); free(acol);
  return ORC_OK;
}

static int64_t find_col(const csr *c, int64_t row, int32_t colv) {
  int64_t lo = c->rowptr[row], hi = c->rowptr[row + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (c->col[mid] == colv) return mid;
    if (c->col[mid] < colv) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

static void galerkin_values(const csr *a, const level_t *lv, int K, csr *c) {
  for (int64_t k = 0; k < c->nnz; ++k) c->val[k] = 0.0;
  for (int64_t i = 0; i < a->n; ++i) {
    int32_t ai = lv->agg[i];
    if (ai < 0) continue;
    const double *qi = lv->Q + (int64_t)lv->slot[i] * K;
    for (int64_t e = a->rowptr[i]; e < a->rowptr[i + 1]; ++e) {
      int32_t j = a->col[e];
      int32_t bj = lv->agg[j];
      if (bj < 0) continue;
      const double *qj = lv->Q + (int64_t)lv->slot[j] * K;
      for (int s = 0; s < lv->kq[ai]; ++s) {
        int64_t r = lv->coff[ai] + s;
        for (int t = 0; t < lv->kq[bj]; ++t) {
          int64_t k = find_col(c, r, (int32_t)(lv->coff[bj] + t));
          c->val[k] = c->val[k] + (qi[s] * a->val[e]) * qj[t];
        }
      }
    }
  }
  /* keep the coarse matrix exactly symmetric: the entry below the diagonal
     takes the value accumulated for its mirror above it */
  for (int64_t q = 0; q < c->n; ++q)
    for (int64_t k = c->rowptr[q]; k < c->rowptr[q + 1]; ++k)
      if (c->col[k] < q) c->val[k] = c->val[find_col(c, c->col[k], (int32_t)q)];
}

/* lambda_max(D^-1 A) by the power method (Sec. 4.5) with a stopping test.
   v <- D^-1 A v / |D^-1 A v| from a positive pseudo-random start (stream 5).
   At step k = power_iters and then every POWER_CHECK steps, with w = A v_k:
   theta = v^T A v / v^T D v (the Rayleigh quotient), u = D^-1 w - theta v
   (the eigen-residual), and the method stops once
   |u|_D <= power_tol * theta * |v|_D, or at step power_max, returning theta.
   |x|_D = sqrt(x^T D x): D^-1 A is self-adjoint in that inner product, so a
   small residual means v is close to an eigenvector. */
#define POWER_CHECK 10
static double power_lmax(const csr *a, const double *diag, const orc_opts *o, int level) {
  int64_t n = a->n;
  double *v = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; ++i)
    v[i] = uniform01(o->seed, 5, ((uint64_t)level << 40) + (uint64_t)i);
  double theta = 0.0;
  for (int it = 0;; ++it) {
    spmv(a, v, w);
    int last = it >= o->power_max;
    if (last || (it >= o->power_iters && (it - o->power_iters) % POWER_CHECK == 0)) {
      double num = dot(n, v, w);
      double den = 0.0;
      for (int64_t i = 0; i < n; ++i) den += v[i] * diag[i] * v[i];
      theta = num / den;
      double res = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        double u = w[i] / diag[i] - theta * v[i];
        res += u * diag[i] * u;
      }
      if (last || sqrt(res) <= o->power_tol * theta * sqrt(den)) break;
    }
    for (int64_t i = 0; i < n; ++i) w[i] = w[i] / diag[i];
    double nrm = sqrt(dot(n, w, w));
    if (!(nrm > 0.0)) break;
    for (int64_t i = 0; i < n; ++i) v[i] = w[i] / nrm;
  }
  free(v); free(w);
  return theta;
}

static int dense_cholesky(hier_t *h) {
  level_t *lv = &h->lev[h->L - 1];
  int64_t n = lv->A.n;
  h->nd = n;
  free(h->chol);
  h->chol = calloc((size_t)((n > 0) ? n * n : 1), sizeof(double));
  double *Lm = h->chol;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = lv->A.rowptr[i]; e < lv->A.rowptr[i + 1]; ++e)
      Lm[i * n + lv->A.col[e]] = lv->A.val[e];
  for (int64_t j = 0; j < n; ++j) {
    double d = Lm[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= Lm[j * n + k] * Lm[j * n + k];
    if (!(d > 0.0)) return ORC_E_BREAKDOWN;
    double ljj = sqrt(d);
    Lm[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; ++i) {
      double s = Lm[i * n + j];
      for (int64_t k = 0; k < j; ++k) s -= Lm[i * n + k] * Lm[j * n + k];
      Lm[i * n + j] = s / ljj;
    }
    for (int64_t i = 0; i < j; ++i) Lm[i * n + j] = 0.0;
  }
  return ORC_OK;
}

static void chol_solve(const hier_t *h, const double *r, double *z) {
  int64_t n = h->nd;
  const double *Lm = h->chol;
  for (int64_t i = 0; i < n; ++i) {
    double s = r[i];
    for (int64_t k = 0; k < i; ++k) s -= Lm[i * n + k] * z[k];
    z[i] = s / Lm[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = z[i];
    for (int64_t k = i + 1; k < n; ++k) s -= Lm[k * n + i] * z[k];
    z[i] = s / Lm[i * n + i];
  }
}

static int copy_csr(csr *dst, int64_t n, const int64_t *rowptr, const int32_t *col,
                    const double *val) {
  dst->n = n;
  dst->nnz = rowptr[n];
  dst->rowptr = malloc(sizeof(int64_t) * (n + 1));
  dst->col = malloc(sizeof(int32_t) * (dst->nnz ? dst->nnz : 1));
  dst->val = malloc(sizeof(double) * (dst->nnz ? dst->nnz : 1));
  if (!dst->rowptr || !dst->col || !dst->val) return ORC_E_NOMEM;
  memcpy(dst->rowptr, rowptr, sizeof(int64_t) * (n + 1));
  memcpy(dst->col, col, sizeof(int32_t) * dst->nnz);
  memcpy(dst->val, val, sizeof(double) * dst->nnz);
  return ORC_OK;
}

/* Setup on the given fine matrix: strength, aggregation, near-kernel, P,
   Galerkin pattern and values, omega per level, dense factor of the last. */
static int finish_level(hier_t *h, int l) {
  level_t *lv = &h->lev[l];
  int64_t nl = lv->A.n;
  lv->diag = malloc(sizeof(double) * (nl ? nl : 1));
  h->tmp[l] = malloc(sizeof(double) * (nl ? nl : 1));
  h->res[l] = malloc(sizeof(double) * (nl ? nl : 1));
  h->rc[l] = malloc(sizeof(double) * (nl ? nl : 1));
  h->zc[l] = malloc(sizeof(double) * (nl ? nl : 1));
  h->dir[l] = malloc(sizeof(double) * (nl ? nl : 1));
  if (!lv->diag || !h->tmp[l] || !h->res[l] || !h->rc[l] || !h->zc[l] || !h->dir[l])
    return ORC_E_NOMEM;
  for (int64_t i = 0; i < nl; ++i) {
    lv->diag[i] = csr_get_diag(&lv->A, i);
    if (!(lv->diag[i] > 0.0)) return ORC_E_BREAKDOWN;
  }
  lv->lmax = nl ? h->o.lmax_scale * power_lmax(&lv->A, lv->diag, &h->o, l) : 0.0;
  lv->omega = nl ? 2.0 / (lv->lmax + h->o.lambda_min) : 0.0;
  if (h->o.smoother == 2) {
    /* rows of each colour in ascending order (greedy colouring in
       descending priority, the order the near-kernel sweeps use) */
    uint64_t *cp = malloc(sizeof(uint64_t) * (nl ? nl : 1));
    int32_t *color = malloc(sizeof(int32_t) * (nl ? nl : 1));
    if (!cp || !color) { free(cp); free(color); return ORC_E_NOMEM; }
    for (int64_t i = 0; i < nl; ++i) cp[i] = prio_key(h->o.seed, 4, l, i);
    lv->sm_colors = orc_color(nl, lv->A.rowptr, lv->A.col, cp, color);
    lv->sm_ptr = calloc(lv->sm_colors + 1, sizeof(int64_t));
    lv->sm_rows = malloc(sizeof(int32_t) * (nl ? nl : 1));
    if (!lv->sm_ptr || !lv->sm_rows) { free(cp); free(color); return ORC_E_NOMEM; }
    for (int64_t i = 0; i < nl; ++i) lv->sm_ptr[color[i] + 1]++;
    for (int c = 0; c < lv->sm_colors; ++c) lv->sm_ptr[c + 1] += lv->sm_ptr[c];
    int64_t *cur = malloc(sizeof(int64_t) * (lv->sm_colors ? lv->sm_colors : 1));
    memcpy(cur, lv->sm_ptr, sizeof(int64_t) * lv->sm_colors);
    for (int64_t i = 0; i < nl; ++i) lv->sm_rows[cur[color[i]]++] = (int32_t)i;
    free(cur); free(cp); free(color);
  }
  return ORC_OK;
}

/* QR of the K candidates restricted to one aggregate (its s rows, ascending)
   by modified Gram-Schmidt (Golub and Van Loan, Sec. 5.2.8): column k has
   its projections on the columns kept so far removed one after another, and
   is kept (normalised) unless what remains is at most ORC_QR_DROP of its
   norm, i.e. it is numerically dependent on the kept ones (always the case
   past s columns). Q [s][K] gets the kept columns (zeros beyond them), R
   [K][K] row j the coefficients of kept column j (R = Q^T B). A zero block
   keeps one normalised all-ones column with R[0][0] = sqrt(s). Returns the
   number of kept columns. With K = 1: Q = b / |b|, R = |b|. */
#define ORC_QR_DROP 1e-8
static int qr_aggregate(const double *B, int K, const int32_t *mem, int64_t s, double *Q,
                        double *R) {
  double *v = malloc(sizeof(double) * (s ? s : 1));
  int kept = 0;
  for (int k = 0; k < K; ++k) {
    double n0 = 0.0;
    for (int64_t t = 0; t < s; ++t) {
      v[t] = B[(int64_t)mem[t] * K + k];
      n0 = n0 + v[t] * v[t];
    }
    n0 = sqrt(n0);
    for (int j = 0; j < kept; ++j) {
      double r = 0.0;
      for (int64_t t = 0; t < s; ++t) r = r + Q[t * K + j] * v[t];
      R[j * K + k] = r;
      for (int64_t t = 0; t < s; ++t) v[t] = v[t] - r * Q[t * K + j];
    }
    double nr = 0.0;
    for (int64_t t = 0; t < s; ++t) nr = nr + v[t] * v[t];
    nr = sqrt(nr);
    if (nr > 0.0 && nr > ORC_QR_DROP * n0) {
      for (int64_t t = 0; t < s; ++t) Q[t * K + kept] = v[t] / nr;
      R[kept * K + k] = nr;
      ++kept;
    }
  }
  if (kept == 0) {
    double sa = sqrt((double)s);
    for (int64_t t = 0; t < s; ++t) Q[t * K] = 1.0 / sa;
    R[0] = sa;
    kept = 1;
  }
  free(v);
  return kept;
}

hier_t *orc_hier_build(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                       const orc_opts *opts, int *status) {
  hier_t *h = calloc(1, sizeof *h);
  if (!h) { *status = ORC_E_NOMEM; return NULL; }
  if (opts) h->o = *opts; else orc_default_opts(&h->o);
  const orc_opts *o = &h->o;
  if (o->max_levels < 1 || o->max_levels > 32 || o->n_cand < 1 || o->n_cand > 8 ||
      o->power_iters < 0 || o->power_max < 0 || !(o->power_tol >= 0.0)) {
    *status = ORC_E_INVALID; free(h); return NULL;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      if (col[e] < 0 || col[e] >= n || (e > rowptr[i] && col[e] <= col[e - 1])) {
        *status = ORC_E_INVALID; free(h); return NULL;
      }
  *status = copy_csr(&h->lev[0].A, n, rowptr, col, val);
  h->L = 1;
  if (*status != ORC_OK) { orc_hier_free(h); return NULL; }
  int force_last = 0, stalled = 0;
  for (int l = 0;; ++l) {
    level_t *lv = &h->lev[l];
    int64_t nl = lv->A.n;
    h->L = l + 1;
    *status = finish_level(h, l);
    if (*status != ORC_OK) { orc_hier_free(h); return NULL; }
    if (force_last || nl <= o->coarse_max || h->L >= o->max_levels) break;
    /* aggregation on the strength graph */
    uint64_t *prio = malloc(sizeof(uint64_t) * nl);
    for (int64_t i = 0; i < nl; ++i) prio[i] = prio_key(o->seed, 3, l, i);
    lv->agg = malloc(sizeof(int32_t) * nl);
    lv->n_agg = orc_aggregate(nl, lv->A.rowptr, lv->A.col, lv->A.val, o->theta, prio, lv->agg,
                              NULL);
    free(prio);
    int64_t na = lv->n_agg;
    if (na == 0) break; /* every row isolated: nothing to coarsen */
    /* candidate on this level: level 0 from Gauss-Seidel sweeps on A x = 0
       (Sec. 4.3) or all ones; deeper levels inherit the norms from above */
    const int K = o->n_cand;
    if (l == 0) {
      lv->B = malloc(sizeof(double) * nl * K);
      if (o->b_mode == 1) {
        for (int64_t i = 0; i < nl * K; ++i) lv->B[i] = 1.0;
      } else {
        double amax = 0.0;
        for (int64_t e = 0; e < lv->A.nnz; ++e)
          if (fabs(lv->A.val[e]) > amax) amax = fabs(lv->A.val[e]);
        uint64_t *cp = malloc(sizeof(uint64_t) * nl);
        for (int64_t i = 0; i < nl; ++i) cp[i] = prio_key(o->seed, 4, 0, i);
        lv->color = malloc(sizeof(int32_t) * nl);
        lv->n_colors = orc_color(nl, lv->A.rowptr, lv->A.col, cp, lv->color);
        free(cp);
        int64_t *cptr = calloc(lv->n_colors + 1, sizeof(int64_t));
        int32_t *crow = malloc(sizeof(int32_t) * nl);
        for (int64_t i = 0; i < nl; ++i) cptr[lv->color[i] + 1]++;
        for (int c = 0; c < lv->n_colors; ++c) cptr[c + 1] += cptr[c];
        int64_t *cc = malloc(sizeof(int64_t) * (lv->n_colors ? lv->n_colors : 1));
        memcpy(cc, cptr, sizeof(int64_t) * lv->n_colors);
        for (int64_t i = 0; i < nl; ++i) crow[cc[lv->color[i]]++] = (int32_t)i;
        /* candidate k: its own random start (index k 2^40 + i of stream 2),
           then the same sweeps */
        double *x = malloc(sizeof(double) * nl);
        for (int k = 0; k < K; ++k) {
          for (int64_t i = 0; i < nl; ++i)
            x[i] = uniform01(o->seed, 2, ((uint64_t)k << 40) + (uint64_t)i) * amax;
          for (int s = 0; s < o->gs_sweeps; ++s)
            gs_sweep_homog(&lv->A, lv->diag, lv->color, lv->n_colors, cptr, crow, x);
          for (int64_t i = 0; i < nl; ++i) lv->B[i * K + k] = x[i];
        }
        free(x); free(cptr); free(crow); free(cc);
      }
    }
    /* injection: QR of the candidates restricted to each aggregate (Sec. 4.1):
       Q -> the aggregate's columns of P, R -> the next level's candidates */
    lv->agg_ptr = calloc(na + 1, sizeof(int64_t));
    lv->agg_mem = malloc(sizeof(int32_t) * (nl ? nl : 1));
    for (int64_t i = 0; i < nl; ++i) if (lv->agg[i] >= 0) lv->agg_ptr[lv->agg[i] + 1]++;
    for (int64_t q = 0; q < na; ++q) lv->agg_ptr[q + 1] += lv->agg_ptr[q];
    {
      int64_t *cur = malloc(sizeof(int64_t) * na);
      memcpy(cur, lv->agg_ptr, sizeof(int64_t) * na);
      for (int64_t i = 0; i < nl; ++i)
        if (lv->agg[i] >= 0) lv->agg_mem[cur[lv->agg[i]]++] = (int32_t)i;
      free(cur);
    }
    int64_t nmem = lv->agg_ptr[na];
    lv->slot = malloc(sizeof(int32_t) * (nl ? nl : 1));
    for (int64_t i = 0; i < nl; ++i) lv->slot[i] = -1;
    for (int64_t m = 0; m < nmem; ++m) lv->slot[lv->agg_mem[m]] = (int32_t)m;
    lv->Q = calloc((size_t)(nmem ? nmem : 1) * K, sizeof(double));
    lv->kq = calloc(na ? na : 1, sizeof(int32_t));
    lv->coff = calloc(na + 1, sizeof(int64_t));
    double *R = calloc((size_t)(na ? na : 1) * K * K, sizeof(double));
    for (int64_t q = 0; q < na; ++q) {
      int kept = qr_aggregate(lv->B, K, lv->agg_mem + lv->agg_ptr[q],
                              lv->agg_ptr[q + 1] - lv->agg_ptr[q],
                              lv->Q + lv->agg_ptr[q] * K, R + q * K * K);
      lv->kq[q] = kept;
      lv->coff[q + 1] = lv->coff[q] + kept;
    }
    int64_t nnext = lv->coff[na];
    double *Bn = malloc(sizeof(double) * (nnext ? nnext : 1) * K);
    for (int64_t q = 0; q < na; ++q)
      for (int j = 0; j < lv->kq[q]; ++j)
        for (int k = 0; k < K; ++k) Bn[(lv->coff[q] + j) * K + k] = R[(q * K + j) * K + k];
    free(R);
    level_t *nx = &h->lev[l + 1];
    *status = galerkin_pattern(&lv->A, lv->agg, na, lv->kq, lv->coff, &nx->A);
    if (*status != ORC_OK) { free(Bn); orc_hier_free(h); return NULL; }
    galerkin_values(&lv->A, lv, K, &nx->A);
    nx->B = Bn;
    if ((double)nnext > 0.95 * (double)nl) force_last = stalled = 1; /* coarsening stalled */
  }
  level_t *last = &h->lev[h->L - 1];
  if (last->A.n <= o->dense_max) {
    h->last_dense = 1;
    *status = dense_cholesky(h);
    if (*status != ORC_OK) { orc_hier_free(h); return NULL; }
  } else if (!stalled) {
    /* every row isolated, or the level cap reached: the smoother is the
       last-level solver */
    h->last_dense = 0;
  } else {
    *status = ORC_E_SETUP; orc_hier_free(h); return NULL;
  }
  *status = ORC_OK;
  return h;
}

/* Solving phase (Sec. 4.4): refresh A_0 values, rebuild every coarse level by
   the Galerkin product and refactor the last level. P and omega are kept. */
int orc_hier_refresh(hier_t *h, const double *val0) {
  memcpy(h->lev[0].A.val, val0, sizeof(double) * h->lev[0].A.nnz);
  for (int l = 0; l < h->L; ++l) {
    level_t *lv = &h->lev[l];
    for (int64_t i = 0; i < lv->A.n; ++i) lv->diag[i] = csr_get_diag(&lv->A, i);
    if (l + 1 < h->L) galerkin_values(&lv->A, lv, h->o.n_cand, &h->lev[l + 1].A);
  }
  for (int l = 0; l < h->L; ++l)
    for (int64_t i = 0; i < h->lev[l].A.n; ++i)
      if (!(h->lev[l].diag[i] > 0.0)) return ORC_E_BREAKDOWN;
  if (h->last_dense) return dense_cholesky(h);
  return ORC_OK;
}

/* Multicolour Gauss-Seidel sweeps for A z = r on level l: within a colour the
   rows are independent, z_i <- (r_i - sum_{j != i, ascending} a_ij z_j) / a_ii;
   colours in ascending order (forward) or descending order (backward). */
static void gs_smooth(hier_t *h, int l, const double *r, double *z, int sweeps, int backward) {
  level_t *lv = &h->lev[l];
  const csr *a = &lv->A;
  for (int s = 0; s < sweeps; ++s)
    for (int q = 0; q < lv->sm_colors; ++q) {
      int c = backward ? lv->sm_colors - 1 - q : q;
      for (int64_t t = lv->sm_ptr[c]; t < lv->sm_ptr[c + 1]; ++t) {
        int32_t i = lv->sm_rows[t];
        double acc = 0.0;
        for (int64_t e = a->rowptr[i]; e < a->rowptr[i + 1]; ++e)
          if (a->col[e] != i) acc = acc + a->val[e] * z[a->col[e]];
        z[i] = (r[i] - acc) / lv->diag[i];
      }
    }
}

/* Chebyshev smoothing on level l: `steps` steps of Chebyshev acceleration of
   Jacobi for A z = r on the eigenvalue interval [a, b] = [lambda_min, lmax]
   of D^-1 A: theta = (b + a)/2, delta = (b - a)/2, sigma = theta/delta,
   rho_0 = 1/sigma, d_0 = (1/theta) D^-1 (r - A z_0), z_1 = z_0 + d_0, and for
   k >= 1: rho_k = 1/(2 sigma - rho_{k-1}),
   d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D^-1 (r - A z_k),
   z_{k+1} = z_k + d_k. from_zero: z_0 = 0 (no product in the first step). */
static void cheb_smooth(hier_t *h, int l, const double *r, double *z, int steps, int from_zero) {
  level_t *lv = &h->lev[l];
  int64_t n = lv->A.n;
  double *t = h->tmp[l], *d = h->dir[l];
  double a = h->o.lambda_min, b = lv->lmax;
  double theta = (b + a) / 2.0, delta = (b - a) / 2.0, sigma = theta / delta;
  double rho = 1.0 / sigma;
  for (int k = 0; k < steps; ++k) {
    double c1 = 0.0, c2 = 1.0 / theta;
    if (k > 0) {
      double rho_new = 1.0 / (2.0 * sigma - rho);
      c1 = rho_new * rho;
      c2 = 2.0 * rho_new / delta;
      rho = rho_new;
    }
    if (k == 0 && from_zero) {
      for (int64_t i = 0; i < n; ++i) {
        d[i] = c2 * (r[i] / lv->diag[i]);
        z[i] = d[i];
      }
      continue;
    }
    spmv(&lv->A, z, t);
    for (int64_t i = 0; i < n; ++i) {
      double ri = (r[i] - t[i]) / lv->diag[i];
      d[i] = (k == 0) ? c2 * ri : c1 * d[i] + c2 * ri;
      z[i] = z[i] + d[i];
    }
  }
}

/* one V-cycle z = V(l, r): pre-smoothing from z = 0, residual, restriction
   P^T, coarse correction, prolongation, post-smoothing; Jacobi sweeps or
   Chebyshev steps */
static void vcycle(hier_t *h, int l, const double *r, double *z) {
  level_t *lv = &h->lev[l];
  int64_t n = lv->A.n;
  if (l == h->L - 1 && h->last_dense) { chol_solve(h, r, z); return; }
  double om = lv->omega;
  double *t = h->tmp[l];
  const int cheb = h->o.smoother == 1, gs = h->o.smoother == 2;
  if (h->o.pre_sweeps == 0) {
    for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
  } else if (gs) {
    for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
    gs_smooth(h, l, r, z, h->o.pre_sweeps, 0);
  } else if (cheb) {
    cheb_smooth(h, l, r, z, h->o.pre_sweeps, 1);
  } else {
    for (int64_t i = 0; i < n; ++i) z[i] = om * (r[i] / lv->diag[i]);
    for (int s = 1; s < h->o.pre_sweeps; ++s) {
      spmv(&lv->A, z, t);
      for (int64_t i = 0; i < n; ++i) z[i] = z[i] + om * ((r[i] - t[i]) / lv->diag[i]);
    }
  }
  if (l + 1 < h->L) {
    double *res = h->res[l];
    spmv(&lv->A, z, t);
    for (int64_t i = 0; i < n; ++i) res[i] = r[i] - t[i];
    int64_t na = lv->n_agg;
    const int K = h->o.n_cand;
    double *rc = h->rc[l + 1], *zc = h->zc[l + 1];
    /* restriction P^T res: coarse unknown (q, s) sums Q_i,s res_i over the
       aggregate's rows in ascending order */
    for (int64_t q = 0; q < na; ++q)
      for (int s = 0; s < lv->kq[q]; ++s) {
        double acc = 0.0;
        for (int64_t m = lv->agg_ptr[q]; m < lv->agg_ptr[q + 1]; ++m)
          acc = acc + lv->Q[m * K + s] * res[lv->agg_mem[m]];
        rc[lv->coff[q] + s] = acc;
      }
    vcycle(h, l + 1, rc, zc);
    /* prolongation z += P zc */
    for (int64_t i = 0; i < n; ++i) {
      int32_t q = lv->agg[i];
      if (q < 0) continue;
      const double *qi = lv->Q + (int64_t)lv->slot[i] * K;
      double acc = 0.0;
      for (int s = 0; s < lv->kq[q]; ++s) acc = acc + qi[s] * zc[lv->coff[q] + s];
      z[i] = z[i] + acc;
    }
  }
  if (gs) {
    gs_smooth(h, l, r, z, h->o.post_sweeps, 1);
  } else if (cheb) {
    cheb_smooth(h, l, r, z, h->o.post_sweeps, 0);
  } else {
    for (int s = 0; s < h->o.post_sweeps; ++s) {
      spmv(&lv->A, z, t);
      for (int64_t i = 0; i < n; ++i) z[i] = z[i] + om * ((r[i] - t[i]) / lv->diag[i]);
    }
  }
}

void orc_hier_vcycle(hier_t *h, const double *r, double *z) { vcycle(h, 0, r, z); }

int orc_hier_levels(const hier_t *h) { return h->L; }
int orc_hier_last_dense(const hier_t *h) { return h->last_dense; }

void orc_hier_level_info(const hier_t *h, int l, int64_t *n, int64_t *nnz, double *omega,
                         int64_t *n_agg, int *n_colors) {
  const level_t *lv = &h->lev[l];
  *n = lv->A.n; *nnz = lv->A.nnz; *omega = lv->omega;
  *n_agg = lv->agg ? lv->n_agg : -1;
  *n_colors = lv->n_colors;
}

void orc_hier_level_matrix(const hier_t *h, int l, int64_t *rowptr, int32_t *col, double *val) {
  const level_t *lv = &h->lev[l];
  if (rowptr) memcpy(rowptr, lv->A.rowptr, sizeof(int64_t) * (lv->A.n + 1));
  if (col) memcpy(col, lv->A.col, sizeof(int32_t) * lv->A.nnz);
  if (val) memcpy(val, lv->A.val, sizeof(double) * lv->A.nnz);
}

/* agg, P's first column (one value per row, 0 for isolated rows) and the
   first candidate of level l (only for levels that have a coarser one) */
int orc_hier_level_transfer(const hier_t *h, int l, int32_t *agg, double *p, double *B) {
  const level_t *lv = &h->lev[l];
  const int K = h->o.n_cand;
  if (!lv->agg) return ORC_E_INVALID;
  if (agg) memcpy(agg, lv->agg, sizeof(int32_t) * lv->A.n);
  for (int64_t i = 0; i < lv->A.n; ++i) {
    if (p) p[i] = lv->slot[i] >= 0 ? lv->Q[(int64_t)lv->slot[i] * K] : 0.0;
    if (B) B[i] = lv->B[i * K];
  }
  return ORC_OK;
}

/* the full transfer of level l: kq [n_agg], coff [n_agg + 1], Q [members][K]
   (member order of the ascending aggregate lists), candidates B [n][K] */
int orc_hier_level_qr(const hier_t *h, int l, int32_t *kq, int64_t *coff, double *Q, double *B) {
  const level_t *lv = &h->lev[l];
  const int K = h->o.n_cand;
  if (!lv->agg) return ORC_E_INVALID;
  if (kq) memcpy(kq, lv->kq, sizeof(int32_t) * lv->n_agg);
  if (coff) memcpy(coff, lv->coff, sizeof(int64_t) * (lv->n_agg + 1));
  if (Q) memcpy(Q, lv->Q, sizeof(double) * lv->agg_ptr[lv->n_agg] * K);
  if (B) memcpy(B, lv->B, sizeof(double) * lv->A.n * K);
  return ORC_OK;
}

/* z = A_L^-1 r with the last level's dense Cholesky factor (a test hook; the
   V-cycle applies the same solve at the last level) */
int orc_hier_coarse_solve(const hier_t *h, const double *r, double *z) {
  if (!h->last_dense) return ORC_E_INVALID;
  chol_solve(h, r, z);
  return ORC_OK;
}

int orc_hier_colors(const hier_t *h, int32_t *color) {
  const level_t *lv = &h->lev[0];
  if (!lv->color) return ORC_E_INVALID;
  memcpy(color, lv->color, sizeof(int32_t) * lv->A.n);
  return lv->n_colors;
}

/* MGPCG (Sec. 4.4): x0 = 0, one V-cycle per iteration as preconditioner
   (identity when precond == 0). force_iters > 0 runs exactly that many
   iterations. Returns ORC_OK, ORC_E_NOT_CONVERGED or ORC_E_BREAKDOWN. */
int orc_pcg(hier_t *h, const double *b, double tol, int max_iters, int precond,
            int force_iters, double *x, int *iters_out, double *ratio_out) {
  const csr *a = &h->lev[0].A;
  int64_t n = a->n;
  double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
  double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
  double *zold = malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
  double bn = sqrt(dot(n, b, b));
  int st = ORC_OK, it = 0;
  double ratio = 0.0;
  if (bn == 0.0) goto done;
  if (precond) vcycle(h, 0, r, z); else memcpy(z, r, sizeof(double) * n);
  memcpy(p, z, sizeof(double) * n);
  double rho = dot(n, r, z);
  int cap = force_iters > 0 ? force_iters : max_iters;
  st = ORC_E_NOT_CONVERGED;
  while (it < cap) {
    if (!(rho > 0.0)) { st = ORC_E_BREAKDOWN; break; }
    spmv(a, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0)) { st = ORC_E_BREAKDOWN; break; }
    double alpha = rho / pq;
    for (int64_t i = 0; i < n; ++i) { x[i] = x[i] + alpha * p[i]; r[i] = r[i] - alpha * q[i]; }
    ++it;
    ratio = sqrt(dot(n, r, r)) / bn;
    if (force_iters > 0) { if (it == force_iters) { st = ORC_OK; break; } }
    else if (ratio <= tol) { st = ORC_OK; break; }
    if (h->o.flexible) memcpy(zold, z, sizeof(double) * n);
    if (precond) vcycle(h, 0, r, z); else memcpy(z, r, sizeof(double) * n);
    double rz = dot(n, r, z);
    double beta;
    if (h->o.flexible) {
      double s = 0.0;
      for (int64_t i = 0; i < n; ++i) s += r[i] * (z[i] - zold[i]);
      beta = s / rho;
    } else {
      beta = rz / rho;
    }
    rho = rz;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
done:
  if (iters_out) *iters_out = it;
  if (ratio_out) *ratio_out = ratio;
  free(r); free(z); free(p); free(q); free(zold);
  return st;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: one frame                                              */
/* ------------------------------------------------------------------ */
void orc_sim_free(orc_sim *s) {
  if (!s) return;
  free(s->rest); free(s->w); free(s->tets); free(s->rv); free(s->rk); free(s->rest_c);
  free(s->arap); free(s->dm_inv);
  free(s->alpha_t); free(s->lambda); free(s->C); free(s->grad); free(s->b_last);
  free(s->vc_ptr); free(s->vc_row); free(s->vc_slot);
  csr_free(&s->A);
  orc_hier_free((hier_t *)s->hier);
  free(s);
}

void *orc_sim_hier(orc_sim *s) { return s->hier; }
const double *orc_sim_lambda_ptr(orc_sim *s) { return s->lambda; }
void orc_sim_get_lambda(const orc_sim *s, double *out) { memcpy(out, s->lambda, sizeof(double) * s->m); }
void orc_sim_get_matrix_values(const orc_sim *s, double *val) {
  memcpy(val, s->A.val, sizeof(double) * s->A.nnz);
}
void orc_sim_set_frame(orc_sim *s, int64_t f) { s->frame = f; }
void orc_sim_get_rhs(const orc_sim *s, double *b) { memcpy(b, s->b_last, sizeof(double) * s->m); }
void orc_sim_invalidate(orc_sim *s) { orc_hier_free((hier_t *)s->hier); s->hier = NULL; }

/* pos[N][3], vel[N][3] in/out. Per iteration outputs (nullable, length
   n_iters): |b|, PCG iterations, final PCG residual ratio, and whether setup
   ran. force_pcg (nullable) fixes the PCG iteration count per iteration. */
int orc_sim_step(orc_sim *s, double *pos, double *vel, int n_iters, double *bnorm_out,
                 int *pcg_iters_out, double *ratio_out, int *setup_out, const int *force_pcg) {
  int64_t N = s->n_verts, m = s->m;
  double dt = s->dt;
  for (int64_t v = 0; v < N; ++v)
    for (int k = 0; k < 3; ++k)
      if (!isfinite(pos[3 * v + k]) || !isfinite(vel[3 * v + k])) return ORC_E_INVALID;
  double *xold = malloc(sizeof(double) * 3 * N);
  double *b = malloc(sizeof(double) * (m ? m : 1));
  double *dl = malloc(sizeof(double) * (m ? m : 1));
  /* semi-implicit Euler predict (Algorithm 1, Eq. 1) */
  for (int64_t v = 0; v < N; ++v)
    for (int k = 0; k < 3; ++k) {
      xold[3 * v + k] = pos[3 * v + k];
      if (s->w[v] > 0.0) {
        vel[3 * v + k] = vel[3 * v + k] + dt * s->g[k];
        pos[3 * v + k] = pos[3 * v + k] + dt * vel[3 * v + k];
      }
    }
  memset(s->lambda, 0, sizeof(double) * (m ? m : 1));
  int st = ORC_OK;
  for (int ite = 0; ite < n_iters; ++ite) {
    orc_sim_constraints(s, pos, s->C, s->grad);
    assemble(s, s->A.val, b);
    double bn = sqrt(dot(m, b, b));
    if (bnorm_out) bnorm_out[ite] = bn;
    memcpy(s->b_last, b, sizeof(double) * m);
    int R = s->o.reuse_interval;
    int due = (s->hier == NULL) || (R <= 0) || (ite == 0 && (s->frame % R) == 0);
    if (setup_out) setup_out[ite] = due;
    if (due) {
      orc_hier_free((hier_t *)s->hier);
      s->hier = orc_hier_build(m, s->A.rowptr, s->A.col, s->A.val, &s->o, &st);
      if (!s->hier) break;
    } else {
      st = orc_hier_refresh((hier_t *)s->hier, s->A.val);
      if (st != ORC_OK) break;
    }
    int its = 0;
    double ratio = 0.0;
    int ps = orc_pcg((hier_t *)s->hier, b, s->o.tol, s->o.max_pcg, 1,
                     force_pcg ? force_pcg[ite] : 0, dl, &its, &ratio);
    if (ps == ORC_E_BREAKDOWN && !due && s->o.resetup_on_breakdown) {
      /* the lazy setup (Sec. 4.2) keeps the hierarchy and the smoother weights
         of Sec. 4.5 while they still precondition A; once they do not (the
         V-cycle is no longer positive definite for this A), set up afresh for
         the current A and solve this iteration again */
      if (setup_out) setup_out[ite] = 2;
      orc_hier_free((hier_t *)s->hier);
      s->hier = orc_hier_build(m, s->A.rowptr, s->A.col, s->A.val, &s->o, &st);
      if (!s->hier) break;
      its = 0;
      ratio = 0.0;
      ps = orc_pcg((hier_t *)s->hier, b, s->o.tol, s->o.max_pcg, 1,
                   force_pcg ? force_pcg[ite] : 0, dl, &its, &ratio);
    }
    if (pcg_iters_out) pcg_iters_out[ite] = its;
    if (ratio_out) ratio_out[ite] = ratio;
    if (ps == ORC_E_BREAKDOWN) { st = ps; break; }
    /* dx = M^-1 gradC^T dlambda (Eq. 5), gathered per vertex over its rows
       in ascending order; lambda += dlambda; x += omega dx */
    for (int64_t v = 0; v < N; ++v) {
      double sx = 0.0, sy = 0.0, sz = 0.0;
      for (int64_t e = s->vc_ptr[v]; e < s->vc_ptr[v + 1]; ++e) {
        int32_t r = s->vc_row[e];
        const double *g = s->grad + 12 * (int64_t)r + 3 * s->vc_slot[e];
        sx = sx + g[0] * dl[r];
        sy = sy + g[1] * dl[r];
        sz = sz + g[2] * dl[r];
      }
      double wv = s->w[v];
      pos[3 * v + 0] = pos[3 * v + 0] + s->o.omega_relax * (wv * sx);
      pos[3 * v + 1] = pos[3 * v + 1] + s->o.omega_relax * (wv * sy);
      pos[3 * v + 2] = pos[3 * v + 2] + s->o.omega_relax * (wv * sz);
    }
    for (int64_t r = 0; r < m; ++r) s->lambda[r] = s->lambda[r] + dl[r];
    if (bn < s->o.eps_b) break;
  }
  /* v = (x - x_old) / dt, the velocity update that ends Algorithm 1 */
  for (int64_t v = 0; v < N; ++v)
    for (int k = 0; k < 3; ++k) vel[3 * v + k] = (pos[3 * v + k] - xold[3 * v + k]) / dt;
  s->frame++;
  free(xold); free(b); free(dl);
  return st;
}
