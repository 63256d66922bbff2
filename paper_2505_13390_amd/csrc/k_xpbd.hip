// Kernels of the simulation loop (Algorithm 1) around the linear solve:
// semi-implicit Euler predict, constraint values and gradients, assembly of
// A = gradC M^-1 gradC^T + alpha~ and b = -C - alpha~ lambda into the fixed
// pattern (Eq. 3, per-entry form of Sec. 4.2), dx = M^-1 gradC^T dlambda
// (Eq. 5) gathered per vertex, lambda += dlambda, and the velocity update.
// Positions and velocities are SoA FP64 arrays.
#include "grad.hpp"
#include "xpbd.hpp"

namespace mgpbd {

__global__ void k_predict(int64_t nv, const double *__restrict__ w, double gx, double gy,
                          double gz, double dt, double *__restrict__ x, double *__restrict__ y,
                          double *__restrict__ z, double *__restrict__ vx, double *__restrict__ vy,
                          double *__restrict__ vz, double *__restrict__ xo,
                          double *__restrict__ yo, double *__restrict__ zo) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double px = x[v], py = y[v], pz = z[v];
  xo[v] = px; yo[v] = py; zo[v] = pz;
  if (w[v] > 0.0) {
    double ux = vx[v] + dt * gx, uy = vy[v] + dt * gy, uz = vz[v] + dt * gz;
    vx[v] = ux; vy[v] = uy; vz[v] = uz;
    x[v] = px + dt * ux; y[v] = py + dt * uy; z[v] = pz + dt * uz;
  }
}
void launch_predict(int64_t nv, const double *w, const double *g, double dt, double *const *xyz,
                    double *const *vxyz, double *const *oxyz, hipStream_t s) {
  if (nv)
    k_predict<<<blocks_for(nv, kBlock), kBlock, 0, s>>>(nv, w, g[0], g[1], g[2], dt, xyz[0], xyz[1],
                                                        xyz[2], vxyz[0], vxyz[1], vxyz[2], oxyz[0],
                                                        oxyz[1], oxyz[2]);
}

// C and gradient of each row (formulas in grad.hpp): edge C = |x_i - x_j| - L0,
// volume C = e1.(e2 x e3)/6 - V0.
__global__ void k_constraints(int64_t m, const int32_t *__restrict__ rv,
                              const int8_t *__restrict__ kind,
                              const double *__restrict__ rest_c, const double *__restrict__ x,
                              const double *__restrict__ y, const double *__restrict__ z,
                              double *__restrict__ C, double *__restrict__ grad) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m || (kind && kind[r])) return;
  const int32_t *v = rv + 4 * r;
  double g[4][3];
  double val;
  if (v[2] < 0) {   // edge rows pad slots 2 and 3 with -1
    const int32_t i = v[0], j = v[1];
    const double pi[3] = {x[i], y[i], z[i]}, pj[3] = {x[j], y[j], z[j]};
    val = edge_grads(pi, pj, g[0], g[1]);
#pragma unroll
    for (int d = 0; d < 3; ++d) g[2][d] = g[3][d] = 0.0;
  } else {
    double p[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int32_t q = v[k];
      p[k][0] = x[q];
      p[k][1] = y[q];
      p[k][2] = z[q];
    }
    val = tet_grads(p[0], p[1], p[2], p[3], g) / 6.0;
  }
  C[r] = val - rest_c[r];
  double *go = grad + 12 * r;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) go[3 * k + d] = g[k][d];
}
void launch_constraints(int64_t m, const int32_t *rv, const int8_t *kind, const double *rest_c,
                        const double *const *xyz, double *C, double *grad, hipStream_t s) {
  if (m)
    k_constraints<<<blocks_for(m, kBlock), kBlock, 0, s>>>(m, rv, kind, rest_c, xyz[0], xyz[1],
                                                           xyz[2], C, grad);
}

// Entry (c, d) of A. meta == 0 marks the diagonal; otherwise bits 0-2 hold
// the number of shared vertices and bits 3 + 4t .. 6 + 4t the local slots
// (slot in c | slot in d << 2) of the t-th shared vertex in ascending vertex id.
template <int G>
__global__ __launch_bounds__(kBlock) void k_assemble(
    int64_t m, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
    const uint32_t *__restrict__ meta, const int32_t *__restrict__ rv,
    const double *__restrict__ w, const double *__restrict__ grad,
    const double *__restrict__ alpha_t, const double *__restrict__ C,
    const double *__restrict__ lambda, double *__restrict__ val, float *__restrict__ val32,
    double *__restrict__ b) {
  constexpr int R = kBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  int64_t lo, hi;
  block_range(m, lo, hi);
  for (int64_t base = lo; base < hi; base += R) {
    int64_t c = base + grp;
    if (c >= hi) continue;
    const double *gc = grad + 12 * c;
    const int32_t *vc = rv + 4 * c;
    const int kc = vc[2] < 0 ? 2 : 4;
    for (int64_t e = rp[c] + sub; e < rp[c + 1]; e += G) {
      uint32_t code = meta[e];
      double acc;
      if (code == 0) {
        acc = 0.0;
        for (int k = 0; k < kc; ++k) {
          const double *gk = gc + 3 * k;
          double gg = (gk[0] * gk[0] + gk[1] * gk[1]) + gk[2] * gk[2];
          double t = w[vc[k]] * gg;
          acc = (k == 0) ? t : acc + t;
        }
        acc = acc + alpha_t[c];
      } else {
        const double *gd = grad + 12 * (int64_t)col[e];
        int cnt = code & 7;
        acc = 0.0;
        for (int t = 0; t < cnt; ++t) {
          int sc = (code >> (3 + 4 * t)) & 3, sd = (code >> (5 + 4 * t)) & 3;
          const double *g1 = gc + 3 * sc, *g2 = gd + 3 * sd;
          double gg = (g1[0] * g2[0] + g1[1] * g2[1]) + g1[2] * g2[2];
          double term = w[vc[sc]] * gg;
          acc = (t == 0) ? term : acc + term;
        }
      }
      val[e] = acc;
      if (val32) val32[e] = (float)acc;
    }
    if (sub == 0) b[c] = -C[c] - alpha_t[c] * lambda[c];
  }
}
void launch_assemble(int64_t m, int lanes, const int64_t *rp, const int32_t *col,
                     const uint32_t *meta, const int32_t *rv, const double *w, const double *grad,
                     const double *alpha_t, const double *C, const double *lambda, double *val,
                     float *val32, double *b, hipStream_t s) {
  if (!m) return;
  int grid = grid_for(m * lanes, kBlock);
#define L_(G)                                                                                   \
  k_assemble<G><<<grid, kBlock, 0, s>>>(m, rp, col, meta, rv, w, grad, alpha_t, C, \
                                        lambda, val, val32, b)
  switch (lanes) {
    case 8: L_(8); break;
    case 32: L_(32); break;
    default: L_(16); break;
  }
#undef L_
}

// dx_v = w_v sum over rows c containing v (ascending) of g_{c,v} dlambda_c;
// x_v += omega dx_v
__global__ void k_dx_update(int64_t nv, const int64_t *__restrict__ vptr,
                            const int32_t *__restrict__ vrow, const int8_t *__restrict__ vslot,
                            const double *__restrict__ grad, const double *__restrict__ dl,
                            const double *__restrict__ w, double omega, double *__restrict__ x,
                            double *__restrict__ y, double *__restrict__ z) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int64_t e = vptr[v]; e < vptr[v + 1]; ++e) {
    int32_t r = vrow[e];
    const double *g = grad + 12 * (int64_t)r + 3 * vslot[e];
    double d = dl[r];
    sx = sx + g[0] * d;
    sy = sy + g[1] * d;
    sz = sz + g[2] * d;
  }
  double wv = w[v];
  x[v] = x[v] + omega * (wv * sx);
  y[v] = y[v] + omega * (wv * sy);
  z[v] = z[v] + omega * (wv * sz);
}
void launch_dx_update(int64_t nv, const int64_t *vptr, const int32_t *vrow, const int8_t *vslot,
                      const double *grad, const double *dl, const double *w, double omega,
                      double *const *xyz, hipStream_t s) {
  if (nv)
    k_dx_update<<<blocks_for(nv, kBlock), kBlock, 0, s>>>(nv, vptr, vrow, vslot, grad, dl, w, omega,
                                                          xyz[0], xyz[1], xyz[2]);
}

__global__ void k_axpy_inplace(int64_t n, double *__restrict__ a, const double *__restrict__ d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = a[i] + d[i];
}
// concatenation of bodies: index arrays shifted by the offset of their body
__global__ void k_offset_i32(int64_t n, const int32_t *__restrict__ in, int32_t add,
                             int32_t *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t v = in[i];
  out[i] = v >= 0 ? v + add : v;
}
__global__ void k_offset_i64(int64_t n, const int64_t *__restrict__ in, int64_t add,
                             int64_t *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] + add;
}
void launch_offset_copy(int64_t n, const int32_t *in, int32_t add, int32_t *out, hipStream_t s) {
  if (n) k_offset_i32<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, in, add, out);
}
void launch_offset_copy(int64_t n, const int64_t *in, int64_t add, int64_t *out, hipStream_t s) {
  if (n) k_offset_i64<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, in, add, out);
}

void launch_lambda_add(int64_t m, double *lambda, const double *dl, hipStream_t s) {
  if (m) k_axpy_inplace<<<blocks_for(m, kBlock), kBlock, 0, s>>>(m, lambda, dl);
}

__global__ void k_velocity(int64_t nv, double dt, const double *__restrict__ x,
                           const double *__restrict__ y, const double *__restrict__ z,
                           const double *__restrict__ xo, const double *__restrict__ yo,
                           const double *__restrict__ zo, double *__restrict__ vx,
                           double *__restrict__ vy, double *__restrict__ vz) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  vx[v] = (x[v] - xo[v]) / dt;
  vy[v] = (y[v] - yo[v]) / dt;
  vz[v] = (z[v] - zo[v]) / dt;
}
void launch_velocity(int64_t nv, double dt, double *const *xyz, double *const *oxyz,
                     double *const *vxyz, hipStream_t s) {
  if (nv)
    k_velocity<<<blocks_for(nv, kBlock), kBlock, 0, s>>>(nv, dt, xyz[0], xyz[1], xyz[2], oxyz[0],
                                                         oxyz[1], oxyz[2], vxyz[0], vxyz[1], vxyz[2]);
}

__global__ void k_check_finite(int64_t n, const double *__restrict__ a, int *bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double v = a[i];
    if (!(v == v) || v > 1.7976931348623157e308 || v < -1.7976931348623157e308) atomicExch(bad, 1);
  }
}
void launch_check_finite(int64_t n, const double *a, int *bad, hipStream_t s) {
  if (n) k_check_finite<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, a, bad);
}

// IEEE check hook: s = sqrt(a), q = a / b (used by the tests to confirm that
// the device's FP64 square root and division round correctly)
__global__ void k_sqrt_div(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                           double *__restrict__ s, double *__restrict__ q) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  s[i] = sqrt(a[i]);
  q[i] = a[i] / b[i];
}
void launch_sqrt_div(int64_t n, const double *a, const double *b, double *s, double *q,
                     hipStream_t st) {
  if (n) k_sqrt_div<<<blocks_for(n, kBlock), kBlock, 0, st>>>(n, a, b, s, q);
}

}  // namespace mgpbd
