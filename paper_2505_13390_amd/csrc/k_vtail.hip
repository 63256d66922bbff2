// The fused coarse end of the V-cycle (Sec. 4.4-4.5): one workgroup per body
// runs the body's levels from the tail's start level down to its dense
// coarsest solve and back up. See tail.hpp.
#include "rowops.hpp"
#include "tail.hpp"

namespace mgpbd {

// One row pass over rows [r0, r0 + n) of a level: G lanes per row, strided
// loads, fixed-tree lane sum, then the epilogue (the order of k_rows).
template <int G, class T, class In, class Op>
__device__ void tail_rows_g(int64_t r0, int64_t n, const TailLevel<T> &L, In x, Op op) {
  constexpr int R = kTailBlock / G;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G;
  double acc = 0.0;
  for (int64_t base = r0; base < r0 + n; base += R) {
    const int64_t i = base + grp;
    const bool ok = i < r0 + n;
    const int64_t a = ok ? L.rp[i] : 0, b = ok ? L.rp[i + 1] : 0;
    T s = 0;
#pragma unroll 4
    for (int64_t e = a + sub; e < b; e += G) s += L.val[e] * x(L.col[e]);
    s = group_sum<G, T>(s);
    if (ok && sub == 0) op(i, s, acc);
  }
}
template <class T, class In, class Op>
__device__ void tail_rows(int64_t r0, int64_t n, const TailLevel<T> &L, In x, Op op) {
  switch (L.G) {
    case 4: tail_rows_g<4>(r0, n, L, x, op); break;
    case 8: tail_rows_g<8>(r0, n, L, x, op); break;
    case 16: tail_rows_g<16>(r0, n, L, x, op); break;
    case 32: tail_rows_g<32>(r0, n, L, x, op); break;
    default: tail_rows_g<64>(r0, n, L, x, op); break;
  }
  __syncthreads();
}

// rc[a] = sum over the members i of aggregate a (ascending) of p_i res_i for
// the aggregates [a0, a0 + na), RL lanes per aggregate (the order of k_restrict)
template <int RL, class T>
__device__ void tail_restrict_g(int64_t a0, int64_t na, const TailLevel<T> &L, T *rc) {
  constexpr int R = kTailBlock / RL;
  const int sub = threadIdx.x % RL, grp = threadIdx.x / RL;
  for (int64_t base = a0; base < a0 + na; base += R) {
    const int64_t a = base + grp;
    const bool ok = a < a0 + na;
    const int64_t b0 = ok ? L.agg_ptr[a] : 0, b1 = ok ? L.agg_ptr[a + 1] : 0;
    T s = 0;
    for (int64_t k = b0 + sub; k < b1; k += RL) {
      const int32_t i = L.agg_mem[k];
      s += L.p[i] * L.res[i];
    }
    s = group_sum<RL>(s);
    if (ok && sub == 0) rc[a] = s;
  }
}
template <class T>
__device__ void tail_restrict(int64_t a0, int64_t na, const TailLevel<T> &L, T *rc) {
  switch (L.rlanes) {
    case 64: tail_restrict_g<64>(a0, na, L, rc); break;
    case 32: tail_restrict_g<32>(a0, na, L, rc); break;
    case 16: tail_restrict_g<16>(a0, na, L, rc); break;
    default: tail_restrict_g<8>(a0, na, L, rc); break;
  }
  __syncthreads();
}

// z = Ainv r on the body's last level: one wavefront per row, lane-strided
// products summed by the wave tree (the order of k_dense_apply_batch)
template <class T>
__device__ void tail_dense(int64_t r0, int64_t n, const double *__restrict__ Ai0,
                           const TailLevel<T> &L) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave, nw = kTailBlock / kWave;
  for (int64_t i = wave; i < n; i += nw) {
    const double *Ai = Ai0 + i * n;
    double s = 0.0;
    for (int64_t k = lane; k < n; k += kWave) s += Ai[k] * (double)L.r[r0 + k];
    s = group_sum<kWave>(s);
    if (lane == 0) L.z[r0 + i] = (T)s;
  }
  __syncthreads();
}

template <class T>
__global__ __launch_bounds__(kTailBlock) void k_vcycle_tail(const TailLevel<T> *__restrict__ lv,
                                                            const TailBody *__restrict__ bodies,
                                                            TailPlan plan,
                                                            const double *__restrict__ ainv,
                                                            const int *done) {
  if (done && *done) return;
  const TailBody &B = bodies[blockIdx.x];
  const int depth = B.depth;
  const bool cheb = plan.smoother == 1;
  const bool fuse = plan.fuse_first && !cheb;
  const int pre = plan.pre, post = plan.post;
  // which of (z, t) holds each level's iterate, and the next write target:
  // the iterate ping-pongs so that the last write of the level lands in z
  const int pre_writes = pre == 0 ? 1 : (fuse && pre >= 2) ? pre - 1 : pre;
  const int writes = pre_writes + post;
  const int w0 = (writes % 2) ? 0 : 1;
  // after pre-smoothing (the same on every level): the buffer holding the
  // iterate and the write counter
  const int c_pre = (w0 + pre_writes - 1) % 2, w_pre = w0 + pre_writes;
  auto buf = [&](const TailLevel<T> &L, int k) { return k ? L.t : L.z; };
  // one smoothing step k from zi into zo over the body's rows of level L
  auto sweep = [&](const TailLevel<T> &L, int64_t r0, int64_t n, int k, const T *zi, T *zo) {
    const InVec<T> in{zi};
    if (cheb)
      tail_rows<T>(r0, n, L, in,
                   OpCheb<T, InVec<T>>{L.r, L.dinv, L.dir, zo, L.cheb, L.rowseg, plan.steps, k,
                                       in});
    else
      tail_rows<T>(r0, n, L, in, OpJacobi<T, InVec<T>>{L.wdinv, L.r, in, zo});
  };

  // down: pre-smoothing, residual, restriction
  int j = 0;
  for (; j < depth; ++j) {
    const TailLevel<T> &L = lv[j];
    const int64_t r0 = B.row0[j], n = B.n[j];
    if (j == depth - 1) {
      tail_dense<T>(r0, n, ainv + B.ainv, L);
      break;
    }
    int w = w0;
    int c = (w++) % 2;
    T *zc = buf(L, c);
    int k0 = 1;
    if (pre == 0) {
      for (int64_t i = r0 + threadIdx.x; i < r0 + n; i += kTailBlock) zc[i] = (T)0;
      __syncthreads();
    } else if (cheb) {
      for (int64_t i = r0 + threadIdx.x; i < r0 + n; i += kTailBlock) {
        const T c2 = L.cheb[2 * (int64_t)(L.rowseg ? L.rowseg[i] : 0) * plan.steps + 1];
        const T dn = c2 * (L.r[i] * L.dinv[i]);
        L.dir[i] = dn;
        zc[i] = dn;
      }
      __syncthreads();
    } else if (fuse && pre >= 2) {
      const InScaled<T> in{L.r, L.wdinv};
      tail_rows<T>(r0, n, L, in, OpJacobi<T, InScaled<T>>{L.wdinv, L.r, in, zc});
      k0 = 2;
    } else {
      for (int64_t i = r0 + threadIdx.x; i < r0 + n; i += kTailBlock) zc[i] = L.r[i] * L.wdinv[i];
      __syncthreads();
    }
    for (int k = k0; k < pre; ++k) {
      const int o = (w++) % 2;
      sweep(L, r0, n, k, buf(L, c), buf(L, o));
      c = o;
    }
    tail_rows<T>(r0, n, L, InVec<T>{buf(L, c)}, OpResidual<T>{L.r, L.res});
    tail_restrict<T>(B.row0[j + 1], B.n[j + 1], L, lv[j + 1].r);
  }
  // up: prolongation, post-smoothing
  for (j = depth - 2; j >= 0; --j) {
    const TailLevel<T> &L = lv[j];
    const int64_t r0 = B.row0[j], n = B.n[j];
    int c = c_pre, w = w_pre;
    T *zc = buf(L, c);
    const T *ec = lv[j + 1].z;
    for (int64_t i = r0 + threadIdx.x; i < r0 + n; i += kTailBlock) {
      const int32_t a = L.agg[i];
      if (a >= 0) zc[i] = zc[i] + L.p[i] * ec[a];
    }
    __syncthreads();
    for (int k = 0; k < post; ++k) {
      const int o = (w++) % 2;
      sweep(L, r0, n, k, buf(L, c), buf(L, o));
      c = o;
    }
  }
}

template <class T>
void launch_vcycle_tail(int nbodies, const TailLevel<T> *levels, const TailBody *bodies,
                        const TailPlan &plan, const double *ainv, const int *done,
                        hipStream_t s) {
  if (nbodies <= 0) return;
  k_vcycle_tail<T><<<nbodies, kTailBlock, 0, s>>>(levels, bodies, plan, ainv, done);
}

template void launch_vcycle_tail<double>(int, const TailLevel<double> *, const TailBody *,
                                         const TailPlan &, const double *, const int *,
                                         hipStream_t);
template void launch_vcycle_tail<float>(int, const TailLevel<float> *, const TailBody *,
                                        const TailPlan &, const double *, const int *,
                                        hipStream_t);

}  // namespace mgpbd
