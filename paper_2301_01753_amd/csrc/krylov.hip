// Krylov kernels: preconditioned MINRES and CG with device-resident scalars.
//
// The paper's exact-FEEC equations of motion need M1^{-1} (eq. exactEOM): a
// global solve (section 3), done here by CG with a diagonal preconditioner
// (the preconditioner type the paper uses for its own PCG, section 5.1).
// The symmetric indefinite block operators are solved by MINRES with a
// symmetric positive block-diagonal preconditioner.
//
// Determinism: every dot product is a two-stage reduction with a fixed
// order (per-block tree, then every consumer block re-reduces the same
// partials in the same order), accumulated in FP64 whatever the vector type.
// No atomics.  The scalar recurrences run redundantly in every block of the
// kernel that needs them; block 0 alone writes the next state slot (double
// buffered: kernels read slot it&1 and write slot (it+1)&1).
#include <hip/hip_runtime.h>

#include <cmath>

#include "krylov.hpp"

namespace gym {

constexpr int kBT = 256;

template <typename T>
__device__ __forceinline__ double todbl(T v) { return static_cast<double>(v); }

// Block sum of `v` (fixed order, see wg_sums); returned in every thread.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  double a[1] = {v};
  wg_sums<kBT, 1>(a, sh);
  return a[0];
}

// Sum of `np` partials, same order in every block.
__device__ __forceinline__ double reduce_partials(const double* part, int np, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += kBT) v += part[i];
  return block_sum(v, sh);
}

// ---- MINRES ---------------------------------------------------------------
// init: r1 = r2 = b; y = dinv .* b; x = w = w1 = w2 = 0; partial (b . y)
template <typename TV>
__global__ void __launch_bounds__(kBT) minres_init_a(MinresVecs<TV> v, const double* __restrict__ dinv,
                                                     long long n, double* part) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  const long long off = (long long)rhs * n;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    TV bi = v.b[off + i];
    double yi = dinv[i] * todbl(bi);
    v.r1[off + i] = bi;
    v.r2[off + i] = bi;
    v.y[off + i] = static_cast<TV>(yi);
    v.x[off + i] = 0;
    v.w[off + i] = 0;
    v.w1[off + i] = 0;
    v.w2[off + i] = 0;
    acc += todbl(bi) * yi;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[rhs * gridDim.x + blockIdx.x] = s;
}

// init: beta1 = sqrt(b . M^-1 b); v = y / beta1
template <typename TV>
__global__ void __launch_bounds__(kBT) minres_init_b(MinresVecs<TV> v, long long n, const double* part,
                                                     int np, MinresState* st0, double tol) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  const long long off = (long long)rhs * n;
  double b2 = reduce_partials(part + rhs * np, np, sh);
  double beta1 = b2 > 0 ? sqrt(b2) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    MinresState s{};
    s.beta1 = beta1;
    s.beta = beta1;
    s.oldb = 0;
    s.dbar = 0;
    s.epsln = 0;
    s.phibar = beta1;
    s.cs = -1;
    s.sn = 0;
    s.tnorm2 = 0;
    s.tol = tol;
    s.itn = 0;
    s.done = (beta1 == 0.0) ? 1 : 0;
    s.flag = (b2 < 0 || b2 != b2) ? -1 : 0;
    if (s.flag) s.done = 1;
    st0[rhs] = s;
  }
  double inv = beta1 > 0 ? 1.0 / beta1 : 0.0;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    v.v[off + i] = static_cast<TV>(todbl(v.y[off + i]) * inv);
}

// Non-diagonal preconditioner: r1 = r2 = b, x = w = w1 = w2 = 0
template <typename TV>
__global__ void __launch_bounds__(kBT) minres_init_vecs(MinresVecs<TV> v, long long n) {
  const long long off = (long long)blockIdx.y * n;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    const TV bi = v.b[off + i];
    v.r1[off + i] = bi;
    v.r2[off + i] = bi;
    v.x[off + i] = 0;
    v.w[off + i] = 0;
    v.w1[off + i] = 0;
    v.w2[off + i] = 0;
  }
}

// per block: pb = y . z, pc = z . r (r may be null); nothing for a
// right-hand side whose state in gate (if given) has converged
template <typename TV>
__global__ void __launch_bounds__(kBT) minres_dot2(const TV* __restrict__ y, const TV* __restrict__ z,
                                                   const TV* __restrict__ r, long long n, double* pb, double* pc,
                                                   const MinresState* gate) {
  __shared__ double sh[2 * kBT];
  if (gate && gate[blockIdx.y].done) return;
  const long long off = (long long)blockIdx.y * n;
  double a = 0.0, c = 0.0;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    const double zi = todbl(z[off + i]);
    a += todbl(y[off + i]) * zi;
    if (r) c += zi * todbl(r[off + i]);
  }
  double t[2] = {a, c};
  wg_sums<kBT, 2>(t, sh);
  if (threadIdx.x == 0) {
    pb[(long long)blockIdx.y * gridDim.x + blockIdx.x] = t[0];
    if (pc) pc[(long long)blockIdx.y * gridDim.x + blockIdx.x] = t[1];
  }
}

// Second kernel of a fused MINRES step.  The operator kernel left
// y = A z_k and per-workgroup partial sums pa of z_k . A z_k.  Every block:
//   1. closes step k-1 (unless `first`): scalar update of state cur with
//      alfa_{k-1} and the sums of the previous pass's partials (beta_k^2 from
//      pb_prev, z_k . r1_k from pc_prev); block 0 stores the state in next;
//   2. alfa_k = (z.Az) / beta_k^2 - (beta_k / beta_{k-1}) (z_k . r1_k) / beta_k;
//   3. one pass over the vectors: y = (A z_k) / beta_k - (beta_k / beta_{k-1}) r1
//      - (alfa_k / beta_k) r2, z_{k+1} = dinv .* y written over zp, step k-1's
//      w_{k-1} = (v_{k-1} - oldeps w_{k-3} - delta w_{k-2}) / gamma with
//      v_{k-1} = zp / beta_{k-1} (zp is read before it is overwritten),
//      x += phi w_{k-1}; partial sums of y . z_{k+1} and z_{k+1} . r2 into
//      pb, pc.
// A converged state is copied forward and nothing else is done.
struct Step2Coef {
  double ys, c1, c, vpinv, phi, denom, oldeps, delta;
};

template <typename TV, bool UPD, bool EXT>
__device__ __forceinline__ void step2_sweep(const MrVecs<TV>& v, const double* __restrict__ dinv, long long n,
                                            long long off, const Step2Coef& k, int blk, int nblk, double& ab,
                                            double& ac) {
  // restrict-qualified locals let the compiler issue every load of an
  // unrolled group before the stores of the previous one.  The stores are
  // non-temporal: the four written vectors are read again only in the next
  // step, after the whole sweep, far beyond what the caches hold (measured
  // on a 95M-unknown Hodge solve: 2% faster per step at 1 rhs, 3.7% at 8;
  // non-temporal loads helped at 1 rhs and hurt at 8)
  TV* __restrict__ y = v.y + off;
  const TV* __restrict__ r1 = v.r1 + off;
  const TV* __restrict__ r2 = v.r2 + off;
  TV* __restrict__ zp = v.zp + off;
  TV* __restrict__ x = v.x + off;
  const TV* __restrict__ wa = v.wa + off;
  const TV* __restrict__ wb = v.wb + off;
  TV* __restrict__ wo = v.wout + off;
  constexpr int U = 4;
  const long long stride = (long long)nblk * kBT;
  long long i0 = (long long)blk * kBT + threadIdx.x;
  auto one = [&](long long i, double yv, double r1v, double r2v, double dv, double zpv, double wav, double wbv,
                 double xv) {
    const TV ys = static_cast<TV>(k.ys * yv - k.c1 * r1v - k.c * r2v);
    __builtin_nontemporal_store(ys, &y[i]);
    if constexpr (UPD) {
      const double vp = todbl(static_cast<TV>(zpv * k.vpinv));
      const TV ws = static_cast<TV>((vp - k.oldeps * wav - k.delta * wbv) * k.denom);
      __builtin_nontemporal_store(ws, &wo[i]);
      __builtin_nontemporal_store(static_cast<TV>(xv + k.phi * todbl(ws)), &x[i]);
    }
    if constexpr (!EXT) {
      const TV zs = static_cast<TV>(dv * todbl(ys));
      __builtin_nontemporal_store(zs, &zp[i]);
      ab += todbl(ys) * todbl(zs);
      ac += todbl(zs) * r2v;
    }
  };
  for (; i0 + (U - 1) * stride < n; i0 += U * stride) {
    double yv[U], r1v[U], r2v[U], dv[U], zpv[U], wav[U], wbv[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * stride;
      yv[u] = todbl(y[i]);
      r1v[u] = todbl(r1[i]);
      r2v[u] = todbl(r2[i]);
      dv[u] = EXT ? 0.0 : dinv[i];
      if constexpr (UPD) {
        zpv[u] = todbl(zp[i]);
        wav[u] = todbl(wa[i]);
        wbv[u] = todbl(wb[i]);
        xv[u] = todbl(x[i]);
      } else {
        zpv[u] = wav[u] = wbv[u] = xv[u] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) one(i0 + u * stride, yv[u], r1v[u], r2v[u], dv[u], zpv[u], wav[u], wbv[u], xv[u]);
  }
  for (; i0 < n; i0 += stride) {
    if constexpr (UPD)
      one(i0, todbl(y[i0]), todbl(r1[i0]), todbl(r2[i0]), EXT ? 0.0 : dinv[i0], todbl(zp[i0]), todbl(wa[i0]),
          todbl(wb[i0]), todbl(x[i0]));
    else
      one(i0, todbl(y[i0]), todbl(r1[i0]), todbl(r2[i0]), EXT ? 0.0 : dinv[i0], 0.0, 0.0, 0.0, 0.0);
  }
}

// blk / nblk: this block and the blocks of this right-hand side.
template <typename TV>
__device__ __forceinline__ void step2_body(const MrVecs<TV>& v, const double* __restrict__ dinv, long long n,
                                           const Step2Io& io, int rhs, int blk, int nblk, double* sh) {
  const bool lead = blk == 0 && threadIdx.x == 0;
  MinresState s = io.cur[rhs];
  if (s.done) {
    if (lead) io.next[rhs] = s;
    return;
  }
  Step2Coef k{};
  double zr1 = 0.0;
  k.vpinv = s.beta > 0 ? 1.0 / s.beta : 0.0;  // 1 / beta_{k-1}
  // the three sums in one block reduction: beta_k^2, z_k . r1_k, z_k . A z_k
  double t3[3] = {0.0, 0.0, 0.0};
  if (!io.first) {
    const double* pb = io.pb_prev + (long long)rhs * io.npb;
    const double* pc = io.pc_prev + (long long)rhs * io.npb;
    for (int i = threadIdx.x; i < io.npb; i += kBT) {
      t3[0] += pb[i];
      t3[1] += pc[i];
    }
  }
  const double* pa = io.pa + (long long)rhs * io.npa;
  for (int i = threadIdx.x; i < io.npa; i += kBT) t3[2] += pa[i];
  wg_sums<kBT, 3>(t3, sh);
  if (!io.first) {
    zr1 = t3[1];
    double vinv;
    minres_scalar_update(s, io.alfa_prev[rhs], t3[0], k.phi, k.denom, k.oldeps, k.delta, vinv);
  }
  if (lead) io.next[rhs] = s;
  const double vinv = s.beta > 0 ? 1.0 / s.beta : 0.0;  // 1 / beta_k
  k.c1 = s.oldb > 0 ? s.beta / s.oldb : 0.0;
  const double zaz = t3[2];
  const double alfa = vinv * vinv * zaz - k.c1 * zr1 * vinv;
  if (lead) io.alfa[rhs] = alfa;
  k.ys = vinv;
  k.c = alfa * vinv;
  const long long off = (long long)rhs * n;
  double ab = 0.0, ac = 0.0;
  if (io.ext) {
    // y and the w, x updates only: z_{k+1} = M^-1 y and its partial sums
    // follow in the caller's kernels
    if (io.first) step2_sweep<TV, false, true>(v, dinv, n, off, k, blk, nblk, ab, ac);
    else step2_sweep<TV, true, true>(v, dinv, n, off, k, blk, nblk, ab, ac);
    return;
  }
  if (io.first) step2_sweep<TV, false, false>(v, dinv, n, off, k, blk, nblk, ab, ac);
  else step2_sweep<TV, true, false>(v, dinv, n, off, k, blk, nblk, ab, ac);
  double t2[2] = {ab, ac};
  wg_sums<kBT, 2>(t2, sh);
  if (threadIdx.x == 0) {
    io.pb[(long long)rhs * nblk + blk] = t2[0];
    io.pc[(long long)rhs * nblk + blk] = t2[1];
  }
}

template <typename TV>
__global__ void __launch_bounds__(kBT) minres_step2(MrVecs<TV> v, const double* __restrict__ dinv, long long n,
                                                    Step2Io io) {
  __shared__ double sh[3 * kBT];
  step2_body<TV>(v, dinv, n, io, blockIdx.y, blockIdx.x, gridDim.x, sh);
}

// Completes a pending step without a further apply (iteration cap reached):
// scalar update, w_k = (v_{k-1} - oldeps w_{k-2} - delta w_{k-1}) / gamma over
// wout, x += phi w_k.  Converged states are copied forward.
template <typename TV>
__global__ void __launch_bounds__(kBT) minres_finish(TV* __restrict__ x, const TV* __restrict__ zprev,
                                                     const TV* __restrict__ wa, const TV* __restrict__ wb,
                                                     TV* __restrict__ wout, long long n, const MinresState* cur,
                                                     MinresState* next, const double* pb, int npb,
                                                     const double* alfa) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  MinresState s = cur[rhs];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (s.done) {
    if (lead) next[rhs] = s;
    return;
  }
  const double vinv_prev = s.beta > 0 ? 1.0 / s.beta : 0.0;
  double phi, denom, oldeps, delta, vinv;
  const double b2 = reduce_partials(pb + (long long)rhs * npb, npb, sh);
  minres_scalar_update(s, alfa[rhs], b2, phi, denom, oldeps, delta, vinv);
  if (lead) next[rhs] = s;
  const long long off = (long long)rhs * n;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    double vp = todbl(static_cast<TV>(todbl(zprev[off + i]) * vinv_prev));
    double wn = (vp - oldeps * todbl(wa[off + i]) - delta * todbl(wb[off + i])) * denom;
    TV ws = static_cast<TV>(wn);
    wout[off + i] = ws;
    x[off + i] = static_cast<TV>(todbl(x[off + i]) + phi * todbl(ws));
  }
}

// ---- CG (SPD mass solves) -------------------------------------------------
template <typename TV>
__global__ void __launch_bounds__(kBT) cg_init(CgVecs<TV> v, const double* __restrict__ dinv, long long n,
                                               double* part) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  const long long off = (long long)rhs * n;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    TV bi = v.b[off + i];
    double zi = dinv[i] * todbl(bi);
    v.r[off + i] = bi;
    v.p[off + i] = static_cast<TV>(zi);
    v.x[off + i] = 0;
    acc += todbl(bi) * zi;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[rhs * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBT) cg_init_b(const double* part, int np, CgState* st0, double tol) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  double rz = reduce_partials(part + rhs * np, np, sh);
  if (threadIdx.x == 0) {
    CgState s{};
    s.rz = rz;
    s.rz0 = rz;
    s.tol = tol;
    s.done = rz == 0.0 ? 1 : 0;
    s.flag = (rz < 0 || rz != rz) ? -1 : 0;
    if (s.flag) s.done = 1;
    st0[rhs] = s;
  }
}

// partial (p . q) after q = A p
template <typename TV>
__global__ void __launch_bounds__(kBT) cg_pq(const TV* __restrict__ p, const TV* __restrict__ q, long long n,
                                             const CgState* cur, double* part_a) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  if (cur[rhs].done) return;
  const long long off = (long long)rhs * n;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    acc += todbl(p[off + i]) * todbl(q[off + i]);
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part_a[rhs * gridDim.x + blockIdx.x] = t;
}

// alpha = rz / (p.q); x += alpha p; r -= alpha q; z = dinv r (into q);
// partial (r . z)
template <typename TV>
__global__ void __launch_bounds__(kBT) cg_update(CgVecs<TV> v, const double* __restrict__ dinv, long long n,
                                                 const CgState* cur, const double* part_a, double* part_b) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  const CgState s = cur[rhs];
  if (s.done) return;
  const int np = gridDim.x;
  const double pq = reduce_partials(part_a + rhs * np, np, sh);
  const double alpha = s.rz / pq;
  const long long off = (long long)rhs * n;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    v.x[off + i] = static_cast<TV>(todbl(v.x[off + i]) + alpha * todbl(v.p[off + i]));
    double ri = todbl(v.r[off + i]) - alpha * todbl(v.q[off + i]);
    TV rs = static_cast<TV>(ri);
    v.r[off + i] = rs;
    double zi = dinv[i] * todbl(rs);
    TV zs = static_cast<TV>(zi);
    v.q[off + i] = zs;
    acc += todbl(rs) * todbl(zs);
  }
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part_b[rhs * gridDim.x + blockIdx.x] = t;
}

// beta = rz_new / rz; p = z + beta p; state update
template <typename TV>
__global__ void __launch_bounds__(kBT) cg_dir(CgVecs<TV> v, long long n, const CgState* cur, CgState* next,
                                              const double* part_b) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  CgState s = cur[rhs];
  if (s.done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) next[rhs] = s;
    return;
  }
  const int np = gridDim.x;
  const double rz = reduce_partials(part_b + rhs * np, np, sh);
  const double beta = rz / s.rz;
  s.itn += 1;
  s.rz = rz;
  if (rz < 0 || !(rz == rz)) {
    s.flag = -1;
    s.done = 1;
  } else if (rz <= s.tol * s.tol * s.rz0) {
    s.flag = 1;
    s.done = 1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) next[rhs] = s;
  const long long off = (long long)rhs * n;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    v.p[off + i] = static_cast<TV>(todbl(v.q[off + i]) + beta * todbl(v.p[off + i]));
}

// ---- small vector utilities -------------------------------------------------
// partial sums of (a - b)^2 style norms: mode 0: a.a, mode 1: (a-b).(a-b)
template <typename TA>
__global__ void __launch_bounds__(kBT) norm2_partial(const TA* __restrict__ a, const double* __restrict__ b,
                                                     long long n, int mode, double* part) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.y;
  const long long off = (long long)rhs * n;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    if (mode == 2) {
      acc += todbl(a[off + i]) * b[off + i];
    } else {
      double d = todbl(a[off + i]) - (mode ? b[off + i] : 0.0);
      acc += d * d;
    }
  }
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[rhs * gridDim.x + blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBT) finish_sums(const double* part, int np, double* out) {
  __shared__ double sh[kBT];
  const int rhs = blockIdx.x;
  double s = reduce_partials(part + rhs * np, np, sh);
  if (threadIdx.x == 0) out[rhs] = s;
}

// y = a - b (all FP64)
__global__ void __launch_bounds__(kBT) sub_kernel(const double* a, const double* b, double* y, long long n) {
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    y[i] = a[i] - b[i];
}

// y = beta y + alpha (d .* x), d = NULL meaning ones (all FP64; beta = 0
// overwrites y)
__global__ void __launch_bounds__(kBT) axpy_diag_kernel(double* y, double beta, double alpha, const double* d,
                                                        const double* x, long long n) {
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) {
    const double v = alpha * (d ? d[i] * x[i] : x[i]);
    y[i] = beta == 0.0 ? v : beta * y[i] + v;
  }
}

// y_j = d .* x_j for the columns j = blockIdx.y of n rows each (all FP64)
__global__ void __launch_bounds__(kBT) diag_cols_kernel(double* y, const double* d, const double* x, long long n) {
  const long long off = n * blockIdx.y;
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    y[off + i] = d[i] * x[off + i];
}

// x += d (all FP64)
__global__ void __launch_bounds__(kBT) add_kernel(const double* d, double* x, long long n) {
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    x[i] += d[i];
}

__global__ void __launch_bounds__(kBT) fill_kernel(double* y, double v, long long n) {
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT) y[i] = v;
}

// y32 = scale[rhs] * a64 (rhs-wise scaling)
__global__ void __launch_bounds__(kBT) to_f32_scaled(const double* a, float* y, long long n, const double* scale) {
  const int rhs = blockIdx.y;
  const long long off = (long long)rhs * n;
  const double s = scale[rhs];
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    y[off + i] = static_cast<float>(a[off + i] * s);
}

// x64 += scale[rhs] * d32
__global__ void __launch_bounds__(kBT) axpy_f32(const float* d, double* x, long long n, const double* scale) {
  const int rhs = blockIdx.y;
  const long long off = (long long)rhs * n;
  const double s = scale[rhs];
  for (long long i = (long long)blockIdx.x * kBT + threadIdx.x; i < n; i += (long long)gridDim.x * kBT)
    x[off + i] += s * static_cast<double>(d[off + i]);
}

// ---- host launchers ---------------------------------------------------------
int vec_grid(long long n, int ncu) {
  long long b = (n + kBT * 4 - 1) / (kBT * 4);
  long long cap = 4LL * ncu;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

#define GYM_LAUNCH(k, g, s, ...) hipLaunchKernelGGL(k, g, dim3(kBT), 0, s, __VA_ARGS__)

template <typename TV>
void minres_launch_init(const MinresVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb, double* part,
                        MinresState* st0, double tol, hipStream_t s) {
  GYM_LAUNCH(minres_init_a<TV>, dim3(nb, nrhs), s, v, dinv, n, part);
  GYM_LAUNCH(minres_init_b<TV>, dim3(nb, nrhs), s, v, n, part, nb, st0, tol);
}

template <typename TV>
void minres_launch_init_vecs(const MinresVecs<TV>& v, long long n, int nrhs, int nb, hipStream_t s) {
  GYM_LAUNCH(minres_init_vecs<TV>, dim3(nb, nrhs), s, v, n);
}

template <typename TV>
void minres_launch_dot2(const TV* y, const TV* z, const TV* r, long long n, int nrhs, int nb, double* pb,
                        double* pc, hipStream_t s, const MinresState* gate) {
  GYM_LAUNCH(minres_dot2<TV>, dim3(nb, nrhs), s, y, z, r, n, pb, pc, gate);
}

template <typename TV>
void minres_launch_init_state(const MinresVecs<TV>& v, long long n, int nrhs, int nb, const double* part,
                              MinresState* st0, double tol, hipStream_t s) {
  GYM_LAUNCH(minres_init_b<TV>, dim3(nb, nrhs), s, v, n, part, nb, st0, tol);
}

template <typename TV>
void minres_launch_step2(const MrVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb, const Step2Io& io,
                         hipStream_t s) {
  GYM_LAUNCH(minres_step2<TV>, dim3(nb, nrhs), s, v, dinv, n, io);
}

template <typename TV>
void minres_launch_finish(TV* x, const TV* zprev, const TV* wa, const TV* wb, TV* wout, long long n, int nrhs,
                          int nb, const MinresState* cur, MinresState* next, const double* pb,
                          const double* alfa, hipStream_t s) {
  GYM_LAUNCH(minres_finish<TV>, dim3(nb, nrhs), s, x, zprev, wa, wb, wout, n, cur, next, pb, nb, alfa);
}

template <typename TV>
void cg_launch_init(const CgVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb, double* part,
                    CgState* st0, double tol, hipStream_t s) {
  GYM_LAUNCH(cg_init<TV>, dim3(nb, nrhs), s, v, dinv, n, part);
  GYM_LAUNCH(cg_init_b, dim3(1, nrhs), s, part, nb, st0, tol);
}

template <typename TV>
void cg_launch_iter_tail(const CgVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb,
                         const CgState* cur, CgState* next, double* pa, double* pb, hipStream_t s) {
  GYM_LAUNCH(cg_pq<TV>, dim3(nb, nrhs), s, v.p, v.q, n, cur, pa);
  GYM_LAUNCH(cg_update<TV>, dim3(nb, nrhs), s, v, dinv, n, cur, pa, pb);
  GYM_LAUNCH(cg_dir<TV>, dim3(nb, nrhs), s, v, n, cur, next, pb);
}

void launch_norm2(const double* a, const double* b, long long n, int nrhs, int nb, int mode, double* part,
                  double* out, hipStream_t s) {
  GYM_LAUNCH(norm2_partial<double>, dim3(nb, nrhs), s, a, b, n, mode, part);
  GYM_LAUNCH(finish_sums, dim3(nrhs), s, part, nb, out);
}

void launch_sub(const double* a, const double* b, double* y, long long n, int nb, hipStream_t s) {
  GYM_LAUNCH(sub_kernel, dim3(nb), s, a, b, y, n);
}

void launch_axpy_diag(double* y, double beta, double alpha, const double* d, const double* x, long long n, int nb,
                      hipStream_t s) {
  GYM_LAUNCH(axpy_diag_kernel, dim3(nb), s, y, beta, alpha, d, x, n);
}

void launch_diag_cols(double* y, const double* d, const double* x, long long n, int ncol, int nb, hipStream_t s) {
  if (n < 1 || ncol < 1) return;
  hipLaunchKernelGGL(diag_cols_kernel, dim3(nb, ncol), dim3(kBT), 0, s, y, d, x, n);
}

void launch_add(const double* d, double* x, long long n, int nb, hipStream_t s) {
  GYM_LAUNCH(add_kernel, dim3(nb), s, d, x, n);
}

void launch_fill(double* y, double v, long long n, int nb, hipStream_t s) {
  GYM_LAUNCH(fill_kernel, dim3(nb), s, y, v, n);
}

void launch_to_f32_scaled(const double* a, float* y, long long n, int nrhs, int nb, const double* scale,
                          hipStream_t s) {
  GYM_LAUNCH(to_f32_scaled, dim3(nb, nrhs), s, a, y, n, scale);
}

void launch_axpy_f32(const float* d, double* x, long long n, int nrhs, int nb, const double* scale,
                     hipStream_t s) {
  GYM_LAUNCH(axpy_f32, dim3(nb, nrhs), s, d, x, n, scale);
}

template void minres_launch_init<double>(const MinresVecs<double>&, const double*, long long, int, int, double*,
                                         MinresState*, double, hipStream_t);
template void minres_launch_init<float>(const MinresVecs<float>&, const double*, long long, int, int, double*,
                                        MinresState*, double, hipStream_t);
template void minres_launch_init_vecs<double>(const MinresVecs<double>&, long long, int, int, hipStream_t);
template void minres_launch_init_vecs<float>(const MinresVecs<float>&, long long, int, int, hipStream_t);
template void minres_launch_dot2<double>(const double*, const double*, const double*, long long, int, int, double*,
                                         double*, hipStream_t, const MinresState*);
template void minres_launch_dot2<float>(const float*, const float*, const float*, long long, int, int, double*,
                                        double*, hipStream_t, const MinresState*);
template void minres_launch_init_state<double>(const MinresVecs<double>&, long long, int, int, const double*,
                                               MinresState*, double, hipStream_t);
template void minres_launch_init_state<float>(const MinresVecs<float>&, long long, int, int, const double*,
                                              MinresState*, double, hipStream_t);
template void minres_launch_step2<double>(const MrVecs<double>&, const double*, long long, int, int, const Step2Io&,
                                          hipStream_t);
template void minres_launch_step2<float>(const MrVecs<float>&, const double*, long long, int, int, const Step2Io&,
                                         hipStream_t);
template void minres_launch_finish<double>(double*, const double*, const double*, const double*, double*,
                                           long long, int, int, const MinresState*, MinresState*,
                                           const double*, const double*, hipStream_t);
template void minres_launch_finish<float>(float*, const float*, const float*, const float*, float*, long long,
                                          int, int, const MinresState*, MinresState*, const double*,
                                          const double*, hipStream_t);
template void cg_launch_init<double>(const CgVecs<double>&, const double*, long long, int, int, double*,
                                     CgState*, double, hipStream_t);
template void cg_launch_iter_tail<double>(const CgVecs<double>&, const double*, long long, int, int,
                                          const CgState*, CgState*, double*, double*, hipStream_t);

}  // namespace gym

// ---- ragged batches (serving) ------------------------------------------------
// One launch covers one MINRES step of several independent solves; every
// request keeps its own block count, partial sums and state, so its result
// is the same whether it runs alone or in a batch.
namespace gym {

__device__ __forceinline__ int find_item(const int* bstart, int nitem, int blk) {
  int lo = 0, hi = nitem;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (bstart[mid] <= blk) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Second kernel of a fused MINRES step for every request of a ragged batch
// (each item: one request, one rhs, its own blocks and partial sums).
__global__ void __launch_bounds__(kBT) batch_step2(const MrItem* items, const int* bstart, int nitem) {
  __shared__ double sh[3 * kBT];
  const int i = find_item(bstart, nitem, blockIdx.x);
  const MrItem it = items[i];
  step2_body<double>(it.v, it.dinv, it.n, it.io, 0, blockIdx.x - bstart[i], it.nb, sh);
}

// N(0,1) right-hand side from a counter-based generator: SplitMix64
// (Steele, Lea & Flood 2014) gives 64-bit words z_k = mix(seed + (k+1) g),
// g = 0x9E3779B97F4A7C15; u = (z >> 11) 2^-53; Box-Muller on (u_{2i}, u_{2i+1}):
// b_i = sqrt(-2 log(1 - u_{2i})) cos(2 pi u_{2i+1}).  Entries below `first`
// are zero (the first unknown block).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed, unsigned long long k) {
  unsigned long long z = seed + (k + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(kBT) rhs_normal(double* b, long long first, long long n, unsigned long long seed) {
  for (long long k = (long long)blockIdx.x * kBT + threadIdx.x; k < n; k += (long long)gridDim.x * kBT) {
    if (k < first) {
      b[k] = 0.0;
      continue;
    }
    unsigned long long i = (unsigned long long)(k - first);
    double u1 = (double)(splitmix64(seed, 2 * i) >> 11) * 0x1.0p-53;
    double u2 = (double)(splitmix64(seed, 2 * i + 1) >> 11) * 0x1.0p-53;
    b[k] = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
  }
}

void launch_batch_step2(const MrItem* items_dev, const int* bstart_dev, int nitem, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(batch_step2, dim3(nblocks), dim3(kBT), 0, s, items_dev, bstart_dev, nitem);
}
void launch_rhs_normal(double* b, long long first, long long n, unsigned long long seed, int nb, hipStream_t s) {
  hipLaunchKernelGGL(rhs_normal, dim3(nb), dim3(kBT), 0, s, b, first, n, seed);
}

}  // namespace gym
