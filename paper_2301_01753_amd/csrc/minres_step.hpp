// MINRES recurrence state and the scalar part of one MINRES step, shared by
// the Krylov vector kernels and the operator kernel that runs a whole MINRES
// step in its epilogue.
#pragma once
#include <hip/hip_runtime.h>

namespace gym {

struct MinresState {
  double beta, oldb, dbar, epsln, phibar, cs, sn, tnorm2, beta1, alfa, tol;
  int itn, done, flag;  // flag: 0 running, 1 converged, -1 breakdown
  int pad;
};

// Sums over a workgroup of NT threads (a multiple of 64) of N values per
// thread, returned in every thread: a butterfly across the 64 lanes of each
// wavefront (cross-lane moves, no LDS, no barrier), then one LDS exchange of
// the per-wavefront sums, which every thread adds up in wavefront order.  The
// order is fixed, so results are reproducible.  sh holds N * NT / 64 doubles
// (any buffer of N * NT doubles is large enough).
template <int NT, int N>
__device__ __forceinline__ void wg_sums(double (&v)[N], double* sh) {
  static_assert(NT % 64 == 0 && NT >= 64 && NT <= 1024, "workgroup size");
  constexpr int NW = NT / 64;
  const int t = threadIdx.x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], off, 64);
  if constexpr (NW > 1) {
    if ((t & 63) == 0)
#pragma unroll
      for (int k = 0; k < N; ++k) sh[k * NW + (t >> 6)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a = sh[k * NW];
#pragma unroll
      for (int w = 1; w < NW; ++w) a += sh[k * NW + w];
      v[k] = a;
    }
    __syncthreads();
  }
}

// Lanczos/Givens scalar recurrence of one MINRES step (Paige & Saunders),
// given alfa = v.(A v - ...) and b2 = r2 . M^-1 r2; returns the update
// coefficients and marks convergence (phibar <= tol beta1) or breakdown.
__device__ __forceinline__ void minres_scalar_update(MinresState& s, double alfa, double b2, double& phi,
                                                     double& denom, double& oldeps, double& delta, double& vinv) {
  s.itn += 1;
  const double oldb = s.beta;
  const double beta = b2 > 0 ? sqrt(b2) : 0.0;
  s.tnorm2 += alfa * alfa + oldb * oldb + beta * beta;
  oldeps = s.epsln;
  delta = s.cs * s.dbar + s.sn * alfa;
  const double gbar = s.sn * s.dbar - s.cs * alfa;
  const double epsln = s.sn * beta;
  const double dbar = -s.cs * beta;
  double gamma = sqrt(gbar * gbar + beta * beta);
  gamma = gamma > 2.2e-308 ? gamma : 2.2e-308;
  const double cs = gbar / gamma, sn = beta / gamma;
  phi = cs * s.phibar;
  const double phibar = sn * s.phibar;
  denom = 1.0 / gamma;
  s.oldb = oldb;
  s.beta = beta;
  s.epsln = epsln;
  s.dbar = dbar;
  s.cs = cs;
  s.sn = sn;
  s.phibar = phibar;
  s.alfa = alfa;
  if (b2 < 0 || !(b2 == b2) || !(phibar == phibar)) {
    s.flag = -1;
    s.done = 1;
  } else if (phibar <= s.tol * s.beta1 || beta == 0.0) {
    s.flag = 1;
    s.done = 1;
  }
  vinv = beta > 0 ? 1.0 / beta : 0.0;
}

// First half of a fused MINRES step, carried by an operator apply of z_k
// (z_k = M^-1 r2_k, so v_k = z_k / beta_k): y receives A z_k, and the epilogue
// adds z_k . (A z_k) over the owned positions into one partial sum per
// workgroup (pa).  The apply needs no scalar of the recurrence (A is linear):
// minres_step2 closes step k-1, then scales by 1 / beta_k.  Workgroups of a
// right-hand side whose state is already converged do nothing.
struct MrStep {
  const MinresState* cur;  // latest state (written by the previous minres_step2)
  double* pa;              // out: one partial sum of z_k . A z_k per workgroup
};

}  // namespace gym
