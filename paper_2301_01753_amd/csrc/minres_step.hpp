// MINRES recurrence state and the scalar part of one MINRES step, shared by
// the Krylov vector kernels and the operator kernel that runs a whole MINRES
// step in its epilogue.
#pragma once
#include <hip/hip_runtime.h>

namespace gym {

struct MinresState {
  double beta, oldb, dbar, epsln, phibar, cs, sn, tnorm2, beta1, alfa, tol;
  // fused driver: coefficients of the w / x update of the step just closed
  // by the scalar update, and z_k . r1_k for the next alfa
  double phi, denom, oldeps, delta, zr1;
  int itn, done, flag;  // flag: 0 running, 1 converged, -1 breakdown
  int fresh;            // fused driver: 1 when the operator kernel produced this state
  int upd;              // fused driver: the w / x update of that step is due
  int pad;
};

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

// First half of a fused MINRES step, carried by an operator apply of
// v_k = z_k / beta_k (z_k is the apply input; y receives A v_k unchanged).
// Unless `first`, every workgroup first closes step k-1: it sums the
// partials pb (beta_k^2) and pc (z_k . r1_k) left by minres_step2 and runs
// the scalar update from alfa_{k-1}; one workgroup stores the new state with
// the w / x coefficients.  The epilogue adds v_k . (A v_k) over the owned
// positions into one partial sum per workgroup (pa); minres_step2 completes
// alfa_k = v_k . (A v_k) - (beta_k / beta_{k-1}) v_k . r1_k.  (Each consumer
// re-adds the partials in the same order: a last-workgroup reduction would
// need a device-scope fence per workgroup, which writes back the L2.)
struct MrStep {
  const MinresState* cur;  // state before the update of step k-1
  MinresState* next;       // state after it
  const double* pb;        // npb partial sums per rhs of beta_k^2
  const double* pc;        // npb partial sums per rhs of z_k . r1_k
  const double* alfa;      // alfa_{k-1} per rhs
  double* pa;              // out: one partial sum of v_k . A v_k per workgroup
  int npb;
  int first;  // 1: no step is pending (fresh start)
};

}  // namespace gym
