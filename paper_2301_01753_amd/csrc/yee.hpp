// Fused generalized Yee step with lumped masses (paper sections 3 and 4.3).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gym {

// With both masses lumped every operator of a Strang step is a lattice
// stencil: Q1 and M2~ are diagonal, and their diagonals are tensor products of
// 1-D row sums, so one pass over the lattice positions does a whole step.
struct YeeParams {
  const double* a_in;  // a before the step (every position the stencil reads)
  double* a_out;       // a after the step (may equal a_in only for the half step)
  double* e;           // e, updated in place
  DevSpace s1;         // Lambda^1 with the perfect-conductor unknowns removed
  const double* w;     // 1-D row sums: nodal ones along axis d at w + wn[d], edge ones at w + we[d]
  int wn[3], we[3];
  double q1s[3];       // metric constant of Lambda^1 component c
  double m2s[3];       // metric constant of Lambda^2 component c
  double te;           // tau c^2: e += te C^T M2~ C a
  double ha;           // then a -= ha Q1 e
  int len[3];          // lattice positions per axis (r N_d + 1)
  unsigned npos;       // len[0] len[1] len[2]
};

// half: only a_out = a_in - ha Q1 e (the first half step in a); else a full
// step e += te C^T M2~ C a_in, a_out = a_in - ha Q1 e.  ncu: compute units
// (sizes the z-chunks of the full step).
int launch_yee(const YeeParams& p, bool half, int ncu, hipStream_t s);

}  // namespace gym
