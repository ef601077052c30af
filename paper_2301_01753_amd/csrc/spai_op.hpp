// SPAI-OP Q1 (paper section 5) on axis-aligned meshes.
#pragma once
#include <hip/hip_runtime.h>

struct gym_space;

namespace gym {

// The symmetric Q1 on the pattern of M1, one slot per offset of the
// (2r + 1)^3 box around each row (dead slots zero), with the 1-D tables the
// apply needs.  Owns q and params_tab (device).
struct SpaiOpQ1 {
  double* q = nullptr;           // n1 x (2r + 1)^3 slots
  double* params_tab = nullptr;  // the 1-D bands of M_a and M_a^2
  long long n1 = 0;
  int r = 0;
  int wrap = 0;                  // periodic axes of the space
  long long off[3] = {0, 0, 0};
  int n[3][3] = {};
  double sc[3] = {0, 0, 0};
  const double* M[3][3] = {};
  const double* M2[3][3] = {};
};

// Solves the SPAI-OP Sylvester system (U Q1 T + T Q1 U = M1 T + T M1 on the
// pattern of M1, U = M1^2, T = 1 + lambda W W^T) by Jacobi-preconditioned CG
// from the symmetrised column-wise SPAI, to relative residual rtol.  W: np
// probing vectors P2 v_k (device, np x n1), MW = M1 W.  Returns 0,
// GYM_W_NOT_CONVERGED at the iteration cap, or an error.
int spai_op_build(const gym_space* s1, const double* W, const double* MW, int np, double lam, double rtol,
                  int maxit, int ncu, hipStream_t s, SpaiOpQ1* out, int* iters, double* rel_res);
// y = Q1 x
void launch_spai_op_apply(const SpaiOpQ1& Q, const double* x, double* y, int ncu, hipStream_t s);
void spai_op_free(SpaiOpQ1* Q);

}  // namespace gym
