// Block preconditioner of the mixed Poisson operator on affine boxes:
// diag(diag(M2), M3 D diag(M2)^-1 D^T M3) applied exactly, the cell block by
// simultaneous diagonalisation of its per-axis factors (schur.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "minres_step.hpp"

struct gym_op;

namespace gym {

struct SchurPrec {
  long long ns = 0, np = 0;     // unknowns of the flux block and of the cell block
  int m[3] = {1, 1, 1};         // cells per axis
  double* dsinv = nullptr;      // ns: 1 / diag(M2)
  double* lam = nullptr;        // m0 + m1 + m2: lam_a / s2_a per axis
  double scale = 1.0;           // 1 / s3^2
  double* fwd64[3] = {};        // Vt_a^T, row-major m_a x m_a (forward transforms)
  double* bwd64[3] = {};        // Vt_a
  float* fwd32[3] = {};
  float* bwd32[3] = {};
  void* work = nullptr;         // two cell-block vectors per right-hand side
  int work_nrhs = 0;
  size_t work_bytes = 0;
  void* mem = nullptr;          // the factors

  template <typename T>
  const T* const* fwd() const {
    if constexpr (sizeof(T) == 8) return fwd64;
    else return fwd32;
  }
  template <typename T>
  const T* const* bwd() const {
    if constexpr (sizeof(T) == 8) return bwd64;
    else return bwd32;
  }
  // k-th work vector (np x nrhs of T)
  template <typename T>
  T* work_vec(int k) const {
    return static_cast<T*>(work) + (size_t)k * (size_t)np * (size_t)work_nrhs;
  }
};

// Set-up for the operator (mixed Poisson, 3-D, affine): GYM_E_UNSUPPORTED
// otherwise.  Host work: three symmetric eigenproblems of size m_a.
int schur_build(const gym_op* op, SchurPrec* out);
// Work vectors for nrhs right-hand sides (grown on demand; the caller
// allocates outside its hot loop).
int schur_reserve(SchurPrec* P, int nrhs, size_t elem_bytes);
void schur_free(SchurPrec* P);
// One request of a ragged batch of FP64 preconditioner applies (serving):
// z = P^-1 y for one right-hand side, with the request's own work vectors,
// followed by the partial sums pb = y . z and pc = z . r2 per elementwise
// block (nb of them), as minres_launch_dot2 forms them.
struct SchurItem {
  long long ns, np;
  int m[3];
  int nb;                   // blocks of this item in the elementwise kernels
  double scale;
  const double* dsinv;
  const double* lam;
  const double* fwd[3];
  const double* bwd[3];
  const double* y;
  double* z;
  double* w0;               // np
  double* w1;               // np
  const double* r2;
  double* pb;
  double* pc;
  const MinresState* gate;  // skip the item once this state has converged
};
// Blocks of item it in the transform along axis a (64 lines x 64 outputs each).
int schur_axis_blocks(const SchurItem& it, int a);
// The batch on the device: items_dev[nitem]; est: prefix sums of the items'
// nb; ast[a]: prefix sums of schur_axis_blocks(., a) (nitem + 1 entries each).
void launch_schur_batch(const SchurItem* items_dev, int nitem, const int* est, int ne, const int* const ast[3],
                        const int na[3], hipStream_t s);

// The operator's preconditioner, set up on first use and kept with the
// operator (freed with it), with work vectors for nrhs right-hand sides.
int ensure_schur(gym_op* op, int nrhs, SchurPrec** out);
// z = P^-1 y for nrhs vectors in the operator's layout [s; p] (stride ns + np).
// gate (optional, one Krylov state per right-hand side): right-hand sides
// whose state has converged are left untouched.
template <typename T>
int launch_schur_apply(const SchurPrec& P, const T* y, T* z, int nrhs, int nb, hipStream_t s,
                       const MinresState* gate = nullptr);

}  // namespace gym
