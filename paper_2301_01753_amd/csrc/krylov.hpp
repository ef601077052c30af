// Krylov kernel interfaces (see krylov.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "minres_step.hpp"

namespace gym {

struct CgState {
  double rz, rz0, tol;
  int itn, done, flag, pad;
};

template <typename TV>
struct MinresVecs {
  const TV* b;
  TV *x, *r1, *r2, *y, *v, *w, *w1, *w2;
};

template <typename TV>
struct CgVecs {
  const TV* b;
  TV *x, *r, *p, *q;  // q holds A p, then z = M^-1 r
};

void launch_rhs_normal(double* b, long long first, long long n, unsigned long long seed, int nb, hipStream_t s);

int vec_grid(long long n, int ncu);

template <typename TV>
void minres_launch_init(const MinresVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb, double* part,
                        MinresState* st0, double tol, hipStream_t s);
// Vectors of the second kernel of a fused MINRES step (rhs-major).
template <typename TV>
struct MrVecs {
  TV *y, *r1, *r2, *zp, *x;
  const TV *wa, *wb;  // w_{k-3}, w_{k-2}
  TV* wout;           // receives w_{k-1} (holds w_{k-4})
};

// Scalars and partial sums of the second kernel of a fused MINRES step
// (see minres_step2): the previous pass's partials are read while the new
// ones are written, so the host alternates two sets.
struct Step2Io {
  const MinresState* cur;  // latest state
  MinresState* next;       // receives the state after closing step k-1
  int first;               // 1: no step to close (fresh start)
  int npa, npb;            // partials per rhs: operator workgroups, step2 blocks
  const double* pa;        // z_k . A z_k partials (operator kernel)
  const double* pb_prev;   // beta_k^2 partials (previous pass)
  const double* pc_prev;   // z_k . r1_k partials (previous pass)
  const double* alfa_prev; // alfa_{k-1} per rhs
  double *pb, *pc;         // out: this pass's partials
  double* alfa;            // out: alfa_k per rhs
  int ext;                 // 1: the preconditioner runs after the kernel
                           // (z_{k+1} and the partials pb, pc come from
                           // the caller: minres_launch_dot2)
};

template <typename TV>
void minres_launch_step2(const MrVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb, const Step2Io& io,
                         hipStream_t s);
// A non-diagonal preconditioner M: the initialisation without z (r1 = r2 = b,
// x = w = w1 = w2 = 0), and after z = M^-1 y the per-block partial sums
// pb = y . z and, if r is not null, pc = z . r, in the layout of
// minres_step2's (nb blocks per rhs).
template <typename TV>
void minres_launch_init_vecs(const MinresVecs<TV>& v, long long n, int nrhs, int nb, hipStream_t s);
// gate (optional): leave right-hand sides whose state there has converged.
template <typename TV>
void minres_launch_dot2(const TV* y, const TV* z, const TV* r, long long n, int nrhs, int nb, double* pb,
                        double* pc, hipStream_t s, const MinresState* gate = nullptr);
// beta_1 from the partials of b . M^-1 b (as minres_launch_init's second half)
template <typename TV>
void minres_launch_init_state(const MinresVecs<TV>& v, long long n, int nrhs, int nb, const double* part,
                              MinresState* st0, double tol, hipStream_t s);

// One request of a ragged batch of fused MINRES steps (FP64, one rhs).
struct MrItem {
  long long n;
  int nb, pad;  // nb: blocks of this request in the batch
  MrVecs<double> v;
  const double* dinv;
  Step2Io io;
};
// minres_step2 for every item; bstart = prefix sums of the items' nb.
void launch_batch_step2(const MrItem* items_dev, const int* bstart_dev, int nitem, int nblocks, hipStream_t s);
// Completes a pending step (iteration cap): state cur -> next, w and x.
template <typename TV>
void minres_launch_finish(TV* x, const TV* zprev, const TV* wa, const TV* wb, TV* wout, long long n, int nrhs,
                          int nb, const MinresState* cur, MinresState* next, const double* pb,
                          const double* alfa, hipStream_t s);
template <typename TV>
void cg_launch_init(const CgVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb, double* part,
                    CgState* st0, double tol, hipStream_t s);
template <typename TV>
void cg_launch_iter_tail(const CgVecs<TV>& v, const double* dinv, long long n, int nrhs, int nb,
                         const CgState* cur, CgState* next, double* pa, double* pb, hipStream_t s);

// per rhs: mode 0 |a|^2, mode 1 |a - b|^2, mode 2 a . b (deterministic two-stage sums)
void launch_norm2(const double* a, const double* b, long long n, int nrhs, int nb, int mode, double* part,
                  double* out, hipStream_t s);
void launch_sub(const double* a, const double* b, double* y, long long n, int nb, hipStream_t s);
void launch_add(const double* d, double* x, long long n, int nb, hipStream_t s);
// y = v (a fill kernel, not a memset, so that it may sit in a captured graph)
void launch_fill(double* y, double v, long long n, int nb, hipStream_t s);
// y = beta y + alpha (d .* x); d = NULL: ones
void launch_axpy_diag(double* y, double beta, double alpha, const double* d, const double* x, long long n, int nb,
                      hipStream_t s);
// y_j = d .* x_j for ncol contiguous columns of n rows (one launch)
void launch_diag_cols(double* y, const double* d, const double* x, long long n, int ncol, int nb, hipStream_t s);
void launch_to_f32_scaled(const double* a, float* y, long long n, int nrhs, int nb, const double* scale,
                          hipStream_t s);
void launch_axpy_f32(const float* d, double* x, long long n, int nrhs, int nb, const double* scale,
                     hipStream_t s);

}  // namespace gym
