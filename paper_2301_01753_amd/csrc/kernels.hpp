// Kernel launch interfaces shared by the host code of the gym library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "minres_step.hpp"

namespace gym {

enum {
  PROB_POISSON = 0,
  PROB_HODGE = 1,
  PROB_MASS_H1 = 10,
  PROB_MASS_HCURL = 11,
  PROB_MASS_HDIV = 12,
  PROB_MASS_L2 = 13,
};

struct DevComp {
  long long offset;  // first index of the component block in the vector
  int start[3];      // first kept lattice position per axis
  int count[3];      // kept positions per axis
};
struct DevSpace {
  DevComp c[3];
};

struct OpParams {
  const void* x;
  void* y;
  long long ndofs;  // stride between right-hand sides
  DevSpace sa, sb;  // first / second block
  int nel[3];
  int m[3];         // lattice cells per axis (r * nel)
  int tiles_x, tiles_y, chunk, nchunks;
  int kron;         // 1: Kronecker (1-D element matrix) form of the masses
  int bf16;         // 1: contraction operands rounded to bf16 (FP32 accumulate)
  int curved;       // 1: per-Gauss-point metric (curved cells)
  const void* qd;   // curved: the Gauss-point metrics (geom.hpp), FP64 or FP32 as the contractions
  long long qfs;    // values per metric field, (q nel_0)(q nel_1)(q nel_2)
  const int* gate;      // batched launches: skip when *gate != 0 (a solve's done flag)
  int tile_budget;  // 0: one 160 KB workgroup per CU, 1: 40 KB workgroups, 2: automatic
  double sc[8];     // constant pointwise metric factors (affine meshes)
  int fused;        // 1: the apply carries the MINRES step `mr`
  MrStep mr;
  int dry;          // 1: launch nothing, only report the grid in *wg_out
  int* wg_out;      // host: workgroups per rhs of the launch (may be null)
};

int upload_tables();
int launch_operator(int prob, int dim, int r, int prec, const OpParams& p, int nrhs, int ncu,
                    hipStream_t s);
// per-unit entry points (op_hodge.hip, op_poisson.hip, op_mass.hip)
int launch_hodge(int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s);
int launch_poisson(int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s);
// the same with the fused MINRES step (p.fused, p.mr; op_hodge_mr.hip, op_poisson_mr.hip)
int launch_hodge_mr(int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s);
int launch_poisson_mr(int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s);
int launch_mass(int prob, int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s);
// ragged batch of affine operators of one problem and degree (FP64); with
// plist_host[0].fused every item carries its fused MINRES step (p.mr)
int launch_op_batch(int prob, int dim, int r, OpParams* plist_host, int* bstart_host, int nreq,
                    OpParams* plist_dev, int* bstart_dev, int ncu, hipStream_t s);
int launch_hodge_batch(int r, OpParams* ph, int* bh, int n, OpParams* pd, int* bd, int ncu, hipStream_t s);
int launch_poisson_batch(int r, OpParams* ph, int* bh, int n, OpParams* pd, int* bd, int ncu, hipStream_t s);
int launch_hodge_batch_mr(int r, OpParams* ph, int* bh, int n, OpParams* pd, int* bd, int ncu, hipStream_t s);
int launch_poisson_batch_mr(int r, OpParams* ph, int* bh, int n, OpParams* pd, int* bd, int ncu, hipStream_t s);
int upload_tables_hodge();
int upload_tables_poisson();
int upload_tables_mass();
int upload_tables_hodge_mr();
int upload_tables_poisson_mr();

// incidence: y = d x or d^T x, bit-reproducible ascending-index sums
struct IncParams {
  const double* x;
  double* y;
  DevSpace in, out;
  int in_ncomp, out_ncomp;
  int dim;
  int op;           // 0 = G, 1 = C, 2 = D
  int transpose;
  int periodic;     // bit a: positions along axis a wrap (count = m_a)
  long long nout;
  int nrhs = 1;     // right-hand sides (grid y), x and y strides below
  long long in_stride = 0, out_stride = 0;
};
int launch_incidence(const IncParams& p, hipStream_t s);

}  // namespace gym
