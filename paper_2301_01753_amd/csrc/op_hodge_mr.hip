// Hodge-Laplacian operator kernels carrying the first half of a fused MINRES
// step (MrStep): instantiation unit.
#include "op_kernel.hpp"

namespace gym {

int launch_hodge_mr(int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  if (dim != 3) return -2;
  if (prec == GYM_F64) return dispatch_r<3, PROB_HODGE, double, double, true>(r, p, nrhs, ncu, s);
  if (prec == GYM_F32) return dispatch_r<3, PROB_HODGE, float, float, true>(r, p, nrhs, ncu, s);
  return -2;
}

int launch_hodge_batch_mr(int r, OpParams* ph, int* bh, int n, OpParams* pd, int* bd, int ncu, hipStream_t s) {
  switch (r) {
    case 1: return launch_op_batch_r<3, 1, PROB_HODGE, double, double, true>(ph, bh, n, pd, bd, ncu, s);
    case 2: return launch_op_batch_r<3, 2, PROB_HODGE, double, double, true>(ph, bh, n, pd, bd, ncu, s);
    case 3: return launch_op_batch_r<3, 3, PROB_HODGE, double, double, true>(ph, bh, n, pd, bd, ncu, s);
    case 4: return launch_op_batch_r<3, 4, PROB_HODGE, double, double, true>(ph, bh, n, pd, bd, ncu, s);
  }
  return -2;
}

int upload_tables_hodge_mr() { return upload_tables_unit(); }

}  // namespace gym
