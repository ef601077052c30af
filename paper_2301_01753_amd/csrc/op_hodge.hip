// Hodge-Laplacian (1-forms) operator kernels: instantiation unit.
#include "op_kernel.hpp"

namespace gym {

int launch_hodge(int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  if (dim != 3) return -2;
  if (prec == GYM_F64) return dispatch_r<3, PROB_HODGE, double, double>(r, p, nrhs, ncu, s);
  if (prec == GYM_F32) return dispatch_r<3, PROB_HODGE, float, float>(r, p, nrhs, ncu, s);
  return -2;
}

int upload_tables_hodge() { return upload_tables_unit(); }

}  // namespace gym
