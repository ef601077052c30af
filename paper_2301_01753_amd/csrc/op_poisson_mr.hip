// Mixed-Poisson operator kernels carrying the first half of a fused MINRES
// step (MrStep): instantiation unit.
#include "op_kernel.hpp"

namespace gym {

int launch_poisson_mr(int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  if (dim == 3) {
    if (prec == GYM_F64) return dispatch_r<3, PROB_POISSON, double, double, true>(r, p, nrhs, ncu, s);
    if (prec == GYM_F32) return dispatch_r<3, PROB_POISSON, float, float, true>(r, p, nrhs, ncu, s);
  } else if (dim == 2 && !p.curved) {
    if (prec == GYM_F64) return dispatch_r<2, PROB_POISSON, double, double, true>(r, p, nrhs, ncu, s);
    if (prec == GYM_F32) return dispatch_r<2, PROB_POISSON, float, float, true>(r, p, nrhs, ncu, s);
  }
  return -2;
}

int upload_tables_poisson_mr() { return upload_tables_unit(); }

}  // namespace gym
