// Single-space mass kernels: instantiation unit.
#include "op_kernel.hpp"

namespace gym {

template <int DIM, typename TV, typename TC>
static int mass_dim(int prob, int r, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  switch (prob) {
    case PROB_MASS_H1: return dispatch_r<DIM, PROB_MASS_H1, TV, TC>(r, p, nrhs, ncu, s);
    case PROB_MASS_HCURL: return dispatch_r<DIM, PROB_MASS_HCURL, TV, TC>(r, p, nrhs, ncu, s);
    case PROB_MASS_HDIV: return dispatch_r<DIM, PROB_MASS_HDIV, TV, TC>(r, p, nrhs, ncu, s);
    case PROB_MASS_L2: return dispatch_r<DIM, PROB_MASS_L2, TV, TC>(r, p, nrhs, ncu, s);
  }
  return -2;
}

int launch_mass(int prob, int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  if (dim == 3) {
    if (prec == GYM_F64) return mass_dim<3, double, double>(prob, r, p, nrhs, ncu, s);
    if (prec == GYM_F32) return mass_dim<3, float, float>(prob, r, p, nrhs, ncu, s);
  } else if (dim == 2 && !p.curved) {
    if (prec == GYM_F64) return mass_dim<2, double, double>(prob, r, p, nrhs, ncu, s);
    if (prec == GYM_F32) return mass_dim<2, float, float>(prob, r, p, nrhs, ncu, s);
  }
  return -2;
}

int upload_tables_mass() { return upload_tables_unit(); }

}  // namespace gym
