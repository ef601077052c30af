// Mixed Poisson apply with bf16 element products on the matrix cores
// (poisson_mfma.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "minres_step.hpp"

namespace gym {

struct PoissonMfmaParams {
  const void* x;        // FP32 input, ndofs per right-hand side
  void* y;              // FP32 output
  void* yel;            // element results: rows x el_rows floats per right-hand side
  long long ndofs;      // unknowns per right-hand side
  long long np_off;     // index of the first cell unknown
  long long el_rows;    // elements (the stride of one local row)
  long long el_stride;  // floats per right-hand side in yel
  int nel[3], m[3];
  DevSpace s;           // flux block layout
  float s2[3];          // h_c^2 / |cell|
  int gather_blocks;    // blocks of the gather kernel (= partial sums per rhs with the fused step)
  MrStep mr;            // fused MINRES step: partial sums of z . A z into mr.pa
};

// Element-local rows (3 (r+1) r^2 flux + r^3 cell values).
int poisson_mfma_rows(int r);
int poisson_mfma_gather_blocks(long long ndofs, int ncu);
// A fragments of the element blocks (M2ref, then B_c^T and B_c per component),
// from the 1-D element masses mn ((r+1)^2) and me (r^2) and s3 = 1 / |cell|.
std::vector<uint16_t> poisson_mfma_fragments(int r, const std::vector<double>& mn, const std::vector<double>& me,
                                             double s3);
int launch_poisson_mfma(const PoissonMfmaParams& q, const uint16_t* frag, int r, int nrhs, bool mr, int ncu,
                        hipStream_t s);

}  // namespace gym
