// Hodge-Laplacian apply (1-forms) on curved cells, degree 3, FP64, with the
// 1-D contractions on the matrix cores (hodge_mfma.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gym {

struct HcParams {
  const void* x;     // FP64 or FP32 (the launch's f32), as y
  void* y;
  long long ndofs;   // stride between right-hand sides
  DevComp f[4];      // sigma (H1_0), u_x, u_y, u_z (H0(curl)), kept positions
  int nel[3];
  const double* verts;  // (nel+1)^3 x 3 cell vertices (x fastest), 16 doubles of padding after
  double* halo;      // tile-boundary partial sums (hodge_mfma_halo_doubles)
  const void* zero;  // 8 zero bytes in device memory (read by lanes outside the kept set)
  int chunk_mode;    // z chunks: 0 automatic, 1 whole columns, 2 one layer each
  // filled by the launch
  int tiles_x, tiles_y, chunk, nchunks, nitems, nrhs;
  long long hx_n, hy_n, hxy_n;  // per right-hand side
};

// Degree of the matrix-core kernel.
constexpr int kHcDegree = 3;
// Doubles of the halo buffer for a mesh of nel cells and nrhs right-hand sides.
long long hodge_mfma_halo_doubles(const int nel[3], int nrhs);
// y = A x for nrhs right-hand sides (x, y in the operator's canonical layout,
// stride ndofs).  Two launches on s: the element kernel, then the sums over
// tile boundaries.  Returns 0, or -1 on a launch failure.
// f32: x and y are FP32 (the arithmetic stays FP64; only the vectors are
// stored in FP32).
int launch_hodge_mfma(const HcParams& p, int nrhs, int ncu, hipStream_t s, bool f32 = false);

}  // namespace gym
