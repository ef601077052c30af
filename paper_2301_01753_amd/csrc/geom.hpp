// Per-Gauss-point metrics of curved cells (geom.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace gym {

// fields per Gauss point: det J, 1/det J, HCURL metric (6), HDIV metric (6)
constexpr int kQFields = 14;
enum { QF_DET = 0, QF_INVDET = 1, QF_HCURL = 2, QF_HDIV = 8 };

struct QPoints {
  double x[8];  // Gauss points on [0, 1]
};

// Fill `out` (kQFields x (q nel_0)(q nel_1)(q nel_2) values, FP64 or FP32 by
// `f32`) from the (nel+1)^3 x 3 vertex array; asynchronous on `s`.
int launch_qdata(const double* verts, const int nel[3], int q, const double* gauss_x, void* out, int f32,
                 hipStream_t s);

}  // namespace gym
