// Pointwise metrics of the mass matrices on curved (multilinear) cells,
// evaluated once per mesh and Gauss rule.
//
// Paper section 2 defines (M_p)_ij = int (Lambda_i, Lambda_j)_p dx.  Pulled
// back to the reference cube through the cell map x(xi) with Jacobian
// J = dx/dxi, the integrand at a Gauss point becomes the reference basis
// values times a 3x3 (or scalar) metric:
//   p = 0 (H1):    det J
//   p = 1 (HCURL): det J J^-1 J^-T = adj(J) adj(J)^T / det J   (covariant)
//   p = 2 (HDIV):  J^T J / det J                                (contravariant)
//   p = 3 (L2):    1 / det J
// The operator kernels read these instead of rebuilding J at every Gauss
// point of every mass, right-hand side and apply.
//
// Layout: field f (0: det, 1: 1/det, 2..7: HCURL metric, 8..13: HDIV metric,
// symmetric entries 00 01 02 11 12 22) is a lattice of Gauss points
// [GZ][GY][GX] with G_a = q nel_a, the point t of element e along axis a at
// q e + t (x fastest), so a row of points along x is contiguous.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "geom.hpp"
#include "gym_internal.hpp"

namespace gym {

namespace {

template <typename TO>
__global__ void __launch_bounds__(256) qdata_kernel(const double* __restrict__ V, int nx, int ny, int nz, int q,
                                                    QPoints gp, TO* __restrict__ out, long long fs) {
  const long long GX = (long long)q * nx, GY = (long long)q * ny;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < fs; g += (long long)gridDim.x * blockDim.x) {
    const long long gx = g % GX, r = g / GX;
    const long long gy = r % GY, gz = r / GY;
    const int ex = (int)(gx / q), ey = (int)(gy / q), ez = (int)(gz / q);
    const double xi[3] = {gp.x[gx - (long long)ex * q], gp.x[gy - (long long)ey * q], gp.x[gz - (long long)ez * q]};
    // corner c = (b0, b1, b2) of the cell at vertex (ex + b0, ey + b1, ez + b2)
    auto vtx = [&](int b0, int b1, int b2, int a) {
      return V[(((long long)(ez + b2) * (ny + 1) + (ey + b1)) * (nx + 1) + (ex + b0)) * 3 + a];
    };
    double J[3][3];
    for (int i = 0; i < 3; ++i) {
      double d[3] = {0, 0, 0};
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
          // derivative along axis a: the difference across a, weighted by the
          // multilinear weights of the other two axes
          const double w0 = (b ? xi[1] : 1 - xi[1]) * (c ? xi[2] : 1 - xi[2]);
          const double w1 = (b ? xi[0] : 1 - xi[0]) * (c ? xi[2] : 1 - xi[2]);
          const double w2 = (b ? xi[0] : 1 - xi[0]) * (c ? xi[1] : 1 - xi[1]);
          d[0] += w0 * (vtx(1, b, c, i) - vtx(0, b, c, i));
          d[1] += w1 * (vtx(b, 1, c, i) - vtx(b, 0, c, i));
          d[2] += w2 * (vtx(b, c, 1, i) - vtx(b, c, 0, i));
        }
      J[i][0] = d[0];
      J[i][1] = d[1];
      J[i][2] = d[2];
    }
    // adj[a][i] = cofactor of J[i][a]
    double adj[3][3];
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
    const double inv = 1.0 / det;
    double f[kQFields];
    f[0] = det;
    f[1] = inv;
    const int sa[6] = {0, 0, 0, 1, 1, 2}, sb[6] = {0, 1, 2, 1, 2, 2};
    for (int s = 0; s < 6; ++s) {
      const int a = sa[s], b = sb[s];
      double hc = 0, hd = 0;
      for (int i = 0; i < 3; ++i) {
        hc += adj[a][i] * adj[b][i];
        hd += J[i][a] * J[i][b];
      }
      f[2 + s] = hc * inv;
      f[8 + s] = hd * inv;
    }
    for (int k = 0; k < kQFields; ++k) out[k * fs + g] = static_cast<TO>(f[k]);
  }
}

}  // namespace

int launch_qdata(const double* verts, const int nel[3], int q, const double* gauss_x, void* out, int f32,
                 hipStream_t s) {
  QPoints gp{};
  for (int t = 0; t < q; ++t) gp.x[t] = gauss_x[t];
  const long long fs = (long long)q * nel[0] * q * nel[1] * q * nel[2];
  const int nb = (int)std::min<long long>((fs + 255) / 256, 65536);
  if (f32)
    hipLaunchKernelGGL(qdata_kernel<float>, dim3(nb), dim3(256), 0, s, verts, nel[0], nel[1], nel[2], q, gp,
                       static_cast<float*>(out), fs);
  else
    hipLaunchKernelGGL(qdata_kernel<double>, dim3(nb), dim3(256), 0, s, verts, nel[0], nel[1], nel[2], q, gp,
                       static_cast<double*>(out), fs);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gym
