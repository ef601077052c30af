// Block kernels of the generalized eigen-solver (LOBPCG, eig.cpp).
//
// Blocks hold up to kEigMaxCols column vectors of length n, column after
// column.  The Gram kernel stages 64 rows of both blocks in LDS and gives
// every thread up to three (row of U^T, column of V) pairs; per-block
// partials are summed by a second kernel in block order, so the result does
// not depend on timing.
#include <algorithm>

#include "eig.hpp"

namespace gym {
namespace {

constexpr int kET = 256;  // threads per block
constexpr int kER = 64;   // rows per LDS tile of the Gram kernel
constexpr int kEP = (kEigMaxCols * kEigMaxCols + kET - 1) / kET;  // pairs per thread

__global__ void __launch_bounds__(kET) gram_partial(const double* __restrict__ U, int p, const double* __restrict__ V,
                                                    int q, long long n, double* __restrict__ part) {
  __shared__ double su[kER][kEigMaxCols];
  __shared__ double sv[kER][kEigMaxCols];
  const int npair = p * q;
  double acc[kEP];
#pragma unroll
  for (int j = 0; j < kEP; ++j) acc[j] = 0.0;
  for (long long r0 = (long long)blockIdx.x * kER; r0 < n; r0 += (long long)gridDim.x * kER) {
    for (int i = threadIdx.x; i < kER * p; i += kET) {
      const int r = i % kER, c = i / kER;
      su[r][c] = r0 + r < n ? U[(long long)c * n + r0 + r] : 0.0;
    }
    for (int i = threadIdx.x; i < kER * q; i += kET) {
      const int r = i % kER, c = i / kER;
      sv[r][c] = r0 + r < n ? V[(long long)c * n + r0 + r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kEP; ++j) {
      const int pr = threadIdx.x + j * kET;
      if (pr < npair) {
        const int a = pr / q, b = pr - a * q;
        double s = 0.0;
#pragma unroll 8
        for (int r = 0; r < kER; ++r) s += su[r][a] * sv[r][b];
        acc[j] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < kEP; ++j) {
    const int pr = threadIdx.x + j * kET;
    if (pr < npair) part[(long long)blockIdx.x * npair + pr] = acc[j];
  }
}

__global__ void __launch_bounds__(kET) gram_reduce(const double* __restrict__ part, int npair, int nb,
                                                   double* __restrict__ G) {
  const int pr = blockIdx.x * kET + threadIdx.x;
  if (pr >= npair) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(long long)b * npair + pr];
  G[pr] = s;
}

__global__ void __launch_bounds__(kET) combine_kernel(const double* __restrict__ U, int m, const double* __restrict__ C,
                                                      int q, long long n, double* __restrict__ Y) {
  __shared__ double sc[kEigMaxCols * kEigMaxCols];
  for (int i = threadIdx.x; i < m * q; i += kET) sc[i] = C[i];
  __syncthreads();
  for (long long row = (long long)blockIdx.x * kET + threadIdx.x; row < n; row += (long long)gridDim.x * kET) {
    double u[kEigMaxCols];
#pragma unroll
    for (int c = 0; c < kEigMaxCols; ++c) {
      u[c] = 0.0;
      if (c < m) u[c] = U[(long long)c * n + row];
    }
    for (int j = 0; j < q; ++j) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < kEigMaxCols; ++c)
        if (c < m) s += u[c] * sc[c * q + j];
      Y[(long long)j * n + row] = s;
    }
  }
}

__global__ void __launch_bounds__(kET) scale_kernel(double* __restrict__ X, const double* __restrict__ f, int k,
                                                    long long n) {
  for (long long i = (long long)blockIdx.x * kET + threadIdx.x; i < (long long)k * n; i += (long long)gridDim.x * kET)
    X[i] *= f[i / n];
}

}  // namespace

namespace {
// one Gram matrix into work slot `slot` (partials and result), copied to the
// host asynchronously on s
int gram_async(const double* U, int p, const double* V, int q, long long n, double* G_host, double* work, int slot,
               int nb, hipStream_t s) {
  if (p < 1 || q < 1 || p > kEigMaxCols || q > kEigMaxCols) return -1;
  const int npair = p * q;
  const long long per = (long long)nb * kEigMaxCols * kEigMaxCols + kEigMaxCols * kEigMaxCols;
  double* part = work + slot * per;
  double* G = part + (long long)nb * kEigMaxCols * kEigMaxCols;
  hipLaunchKernelGGL(gram_partial, dim3(nb), dim3(kET), 0, s, U, p, V, q, n, part);
  hipLaunchKernelGGL(gram_reduce, dim3((npair + kET - 1) / kET), dim3(kET), 0, s, part, npair, nb, G);
  return hipMemcpyAsync(G_host, G, sizeof(double) * npair, hipMemcpyDeviceToHost, s) == hipSuccess ? 0 : -1;
}
}  // namespace

int eig_grid(long long n, int ncu) {
  long long b = (n + kET - 1) / kET;
  const long long cap = 4LL * ncu;
  return (int)std::max(1LL, std::min(b, cap));
}

long long eig_gram_work(int nb) {
  return 2 * ((long long)nb * kEigMaxCols * kEigMaxCols + kEigMaxCols * kEigMaxCols);
}

int eig_gram(const double* U, int p, const double* V, int q, long long n, double* G_host, double* work, int nb,
             hipStream_t s) {
  if (gram_async(U, p, V, q, n, G_host, work, 0, nb, s)) return -1;
  return hipStreamSynchronize(s) == hipSuccess ? 0 : -1;
}

int eig_gram2(const double* U1, int p1, const double* V1, int q1, double* G1_host, const double* U2, int p2,
              const double* V2, int q2, double* G2_host, long long n, double* work, int nb, hipStream_t s) {
  if (gram_async(U1, p1, V1, q1, n, G1_host, work, 0, nb, s)) return -1;
  if (gram_async(U2, p2, V2, q2, n, G2_host, work, 1, nb, s)) return -1;
  return hipStreamSynchronize(s) == hipSuccess ? 0 : -1;
}

void eig_combine(const double* U, int m, const double* C_dev, int q, long long n, double* Y, int nb, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(nb), dim3(kET), 0, s, U, m, C_dev, q, n, Y);
}

void eig_scale(double* X, const double* f_dev, int k, long long n, int nb, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(kET), 0, s, X, f_dev, k, n);
}

}  // namespace gym
