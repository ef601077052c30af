// Block preconditioner of the mixed Poisson operator on affine boxes (device
// part; the set-up is schur.cpp).
//
// For A = [[M2, -D^T M3], [-M3 D, 0]] (paper section 2 objects: the mass
// matrices M_p and the incidence D) the block-diagonal preconditioner
//   P = diag(diag(M2), S),  S = M3 D diag(M2)^-1 D^T M3,
// keeps the spectrum of P^-1 A in mesh-independent intervals: diag(M2) is
// spectrally equivalent to M2 (each 1-D factor by a factor <= 3), and S is then
// the Schur complement of the same block system.  On an axis-aligned box S has
// Kronecker structure: with per-axis 1-D factors, D diag(M2)^-1 D^T is a sum
// over axes of (tridiagonal T_a on axis a) x (diagonal W_b on the others), and
// M3 = s3 (x)_a Me_a.  Simultaneous diagonalisation (Lynch, Rice & Thomas 1964)
// then gives S^-1 = s3^-2 (x)_a Vt_a  Lambda^-1  (x)_a Vt_a^T with dense m_a x m_a
// factors Vt_a = Me_a^-1 V_a (V_a^T T_a V_a = diag(lam_a), V_a^T W_a V_a = I) and
// Lambda = sum_a lam_a / s2_a on the cell lattice.
//
// The cell block is applied as six dense 1-D transforms along the three axes
// (axis_gemm) and one pointwise division; the flux block as a diagonal.
#include <hip/hip_runtime.h>

#include "gym_internal.hpp"
#include "minres_step.hpp"
#include "schur.hpp"

namespace gym {

namespace {

constexpr int kTL = 64;  // lines per tile
constexpr int kTI = 64;  // outputs per tile
constexpr int kTK = 16;  // contraction chunk
constexpr int kGT = 256; // threads

// out[line][i] = sum_l A[i][l] in[line][l] along axis AX of an m0 x m1 x m2
// lattice (x fastest), A row-major m_a x m_a.  blockIdx.z: right-hand side.
// A thread computes 4 lines x 4 outputs; lanes run along the outputs for the
// x axis (contiguous in memory) and along the lines for y and z.  Every
// kernel here does nothing for a right-hand side whose Krylov state in `gate`
// (if given) has converged.
template <int AX, typename T>
__global__ void __launch_bounds__(kGT) axis_gemm(const T* __restrict__ in, T* __restrict__ out,
                                                 const T* __restrict__ A, int m0, int m1, int m2, long long vin,
                                                 long long vout, const MinresState* gate) {
  __shared__ T s_in[kTK][kTL + 4];
  __shared__ T sa[kTK][kTI + 4];
  if (gate && gate[blockIdx.z].done) return;
  const int ma = AX == 0 ? m0 : (AX == 1 ? m1 : m2);
  const long long nlines = (long long)m0 * m1 * m2 / ma;
  const long long stride = AX == 0 ? 1 : (AX == 1 ? (long long)m0 : (long long)m0 * m1);
  const long long L0 = (long long)blockIdx.x * kTL;
  const int i0 = blockIdx.y * kTI;
  in += (long long)blockIdx.z * vin;
  out += (long long)blockIdx.z * vout;
  // memory offset of the first entry of line L
  auto base = [&](long long L) -> long long {
    if (AX == 0) return L * m0;
    if (AX == 1) return (L % m0) + (long long)m0 * m1 * (L / m0);
    return L;
  };
  const int t = threadIdx.x;
  const int a = AX == 0 ? t / 16 : t % 16;  // line group
  const int b = AX == 0 ? t % 16 : t / 16;  // output group
  T acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0;
  for (int k0 = 0; k0 < ma; k0 += kTK) {
    // stage kTK contraction entries of kTL lines and of kTI rows of A
    for (int e = t; e < kTK * kTL; e += kGT) {
      int kk, ll;
      if (AX == 0) {
        ll = e / kTK;
        kk = e % kTK;
      } else {
        ll = e % kTL;
        kk = e / kTL;
      }
      const long long L = L0 + ll;
      const int k = k0 + kk;
      s_in[kk][ll] = (L < nlines && k < ma) ? in[base(L) + stride * k] : T(0);
    }
    for (int e = t; e < kTK * kTI; e += kGT) {
      const int ii = e / kTK, kk = e % kTK;
      const int i = i0 + ii, k = k0 + kk;
      sa[kk][ii] = (i < ma && k < ma) ? A[(long long)i * ma + k] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTK; ++kk) {
      T x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = s_in[kk][4 * a + u];
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] = sa[kk][4 * b + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += y[v] * x[u];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long long L = L0 + 4 * a + u;
    if (L >= nlines) continue;
    const long long o = base(L);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 4 * b + v;
      if (i < ma) out[o + stride * i] = acc[u][v];
    }
  }
}

// y[i, j, k] *= scale / (lam0[i] + lam1[j] + lam2[k]) on the cell lattice
template <typename T>
__global__ void __launch_bounds__(256) lam_scale(T* __restrict__ y, const double* __restrict__ lam, int m0, int m1,
                                                 int m2, double scale, long long vstride, const MinresState* gate) {
  if (gate && gate[blockIdx.y].done) return;
  const long long n = (long long)m0 * m1 * m2;
  y += (long long)blockIdx.y * vstride;
  for (long long g = (long long)blockIdx.x * 256 + threadIdx.x; g < n; g += (long long)gridDim.x * 256) {
    const int i = (int)(g % m0);
    const long long r = g / m0;
    const int j = (int)(r % m1), k = (int)(r / m1);
    y[g] = static_cast<T>(static_cast<double>(y[g]) * (scale / (lam[i] + lam[m0 + j] + lam[m0 + m1 + k])));
  }
}

// z = d .* y on the flux block
template <typename T>
__global__ void __launch_bounds__(256) diag_scale(const T* __restrict__ y, T* __restrict__ z,
                                                  const double* __restrict__ d, long long n, long long vstride,
                                                  const MinresState* gate) {
  if (gate && gate[blockIdx.y].done) return;
  y += (long long)blockIdx.y * vstride;
  z += (long long)blockIdx.y * vstride;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    z[i] = static_cast<T>(d[i] * static_cast<double>(y[i]));
}

template <int AX, typename T>
void axis_launch(const T* in, long long vin, T* out, long long vout, const T* A, const int m[3], int nrhs,
                 const MinresState* gate, hipStream_t s) {
  const long long nlines = (long long)m[0] * m[1] * m[2] / m[AX];
  dim3 grid((unsigned)((nlines + kTL - 1) / kTL), (unsigned)((m[AX] + kTI - 1) / kTI), (unsigned)nrhs);
  hipLaunchKernelGGL((axis_gemm<AX, T>), grid, dim3(kGT), 0, s, in, out, A, m[0], m[1], m[2], vin, vout, gate);
}

}  // namespace

template <typename T>
int launch_schur_apply(const SchurPrec& P, const T* y, T* z, int nrhs, int nb, hipStream_t s,
                       const MinresState* gate) {
  const T* const* F = P.template fwd<T>();
  const T* const* B = P.template bwd<T>();
  if (nrhs > P.work_nrhs) return -1;
  T* w0 = P.template work_vec<T>(0);
  T* w1 = P.template work_vec<T>(1);
  const long long n = P.ns + P.np, np = P.np;
  // flux block
  hipLaunchKernelGGL((diag_scale<T>), dim3(nb, nrhs), dim3(256), 0, s, y, z, P.dsinv, P.ns, n, gate);
  // cell block: forward transforms, division, backward transforms
  const T* yp = y + P.ns;
  T* zp = z + P.ns;
  axis_launch<0, T>(yp, n, w0, np, F[0], P.m, nrhs, gate, s);
  axis_launch<1, T>(w0, np, w1, np, F[1], P.m, nrhs, gate, s);
  axis_launch<2, T>(w1, np, w0, np, F[2], P.m, nrhs, gate, s);
  hipLaunchKernelGGL((lam_scale<T>), dim3(nb, nrhs), dim3(256), 0, s, w0, P.lam, P.m[0], P.m[1], P.m[2], P.scale,
                     np, gate);
  axis_launch<2, T>(w0, np, w1, np, B[2], P.m, nrhs, gate, s);
  axis_launch<1, T>(w1, np, w0, np, B[1], P.m, nrhs, gate, s);
  axis_launch<0, T>(w0, np, zp, n, B[0], P.m, nrhs, gate, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_schur_apply<double>(const SchurPrec&, const double*, double*, int, int, hipStream_t,
                                        const MinresState*);
template int launch_schur_apply<float>(const SchurPrec&, const float*, float*, int, int, hipStream_t,
                                       const MinresState*);

}  // namespace gym
