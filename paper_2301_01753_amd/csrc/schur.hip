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
// A workgroup computes 16 RT lines x 16 RT outputs (RT = 4), a thread RT x RT
// of them, interleaved (lines a + 16 u, outputs b + 16 v): lanes run along the
// outputs for the x axis (contiguous in memory) and along the lines for y
// and z, so the LDS reads of a k step are consecutive words and the stores
// are coalesced.  Each output sums its k terms in ascending order whatever
// RT.  Every kernel here does nothing for a right-hand side whose Krylov
// state in `gate` (if given) has converged.
// Block (bx: line block, by: output block) of the transform of one vector.
template <int AX, typename T, int RT = 4>
__device__ __forceinline__ void axis_gemm_block(const T* __restrict__ in, T* __restrict__ out,
                                                const T* __restrict__ A, int m0, int m1, int m2, long long bx,
                                                int by) {
  constexpr int TL = 16 * RT, TI = 16 * RT;
  __shared__ T s_in[kTK][TL + 4];
  __shared__ T sa[kTK][TI + 4];
  const int ma = AX == 0 ? m0 : (AX == 1 ? m1 : m2);
  const long long nlines = (long long)m0 * m1 * m2 / ma;
  const long long stride = AX == 0 ? 1 : (AX == 1 ? (long long)m0 : (long long)m0 * m1);
  const long long L0 = bx * TL;
  const int i0 = by * TI;
  // memory offset of the first entry of line L
  auto base = [&](long long L) -> long long {
    if (AX == 0) return L * m0;
    if (AX == 1) return (L % m0) + (long long)m0 * m1 * (L / m0);
    return L;
  };
  const int t = threadIdx.x;
  const int a = AX == 0 ? t / 16 : t % 16;  // line group
  const int b = AX == 0 ? t % 16 : t / 16;  // output group
  T acc[RT][RT];
#pragma unroll
  for (int u = 0; u < RT; ++u)
#pragma unroll
    for (int v = 0; v < RT; ++v) acc[u][v] = 0;
  for (int k0 = 0; k0 < ma; k0 += kTK) {
    // stage kTK contraction entries of TL lines and of TI rows of A
    for (int e = t; e < kTK * TL; e += kGT) {
      int kk, ll;
      if (AX == 0) {
        ll = e / kTK;
        kk = e % kTK;
      } else {
        ll = e % TL;
        kk = e / TL;
      }
      const long long L = L0 + ll;
      const int k = k0 + kk;
      s_in[kk][ll] = (L < nlines && k < ma) ? in[base(L) + stride * k] : T(0);
    }
    for (int e = t; e < kTK * TI; e += kGT) {
      const int ii = e / kTK, kk = e % kTK;
      const int i = i0 + ii, k = k0 + kk;
      sa[kk][ii] = (i < ma && k < ma) ? A[(long long)i * ma + k] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTK; ++kk) {
      T x[RT], y[RT];
#pragma unroll
      for (int u = 0; u < RT; ++u) x[u] = s_in[kk][a + 16 * u];
#pragma unroll
      for (int v = 0; v < RT; ++v) y[v] = sa[kk][b + 16 * v];
#pragma unroll
      for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int v = 0; v < RT; ++v) acc[u][v] += y[v] * x[u];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < RT; ++u) {
    const long long L = L0 + a + 16 * u;
    if (L >= nlines) continue;
    const long long o = base(L);
#pragma unroll
    for (int v = 0; v < RT; ++v) {
      const int i = i0 + b + 16 * v;
      if (i < ma) out[o + stride * i] = acc[u][v];
    }
  }
}

template <int AX, typename T, int RT>
__global__ void __launch_bounds__(kGT) axis_gemm(const T* __restrict__ in, T* __restrict__ out,
                                                 const T* __restrict__ A, int m0, int m1, int m2, long long vin,
                                                 long long vout, const MinresState* gate) {
  if (gate && gate[blockIdx.z].done) return;
  axis_gemm_block<AX, T, RT>(in + (long long)blockIdx.z * vin, out + (long long)blockIdx.z * vout, A, m0, m1, m2,
                             blockIdx.x, blockIdx.y);
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
  // (8 x 8 per thread, 128 x 128 tiles, measured no faster on the 256-cell
  // axes of the 64^3 degree-4 mesh: 2.28 against 2.08 ms per FP64 apply)
  dim3 grid((unsigned)((nlines + kTL - 1) / kTL), (unsigned)((m[AX] + kTI - 1) / kTI), (unsigned)nrhs);
  hipLaunchKernelGGL((axis_gemm<AX, T, 4>), grid, dim3(kGT), 0, s, in, out, A, m[0], m[1], m[2], vin, vout, gate);
}

__device__ __forceinline__ int item_of(const int* start, int nitem, int blk) {
  int lo = 0, hi = nitem;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= blk) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Ragged batch, elementwise parts: stage 0 the flux diagonal, stage 1 the
// division by the eigenvalue sums, stage 2 the partial sums y . z, z . r2.
template <int STAGE>
__global__ void __launch_bounds__(256) schur_batch_elem(const SchurItem* items, const int* start, int nitem) {
  __shared__ double sh[2 * 256];
  const int i = item_of(start, nitem, blockIdx.x);
  const SchurItem& it = items[i];
  if (it.gate && it.gate->done) return;
  const int blk = blockIdx.x - start[i];
  const long long stride = (long long)it.nb * 256;
  if constexpr (STAGE == 0) {
    for (long long g = (long long)blk * 256 + threadIdx.x; g < it.ns; g += stride) it.z[g] = it.dsinv[g] * it.y[g];
  } else if constexpr (STAGE == 1) {
    const int m0 = it.m[0], m1 = it.m[1];
    for (long long g = (long long)blk * 256 + threadIdx.x; g < it.np; g += stride) {
      const int a = (int)(g % m0);
      const long long r = g / m0;
      const int b = (int)(r % m1), c = (int)(r / m1);
      it.w0[g] *= it.scale / (it.lam[a] + it.lam[m0 + b] + it.lam[m0 + m1 + c]);
    }
  } else {
    const long long n = it.ns + it.np;
    double a = 0.0, c = 0.0;
    for (long long g = (long long)blk * 256 + threadIdx.x; g < n; g += stride) {
      const double zi = it.z[g];
      a += it.y[g] * zi;
      c += zi * it.r2[g];
    }
    double t[2] = {a, c};
    wg_sums<256, 2>(t, sh);
    if (threadIdx.x == 0) {
      it.pb[blk] = t[0];
      it.pc[blk] = t[1];
    }
  }
}

// Ragged batch, one 1-D transform along AX: FWD y_p -> w0 (x), w0 -> w1 (y),
// w1 -> w0 (z); backward w0 -> w1 (z), w1 -> w0 (y), w0 -> z_p (x).
template <int AX, bool FWD>
__global__ void __launch_bounds__(kGT) schur_batch_axis(const SchurItem* items, const int* start, int nitem) {
  const int i = item_of(start, nitem, blockIdx.x);
  const SchurItem& it = items[i];
  if (it.gate && it.gate->done) return;
  const int blk = blockIdx.x - start[i];
  const int nob = (it.m[AX] + kTI - 1) / kTI;
  const double* in;
  double* out;
  if constexpr (FWD) {
    in = AX == 0 ? it.y + it.ns : (AX == 1 ? it.w0 : it.w1);
    out = AX == 0 ? it.w0 : (AX == 1 ? it.w1 : it.w0);
  } else {
    in = AX == 2 ? it.w0 : (AX == 1 ? it.w1 : it.w0);
    out = AX == 2 ? it.w1 : (AX == 1 ? it.w0 : it.z + it.ns);
  }
  axis_gemm_block<AX, double>(in, out, FWD ? it.fwd[AX] : it.bwd[AX], it.m[0], it.m[1], it.m[2], blk / nob,
                              blk % nob);
}

}  // namespace

int schur_axis_blocks(const SchurItem& it, int a) {
  const long long nlines = (long long)it.m[0] * it.m[1] * it.m[2] / it.m[a];
  return (int)(((nlines + kTL - 1) / kTL) * ((it.m[a] + kTI - 1) / kTI));
}

void launch_schur_batch(const SchurItem* items, int nitem, const int* est, int ne, const int* const ast[3],
                        const int na[3], hipStream_t s) {
  hipLaunchKernelGGL((schur_batch_elem<0>), dim3(ne), dim3(256), 0, s, items, est, nitem);
  hipLaunchKernelGGL((schur_batch_axis<0, true>), dim3(na[0]), dim3(kGT), 0, s, items, ast[0], nitem);
  hipLaunchKernelGGL((schur_batch_axis<1, true>), dim3(na[1]), dim3(kGT), 0, s, items, ast[1], nitem);
  hipLaunchKernelGGL((schur_batch_axis<2, true>), dim3(na[2]), dim3(kGT), 0, s, items, ast[2], nitem);
  hipLaunchKernelGGL((schur_batch_elem<1>), dim3(ne), dim3(256), 0, s, items, est, nitem);
  hipLaunchKernelGGL((schur_batch_axis<2, false>), dim3(na[2]), dim3(kGT), 0, s, items, ast[2], nitem);
  hipLaunchKernelGGL((schur_batch_axis<1, false>), dim3(na[1]), dim3(kGT), 0, s, items, ast[1], nitem);
  hipLaunchKernelGGL((schur_batch_axis<0, false>), dim3(na[0]), dim3(kGT), 0, s, items, ast[0], nitem);
  hipLaunchKernelGGL((schur_batch_elem<2>), dim3(ne), dim3(256), 0, s, items, est, nitem);
}

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
