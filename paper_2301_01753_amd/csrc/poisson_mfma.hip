// Mixed Poisson operator with bf16 contractions on the matrix cores
// (affine 3-D boxes, degree r >= 3; the GYM_BF16 precision of gym_op_apply).
//
// On an axis-aligned box every element carries the same element operator,
// assembled from the paper's section 2 objects restricted to one element:
//   y_s,c = s2_c M2ref s_c + B_c^T p      (flux component c, (r+1) r^2 values)
//   y_p   = sum_c B_c s_c                 (cell values, r^3)
// with M2ref = Mn (x) Me (x) Me in each component's own order (its normal axis
// first, so the three components share one matrix; s2_c = h_c^2 / |cell|) and
// B_c = -M3 D_c the element's -M3 times its divergence.  A batch of 32
// elements is one dense product per block, [rows x K] x [K x 32]: the
// element matrices are the A operand of v_mfma_f32_32x32x16_bf16 (pre-packed
// on the host in the instruction's lane order, rounded to bf16), the gathered
// element coefficients (FP32 vectors rounded to bf16) the B operand, FP32
// accumulation.  For r = 4 that is 111 matrix-core instructions per batch,
// 0.1 MFLOP per element.
//
// The element results go to an element-local buffer (row-major over local
// rows, elements contiguous, so every store of a batch is coalesced); a second
// kernel, one thread per global unknown, sums its contributions in a fixed
// order (the lower element first, at most two for a flux unknown on an
// element face) and writes y: deterministic, no atomics.  With the fused MINRES step it also
// adds z . A z per block.
//
// Lane layouts (gfx950, checked on the device): A is 32 x 16 with lane l
// holding A[l % 32][8 (l / 32) + j], j < 8; B is 16 x 32 with lane l holding
// B[8 (l / 32) + j][l % 32]; the 32 x 32 result D holds, in lane l and
// register v, D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "gym_internal.hpp"
#include "kernels.hpp"
#include "poisson_mfma.hpp"
#include "tile.hpp"

namespace gym {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int kBatch = 32;

// local flux index of component c: position along the normal axis c fastest,
// then axis (c+1)%3, then (c+2)%3
__host__ __device__ inline int flux_local(int r, int i_n, int i_1, int i_2) { return i_n + (r + 1) * (i_1 + r * i_2); }

template <int R>
struct Dims {
  static constexpr int NF = (R + 1) * R * R;   // flux values per component
  static constexpr int NC = R * R * R;         // cell values
  static constexpr int KF = (NF + 15) / 16;    // k-steps over a flux component
  static constexpr int KC = (NC + 15) / 16;    // k-steps over the cells
  static constexpr int TF = (NF + 31) / 32;    // 32-row tiles of a flux block
  static constexpr int TC = (NC + 31) / 32;    // 32-row tiles of the cell block
  static constexpr int ROWS = 3 * NF + NC;     // local rows of the element buffer
};

__device__ inline bf16x8 ld_frag(const uint16_t* p, int lane) {
  const uint4 v = reinterpret_cast<const uint4*>(p)[lane];
  bf16x8 f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return f;
}

// Element products of a batch of 32 elements; one wavefront per batch.
template <int R, bool MR>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) elem_kernel(const float* __restrict__ x, float* __restrict__ yel,
                                                  const uint16_t* __restrict__ frag, PoissonMfmaParams q) {
  using D = Dims<R>;
  const int lane = threadIdx.x;
  const long long E = (long long)q.nel[0] * q.nel[1] * q.nel[2];
  const long long e0 = (long long)blockIdx.x * kBatch;
  const int rhs = blockIdx.y;
  const float* xr = x + (long long)rhs * q.ndofs;
  float* yr = yel + (long long)rhs * q.el_stride;
  const long long e = e0 + (lane % 32);
  const bool live = e < E;
  int ec[3] = {0, 0, 0};
  if (live) {
    ec[0] = (int)(e % q.nel[0]);
    ec[1] = (int)((e / q.nel[0]) % q.nel[1]);
    ec[2] = (int)(e / ((long long)q.nel[0] * q.nel[1]));
  }
  const int kh = 8 * (lane / 32);  // this lane's first k within a 16-step
  // B fragments of the cell values, bf16 (those of a flux component are
  // gathered inside the component loop, so only one component is live)
  bf16x8 bp[D::KC];
  {
    const long long base = q.np_off;
    const long long m0 = q.m[0], m1 = q.m[1];
#pragma unroll
    for (int kt = 0; kt < D::KC; ++kt) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 16 * kt + kh + j;
        float v = 0.f;
        if (live && k < D::NC) {
          const int ix = k % R, iy = (k / R) % R, iz = k / (R * R);
          v = xr[base + (R * ec[0] + ix) + m0 * ((R * ec[1] + iy) + m1 * (R * ec[2] + iz))];
        }
        bp[kt][j] = (__bf16)v;
      }
    }
  }
  // fragment tables: M2ref [TF][KF], then per component B_c^T [TF][KC] and
  // B_c [TC][KF]; 512 bf16 per fragment
  const uint16_t* fM2 = frag;
  const uint16_t* fBT = fM2 + (size_t)D::TF * D::KF * 512;
  const uint16_t* fB = fBT + (size_t)3 * D::TF * D::KC * 512;
  floatx16 accp[D::TC];
#pragma unroll
  for (int t = 0; t < D::TC; ++t) accp[t] = floatx16{};
  const long long col = e0 + (lane % 32);
  const int rq = 4 * (lane / 32);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    bf16x8 bs[D::KF];
    {
      const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
      const DevComp& cd = q.s.c[c];
#pragma unroll
      for (int kt = 0; kt < D::KF; ++kt) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = 16 * kt + kh + j;
          float v = 0.f;
          if (live && k < D::NF) {
            const int i_n = k % (R + 1), t = k / (R + 1);
            const int i_1 = t % R, i_2 = t / R;
            int p[3];
            p[c] = R * ec[c] + i_n;
            p[a1] = R * ec[a1] + i_1;
            p[a2] = R * ec[a2] + i_2;
            v = xr[cd.offset + p[0] + (long long)cd.count[0] * (p[1] + (long long)cd.count[1] * p[2])];
          }
          bs[kt][j] = (__bf16)v;
        }
      }
    }
    floatx16 a1[D::TF], a2[D::TF];
#pragma unroll
    for (int t = 0; t < D::TF; ++t) {
      a1[t] = floatx16{};
      a2[t] = floatx16{};
#pragma unroll
      for (int kt = 0; kt < D::KF; ++kt)
        a1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld_frag(fM2 + (size_t)(t * D::KF + kt) * 512, lane),
                                                       bs[kt], a1[t], 0, 0, 0);
#pragma unroll
      for (int kt = 0; kt < D::KC; ++kt)
        a2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            ld_frag(fBT + (size_t)((c * D::TF + t) * D::KC + kt) * 512, lane), bp[kt], a2[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < D::TC; ++t)
#pragma unroll
      for (int kt = 0; kt < D::KF; ++kt)
        accp[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            ld_frag(fB + (size_t)((c * D::TC + t) * D::KF + kt) * 512, lane), bs[kt], accp[t], 0, 0, 0);
    // y_s,c = s2_c (M2ref s_c) + B_c^T p, rows c NF + local
    if (live) {
      const float s2 = q.s2[c];
#pragma unroll
      for (int t = 0; t < D::TF; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = 32 * t + 8 * (v / 4) + rq + v % 4;
          if (row < D::NF) yr[(long long)(c * D::NF + row) * q.el_rows + col] = s2 * a1[t][v] + a2[t][v];
        }
    }
  }
  if (live) {
#pragma unroll
    for (int t = 0; t < D::TC; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = 32 * t + 8 * (v / 4) + rq + v % 4;
        if (row < D::NC) yr[(long long)(3 * D::NF + row) * q.el_rows + col] = accp[t][v];
      }
  }
}

// Sum the element contributions of every global unknown into y: one thread
// per unknown, in the vector's own order, so every store of y is coalesced and
// each 64-byte line of it is written once; the reads of the element buffer come
// as a few contiguous runs per wavefront (a run per local row, elements
// contiguous).  A flux unknown on an interior face (normal position a multiple
// of r, not on the boundary) sums the lower element's upper-face row and the
// upper element's lower-face row, in that order; every other unknown has one
// contribution.  With MR also partial sums of z . (A z) per block.
template <int R, bool MR>
__global__ void __launch_bounds__(256) gather_kernel(const float* __restrict__ x, float* __restrict__ y,
                                                     const float* __restrict__ yel, PoissonMfmaParams q) {
  using D = Dims<R>;
  const int rhs = blockIdx.y;
  const float* yr = yel + (long long)rhs * q.el_stride;
  const long long off = (long long)rhs * q.ndofs;
  const long long E = q.el_rows;
  const unsigned n0 = (unsigned)q.nel[0], n01 = (unsigned)q.nel[0] * (unsigned)q.nel[1];
  double acc = 0.0;
  for (long long g = (long long)blockIdx.x * 256 + threadIdx.x; g < q.ndofs; g += (long long)gridDim.x * 256) {
    float v;
    if (g >= q.np_off) {
      const unsigned idx = (unsigned)(g - q.np_off);
      const unsigned m0 = (unsigned)q.m[0], m1 = (unsigned)q.m[1];
      const unsigned px = idx % m0, t = idx / m0, py = t % m1, pz = t / m1;
      const long long e = (long long)(px / R) + n0 * (py / R) + (long long)n01 * (pz / R);
      const int k = (int)(px % R) + R * ((int)(py % R) + R * (int)(pz % R));
      v = yr[(long long)(3 * D::NF + k) * E + e];
    } else {
      const int c = g >= q.s.c[2].offset ? 2 : (g >= q.s.c[1].offset ? 1 : 0);
      const DevComp& cd = q.s.c[c];
      const unsigned idx = (unsigned)(g - cd.offset);
      const unsigned c0 = (unsigned)cd.count[0], c1 = (unsigned)cd.count[1];
      const unsigned q0 = idx % c0, t = idx / c0, q1 = t % c1, q2 = t / c1;
      // positions along the normal axis c and the tangential axes c+1, c+2
      const unsigned pn = c == 0 ? q0 : (c == 1 ? q1 : q2);
      const unsigned pt1 = c == 0 ? q1 : (c == 1 ? q2 : q0);
      const unsigned pt2 = c == 0 ? q2 : (c == 1 ? q0 : q1);
      const int nc = c == 0 ? q.nel[0] : (c == 1 ? q.nel[1] : q.nel[2]);
      int en = (int)(pn / R), i_n = (int)(pn % R);
      if (en == nc) {  // upper boundary face: the last element's upper row
        en = nc - 1;
        i_n = R;
      }
      const unsigned e1 = pt1 / R, e2 = pt2 / R;
      const int i_1 = (int)(pt1 % R), i_2 = (int)(pt2 % R);
      const unsigned ex = c == 0 ? (unsigned)en : (c == 1 ? e2 : e1);
      const unsigned ey = c == 0 ? e1 : (c == 1 ? (unsigned)en : e2);
      const unsigned ez = c == 0 ? e2 : (c == 1 ? e1 : (unsigned)en);
      const long long e = (long long)ex + (long long)n0 * ey + (long long)n01 * ez;
      const int row = c * D::NF + flux_local(R, i_n, i_1, i_2);
      v = yr[(long long)row * E + e];
      if (i_n == 0 && en > 0) {
        const long long se = c == 0 ? 1 : (c == 1 ? (long long)n0 : (long long)n01);
        v = yr[(long long)(row + R) * E + (e - se)] + v;
      }
    }
    y[off + g] = v;
    if constexpr (MR) acc += (double)x[off + g] * (double)v;
  }
  if constexpr (MR) {
    __shared__ double sh[256];
    double a[1] = {acc};
    wg_sums<256, 1>(a, sh);
    if (threadIdx.x == 0) q.mr.pa[(long long)rhs * gridDim.x + blockIdx.x] = a[0];
  }
}

// Host: round to bf16 (nearest even)
uint16_t bf16_bits(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Pack a rows x cols row-major matrix into 32 x 16 A fragments [tile][kstep]
void pack(const std::vector<double>& M, int rows, int cols, std::vector<uint16_t>& out) {
  const int T = (rows + 31) / 32, K = (cols + 15) / 16;
  for (int t = 0; t < T; ++t)
    for (int kt = 0; kt < K; ++kt)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const int i = 32 * t + l % 32, k = 16 * kt + 8 * (l / 32) + j;
          out.push_back(bf16_bits(i < rows && k < cols ? (float)M[(size_t)i * cols + k] : 0.f));
        }
}

template <int R>
int launch_r(const PoissonMfmaParams& q, const uint16_t* frag, int nrhs, bool mr, int ncu, hipStream_t s) {
  const long long E = (long long)q.nel[0] * q.nel[1] * q.nel[2];
  dim3 g1((unsigned)((E + kBatch - 1) / kBatch), (unsigned)nrhs);
  dim3 g2((unsigned)q.gather_blocks, (unsigned)nrhs);
  const float* x = static_cast<const float*>(q.x);
  float* y = static_cast<float*>(q.y);
  float* yel = static_cast<float*>(q.yel);
  hipLaunchKernelGGL((elem_kernel<R, false>), g1, dim3(64), 0, s, x, yel, frag, q);
  if (mr) hipLaunchKernelGGL((gather_kernel<R, true>), g2, dim3(256), 0, s, x, y, yel, q);
  else hipLaunchKernelGGL((gather_kernel<R, false>), g2, dim3(256), 0, s, x, y, yel, q);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int poisson_mfma_rows(int r) { return 3 * (r + 1) * r * r + r * r * r; }

int poisson_mfma_gather_blocks(long long ndofs, int ncu) {
  long long b = (ndofs + 255) / 256;
  const long long cap = 8LL * ncu;
  return (int)(b < cap ? b : cap);
}

std::vector<uint16_t> poisson_mfma_fragments(int r, const std::vector<double>& mn, const std::vector<double>& me,
                                             double s3) {
  const int NF = (r + 1) * r * r, NC = r * r * r;
  // M2ref = Mn (x) Me (x) Me in the local order (normal index fastest)
  std::vector<double> M2((size_t)NF * NF);
  for (int a = 0; a < NF; ++a)
    for (int b = 0; b < NF; ++b) {
      const int an = a % (r + 1), at = a / (r + 1), a1 = at % r, a2 = at / r;
      const int bn = b % (r + 1), bt = b / (r + 1), b1 = bt % r, b2 = bt / r;
      M2[(size_t)a * NF + b] = mn[an * (r + 1) + bn] * me[a1 * r + b1] * me[a2 * r + b2];
    }
  // element M3 = s3 Me (x) Me (x) Me over cells (x fastest)
  std::vector<double> M3((size_t)NC * NC);
  for (int a = 0; a < NC; ++a)
    for (int b = 0; b < NC; ++b) {
      const int ax = a % r, ay = (a / r) % r, az = a / (r * r);
      const int bx = b % r, by = (b / r) % r, bz = b / (r * r);
      M3[(size_t)a * NC + b] = s3 * me[ax * r + bx] * me[ay * r + by] * me[az * r + bz];
    }
  std::vector<uint16_t> out;
  pack(M2, NF, NF, out);
  std::vector<std::vector<double>> B(3, std::vector<double>((size_t)NC * NF, 0.0));
  for (int c = 0; c < 3; ++c) {
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    // D_c: cell (i, j, k) <- flux at +1 minus flux at 0 along c
    std::vector<double> Dc((size_t)NC * NF, 0.0);
    for (int cell = 0; cell < NC; ++cell) {
      int id[3] = {cell % r, (cell / r) % r, cell / (r * r)};
      for (int sgn = 0; sgn < 2; ++sgn) {
        const int k = flux_local(r, id[c] + sgn, id[a1], id[a2]);
        Dc[(size_t)cell * NF + k] += sgn ? 1.0 : -1.0;
      }
    }
    for (int a = 0; a < NC; ++a)
      for (int b = 0; b < NF; ++b) {
        double s = 0.0;
        for (int k = 0; k < NC; ++k) s += M3[(size_t)a * NC + k] * Dc[(size_t)k * NF + b];
        B[c][(size_t)a * NF + b] = -s;
      }
  }
  for (int c = 0; c < 3; ++c) {
    std::vector<double> BT((size_t)NF * NC);
    for (int a = 0; a < NC; ++a)
      for (int b = 0; b < NF; ++b) BT[(size_t)b * NC + a] = B[c][(size_t)a * NF + b];
    pack(BT, NF, NC, out);
  }
  for (int c = 0; c < 3; ++c) pack(B[c], NC, NF, out);
  return out;
}

int launch_poisson_mfma(const PoissonMfmaParams& q, const uint16_t* frag, int r, int nrhs, bool mr, int ncu,
                        hipStream_t s) {
  switch (r) {
    case 3: return launch_r<3>(q, frag, nrhs, mr, ncu, s);
    case 4: return launch_r<4>(q, frag, nrhs, mr, ncu, s);
  }
  return -2;
}

}  // namespace gym
