// Mass applies on curved cells (included by op_kernel.hpp).
//
// The element mass of paper section 2, (M_p)_ij = int (Lambda_i, Lambda_j)_p,
// pulled back to the reference cube: three 1-D contractions of the lattice
// coefficients to the Gauss points (tables phi, e at q = r + 1 points), the
// pointwise metric of the cell map (geom.hpp: det J, 1/det J, or the 3x3
// Piola metrics, precomputed per Gauss point), and the three transposed
// contractions with Gauss-weighted tables.
//
// Each contraction stage gives a thread one 1-D line: the n coefficients of
// one element along the axis in, its q Gauss-point values out (or the
// reverse).  The table entries are then compile-time indices, so they are
// uniform over the wavefront and sit in scalar registers, and every value read
// from LDS feeds q (or n) fused multiply-adds.  The z contraction, the metric
// and the transposed z contraction run as one stage: a thread owns the q
// Gauss points of one (x, y) column of a layer, for all three components of a
// vector field, so the metric mixes components in registers.  Positions shared
// by neighbouring elements (nodal axes) are summed by the thread of the upper
// element in a fixed order: lower element first.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/gym.h"
#include "geom.hpp"
#include "tile.hpp"

namespace gym {

// The x Gauss-point dimension of the work arrays (QX = Q EX entries) is stored
// point-major: Gauss point t of local element e at t EX + e.  The x stages give
// consecutive lanes consecutive elements, so their LDS accesses are
// consecutive words (element-major, Q words apart, they collide in banks).
template <class C>
__device__ __forceinline__ constexpr int xq(int e, int t) {
  return t * C::EX + e;
}

// Where a layer's Gauss points sit in the metric lattice of geom.hpp.
template <typename TC>
struct QGeom {
  const TC* qd;       // field-major Gauss-point metrics
  long long fs;       // values per field
  int gx0, gy0, gz0;  // lattice index of the closure's first point in x, y; the layer's first in z
  int GX, GY;         // points per row and per column of the metric lattice
};

// x: in [NX][NY][NZ] lattice -> out [QX][NY][NZ]; line l = (element, row)
// Gauss-point values of elements outside the mesh are not masked here: the z
// stage (cz_scalar, cz_vector) replaces every column of such an element by
// zeros, so whatever these stages computed for it is never used.
template <class C, int TM, typename TC>
__device__ __forceinline__ void cfwd_x(const TC* __restrict__ in, TC* __restrict__ out, int l) {
  constexpr int NX = C::nx(TM), R = C::R, Q = C::Q;
  constexpr bool N = TM & 1;
  constexpr int n = N ? R + 1 : R;
  const int e = l % C::EX, rest = l / C::EX;
  const TC* s = in + rest * NX + R * e;
  TC v[n];
#pragma unroll
  for (int i = 0; i < n; ++i) v[i] = s[i];
  TC* o = out + rest * C::QX + e;
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    TC acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += ctab<TC, R, N, false>(t, i) * v[i];
    o[xq<C>(0, t)] = acc;
  }
}

// y: in [QX][NY][NZ] -> out [QX][QY][NZ]; line l = (qx, element, z row), qx
// the stored x index (xq)
template <class C, int TM, typename TC>
__device__ __forceinline__ void cfwd_y(const TC* __restrict__ in, TC* __restrict__ out, int l) {
  constexpr int NY = C::ny(TM), R = C::R, Q = C::Q, QX = C::QX;
  constexpr bool N = TM & 2;
  constexpr int n = N ? R + 1 : R;
  const int qx = l % QX, r2 = l / QX;
  const int e = r2 % C::EY, k = r2 / C::EY;
  const TC* s = in + qx + QX * (R * e + NY * k);
  TC v[n];
#pragma unroll
  for (int i = 0; i < n; ++i) v[i] = s[QX * i];
  TC* o = out + qx + QX * (Q * e + C::QY * k);
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    TC acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += ctab<TC, R, N, false>(t, i) * v[i];
    o[QX * t] = acc;
  }
}

// z forward contraction of one column p of B ([QX][QY][NZ]) into u[0..Q)
template <class C, int TM, typename TC>
__device__ __forceinline__ void cz_fwd(const TC* __restrict__ B, int p, TC (&u)[C::Q]) {
  constexpr int P = C::QX * C::QY, R = C::R, Q = C::Q;
  constexpr bool N = TM & 4;
  constexpr int n = N ? R + 1 : R;
  TC v[n];
#pragma unroll
  for (int i = 0; i < n; ++i) v[i] = B[p + P * i];
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    TC acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += ctab<TC, R, N, false>(t, i) * v[i];
    u[t] = acc;
  }
}

// transposed weighted z contraction of u back into column p of B
template <class C, int TM, typename TC>
__device__ __forceinline__ void cz_bwd(TC* __restrict__ B, int p, const TC (&u)[C::Q]) {
  constexpr int P = C::QX * C::QY, R = C::R, Q = C::Q;
  constexpr bool N = TM & 4;
  constexpr int NZ = C::nz(TM);
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    TC acc = 0;
#pragma unroll
    for (int t = 0; t < Q; ++t) acc += ctab<TC, R, N, true>(t, k) * u[t];
    B[p + P * k] = acc;
  }
}

// Gauss-point metric lattice offset of column p of the layer (point t = 0),
// or -1 when the column belongs to an element outside the mesh
template <class C, typename TC>
__device__ __forceinline__ long long cz_base(int p, const ElemRange& er, const QGeom<TC>& g) {
  const int qxs = p % C::QX, qy = p / C::QX;
  const int ex = qxs % C::EX, tx = qxs / C::EX, ey = qy / C::Q;
  if (ex < er.xlo || ex >= er.xhi || ey < er.ylo || ey >= er.yhi) return -1;
  return (long long)(g.gx0 + C::Q * ex + tx) + (long long)g.GX * ((long long)(g.gy0 + qy) + (long long)g.GY * g.gz0);
}

// z stage of a scalar mass (H1: det J, L2: 1/det J) on column p, in place
template <class C, int TM, int KIND, typename TC>
__device__ __forceinline__ void cz_scalar(TC* B, int p, const ElemRange& er, const QGeom<TC>& g, TC sign) {
  constexpr int Q = C::Q;
  TC u[Q];
  cz_fwd<C, TM>(B, p, u);
  const long long base = cz_base<C>(p, er, g);
  if (base >= 0) {
    const TC* m = g.qd + (KIND == GYM_H1 ? QF_DET : QF_INVDET) * g.fs + base;
    const long long plane = (long long)g.GX * g.GY;
#pragma unroll
    for (int t = 0; t < Q; ++t) u[t] *= sign * m[plane * t];
  } else {
#pragma unroll
    for (int t = 0; t < Q; ++t) u[t] = 0;
  }
  cz_bwd<C, TM>(B, p, u);
}

// z stage of a vector mass (HCURL or HDIV metric, symmetric 3x3) on column p
// of the three component arrays, in place
template <class C, int KIND, int T0, int T1, int T2, typename TC>
__device__ __forceinline__ void cz_vector(TC* const B[3], int p, const ElemRange& er, const QGeom<TC>& g, TC sign) {
  constexpr int Q = C::Q;
  TC u0[Q], u1[Q], u2[Q];
  cz_fwd<C, T0>(B[0], p, u0);
  cz_fwd<C, T1>(B[1], p, u1);
  cz_fwd<C, T2>(B[2], p, u2);
  const long long base = cz_base<C>(p, er, g);
  if (base >= 0) {
    const long long fs = g.fs, plane = (long long)g.GX * g.GY;
    const TC* m = g.qd + (KIND == GYM_HCURL ? QF_HCURL : QF_HDIV) * fs + base;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const TC* mt = m + plane * t;
      const TC m00 = mt[0], m01 = mt[fs], m02 = mt[2 * fs], m11 = mt[3 * fs], m12 = mt[4 * fs], m22 = mt[5 * fs];
      const TC a = u0[t], b = u1[t], c = u2[t];
      u0[t] = sign * (m00 * a + m01 * b + m02 * c);
      u1[t] = sign * (m01 * a + m11 * b + m12 * c);
      u2[t] = sign * (m02 * a + m12 * b + m22 * c);
    }
  } else {
#pragma unroll
    for (int t = 0; t < Q; ++t) u0[t] = u1[t] = u2[t] = 0;
  }
  cz_bwd<C, T0>(B[0], p, u0);
  cz_bwd<C, T1>(B[1], p, u1);
  cz_bwd<C, T2>(B[2], p, u2);
}

// transposed y: in [QX][QY][NZ] -> out [QX][NY][NZ]; line l = (qx, element, z row)
template <class C, int TM, typename TC>
__device__ __forceinline__ void cbwd_y(const TC* __restrict__ in, TC* __restrict__ out, int l) {
  constexpr int NY = C::ny(TM), R = C::R, Q = C::Q, QX = C::QX;
  constexpr bool N = TM & 2;
  const int qx = l % QX, r2 = l / QX;
  const int e = r2 % C::EY, k = r2 / C::EY;
  const TC* s = in + qx + QX * (Q * e + C::QY * k);
  TC c[Q];
#pragma unroll
  for (int t = 0; t < Q; ++t) c[t] = s[QX * t];
  TC* o = out + qx + QX * (R * e + NY * k);
  if constexpr (N) {
    TC lower = 0;  // the lower element's contribution to the shared position R e
    if (e > 0) {
#pragma unroll
      for (int t = 0; t < Q; ++t) lower += ctab<TC, R, N, true>(t, R) * s[QX * (t - Q)];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < Q; ++t) acc += ctab<TC, R, N, true>(t, i) * c[t];
      o[QX * i] = i == 0 ? lower + acc : acc;
    }
    if (e == C::EY - 1) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < Q; ++t) acc += ctab<TC, R, N, true>(t, R) * c[t];
      o[QX * R] = acc;
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < Q; ++t) acc += ctab<TC, R, N, true>(t, i) * c[t];
      o[QX * i] = acc;
    }
  }
}

// transposed x: in [QX][NY][NZ] -> lattice out [NX][NY][NZ] (= or +=);
// line l = (element, row)
template <class C, int TM, bool ADD, typename TC>
__device__ __forceinline__ void cbwd_x(const TC* __restrict__ in, TC* __restrict__ out, int l) {
  constexpr int NX = C::nx(TM), R = C::R, Q = C::Q;
  constexpr bool N = TM & 1;
  const int e = l % C::EX, rest = l / C::EX;
  const TC* s = in + rest * C::QX + e;
  TC c[Q];
#pragma unroll
  for (int t = 0; t < Q; ++t) c[t] = s[xq<C>(0, t)];
  TC* o = out + rest * NX + R * e;
  auto put = [&](int i, TC v) {
    if constexpr (ADD) o[i] += v;
    else o[i] = v;
  };
  if constexpr (N) {
    TC lower = 0;
    if (e > 0) {
#pragma unroll
      for (int t = 0; t < Q; ++t) lower += ctab<TC, R, N, true>(t, R) * s[xq<C>(0, t) - 1];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < Q; ++t) acc += ctab<TC, R, N, true>(t, i) * c[t];
      put(i, i == 0 ? lower + acc : acc);
    }
    if (e == C::EX - 1) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < Q; ++t) acc += ctab<TC, R, N, true>(t, R) * c[t];
      put(R, acc);
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < Q; ++t) acc += ctab<TC, R, N, true>(t, i) * c[t];
      put(i, acc);
    }
  }
}

// The thread index, passed through an empty asm: the loop predicates of the
// stages (thread index < item count) are then evaluated where the stage runs,
// instead of being hoisted out of the layer loop, where dozens of them would
// stay live as 64-bit lane masks and spill to VGPR lanes.
__device__ __forceinline__ int stage_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// One stage over up to three components: items [0, n0) go to f0, then n1
// items to f1, n2 to f2, spread over the workgroup.
template <int NT, int N0, int N1, int N2, class F0, class F1, class F2>
__device__ __forceinline__ void stage3(F0&& f0, F1&& f1, F2&& f2) {
  for (int idx = stage_tid(); idx < N0 + N1 + N2; idx += NT) {
    if (idx < N0) f0(idx);
    else if (N1 > 0 && idx < N0 + N1) f1(idx - N0);
    else if (N2 > 0) f2(idx - N0 - N1);
  }
}

}  // namespace gym
