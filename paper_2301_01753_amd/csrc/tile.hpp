// Device building blocks of the matrix-free operator kernels (gfx950).
//
// Work decomposition ("2.5-D blocking"): a workgroup owns an x-y tile of
// BX x BY elements and marches through a chunk of element layers in z.  For
// each layer it holds, in LDS, every field on the lattice closure of the
// layer's (BX+1) x (BY+1) elements: the extra element column/row on the low
// side is recomputed so that the tile's own low boundary positions receive
// every contribution without atomics.  Positions shared between consecutive
// layers (the top lattice plane of nodal-in-z fields) are carried in LDS to
// the next layer.  Every output position is therefore written exactly once,
// by its owner, with a fixed summation order: results are deterministic.
//
// Mass matrices (paper section 2: (M_p)_ij = int (Lambda_i, Lambda_j)_p dx)
// are applied by sum factorisation: three 1-D contractions from lattice
// coefficients to Gauss points (tables phi / e at q = r + 1 points), the
// pointwise metric, three transposed contractions with weighted tables.
// Incidence (eq. discreteDeRham) is applied on the closure as +-1 sums.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gen/tables_const.hpp"
#include "kernels.hpp"

namespace gym {

// Threads per workgroup of the small-tile (40 KB) tilings; the whole-CU
// tilings choose theirs per problem, degree and form (op_kernel.hpp).
constexpr int kNTSmall = 256;

// 1-D tables for degree r (index r - 1).  Row t = Gauss point.
template <typename T>
struct TabSet {
  T phi[6][5];    // nodal values       (q x (r + 1))
  T edge[6][4];   // edge values        (q x r)
  T phiw[6][5];   // w_t * nodal values
  T edgew[6][4];  // w_t * edge values
  T w[6];
  T gx[6];
  T mn[5][5];     // 1-D element mass of the nodal functions (Gauss, q = r + 1)
  T me[4][4];     // 1-D element mass of the edge functions
};

// Every translation unit that launches kernels holds its own copy of the
// tables (no relocatable device code); see upload_tables_unit().
static __constant__ TabSet<double> c_tab_d[4];   // q = r + 1
static __constant__ TabSet<float> c_tab_f[4];
static __constant__ TabSet<float> c_tab_b[4];    // FP32 values rounded to bf16
static __constant__ TabSet<double> c_tabL_d[4];  // q = r + 2 (load vectors)

// Host: fill the table sets for r = 1..4 (op_common.hip); hb receives the
// FP32 tables rounded to bf16.
void fill_tables(TabSet<double>* hd, TabSet<double>* hl, TabSet<float>* hf, TabSet<float>* hb);

// bf16 rounding (round to nearest, ties to even) of an FP32 value, kept in
// FP32 storage: the BF16 mode rounds every contraction operand this way and
// accumulates in FP32.
__host__ __device__ inline float round_bf16(float x) {
  union {
    float f;
    unsigned u;
  } v;
  v.f = x;
  unsigned lsb = (v.u >> 16) & 1u;
  v.u += 0x7FFFu + lsb;
  v.u &= 0xFFFF0000u;
  return v.f;
}

template <bool BF, typename TC>
__device__ __forceinline__ TC rd(TC x) {
  if constexpr (BF) return round_bf16(x);
  else return x;
}

template <typename T>
__device__ __forceinline__ const TabSet<T>& tabs(int r);
template <>
__device__ __forceinline__ const TabSet<double>& tabs<double>(int r) { return c_tab_d[r - 1]; }
template <>
__device__ __forceinline__ const TabSet<float>& tabs<float>(int r) { return c_tab_f[r - 1]; }

template <bool BF, typename TC>
__device__ __forceinline__ const TabSet<TC>& ktabs(int r) {
  if constexpr (BF) return c_tab_b[r - 1];
  else return tabs<TC>(r);
}

// Compile-time geometry of one layer of a tile.
template <int R_, int BX_, int BY_, int DIM_, int NT_ = kNTSmall>
struct Cfg {
  static constexpr int R = R_, Q = R_ + 1, BX = BX_, BY = BY_, DIM = DIM_, NT = NT_;
  static constexpr int EX = BX + 1, EY = BY + 1;
  static constexpr int QX = Q * EX, QY = Q * EY, QZ = DIM == 3 ? Q : 1;
  static constexpr int nx(int tm) { return (tm & 1) ? R * EX + 1 : R * EX; }
  static constexpr int ny(int tm) { return (tm & 2) ? R * EY + 1 : R * EY; }
  static constexpr int nz(int tm) { return DIM == 2 ? 1 : ((tm & 4) ? R + 1 : R); }
  static constexpr int lat(int tm) { return nx(tm) * ny(tm) * nz(tm); }
  static constexpr int plane(int tm) { return nx(tm) * ny(tm); }
  // temporaries of one scalar sum-factorised mass apply
  static constexpr int tmpA() {
    int a = QX * QY * QZ;
    int b = QX * (R * EY + 1) * (DIM == 3 ? R + 1 : 1);
    return a > b ? a : b;
  }
  static constexpr int tmpB() { return QX * QY * (DIM == 3 ? R + 1 : 1); }
};

// The contraction tables of degree R (q = R + 1) as compile-time constants,
// generated at build time from the same make_tables() as the run-time copies:
// with the loops unrolled every entry is a literal, so no scalar-memory load
// (and no wait on one) sits in a contraction.
template <typename TC, int R, bool NODAL, bool WEIGHTED>
__device__ __forceinline__ constexpr TC ctab(int q, int i) {
  using T = ctabs::Tab<R>;
  if constexpr (NODAL) return static_cast<TC>(WEIGHTED ? T::phiw[q][i] : T::phi[q][i]);
  else return static_cast<TC>(WEIGHTED ? T::edgew[q][i] : T::edge[q][i]);
}

template <typename TC, bool NODAL, bool WEIGHTED>
__device__ __forceinline__ TC tab(const TabSet<TC>& t, int q, int i) {
  if constexpr (NODAL) return WEIGHTED ? t.phiw[q][i] : t.phi[q][i];
  else return WEIGHTED ? t.edgew[q][i] : t.edge[q][i];
}

// ---- forward contractions (coefficients -> Gauss points) ----------------
// in: [nx][ny][nz] lattice (x fastest) -> out: [QX][ny][nz]
// Elements of the closure that lie outside the mesh (the low-side halo of the
// first tile, the ragged end of the last one) see nonzero values on the
// domain's boundary positions; their Gauss-point values are forced to zero
// here so that they contribute nothing.  Valid local elements: [lo, hi).
struct ElemRange {
  int xlo, xhi, ylo, yhi;
};

template <class C, int TM, typename TC>
__device__ __forceinline__ void fwd_x(const TC* __restrict__ in, TC* __restrict__ out, const ElemRange& er) {
  constexpr int NX = C::nx(TM), NY = C::ny(TM), NZ = C::nz(TM);
  constexpr bool N = TM & 1;
  constexpr int n = N ? C::R + 1 : C::R;
  for (int idx = threadIdx.x; idx < C::QX * NY * NZ; idx += C::NT) {
    int qx = idx % C::QX, rest = idx / C::QX;
    int e = qx / C::Q, t = qx - e * C::Q;
    const TC* s = in + rest * NX + C::R * e;
    TC acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += ctab<TC, C::R, N, false>(t, i) * s[i];
    out[idx] = (e >= er.xlo && e < er.xhi) ? acc : TC(0);
  }
}

// in: [QX][ny][nz] -> out: [QX][QY][nz]
template <class C, int TM, typename TC>
__device__ __forceinline__ void fwd_y(const TC* __restrict__ in, TC* __restrict__ out, const ElemRange& er) {
  constexpr int NY = C::ny(TM), NZ = C::nz(TM);
  constexpr bool N = TM & 2;
  constexpr int n = N ? C::R + 1 : C::R;
  for (int idx = threadIdx.x; idx < C::QX * C::QY * NZ; idx += C::NT) {
    int qx = idx % C::QX, r2 = idx / C::QX;
    int qy = r2 % C::QY, k = r2 / C::QY;
    int e = qy / C::Q, t = qy - e * C::Q;
    const TC* s = in + qx + C::QX * (C::R * e + NY * k);
    TC acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += ctab<TC, C::R, N, false>(t, i) * s[C::QX * i];
    out[idx] = (e >= er.ylo && e < er.yhi) ? acc : TC(0);
  }
}

// in: [QX][QY][nz] -> out: [QX][QY][QZ] (one element layer in z)
template <class C, int TM, typename TC>
__device__ __forceinline__ void fwd_z(const TC* __restrict__ in, TC* __restrict__ out) {
  constexpr int P = C::QX * C::QY;
  if constexpr (C::DIM == 2) {
    for (int idx = threadIdx.x; idx < P; idx += C::NT) out[idx] = in[idx];
  } else {
    constexpr bool N = TM & 4;
    constexpr int n = N ? C::R + 1 : C::R;
    for (int idx = threadIdx.x; idx < P * C::Q; idx += C::NT) {
      int p = idx % P, t = idx / P;
      TC acc = 0;
#pragma unroll
      for (int i = 0; i < n; ++i) acc += ctab<TC, C::R, N, false>(t, i) * in[p + P * i];
      out[idx] = acc;
    }
  }
}

// ---- backward (transposed, weighted) contractions -----------------------
// in: [QX][QY][QZ] -> out: [QX][QY][nz]
template <class C, int TM, typename TC>
__device__ __forceinline__ void bwd_z(const TC* __restrict__ in, TC* __restrict__ out) {
  constexpr int P = C::QX * C::QY;
  if constexpr (C::DIM == 2) {
    for (int idx = threadIdx.x; idx < P; idx += C::NT) out[idx] = in[idx];
  } else {
    constexpr bool N = TM & 4;
    constexpr int NZ = C::nz(TM);
    for (int idx = threadIdx.x; idx < P * NZ; idx += C::NT) {
      int p = idx % P, k = idx / P;
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < C::Q; ++t) acc += ctab<TC, C::R, N, true>(t, k) * in[p + P * t];
      out[idx] = acc;
    }
  }
}

// Contributions to lattice position j from the elements of a 1-D run of E
// elements: for nodal types the position j = R*e is shared by elements e-1
// (local index R) and e (local index 0); summed in that order.
template <int R, int E, bool NODAL, class F>
__device__ __forceinline__ auto gather1d(int j, F&& term) {
  int e = j / R, i = j - R * e;
  decltype(term(0, 0)) acc = 0;
  if constexpr (NODAL) {
    if (i == 0 && e > 0) acc += term(e - 1, R);
    if (e < E) acc += term(e, i);
  } else {
    acc += term(e, i);
  }
  return acc;
}

// in: [QX][QY][nz] -> out: [QX][ny][nz]
template <class C, int TM, typename TC>
__device__ __forceinline__ void bwd_y(const TC* __restrict__ in, TC* __restrict__ out) {
  constexpr int NY = C::ny(TM), NZ = C::nz(TM);
  constexpr bool N = TM & 2;
  for (int idx = threadIdx.x; idx < C::QX * NY * NZ; idx += C::NT) {
    int qx = idx % C::QX, r2 = idx / C::QX;
    int j = r2 % NY, k = r2 / NY;
    const TC* base = in + qx + C::QX * C::QY * k;
    // i varies over the lanes: a table lookup, not a literal
    const TabSet<TC>& T = tabs<TC>(C::R);
    out[idx] = gather1d<C::R, C::EY, N>(j, [&](int e, int i) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < C::Q; ++t) acc += tab<TC, N, true>(T, t, i) * base[C::QX * (C::Q * e + t)];
      return acc;
    });
  }
}

// in: [QX][ny][nz] -> lattice out [nx][ny][nz]; out = scale * acc (STORE) or
// out += scale * acc (ADD)
template <class C, int TM, bool ADD, typename TC>
__device__ __forceinline__ void bwd_x(const TC* __restrict__ in, TC* __restrict__ out, TC scale) {
  constexpr int NX = C::nx(TM), NY = C::ny(TM), NZ = C::nz(TM);
  constexpr bool N = TM & 1;
  for (int idx = threadIdx.x; idx < NX * NY * NZ; idx += C::NT) {
    int j = idx % NX, rest = idx / NX;
    const TC* base = in + C::QX * rest;
    const TabSet<TC>& T = tabs<TC>(C::R);  // i varies over the lanes
    TC v = gather1d<C::R, C::EX, N>(j, [&](int e, int i) {
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < C::Q; ++t) acc += tab<TC, N, true>(T, t, i) * base[C::Q * e + t];
      return acc;
    });
    if constexpr (ADD) out[idx] += scale * v;
    else out[idx] = scale * v;
  }
}

// One scalar mass apply on uniform (affine, axis-aligned) cells, where the
// pointwise metric is a constant folded into `scale`:
// out (=|+=) scale * B^T W B in.   A, B: temporaries (Cfg::tmpA/tmpB).
template <class C, int TM, bool ADD, typename TC>
__device__ __forceinline__ void mass_uniform(const TC* in, TC* out, TC scale, TC* A, TC* B,
                                             const ElemRange& er) {
  fwd_x<C, TM>(in, A, er);
  __syncthreads();
  fwd_y<C, TM>(A, B, er);
  __syncthreads();
  fwd_z<C, TM>(B, A);
  __syncthreads();
  bwd_z<C, TM>(A, B);
  __syncthreads();
  bwd_y<C, TM>(B, A);
  __syncthreads();
  bwd_x<C, TM, ADD>(A, out, scale);
  __syncthreads();
}

// Kronecker form of the same mass apply on affine, axis-aligned cells: with a
// constant metric the element matrix factors into 1-D element matrices
// M_a = B_a^T W B_a (evaluated once from the same Gauss rule), so
//   out (=|+=) scale * (M_x (x) M_y (x) M_z) in
// assembled over the tile's valid elements.  Three banded lattice stages
// replace the six Gauss-point stages; the result equals mass_uniform up to
// rounding.  A, B: lattice-sized temporaries.
template <typename TC, bool NODAL>
__device__ __forceinline__ TC kmat(const TabSet<TC>& t, int i, int j) {
  if constexpr (NODAL) return t.mn[i][j];
  else return t.me[i][j];
}

template <class C, int TM, bool ADD, typename TC>
__device__ __forceinline__ void mass_kron(const TC* in, TC* out, TC scale, TC* A, TC* B, const ElemRange& er) {
  constexpr int NX = C::nx(TM), NY = C::ny(TM), NZ = C::nz(TM);
  constexpr int R = C::R;
  const TabSet<TC>& T = tabs<TC>(R);
  {
    constexpr bool N = TM & 1;
    constexpr int n = N ? R + 1 : R;
    for (int idx = threadIdx.x; idx < NX * NY * NZ; idx += C::NT) {
      int j = idx % NX;
      const TC* s = in + (idx - j);
      A[idx] = gather1d<R, C::EX, N>(j, [&](int e, int i) {
        TC acc = 0;
        if (e >= er.xlo && e < er.xhi) {
#pragma unroll
          for (int k = 0; k < n; ++k) acc += kmat<TC, N>(T, i, k) * s[R * e + k];
        }
        return acc;
      });
    }
  }
  __syncthreads();
  {
    constexpr bool N = TM & 2;
    constexpr int n = N ? R + 1 : R;
    for (int idx = threadIdx.x; idx < NX * NY * NZ; idx += C::NT) {
      int x = idx % NX, r2 = idx / NX;
      int j = r2 % NY, k = r2 / NY;
      const TC* s = A + x + NX * NY * k;
      B[idx] = gather1d<R, C::EY, N>(j, [&](int e, int i) {
        TC acc = 0;
        if (e >= er.ylo && e < er.yhi) {
#pragma unroll
          for (int m = 0; m < n; ++m) acc += kmat<TC, N>(T, i, m) * s[NX * (R * e + m)];
        }
        return acc;
      });
    }
  }
  __syncthreads();
  {
    constexpr int P = NX * NY;
    for (int idx = threadIdx.x; idx < P * NZ; idx += C::NT) {
      TC v;
      if constexpr (C::DIM == 2) {
        v = B[idx];
      } else {
        constexpr bool N = TM & 4;
        int p = idx % P, k = idx / P;
        v = 0;
#pragma unroll
        for (int m = 0; m < NZ; ++m) v += kmat<TC, N>(T, k, m) * B[p + P * m];
      }
      if constexpr (ADD) out[idx] += scale * v;
      else out[idx] = scale * v;
    }
  }
  __syncthreads();
}

// Column-register form of the Kronecker mass, for up to three components at
// once (masks T0, T1, T2; NCOMP of them used).  Stage 1: every thread owns
// lattice columns (x, y) of one component and applies M_x along x for all
// z values of the column.  Stage 2: the same columns apply M_y along y and,
// in registers, M_z along the column.  Two barriers per call whatever the
// number of components.  in[c] == out[c] is allowed.
template <class C, int TM, bool BF, typename TC>
__device__ __forceinline__ void kron_x_col(const TC* __restrict__ in, TC* __restrict__ A, int col, const ElemRange& er) {
  constexpr int NX = C::nx(TM), NY = C::ny(TM), NZ = C::nz(TM);
  constexpr int R = C::R;
  constexpr bool N = TM & 1;
  constexpr int n = N ? R + 1 : R;
  const TabSet<TC>& T = ktabs<BF, TC>(R);
  const int j = col % NX, y = col / NX;
  TC acc[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) acc[k] = 0;
  auto term = [&](int e, int i) {
    if (e < er.xlo || e >= er.xhi) return;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      const TC c = kmat<TC, N>(T, i, m);
#pragma unroll
      for (int k = 0; k < NZ; ++k) acc[k] += c * rd<BF>(in[(R * e + m) + NX * (y + NY * k)]);
    }
  };
  {
    int e = j / R, i = j - R * e;
    if constexpr (N) {
      if (i == 0 && e > 0) term(e - 1, R);
      if (e < C::EX) term(e, i);
    } else {
      term(e, i);
    }
  }
#pragma unroll
  for (int k = 0; k < NZ; ++k) A[j + NX * (y + NY * k)] = acc[k];
}

template <class C, int TM, bool ADD, bool BF, typename TC>
__device__ __forceinline__ void kron_yz_col(const TC* __restrict__ A, TC* __restrict__ out, TC scale, int col,
                                            const ElemRange& er) {
  constexpr int NX = C::nx(TM), NY = C::ny(TM), NZ = C::nz(TM);
  constexpr int R = C::R;
  constexpr bool N = TM & 2;
  constexpr int n = N ? R + 1 : R;
  const TabSet<TC>& T = ktabs<BF, TC>(R);
  const int x = col % NX, j = col / NX;
  TC b[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) b[k] = 0;
  auto term = [&](int e, int i) {
    if (e < er.ylo || e >= er.yhi) return;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      const TC c = kmat<TC, N>(T, i, m);
#pragma unroll
      for (int k = 0; k < NZ; ++k) b[k] += c * rd<BF>(A[x + NX * ((R * e + m) + NY * k)]);
    }
  };
  {
    int e = j / R, i = j - R * e;
    if constexpr (N) {
      if (i == 0 && e > 0) term(e - 1, R);
      if (e < C::EY) term(e, i);
    } else {
      term(e, i);
    }
  }
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    TC v;
    if constexpr (C::DIM == 2) {
      v = b[k];
    } else {
      constexpr bool NZB = TM & 4;
      v = 0;
#pragma unroll
      for (int m = 0; m < NZ; ++m) v += kmat<TC, NZB>(T, k, m) * rd<BF>(b[m]);
    }
    TC* o = out + x + NX * (j + NY * k);
    if constexpr (ADD) *o += scale * v;
    else *o = scale * v;
  }
}

template <class C, int NCOMP, int T0, int T1, int T2, bool ADD, bool BF, typename TC>
__device__ __forceinline__ void kron_cols(TC* const in[3], TC* const out[3], const TC sc[3], TC* const A[3],
                                          const ElemRange& er) {
  constexpr int n0 = C::nx(T0) * C::ny(T0);
  constexpr int n1 = NCOMP > 1 ? C::nx(T1) * C::ny(T1) : 0;
  constexpr int n2 = NCOMP > 2 ? C::nx(T2) * C::ny(T2) : 0;
  for (int idx = threadIdx.x; idx < n0 + n1 + n2; idx += C::NT) {
    if (idx < n0) kron_x_col<C, T0, BF>(in[0], A[0], idx, er);
    else if (NCOMP > 1 && idx < n0 + n1) kron_x_col<C, T1, BF>(in[1], A[1], idx - n0, er);
    else if (NCOMP > 2) kron_x_col<C, T2, BF>(in[2], A[2], idx - n0 - n1, er);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n0 + n1 + n2; idx += C::NT) {
    if (idx < n0) kron_yz_col<C, T0, ADD, BF>(A[0], out[0], sc[0], idx, er);
    else if (NCOMP > 1 && idx < n0 + n1) kron_yz_col<C, T1, ADD, BF>(A[1], out[1], sc[1], idx - n0, er);
    else if (NCOMP > 2) kron_yz_col<C, T2, ADD, BF>(A[2], out[2], sc[2], idx - n0 - n1, er);
  }
  __syncthreads();
}

template <class C, int TM, bool ADD, bool KRON, typename TC>
__device__ __forceinline__ void mass(const TC* in, TC* out, TC scale, TC* A, TC* B, const ElemRange& er) {
  if constexpr (KRON) mass_kron<C, TM, ADD>(in, out, scale, A, B, er);
  else mass_uniform<C, TM, ADD>(in, out, scale, A, B, er);
}

// Lattice index inside the layer closure.
template <class C, int TM>
__device__ __forceinline__ int lidx(int x, int y, int z) {
  return x + C::nx(TM) * (y + C::ny(TM) * z);
}

template <class C, int TM>
__device__ __forceinline__ void lpos(int idx, int& x, int& y, int& z) {
  x = idx % C::nx(TM);
  int r = idx / C::nx(TM);
  y = r % C::ny(TM);
  z = r / C::ny(TM);
}

}  // namespace gym
