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

#include "kernels.hpp"

namespace gym {

constexpr int kNT = 256;  // threads per workgroup

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
static __constant__ TabSet<double> c_tabL_d[4];  // q = r + 2 (load vectors)

// Host: fill the table sets for r = 1..4 (op_common.hip).
void fill_tables(TabSet<double>* hd, TabSet<double>* hl, TabSet<float>* hf);

template <typename T>
__device__ __forceinline__ const TabSet<T>& tabs(int r);
template <>
__device__ __forceinline__ const TabSet<double>& tabs<double>(int r) { return c_tab_d[r - 1]; }
template <>
__device__ __forceinline__ const TabSet<float>& tabs<float>(int r) { return c_tab_f[r - 1]; }

// Compile-time geometry of one layer of a tile.
template <int R_, int BX_, int BY_, int DIM_>
struct Cfg {
  static constexpr int R = R_, Q = R_ + 1, BX = BX_, BY = BY_, DIM = DIM_;
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
  const TabSet<TC>& T = tabs<TC>(C::R);
  for (int idx = threadIdx.x; idx < C::QX * NY * NZ; idx += kNT) {
    int qx = idx % C::QX, rest = idx / C::QX;
    int e = qx / C::Q, t = qx - e * C::Q;
    const TC* s = in + rest * NX + C::R * e;
    TC acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += tab<TC, N, false>(T, t, i) * s[i];
    out[idx] = (e >= er.xlo && e < er.xhi) ? acc : TC(0);
  }
}

// in: [QX][ny][nz] -> out: [QX][QY][nz]
template <class C, int TM, typename TC>
__device__ __forceinline__ void fwd_y(const TC* __restrict__ in, TC* __restrict__ out, const ElemRange& er) {
  constexpr int NY = C::ny(TM), NZ = C::nz(TM);
  constexpr bool N = TM & 2;
  constexpr int n = N ? C::R + 1 : C::R;
  const TabSet<TC>& T = tabs<TC>(C::R);
  for (int idx = threadIdx.x; idx < C::QX * C::QY * NZ; idx += kNT) {
    int qx = idx % C::QX, r2 = idx / C::QX;
    int qy = r2 % C::QY, k = r2 / C::QY;
    int e = qy / C::Q, t = qy - e * C::Q;
    const TC* s = in + qx + C::QX * (C::R * e + NY * k);
    TC acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += tab<TC, N, false>(T, t, i) * s[C::QX * i];
    out[idx] = (e >= er.ylo && e < er.yhi) ? acc : TC(0);
  }
}

// in: [QX][QY][nz] -> out: [QX][QY][QZ] (one element layer in z)
template <class C, int TM, typename TC>
__device__ __forceinline__ void fwd_z(const TC* __restrict__ in, TC* __restrict__ out) {
  constexpr int P = C::QX * C::QY;
  if constexpr (C::DIM == 2) {
    for (int idx = threadIdx.x; idx < P; idx += kNT) out[idx] = in[idx];
  } else {
    constexpr bool N = TM & 4;
    constexpr int n = N ? C::R + 1 : C::R;
    const TabSet<TC>& T = tabs<TC>(C::R);
    for (int idx = threadIdx.x; idx < P * C::Q; idx += kNT) {
      int p = idx % P, t = idx / P;
      TC acc = 0;
#pragma unroll
      for (int i = 0; i < n; ++i) acc += tab<TC, N, false>(T, t, i) * in[p + P * i];
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
    for (int idx = threadIdx.x; idx < P; idx += kNT) out[idx] = in[idx];
  } else {
    constexpr bool N = TM & 4;
    constexpr int NZ = C::nz(TM);
    const TabSet<TC>& T = tabs<TC>(C::R);
    for (int idx = threadIdx.x; idx < P * NZ; idx += kNT) {
      int p = idx % P, k = idx / P;
      TC acc = 0;
#pragma unroll
      for (int t = 0; t < C::Q; ++t) acc += tab<TC, N, true>(T, t, k) * in[p + P * t];
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
  const TabSet<TC>& T = tabs<TC>(C::R);
  for (int idx = threadIdx.x; idx < C::QX * NY * NZ; idx += kNT) {
    int qx = idx % C::QX, r2 = idx / C::QX;
    int j = r2 % NY, k = r2 / NY;
    const TC* base = in + qx + C::QX * C::QY * k;
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
  const TabSet<TC>& T = tabs<TC>(C::R);
  for (int idx = threadIdx.x; idx < NX * NY * NZ; idx += kNT) {
    int j = idx % NX, rest = idx / NX;
    const TC* base = in + C::QX * rest;
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
    for (int idx = threadIdx.x; idx < NX * NY * NZ; idx += kNT) {
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
    for (int idx = threadIdx.x; idx < NX * NY * NZ; idx += kNT) {
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
    for (int idx = threadIdx.x; idx < P * NZ; idx += kNT) {
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
