// Hodge-Laplacian (1-forms) on curved cells, degree 3, FP64: the element
// contractions on the matrix cores.
//
// Operator (masses M_p of paper section 2, incidence of eq. discreteDeRham):
//   y_sigma = -M0 sigma + G^T M1 u,   y_u = M1 G sigma + C^T M2 C u.
// On one cell, with N and E the nodal and edge functions at the q = 4 Gauss
// points of an axis and D the derivatives of the nodal functions written in
// the edge basis (D(t, i) = E(t, i - 1) - E(t, i), which is how G and C act
// on the coefficients), every term is a product of three 1-D tables (x, y,
// z), the pointwise metric (det J and the HCURL and HDIV Piola metrics of the
// cell map, geom.hip), and the transposed tables weighted by the Gauss
// weights:
//   Gauss values   s = NNN sigma, grad sigma = (DNN, NDN, NND) sigma,
//                  u = (ENN u_x, NEN u_y, NNE u_z),
//                  curl u = (NDE u_z - NED u_y, END u_x - DNE u_z, DEN u_y - EDN u_x)
//   metric         p = -det s, h = G1 u, g = G1 grad sigma, v = G2 curl u
//   outputs        y_sigma = NNN' p + DNN' h_x + NDN' h_y + NND' h_z
//                  y_ux = ENN' g_x + END' v_y - EDN' v_z   (and cyclically)
//
// Work mapping: a wavefront computes four cells, one per block of
// v_mfma_f64_4x4x4_4b (16 lanes each).  Lane 16 r + 4 blk + c of block blk
// holds entry (r, c) of a 4 x 4 plane of its cell: the x-y coefficients
// (a, b) = (r, c) of one z level, or the Gauss point (i, j) = (c, r).  The z
// direction lives in registers.  The instruction D = A B + C reads a lane's
// value X as A = X^T or as B = X and returns D in the same placement, so the
// four 1-D stages chain without moving data between lanes:
//   x forward   D[b][i] = sum_a X[a][b] T(i, a)          A = X,   B = F_T
//   y forward   D[j][i] = sum_b T(j, b) X[b][i]          A = F_T, B = X
//   y backward  D[i][b] = sum_j X[j][i] w_j T(j, b)      A = X,   B = W_T
//   x backward  D[a][b] = sum_i w_i T(i, a) X[i][b]      A = W_T, B = X
// with the per-lane table operands F_T(r, c) = T(c, r) and W_T(r, c) =
// w_r T(r, c).  The z contractions and the metric are FMAs in registers with
// the table entries as compile-time constants.
//
// Metric: computed in registers from the cell's 8 vertices (J, adj J, det J,
// G1, G2 at each Gauss point); a wavefront loads its cells' vertex rows for
// the next layer straight into its own LDS rows (global-to-LDS loads, no
// registers, no barrier).  No per-Gauss-point metric is read from memory:
// read per right-hand side, it cost more than the rest of the kernel.
//
// Sums over cells: a workgroup owns a TX x TY tile of cells and marches
// through a chunk of layers in z.  The top z plane of a cell is carried in
// registers into the cell above (the layer below a chunk is recomputed to
// start the carry).  A position shared in x or y by cells of the tile is
// collected in LDS by one lane (the cell that has it at its low side, or the
// last cell of the tile) in a fixed order.  Positions on a tile's high x or y
// face belong to the next tile: the collected sum goes to a halo slot (one
// per position and neighbour direction), and a second kernel adds the at
// most three halo values to the owner's sum in a fixed order, so results are
// deterministic and no cell is computed twice.
#include "hodge_mfma.hpp"

#include <algorithm>
#include <utility>

#include "gen/tables_const.hpp"
#include "geom.hpp"

namespace gym {
namespace {

constexpr int R = kHcDegree, Q = R + 1;
static_assert(Q == 4, "one 4 x 4 matrix-core block per cell plane");
using Tab = ctabs::Tab<R>;

// 1-D tables: Gauss point t, function i; W: times the Gauss weight of t.
// E is padded with a zero column (i = R), D is the nodal derivative.
template <bool W>
__host__ __device__ constexpr double tN(int t, int i) {
  return W ? Tab::phiw[t][i] : Tab::phi[t][i];
}
template <bool W>
__host__ __device__ constexpr double tE(int t, int i) {
  return i < R ? (W ? Tab::edgew[t][i] : Tab::edge[t][i]) : 0.0;
}
template <bool W>
__host__ __device__ constexpr double tD(int t, int i) {
  return (i > 0 ? tE<W>(t, i - 1) : 0.0) - tE<W>(t, i);
}
enum { TN = 0, TD = 1, TE = 2 };
template <int T, bool W>
__host__ __device__ constexpr double tab(int t, int i) {
  return T == TN ? tN<W>(t, i) : T == TD ? tD<W>(t, i) : tE<W>(t, i);
}

// entry (t, i) of a table for a lane-dependent (t, i)
template <int T, bool W>
__device__ double lane_tab(int t, int i) {
  double v = 0;
#pragma unroll
  for (int tt = 0; tt < 4; ++tt)
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
      if (tt == t && ii == i) v = tab<T, W>(tt, ii);
  return v;
}

__device__ __forceinline__ double mma(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

enum { SET = 0, ADD = 1, SUB = 2, NSET = 3 };

// A table as 16 scalar-register constants, materialised where it is used.
// Each entry is written by two s_mov_b32 of its bit pattern inside volatile
// asm: the compiler can then neither hoist the entries out of the layer loop
// (all tables together do not fit the scalar registers and would be spilled
// and reloaded lane by lane) nor keep them across the loop.
template <int T, bool W, int t, int i>
__device__ __forceinline__ double kconst() {
  constexpr unsigned long long b = __builtin_bit_cast(unsigned long long, tab<T, W>(t, i));
  unsigned lo, hi;
  asm volatile("s_mov_b32 %0, %1" : "=s"(lo) : "i"((unsigned)(b & 0xffffffffu)));
  asm volatile("s_mov_b32 %0, %1" : "=s"(hi) : "i"((unsigned)(b >> 32)));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int T, bool W>
struct KTab {
  double k[4][4];
  __device__ __forceinline__ KTab() { fill(std::make_integer_sequence<int, 16>{}); }
  template <int... I>
  __device__ __forceinline__ void fill(std::integer_sequence<int, I...>) {
    ((k[I / 4][I % 4] = (T == TE && I % 4 == R) ? 0.0 : kconst<T, W, I / 4, I % 4>()), ...);
  }
};
// z forward: g[k] (=, +=, -=, = -) sum_{c < NC} T(k, c) y[c]
template <int NC, int MODE, class K>
__device__ __forceinline__ void zf(const K& K_, const double (&y)[4], double (&g)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double acc = (MODE == ADD || MODE == SUB) ? g[k] : 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      constexpr bool neg = MODE == SUB || MODE == NSET;
      acc = __builtin_fma(neg ? -K_.k[k][c] : K_.k[k][c], y[c], acc);
    }
    g[k] = acc;
  }
}
// z backward: w[c] (=, +=, -=, = -) sum_k w_k T(k, c) v[k], c < NC (K weighted)
template <int NC, int MODE, class K>
__device__ __forceinline__ void zb(const K& K_, const double (&v)[4], double (&w)[4]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double acc = (MODE == ADD || MODE == SUB) ? w[c] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      constexpr bool neg = MODE == SUB || MODE == NSET;
      acc = __builtin_fma(neg ? -K_.k[k][c] : K_.k[k][c], v[k], acc);
    }
    w[c] = acc;
  }
}

// Fields: 0 sigma (nodal x y z), 1 u_x (edge x), 2 u_y (edge y), 3 u_z (edge z).
constexpr bool kNX[4] = {true, false, true, true};
constexpr bool kNY[4] = {true, true, false, true};
constexpr bool kNZ[4] = {true, true, true, false};
// slot numbers of the fields shared along x, along y, and along both
constexpr int kSX[4] = {0, -1, 1, 2};
constexpr int kSY[4] = {0, 1, -1, 2};
constexpr int kSXY[4] = {0, -1, -1, 1};

__device__ __forceinline__ long long kept_index(const DevComp& d, int g0, int g1, int g2) {
  const int l0 = g0 - d.start[0], l1 = g1 - d.start[1], l2 = g2 - d.start[2];
  if (l0 < 0 || l0 >= d.count[0] || l1 < 0 || l1 >= d.count[1] || l2 < 0 || l2 >= d.count[2]) return -1;
  return d.offset + l0 + (long long)d.count[0] * (l1 + (long long)d.count[1] * l2);
}

// Gauss points on [0, 1] of the rule the tables use
__host__ __device__ constexpr double gpt(int t) { return Tab::gx[t]; }

// Workgroup tile of cells: TX x TY, four cells (a row of four along x) per
// wavefront.
// Workgroup tile: 16 x 2 cells, 8 wavefronts.  Tile boundaries across x cost
// the second kernel a read-modify-write of y one row apart per position; across
// y they are contiguous rows: 16 x 2 took 13.8 ms on the 96^3 workload (second
// kernel 1.4 ms) against 14.5 ms (1.7 ms) for 8 x 4.
constexpr int kTX = 16, kTY = 2;

// LDS slots of the values a cell hands to a neighbour in its layer, per
// cell (cell-major, 87 doubles): x senders (sigma b 0-3, u_y b 0-2, u_z b 0-3),
// y senders (sigma a 0-3, u_x a 0-2, u_z a 0-3), xy senders (sigma, u_z),
// each by z plane (4 planes, 3 for u_z).  Two copies, used by alternate
// layers, so one barrier per layer separates the senders from the collectors.
template <int TX, int TY>
struct Slots {
  static constexpr int kCell = 87, kN = kCell * TX * TY;
  static constexpr int kBX[4] = {0, -1, 16, 28}, kBY[4] = {40, 56, -1, 68};
  static constexpr int kBXY[4] = {80, -1, -1, 84};
  static constexpr int kNZP[4] = {4, 4, 4, 3};
  static __device__ __forceinline__ int cell(int ly, int lx) { return (ly * TX + lx) * kCell; }
  template <int F>
  static __device__ __forceinline__ int sx(int ly, int lx, int b) { return cell(ly, lx) + kBX[F] + b * kNZP[F]; }
  template <int F>
  static __device__ __forceinline__ int sy(int ly, int lx, int a) { return cell(ly, lx) + kBY[F] + a * kNZP[F]; }
  template <int F>
  static __device__ __forceinline__ int sxy(int ly, int lx) { return cell(ly, lx) + kBXY[F]; }
};

// Roles of a lane for one field in the x-y sums (3 bits), and the
// neighbours it receives from (3 bits: x, y, xy).
enum { ROLE_NONE = 0, ROLE_SX = 1, ROLE_SY = 2, ROLE_SXY = 3, ROLE_Y = 4, ROLE_HX = 5, ROLE_HY = 6, ROLE_HXY = 7 };
constexpr int kCodeBits = 6;  // per field: role (3 bits), then the neighbours received from (3 bits)

// WPE: wavefronts per SIMD the registers are budgeted for (2: about 250
// VGPRs; 3 and 4 spill and measured slower).
// TV: the vectors' type (the arithmetic is FP64 either way).
template <int TX, int TY, int WPE, typename TV>
__global__ void __launch_bounds__(TX * TY * 16, WPE) hodge_mfma_kernel(HcParams p) {
  static_assert(TX % 4 == 0, "four cells per wavefront along x");
  constexpr int WX = TX / 4;
  using SL = Slots<TX, TY>;
  constexpr int NW = TX * TY / 4;
  __shared__ double slots[2][SL::kN];
  // per wavefront, two layers: the vertices of its four cells, rows (z, y) of
  // 16 doubles from the first cell's low x vertex (5 vertices, 3
  // coordinates each), filled by direct global-to-LDS loads a layer ahead
  __shared__ double vrow[NW][2][64];

  // blocks b, b + 8, ... run on one XCD: the right-hand sides of an item
  // are consecutive there
  const int blk_id = blockIdx.x;
  const int rhs = (blk_id >> 3) % p.nrhs;
  const int item = (blk_id & 7) + 8 * (blk_id / (8 * p.nrhs));
  if (item >= p.nitems) return;
  const int ntiles = p.tiles_x * p.tiles_y;
  const int tile = item % ntiles, chunk = item / ntiles;
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int blk = (lane >> 2) & 3, r = lane >> 4, c = lane & 3;
  const int lx = 4 * (wv % WX) + blk, ly = wv / WX;
  const int Nx = p.nel[0], Ny = p.nel[1], Nz = p.nel[2];
  const int ex = tx * TX + lx, ey = ty * TY + ly;
  const bool ev = ex < Nx && ey < Ny;

  const double fN = lane_tab<TN, false>(c, r), fD = lane_tab<TD, false>(c, r), fE = lane_tab<TE, false>(c, r);
  const double bN = lane_tab<TN, true>(r, c), bD = lane_tab<TD, true>(r, c), bE = lane_tab<TE, true>(r, c);

  const TV* __restrict__ x = static_cast<const TV*>(p.x) + (long long)rhs * p.ndofs;
  TV* __restrict__ y = static_cast<TV*>(p.y) + (long long)rhs * p.ndofs;
  double* __restrict__ hx = p.halo + (long long)rhs * (p.hx_n + p.hy_n + p.hxy_n);
  double* __restrict__ hy = hx + p.hx_n;
  double* __restrict__ hxy = hy + p.hy_n;
  const int LX = R * Nx + 1, LY = R * Ny + 1, LZ = R * Nz + 1;

  // vertex rows of the wavefront's cells: x from vertex xs (a cell beyond
  // the mesh uses the last cell's vertices: its inputs are zero), y from ey'
  const int x0w = tx * TX + 4 * (wv % WX);
  const int xs = min(x0w, Nx - 1), eyv = min(ey, Ny - 1);
  const int vx = min(ex, Nx - 1) - xs;  // the lane's cell, 0..3, within the rows
  auto prefetch_verts = [&](int ezq) {
    // lanes 0-31: row L / 8 = (z, y) bits, doubles 2 (L % 8), + 1
    if (lane < 32) {
      const int row = lane >> 3, b2 = row >> 1, b1 = row & 1;
      const double* src =
          p.verts + (((long long)(ezq + b2) * (Ny + 1) + (eyv + b1)) * (Nx + 1) + xs) * 3 + 2 * (lane & 7);
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)&vrow[wv][ezq & 1][0], 16, 0, 0);
    }
  };
  // Gauss points of the lane's (i, j) = (c, r)
  double xi1 = 0, xi2 = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (c == t) xi1 = gpt(t);
    if (r == t) xi2 = gpt(t);
  }

  const int zfirst = chunk * p.chunk;
  const int zend = min(zfirst + p.chunk, Nz);
  const int zbeg = zfirst > 0 ? zfirst - 1 : 0;

  // lane's coefficient position (a, b) = (r, c) in the cell
  const int a = r, bb = c;
  const int ga = R * ex + a, gb = R * ey + bb;

  // the lane's coefficient column of each field: kept in x and y, index of
  // its z = 0 position, positions per z step
  long long fbase[4];
  bool fok[4];
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    const DevComp& d = p.f[F];
    const int na = kNX[F] ? R + 1 : R, nb = kNY[F] ? R + 1 : R;
    const int l0 = ga - d.start[0], l1 = gb - d.start[1];
    fok[F] = ev && a < na && bb < nb && l0 >= 0 && l0 < d.count[0] && l1 >= 0 && l1 < d.count[1];
    fbase[F] = d.offset + l0 + (long long)d.count[0] * (l1 - (long long)d.count[1] * d.start[2]);
  }
  // the lane's input column: position gz at xcol[F][zsl[F] gz]; a lane
  // outside the kept set reads the zero (stride 0)
  const TV* xcol[4];
  int zsl[4];
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    xcol[F] = fok[F] ? x + fbase[F] : static_cast<const TV*>(p.zero);
    zsl[F] = fok[F] ? p.f[F].count[0] * p.f[F].count[1] : 0;
  }
  // is lattice plane gz of field F kept (uniform)
  auto zkept = [&](int F, int gz) { return gz >= p.f[F].start[2] && gz < p.f[F].start[2] + p.f[F].count[2]; };

  // roles in the x-y sums, 6 bits per field
  int code0 = 0;
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    const int na = kNX[F] ? R + 1 : R, nb = kNY[F] ? R + 1 : R;
    const bool valid = ev && a < na && bb < nb;
    const bool xs = kNX[F] && a == R && lx + 1 < TX && ex + 1 < Nx;
    const bool ys = kNY[F] && bb == R && ly + 1 < TY && ey + 1 < Ny;
    const bool hxf = kNX[F] && a == R && ex + 1 < Nx;  // on the next tile in x
    const bool hyf = kNY[F] && bb == R && ey + 1 < Ny;
    int role = ROLE_NONE, rm = 0;
    if (valid) {
      if (xs || ys) {
        role = xs && ys ? ROLE_SXY : xs ? ROLE_SX : ROLE_SY;
      } else {
        role = hxf && hyf ? ROLE_HXY : hxf ? ROLE_HX : hyf ? ROLE_HY : (fok[F] ? ROLE_Y : ROLE_NONE);
        if (kNX[F] && a == 0 && lx > 0) rm |= 1;
        if (kNY[F] && bb == 0 && ly > 0) rm |= 2;
        if (kNX[F] && kNY[F] && a == 0 && bb == 0 && lx > 0 && ly > 0) rm |= 4;
      }
    }
    code0 |= (role | rm << 3) << (kCodeBits * F);
  }

  double cS = 0, cX = 0, cY = 0;  // top planes carried into the cell above

  prefetch_verts(zbeg);
  for (int ez = zbeg; ez < zend; ++ez) {
    // the next layer's vertices, issued before this layer's inputs (whose
    // wait then covers them)
    if (ez + 1 < zend) prefetch_verts(ez + 1);
    // ---- inputs: the cell's coefficients, planes along z
    double iS[4], iX[4], iY[4], iZ[4];
    {
      // unconditional loads (a plane outside the kept set reads the zero
      // slot), all issued before the first conversion (the scheduling
      // barrier keeps them from being interleaved with their conversions
      // field by field, each group waited for in turn); z offsets in 32 bits
      // (operators of fewer than 2^31 unknowns), advanced by additions
      const TV* zero = static_cast<const TV*>(p.zero);
      TV raw[4][4];
#pragma unroll
      for (int F = 0; F < 4; ++F) {
        const int nz = F == 3 ? 3 : 4;
        unsigned o = (unsigned)zsl[F] * (unsigned)(R * ez);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int gz = R * ez + k;
          raw[F][k] = *((k < nz && zkept(F, gz)) ? xcol[F] + o : zero);
          o += (unsigned)zsl[F];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        iS[k] = static_cast<double>(raw[0][k]);
        iX[k] = static_cast<double>(raw[1][k]);
        iY[k] = static_cast<double>(raw[2][k]);
        iZ[k] = static_cast<double>(raw[3][k]);
      }
    }

    // ---- forward: x and y contractions on the matrix cores, all fields
    double YNN[4], YND[4], YDN[4];  // sigma: (x table, y table) per z plane
    double YEN[4], YED[4];          // u_x
    double YNE[4], YDE[4];          // u_y
    double ZNN[4], ZND[4], ZDN[4];  // u_z (three planes)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double xn = mma(iS[k], fN, 0.0), xd = mma(iS[k], fD, 0.0);
      YNN[k] = mma(fN, xn, 0.0);
      YND[k] = mma(fD, xn, 0.0);
      YDN[k] = mma(fN, xd, 0.0);
      const double xe = mma(iX[k], fE, 0.0);
      YEN[k] = mma(fN, xe, 0.0);
      YED[k] = mma(fD, xe, 0.0);
      const double yn = mma(iY[k], fN, 0.0), yd = mma(iY[k], fD, 0.0);
      YNE[k] = mma(fE, yn, 0.0);
      YDE[k] = mma(fE, yd, 0.0);
      if (k < 3) {
        const double zn = mma(iZ[k], fN, 0.0), zd = mma(iZ[k], fD, 0.0);
        ZNN[k] = mma(fN, zn, 0.0);
        ZND[k] = mma(fD, zn, 0.0);
        ZDN[k] = mma(fN, zd, 0.0);
      }
    }
    ZNN[3] = ZND[3] = ZDN[3] = 0;
    // z contractions, one table at a time: Gauss-point values of sigma (sg),
    // its gradient, u and curl u
    double sg[4], gx[4], gy[4], gz[4];
    double ux[4], uy[4], uz[4], cx[4], cy[4], cz[4];
    {
      const KTab<TN, false> K;
      zf<4, SET>(K, YNN, sg);
      zf<4, SET>(K, YDN, gx);
      zf<4, SET>(K, YND, gy);
      zf<4, SET>(K, YEN, ux);
      zf<4, NSET>(K, YED, cz);  // -d/dy u_x
      zf<4, SET>(K, YNE, uy);
      zf<4, ADD>(K, YDE, cz);   // +d/dx u_y
    }
    {
      const KTab<TD, false> K;
      zf<4, SET>(K, YNN, gz);
      zf<4, SET>(K, YEN, cy);   // +d/dz u_x
      zf<4, NSET>(K, YNE, cx);  // -d/dz u_y
    }
    {
      const KTab<TE, false> K;
      zf<3, SET>(K, ZNN, uz);
      zf<3, ADD>(K, ZND, cx);   // +d/dy u_z
      zf<3, SUB>(K, ZDN, cy);   // -d/dx u_z
    }

    // ---- pointwise metric, from the cell's vertices (paper section 2: the
    // masses pulled back through the multilinear cell map with Jacobian J):
    // det J, G1 = adj(J) adj(J)^T / det J (HCURL), G2 = J^T J / det J (HDIV,
    // applied as J^T (J v) / det J).
    // Column d of J is the derivative along reference axis d, a bilinear
    // interpolation of the cell's edge vectors along d in the other two
    // coordinates; with (xi1, xi2) fixed per lane, columns 0 and 1 are linear
    // in xi3 and column 2 is constant over the lane's z column.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the vertex rows have landed
    asm volatile("" ::: "memory");
    {
      const double* V = &vrow[wv][ez & 1][0];
      auto vtx = [&](int b0, int b1, int b2, int comp) { return V[(b2 * 2 + b1) * 16 + (vx + b0) * 3 + comp]; };
      double A0[3], dA[3], B0[3], dB[3], Cc[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        // d/dxi1: edges along x at (y, z) corners, interpolated in xi2, then xi3
        const double e00 = vtx(1, 0, 0, i) - vtx(0, 0, 0, i), e10 = vtx(1, 1, 0, i) - vtx(0, 1, 0, i);
        const double e01 = vtx(1, 0, 1, i) - vtx(0, 0, 1, i), e11 = vtx(1, 1, 1, i) - vtx(0, 1, 1, i);
        const double a0 = e00 + xi2 * (e10 - e00), a1 = e01 + xi2 * (e11 - e01);
        A0[i] = a0;
        dA[i] = a1 - a0;
        // d/dxi2: edges along y at (x, z) corners, interpolated in xi1, then xi3
        const double f00 = vtx(0, 1, 0, i) - vtx(0, 0, 0, i), f10 = vtx(1, 1, 0, i) - vtx(1, 0, 0, i);
        const double f01 = vtx(0, 1, 1, i) - vtx(0, 0, 1, i), f11 = vtx(1, 1, 1, i) - vtx(1, 0, 1, i);
        const double b0 = f00 + xi1 * (f10 - f00), b1 = f01 + xi1 * (f11 - f01);
        B0[i] = b0;
        dB[i] = b1 - b0;
        // d/dxi3: edges along z at (x, y) corners, interpolated in xi1, xi2
        const double g00 = vtx(0, 0, 1, i) - vtx(0, 0, 0, i), g10 = vtx(1, 0, 1, i) - vtx(1, 0, 0, i);
        const double g01 = vtx(0, 1, 1, i) - vtx(0, 1, 0, i), g11 = vtx(1, 1, 1, i) - vtx(1, 1, 0, i);
        const double c0 = g00 + xi1 * (g10 - g00), c1 = g01 + xi1 * (g11 - g01);
        Cc[i] = c0 + xi2 * (c1 - c0);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double xi3 = gpt(k);
        double J[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          J[i][0] = A0[i] + xi3 * dA[i];
          J[i][1] = B0[i] + xi3 * dB[i];
          J[i][2] = Cc[i];
        }
        // adj[a][i] = cofactor of J[i][a]
        const double a00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], a01 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
                     a02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        const double a10 = J[1][2] * J[2][0] - J[1][0] * J[2][2], a11 = J[0][0] * J[2][2] - J[0][2] * J[2][0],
                     a12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        const double a20 = J[1][0] * J[2][1] - J[1][1] * J[2][0], a21 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
                     a22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * a00 + J[0][1] * a10 + J[0][2] * a20;
        // 1 / det J: hardware reciprocal and two Newton steps (error about
        // one ulp; the division sequence cost three times the instructions)
        double inv = __builtin_amdgcn_rcp(det);
        inv = __builtin_fma(inv, __builtin_fma(-det, inv, 1.0), inv);
        inv = __builtin_fma(inv, __builtin_fma(-det, inv, 1.0), inv);
        const double m00 = (a00 * a00 + a01 * a01 + a02 * a02) * inv, m01 = (a00 * a10 + a01 * a11 + a02 * a12) * inv,
                     m02 = (a00 * a20 + a01 * a21 + a02 * a22) * inv, m11 = (a10 * a10 + a11 * a11 + a12 * a12) * inv,
                     m12 = (a10 * a20 + a11 * a21 + a12 * a22) * inv, m22 = (a20 * a20 + a21 * a21 + a22 * a22) * inv;
        sg[k] = -det * sg[k];
        double t0 = ux[k], t1 = uy[k], t2 = uz[k];
        ux[k] = m00 * t0 + m01 * t1 + m02 * t2;
        uy[k] = m01 * t0 + m11 * t1 + m12 * t2;
        uz[k] = m02 * t0 + m12 * t1 + m22 * t2;
        t0 = gx[k], t1 = gy[k], t2 = gz[k];
        gx[k] = m00 * t0 + m01 * t1 + m02 * t2;
        gy[k] = m01 * t0 + m11 * t1 + m12 * t2;
        gz[k] = m02 * t0 + m12 * t1 + m22 * t2;
        // G2 v = J^T (J v) / det J: two matrix-vector products
        t0 = cx[k], t1 = cy[k], t2 = cz[k];
        const double w0 = (J[0][0] * t0 + J[0][1] * t1 + J[0][2] * t2) * inv,
                     w1 = (J[1][0] * t0 + J[1][1] * t1 + J[1][2] * t2) * inv,
                     w2 = (J[2][0] * t0 + J[2][1] * t1 + J[2][2] * t2) * inv;
        cx[k] = J[0][0] * w0 + J[1][0] * w1 + J[2][0] * w2;
        cy[k] = J[0][1] * w0 + J[1][1] * w1 + J[2][1] * w2;
        cz[k] = J[0][2] * w0 + J[1][2] * w1 + J[2][2] * w2;
      }
    }

    // ---- backward: p = sg, h = u, g = grad, v = curl (metric applied).
    // z contractions (weighted tables) grouped by the (x, y) tables of a term:
    //   y_sigma = NNN' p + DNN' h_x + NDN' h_y + NND' h_z
    //   y_ux    = ENN' g_x + END' v_y - EDN' v_z
    //   y_uy    = NEN' g_y + DEN' v_z - NED' v_x
    //   y_uz    = NNE' g_z + NDE' v_x - DNE' v_y
    double wNN[4], wDN[4], wND[4], wEN[4], wED[4], wNE[4], wDE[4], vNN[4], vND[4], vDN[4];
    {
      const KTab<TN, true> K;
      zb<4, SET>(K, sg, wNN);
      zb<4, SET>(K, ux, wDN);
      zb<4, SET>(K, uy, wND);
      zb<4, SET>(K, gx, wEN);
      zb<4, NSET>(K, cz, wED);
      zb<4, SET>(K, gy, wNE);
      zb<4, SET>(K, cz, wDE);
    }
    {
      const KTab<TD, true> K;
      zb<4, ADD>(K, uz, wNN);
      zb<4, ADD>(K, cy, wEN);
      zb<4, SUB>(K, cx, wNE);
    }
    {
      const KTab<TE, true> K;
      zb<3, SET>(K, gz, vNN);
      zb<3, SET>(K, cx, vND);
      zb<3, NSET>(K, cy, vDN);
    }
    // y and x contractions on the matrix cores
    double oS[4], oX[4], oY[4], oZ[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double sN = mma(wND[k], bD, mma(wNN[k], bN, 0.0)), sD = mma(wDN[k], bN, 0.0);
      oS[k] = mma(bD, sD, mma(bN, sN, 0.0));
      const double xE = mma(wED[k], bD, mma(wEN[k], bN, 0.0));
      oX[k] = mma(bE, xE, 0.0);
      const double yN = mma(wNE[k], bE, 0.0), yD = mma(wDE[k], bE, 0.0);
      oY[k] = mma(bD, yD, mma(bN, yN, 0.0));
      if (k < 3) {
        const double zN = mma(vND[k], bD, mma(vNN[k], bN, 0.0)), zD = mma(vDN[k], bN, 0.0);
        oZ[k] = mma(bD, zD, mma(bN, zN, 0.0));
      }
    }
    oZ[3] = 0;

    // ---- z: add the plane carried from the cell below, carry the top one
    oS[0] += cS;
    oX[0] += cX;
    oY[0] += cY;
    cS = oS[R];
    cX = oX[R];
    cY = oY[R];
    if (ez < zfirst) continue;  // the recomputed layer below the chunk only starts the carry
    const bool top = ez == Nz - 1;

    // ---- x-y sums: senders to LDS, then collectors (planes of this layer:
    // 0 .. R - 1, and R for nodal-z fields at the top of the mesh)
    const int nout4 = top ? R + 1 : R;
    double* lds = slots[ez & 1];
    // the roles, re-read each layer: their lane masks would otherwise be
    // hoisted out of the loop and spilled
    int code = code0;
    asm volatile("" : "+v"(code));
    auto send = [&](auto fc, const double(&o)[4]) {
      constexpr int F = decltype(fc)::value;
      const int role = (code >> (kCodeBits * F)) & 7;
      if (role < ROLE_SX || role > ROLE_SXY) return;
      int off = 0;
      if constexpr (kSX[F] >= 0) {
        if (role == ROLE_SX) off = SL::template sx<F>(ly, lx, bb);
      }
      if constexpr (kSY[F] >= 0) {
        if (role == ROLE_SY) off = SL::template sy<F>(ly, lx, a);
      }
      if constexpr (kSXY[F] >= 0) {
        if (role == ROLE_SXY) off = SL::template sxy<F>(ly, lx);
      }
      const int nout = kNZ[F] ? nout4 : R;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < nout) lds[off + k] = o[k];
    };
    auto collect = [&](auto fc, const double(&o)[4]) {
      constexpr int F = decltype(fc)::value;
      const int role = (code >> (kCodeBits * F)) & 7, rm = (code >> (kCodeBits * F + 3)) & 7;
      if (role < ROLE_Y) return;
      const int nout = kNZ[F] ? nout4 : R;
      double v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = o[k];
      if constexpr (kSX[F] >= 0) {
        if (rm & 1) {
          const int off = SL::template sx<F>(ly, lx - 1, bb);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < nout) v[k] += lds[off + k];
        }
      }
      if constexpr (kSY[F] >= 0) {
        if (rm & 2) {
          const int off = SL::template sy<F>(ly - 1, lx, a);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < nout) v[k] += lds[off + k];
        }
      }
      if constexpr (kSXY[F] >= 0) {
        if (rm & 4) {
          const int off = SL::template sxy<F>(ly - 1, lx - 1);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < nout) v[k] += lds[off + k];
        }
      }
      // destination column: the vector, or a halo slot of the next tile (FP64)
      if (role == ROLE_Y) {  // a kept column: the input's, in y
        const DevComp& d = p.f[F];
        TV* dst = y + (xcol[F] - x);
        const int zs = d.count[0] * d.count[1];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int gz = R * ez + k;
          if (k < nout && gz >= d.start[2] && gz < d.start[2] + d.count[2]) dst[(long long)zs * gz] = static_cast<TV>(v[k]);
        }
        return;
      }
      double* dst;
      int zs;
      if (role == ROLE_HX) {
        dst = hx + ((kSX[F] * (p.tiles_x - 1) + tx) * LZ) * LY + gb;
        zs = LY;
      } else if (role == ROLE_HY) {
        dst = hy + ((kSY[F] * (p.tiles_y - 1) + ty) * LZ) * LX + ga;
        zs = LX;
      } else {
        dst = hxy + ((kSXY[F] * (p.tiles_x - 1) + tx) * (p.tiles_y - 1) + ty) * LZ;
        zs = 1;
      }
      unsigned zo = (unsigned)zs * (unsigned)(R * ez);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < nout) dst[zo] = v[k];
        zo += (unsigned)zs;
      }
    };
    send(std::integral_constant<int, 0>{}, oS);
    send(std::integral_constant<int, 1>{}, oX);
    send(std::integral_constant<int, 2>{}, oY);
    send(std::integral_constant<int, 3>{}, oZ);
    __syncthreads();
    collect(std::integral_constant<int, 0>{}, oS);
    collect(std::integral_constant<int, 1>{}, oX);
    collect(std::integral_constant<int, 2>{}, oY);
    collect(std::integral_constant<int, 3>{}, oZ);
  }
}

// kept_index of field f (runtime f): each case reads its own kernel-argument
// fields, so the argument block is not copied to per-thread memory for a
// dynamically indexed reference
__device__ __forceinline__ long long field_index(const HcParams& p, int f, int g0, int g1, int g2) {
  switch (f) {
    case 0: return kept_index(p.f[0], g0, g1, g2);
    case 1: return kept_index(p.f[1], g0, g1, g2);
    case 2: return kept_index(p.f[2], g0, g1, g2);
    default: return kept_index(p.f[3], g0, g1, g2);
  }
}

// Tile-boundary sums of one right-hand side (blockIdx.y), in the order own,
// x, y, xy; positions are numbered line by line (line length LM), lines:
// Part A: the x boundary planes of the fields nodal in x (sigma, u_y, u_z),
// lines along y: y += HX (+ HY + HXY where the position is on a y boundary
// too).  Part B: the y boundary planes of the fields nodal in y (sigma, u_x,
// u_z), lines along x: y += HY, except where part A adds.
template <typename TV>
__global__ void __launch_bounds__(256) hodge_mfma_fixup(HcParams p, int TX, int TY) {
  const int Nx = p.nel[0], Ny = p.nel[1], Nz = p.nel[2];
  const int LX = R * Nx + 1, LY = R * Ny + 1, LZ = R * Nz + 1, LM = max(LX, LY);
  const int bxn = p.tiles_x - 1, byn = p.tiles_y - 1;
  const int ra = 3 * bxn * LZ, rb = 3 * byn * LZ;
  const int rhs = blockIdx.y;
  TV* y = static_cast<TV*>(p.y) + (long long)rhs * p.ndofs;
  const double* hx = p.halo + (long long)rhs * (p.hx_n + p.hy_n + p.hxy_n);
  const double* hy = hx + p.hx_n;
  const double* hxy = hy + p.hy_n;
  const int total = (ra + rb) * LM;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const int row = t / LM, g = t - row * LM;
    if (row < ra) {
      const int fs = row / (bxn * LZ), rem = row - fs * bxn * LZ;
      const int bx = rem / LZ, gz = rem - bx * LZ;
      const int gy = g;
      if (gy >= LY) continue;
      const int F = fs == 0 ? 0 : fs + 1;  // sigma, u_y, u_z
      const int gx = R * TX * (bx + 1);
      const long long id = field_index(p, F, gx, gy, gz);
      if (id < 0) continue;
      double val = static_cast<double>(y[id]) + hx[((long long)(fs * bxn + bx) * LZ + gz) * LY + gy];
      if (F != 2 && gy % (R * TY) == 0 && gy > 0 && gy < R * Ny) {
        const int by = gy / (R * TY) - 1;
        const int fy = F == 0 ? 0 : 2, fxy = F == 0 ? 0 : 1;
        val += hy[((long long)(fy * byn + by) * LZ + gz) * LX + gx];
        val += hxy[((long long)(fxy * bxn + bx) * byn + by) * LZ + gz];
      }
      y[id] = static_cast<TV>(val);
    } else {
      const int r2 = row - ra;
      const int fs = r2 / (byn * LZ), rem = r2 - fs * byn * LZ;
      const int by = rem / LZ, gz = rem - by * LZ;
      const int gx = g;
      if (gx >= LX) continue;
      const int F = fs == 0 ? 0 : (fs == 1 ? 1 : 3);  // sigma, u_x, u_z
      if (F != 1 && gx % (R * TX) == 0 && gx > 0 && gx < R * Nx) continue;  // part A's
      const int gy = R * TY * (by + 1);
      const long long id = field_index(p, F, gx, gy, gz);
      if (id < 0) continue;
      y[id] = static_cast<TV>(static_cast<double>(y[id]) + hy[((long long)(fs * byn + by) * LZ + gz) * LX + gx]);
    }
  }
}

struct HaloDims {
  int tiles_x, tiles_y;
  long long hx, hy, hxy;
};
HaloDims halo_dims(const int nel[3]) {
  HaloDims h;
  h.tiles_x = (nel[0] + kTX - 1) / kTX;
  h.tiles_y = (nel[1] + kTY - 1) / kTY;
  const long long LX = R * (long long)nel[0] + 1, LY = R * (long long)nel[1] + 1, LZ = R * (long long)nel[2] + 1;
  h.hx = 3LL * (h.tiles_x - 1) * LZ * LY;
  h.hy = 3LL * (h.tiles_y - 1) * LZ * LX;
  h.hxy = 2LL * (h.tiles_x - 1) * (h.tiles_y - 1) * LZ;
  return h;
}

}  // namespace

long long hodge_mfma_halo_doubles(const int nel[3], int nrhs) {
  const HaloDims h = halo_dims(nel);
  return (long long)nrhs * (h.hx + h.hy + h.hxy);
}

int launch_hodge_mfma(const HcParams& p0, int nrhs, int ncu, hipStream_t s, bool f32) {
  HcParams p = p0;
  const HaloDims h = halo_dims(p.nel);
  p.nrhs = nrhs;
  p.tiles_x = h.tiles_x;
  p.tiles_y = h.tiles_y;
  p.hx_n = h.hx;
  p.hy_n = h.hy;
  p.hxy_n = h.hxy;
  const int ntiles = p.tiles_x * p.tiles_y, nz = p.nel[2];
  // z chunks: a chunk of c layers costs c + 1 (the recomputed layer below);
  // one workgroup per CU, ceil(workgroups / ncu) rounds
  long long best = -1;
  int bc = nz;
  for (int c = 1; c <= nz && p.chunk_mode == 0; ++c) {
    const long long nch = (nz + c - 1) / c;
    const long long wg = (long long)ntiles * nch * nrhs;
    const long long rounds = (wg + ncu - 1) / ncu;
    const long long cost = rounds * (c + (nch > 1 ? 1 : 0));
    if (best < 0 || cost < best || (cost == best && c > bc)) {
      best = cost;
      bc = c;
    }
  }
  if (p.chunk_mode == 2) bc = 1;
  p.chunk = bc;
  p.nchunks = (nz + bc - 1) / bc;
  p.nitems = ntiles * p.nchunks;
  const long long nblk = (long long)((p.nitems + 7) / 8) * 8 * nrhs;
  if (nblk >= (1LL << 31)) return -1;
  if (f32)
    hipLaunchKernelGGL((hodge_mfma_kernel<kTX, kTY, 2, float>), dim3((unsigned)nblk), dim3(kTX * kTY * 16), 0, s, p);
  else
    hipLaunchKernelGGL((hodge_mfma_kernel<kTX, kTY, 2, double>), dim3((unsigned)nblk), dim3(kTX * kTY * 16), 0, s, p);
  if (hipGetLastError() != hipSuccess) return -1;
  const int LX = R * p.nel[0] + 1, LY = R * p.nel[1] + 1, LZ = R * p.nel[2] + 1;
  const long long rows = 3LL * (p.tiles_x - 1) * LZ + 3LL * (p.tiles_y - 1) * LZ;
  const long long total = rows * std::max(LX, LY);
  if (total >= (1LL << 31)) return -1;
  if (total > 0) {
    const dim3 grid((unsigned)std::min<long long>((total + 255) / 256, 4LL * ncu), (unsigned)nrhs);
    if (f32)
      hipLaunchKernelGGL(hodge_mfma_fixup<float>, grid, dim3(256), 0, s, p, kTX, kTY);
    else
      hipLaunchKernelGGL(hodge_mfma_fixup<double>, grid, dim3(256), 0, s, p, kTX, kTY);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  return 0;
}

}  // namespace gym
