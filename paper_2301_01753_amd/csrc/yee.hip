// Fused generalized Yee step with lumped masses (paper sections 3, 4 and 4.3).
//
// On the refined lattice of a degree-r space (r N_d cells per axis, integral
// unknowns) the incidence C is the lattice curl, and the lumped M1 and M2~
// are diagonal.  So the P2 shear e += tau c^2 C^T M2~ C a and the Q1 shear
// a -= h Q1 e of one Strang step form a single stencil: at each lattice
// position the (up to three) Lambda^1 unknowns bound nine faces; their
// circulations b = C a, weighted by the lumped face masses, give C^T M2~ C a
// at the position, and e and then a are updated there.  Neighbours read a, so
// a goes from one buffer into another.  The lumped diagonals are recomputed
// from their 1-D row-sum factors, so a step moves a and e in and out once:
// 32 bytes per unknown.
//
// Blocks are renumbered so that the blocks one XCD runs (hardware dispatch
// hands block b to XCD b mod 8) cover one contiguous range of z-planes: the
// neighbour planes a block reads are then mostly in that XCD's own L2.
#include "yee.hpp"

#include <type_traits>

namespace gym {
namespace {

__device__ __forceinline__ bool kept(const DevComp& c, int x, int y, int z) {
  return (unsigned)(x - c.start[0]) < (unsigned)c.count[0] && (unsigned)(y - c.start[1]) < (unsigned)c.count[1] &&
         (unsigned)(z - c.start[2]) < (unsigned)c.count[2];
}

__device__ __forceinline__ long long at(const DevComp& c, int x, int y, int z) {
  return c.offset + (x - c.start[0]) +
         (long long)c.count[0] * ((y - c.start[1]) + (long long)c.count[1] * (z - c.start[2]));
}

template <class Fn>
__device__ __forceinline__ void static_for_comp(Fn&& fn) {
  fn(std::integral_constant<int, 0>{});
  fn(std::integral_constant<int, 1>{});
  fn(std::integral_constant<int, 2>{});
}

// a_c at lattice position (x, y, z); zero at the unknowns the conductor removes
template <int C>
__device__ __forceinline__ double lda(const YeeParams& p, int x, int y, int z) {
  const DevComp& d = p.s1.c[C];
  return kept(d, x, y, z) ? p.a_in[at(d, x, y, z)] : 0.0;
}

// Lumped mass: sc times the 1-D row sums along each axis, nodal along the
// axes whose bit is set in NODAL and edge along the others (the product taken
// in axis order, as the host builds the diagonals).
template <int NODAL>
__device__ __forceinline__ double lumped(const YeeParams& p, double sc, int x, int y, int z) {
  double v = sc;
  v *= p.w[((NODAL & 1) ? p.wn[0] : p.we[0]) + x];
  v *= p.w[((NODAL & 2) ? p.wn[1] : p.we[1]) + y];
  v *= p.w[((NODAL & 4) ? p.wn[2] : p.we[2]) + z];
  return v;
}

// The first half step in a, a <- a - ha Q1 e: pointwise, one thread per lattice position.
__global__ void __launch_bounds__(256) yee_half_kernel(const YeeParams p) {
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= p.npos) return;
  const unsigned row = t / (unsigned)p.len[0];
  const int x = (int)(t - row * (unsigned)p.len[0]);
  const int z = (int)(row / (unsigned)p.len[1]);
  const int y = (int)(row - (unsigned)z * (unsigned)p.len[1]);
  static_for_comp([&](auto cc) {
    constexpr int C = decltype(cc)::value;
    const DevComp& d = p.s1.c[C];
    if (!kept(d, x, y, z)) return;
    const long long i = at(d, x, y, z);
    const double q = p.e[i] * (1.0 / lumped<7 & ~(1 << C)>(p, p.q1s[C], x, y, z));
    p.a_out[i] = fma(-p.ha, q, p.a_in[i]);
  });
}

// 1-D lumped factor along axis D at lattice index i, nodal (i in [0, M_D]) or
// edge (i in [0, M_D)); zero where no such position exists.
template <int D, bool NODAL>
__device__ __forceinline__ double wfac(const YeeParams& p, int i) {
  const int m = p.len[D] - 1;
  if constexpr (NODAL) return (i >= 0 && i <= m) ? p.w[p.wn[D] + i] : 0.0;
  else return (i >= 0 && i < m) ? p.w[p.we[D] + i] : 0.0;
}

// A full Strang step, one thread per lattice column (x, y) and chunk of
// z-planes.  Going up the column, the thread carries a_x and a_y of its own
// column and of the columns at x - 1 and y - 1 from plane z + 1 to plane z,
// and the circulations of its x- and y-faces from plane z to the plane above,
// where they are the faces below.  Per plane it loads 15 values of a (its own
// a_z, and a of the neighbouring columns the nine faces reach), forms seven
// faces, applies C^T to the four faces around each of its unknowns, and
// updates e and a.  The x-y factors of the lumped masses are fixed along a
// column.  Neighbouring threads are neighbouring x, so every load and store
// of a wave is one contiguous row segment.
__global__ void __launch_bounds__(256) yee_column_kernel(const YeeParams p, int zc, unsigned ncol, unsigned nthr) {
  const unsigned nb = gridDim.x, b = blockIdx.x, xcd = b & 7u;
  const unsigned per = nb >> 3, rem = nb & 7u;
  const unsigned blk = xcd * per + min(xcd, rem) + (b >> 3);
  const unsigned t = blk * 256u + threadIdx.x;
  if (t >= nthr) return;
  const unsigned zch = t / ncol;
  const unsigned col = t - zch * ncol;
  const int x = (int)(col % (unsigned)p.len[0]);
  const int y = (int)(col / (unsigned)p.len[0]);
  const int z0 = (int)zch * zc;
  const int z1 = min(z0 + zc, p.len[2]);
  const DevComp& d0 = p.s1.c[0];
  const DevComp& d1 = p.s1.c[1];
  const DevComp& d2 = p.s1.c[2];
  auto okxy = [&](const DevComp& d, int dx, int dy) {
    return (unsigned)(x + dx - d.start[0]) < (unsigned)d.count[0] &&
           (unsigned)(y + dy - d.start[1]) < (unsigned)d.count[1];
  };
  // index within the component block (a component has fewer than 2^31
  // unknowns: the host launches this kernel only then)
  auto idx = [&](const DevComp& d, int dx, int dy, int z) {
    return (x + dx - d.start[0]) + d.count[0] * ((y + dy - d.start[1]) + d.count[1] * (z - d.start[2]));
  };
  const double* __restrict__ ain[3] = {p.a_in + d0.offset, p.a_in + d1.offset, p.a_in + d2.offset};
  // a of component C in column (x + dx, y + dy) at plane z; zero at removed unknowns
  auto A = [&](auto cc, int dx, int dy, int z) {
    constexpr int C = decltype(cc)::value;
    const DevComp& d = p.s1.c[C];
    return (okxy(d, dx, dy) && (unsigned)(z - d.start[2]) < (unsigned)d.count[2]) ? ain[C][idx(d, dx, dy, z)] : 0.0;
  };
  constexpr std::integral_constant<int, 0> X{};
  constexpr std::integral_constant<int, 1> Y{};
  constexpr std::integral_constant<int, 2> Z{};
  // x-y factors of the face masses (component: nodal along itself, edge along the others)
  const double rnx = wfac<0, true>(p, x), rex = wfac<0, false>(p, x), rexm = wfac<0, false>(p, x - 1);
  const double rny = wfac<1, true>(p, y), rey = wfac<1, false>(p, y), reym = wfac<1, false>(p, y - 1);
  const double whx = p.m2s[0] * rnx * rey, whx_y = p.m2s[0] * rnx * reym;
  const double why = p.m2s[1] * rex * rny, why_x = p.m2s[1] * rexm * rny;
  const double whz = p.m2s[2] * rex * rey, whz_y = p.m2s[2] * rex * reym, whz_x = p.m2s[2] * rexm * rey;
  // x-y factors of the edge masses (component: edge along itself, nodal along the others)
  const double wq0 = p.q1s[0] * rex * rny, wq1 = p.q1s[1] * rnx * rey, wq2 = p.q1s[2] * rnx * rny;
  const bool own0 = okxy(d0, 0, 0), own1 = okxy(d1, 0, 0), own2 = okxy(d2, 0, 0);

  double ax = A(X, 0, 0, z0), ay = A(Y, 0, 0, z0);  // a_x, a_y of this column at plane z
  double axm = A(X, -1, 0, z0), aym = A(Y, 0, -1, z0);  // a_x at x - 1, a_y at y - 1
  double hxb = 0.0, hyb = 0.0;  // x- and y-faces of this column below plane z
  if (z0 > 0) {
    const int zb = z0 - 1;
    const double reb = wfac<2, false>(p, zb), azb = A(Z, 0, 0, zb);
    hxb = whx * reb * ((A(Z, 0, 1, zb) - azb) - (ay - A(Y, 0, 0, zb)));
    hyb = why * reb * ((ax - A(X, 0, 0, zb)) - (A(Z, 1, 0, zb) - azb));
  }
  for (int z = z0; z < z1; ++z) {
    const double rez = wfac<2, false>(p, z), rnz = wfac<2, true>(p, z);
    const double az = A(Z, 0, 0, z);
    const double axu = A(X, 0, 0, z + 1), ayu = A(Y, 0, 0, z + 1);
    const double axmu = A(X, -1, 0, z + 1), aymu = A(Y, 0, -1, z + 1);
    const double az_xm = A(Z, -1, 0, z), ay_xm = A(Y, -1, 0, z);
    const double az_ym = A(Z, 0, -1, z), ax_ym = A(X, 0, -1, z);
    const double az_xp = A(Z, 1, 0, z), ay_xp = A(Y, 1, 0, z);
    const double az_yp = A(Z, 0, 1, z), ax_yp = A(X, 0, 1, z);
    const double ay_xp_ym = A(Y, 1, -1, z), ax_xm_yp = A(X, -1, 1, z);
    // faces at (x, y, z) and at the neighbours the unknowns of (x, y, z) bound
    const double hx = whx * rez * ((az_yp - az) - (ayu - ay));
    const double hy = why * rez * ((axu - ax) - (az_xp - az));
    const double hz = whz * rnz * ((ay_xp - ay) - (ax_yp - ax));
    const double hx_y = whx_y * rez * ((az - az_ym) - (aymu - aym));
    const double hy_x = why_x * rez * ((axmu - axm) - (az - az_xm));
    const double hz_y = whz_y * rnz * ((ay_xp_ym - aym) - (ax - ax_ym));
    const double hz_x = whz_x * rnz * ((ay - ay_xm) - (ax_xm_yp - axm));
    const double tv[3] = {(hz - hz_y) - (hy - hyb), (hx - hxb) - (hz - hz_x), (hy - hy_x) - (hx - hx_y)};
    const double av[3] = {ax, ay, az};
    const double wq[3] = {wq0 * rnz, wq1 * rnz, wq2 * rez};
    const bool own[3] = {own0, own1, own2};
    static_for_comp([&](auto cc) {
      constexpr int C = decltype(cc)::value;
      const DevComp& d = p.s1.c[C];
      if (!own[C] || (unsigned)(z - d.start[2]) >= (unsigned)d.count[2]) return;
      const long long i = d.offset + idx(d, 0, 0, z);
      const double ev = fma(p.te, tv[C], p.e[i]);
      p.e[i] = ev;
      p.a_out[i] = fma(-p.ha, ev * (1.0 / wq[C]), av[C]);
    });
    hxb = hx;
    hyb = hy;
    ax = axu;
    ay = ayu;
    axm = axmu;
    aym = aymu;
  }
}

}  // namespace

int launch_yee(const YeeParams& p, bool half, int ncu, hipStream_t s) {
  if (p.npos == 0) return 0;
  if (half) {
    hipLaunchKernelGGL(yee_half_kernel, dim3((p.npos + 255u) / 256u), dim3(256), 0, s, p);
  } else {
    // z-chunks short enough for about eight blocks per CU, 2..8 planes long
    // (measured best on MI355X: 2 planes at 65^3 positions, 4 at 129^3, 8 at 257^3)
    const unsigned ncol = (unsigned)p.len[0] * (unsigned)p.len[1];
    long long zc = (long long)p.npos / (8LL * ncu * 256);
    zc = zc < 2 ? 2 : (zc > 8 ? 8 : zc);
    const unsigned nzc = (unsigned)((p.len[2] + zc - 1) / zc);
    const unsigned nthr = ncol * nzc;
    hipLaunchKernelGGL(yee_column_kernel, dim3((nthr + 255u) / 256u), dim3(256), 0, s, p, (int)zc, ncol, nthr);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gym
