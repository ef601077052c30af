// Fused generalized Yee step with lumped masses (paper sections 3, 4 and 4.3).
//
// On the refined lattice of a degree-r space (r N_d cells per axis, integral
// unknowns) the incidence C is the lattice curl, and the lumped M1 and M2~
// are diagonal.  So the P2 shear e += tau c^2 C^T M2~ C a and the Q1 shear
// a -= h Q1 e of one Strang step form a single stencil.  One thread per
// lattice position p holds the (up to three) Lambda^1 unknowns at p.  It forms
// the nine face circulations b = C a that they bound, weights each by its
// lumped face mass, applies C^T, and updates e and then a at p.  Neighbours
// read a, so a goes from one buffer into another.  The lumped diagonals are
// recomputed from their 1-D row-sum factors, so a step moves a and e in and
// out once: 32 bytes per unknown.
//
// Blocks are renumbered so that the blocks one XCD runs (hardware dispatch
// hands block b to XCD b mod 8) cover one contiguous range of z-planes: the
// neighbour planes a block reads are then mostly in that XCD's own L2.
#include "yee.hpp"

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

// (M2~ C a) on the face of component C at (x, y, z):
// b_C = (a_C2(q + e_C1) - a_C2(q)) - (a_C1(q + e_C2) - a_C1(q)), C1 = C + 1, C2 = C + 2 (mod 3).
template <int C>
__device__ __forceinline__ double face(const YeeParams& p, int x, int y, int z) {
  constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
  const double b = (lda<C2>(p, x + (C1 == 0), y + (C1 == 1), z + (C1 == 2)) - lda<C2>(p, x, y, z)) -
                   (lda<C1>(p, x + (C2 == 0), y + (C2 == 1), z + (C2 == 2)) - lda<C1>(p, x, y, z));
  return lumped<1 << C>(p, p.m2s[C], x, y, z) * b;
}

template <int C, bool HALF>
__device__ __forceinline__ void update(const YeeParams& p, int x, int y, int z, double t) {
  const long long i = at(p.s1.c[C], x, y, z);
  double ev = p.e[i];
  if constexpr (!HALF) {
    ev = fma(p.te, t, ev);
    p.e[i] = ev;
  }
  const double q = ev * (1.0 / lumped<7 & ~(1 << C)>(p, p.q1s[C], x, y, z));
  p.a_out[i] = fma(-p.ha, q, p.a_in[i]);
}

template <bool HALF>
__global__ void __launch_bounds__(256) yee_kernel(const YeeParams p) {
  const unsigned nb = gridDim.x, b = blockIdx.x, xcd = b & 7u;
  const unsigned per = nb >> 3, rem = nb & 7u;
  const unsigned blk = xcd * per + min(xcd, rem) + (b >> 3);
  const unsigned t = blk * 256u + threadIdx.x;
  if (t >= p.npos) return;
  const unsigned row = t / (unsigned)p.len[0];
  const int x = (int)(t - row * (unsigned)p.len[0]);
  const int z = (int)(row / (unsigned)p.len[1]);
  const int y = (int)(row - (unsigned)z * (unsigned)p.len[1]);
  const bool k0 = kept(p.s1.c[0], x, y, z), k1 = kept(p.s1.c[1], x, y, z), k2 = kept(p.s1.c[2], x, y, z);
  if (!(k0 || k1 || k2)) return;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  if constexpr (!HALF) {
    // C^T h at p (h = M2~ C a): each Lambda^1 unknown bounds four faces.  A
    // face is formed only when an unknown kept at p needs it; those faces all
    // exist in Lambda^2.
    const double hx = (k1 || k2) ? face<0>(p, x, y, z) : 0.0;
    const double hx_z = k1 ? face<0>(p, x, y, z - 1) : 0.0;
    const double hx_y = k2 ? face<0>(p, x, y - 1, z) : 0.0;
    const double hy = (k0 || k2) ? face<1>(p, x, y, z) : 0.0;
    const double hy_z = k0 ? face<1>(p, x, y, z - 1) : 0.0;
    const double hy_x = k2 ? face<1>(p, x - 1, y, z) : 0.0;
    const double hz = (k0 || k1) ? face<2>(p, x, y, z) : 0.0;
    const double hz_y = k0 ? face<2>(p, x, y - 1, z) : 0.0;
    const double hz_x = k1 ? face<2>(p, x - 1, y, z) : 0.0;
    t0 = (hz - hz_y) - (hy - hy_z);
    t1 = (hx - hx_z) - (hz - hz_x);
    t2 = (hy - hy_x) - (hx - hx_y);
  }
  if (k0) update<0, HALF>(p, x, y, z, t0);
  if (k1) update<1, HALF>(p, x, y, z, t1);
  if (k2) update<2, HALF>(p, x, y, z, t2);
}

}  // namespace

int launch_yee(const YeeParams& p, bool half, hipStream_t s) {
  if (p.npos == 0) return 0;
  const unsigned blocks = (p.npos + 255u) / 256u;
  if (half) hipLaunchKernelGGL(yee_kernel<true>, dim3(blocks), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(yee_kernel<false>, dim3(blocks), dim3(256), 0, s, p);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gym
