// Fused matrix-free operator kernels on affine (axis-aligned) meshes.
//
// Problems (unknown blocks in canonical layout, paper section 2 objects):
//   POISSON : [s in HDIV; p in L2]      y_s = M2 s - D^T M3 p,  y_p = -M3 D s
//   HODGE   : [sigma in H1_0; u in H0(curl)]
//             y_sigma = -M0 sigma + G^T M1 u,  y_u = M1 G sigma + C^T M2 C u
//   MASS_k  : y = M_k x for one space
// Per element layer of a tile (see tile.hpp) the incidence is applied on the
// closure (+-1 sums), each mass block by sum factorisation, and the
// transposed incidence on the closure; this equals the sum over elements of
// the element-local operators because incidence commutes with restriction
// to an element.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gym_internal.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace gym {

__constant__ TabSet<double> c_tab_d[4];
__constant__ TabSet<float> c_tab_f[4];
__constant__ TabSet<double> c_tabL_d[4];

// ---- field lists ---------------------------------------------------------
// tm: nodal mask of the field's lattice; sp: 0 = first block, 1 = second
// block of the operator vector; cp: component within its space.
template <int PROB, int DIM>
struct Fields;

template <>
struct Fields<PROB_HODGE, 3> {
  static constexpr int NF = 4;
  static constexpr int tm[4] = {7, 6, 5, 3};
  static constexpr int sp[4] = {0, 1, 1, 1};
  static constexpr int cp[4] = {0, 0, 1, 2};
};
template <>
struct Fields<PROB_POISSON, 3> {
  static constexpr int NF = 4;
  static constexpr int tm[4] = {1, 2, 4, 0};
  static constexpr int sp[4] = {0, 0, 0, 1};
  static constexpr int cp[4] = {0, 1, 2, 0};
};
template <>
struct Fields<PROB_POISSON, 2> {
  static constexpr int NF = 3;
  static constexpr int tm[3] = {1, 2, 0};
  static constexpr int sp[3] = {0, 0, 1};
  static constexpr int cp[3] = {0, 1, 0};
};
template <>
struct Fields<PROB_MASS_H1, 3> {
  static constexpr int NF = 1;
  static constexpr int tm[1] = {7};
  static constexpr int sp[1] = {0};
  static constexpr int cp[1] = {0};
};
template <>
struct Fields<PROB_MASS_H1, 2> {
  static constexpr int NF = 1;
  static constexpr int tm[1] = {3};
  static constexpr int sp[1] = {0};
  static constexpr int cp[1] = {0};
};
template <>
struct Fields<PROB_MASS_HCURL, 3> {
  static constexpr int NF = 3;
  static constexpr int tm[3] = {6, 5, 3};
  static constexpr int sp[3] = {0, 0, 0};
  static constexpr int cp[3] = {0, 1, 2};
};
template <>
struct Fields<PROB_MASS_HCURL, 2> {
  static constexpr int NF = 2;
  static constexpr int tm[2] = {2, 1};
  static constexpr int sp[2] = {0, 0};
  static constexpr int cp[2] = {0, 1};
};
template <>
struct Fields<PROB_MASS_HDIV, 3> {
  static constexpr int NF = 3;
  static constexpr int tm[3] = {1, 2, 4};
  static constexpr int sp[3] = {0, 0, 0};
  static constexpr int cp[3] = {0, 1, 2};
};
template <>
struct Fields<PROB_MASS_HDIV, 2> {
  static constexpr int NF = 2;
  static constexpr int tm[2] = {1, 2};
  static constexpr int sp[2] = {0, 0};
  static constexpr int cp[2] = {0, 1};
};
template <>
struct Fields<PROB_MASS_L2, 3> {
  static constexpr int NF = 1;
  static constexpr int tm[1] = {0};
  static constexpr int sp[1] = {0};
  static constexpr int cp[1] = {0};
};
template <>
struct Fields<PROB_MASS_L2, 2> {
  static constexpr int NF = 1;
  static constexpr int tm[1] = {0};
  static constexpr int sp[1] = {0};
  static constexpr int cp[1] = {0};
};

template <int I, int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, N>(fn);
  }
}

// ---- LDS layout ------------------------------------------------------------
template <class C, class F, bool KRON>
struct Layout {
  static constexpr int lat(int f) { return C::lat(F::tm[f]); }
  static constexpr bool carries(int f) { return C::DIM == 3 && (F::tm[f] & 4); }
  static constexpr int in_off(int f) {
    int o = 0;
    for (int g = 0; g < f; ++g) o += lat(g);
    return o;
  }
  static constexpr int out_off(int f) { return in_off(F::NF) + in_off(f); }
  static constexpr int car_off(int f) {
    int o = 2 * in_off(F::NF);
    for (int g = 0; g < f; ++g) o += carries(g) ? C::plane(F::tm[g]) : 0;
    return o;
  }
  static constexpr int maxlat() {
    int m = 0;
    for (int t = 0; t < 8; ++t) m = C::lat(t) > m ? C::lat(t) : m;
    return m;
  }
  static constexpr int A_off() { return car_off(F::NF); }
  static constexpr int B_off() { return A_off() + (KRON ? maxlat() : C::tmpA()); }
  static constexpr int L1_off() { return B_off() + (KRON ? maxlat() : C::tmpB()); }
  static constexpr int L2_off() { return L1_off() + maxlat(); }
  static constexpr int total() { return L2_off() + maxlat(); }
};

// extent of the lattice of mask TM along axis a
template <class C, int TM>
__device__ __forceinline__ int ext(int a) {
  return a == 0 ? C::nx(TM) : (a == 1 ? C::ny(TM) : C::nz(TM));
}

// ---- the kernel ------------------------------------------------------------
template <class C, int PROB, bool KRON, typename TV, typename TC>
__global__ void __launch_bounds__(kNT) op_kernel(const OpParams p) {
  using F = Fields<PROB, C::DIM>;
  using L = Layout<C, F, KRON>;
  constexpr int R = C::R;
  __shared__ TC smem[L::total()];
  TC* A = smem + L::A_off();
  TC* B = smem + L::B_off();
  TC* L1 = smem + L::L1_off();
  TC* L2 = smem + L::L2_off();

  // XCD-aware tile order: consecutive hardware block ids go round-robin over
  // the 8 XCDs; remap so that each XCD receives a contiguous run of tiles.
  const int nt = p.tiles_x * p.tiles_y;
  int b = blockIdx.x;
  if (nt % 8 == 0) b = (b % 8) * (nt / 8) + b / 8;
  const int tx = b % p.tiles_x, ty = b / p.tiles_x;
  const int X0 = tx * C::BX, Y0 = ty * C::BY;
  const int rhs = blockIdx.z;
  const TV* __restrict__ xin = reinterpret_cast<const TV*>(p.x) + (long long)rhs * p.ndofs;
  TV* __restrict__ yout = reinterpret_cast<TV*>(p.y) + (long long)rhs * p.ndofs;
  const int gx0 = R * (X0 - 1), gy0 = R * (Y0 - 1);
  // local element e <-> global X0 - 1 + e
  const ElemRange er{max(0, 1 - X0), min(C::EX, p.nel[0] - X0 + 1), max(0, 1 - Y0),
                     min(C::EY, p.nel[1] - Y0 + 1)};

  int zfirst = 0, zbeg = 0, zend = 1;
  if constexpr (C::DIM == 3) {
    zfirst = blockIdx.y * p.chunk;
    zend = min(zfirst + p.chunk, p.nel[2]);
    zbeg = zfirst > 0 ? zfirst - 1 : 0;
  }

  static_for<0, F::NF>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    if constexpr (L::carries(f)) {
      TC* car = smem + L::car_off(f);
      for (int i = threadIdx.x; i < C::plane(F::tm[f]); i += kNT) car[i] = 0;
    }
  });

  for (int ez = zbeg; ez < zend; ++ez) {
    const int gz0 = C::DIM == 3 ? R * ez : 0;
    // ---- load inputs, zero outputs
    static_for<0, F::NF>([&](auto fc) {
      constexpr int f = decltype(fc)::value;
      constexpr int TM = F::tm[f];
      const DevComp& cd = (F::sp[f] == 0 ? p.sa : p.sb).c[F::cp[f]];
      TC* in = smem + L::in_off(f);
      TC* out = smem + L::out_off(f);
      for (int i = threadIdx.x; i < C::lat(TM); i += kNT) {
        int lx, ly, lz;
        lpos<C, TM>(i, lx, ly, lz);
        int g0 = gx0 + lx - cd.start[0], g1 = gy0 + ly - cd.start[1], g2 = gz0 + lz - cd.start[2];
        TC v = 0;
        if (g0 >= 0 && g0 < cd.count[0] && g1 >= 0 && g1 < cd.count[1] && g2 >= 0 && g2 < cd.count[2])
          v = static_cast<TC>(xin[cd.offset + g0 + (long long)cd.count[0] * (g1 + (long long)cd.count[1] * g2)]);
        in[i] = v;
        out[i] = 0;
      }
    });
    __syncthreads();

    TC* in0 = smem + L::in_off(0);
    TC* out0 = smem + L::out_off(0);

    if constexpr (PROB == PROB_HODGE) {
      // -M0 sigma
      mass<C, 7, true, KRON>(in0, out0, (TC)-p.sc[0], A, B, er);
      // G^T (M1 u): v_c = M1_c u_c on the closure, then y_sigma(q) += v_c(q-e_c) - v_c(q)
      static_for<0, 3>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int TE = 7 & ~(1 << c);
        mass<C, TE, false, KRON>(smem + L::in_off(1 + c), L1, (TC)p.sc[1 + c], A, B, er);
        for (int i = threadIdx.x; i < C::lat(7); i += kNT) {
          int q[3];
          lpos<C, 7>(i, q[0], q[1], q[2]);
          TC acc = 0;
          const int qc = q[c];
          if (qc >= 1) {
            int s[3] = {q[0], q[1], q[2]};
            s[c] -= 1;
            acc += L1[lidx<C, TE>(s[0], s[1], s[2])];
          }
          if (qc < ext<C, TE>(c)) acc -= L1[lidx<C, TE>(q[0], q[1], q[2])];
          out0[i] += acc;
        }
        __syncthreads();
      });
      // M1 G sigma
      static_for<0, 3>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int TE = 7 & ~(1 << c);
        for (int i = threadIdx.x; i < C::lat(TE); i += kNT) {
          int q[3];
          lpos<C, TE>(i, q[0], q[1], q[2]);
          int s[3] = {q[0], q[1], q[2]};
          s[c] += 1;
          TC g = -in0[lidx<C, 7>(q[0], q[1], q[2])];
          g += in0[lidx<C, 7>(s[0], s[1], s[2])];
          L1[i] = g;
        }
        __syncthreads();
        mass<C, TE, true, KRON>(L1, smem + L::out_off(1 + c), (TC)p.sc[1 + c], A, B, er);
      });
      // C^T M2 C u
      static_for<0, 3>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        constexpr int TF = 1 << c;
        constexpr int T1 = 7 & ~(1 << c1), T2 = 7 & ~(1 << c2);
        const TC* a1 = smem + L::in_off(1 + c1);
        const TC* a2 = smem + L::in_off(1 + c2);
        // b_c(p) = a_c2(p + e_c1) - a_c2(p) - a_c1(p + e_c2) + a_c1(p)
        for (int i = threadIdx.x; i < C::lat(TF); i += kNT) {
          int q[3];
          lpos<C, TF>(i, q[0], q[1], q[2]);
          int s1[3] = {q[0], q[1], q[2]}, s2[3] = {q[0], q[1], q[2]};
          s1[c1] += 1;
          s2[c2] += 1;
          TC v = a2[lidx<C, T2>(s1[0], s1[1], s1[2])];
          v -= a2[lidx<C, T2>(q[0], q[1], q[2])];
          v -= a1[lidx<C, T1>(s2[0], s2[1], s2[2])];
          v += a1[lidx<C, T1>(q[0], q[1], q[2])];
          L1[i] = v;
        }
        __syncthreads();
        mass<C, TF, false, KRON>(L1, L2, (TC)p.sc[4 + c], A, B, er);
        // (C^T z)_c2(q) = z_c(q - e_c1) - z_c(q); (C^T z)_c1(q) = z_c(q) - z_c(q - e_c2)
        TC* o2 = smem + L::out_off(1 + c2);
        for (int i = threadIdx.x; i < C::lat(T2); i += kNT) {
          int q[3];
          lpos<C, T2>(i, q[0], q[1], q[2]);
          TC acc = 0;
          if (q[c1] >= 1) {
            int s[3] = {q[0], q[1], q[2]};
            s[c1] -= 1;
            acc += L2[lidx<C, TF>(s[0], s[1], s[2])];
          }
          if (q[c1] < ext<C, TF>(c1)) acc -= L2[lidx<C, TF>(q[0], q[1], q[2])];
          o2[i] += acc;
        }
        TC* o1 = smem + L::out_off(1 + c1);
        for (int i = threadIdx.x; i < C::lat(T1); i += kNT) {
          int q[3];
          lpos<C, T1>(i, q[0], q[1], q[2]);
          TC acc = 0;
          if (q[c2] < ext<C, TF>(c2)) acc += L2[lidx<C, TF>(q[0], q[1], q[2])];
          if (q[c2] >= 1) {
            int s[3] = {q[0], q[1], q[2]};
            s[c2] -= 1;
            acc -= L2[lidx<C, TF>(s[0], s[1], s[2])];
          }
          o1[i] += acc;
        }
        __syncthreads();
      });
    } else if constexpr (PROB == PROB_POISSON) {
      constexpr int D = C::DIM;
      constexpr int NS = D;                    // flux components
      TC* inp = smem + L::in_off(NS);
      TC* outp = smem + L::out_off(NS);
      // M2 s
      static_for<0, NS>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        mass<C, F::tm[c], true, KRON>(smem + L::in_off(c), smem + L::out_off(c), (TC)p.sc[c], A, B, er);
      });
      // -D^T (M3 p): y_s_c(q) += w(q) - w(q - e_c)
      mass<C, 0, false, KRON>(inp, L1, (TC)p.sc[3], A, B, er);
      static_for<0, NS>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int TF = F::tm[c];
        TC* o = smem + L::out_off(c);
        for (int i = threadIdx.x; i < C::lat(TF); i += kNT) {
          int q[3];
          lpos<C, TF>(i, q[0], q[1], q[2]);
          TC acc = 0;
          if (q[c] < ext<C, 0>(c)) acc += L1[lidx<C, 0>(q[0], q[1], q[2])];
          if (q[c] >= 1) {
            int s[3] = {q[0], q[1], q[2]};
            s[c] -= 1;
            acc -= L1[lidx<C, 0>(s[0], s[1], s[2])];
          }
          o[i] += acc;
        }
      });
      __syncthreads();
      // -M3 (D s): div(p) = sum_c s_c(p + e_c) - s_c(p)
      for (int i = threadIdx.x; i < C::lat(0); i += kNT) {
        int q[3];
        lpos<C, 0>(i, q[0], q[1], q[2]);
        TC v = 0;
        static_for<0, NS>([&](auto cc) {
          constexpr int c = decltype(cc)::value;
          constexpr int TF = F::tm[c];
          const TC* s = smem + L::in_off(c);
          int t[3] = {q[0], q[1], q[2]};
          t[c] += 1;
          v -= s[lidx<C, TF>(q[0], q[1], q[2])];
          v += s[lidx<C, TF>(t[0], t[1], t[2])];
        });
        L1[i] = v;
      }
      __syncthreads();
      mass<C, 0, true, KRON>(L1, outp, (TC)-p.sc[3], A, B, er);
    } else {
      static_for<0, F::NF>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        mass<C, F::tm[f], true, KRON>(smem + L::in_off(f), smem + L::out_off(f), (TC)p.sc[f], A, B, er);
      });
    }

    // ---- carry the shared top plane to the next layer
    if constexpr (C::DIM == 3) {
      static_for<0, F::NF>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        if constexpr (L::carries(f)) {
          constexpr int PL = C::plane(F::tm[f]);
          TC* out = smem + L::out_off(f);
          TC* car = smem + L::car_off(f);
          for (int i = threadIdx.x; i < PL; i += kNT) {
            out[i] += car[i];
            car[i] = out[i + R * PL];
          }
        }
      });
      __syncthreads();
    }

    // ---- write owned positions
    if (ez >= zfirst) {
      static_for<0, F::NF>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        constexpr int TM = F::tm[f];
        const DevComp& cd = (F::sp[f] == 0 ? p.sa : p.sb).c[F::cp[f]];
        const TC* out = smem + L::out_off(f);
        for (int i = threadIdx.x; i < C::lat(TM); i += kNT) {
          int lx, ly, lz;
          lpos<C, TM>(i, lx, ly, lz);
          int G0 = gx0 + lx, G1 = gy0 + ly, G2 = gz0 + lz;
          bool own = G0 >= R * X0 && (G0 < R * (X0 + C::BX) || G0 == p.m[0]) &&
                     G1 >= R * Y0 && (G1 < R * (Y0 + C::BY) || G1 == p.m[1]);
          if constexpr (C::DIM == 3) own = own && (G2 < gz0 + R || G2 == p.m[2]);
          int g0 = G0 - cd.start[0], g1 = G1 - cd.start[1], g2 = G2 - cd.start[2];
          if (own && g0 >= 0 && g0 < cd.count[0] && g1 >= 0 && g1 < cd.count[1] && g2 >= 0 &&
              g2 < cd.count[2])
            yout[cd.offset + g0 + (long long)cd.count[0] * (g1 + (long long)cd.count[1] * g2)] =
                static_cast<TV>(out[i]);
        }
      });
    }
    __syncthreads();
  }
}

// ---- tile-size selection ----------------------------------------------------
// Largest square tile whose LDS footprint fits `budget` bytes (2..8 per side;
// up to 16 in 2-D).  Two budgets are compiled: the whole 160 KB of a CU (one
// workgroup per CU, least halo recomputation) and 40 KB (four workgroups per
// CU, more waves to hide LDS latency).
template <int DIM, int R, int PROB, bool KRON, typename TC, int BUDGET>
struct TileSel {
  template <int B>
  static constexpr int bytes() {
    using C = Cfg<R, B, B, DIM>;
    return Layout<C, Fields<PROB, DIM>, KRON>::total() * (int)sizeof(TC);
  }
  static constexpr int B = DIM == 2 ? (bytes<16>() <= BUDGET ? 16 : (bytes<8>() <= BUDGET ? 8 : (bytes<4>() <= BUDGET ? 4 : 2)))
                           : bytes<8>() <= BUDGET ? 8
                           : bytes<6>() <= BUDGET ? 6
                           : bytes<4>() <= BUDGET ? 4
                           : bytes<3>() <= BUDGET ? 3
                                                  : 2;
};

template <int DIM, int R, int PROB, bool KRON, typename TV, typename TC, int BUDGET>
int launch_op_b(const OpParams& p0, int nrhs, int ncu, hipStream_t stream) {
  constexpr int B = TileSel<DIM, R, PROB, KRON, TC, BUDGET>::B;
  using C = Cfg<R, B, B, DIM>;
  static_assert(Layout<C, Fields<PROB, DIM>, KRON>::total() * sizeof(TC) <= 160 * 1024, "LDS");
  OpParams p = p0;
  p.tiles_x = (p.nel[0] + B - 1) / B;
  p.tiles_y = (p.nel[1] + B - 1) / B;
  const int nt = p.tiles_x * p.tiles_y;
  int nchunks = 1;
  p.chunk = 1;
  if (DIM == 3) {
    // enough workgroups for two per CU, but chunks of at least 4 layers so
    // that the recomputed halo layer costs at most a quarter
    const int target = 2 * ncu;
    nchunks = (target + nt * nrhs - 1) / (nt * nrhs);
    int maxch = p.nel[2] / 4;
    if (nchunks > maxch) nchunks = maxch;
    if (nchunks < 1) nchunks = 1;
    p.chunk = (p.nel[2] + nchunks - 1) / nchunks;
    nchunks = (p.nel[2] + p.chunk - 1) / p.chunk;
  }
  dim3 grid(nt, nchunks, nrhs);
  hipLaunchKernelGGL((op_kernel<C, PROB, KRON, TV, TC>), grid, dim3(kNT), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int DIM, int R, int PROB, typename TV, typename TC>
int launch_op(const OpParams& p, int nrhs, int ncu, hipStream_t stream) {
  if (p.kron) {
    if (p.tile_budget == 0) return launch_op_b<DIM, R, PROB, true, TV, TC, 160 * 1024>(p, nrhs, ncu, stream);
    return launch_op_b<DIM, R, PROB, true, TV, TC, 40 * 1024>(p, nrhs, ncu, stream);
  }
  if (p.tile_budget == 0) return launch_op_b<DIM, R, PROB, false, TV, TC, 160 * 1024>(p, nrhs, ncu, stream);
  return launch_op_b<DIM, R, PROB, false, TV, TC, 40 * 1024>(p, nrhs, ncu, stream);
}

template <int DIM, int PROB, typename TV, typename TC>
int dispatch_r(int r, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  switch (r) {
    case 1: return launch_op<DIM, 1, PROB, TV, TC>(p, nrhs, ncu, s);
    case 2: return launch_op<DIM, 2, PROB, TV, TC>(p, nrhs, ncu, s);
    case 3: return launch_op<DIM, 3, PROB, TV, TC>(p, nrhs, ncu, s);
    case 4: return launch_op<DIM, 4, PROB, TV, TC>(p, nrhs, ncu, s);
  }
  return -2;
}

template <typename TV, typename TC>
int dispatch_prob(int prob, int dim, int r, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  if (dim == 3) {
    switch (prob) {
      case PROB_HODGE: return dispatch_r<3, PROB_HODGE, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_POISSON: return dispatch_r<3, PROB_POISSON, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_H1: return dispatch_r<3, PROB_MASS_H1, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_HCURL: return dispatch_r<3, PROB_MASS_HCURL, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_HDIV: return dispatch_r<3, PROB_MASS_HDIV, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_L2: return dispatch_r<3, PROB_MASS_L2, TV, TC>(r, p, nrhs, ncu, s);
    }
  } else if (dim == 2) {
    switch (prob) {
      case PROB_POISSON: return dispatch_r<2, PROB_POISSON, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_H1: return dispatch_r<2, PROB_MASS_H1, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_HCURL: return dispatch_r<2, PROB_MASS_HCURL, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_HDIV: return dispatch_r<2, PROB_MASS_HDIV, TV, TC>(r, p, nrhs, ncu, s);
      case PROB_MASS_L2: return dispatch_r<2, PROB_MASS_L2, TV, TC>(r, p, nrhs, ncu, s);
    }
  }
  return -2;
}

int launch_operator(int prob, int dim, int r, int prec, const OpParams& p, int nrhs, int ncu,
                    hipStream_t s) {
  if (prec == GYM_F64) return dispatch_prob<double, double>(prob, dim, r, p, nrhs, ncu, s);
  if (prec == GYM_F32) return dispatch_prob<float, float>(prob, dim, r, p, nrhs, ncu, s);
  return -2;
}

int upload_tables() {
  TabSet<double> hd[4] = {}, hl[4] = {};
  TabSet<float> hf[4] = {};
  for (int r = 1; r <= 4; ++r) {
    for (int which = 0; which < 2; ++which) {
      int q = r + 1 + which;
      Tables1D t = make_tables(r, q);
      TabSet<double>& d = which == 0 ? hd[r - 1] : hl[r - 1];
      for (int s = 0; s < q; ++s) {
        d.w[s] = t.gw[s];
        d.gx[s] = t.gx[s];
        for (int i = 0; i <= r; ++i) {
          d.phi[s][i] = t.phi[s * (r + 1) + i];
          d.phiw[s][i] = t.gw[s] * t.phi[s * (r + 1) + i];
        }
        for (int j = 0; j < r; ++j) {
          d.edge[s][j] = t.edge[s * r + j];
          d.edgew[s][j] = t.gw[s] * t.edge[s * r + j];
        }
      }
      for (int i = 0; i <= r; ++i)
        for (int j = 0; j <= r; ++j) {
          double acc = 0;
          for (int s = 0; s < q; ++s) acc += t.gw[s] * t.phi[s * (r + 1) + i] * t.phi[s * (r + 1) + j];
          d.mn[i][j] = acc;
        }
      for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) {
          double acc = 0;
          for (int s = 0; s < q; ++s) acc += t.gw[s] * t.edge[s * r + i] * t.edge[s * r + j];
          d.me[i][j] = acc;
        }
    }
    TabSet<float>& f = hf[r - 1];
    const TabSet<double>& d = hd[r - 1];
    for (int s = 0; s < 6; ++s) {
      f.w[s] = (float)d.w[s];
      f.gx[s] = (float)d.gx[s];
      for (int i = 0; i < 5; ++i) f.phi[s][i] = (float)d.phi[s][i], f.phiw[s][i] = (float)d.phiw[s][i];
      for (int j = 0; j < 4; ++j) f.edge[s][j] = (float)d.edge[s][j], f.edgew[s][j] = (float)d.edgew[s][j];
    }
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) f.mn[i][j] = (float)d.mn[i][j];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) f.me[i][j] = (float)d.me[i][j];
  }
  GYM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tab_d), hd, sizeof(hd)));
  GYM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tabL_d), hl, sizeof(hl)));
  GYM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tab_f), hf, sizeof(hf)));
  return 0;
}

}  // namespace gym
