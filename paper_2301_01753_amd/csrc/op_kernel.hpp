// Fused matrix-free operator kernel (included by the op_*.hip units).
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
//
// Mass forms (template FORM):
//   FORM_GAUSS  Gauss-point contractions, constant metric (affine cells)
//   FORM_KRON   Kronecker product of 1-D element masses (affine cells)
//   FORM_CURVED Gauss-point contractions with the metric of the multilinear
//               cell map evaluated at every Gauss point (curved cells)
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "curved.hpp"
#include "gym_internal.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace gym {

enum { FORM_GAUSS = 0, FORM_KRON = 1, FORM_CURVED = 2, FORM_KRON_BF16 = 3 };
// FORM_KRON_BF16: the Kronecker form with every contraction operand rounded
// to bf16 (FP32 accumulation, FP32 vectors)
constexpr bool is_kron(int form) { return form == FORM_KRON || form == FORM_KRON_BF16; }

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
// Per field: the input and output lattice closures of the layer, the carried
// top plane (nodal-in-z fields), then the work arrays of the mass form:
//   affine forms: A, B (and T2 for the Kronecker form), three lattice
//     temporaries L for the incidence stages;
//   curved form: the three lattice temporaries L, then per vector component
//     an x-contracted array WA ([QX][ny][nz]) and an x-y-contracted one WB
//     ([QX][QY][nz]).
template <class C, class F, int FORM>
struct Layout {
  static constexpr bool CURVED = FORM == FORM_CURVED;
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
  static constexpr int B_off() { return A_off() + (CURVED ? 0 : is_kron(FORM) ? maxlat() : C::tmpA()); }
  // Kronecker form: a third lattice temporary (one per vector component)
  static constexpr int T2_off() { return B_off() + (CURVED ? 0 : is_kron(FORM) ? maxlat() : C::tmpB()); }
  static constexpr int L_off(int k) { return T2_off() + (is_kron(FORM) ? maxlat() : 0) + k * maxlat(); }
  // curved form: contraction work arrays per component
  static constexpr int wa() { return C::QX * (C::R * C::EY + 1) * C::nz(7); }
  static constexpr int wb() { return C::QX * C::QY * C::nz(7); }
  static constexpr int WA_off(int k) { return L_off(3) + k * wa(); }
  static constexpr int WB_off(int k) { return WA_off(3) + k * wb(); }
  static constexpr int total() { return CURVED ? WB_off(3) : L_off(3); }
};

// extent of the lattice of mask TM along axis a
template <class C, int TM>
__device__ __forceinline__ int ext(int a) {
  return a == 0 ? C::nx(TM) : (a == 1 ? C::ny(TM) : C::nz(TM));
}

// Work buffers of one layer.
template <typename TC>
struct Work {
  TC *A, *B, *T2, *L[3];
  TC *WA[3], *WB[3];  // curved form
  QGeom<TC> g;        // curved form: the layer's Gauss-point metrics
  ElemRange er;
};

// ---- curved cells (curved.hpp stages) -----------------------------------------
template <class C, int TM, int KIND, bool ADD, typename TC>
__device__ __forceinline__ void cmass_scalar(const TC* in, TC* out, TC sign, const Work<TC>& w) {
  constexpr int NY = C::ny(TM), NZ = C::nz(TM);
  for (int l = stage_tid(); l < C::EX * NY * NZ; l += C::NT) cfwd_x<C, TM>(in, w.WA[0], l);
  __syncthreads();
  for (int l = stage_tid(); l < C::QX * C::EY * NZ; l += C::NT) cfwd_y<C, TM>(w.WA[0], w.WB[0], l);
  __syncthreads();
  for (int p = stage_tid(); p < C::QX * C::QY; p += C::NT) cz_scalar<C, TM, KIND>(w.WB[0], p, w.er, w.g, sign);
  __syncthreads();
  for (int l = stage_tid(); l < C::QX * C::EY * NZ; l += C::NT) cbwd_y<C, TM>(w.WB[0], w.WA[0], l);
  __syncthreads();
  for (int l = stage_tid(); l < C::EX * NY * NZ; l += C::NT) cbwd_x<C, TM, ADD>(w.WA[0], out, l);
  __syncthreads();
}

// in == out is allowed: the inputs are consumed by the first stage.
template <class C, int KIND, int T0, int T1, int T2, bool ADD, typename TC>
__device__ __forceinline__ void cmass_vector(TC* const in[3], TC* const out[3], TC sign, const Work<TC>& w) {
  constexpr int NT = C::NT;
  constexpr int X0 = C::EX * C::ny(T0) * C::nz(T0), X1 = C::EX * C::ny(T1) * C::nz(T1),
                X2 = C::EX * C::ny(T2) * C::nz(T2);
  constexpr int Y0 = C::QX * C::EY * C::nz(T0), Y1 = C::QX * C::EY * C::nz(T1), Y2 = C::QX * C::EY * C::nz(T2);
  stage3<NT, X0, X1, X2>([&](int l) { cfwd_x<C, T0>(in[0], w.WA[0], l); },
                         [&](int l) { cfwd_x<C, T1>(in[1], w.WA[1], l); },
                         [&](int l) { cfwd_x<C, T2>(in[2], w.WA[2], l); });
  __syncthreads();
  stage3<NT, Y0, Y1, Y2>([&](int l) { cfwd_y<C, T0>(w.WA[0], w.WB[0], l); },
                         [&](int l) { cfwd_y<C, T1>(w.WA[1], w.WB[1], l); },
                         [&](int l) { cfwd_y<C, T2>(w.WA[2], w.WB[2], l); });
  __syncthreads();
  for (int p = stage_tid(); p < C::QX * C::QY; p += NT) cz_vector<C, KIND, T0, T1, T2>(w.WB, p, w.er, w.g, sign);
  __syncthreads();
  stage3<NT, Y0, Y1, Y2>([&](int l) { cbwd_y<C, T0>(w.WB[0], w.WA[0], l); },
                         [&](int l) { cbwd_y<C, T1>(w.WB[1], w.WA[1], l); },
                         [&](int l) { cbwd_y<C, T2>(w.WB[2], w.WA[2], l); });
  __syncthreads();
  stage3<NT, X0, X1, X2>([&](int l) { cbwd_x<C, T0, ADD>(w.WA[0], out[0], l); },
                         [&](int l) { cbwd_x<C, T1, ADD>(w.WA[1], out[1], l); },
                         [&](int l) { cbwd_x<C, T2, ADD>(w.WA[2], out[2], l); });
  __syncthreads();
}

// Scalar mass apply of kind KIND on a field of mask TM.
template <class C, int TM, int KIND, bool ADD, int FORM, typename TC>
__device__ __forceinline__ void smass(const TC* in, TC* out, TC scale, const Work<TC>& w) {
  if constexpr (FORM == FORM_CURVED) {
    cmass_scalar<C, TM, KIND, ADD>(in, out, scale, w);
  } else if constexpr (is_kron(FORM)) {
    TC* const i3[3] = {const_cast<TC*>(in), nullptr, nullptr};
    TC* const o3[3] = {out, nullptr, nullptr};
    TC* const t3[3] = {w.A, w.B, w.T2};
    const TC s3[3] = {scale, 0, 0};
    kron_cols<C, 1, TM, TM, TM, ADD, FORM == FORM_KRON_BF16>(i3, o3, s3, t3, w.er);
  } else {
    mass<C, TM, ADD, false>(in, out, scale, w.A, w.B, w.er);
  }
}

// Vector mass apply (three components of masks T0, T1, T2).  On affine
// cells the metric is diagonal and the components decouple; on curved
// cells all three reach the Gauss points before the metric mixes them.
// in == out is allowed: inputs are consumed before outputs are written.
template <class C, int KIND, int T0, int T1, int T2, bool ADD, int FORM, typename TC>
__device__ __forceinline__ void vmass(TC* const in[3], TC* const out[3], const TC sc[3], const Work<TC>& w) {
  if constexpr (FORM == FORM_CURVED) {
    cmass_vector<C, KIND, T0, T1, T2, ADD>(in, out, sc[0], w);
  } else if constexpr (is_kron(FORM)) {
    TC* const t3[3] = {w.A, w.B, w.T2};
    kron_cols<C, 3, T0, T1, T2, ADD, FORM == FORM_KRON_BF16>(in, out, sc, t3, w.er);
  } else {
    mass<C, T0, ADD, false>(in[0], out[0], sc[0], w.A, w.B, w.er);
    mass<C, T1, ADD, false>(in[1], out[1], sc[1], w.A, w.B, w.er);
    mass<C, T2, ADD, false>(in[2], out[2], sc[2], w.A, w.B, w.er);
  }
}

// 2-D vector mass (affine forms only)
template <class C, int T0, int T1, bool ADD, int FORM, typename TC>
__device__ __forceinline__ void vmass2(TC* const in[2], TC* const out[2], const TC sc[2], const Work<TC>& w) {
  if constexpr (is_kron(FORM)) {
    TC* const i3[3] = {in[0], in[1], nullptr};
    TC* const o3[3] = {out[0], out[1], nullptr};
    TC* const t3[3] = {w.A, w.B, w.T2};
    const TC s3[3] = {sc[0], sc[1], 0};
    kron_cols<C, 2, T0, T1, T1, ADD, FORM == FORM_KRON_BF16>(i3, o3, s3, t3, w.er);
  } else {
    mass<C, T0, ADD, false>(in[0], out[0], sc[0], w.A, w.B, w.er);
    mass<C, T1, ADD, false>(in[1], out[1], sc[1], w.A, w.B, w.er);
  }
}

// ---- fused MINRES step -------------------------------------------------------
// Sum over the workgroup in a fixed order (see wg_sums).
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* sh) {
  double a[1] = {v};
  wg_sums<NT, 1>(a, sh);
  return a[0];
}

// Most lattice values of one field a thread loads per layer.
template <class C, class F>
constexpr int max_per_thread() {
  int m = 1;
  for (int f = 0; f < F::NF; ++f) {
    const int k = (C::lat(F::tm[f]) + C::NT - 1) / C::NT;
    m = k > m ? k : m;
  }
  return m;
}

// ---- the kernel body -------------------------------------------------------
// (bx, by, bz) = (tile, z-chunk, right-hand side) of this workgroup.  remap:
// spread the tiles over the XCDs in contiguous runs (the launch did not).
template <class C, int PROB, int FORM, typename TV, typename TC, bool MR>
__device__ __forceinline__ void op_body(const OpParams& p, int bx, int by, int bz, TC* smem, bool remap = true) {
  using F = Fields<PROB, C::DIM>;
  using L = Layout<C, F, FORM>;
  constexpr int R = C::R;
  static_assert(FORM != FORM_CURVED || C::DIM == 3, "curved cells are 3-D");

  // XCD-aware tile order: consecutive hardware block ids go round-robin over
  // the 8 XCDs; remap so that each XCD receives a contiguous run of tiles.
  const int nt = p.tiles_x * p.tiles_y;
  int b = bx;
  if (remap && nt % 8 == 0) b = (b % 8) * (nt / 8) + b / 8;
  const int tx = b % p.tiles_x, ty = b / p.tiles_x;
  const int X0 = tx * C::BX, Y0 = ty * C::BY;
  const int rhs = bz;
  const long long voff = (long long)rhs * p.ndofs;
  const TV* __restrict__ xin = reinterpret_cast<const TV*>(p.x) + voff;
  TV* __restrict__ yout = reinterpret_cast<TV*>(p.y) + voff;
  const int gx0 = R * (X0 - 1), gy0 = R * (Y0 - 1);

  // ---- fused MINRES step: nothing to do once this rhs has converged
  double mr_acc = 0.0;
  if constexpr (MR) {
    if (p.mr.cur[rhs].done) return;
  }

  Work<TC> w;
  w.A = smem + L::A_off();
  w.B = smem + L::B_off();
  w.T2 = smem + L::T2_off();
  for (int k = 0; k < 3; ++k) w.L[k] = smem + L::L_off(k);
  if constexpr (FORM == FORM_CURVED) {
    for (int k = 0; k < 3; ++k) {
      w.WA[k] = smem + L::WA_off(k);
      w.WB[k] = smem + L::WB_off(k);
    }
    w.g.qd = static_cast<const TC*>(p.qd);
    w.g.fs = p.qfs;
    w.g.GX = C::Q * p.nel[0];
    w.g.GY = C::Q * p.nel[1];
    w.g.gx0 = C::Q * (X0 - 1);
    w.g.gy0 = C::Q * (Y0 - 1);
    w.g.gz0 = 0;
  } else {
    for (int k = 0; k < 3; ++k) w.WA[k] = w.WB[k] = nullptr;
    w.g = QGeom<TC>{};
  }
  // local element e <-> global X0 - 1 + e
  w.er = ElemRange{max(0, 1 - X0), min(C::EX, p.nel[0] - X0 + 1), max(0, 1 - Y0), min(C::EY, p.nel[1] - Y0 + 1)};

  int zfirst = 0, zbeg = 0, zend = 1;
  if constexpr (C::DIM == 3) {
    zfirst = by * p.chunk;
    zend = min(zfirst + p.chunk, p.nel[2]);
    zbeg = zfirst > 0 ? zfirst - 1 : 0;
  }

  static_for<0, F::NF>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    if constexpr (L::carries(f)) {
      TC* car = smem + L::car_off(f);
      for (int i = threadIdx.x; i < C::plane(F::tm[f]); i += C::NT) car[i] = 0;
    }
  });

  // Layout descriptors of the fields, staged in LDS: read from there in the
  // load and write stages, they stay live only within those stages instead
  // of occupying scalar registers across the layer loop (where they spilled).
  __shared__ DevComp sh_comp[F::NF];
  static_for<0, F::NF>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    if (threadIdx.x == f) sh_comp[f] = (F::sp[f] == 0 ? p.sa : p.sb).c[F::cp[f]];
  });
  __syncthreads();

  auto IN = [&](int f) { return smem + L::in_off(f); };
  auto OUT = [&](int f) { return smem + L::out_off(f); };

  // Inputs of a layer are loaded into registers one layer ahead (a thread
  // holds at most KMAX values per field), so the global loads of layer ez + 1
  // are in flight while layer ez is computed.  For workgroups of up to 512
  // threads, and for the curved form (its contraction tables are immediates,
  // which leaves the registers for it; the perturbed 96^3 degree-3 apply
  // measured 6% faster).  The wider Kronecker and Gauss-point workgroups are
  // at their register limit: there the extra registers spill to scratch
  // (measured slower).
  constexpr bool PREFETCH = C::NT <= 512 || FORM == FORM_CURVED;
  constexpr int KMAX = PREFETCH ? max_per_thread<C, F>() : 1;
  TC pre[F::NF][KMAX];
  auto prefetch = [&](int ez) {
    const int gz0 = C::DIM == 3 ? R * ez : 0;
    static_for<0, F::NF>([&](auto fc) {
      constexpr int f = decltype(fc)::value;
      constexpr int TM = F::tm[f];
      constexpr int K = (C::lat(TM) + C::NT - 1) / C::NT;
      const DevComp& cd = sh_comp[f];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * C::NT;
        TC v = 0;
        if (i < C::lat(TM)) {
          int lx, ly, lz;
          lpos<C, TM>(i, lx, ly, lz);
          int g0 = gx0 + lx - cd.start[0], g1 = gy0 + ly - cd.start[1], g2 = gz0 + lz - cd.start[2];
          if (g0 >= 0 && g0 < cd.count[0] && g1 >= 0 && g1 < cd.count[1] && g2 >= 0 && g2 < cd.count[2])
            v = static_cast<TC>(xin[cd.offset + g0 + (long long)cd.count[0] * (g1 + (long long)cd.count[1] * g2)]);
        }
        pre[f][k] = v;
      }
    });
  };
  if constexpr (PREFETCH) prefetch(zbeg);

  for (int ez = zbeg; ez < zend; ++ez) {
    const int gz0 = C::DIM == 3 ? R * ez : 0;
    // ---- stage the inputs, zero outputs (and the cell vertices when curved)
    static_for<0, F::NF>([&](auto fc) {
      constexpr int f = decltype(fc)::value;
      constexpr int TM = F::tm[f];
      TC* in = smem + L::in_off(f);
      TC* out = smem + L::out_off(f);
      if constexpr (PREFETCH) {
        constexpr int K = (C::lat(TM) + C::NT - 1) / C::NT;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int i = threadIdx.x + k * C::NT;
          if (i < C::lat(TM)) {
            in[i] = pre[f][k];
            out[i] = 0;
          }
        }
      } else {
        const DevComp& cd = sh_comp[f];
        for (int i = threadIdx.x; i < C::lat(TM); i += C::NT) {
          int lx, ly, lz;
          lpos<C, TM>(i, lx, ly, lz);
          int g0 = gx0 + lx - cd.start[0], g1 = gy0 + ly - cd.start[1], g2 = gz0 + lz - cd.start[2];
          TC v = 0;
          if (g0 >= 0 && g0 < cd.count[0] && g1 >= 0 && g1 < cd.count[1] && g2 >= 0 && g2 < cd.count[2])
            v = static_cast<TC>(xin[cd.offset + g0 + (long long)cd.count[0] * (g1 + (long long)cd.count[1] * g2)]);
          in[i] = v;
          out[i] = 0;
        }
      }
    });
    if constexpr (FORM == FORM_CURVED) w.g.gz0 = C::Q * ez;
    __syncthreads();
    if constexpr (PREFETCH) {
      if (ez + 1 < zend) prefetch(ez + 1);
    }

    if constexpr (PROB == PROB_HODGE) {
      TC* in_u[3] = {IN(1), IN(2), IN(3)};
      TC* out_u[3] = {OUT(1), OUT(2), OUT(3)};
      TC* Lb[3] = {w.L[0], w.L[1], w.L[2]};
      const TC s1[3] = {(TC)p.sc[1], (TC)p.sc[2], (TC)p.sc[3]};
      const TC s2[3] = {(TC)p.sc[4], (TC)p.sc[5], (TC)p.sc[6]};
      // -M0 sigma
      smass<C, 7, GYM_H1, true, FORM>(IN(0), OUT(0), (TC)-p.sc[0], w);
      // G^T (M1 u): v = M1 u on the closure, y_sigma(q) += sum_c v_c(q-e_c) - v_c(q)
      vmass<C, GYM_HCURL, 6, 5, 3, false, FORM>(in_u, Lb, s1, w);
      for (int i = threadIdx.x; i < C::lat(7); i += C::NT) {
        int q[3];
        lpos<C, 7>(i, q[0], q[1], q[2]);
        TC acc = 0;
        static_for<0, 3>([&](auto cc) {
          constexpr int c = decltype(cc)::value;
          constexpr int TE = 7 & ~(1 << c);
          if (q[c] >= 1) {
            int s[3] = {q[0], q[1], q[2]};
            s[c] -= 1;
            acc += Lb[c][lidx<C, TE>(s[0], s[1], s[2])];
          }
          if (q[c] < ext<C, TE>(c)) acc -= Lb[c][lidx<C, TE>(q[0], q[1], q[2])];
        });
        OUT(0)[i] += acc;
      }
      __syncthreads();
      // M1 G sigma: g_c(q) = sigma(q + e_c) - sigma(q)
      static_for<0, 3>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int TE = 7 & ~(1 << c);
        const TC* sg = IN(0);
        for (int i = threadIdx.x; i < C::lat(TE); i += C::NT) {
          int q[3];
          lpos<C, TE>(i, q[0], q[1], q[2]);
          int s[3] = {q[0], q[1], q[2]};
          s[c] += 1;
          TC g = -sg[lidx<C, 7>(q[0], q[1], q[2])];
          g += sg[lidx<C, 7>(s[0], s[1], s[2])];
          Lb[c][i] = g;
        }
      });
      __syncthreads();
      vmass<C, GYM_HCURL, 6, 5, 3, true, FORM>(Lb, out_u, s1, w);
      // C^T M2 C u: b_c(p) = a_c2(p + e_c1) - a_c2(p) - a_c1(p + e_c2) + a_c1(p)
      static_for<0, 3>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        constexpr int TF = 1 << c;
        constexpr int T1 = 7 & ~(1 << c1), T2 = 7 & ~(1 << c2);
        const TC* a1 = in_u[c1];
        const TC* a2 = in_u[c2];
        for (int i = threadIdx.x; i < C::lat(TF); i += C::NT) {
          int q[3];
          lpos<C, TF>(i, q[0], q[1], q[2]);
          int t1[3] = {q[0], q[1], q[2]}, t2[3] = {q[0], q[1], q[2]};
          t1[c1] += 1;
          t2[c2] += 1;
          TC v = a2[lidx<C, T2>(t1[0], t1[1], t1[2])];
          v -= a2[lidx<C, T2>(q[0], q[1], q[2])];
          v -= a1[lidx<C, T1>(t2[0], t2[1], t2[2])];
          v += a1[lidx<C, T1>(q[0], q[1], q[2])];
          Lb[c][i] = v;
        }
      });
      __syncthreads();
      vmass<C, GYM_HDIV, 1, 2, 4, false, FORM>(Lb, Lb, s2, w);  // z = M2 c in place
      // (C^T z)_e(q) = [z_{e1}(q - e_{e2}) - z_{e1}(q)] + [z_{e2}(q) - z_{e2}(q - e_{e1})]
      // with (e1, e2) the cyclic successors of edge component e
      static_for<0, 3>([&](auto ce) {
        constexpr int e = decltype(ce)::value;
        constexpr int e1 = (e + 1) % 3, e2 = (e + 2) % 3;
        constexpr int TE = 7 & ~(1 << e);
        constexpr int TF1 = 1 << e1, TF2 = 1 << e2;
        TC* o = out_u[e];
        for (int i = threadIdx.x; i < C::lat(TE); i += C::NT) {
          int q[3];
          lpos<C, TE>(i, q[0], q[1], q[2]);
          TC acc = 0;
          // face component e1 (nodal along e1, edge along e and e2)
          if (q[e2] >= 1) {
            int s[3] = {q[0], q[1], q[2]};
            s[e2] -= 1;
            acc += Lb[e1][lidx<C, TF1>(s[0], s[1], s[2])];
          }
          if (q[e2] < ext<C, TF1>(e2)) acc -= Lb[e1][lidx<C, TF1>(q[0], q[1], q[2])];
          // face component e2 (nodal along e2, edge along e and e1)
          if (q[e1] < ext<C, TF2>(e1)) acc += Lb[e2][lidx<C, TF2>(q[0], q[1], q[2])];
          if (q[e1] >= 1) {
            int s[3] = {q[0], q[1], q[2]};
            s[e1] -= 1;
            acc -= Lb[e2][lidx<C, TF2>(s[0], s[1], s[2])];
          }
          o[i] += acc;
        }
      });
      __syncthreads();
    } else if constexpr (PROB == PROB_POISSON) {
      constexpr int D = C::DIM;
      constexpr int NS = D;  // flux components
      TC* L1 = w.L[0];
      // M2 s
      if constexpr (D == 3) {
        TC* in_s[3] = {IN(0), IN(1), IN(2)};
        TC* out_s[3] = {OUT(0), OUT(1), OUT(2)};
        const TC s2[3] = {(TC)p.sc[0], (TC)p.sc[1], (TC)p.sc[2]};
        vmass<C, GYM_HDIV, 1, 2, 4, true, FORM>(in_s, out_s, s2, w);
      } else {
        TC* in_s[2] = {IN(0), IN(1)};
        TC* out_s[2] = {OUT(0), OUT(1)};
        const TC s2[2] = {(TC)p.sc[0], (TC)p.sc[1]};
        vmass2<C, 1, 2, true, FORM>(in_s, out_s, s2, w);
      }
      // -D^T (M3 p): y_s_c(q) += w(q) - w(q - e_c)
      smass<C, 0, GYM_L2, false, FORM>(IN(NS), L1, (TC)p.sc[3], w);
      static_for<0, NS>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int TF = F::tm[c];
        TC* o = OUT(c);
        for (int i = threadIdx.x; i < C::lat(TF); i += C::NT) {
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
      for (int i = threadIdx.x; i < C::lat(0); i += C::NT) {
        int q[3];
        lpos<C, 0>(i, q[0], q[1], q[2]);
        TC v = 0;
        static_for<0, NS>([&](auto cc) {
          constexpr int c = decltype(cc)::value;
          constexpr int TF = F::tm[c];
          const TC* s = IN(c);
          int t[3] = {q[0], q[1], q[2]};
          t[c] += 1;
          v -= s[lidx<C, TF>(q[0], q[1], q[2])];
          v += s[lidx<C, TF>(t[0], t[1], t[2])];
        });
        L1[i] = v;
      }
      __syncthreads();
      smass<C, 0, GYM_L2, true, FORM>(L1, OUT(NS), (TC)-p.sc[3], w);
    } else {
      constexpr int KIND = PROB - PROB_MASS_H1;
      if constexpr (F::NF == 1) {
        smass<C, F::tm[0], KIND, true, FORM>(IN(0), OUT(0), (TC)p.sc[0], w);
      } else if constexpr (F::NF == 3) {
        TC* in_v[3] = {IN(0), IN(1), IN(2)};
        TC* out_v[3] = {OUT(0), OUT(1), OUT(2)};
        const TC sv[3] = {(TC)p.sc[0], (TC)p.sc[1], (TC)p.sc[2]};
        vmass<C, KIND, F::tm[0], F::tm[1], F::tm[2], true, FORM>(in_v, out_v, sv, w);
      } else {
        TC* in_v[2] = {IN(0), IN(1)};
        TC* out_v[2] = {OUT(0), OUT(1)};
        const TC sv[2] = {(TC)p.sc[0], (TC)p.sc[1]};
        vmass2<C, F::tm[0], F::tm[1], true, FORM>(in_v, out_v, sv, w);
      }
    }

    // ---- carry the shared top plane to the next layer
    if constexpr (C::DIM == 3) {
      static_for<0, F::NF>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        if constexpr (L::carries(f)) {
          constexpr int PL = C::plane(F::tm[f]);
          TC* out = smem + L::out_off(f);
          TC* car = smem + L::car_off(f);
          for (int i = threadIdx.x; i < PL; i += C::NT) {
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
        const DevComp& cd = sh_comp[f];
        const TC* out = smem + L::out_off(f);
        const TC* in = smem + L::in_off(f);
        for (int i = threadIdx.x; i < C::lat(TM); i += C::NT) {
          int lx, ly, lz;
          lpos<C, TM>(i, lx, ly, lz);
          int G0 = gx0 + lx, G1 = gy0 + ly, G2 = gz0 + lz;
          bool own = G0 >= R * X0 && (G0 < R * (X0 + C::BX) || G0 == p.m[0]) && G1 >= R * Y0 &&
                     (G1 < R * (Y0 + C::BY) || G1 == p.m[1]);
          if constexpr (C::DIM == 3) own = own && (G2 < gz0 + R || G2 == p.m[2]);
          int g0 = G0 - cd.start[0], g1 = G1 - cd.start[1], g2 = G2 - cd.start[2];
          if (own && g0 >= 0 && g0 < cd.count[0] && g1 >= 0 && g1 < cd.count[1] && g2 >= 0 && g2 < cd.count[2]) {
            const long long gi = cd.offset + g0 + (long long)cd.count[0] * (g1 + (long long)cd.count[1] * g2);
            const TV ys = static_cast<TV>(out[i]);
            yout[gi] = ys;
            if constexpr (MR) mr_acc += static_cast<double>(in[i]) * static_cast<double>(ys);  // z_k . A z_k
          }
        }
      });
    }
    __syncthreads();
  }
  if constexpr (MR) {
    const double t = wg_sum<C::NT>(mr_acc, reinterpret_cast<double*>(smem));
    if (threadIdx.x == 0) p.mr.pa[(long long)rhs * nt * p.nchunks + bx + nt * by] = t;
  }
}

template <class C, int PROB, int FORM, typename TV, typename TC, bool MR>
__global__ void __launch_bounds__(C::NT) op_kernel(const OpParams p) {
  constexpr int kWords = Layout<C, Fields<PROB, C::DIM>, FORM>::total();
  static_assert(kWords * sizeof(TC) >= C::NT * sizeof(double), "LDS holds the workgroup sums");
  __shared__ __align__(16) TC smem[kWords];
  op_body<C, PROB, FORM, TV, TC, MR>(p, blockIdx.x, blockIdx.y, blockIdx.z, smem);
}

// Several right-hand sides sharing per-point data (the curved form's
// Gauss-point metrics): a 1-D grid of tiles x chunks x nrhs workgroups,
// numbered so that the nrhs workgroups of one tile and chunk run on the same
// XCD (the hardware deals block b to XCD b mod 8) and are dispatched one after
// another.  They then read the same metric values within a short time, and
// all but the first find them in that XCD's L2.  The host checks that the
// workgroup count is a multiple of 8.
template <class C, int PROB, int FORM, typename TV, typename TC, bool MR>
__global__ void __launch_bounds__(C::NT) op_kernel_rhs(const OpParams p, int nrhs) {
  __shared__ __align__(16) TC smem[Layout<C, Fields<PROB, C::DIM>, FORM>::total()];
  const int nt = p.tiles_x * p.tiles_y;
  const int per_xcd = nt * p.nchunks * nrhs / 8;
  const int slot = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);  // (tile, chunk, rhs), rhs fastest
  const int rhs = slot % nrhs, tc = slot / nrhs;
  op_body<C, PROB, FORM, TV, TC, MR>(p, tc % nt, tc / nt, rhs, smem, false);
}

// Ragged batch: one launch over the workgroups of several operators of the
// same kind and degree (different meshes and vectors).  bstart holds the
// prefix sums of the per-request workgroup counts (nreq + 1 entries).
template <class C, int PROB, int FORM, typename TV, typename TC, bool MR>
__global__ void __launch_bounds__(C::NT) op_kernel_batch(const OpParams* __restrict__ plist,
                                                       const int* __restrict__ bstart, int nreq) {
  __shared__ __align__(16) TC smem[Layout<C, Fields<PROB, C::DIM>, FORM>::total()];
  const int blk = blockIdx.x;
  int lo = 0, hi = nreq;  // bstart[lo] <= blk < bstart[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (bstart[mid] <= blk) lo = mid;
    else hi = mid;
  }
  const OpParams p = plist[lo];
  if constexpr (!MR) {
    if (p.gate && *p.gate) return;  // that request has converged: leave its vectors alone
  }
  const int local = blk - bstart[lo];
  const int nt = p.tiles_x * p.tiles_y;
  const int bx = local % nt, r2 = local / nt;
  op_body<C, PROB, FORM, TV, TC, MR>(p, bx, r2 % p.nchunks, r2 / p.nchunks, smem);
}

// ---- tile-size selection ----------------------------------------------------
// Largest square tile whose LDS footprint fits `budget` bytes (2..8 per side;
// up to 16 in 2-D).  Two budgets are compiled: the whole 160 KB of a CU (one
// workgroup per CU, least halo recomputation) and 40 KB (several workgroups
// per CU, more waves to hide LDS latency).
template <int DIM, int R, int PROB, int FORM, typename TC, int BUDGET>
struct TileSel {
  template <int B>
  static constexpr int bytes() {
    using C = Cfg<R, B, B, DIM>;
    return Layout<C, Fields<PROB, DIM>, FORM>::total() * (int)sizeof(TC);
  }
  static constexpr int B = DIM == 2 ? (bytes<16>() <= BUDGET ? 16 : (bytes<8>() <= BUDGET ? 8 : (bytes<4>() <= BUDGET ? 4 : 2)))
                           : bytes<8>() <= BUDGET ? 8
                           : bytes<6>() <= BUDGET ? 6
                           : bytes<4>() <= BUDGET ? 4
                           : bytes<3>() <= BUDGET ? 3
                           : bytes<2>() <= BUDGET ? 2
                                                  : 1;
};

// Tiles and z-chunks of one operator for tile size B; returns the number of
// workgroups (tiles x chunks x nrhs).  A chunk of c element layers costs its
// workgroup c + 1 layers (the halo layer below it is recomputed), except the
// bottom chunk.  Modes:
//   kTileWhole  whole-CU tiles, `occ` workgroups per CU (one in FP64, two
//               for some FP32 kernels): the launch runs in
//               ceil(workgroups / (occ ncu)) rounds of one chunk each, so the
//               chunk minimises rounds x (c + 1), a cost that tracks the
//               measured kernel times on MI355X.
//   kTileSmall  40 KB tiles, several workgroups per CU: about four
//               workgroups per CU, chunks of at least two layers.
//   kTileBatch  the ragged serving batch, where many requests fill the GPU
//               together: about two workgroups per CU and request, chunks of
//               at least four layers.
enum { kTileWhole = 0, kTileSmall = 1, kTileBatch = 2 };
inline int op_tiling(OpParams& p, int B, int dim, int nrhs, int ncu, int mode, int occ = 1) {
  p.tiles_x = (p.nel[0] + B - 1) / B;
  p.tiles_y = (p.nel[1] + B - 1) / B;
  const int nt = p.tiles_x * p.tiles_y;
  int nchunks = 1;
  p.chunk = 1;
  if (dim == 3) {
    const int nz = p.nel[2];
    if (mode == kTileWhole) {
      long long best = -1;
      for (int c = 1; c <= nz; ++c) {
        const int nch = (nz + c - 1) / c;
        if ((nz + nch - 1) / nch != c) continue;  // the same split as a smaller c
        const long long slots = (long long)occ * ncu;
        const long long rounds = ((long long)nt * nrhs * nch + slots - 1) / slots;
        const long long cost = rounds * (c + (nch > 1 ? 1 : 0));
        if (best < 0 || cost < best) {
          best = cost;
          p.chunk = c;
        }
      }
    } else {
      const int target = (mode == kTileSmall ? 4 : 2) * ncu;
      nchunks = (target + nt * nrhs - 1) / (nt * nrhs);
      int maxch = nz / (mode == kTileSmall ? 2 : 4);
      if (nchunks > maxch) nchunks = maxch;
      if (nchunks < 1) nchunks = 1;
      p.chunk = (nz + nchunks - 1) / nchunks;
    }
    nchunks = (nz + p.chunk - 1) / p.chunk;
  }
  p.nchunks = nchunks;
  return nt * nchunks * nrhs;
}

// Threads of a whole-CU workgroup (one per CU: its waves alone must hide the
// LDS latency).  Measured on MI355X at about 8M unknowns per operator for
// 512, 768 and 1024 threads: degree 1 has too little work per stage for more
// than 512; Gauss-point and the FP32/BF16 Kronecker contractions gain up to
// 1024; the FP64 Kronecker Hodge kernel at degree >= 3 runs out of registers
// beyond 768.  The curved kernels fit 1024 threads (at most 128 VGPRs, no
// scratch) since their tables are immediates: the perturbed 96^3 degree-3
// apply took 48.5 ms at 1024 against 53.1 ms at 768.
template <int DIM, int R, int PROB, int FORM, typename TC>
constexpr int big_threads() {
  if (DIM == 2 || PROB >= PROB_MASS_H1) return 512;
  if (R == 1) return FORM == FORM_CURVED ? 768 : 512;
  if (FORM == FORM_CURVED) return 1024;
  if (FORM == FORM_GAUSS) return 1024;
  if (FORM == FORM_KRON && std::is_same<TC, double>::value) return (PROB == PROB_HODGE && R >= 3) ? 768 : 1024;
  return R == 2 ? 768 : 1024;
}

template <int DIM, int R, int PROB, int FORM, typename TC, int BUDGET>
struct OpCfg {
  static constexpr int B = TileSel<DIM, R, PROB, FORM, TC, BUDGET>::B;
  // one workgroup per CU on the whole-CU budget: widen it to keep enough
  // waves in flight to hide LDS latency
  using C = Cfg<R, B, B, DIM, (BUDGET > 40 * 1024 ? big_threads<DIM, R, PROB, FORM, TC>() : kNTSmall)>;
};

// Workgroups of one operator kernel that fit on a CU at once (LDS, waves and
// registers), asked of the runtime once per kernel.
template <class C, int PROB, int FORM, typename TV, typename TC, bool MR>
int op_occupancy() {
  static const int occ = [] {
    int k = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, reinterpret_cast<const void*>(&op_kernel<C, PROB, FORM, TV, TC, MR>),
                                                     C::NT, 0) != hipSuccess) {
      (void)hipGetLastError();
      k = 1;
    }
    return k < 1 ? 1 : k;
  }();
  return occ;
}

template <int DIM, int R, int PROB, int FORM, typename TV, typename TC, int BUDGET, bool MR>
int launch_op_b(const OpParams& p0, int nrhs, int ncu, hipStream_t stream) {
  using OC = OpCfg<DIM, R, PROB, FORM, TC, BUDGET>;
  constexpr int B = OC::B;
  using C = typename OC::C;
  static_assert(Layout<C, Fields<PROB, DIM>, FORM>::total() * sizeof(TC) <= 160 * 1024, "LDS");
  OpParams p = p0;
  if constexpr (BUDGET > 40 * 1024) op_tiling(p, B, DIM, nrhs, ncu, kTileWhole, op_occupancy<C, PROB, FORM, TV, TC, MR>());
  else op_tiling(p, B, DIM, nrhs, ncu, kTileSmall);
  if (p0.wg_out) *p0.wg_out = p.tiles_x * p.tiles_y * p.nchunks;
  if (p0.dry) return 0;
  const long long nwg = (long long)p.tiles_x * p.tiles_y * p.nchunks * nrhs;
  if constexpr (FORM == FORM_CURVED) {
    if (nrhs > 1 && nwg % 8 == 0 && nwg < (1LL << 31)) {
      hipLaunchKernelGGL((op_kernel_rhs<C, PROB, FORM, TV, TC, MR>), dim3((unsigned)nwg), dim3(C::NT), 0, stream, p,
                         nrhs);
      return hipGetLastError() == hipSuccess ? 0 : -1;
    }
  }
  dim3 grid(p.tiles_x * p.tiles_y, p.nchunks, nrhs);
  hipLaunchKernelGGL((op_kernel<C, PROB, FORM, TV, TC, MR>), grid, dim3(C::NT), 0, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Batched launch (affine Kronecker form, small tiles, one rhs per request):
// tile each request, fill the device parameter list and prefix table, launch.
template <int DIM, int R, int PROB, typename TV, typename TC, bool MR = false>
int launch_op_batch_r(OpParams* plist_host, int* bstart_host, int nreq, OpParams* plist_dev, int* bstart_dev,
                      int ncu, hipStream_t stream) {
  constexpr int B = TileSel<DIM, R, PROB, FORM_KRON, TC, 40 * 1024>::B;
  using C = Cfg<R, B, B, DIM>;
  bstart_host[0] = 0;
  for (int i = 0; i < nreq; ++i) bstart_host[i + 1] = bstart_host[i] + op_tiling(plist_host[i], B, DIM, 1, ncu, kTileBatch);
  if (hipMemcpyAsync(plist_dev, plist_host, sizeof(OpParams) * nreq, hipMemcpyHostToDevice, stream) != hipSuccess)
    return -1;
  if (hipMemcpyAsync(bstart_dev, bstart_host, sizeof(int) * (nreq + 1), hipMemcpyHostToDevice, stream) != hipSuccess)
    return -1;
  hipLaunchKernelGGL((op_kernel_batch<C, PROB, FORM_KRON, TV, TC, MR>), dim3(bstart_host[nreq]), dim3(C::NT), 0, stream,
                     plist_dev, bstart_dev, nreq);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Tile budget 0: whole-CU tiles; 1: small tiles; 2: whole-CU tiles when their
// best chunking fills at least half of the slots they have on the GPU, small
// tiles otherwise (small meshes).
template <int DIM, int R, int PROB, int FORM, typename TV, typename TC, bool MR>
int launch_form(const OpParams& p, int nrhs, int ncu, hipStream_t stream) {
  constexpr int kBig = 160 * 1024, kSmall = 40 * 1024;
  bool large = p.tile_budget == 0;
  if (p.tile_budget == 2) {
    using OC = OpCfg<DIM, R, PROB, FORM, TC, kBig>;
    const int occ = op_occupancy<typename OC::C, PROB, FORM, TV, TC, MR>();
    OpParams q = p;
    large = 2 * op_tiling(q, OC::B, DIM, nrhs, ncu, kTileWhole, occ) >= occ * ncu;
  }
  if (large) return launch_op_b<DIM, R, PROB, FORM, TV, TC, kBig, MR>(p, nrhs, ncu, stream);
  return launch_op_b<DIM, R, PROB, FORM, TV, TC, kSmall, MR>(p, nrhs, ncu, stream);
}

template <int DIM, int R, int PROB, typename TV, typename TC, bool MR>
int launch_op(const OpParams& p, int nrhs, int ncu, hipStream_t stream) {
  if (p.curved) {
    if (p.bf16) return -2;  // bf16 contractions exist in the Kronecker form only
    if constexpr (DIM == 3) return launch_form<DIM, R, PROB, FORM_CURVED, TV, TC, MR>(p, nrhs, ncu, stream);
    return -2;
  }
  if (p.kron) {
    if constexpr (std::is_same<TC, float>::value) {
      if (p.bf16) return launch_form<DIM, R, PROB, FORM_KRON_BF16, TV, TC, MR>(p, nrhs, ncu, stream);
    }
    return launch_form<DIM, R, PROB, FORM_KRON, TV, TC, MR>(p, nrhs, ncu, stream);
  }
  if (p.bf16) return -2;  // bf16 contractions exist in the Kronecker form only
  return launch_form<DIM, R, PROB, FORM_GAUSS, TV, TC, MR>(p, nrhs, ncu, stream);
}

template <int DIM, int PROB, typename TV, typename TC, bool MR = false>
int dispatch_r(int r, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  switch (r) {
    case 1: return launch_op<DIM, 1, PROB, TV, TC, MR>(p, nrhs, ncu, s);
    case 2: return launch_op<DIM, 2, PROB, TV, TC, MR>(p, nrhs, ncu, s);
    case 3: return launch_op<DIM, 3, PROB, TV, TC, MR>(p, nrhs, ncu, s);
    case 4: return launch_op<DIM, 4, PROB, TV, TC, MR>(p, nrhs, ncu, s);
  }
  return -2;
}

// Each translation unit owns a private copy of the constant tables; the
// definitions below give every unit its own and the upload helper fills it.
static int upload_tables_unit() {
  TabSet<double> hd[4] = {}, hl[4] = {};
  TabSet<float> hf[4] = {}, hb[4] = {};
  fill_tables(hd, hl, hf, hb);
  GYM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tab_b), hb, sizeof(hb)));
  GYM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tab_d), hd, sizeof(hd)));
  GYM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tabL_d), hl, sizeof(hl)));
  GYM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tab_f), hf, sizeof(hf)));
  return 0;
}

}  // namespace gym
