// SPAI-OP, the operator-probed sparse approximate inverse of M1 (paper
// section 5, eqs. SPAIOPobjective to diagonalPreconditioner), on axis-aligned
// meshes.
//
// Q1 lives on S = S(M1): in a component block, row i couples to the j with
// M1_ij != 0, a box of (2r + 1)^3 offsets of which the 1-D masses mark the
// live ones.  The unknowns q are stored row by row, one slot per box offset
// (dead slots stay zero).  The symmetric Q1 that minimises
// ||M1 Q1 - 1||_F^2 + lambda sum_k ||(M1 Q1 - 1) W_k||^2, W = P2 V, solves
// (U Q1 T + T Q1 U)_ij = R_ij on S with U = M1^2, T = 1 + lambda W W^T and
// R = M1 T + T M1.  The operator is applied matrix-free:
//   (U Q)_ij = sum_m U_im Q_mj over the m with Q_mj in the box of row m,
//   (Q U)_ij = sum_m Q_im U_mj over the box of row i,
// U_im a product of 1-D entries of M_a^2 (Kronecker structure of M1 per
// component), and the rank-n_probe parts through X = U Q W and
// Y = U Q^T W.  Jacobi-preconditioned CG solves it, started from the
// symmetrised column-wise SPAI; the operator is two box contractions with
// U's 1-D factors (rows for Q U, columns for U Q), one thread per row in the
// stencil applies.
#include "spai_op.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

#include "gym_internal.hpp"
#include "krylov.hpp"
#include "spai.hpp"

namespace gym {
namespace {

struct OpComp {
  long long off;         // first row of the block
  int n[3];              // kept positions per axis
  int wrap;              // bit a: axis a periodic (positions taken modulo n[a]; n[a] > 4r)
  double sc;             // M1 block = sc (x)_a M_a
  const double* M[3];    // n[a] x (2r + 1): M_a band
  const double* M2[3];   // n[a] x (4r + 1): (M_a^2) band
};

struct SylvParams {
  OpComp c[3];
  long long n1;
  int r;
  int np;            // probes
  const double* W;   // np x n1: P2 v_k
  const double* X;   // np x n1: U Q W  (for the current direction)
  const double* Y;   // np x n1: U Q^T W
  const double* MW;  // np x n1: M1 W
  double lam, eps;
};

__device__ __forceinline__ int comp_of(const SylvParams& p, long long g) {
  return (g >= p.c[1].off) + (g >= p.c[2].off);
}

__device__ __forceinline__ void decode(const OpComp& d, long long g, int& x, int& y, int& z) {
  const long long loc = g - d.off;
  x = (int)(loc % d.n[0]);
  const long long rest = loc / d.n[0];
  y = (int)(rest % d.n[1]);
  z = (int)(rest / d.n[1]);
}

// A position along axis a brought back into [0, n[a]) on a periodic axis
// (shifts here are at most 2r < n[a]); unchanged otherwise.
__device__ __forceinline__ int wrap_pos(const OpComp& d, int a, int v) {
  if (!((d.wrap >> a) & 1)) return v;
  const int n = d.n[a];
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

__device__ __forceinline__ long long at(const OpComp& d, int x, int y, int z) {
  x = wrap_pos(d, 0, x);
  y = wrap_pos(d, 1, y);
  z = wrap_pos(d, 2, z);
  return d.off + x + (long long)d.n[0] * (y + (long long)d.n[1] * z);
}

// every position of a periodic axis is inside
__device__ __forceinline__ bool inside(const OpComp& d, int x, int y, int z) {
  return ((d.wrap & 1) || (unsigned)x < (unsigned)d.n[0]) && ((d.wrap & 2) || (unsigned)y < (unsigned)d.n[1]) &&
         ((d.wrap & 4) || (unsigned)z < (unsigned)d.n[2]);
}

// M1_ij / sc for j = i + (dx, dy, dz) (zero off the pattern); the bands hold
// raw offsets, so on a periodic axis only the row position wraps
__device__ __forceinline__ double m1_rel(const OpComp& d, int r, int x, int y, int z, int dx, int dy, int dz) {
  const int L = 2 * r + 1;
  x = wrap_pos(d, 0, x);
  y = wrap_pos(d, 1, y);
  z = wrap_pos(d, 2, z);
  return d.M[0][(long long)x * L + dx + r] * d.M[1][(long long)y * L + dy + r] * d.M[2][(long long)z * L + dz + r];
}

// U_ij / sc^2 for j = i + (dx, dy, dz), |d_a| <= 2r
__device__ __forceinline__ double u_rel(const OpComp& d, int r, int x, int y, int z, int dx, int dy, int dz) {
  const int L2 = 4 * r + 1;
  x = wrap_pos(d, 0, x);
  y = wrap_pos(d, 1, y);
  z = wrap_pos(d, 2, z);
  return d.M2[0][(long long)x * L2 + dx + 2 * r] * d.M2[1][(long long)y * L2 + dy + 2 * r] *
         d.M2[2][(long long)z * L2 + dz + 2 * r];
}

__device__ __forceinline__ int slot(int r, int dx, int dy, int dz) {
  const int L = 2 * r + 1;
  return ((dz + r) * L + (dy + r)) * L + (dx + r);
}

// One half of A q per launch: a (2r + 1)^3-box to box contraction with the
// Kronecker factors of U, applied one axis at a time (3 (2r + 1)^4 terms per
// box instead of (2r + 1)^6).  A workgroup stages `per` boxes in LDS.
//  ROWS (Q U): for row i, (Q U)_{i, i+e'} = sum_e Q_{i, i+e} U_{i+e, i+e'};
//    writes every slot of the row: sc^2 (Q U) + the probe terms + eps q on
//    live slots, zero on dead ones.
//  columns (U Q): for column j, (U Q)_{j-e', j} = sum_e U_{j-e', j-e} Q_{j-e, j},
//    the box of column j gathered from the rows j - e; adds sc^2 (U Q) into
//    the live slot e' of row j - e'.
// Each (i, j) has one owner in either pass, so the ROWS launch followed by
// the columns launch on one stream needs no atomics.
template <int R, bool ROWS>
__global__ void __launch_bounds__(256) sylv_box(const SylvParams p, const double* __restrict__ q,
                                                double* __restrict__ out, int per) {
  constexpr int L = 2 * R + 1, L2 = 4 * R + 1, L3 = L * L * L;
  constexpr int sg = ROWS ? 1 : -1;
  extern __shared__ double sb[];
  __shared__ int pos[256][4];  // lattice position and component of each box centre
  double* g = sb;
  double* h = sb + per * L3;
  for (long long c0 = (long long)blockIdx.x * per; c0 < p.n1; c0 += (long long)gridDim.x * per) {
    const int cnt = (int)(p.n1 - c0 < per ? p.n1 - c0 : per);
    if (threadIdx.x < cnt) {
      const long long c = c0 + threadIdx.x;
      const int cc = comp_of(p, c);
      decode(p.c[cc], c, pos[threadIdx.x][0], pos[threadIdx.x][1], pos[threadIdx.x][2]);
      pos[threadIdx.x][3] = cc;
    }
    __syncthreads();
    // the box of row / column c: g(e) = Q_{c, c+e} or Q_{c-e, c}
    for (int u = threadIdx.x; u < cnt * L3; u += 256) {
      const int k = u / L3, t = u - k * L3;
      const long long c = c0 + k;
      double v = 0.0;
      if constexpr (ROWS) {
        v = q[c * L3 + t];
      } else {
        const OpComp& d = p.c[pos[k][3]];
        const int x = pos[k][0], y = pos[k][1], z = pos[k][2];
        const int mx = x - (t % L - R), my = y - ((t / L) % L - R), mz = z - (t / (L * L) - R);
        if (inside(d, mx, my, mz)) v = q[at(d, mx, my, mz) * L3 + t];
      }
      g[u] = v;
    }
    __syncthreads();
    // axis a: out(.., e'_a, ..) = sum_{e_a} U_a(c_a + sg e'_a, c_a + sg e_a) in(.., e_a, ..)
    auto pass = [&](const double* in, double* o, int a) {
      const int st = a == 0 ? 1 : a == 1 ? L : L * L;  // slot stride of axis a
      for (int u = threadIdx.x; u < cnt * L3; u += 256) {
        const int k = u / L3, t = u - k * L3;
        const OpComp& d = p.c[pos[k][3]];
        const int ca = pos[k][a];
        const int e_out = (t / st) % L - R;
        const int base = t - (e_out + R) * st;
        const int pp = ca + sg * e_out;
        const bool wa = (d.wrap >> a) & 1;
        double acc = 0.0;
        if (wa || (unsigned)pp < (unsigned)d.n[a]) {
          const double* band = d.M2[a] + (long long)wrap_pos(d, a, pp) * L2 + 2 * R;
#pragma unroll
          for (int e = -R; e <= R; ++e) {
            const int qq = ca + sg * e;
            if (wa || (unsigned)qq < (unsigned)d.n[a]) acc += band[qq - pp] * in[k * L3 + base + (e + R) * st];
          }
        }
        o[u] = acc;
      }
      __syncthreads();
    };
    pass(g, h, 0);
    pass(h, g, 1);
    pass(g, h, 2);
    for (int u = threadIdx.x; u < cnt * L3; u += 256) {
      const int k = u / L3, t = u - k * L3;
      const long long c = c0 + k;
      const OpComp& d = p.c[pos[k][3]];
      const int x = pos[k][0], y = pos[k][1], z = pos[k][2];
      const int dx = t % L - R, dy = (t / L) % L - R, dz = t / (L * L) - R;
      const double v = d.sc * d.sc * h[u];
      if constexpr (ROWS) {
        const long long idx = c * L3 + t;
        if (!inside(d, x + dx, y + dy, z + dz) || m1_rel(d, R, x, y, z, dx, dy, dz) == 0.0) {
          out[idx] = 0.0;
          continue;
        }
        const long long j = at(d, x + dx, y + dy, z + dz);
        double acc = v;
        for (int kk = 0; kk < p.np; ++kk) {
          const long long o = (long long)kk * p.n1;
          acc += p.lam * (p.X[o + c] * p.W[o + j] + p.W[o + c] * p.Y[o + j]);
        }
        out[idx] = acc + p.eps * q[idx];
      } else {
        const int ix = x - dx, iy = y - dy, iz = z - dz;  // row i = j - e'
        if (inside(d, ix, iy, iz) && m1_rel(d, R, ix, iy, iz, dx, dy, dz) != 0.0) out[at(d, ix, iy, iz) * L3 + t] += v;
      }
    }
    __syncthreads();  // h and g are refilled by the next boxes
  }
}

template <int R>
void launch_sylv(const SylvParams& p, const double* q, double* out, int ncu, hipStream_t s) {
  constexpr int L3 = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
  const int per = L3 >= 256 ? 1 : 256 / L3;
  long long nb = (p.n1 + per - 1) / per;
  if (nb > 8LL * ncu) nb = 8LL * ncu;
  const size_t lds = sizeof(double) * 2 * per * L3;
  hipLaunchKernelGGL((sylv_box<R, true>), dim3((int)nb), dim3(256), lds, s, p, q, out, per);
  hipLaunchKernelGGL((sylv_box<R, false>), dim3((int)nb), dim3(256), lds, s, p, q, out, per);
}

// out = A q on S (+ eps q)
void sylv_apply(const SylvParams& p, const double* q, double* out, int ncu, hipStream_t s) {
  switch (p.r) {
    case 1: launch_sylv<1>(p, q, out, ncu, s); break;
    case 2: launch_sylv<2>(p, q, out, ncu, s); break;
    case 3: launch_sylv<3>(p, q, out, ncu, s); break;
    default: launch_sylv<4>(p, q, out, ncu, s); break;
  }
}

// right-hand side R = M1 T + T M1 on S, and the Jacobi preconditioner
// (its inverse; 1 on dead slots, whose right-hand side is zero)
__global__ void __launch_bounds__(256) sylv_setup(const SylvParams p, double* __restrict__ rhs,
                                                  double* __restrict__ pinv) {
  const int r = p.r, L = 2 * r + 1, L3 = L * L * L;
  const long long total = p.n1 * L3;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
    const long long i = t / L3;
    const int s = (int)(t - i * L3);
    const int dx = s % L - r, dy = (s / L) % L - r, dz = s / (L * L) - r;
    const OpComp& d = p.c[comp_of(p, i)];
    int x, y, z;
    decode(d, i, x, y, z);
    const double m = m1_rel(d, r, x, y, z, dx, dy, dz);
    if (m == 0.0) {
      rhs[t] = 0.0;
      pinv[t] = 1.0;
      continue;
    }
    const long long j = at(d, x + dx, y + dy, z + dz);
    double rv = 2.0 * d.sc * m, ti = 1.0, tj = 1.0;
    for (int k = 0; k < p.np; ++k) {
      const long long o = (long long)k * p.n1;
      rv += p.lam * (p.MW[o + i] * p.W[o + j] + p.W[o + i] * p.MW[o + j]);
      ti += p.lam * p.W[o + i] * p.W[o + i];
      tj += p.lam * p.W[o + j] * p.W[o + j];
    }
    rhs[t] = rv;
    const double uii = d.sc * d.sc * u_rel(d, r, x, y, z, 0, 0, 0);
    int jx, jy, jz;
    decode(d, j, jx, jy, jz);
    const double ujj = d.sc * d.sc * u_rel(d, r, jx, jy, jz, 0, 0, 0);
    pinv[t] = 1.0 / (uii * tj + ti * ujj + p.eps);
  }
}

// The stencil applies do (2r + 1)^3 or (4r + 1)^3 terms per row: one wave per
// workgroup and one row per thread, so that a small mesh still spreads over
// every CU.
constexpr int kRowBT = 64;
int row_grid(long long n) {
  long long b = (n + kRowBT - 1) / kRowBT;
  return (int)(b > 65536 ? 65536 : b < 1 ? 1 : b);
}

// y = Q x (transpose = 0) or Q^T x (transpose = 1), Q from the slots q
__global__ void __launch_bounds__(kRowBT) box_apply(const SylvParams p, const double* __restrict__ q,
                                                 const double* __restrict__ xv, double* __restrict__ yv,
                                                 int transpose) {
  const int r = p.r, L = 2 * r + 1, L3 = L * L * L;
  for (long long i = (long long)blockIdx.x * kRowBT + threadIdx.x; i < p.n1; i += (long long)gridDim.x * kRowBT) {
    const OpComp& d = p.c[comp_of(p, i)];
    int x, y, z;
    decode(d, i, x, y, z);
    double acc = 0.0;
    for (int ez = -r; ez <= r; ++ez)
      for (int ey = -r; ey <= r; ++ey)
        for (int ex = -r; ex <= r; ++ex) {
          const int nx = x + ex, ny = y + ey, nz = z + ez;
          if (!inside(d, nx, ny, nz)) continue;
          const long long m = at(d, nx, ny, nz);
          const double c = transpose ? q[m * L3 + slot(r, -ex, -ey, -ez)] : q[i * L3 + slot(r, ex, ey, ez)];
          acc += c * xv[m];
        }
    yv[i] = acc;
  }
}

// One factor of U = M1^2 = sc^2 (M_x^2 (x) M_y^2 (x) M_z^2) per component:
// y = (M_a^2 along axis a) x, times sc^2 when `last`.  Three launches, one
// per axis, apply U with 3 (4r + 1) terms per row.
__global__ void __launch_bounds__(kRowBT) u_axis(const SylvParams p, const double* __restrict__ xv,
                                              double* __restrict__ yv, int a, int last) {
  const int r = p.r, L2 = 4 * r + 1;
  for (long long i = (long long)blockIdx.x * kRowBT + threadIdx.x; i < p.n1; i += (long long)gridDim.x * kRowBT) {
    const OpComp& d = p.c[comp_of(p, i)];
    int xyz[3];
    decode(d, i, xyz[0], xyz[1], xyz[2]);
    const int pa = a == 0 ? xyz[0] : a == 1 ? xyz[1] : xyz[2];
    const int na = d.n[a];
    const bool wa = (d.wrap >> a) & 1;
    const long long st = a == 0 ? 1 : a == 1 ? (long long)d.n[0] : (long long)d.n[0] * d.n[1];
    const double* band = d.M2[a] + (long long)pa * L2 + 2 * r;
    double acc = 0.0;
    for (int k = -2 * r; k <= 2 * r; ++k)
      if (wa || (unsigned)(pa + k) < (unsigned)na) acc += band[k] * xv[i + (long long)(wrap_pos(d, a, pa + k) - pa) * st];
    yv[i] = last ? d.sc * d.sc * acc : acc;
  }
}

// the symmetrised column-wise SPAI written into the slots (the warm start)
__global__ void __launch_bounds__(256) spai_to_slots(const SylvParams p, const SpaiParams sp, double* __restrict__ q) {
  const int r = p.r, L = 2 * r + 1, L3 = L * L * L;
  const long long total = p.n1 * L3;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
    const long long i = t / L3;
    const int s = (int)(t - i * L3);
    const int dx = s % L - r, dy = (s / L) % L - r, dz = s / (L * L) - r;
    const int c = comp_of(p, i);
    const OpComp& d = p.c[c];
    int x, y, z;
    decode(d, i, x, y, z);
    const SpaiComp& a = sp.c[c];
    double v = 0.0;
    if (inside(d, x + dx, y + dy, z + dz) && m1_rel(d, r, x, y, z, dx, dy, dz) != 0.0) {
      v = a.band[0][0][(long long)x * L + dx + r] * a.band[0][1][(long long)y * L + dy + r] *
              a.band[0][2][(long long)z * L + dz + r] +
          a.band[1][0][(long long)x * L + dx + r] * a.band[1][1][(long long)y * L + dy + r] *
              a.band[1][2][(long long)z * L + dz + r];
      v *= a.scale;
    }
    q[t] = v;
  }
}

}  // namespace

int spai_op_build(const gym_space* s1, const double* Wdev, const double* MWdev, int np, double lam, double rtol,
                  int maxit, int ncu, hipStream_t s, SpaiOpQ1* out, int* iters, double* rel_res) {
  const SpaceDesc& sd = s1->desc;
  const gym_mesh* m = s1->mesh;
  if (sd.kind != GYM_HCURL || sd.ncomp != m->dim) return fail(GYM_E_ARG, "SPAI-OP: Lambda^1 only");
  const int r = sd.r, L = 2 * r + 1, L2 = 4 * r + 1, L3 = L * L * L;
  for (int a = 0; a < sd.dim; ++a)
    if (((sd.periodic >> a) & 1) && sd.m[a] <= 4 * r)
      return fail(GYM_E_UNSUPPORTED, "SPAI-OP: a periodic axis needs more than 4r positions");
  const long long n1 = sd.ndofs, nq = n1 * L3;
  const LumpedTables lt = lumped_tables_host(s1);
  // 1-D bands of M_a and M_a^2 per component and axis
  std::vector<double> host;
  size_t offM[3][3] = {}, offM2[3][3] = {};
  for (int c = 0; c < sd.ncomp; ++c)
    for (int a = 0; a < 3; ++a) {
      const CompDesc& cd = sd.comp[c];
      const int cnt = (int)cd.count[a];
      const bool per = (sd.periodic >> a) & 1;
      std::vector<double> A, A2((size_t)cnt * L2, 0.0);
      if (a >= sd.dim) {  // no such axis: the identity (one position)
        A.assign(L, 0.0);
        A[r] = 1.0;
        A2[2 * r] = 1.0;
      } else {
        A = mass1d_band(r, (int)m->nel[a], (cd.nodal_mask >> a) & 1, (int)cd.start[a], cnt, per);
        for (int i = 0; i < cnt; ++i)
          for (int k = -r; k <= r; ++k) {
            int mm = i + k;
            if (per) mm = mm < 0 ? mm + cnt : (mm >= cnt ? mm - cnt : mm);
            else if (mm < 0 || mm >= cnt) continue;
            for (int k2 = -r; k2 <= r; ++k2) {
              // raw offset k + k2 (on a periodic axis, cnt > 4r keeps them apart)
              if (!per && (mm + k2 < 0 || mm + k2 >= cnt)) continue;
              A2[(size_t)i * L2 + (k + k2 + 2 * r)] += A[(size_t)i * L + k + r] * A[(size_t)mm * L + k2 + r];
            }
          }
      }
      offM[c][a] = host.size();
      host.insert(host.end(), A.begin(), A.end());
      offM2[c][a] = host.size();
      host.insert(host.end(), A2.begin(), A2.end());
    }
  std::vector<void*> pool;
  auto alloc = [&](long long cnt) -> double* {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(double) * cnt) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    pool.push_back(p);
    return (double*)p;
  };
  auto release = [&](bool keep_first) {
    for (size_t i = keep_first ? 2 : 0; i < pool.size(); ++i) (void)hipFree(pool[i]);
  };
  // the first two allocations (tables, the solution q) outlive the call
  double* tab = alloc((long long)host.size());
  double* q = alloc(nq);
  double* rv = alloc(2 * nq);  // r, then z = Pinv r
  double* pv = alloc(nq);
  double* ap = alloc(nq);
  double* pinv = alloc(nq);
  double* X = alloc(std::max(1, np) * n1);
  double* Y = alloc(std::max(1, np) * n1);
  double* tmp = alloc(n1);
  double* tmp2 = alloc(n1);
  const int nb = vec_grid(nq, ncu);
  double* gw = alloc(2LL * nb + 2);  // dot-product partials and results
  if (!tab || !q || !rv || !pv || !ap || !pinv || !X || !Y || !tmp || !tmp2 || !gw) {
    release(false);
    return fail(GYM_E_OOM, "SPAI-OP: device allocation failed");
  }
  if (hipMemcpy(tab, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    release(false);
    return fail(GYM_E_HIP, "SPAI-OP: upload failed");
  }
  SylvParams P{};
  double dmax = 0.0;  // largest diagonal of U, for the Tikhonov shift
  for (int c = 0; c < 3; ++c) {
    OpComp& d = P.c[c];
    if (c >= sd.ncomp) {  // 2-D: no third component (never selected)
      d.off = n1;
      for (int a = 0; a < 3; ++a) {
        d.n[a] = 1;
        d.M[a] = tab + offM[0][a];
        d.M2[a] = tab + offM2[0][a];
      }
      continue;
    }
    d.off = sd.comp[c].offset;
    d.wrap = sd.periodic;
    for (int a = 0; a < 3; ++a) {
      d.n[a] = (int)sd.comp[c].count[a];
      d.M[a] = tab + offM[c][a];
      d.M2[a] = tab + offM2[c][a];
    }
    d.sc = lt.sc[c];
    double u = d.sc * d.sc;
    for (int a = 0; a < 3; ++a) {
      double mx = 0.0;
      for (int i = 0; i < d.n[a]; ++i) mx = std::max(mx, host[offM2[c][a] + (size_t)i * L2 + 2 * r]);
      u *= mx;
    }
    dmax = std::max(dmax, u);
  }
  P.n1 = n1;
  P.r = r;
  P.np = np;
  P.W = Wdev;
  P.MW = MWdev;
  P.X = X;
  P.Y = Y;
  P.lam = lam;
  P.eps = 1e-12 * dmax;
  const int nbr = row_grid(n1);
  // out = U t, axis by axis: t -> tmp2 -> t -> out (t is overwritten)
  auto u_apply = [&](double* t, double* out) {
    hipLaunchKernelGGL(u_axis, dim3(nbr), dim3(kRowBT), 0, s, P, t, tmp2, 0, 0);
    hipLaunchKernelGGL(u_axis, dim3(nbr), dim3(kRowBT), 0, s, P, tmp2, t, 1, 0);
    hipLaunchKernelGGL(u_axis, dim3(nbr), dim3(kRowBT), 0, s, P, t, out, 2, 1);
  };
  // A v for a slot vector v: X = U V W, Y = U V^T W, then the Sylvester operator
  auto apply = [&](const double* v, double* out) {
    for (int k = 0; k < np; ++k) {
      double* xk = X + (long long)k * n1;
      double* yk = Y + (long long)k * n1;
      hipLaunchKernelGGL(box_apply, dim3(nbr), dim3(kRowBT), 0, s, P, v, Wdev + (long long)k * n1, tmp, 0);
      u_apply(tmp, xk);
      hipLaunchKernelGGL(box_apply, dim3(nbr), dim3(kRowBT), 0, s, P, v, Wdev + (long long)k * n1, tmp, 1);
      u_apply(tmp, yk);
    }
    sylv_apply(P, v, out, ncu, s);
  };
  // dot products a1 . b1 (and a2 . b2): deterministic two-stage sums into the
  // work buffer, one copy to the host
  auto dot2 = [&](const double* a1, const double* b1, const double* a2, const double* b2, double* res) {
    double* part = gw;
    double* dres = gw + 2LL * nb;
    launch_norm2(a1, b1, nq, 1, nb, 2, part, dres, s);
    if (a2) launch_norm2(a2, b2, nq, 1, nb, 2, part + nb, dres + 1, s);
    if (hipMemcpyAsync(res, dres, sizeof(double) * (a2 ? 2 : 1), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    return hipStreamSynchronize(s) != hipSuccess ? -1 : 0;
  };
  auto dot = [&](const double* a, const double* b, double* res) { return dot2(a, b, nullptr, nullptr, res); };
  // rhs into pv for now (pv is free until the first direction)
  hipLaunchKernelGGL(sylv_setup, dim3(nb), dim3(256), 0, s, P, pv, pinv);
  SpaiParams spp{};
  double* spmem = nullptr;
  if (int rc = build_spai_q1(s1, 1, &spp, &spmem)) {
    release(false);
    return rc;
  }
  hipLaunchKernelGGL(spai_to_slots, dim3(nb), dim3(256), 0, s, P, spp, q);
  // r = b - A q
  apply(q, ap);
  launch_axpy_diag(rv, 0.0, 1.0, nullptr, pv, nq, nb, s);
  launch_axpy_diag(rv, 1.0, -1.0, nullptr, ap, nq, nb, s);
  double* zv = rv + nq;
  double bn2 = 0.0, rrz[2] = {0.0, 0.0};
  int status = 0, it = 0;
  if (dot(pv, pv, &bn2)) status = -1;
  // z = Pinv r, p = z
  launch_axpy_diag(zv, 0.0, 1.0, pinv, rv, nq, nb, s);
  launch_axpy_diag(pv, 0.0, 1.0, nullptr, zv, nq, nb, s);
  if (!status && dot2(rv, rv, zv, rv, rrz)) status = -1;
  double rz = rrz[1];
  const double bn = std::sqrt(bn2);
  double rel = bn > 0 ? std::sqrt(rrz[0]) / bn : 0.0;
  while (!status && rel > rtol && it < maxit) {
    apply(pv, ap);
    double pap = 0.0;
    if (dot(pv, ap, &pap)) {
      status = -1;
      break;
    }
    if (!(pap > 0)) {
      status = fail(GYM_E_BREAKDOWN, "SPAI-OP: the Sylvester operator is not positive definite");
      break;
    }
    const double al = rz / pap;
    launch_axpy_diag(q, 1.0, al, nullptr, pv, nq, nb, s);
    launch_axpy_diag(rv, 1.0, -al, nullptr, ap, nq, nb, s);
    ++it;
    // z = Pinv r; r . r and r . z with one host round trip; p = z + beta p
    launch_axpy_diag(zv, 0.0, 1.0, pinv, rv, nq, nb, s);
    if (dot2(rv, rv, zv, rv, rrz)) {
      status = -1;
      break;
    }
    rel = std::sqrt(rrz[0]) / bn;
    const double rzn = rrz[1];
    launch_axpy_diag(pv, rzn / rz, 1.0, nullptr, zv, nq, nb, s);
    rz = rzn;
  }
  (void)hipFree(spmem);
  if (status == -1) status = hip_fail(hipGetLastError(), "SPAI-OP");
  if (status) {
    release(false);
    return status;
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    release(false);
    return hip_fail(hipGetLastError(), "SPAI-OP");
  }
  release(true);
  out->params_tab = tab;
  out->q = q;
  out->r = r;
  out->n1 = n1;
  out->wrap = sd.periodic;
  for (int c = 0; c < 3; ++c) {
    out->off[c] = P.c[c].off;
    for (int a = 0; a < 3; ++a) {
      out->n[c][a] = P.c[c].n[a];
      out->M[c][a] = P.c[c].M[a];
      out->M2[c][a] = P.c[c].M2[a];
    }
    out->sc[c] = P.c[c].sc;
  }
  *iters = it;
  *rel_res = rel;
  return rel <= rtol ? 0 : GYM_W_NOT_CONVERGED;
}

void launch_spai_op_apply(const SpaiOpQ1& Q, const double* x, double* y, int ncu, hipStream_t s) {
  SylvParams P{};
  for (int c = 0; c < 3; ++c) {
    P.c[c].off = Q.off[c];
    P.c[c].wrap = Q.off[c] < Q.n1 ? Q.wrap : 0;
    for (int a = 0; a < 3; ++a) {
      P.c[c].n[a] = Q.n[c][a];
      P.c[c].M[a] = Q.M[c][a];
      P.c[c].M2[a] = Q.M2[c][a];
    }
    P.c[c].sc = Q.sc[c];
  }
  P.n1 = Q.n1;
  P.r = Q.r;
  hipLaunchKernelGGL(box_apply, dim3(row_grid(Q.n1)), dim3(kRowBT), 0, s, P, Q.q, x, y, 0);
}

void spai_op_free(SpaiOpQ1* Q) {
  if (Q->q) (void)hipFree(Q->q);
  if (Q->params_tab) (void)hipFree(Q->params_tab);
  Q->q = nullptr;
  Q->params_tab = nullptr;
}

}  // namespace gym
