// Set-up of the mixed Poisson block preconditioner (see schur.hip for the
// operator it applies).  All factors come from the 1-D element matrices of
// the same Gauss rule as the operator (q = r + 1), assembled per axis:
//   dn_a  diagonal of the nodal mass (r N_a + 1 positions),
//   de_a  diagonal of the edge mass (r N_a cells),
//   Me_a  the edge mass itself (block diagonal, r x r per element),
// with the metric constants of the box: M2's component c carries
// s2_c = h_c^2 / (h_0 h_1 h_2), M3 carries s3 = 1 / (h_0 h_1 h_2).
//   diag(M2)_c = s2_c dn_c (x) (x)_{b != c} de_b
//   D diag(M2)^-1 D^T = sum_c (1 / s2_c) T_c (x) (x)_{b != c} W_b,
//   T_a = D1 diag(dn_a)^-1 D1^T (tridiagonal, D1 the 1-D difference),
//   W_a = diag(de_a)^-1.
// Per axis the symmetric tridiagonal C_a = W_a^-1/2 T_a W_a^-1/2 = U diag(lam) U^T
// gives V_a = W_a^-1/2 U with V^T W V = 1 and V^T T V = diag(lam).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "eig.hpp"
#include "gym_internal.hpp"
#include "schur.hpp"

namespace gym {

namespace {

// 1-D element masses of degree r (nodal (r+1)^2, edge r^2), Gauss q = r + 1
void element_masses(int r, std::vector<double>& mn, std::vector<double>& me) {
  Tables1D t = make_tables(r, r + 1);
  const int q = r + 1;
  mn.assign((r + 1) * (r + 1), 0.0);
  me.assign(r * r, 0.0);
  for (int k = 0; k < q; ++k) {
    for (int i = 0; i <= r; ++i)
      for (int j = 0; j <= r; ++j) mn[i * (r + 1) + j] += t.gw[k] * t.phi[k * (r + 1) + i] * t.phi[k * (r + 1) + j];
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) me[i * r + j] += t.gw[k] * t.edge[k * r + i] * t.edge[k * r + j];
  }
}

// In-place inverse of a small SPD matrix (Gauss-Jordan; r <= 4)
bool invert_small(std::vector<double>& a, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[p * n + c])) p = r;
    if (a[p * n + c] == 0.0) return false;
    for (int j = 0; j < n; ++j) {
      std::swap(a[c * n + j], a[p * n + j]);
      std::swap(inv[c * n + j], inv[p * n + j]);
    }
    const double d = 1.0 / a[c * n + c];
    for (int j = 0; j < n; ++j) {
      a[c * n + j] *= d;
      inv[c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[r * n + j] -= f * a[c * n + j];
        inv[r * n + j] -= f * inv[c * n + j];
      }
    }
  }
  a.swap(inv);
  return true;
}

struct Axis {
  std::vector<double> dn, de, lam, Vt;  // Vt: m x m row-major, Me^-1 V
};

Axis build_axis(int r, int64_t nel) {
  std::vector<double> mn, me;
  element_masses(r, mn, me);
  const int m = (int)(r * nel);
  Axis A;
  A.dn.assign(m + 1, 0.0);
  A.de.assign(m, 0.0);
  for (int64_t e = 0; e < nel; ++e) {
    for (int i = 0; i <= r; ++i) A.dn[r * e + i] += mn[i * (r + 1) + i];
    for (int i = 0; i < r; ++i) A.de[r * e + i] = me[i * r + i];
  }
  // C = diag(sqrt de) T diag(sqrt de), T[i][i] = 1/dn_i + 1/dn_{i+1},
  // T[i][i+1] = T[i+1][i] = -1/dn_{i+1}: symmetric tridiagonal
  std::vector<double> cd(m), ce(m > 1 ? m - 1 : 1, 0.0), sq(m);
  for (int i = 0; i < m; ++i) sq[i] = std::sqrt(A.de[i]);
  for (int i = 0; i < m; ++i) {
    cd[i] = (1.0 / A.dn[i] + 1.0 / A.dn[i + 1]) * sq[i] * sq[i];
    if (i + 1 < m) ce[i] = -1.0 / A.dn[i + 1] * sq[i] * sq[i + 1];
  }
  std::vector<double> U;
  tridiag_eig(cd, ce, m, A.lam, U);
  // V = diag(sqrt de) U, then Vt = Me^-1 V block by block (Me is block
  // diagonal, one r x r block per element)
  std::vector<double> mei = me;
  invert_small(mei, r);
  A.Vt.assign((size_t)m * m, 0.0);
  for (int64_t e = 0; e < nel; ++e)
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += mei[i * r + k] * sq[r * e + k] * U[(size_t)(r * e + k) * m + j];
        A.Vt[(size_t)(r * e + i) * m + j] = s;
      }
  return A;
}

}  // namespace

int schur_build(const gym_op* op, SchurPrec* out) {
  const gym_mesh* msh = op->mesh;
  if (op->problem != GYM_MIXED_POISSON || msh->dim != 3 || msh->curved)
    return fail(GYM_E_UNSUPPORTED, "the Schur preconditioner is built for mixed Poisson on affine 3-D boxes");
  const int r = op->r;
  SchurPrec P;
  P.ns = op->na;
  P.np = op->nb;
  Axis ax[3];
  double det = 1.0;
  for (int a = 0; a < 3; ++a) {
    P.m[a] = (int)(r * msh->nel[a]);
    if (P.m[a] > 4096) return fail(GYM_E_UNSUPPORTED, "the Schur preconditioner needs at most 4096 cells per axis");
    det *= msh->h[a];
  }
  double s2[3];
  for (int a = 0; a < 3; ++a) {
    int same = -1;  // an earlier axis with the same element count has the same factors
    for (int b = 0; b < a; ++b)
      if (msh->nel[b] == msh->nel[a]) same = b;
    ax[a] = same >= 0 ? ax[same] : build_axis(r, msh->nel[a]);
    s2[a] = msh->h[a] * msh->h[a] / det;
  }
  const double s3 = 1.0 / det;
  P.scale = 1.0 / (s3 * s3);
  // 1 / diag(M2) in the canonical order of the flux block
  std::vector<double> ds;
  ds.reserve(P.ns);
  const SpaceDesc& sd = op->sa;
  for (int c = 0; c < sd.ncomp; ++c) {
    const CompDesc& cd = sd.comp[c];
    for (int64_t k = 0; k < cd.count[2]; ++k)
      for (int64_t j = 0; j < cd.count[1]; ++j)
        for (int64_t i = 0; i < cd.count[0]; ++i) {
          const int64_t p[3] = {cd.start[0] + i, cd.start[1] + j, cd.start[2] + k};
          double v = s2[c];
          for (int a = 0; a < 3; ++a) v *= a == c ? ax[a].dn[p[a]] : ax[a].de[p[a]];
          ds.push_back(1.0 / v);
        }
  }
  std::vector<double> lam;
  for (int a = 0; a < 3; ++a)
    for (double l : ax[a].lam) lam.push_back(l / s2[a]);
  // one allocation: dsinv, lam, then per axis Vt^T and Vt in FP64 and FP32
  size_t bytes = sizeof(double) * (ds.size() + lam.size());
  for (int a = 0; a < 3; ++a) bytes += 2 * (sizeof(double) + sizeof(float)) * (size_t)P.m[a] * P.m[a];
  if (int rc = [&] {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          return fail(GYM_E_OOM, "Schur preconditioner factors");
        }
        P.mem = p;
        return 0;
      }())
    return rc;
  char* q = static_cast<char*>(P.mem);
  auto put = [&](const void* src, size_t n) {
    void* dst = q;
    q += n;
    return hipMemcpy(dst, src, n, hipMemcpyHostToDevice) == hipSuccess ? dst : nullptr;
  };
  bool ok = true;
  P.dsinv = static_cast<double*>(put(ds.data(), sizeof(double) * ds.size()));
  P.lam = static_cast<double*>(put(lam.data(), sizeof(double) * lam.size()));
  ok = P.dsinv && P.lam;
  for (int a = 0; a < 3 && ok; ++a) {
    const int m = P.m[a];
    std::vector<double> F((size_t)m * m);  // Vt^T
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) F[(size_t)i * m + j] = ax[a].Vt[(size_t)j * m + i];
    std::vector<float> F32(F.begin(), F.end()), B32(ax[a].Vt.begin(), ax[a].Vt.end());
    P.fwd64[a] = static_cast<double*>(put(F.data(), sizeof(double) * F.size()));
    P.bwd64[a] = static_cast<double*>(put(ax[a].Vt.data(), sizeof(double) * F.size()));
    P.fwd32[a] = static_cast<float*>(put(F32.data(), sizeof(float) * F.size()));
    P.bwd32[a] = static_cast<float*>(put(B32.data(), sizeof(float) * F.size()));
    ok = P.fwd64[a] && P.bwd64[a] && P.fwd32[a] && P.bwd32[a];
  }
  if (!ok) {
    schur_free(&P);
    return fail(GYM_E_HIP, "upload of the Schur preconditioner factors");
  }
  *out = P;
  return 0;
}

int schur_reserve(SchurPrec* P, int nrhs, size_t elem_bytes) {
  const size_t need = 2 * (size_t)P->np * (size_t)nrhs * elem_bytes;
  if (P->work && P->work_nrhs >= nrhs && P->work_bytes >= need) return 0;
  if (P->work) (void)hipFree(P->work);
  P->work = nullptr;
  P->work_nrhs = 0;
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GYM_E_OOM, "Schur preconditioner work vectors");
  }
  P->work = p;
  P->work_nrhs = nrhs;
  P->work_bytes = need;
  return 0;
}

void schur_free(SchurPrec* P) {
  if (P->mem) (void)hipFree(P->mem);
  if (P->work) (void)hipFree(P->work);
  *P = SchurPrec{};
}

}  // namespace gym
