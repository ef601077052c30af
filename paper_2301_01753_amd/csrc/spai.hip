// Sparse approximate inverse Q1 of M1 on axis-aligned meshes (paper section
// 5): host construction from 1-D factors, and the device apply.
#include "spai.hpp"

#include <cmath>

#include "gym_internal.hpp"
#include "krylov.hpp"

namespace gym {

// Assembled 1-D mass of nel elements of degree r (reference element: the
// spacing sits in the metric constant), nodal (r nel + 1) or edge (r nel),
// restricted to [start, start + count): row-major dense band of half width
// r, A[i][k + r] = A_{i, i+k}.
std::vector<double> mass1d_band(int r, int nel, bool nodal, int start, int count) {
  const Tables1D t = make_tables(r, r + 1);
  const int nb = nodal ? r + 1 : r;
  std::vector<double> el((size_t)nb * nb, 0.0);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j)
      for (int k = 0; k <= r; ++k) {
        const double fi = nodal ? t.phi[k * (r + 1) + i] : t.edge[k * r + i];
        const double fj = nodal ? t.phi[k * (r + 1) + j] : t.edge[k * r + j];
        el[(size_t)i * nb + j] += t.gw[k] * fi * fj;
      }
  const int L = 2 * r + 1;
  std::vector<double> band((size_t)count * L, 0.0);
  for (int e = 0; e < nel; ++e)
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        const int gi = r * e + i - start, gj = r * e + j - start;
        if (gi < 0 || gi >= count || gj < 0 || gj >= count) continue;
        band[(size_t)gi * L + (gj - gi + r)] += el[(size_t)i * nb + j];
      }
  return band;
}

namespace {

// 1-D SPAI of the banded symmetric A (count x count, half width r): column l
// minimises || A[:, I_l] q - e_l ||_2 over its pattern I_l ({l}, or the
// nonzero rows of A's column l), by its normal equations (a Cholesky solve of
// at most 2r + 1 unknowns).  Returns the bands of Q and of Q^T (half width r).
void spai1d(const std::vector<double>& A, int count, int r, int pattern, std::vector<double>& Qb,
            std::vector<double>& QTb) {
  const int L = 2 * r + 1;
  auto a = [&](int i, int j) -> double {
    if (i < 0 || j < 0 || i >= count || j >= count || std::abs(i - j) > r) return 0.0;
    return A[(size_t)i * L + (j - i + r)];
  };
  Qb.assign((size_t)count * L, 0.0);
  QTb.assign((size_t)count * L, 0.0);
  for (int l = 0; l < count; ++l) {
    std::vector<int> I;
    if (pattern == 0) I.push_back(l);
    else
      for (int i = l - r; i <= l + r; ++i)
        if (a(i, l) != 0.0) I.push_back(i);
    const int p = (int)I.size();
    // G = A[:, I]^T A[:, I], b = A[:, I]^T e_l (rows of A[:, I] lie in l - 2r .. l + 2r)
    std::vector<double> G((size_t)p * p, 0.0), b(p, 0.0);
    for (int u = 0; u < p; ++u) {
      b[u] = a(l, I[u]);
      for (int v = 0; v < p; ++v) {
        double s = 0.0;
        for (int row = l - 2 * r; row <= l + 2 * r; ++row) s += a(row, I[u]) * a(row, I[v]);
        G[(size_t)u * p + v] = s;
      }
    }
    // Cholesky solve
    for (int j = 0; j < p; ++j) {
      double d = G[(size_t)j * p + j];
      for (int k = 0; k < j; ++k) d -= G[(size_t)j * p + k] * G[(size_t)j * p + k];
      d = std::sqrt(d);
      G[(size_t)j * p + j] = d;
      for (int i = j + 1; i < p; ++i) {
        double v = G[(size_t)i * p + j];
        for (int k = 0; k < j; ++k) v -= G[(size_t)i * p + k] * G[(size_t)j * p + k];
        G[(size_t)i * p + j] = v / d;
      }
    }
    std::vector<double> z(p), q(p);
    for (int i = 0; i < p; ++i) {
      double v = b[i];
      for (int k = 0; k < i; ++k) v -= G[(size_t)i * p + k] * z[k];
      z[i] = v / G[(size_t)i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {
      double v = z[i];
      for (int k = i + 1; k < p; ++k) v -= G[(size_t)k * p + i] * q[k];
      q[i] = v / G[(size_t)i * p + i];
    }
    for (int u = 0; u < p; ++u) {
      const int i = I[u];  // Q_{i, l} = q[u]
      Qb[(size_t)i * L + (l - i + r)] = q[u];
      QTb[(size_t)l * L + (i - l + r)] = q[u];
    }
  }
}

// One 1-D factor of a Kronecker term of Q1: y = (Q_a or Q_a^T along axis a) x
// over every block; `last` finishes the second term: y = scale (y + acc).
__global__ void __launch_bounds__(256) spai_axis_kernel(const SpaiParams p, int t, int a, int last,
                                                        const double* __restrict__ x, double* __restrict__ y) {
  for (long long g = (long long)blockIdx.x * 256 + threadIdx.x; g < p.n; g += (long long)gridDim.x * 256) {
    const int c = (g >= p.c[1].offset) + (g >= p.c[2].offset);
    const SpaiComp& d = p.c[c];
    // 32-bit position arithmetic: a block holds fewer than 2^31 unknowns
    const unsigned loc = (unsigned)(g - d.offset);
    const unsigned c0 = (unsigned)d.count[0], plane = c0 * (unsigned)d.count[1];
    const int pos = a == 0 ? (int)(loc % c0) : a == 1 ? (int)((loc / c0) % (unsigned)d.count[1]) : (int)(loc / plane);
    const long long st = a == 0 ? 1 : a == 1 ? (long long)c0 : (long long)plane;
    const int w = d.w, L = 2 * w + 1;
    const double* __restrict__ band = d.band[t][a] + (long long)pos * L + w;
    double acc = 0.0;
    for (int k = -w; k <= w; ++k)
      if ((unsigned)(pos + k) < (unsigned)d.count[a]) acc += band[k] * x[g + k * st];
    y[g] = last ? d.scale * (y[g] + acc) : acc;
  }
}

}  // namespace

int build_spai_q1(const gym_space* s1, int pattern, SpaiParams* out, double** mem) {
  const SpaceDesc& sd = s1->desc;
  const gym_mesh* m = s1->mesh;
  if (sd.ncomp != 3 || m->dim != 3) return fail(GYM_E_ARG, "SPAI Q1: 3-D Lambda^1 only");
  if (sd.ndofs >= (1LL << 31)) return fail(GYM_E_ARG, "SPAI Q1: more than 2^31 unknowns");
  const int r = sd.r;
  const LumpedTables lt = lumped_tables_host(s1);  // sc[c]: the metric constants
  std::vector<double> host;
  size_t off[3][2][3];
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a) {
      const CompDesc& cd = sd.comp[c];
      const bool nodal = (cd.nodal_mask >> a) & 1;
      const std::vector<double> A = mass1d_band(r, (int)m->nel[a], nodal, (int)cd.start[a], (int)cd.count[a]);
      std::vector<double> Qb, QTb;
      spai1d(A, (int)cd.count[a], r, pattern, Qb, QTb);
      off[c][0][a] = host.size();
      host.insert(host.end(), Qb.begin(), Qb.end());
      off[c][1][a] = host.size();
      host.insert(host.end(), QTb.begin(), QTb.end());
    }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(double) * (host.size() + 2 * (size_t)sd.ndofs)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GYM_E_OOM, "SPAI Q1: device allocation failed");
  }
  if (hipMemcpy(p, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p);
    return fail(GYM_E_HIP, "SPAI Q1: upload failed");
  }
  double* d = (double*)p;
  for (int c = 0; c < 3; ++c) {
    SpaiComp& sc = out->c[c];
    sc.offset = sd.comp[c].offset;
    for (int a = 0; a < 3; ++a) sc.count[a] = (int)sd.comp[c].count[a];
    sc.w = r;
    sc.scale = 0.5 / lt.sc[c];
    for (int t = 0; t < 2; ++t)
      for (int a = 0; a < 3; ++a) sc.band[t][a] = d + off[c][t][a];
  }
  out->n = sd.ndofs;
  out->tmp[0] = d + host.size();
  out->tmp[1] = d + host.size() + sd.ndofs;
  *mem = d;
  return 0;
}

void launch_spai_apply(const SpaiParams& p, const double* x, double* y, int nb, hipStream_t s) {
  // one row per thread: each pass has a single load chain per row, so the
  // loads in flight come from the number of resident waves
  const long long rows = (p.n + 255) / 256;
  if (rows > nb) nb = (int)(rows < (1LL << 20) ? rows : (1LL << 20));
  for (int t = 0; t < 2; ++t) {  // Q_x (x) Q_y (x) Q_z, then the transposed term
    hipLaunchKernelGGL(spai_axis_kernel, dim3(nb), dim3(256), 0, s, p, t, 0, 0, x, p.tmp[0]);
    hipLaunchKernelGGL(spai_axis_kernel, dim3(nb), dim3(256), 0, s, p, t, 1, 0, (const double*)p.tmp[0], p.tmp[1]);
    hipLaunchKernelGGL(spai_axis_kernel, dim3(nb), dim3(256), 0, s, p, t, 2, t, (const double*)p.tmp[1], y);
  }
}

}  // namespace gym
