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
std::vector<double> mass1d_band(int r, int nel, bool nodal, int start, int count, bool periodic) {
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
        if (periodic) {
          const int gi = (r * e + i) % count;
          band[(size_t)gi * L + (j - i + r)] += el[(size_t)i * nb + j];
          continue;
        }
        const int gi = r * e + i - start, gj = r * e + j - start;
        if (gi < 0 || gi >= count || gj < 0 || gj >= count) continue;
        band[(size_t)gi * L + (gj - gi + r)] += el[(size_t)i * nb + j];
      }
  return band;
}

void mass1d_diag_rowsum(int r, int nel, bool nodal, int start, int count, bool periodic, std::vector<double>& diag,
                        std::vector<double>& rowsum) {
  const std::vector<double> b = mass1d_band(r, nel, nodal, start, count, periodic);
  const int L = 2 * r + 1;
  diag.assign(count, 0.0);
  rowsum.assign(count, 0.0);
  for (int i = 0; i < count; ++i)
    for (int k = -r; k <= r; ++k) {
      const double v = b[(size_t)i * L + k + r];
      rowsum[i] += v;
      if (periodic ? ((k % count) + count) % count == 0 : k == 0) diag[i] += v;
    }
}

namespace {

// Solution of the symmetric positive definite system G q = b (p unknowns,
// G row-major) by Cholesky.
std::vector<double> spd_solve(std::vector<double> G, const std::vector<double>& b, int p) {
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
  return q;
}

// 1-D SPAI of the banded symmetric A (count x count, half width r): column l
// minimises || A[:, I_l] q - e_l ||_2 over its pattern I_l ({l}, or the
// nonzero rows of A's column l), by its normal equations (a Cholesky solve of
// at most 2r + 1 unknowns).  Returns the bands of Q and of Q^T (half width r).
void spai1d(const std::vector<double>& A, int count, int r, int pattern, std::vector<double>& Qb,
            std::vector<double>& QTb, bool periodic = false) {
  const int L = 2 * r + 1;
  if (periodic) {
    // the periodic matrix as a dense one (entries that wrap onto the same
    // column summed), the column-wise least squares on it, and the result
    // back in band form (raw offsets |k| <= r, one of them per column)
    std::vector<double> D((size_t)count * count, 0.0);
    for (int i = 0; i < count; ++i)
      for (int k = -r; k <= r; ++k) D[(size_t)i * count + (((i + k) % count) + count) % count] += A[(size_t)i * L + k + r];
    Qb.assign((size_t)count * L, 0.0);
    QTb.assign((size_t)count * L, 0.0);
    for (int l = 0; l < count; ++l) {
      std::vector<int> I;
      if (pattern == 0) I.push_back(l);
      else
        for (int i = 0; i < count; ++i)
          if (D[(size_t)i * count + l] != 0.0) I.push_back(i);
      const int p = (int)I.size();
      std::vector<double> G((size_t)p * p, 0.0), b(p, 0.0);
      for (int u = 0; u < p; ++u) {
        b[u] = D[(size_t)l * count + I[u]];
        for (int v = 0; v < p; ++v) {
          double s = 0.0;
          for (int row = 0; row < count; ++row) s += D[(size_t)row * count + I[u]] * D[(size_t)row * count + I[v]];
          G[(size_t)u * p + v] = s;
        }
      }
      std::vector<double> q = spd_solve(G, b, p);
      for (int u = 0; u < p; ++u) {
        const int i = I[u];  // Q_{i, l} = q[u]
        int kq = -r;         // an offset of row i that reaches column l
        while (kq <= r && (((i + kq) % count) + count) % count != l) ++kq;
        int kt = -r;         // an offset of row l that reaches column i
        while (kt <= r && (((l + kt) % count) + count) % count != i) ++kt;
        Qb[(size_t)i * L + kq + r] += q[u];
        QTb[(size_t)l * L + kt + r] += q[u];
      }
    }
    return;
  }
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
    const std::vector<double> q = spd_solve(G, b, p);
    for (int u = 0; u < p; ++u) {
      const int i = I[u];  // Q_{i, l} = q[u]
      Qb[(size_t)i * L + (l - i + r)] = q[u];
      QTb[(size_t)l * L + (i - l + r)] = q[u];
    }
  }
}

// One 1-D factor of a Kronecker term: y = (Q_a or Q_a^T along axis a) x over
// every block.  mode 0: y = acc; 1 (closing the second of two terms):
// y = scale (y + acc); 2 (closing a single term): y = scale acc.
__global__ void __launch_bounds__(256) spai_axis_kernel(const SpaiParams p, int t, int a, int mode,
                                                        const double* __restrict__ x, double* __restrict__ y) {
  for (long long g = (long long)blockIdx.x * 256 + threadIdx.x; g < p.n; g += (long long)gridDim.x * 256) {
    const int c = (g >= p.c[1].offset) + (g >= p.c[2].offset);
    const SpaiComp& d = p.c[c];
    // 32-bit position arithmetic: a block holds fewer than 2^31 unknowns
    const unsigned loc = (unsigned)(g - d.offset);
    const unsigned c0 = (unsigned)d.count[0], plane = c0 * (unsigned)d.count[1];
    const int pos = a == 0 ? (int)(loc % c0) : a == 1 ? (int)((loc / c0) % (unsigned)d.count[1]) : (int)(loc / plane);
    const long long st = a == 0 ? 1 : a == 1 ? (long long)c0 : (long long)plane;
    const int w = d.w, L = 2 * w + 1, cnt = d.count[a];
    const double* __restrict__ band = d.band[t][a] + (long long)pos * L + w;
    double acc = 0.0;
    if ((d.wrap >> a) & 1) {
      for (int k = -w; k <= w; ++k) {
        const int q = ((pos + k) % cnt + cnt) % cnt;
        acc += band[k] * x[g + (long long)(q - pos) * st];
      }
    } else {
      for (int k = -w; k <= w; ++k)
        if ((unsigned)(pos + k) < (unsigned)cnt) acc += band[k] * x[g + k * st];
    }
    y[g] = mode == 0 ? acc : (mode == 1 ? d.scale * (y[g] + acc) : d.scale * acc);
  }
}

// 1-D band of the identity (axes beyond the mesh dimension: one position)
std::vector<double> identity_band(int count, int w) {
  std::vector<double> b((size_t)count * (2 * w + 1), 0.0);
  for (int i = 0; i < count; ++i) b[(size_t)i * (2 * w + 1) + w] = 1.0;
  return b;
}

// Upload the bands (and two n-vectors of scratch) and fill the component
// descriptors.  bands[c][t][a] for the first ncomp components.
int upload_bands(const SpaceDesc& sd, const std::vector<double> (&bands)[3][2][3], int terms, const double* scale,
                 SpaiParams* out, double** mem, const char* what) {
  std::vector<double> host;
  size_t off[3][2][3] = {};
  for (int c = 0; c < sd.ncomp; ++c)
    for (int t = 0; t < terms; ++t)
      for (int a = 0; a < 3; ++a) {
        off[c][t][a] = host.size();
        host.insert(host.end(), bands[c][t][a].begin(), bands[c][t][a].end());
      }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(double) * (host.size() + 2 * (size_t)sd.ndofs)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GYM_E_OOM, std::string(what) + ": device allocation failed");
  }
  if (hipMemcpy(p, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p);
    return fail(GYM_E_HIP, std::string(what) + ": upload failed");
  }
  double* d = (double*)p;
  for (int c = 0; c < 3; ++c) {
    SpaiComp& sc = out->c[c];
    sc = SpaiComp{};
    if (c >= sd.ncomp) {
      sc.offset = sd.ndofs;  // never selected
      continue;
    }
    sc.offset = sd.comp[c].offset;
    for (int a = 0; a < 3; ++a) sc.count[a] = (int)sd.comp[c].count[a];
    sc.w = sd.r;
    sc.wrap = sd.periodic;
    sc.scale = scale[c];
    for (int t = 0; t < terms; ++t)
      for (int a = 0; a < 3; ++a) sc.band[t][a] = d + off[c][t][a];
  }
  out->n = sd.ndofs;
  out->terms = terms;
  out->tmp[0] = d + host.size();
  out->tmp[1] = d + host.size() + sd.ndofs;
  *mem = d;
  return 0;
}

}  // namespace

int build_spai_q1(const gym_space* s1, int pattern, SpaiParams* out, double** mem) {
  const SpaceDesc& sd = s1->desc;
  const gym_mesh* m = s1->mesh;
  if (sd.kind != GYM_HCURL || sd.ncomp != m->dim) return fail(GYM_E_ARG, "SPAI Q1: Lambda^1 only");
  if (sd.ndofs >= (1LL << 31)) return fail(GYM_E_ARG, "SPAI Q1: more than 2^31 unknowns");
  const int r = sd.r;
  const LumpedTables lt = lumped_tables_host(s1);  // sc[c]: the metric constants
  std::vector<double> bands[3][2][3];
  double scale[3] = {0, 0, 0};
  for (int c = 0; c < sd.ncomp; ++c) {
    const CompDesc& cd = sd.comp[c];
    scale[c] = 0.5 / lt.sc[c];
    for (int a = 0; a < 3; ++a) {
      if (a >= sd.dim) {
        bands[c][0][a] = bands[c][1][a] = identity_band(1, r);
        continue;
      }
      const bool nodal = (cd.nodal_mask >> a) & 1, per = (sd.periodic >> a) & 1;
      const std::vector<double> A = mass1d_band(r, (int)m->nel[a], nodal, (int)cd.start[a], (int)cd.count[a], per);
      spai1d(A, (int)cd.count[a], r, pattern, bands[c][0][a], bands[c][1][a], per);
    }
  }
  return upload_bands(sd, bands, 2, scale, out, mem, "SPAI Q1");
}

int build_band_mass(const gym_space* sp, SpaiParams* out, double** mem) {
  const SpaceDesc& sd = sp->desc;
  const gym_mesh* m = sp->mesh;
  if (m->curved) return fail(GYM_E_UNSUPPORTED, "band mass: affine meshes only");
  if (sd.ndofs >= (1LL << 31)) return fail(GYM_E_ARG, "band mass: more than 2^31 unknowns");
  const LumpedTables lt = lumped_tables_host(sp);
  std::vector<double> bands[3][2][3];
  double scale[3] = {0, 0, 0};
  for (int c = 0; c < sd.ncomp; ++c) {
    const CompDesc& cd = sd.comp[c];
    scale[c] = lt.sc[c];
    for (int a = 0; a < 3; ++a) {
      if (a >= sd.dim) {
        bands[c][0][a] = identity_band(1, sd.r);
        continue;
      }
      const bool nodal = (cd.nodal_mask >> a) & 1, per = (sd.periodic >> a) & 1;
      bands[c][0][a] = mass1d_band(sd.r, (int)m->nel[a], nodal, (int)cd.start[a], (int)cd.count[a], per);
    }
  }
  return upload_bands(sd, bands, 1, scale, out, mem, "band mass");
}

void launch_spai_apply(const SpaiParams& p, const double* x, double* y, int nb, hipStream_t s) {
  // one row per thread: each pass has a single load chain per row, so the
  // loads in flight come from the number of resident waves
  const long long rows = (p.n + 255) / 256;
  if (rows > nb) nb = (int)(rows < (1LL << 20) ? rows : (1LL << 20));
  for (int t = 0; t < p.terms; ++t) {  // Q_x (x) Q_y (x) Q_z, then (two terms) the transposed one
    const int close = p.terms == 1 ? 2 : t;
    hipLaunchKernelGGL(spai_axis_kernel, dim3(nb), dim3(256), 0, s, p, t, 0, 0, x, p.tmp[0]);
    hipLaunchKernelGGL(spai_axis_kernel, dim3(nb), dim3(256), 0, s, p, t, 1, 0, (const double*)p.tmp[0], p.tmp[1]);
    hipLaunchKernelGGL(spai_axis_kernel, dim3(nb), dim3(256), 0, s, p, t, 2, close, (const double*)p.tmp[1], y);
  }
}

}  // namespace gym
