// C ABI entry points of the gym library (declared in include/gym.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "geom.hpp"
#include "gym_internal.hpp"
#include "kernels.hpp"
#include "krylov.hpp"
#include "hodge_mfma.hpp"
#include "poisson_mfma.hpp"
#include "schur.hpp"
#include "spai.hpp"

namespace gym {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string("HIP error: ") + hipGetErrorString(e) + " in " + what;
  return GYM_E_HIP;
}

namespace {

DevSpace to_dev(const SpaceDesc& s, long long base) {
  DevSpace d{};
  for (int c = 0; c < 3; ++c) {
    const CompDesc& cd = s.comp[c < s.ncomp ? c : 0];
    d.c[c].offset = base + (c < s.ncomp ? cd.offset : 0);
    for (int a = 0; a < 3; ++a) {
      d.c[c].start[a] = (int)cd.start[a];
      d.c[c].count[a] = (int)cd.count[a];
    }
  }
  return d;
}

// constant pointwise metric of one component on an axis-aligned box cell
double metric_const(int kind, int comp, const gym_mesh* m) {
  double det = 1.0;
  for (int a = 0; a < m->dim; ++a) det *= m->h[a];
  switch (kind) {
    case GYM_H1: return det;
    case GYM_HCURL: return det / (m->h[comp] * m->h[comp]);
    case GYM_HDIV: return m->h[comp] * m->h[comp] / det;
    default: return 1.0 / det;
  }
}

// Diagonals of the global 1-D reference matrices along one axis:
// nodal mass, edge mass and the nodal stiffness Delta^T M_e Delta.
struct Diag1D {
  std::vector<double> dn, de, dk;
};

Diag1D diag1d(int r, int64_t nel) {
  Tables1D t = make_tables(r, r + 1);
  int q = r + 1;
  std::vector<double> mn(r + 1), me(r), kk(r + 1, 0.0);
  for (int i = 0; i <= r; ++i) {
    double s = 0;
    for (int k = 0; k < q; ++k) s += t.gw[k] * t.phi[k * (r + 1) + i] * t.phi[k * (r + 1) + i];
    mn[i] = s;
  }
  std::vector<double> Me(r * r);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0;
      for (int k = 0; k < q; ++k) s += t.gw[k] * t.edge[k * r + i] * t.edge[k * r + j];
      Me[i * r + j] = s;
    }
  for (int i = 0; i < r; ++i) me[i] = Me[i * r + i];
  // (Delta u)_j = u_{j+1} - u_j; diag of Delta^T Me Delta at node i:
  for (int i = 0; i <= r; ++i) {
    double s = 0;
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < r; ++b) {
        double ea = (i == a + 1) ? 1.0 : (i == a ? -1.0 : 0.0);
        double eb = (i == b + 1) ? 1.0 : (i == b ? -1.0 : 0.0);
        s += ea * Me[a * r + b] * eb;
      }
    kk[i] = s;
  }
  int64_t m = r * nel;
  Diag1D d;
  d.dn.assign(m + 1, 0.0);
  d.dk.assign(m + 1, 0.0);
  d.de.assign(m, 0.0);
  for (int64_t e = 0; e < nel; ++e) {
    for (int i = 0; i <= r; ++i) {
      d.dn[r * e + i] += mn[i];
      d.dk[r * e + i] += kk[i];
    }
    for (int j = 0; j < r; ++j) d.de[r * e + j] = me[j];
  }
  return d;
}

// Row sums of the global 1-D reference mass matrices along one axis, without
// boundary conditions: nodal (r nel + 1 entries), edge (r nel).
void rowsum1d(int r, int64_t nel, std::vector<double>& rn, std::vector<double>& re) {
  Tables1D t = make_tables(r, r + 1);
  const int q = r + 1;
  std::vector<double> sn(r + 1, 0.0), se(r, 0.0);
  for (int i = 0; i <= r; ++i)
    for (int j = 0; j <= r; ++j)
      for (int k = 0; k < q; ++k) sn[i] += t.gw[k] * t.phi[k * (r + 1) + i] * t.phi[k * (r + 1) + j];
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j)
      for (int k = 0; k < q; ++k) se[i] += t.gw[k] * t.edge[k * r + i] * t.edge[k * r + j];
  const int64_t m = r * nel;
  rn.assign(m + 1, 0.0);
  re.assign(m, 0.0);
  for (int64_t e = 0; e < nel; ++e) {
    for (int i = 0; i <= r; ++i) rn[r * e + i] += sn[i];
    for (int j = 0; j < r; ++j) re[r * e + j] = se[j];
  }
}

// Preconditioner diagonal on affine meshes (see gym_op_precond_diag).
std::vector<double> precond_diag_host(const gym_op* op) {
  const gym_mesh* m = op->mesh;
  const int dim = m->dim;
  std::vector<Diag1D> D;
  for (int a = 0; a < 3; ++a) D.push_back(diag1d(op->r, a < dim ? m->nel[a] : 1));
  std::vector<double> out(op->na + op->nb, 0.0);
  auto loop = [&](const SpaceDesc& s, int64_t base, auto&& fn) {
    for (int c = 0; c < s.ncomp; ++c) {
      const CompDesc& cd = s.comp[c];
      int64_t idx = base + cd.offset;
      for (int64_t k = 0; k < cd.count[2]; ++k)
        for (int64_t j = 0; j < cd.count[1]; ++j)
          for (int64_t i = 0; i < cd.count[0]; ++i) {
            int64_t p[3] = {cd.start[0] + i, cd.start[1] + j, cd.start[2] + k};
            out[idx++] = fn(c, p);
          }
    }
  };
  auto dn = [&](int a, int64_t p) { return a < dim ? D[a].dn[p] : 1.0; };
  auto de = [&](int a, int64_t p) { return a < dim ? D[a].de[p] : 1.0; };
  auto dk = [&](int a, int64_t p) { return D[a].dk[p]; };
  if (op->problem == GYM_MIXED_POISSON) {
    const double s3 = metric_const(GYM_L2, 0, m);
    loop(op->sa, 0, [&](int c, const int64_t* p) {
      double rest = 1.0;
      for (int a = 0; a < dim; ++a)
        if (a != c) rest *= de(a, p[a]);
      return metric_const(GYM_HDIV, c, m) * dn(c, p[c]) * rest + s3 * dk(c, p[c]) * rest;
    });
    loop(op->sb, op->na, [&](int, const int64_t* p) {
      double v = s3;
      for (int a = 0; a < dim; ++a) v *= de(a, p[a]);
      return v;
    });
  } else {
    loop(op->sa, 0, [&](int, const int64_t* p) {
      double v = metric_const(GYM_H1, 0, m);
      for (int a = 0; a < 3; ++a) v *= dn(a, p[a]);
      for (int c = 0; c < 3; ++c) {
        double t = metric_const(GYM_HCURL, c, m) * dk(c, p[c]);
        for (int a = 0; a < 3; ++a)
          if (a != c) t *= dn(a, p[a]);
        v += t;
      }
      return v;
    });
    loop(op->sb, op->na, [&](int c, const int64_t* p) {
      int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      double v = metric_const(GYM_HCURL, c, m) * de(c, p[c]) * dn(c1, p[c1]) * dn(c2, p[c2]);
      v += metric_const(GYM_HDIV, c1, m) * de(c, p[c]) * dn(c1, p[c1]) * dk(c2, p[c2]);
      v += metric_const(GYM_HDIV, c2, m) * de(c, p[c]) * dn(c2, p[c2]) * dk(c1, p[c1]);
      return v;
    });
  }
  return out;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

int dalloc(void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(GYM_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return 0;
}

int check_mesh_jacobians(const gym_mesh* m) {
  // det J > 0 at the corners and the 5-point Gauss points of every cell;
  // the cell layers are split over host threads
  std::vector<double> gx, gw;
  gauss_rule(5, gx, gw);
  std::vector<double> pts = {0.0};
  pts.insert(pts.end(), gx.begin(), gx.end());
  pts.push_back(1.0);
  const int d = m->dim;
  const int64_t nx = m->nel[0], ny = m->nel[1], nz = d == 3 ? m->nel[2] : 1;
  const double* V = m->vertices.data();
  auto vtx = [&](int64_t i, int64_t j, int64_t k, int a) {
    return V[((k * (ny + 1) + j) * (nx + 1) + i) * d + a];
  };
  const std::vector<double> zpts = d == 3 ? pts : std::vector<double>{0.5};
  // first bad cell (linear index), or -1
  auto check_layer = [&](int64_t k) -> int64_t {
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i)
        for (double z : zpts)
          for (double y : pts)
            for (double x : pts) {
              double J[3][3] = {{0}};
              double xi[3] = {x, y, z};
              for (int corner = 0; corner < (1 << d); ++corner) {
                int b[3] = {corner & 1, (corner >> 1) & 1, (corner >> 2) & 1};
                for (int a = 0; a < d; ++a) {
                  double g = 1.0;
                  for (int c = 0; c < d; ++c) {
                    if (c == a) g *= b[c] ? 1.0 : -1.0;
                    else g *= b[c] ? xi[c] : 1.0 - xi[c];
                  }
                  for (int comp = 0; comp < d; ++comp)
                    J[comp][a] += g * vtx(i + b[0], j + b[1], k + (d == 3 ? b[2] : 0), comp);
                }
              }
              double det = d == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                                  : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
              if (!(det > 0)) return i + nx * (j + ny * k);
            }
    return -1;
  };
  const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(nz, std::max(1u, std::thread::hardware_concurrency())));
  std::atomic<int64_t> bad{-1};
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    for (int64_t k; (k = next.fetch_add(1)) < nz && bad.load() < 0;) {
      int64_t c = check_layer(k);
      if (c >= 0) {
        int64_t expect = -1;
        bad.compare_exchange_strong(expect, c);
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nth; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
  const int64_t c = bad.load();
  if (c >= 0)
    return fail(GYM_E_INVALID_MESH, "det J <= 0 in cell (" + std::to_string(c % nx) + "," +
                                        std::to_string((c / nx) % ny) + "," + std::to_string(c / (nx * ny)) + ")");
  return 0;
}

void set_form(OpParams& p, const gym_ctx* ctx, const gym_mesh* m) {
  p.kron = (ctx->mass_form == 0 && !m->curved) ? 1 : 0;
  // auto: whole-CU tiles (least halo recomputation) unless the mesh is too
  // small to give every CU one of them; decided at launch
  p.tile_budget = ctx->tile == 1 ? 0 : ctx->tile == 2 ? 1 : 2;
  p.curved = m->curved ? 1 : 0;
}

// Curved meshes: the Gauss-point metrics of degree r in the precision of the
// contractions (FP32 also for the bf16-operand mode, which curved kernels
// refuse anyway).
int set_qdata(OpParams& p, const gym_mesh* m, int r, int prec) {
  if (!m->curved || m->dim != 3) return 0;
  const void* q = nullptr;
  if (int rc = mesh_qdata(m, r, prec == GYM_F64 ? 0 : 1, &q)) return rc;
  p.qd = q;
  p.qfs = (long long)(r + 1) * m->nel[0] * (r + 1) * m->nel[1] * (r + 1) * m->nel[2];
  return 0;
}

// On curved cells the metric is evaluated per Gauss point; the per-block
// factors only carry signs.
void curved_scales(OpParams& p) {
  for (double& v : p.sc) v = 1.0;
}

}  // namespace

int mesh_qdata(const gym_mesh* m, int r, int f32, const void** out) {
  *out = nullptr;
  if (!m->curved || m->dim != 3 || r < 1 || r > kMaxR)
    return fail(GYM_E_UNSUPPORTED, "Gauss-point metrics exist for curved 3-D meshes only");
  void*& slot = m->qd[f32 ? 1 : 0][r];
  if (!slot) {
    const int q = r + 1;
    const int nel[3] = {(int)m->nel[0], (int)m->nel[1], (int)m->nel[2]};
    const long long fs = (long long)q * nel[0] * q * nel[1] * q * nel[2];
    if (int rc = dalloc(&slot, (size_t)kQFields * fs * (f32 ? sizeof(float) : sizeof(double)))) return rc;
    Tables1D t = make_tables(r, q);
    if (launch_qdata(m->d_vertices, nel, q, t.gx.data(), slot, f32 ? 1 : 0, nullptr)) {
      (void)hipFree(slot);
      slot = nullptr;
      return fail(GYM_E_HIP, "Gauss-point metric kernel launch failed");
    }
    GYM_HIP(hipDeviceSynchronize());
  }
  *out = slot;
  return 0;
}

// Kernel parameters of a block operator apply (shared with the server).
void build_op_params(const gym_op* op, const void* x, void* y, OpParams& p, int& prob) {
  const gym_mesh* m = op->mesh;
  p = OpParams{};
  set_form(p, op->ctx, m);
  p.x = x;
  p.y = y;
  p.ndofs = op->na + op->nb;
  p.sa = to_dev(op->sa, 0);
  p.sb = to_dev(op->sb, op->na);
  for (int a = 0; a < 3; ++a) {
    p.nel[a] = a < m->dim ? (int)m->nel[a] : 1;
    p.m[a] = a < m->dim ? (int)(op->r * m->nel[a]) : 1;
  }
  if (op->problem == GYM_MIXED_POISSON) {
    prob = PROB_POISSON;
    for (int c = 0; c < m->dim; ++c) p.sc[c] = metric_const(GYM_HDIV, c, m);
    p.sc[3] = metric_const(GYM_L2, 0, m);
  } else {
    prob = PROB_HODGE;
    p.sc[0] = metric_const(GYM_H1, 0, m);
    for (int c = 0; c < 3; ++c) {
      p.sc[1 + c] = metric_const(GYM_HCURL, c, m);
      p.sc[4 + c] = metric_const(GYM_HDIV, c, m);
    }
  }
  if (m->curved) curved_scales(p);
}

namespace {

// bf16 element products on the matrix cores: mixed Poisson, affine 3-D, r >= 3
bool mfma_path(const gym_op* op, int prec) {
  return prec == GYM_BF16 && op->problem == GYM_MIXED_POISSON && op->mesh->dim == 3 && !op->mesh->curved &&
         op->r >= 3;
}

struct MfmaState {
  uint16_t* frag = nullptr;
  float* yel = nullptr;
  int nrhs = 0;
};

int mfma_launch(const gym_op* op, int nrhs, const void* x, void* y, hipStream_t s, const MrStep* mr, int* wg_out) {
  const gym_mesh* m = op->mesh;
  const long long E = m->nel[0] * m->nel[1] * m->nel[2];
  const int rows = poisson_mfma_rows(op->r);
  PoissonMfmaParams q{};
  q.ndofs = op->na + op->nb;
  q.gather_blocks = poisson_mfma_gather_blocks(q.ndofs, op->ctx->ncu);
  if (wg_out) {
    *wg_out = q.gather_blocks;
    return 0;
  }
  gym_op* mop = const_cast<gym_op*>(op);  // lazily built apply state
  MfmaState* st = static_cast<MfmaState*>(mop->mfma);
  if (!st) {
    st = new MfmaState;
    std::vector<double> mn, me;
    element_masses_1d(op->r, mn, me);
    const double s3 = metric_const(GYM_L2, 0, m);
    std::vector<uint16_t> f = poisson_mfma_fragments(op->r, mn, me, s3);
    if (int rc = dalloc((void**)&st->frag, sizeof(uint16_t) * f.size())) {
      delete st;
      return rc;
    }
    if (hipMemcpy(st->frag, f.data(), sizeof(uint16_t) * f.size(), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(st->frag);
      delete st;
      return fail(GYM_E_HIP, "upload of the element fragments");
    }
    mop->mfma = st;
  }
  if (st->nrhs < nrhs) {
    if (st->yel) (void)hipFree(st->yel);
    st->yel = nullptr;
    st->nrhs = 0;
    if (int rc = dalloc((void**)&st->yel, sizeof(float) * (size_t)rows * E * nrhs)) return rc;
    st->nrhs = nrhs;
  }
  q.x = x;
  q.y = y;
  q.yel = st->yel;
  q.np_off = op->na;
  q.el_rows = E;
  q.el_stride = (long long)rows * E;
  for (int a = 0; a < 3; ++a) {
    q.nel[a] = (int)m->nel[a];
    q.m[a] = (int)(op->r * m->nel[a]);
    q.s2[a] = (float)metric_const(GYM_HDIV, a, m);
  }
  q.s = to_dev(op->sa, 0);
  if (mr) q.mr = *mr;
  if (launch_poisson_mfma(q, st->frag, op->r, nrhs, mr != nullptr, op->ctx->ncu, s))
    return fail(GYM_E_HIP, "matrix-core operator launch failed");
  return 0;
}

// Curved Hodge apply of degree 3 on the matrix cores, FP64 arithmetic with
// FP64 or FP32 vectors (fewer than 2^31 unknowns: the kernel's z offsets are
// 32-bit).
bool hc_path(const gym_op* op, int prec) {
  const gym_mesh* m = op->mesh;
  return (prec == GYM_F64 || prec == GYM_F32) && op->problem != GYM_MIXED_POISSON && m->curved && m->dim == 3 &&
         !m->periodic && op->r == kHcDegree && op->ctx->curved_kernel == 0 && op->na + op->nb < (1LL << 31);
}

int hc_launch(const gym_op* op, int prec, int nrhs, const void* x, void* y, hipStream_t s) {
  const gym_mesh* m = op->mesh;
  HcParams q{};
  q.x = x;
  q.y = y;
  q.ndofs = op->na + op->nb;
  const DevSpace a = to_dev(op->sa, 0), b = to_dev(op->sb, op->na);
  q.f[0] = a.c[0];
  for (int c = 0; c < 3; ++c) q.f[1 + c] = b.c[c];
  for (int i = 0; i < 3; ++i) q.nel[i] = (int)m->nel[i];
  q.verts = m->d_vertices;
  gym_op* mop = const_cast<gym_op*>(op);  // lazily sized apply state
  const long long need = hodge_mfma_halo_doubles(q.nel, nrhs);
  if (mop->hc_halo_n < need) {
    if (mop->hc_halo) (void)hipFree(mop->hc_halo);
    mop->hc_halo = nullptr;
    mop->hc_halo_n = 0;
    // the halo slots, then one zero that the kernel only reads
    if (int rc = dalloc((void**)&mop->hc_halo, sizeof(double) * (size_t)(need + 1))) return rc;
    if (hipMemset(mop->hc_halo + need, 0, sizeof(double)) != hipSuccess) {
      (void)hipFree(mop->hc_halo);
      mop->hc_halo = nullptr;
      return fail(GYM_E_HIP, "matrix-core operator: workspace set-up failed");
    }
    mop->hc_halo_n = need;
  }
  q.halo = mop->hc_halo;
  q.zero = mop->hc_halo + mop->hc_halo_n;
  q.chunk_mode = op->ctx->tile;  // large tiles: whole z columns; small: one layer per workgroup
  if (launch_hodge_mfma(q, nrhs, op->ctx->ncu, s, prec == GYM_F32))
    return fail(GYM_E_HIP, "matrix-core operator launch failed");
  return 0;
}

// matrix_core: the curved Hodge apply may take the matrix-core kernel, whose
// tile-boundary buffer is allocated on first use (callers that must not
// allocate pass false and get the tile kernel).
int op_launch(const gym_op* op, int prec, int nrhs, const void* x, void* y, hipStream_t s, const MrStep* mr,
              int* wg_out, bool matrix_core) {
  if (mfma_path(op, prec)) return mfma_launch(op, nrhs, x, y, s, mr, wg_out);
  if (matrix_core && hc_path(op, prec)) {
    // With a MINRES step the apply is followed by the step's first half as a
    // kernel of its own: partial sums of z . A z over vec_grid blocks per
    // right-hand side, skipping converged ones (the layout minres_step2 reads).
    const long long n = op->na + op->nb;
    const int np = vec_grid(n, op->ctx->ncu);
    if (wg_out) {
      *wg_out = np;
      return 0;
    }
    if (int rc = hc_launch(op, prec, nrhs, x, y, s)) return rc;
    if (mr) {
      if (prec == GYM_F64)
        minres_launch_dot2<double>(static_cast<const double*>(x), static_cast<const double*>(y), nullptr, n, nrhs,
                                   np, mr->pa, nullptr, s, mr->cur);
      else
        minres_launch_dot2<float>(static_cast<const float*>(x), static_cast<const float*>(y), nullptr, n, nrhs, np,
                                  mr->pa, nullptr, s, mr->cur);
    }
    return 0;
  }
  OpParams p;
  int prob;
  build_op_params(op, x, y, p, prob);
  if (int rc = set_qdata(p, op->mesh, op->r, prec)) return rc;
  if (prec == GYM_BF16) {
    p.bf16 = 1;  // FP32 vectors, bf16 contraction operands
    prec = GYM_F32;
  }
  if (mr) {
    p.fused = 1;
    p.mr = *mr;
  }
  p.wg_out = wg_out;
  p.dry = wg_out ? 1 : 0;
  int rc = launch_operator(prob, op->mesh->dim, op->r, prec, p, nrhs, op->ctx->ncu, s);
  if (rc == -2) return fail(GYM_E_UNSUPPORTED, "no kernel for this problem/degree/precision");
  if (rc) return fail(GYM_E_HIP, "operator kernel launch failed");
  return 0;
}
}  // namespace

int launch_op_apply(const gym_op* op, int prec, int nrhs, const void* x, void* y, hipStream_t s, const MrStep* mr,
                    bool matrix_core) {
  return op_launch(op, prec, nrhs, x, y, s, mr, nullptr, matrix_core);
}

int op_workgroups(const gym_op* op, int prec, int nrhs, int* wg, bool matrix_core) {
  *wg = 0;
  if (int rc = op_launch(op, prec, nrhs, nullptr, nullptr, nullptr, nullptr, wg, matrix_core)) return rc;
  return *wg > 0 ? 0 : fail(GYM_E_HIP, "operator tiling query failed");
}

namespace {

int launch_mass_apply(const gym_space* sp, int prec, int nrhs, const void* x, void* y, hipStream_t s) {
  const gym_mesh* m = sp->mesh;
  if (sp->desc.periodic) {
    // periodic axes: the mass as a Kronecker product of assembled 1-D bands
    // with wrap-around (FP64), built on first use and kept with the space
    if (prec != GYM_F64) return fail(GYM_E_UNSUPPORTED, "mass apply on a periodic space: FP64 only");
    gym_space* w = const_cast<gym_space*>(sp);  // cache only
    if (!w->band) {
      SpaiParams* bp = new SpaiParams{};
      if (int rc = build_band_mass(sp, bp, &w->band_mem)) {
        delete bp;
        return rc;
      }
      w->band = bp;
    }
    const SpaiParams& bp = *static_cast<const SpaiParams*>(sp->band);
    const long long n = sp->desc.ndofs;
    for (int k = 0; k < nrhs; ++k)
      launch_spai_apply(bp, static_cast<const double*>(x) + k * n, static_cast<double*>(y) + k * n,
                        vec_grid(n, sp->ctx->ncu), s);
    GYM_HIP(hipGetLastError());
    return 0;
  }
  OpParams p{};
  set_form(p, sp->ctx, m);
  p.x = x;
  p.y = y;
  p.ndofs = sp->desc.ndofs;
  p.sa = to_dev(sp->desc, 0);
  p.sb = p.sa;
  for (int a = 0; a < 3; ++a) {
    p.nel[a] = a < m->dim ? (int)m->nel[a] : 1;
    p.m[a] = a < m->dim ? (int)(sp->desc.r * m->nel[a]) : 1;
  }
  for (int c = 0; c < sp->desc.ncomp; ++c) p.sc[c] = metric_const(sp->desc.kind, c, m);
  if (m->curved) curved_scales(p);
  if (int rc = set_qdata(p, m, sp->desc.r, prec)) return rc;
  int prob = PROB_MASS_H1 + sp->desc.kind;
  if (prec == GYM_BF16) {
    p.bf16 = 1;
    prec = GYM_F32;
  }
  int rc = launch_operator(prob, m->dim, sp->desc.r, prec, p, nrhs, sp->ctx->ncu, s);
  if (rc == -2) return fail(GYM_E_UNSUPPORTED, "no mass kernel for this space/precision");
  if (rc) return fail(GYM_E_HIP, "mass kernel launch failed");
  return 0;
}

// ---- Krylov drivers ---------------------------------------------------------
template <typename TV>
struct MinresWork {
  TV *r1 = nullptr, *r2 = nullptr, *y = nullptr, *z = nullptr, *zp = nullptr, *w = nullptr, *w1 = nullptr,
     *w2 = nullptr;
  // partial sums (fused apply: pa; minres_step2: two alternating sets of
  // pb, pc and alfa per rhs)
  double *pa = nullptr, *pb[2] = {}, *pc[2] = {}, *alfa[2] = {};
  int npa_cap = 0;
  MinresState* st = nullptr;
  MinresState* host = nullptr;
};

template <typename TV>
int alloc_minres(std::vector<void*>& pool, MinresWork<TV>& w, long long n, int nrhs) {
  TV** vecs[8] = {&w.r1, &w.r2, &w.y, &w.z, &w.zp, &w.w, &w.w1, &w.w2};
  for (TV** v : vecs) {
    void* p;
    if (int rc = dalloc(&p, sizeof(TV) * n * nrhs)) return rc;
    pool.push_back(p);
    *v = (TV*)p;
  }
  void* p;
  if (int rc = dalloc(&p, sizeof(MinresState) * 2 * nrhs)) return rc;
  pool.push_back(p);
  w.st = (MinresState*)p;
  GYM_HIP(hipHostMalloc((void**)&w.host, sizeof(MinresState) * 2 * nrhs, hipHostMallocDefault));
  return 0;
}

// Partial-sum buffers for a fused apply of npa workgroups per rhs (grown
// when the tiling changes, e.g. after a context option).
template <typename TV>
int ensure_partials(std::vector<void*>& pool, MinresWork<TV>& w, int npa, int nb, int nrhs) {
  if (npa <= w.npa_cap) return 0;
  void* p;
  if (int rc = dalloc(&p, sizeof(double) * ((long long)(npa + 4 * nb + 2) * nrhs))) return rc;
  pool.push_back(p);
  w.pa = (double*)p;
  double* q = w.pa + (long long)npa * nrhs;
  for (int k = 0; k < 2; ++k) {
    w.pb[k] = q;
    w.pc[k] = q + (long long)nb * nrhs;
    w.alfa[k] = q + 2LL * nb * nrhs;
    q += (2LL * nb + 1) * nrhs;
  }
  w.npa_cap = npa;
  return 0;
}

// Preconditioned MINRES from x = 0, two launches per step: the operator
// apply carrying the first half of the step (MrStep) and minres_step2.  The
// host reads the states every check_every steps; on exit x is complete (a
// step still pending at the iteration cap is finished by minres_finish).
// npa = workgroups per rhs of the fused apply.
// A non-diagonal preconditioner: out = M^-1 in for all right-hand sides,
// leaving those whose Krylov state in gate (if not null) has converged.
template <typename TV>
using PrecFn = std::function<int(const TV*, TV*, const MinresState*)>;

template <typename TV, typename Apply>
int run_minres(Apply&& apply, long long n, int nrhs, int nb, int npa, const TV* b, TV* x, const double* dinv,
               double tol, int maxit, int check_every, MinresWork<TV>& wk, hipStream_t s, int* iters_out,
               int* flag_out, const PrecFn<TV>* ext = nullptr) {
  if (npa > wk.npa_cap) return fail(GYM_E_HIP, "MINRES partial-sum buffer too small for this launch");
  // init: r1 = r2 = b, z = M^-1 b (into wk.z), beta_1 in slot 0
  MinresVecs<TV> V{b, x, wk.r1, wk.r2, wk.z, wk.y, wk.w, wk.w1, wk.w2};
  if (ext) {
    minres_launch_init_vecs<TV>(V, n, nrhs, nb, s);
    if (int rc = (*ext)(b, wk.z, nullptr)) return rc;
    minres_launch_dot2<TV>(b, wk.z, nullptr, n, nrhs, nb, wk.pb[0], nullptr, s);
    minres_launch_init_state<TV>(V, n, nrhs, nb, wk.pb[0], wk.st, tol, s);
  } else {
    minres_launch_init<TV>(V, dinv, n, nrhs, nb, wk.pb[0], wk.st, tol, s);
  }
  int par = 0;  // set of step2 partials written last
  if (check_every < 1) check_every = 1;
  int it = 0, slot = 0;
  bool all_done = false, pending = false;
  while (it < maxit && !all_done) {
    MinresState* cur = wk.st + slot * nrhs;
    MinresState* next = wk.st + (slot ^ 1) * nrhs;
    const MrStep m{cur, wk.pa};
    if (int rc = apply(wk.z, wk.y, m)) return rc;
    const MrVecs<TV> mv{wk.y, wk.r1, wk.r2, wk.zp, x, wk.w2, wk.w, wk.w1};
    const Step2Io io{cur, next, pending ? 0 : 1, npa, nb, wk.pa, wk.pb[par], wk.pc[par], wk.alfa[par],
                     wk.pb[par ^ 1], wk.pc[par ^ 1], wk.alfa[par ^ 1], ext ? 1 : 0};
    minres_launch_step2<TV>(mv, dinv, n, nrhs, nb, io, s);
    if (ext) {
      // z_{k+1} = M^-1 y over zp (read by step2 already), and the partial
      // sums step2 leaves to us: y . z_{k+1}, z_{k+1} . r2
      if (int rc = (*ext)(wk.y, wk.zp, cur)) return rc;
      minres_launch_dot2<TV>(wk.y, wk.zp, wk.r2, n, nrhs, nb, io.pb, io.pc, s, cur);
    }
    par ^= 1;
    if (pending) {  // the newest w was written over the oldest
      TV *ow = wk.w, *ow1 = wk.w1, *ow2 = wk.w2;
      wk.w = ow1;
      wk.w1 = ow2;
      wk.w2 = ow;
    }
    std::swap(wk.z, wk.zp);  // z_{k+1} becomes the apply input, z_k the previous one
    TV* old_r1 = wk.r1;
    wk.r1 = wk.r2;
    wk.r2 = wk.y;
    wk.y = old_r1;
    pending = true;
    slot ^= 1;
    ++it;
    if (it % check_every == 0 || it == maxit) {
      GYM_HIP(hipMemcpyAsync(wk.host, wk.st + slot * nrhs, sizeof(MinresState) * nrhs, hipMemcpyDeviceToHost, s));
      GYM_HIP(hipStreamSynchronize(s));
      all_done = true;
      for (int r = 0; r < nrhs; ++r) all_done = all_done && wk.host[r].done;
    }
  }
  if (!all_done && pending) {
    minres_launch_finish<TV>(x, wk.zp, wk.w2, wk.w, wk.w1, n, nrhs, nb, wk.st + slot * nrhs,
                             wk.st + (slot ^ 1) * nrhs, wk.pb[par], wk.alfa[par], s);
    slot ^= 1;
  }
  GYM_HIP(hipGetLastError());
  GYM_HIP(hipMemcpyAsync(wk.host, wk.st + slot * nrhs, sizeof(MinresState) * nrhs, hipMemcpyDeviceToHost, s));
  GYM_HIP(hipStreamSynchronize(s));
  int maxitn = 0, flag = 1;
  for (int r = 0; r < nrhs; ++r) {
    maxitn = std::max(maxitn, wk.host[r].itn);
    if (wk.host[r].flag < 0) flag = -1;
    else if (wk.host[r].flag == 0 && flag > 0) flag = 0;
  }
  *iters_out = maxitn;
  *flag_out = flag;
  return 0;
}

int relres_f64(const gym_op* op, int nrhs, const double* b, const double* x, double* tmp, double* part,
               double* sums, int nb, hipStream_t s, std::vector<double>& rel, std::vector<double>* rnorm = nullptr,
               bool matrix_core = true) {
  long long n = op->na + op->nb;
  if (int rc = launch_op_apply(op, GYM_F64, nrhs, x, tmp, s, nullptr, matrix_core)) return rc;
  launch_norm2(tmp, b, n, nrhs, nb, 1, part, sums, s);
  launch_norm2(b, nullptr, n, nrhs, nb, 0, part, sums + nrhs, s);
  std::vector<double> h(2 * nrhs);
  GYM_HIP(hipMemcpyAsync(h.data(), sums, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
  GYM_HIP(hipStreamSynchronize(s));
  rel.assign(nrhs, 0.0);
  if (rnorm) rnorm->assign(nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r) {
    double rn = std::sqrt(h[r]), bn = std::sqrt(h[nrhs + r]);
    rel[r] = bn > 0 ? rn / bn : rn;
    if (rnorm) (*rnorm)[r] = rn;
  }
  return 0;
}

// Brackets every `period`-th operator apply with a HIP event pair
// (pre-created pool) and sums their elapsed times once the stream has been
// synchronised.  An event pair costs several microseconds of stream time, so
// sampling keeps the measurement from slowing the solve it measures.
struct ApplyTimer {
  int period = 0;  // 0: off
  long long count = 0;
  bool open = false;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  ~ApplyTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  int begin(hipStream_t s) {
    open = period > 0 && (count++ % period) == 0;
    if (!open) return 0;
    if (used + 2 > ev.size()) {
      for (int k = 0; k < 256; ++k) {
        hipEvent_t e;
        GYM_HIP(hipEventCreate(&e));
        ev.push_back(e);
      }
    }
    GYM_HIP(hipEventRecord(ev[used], s));
    return 0;
  }
  int end(hipStream_t s) {
    if (!open) return 0;
    GYM_HIP(hipEventRecord(ev[used + 1], s));
    used += 2;
    return 0;
  }
  // call after the stream is synchronised
  int collect(int* n, double* ms) {
    double tot = 0;
    for (size_t k = 0; k + 1 < used; k += 2) {
      float t = 0;
      GYM_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      tot += t;
    }
    *n = (int)(used / 2);
    *ms = tot;
    used = 0;
    return 0;
  }
};

}  // namespace

// Workspace held by an operator between solves.
struct OpWork {
  long long n = 0;
  int nrhs = 0, nb = 0;
  MinresWork<double> m64;
  MinresWork<float> m32;
  double *tmp = nullptr, *part = nullptr, *sums = nullptr, *r64 = nullptr, *d64 = nullptr, *scale = nullptr;
  float *r32 = nullptr, *x32 = nullptr;
  double* ones = nullptr;  // the identity "diagonal" of GYM_PRECOND_NONE
  std::vector<void*> pool;
  bool matrix_core = true;  // false: applies that allocate nothing (launch_op_apply)
};

int ensure_schur(gym_op* op, int nrhs, SchurPrec** out) {
  if (!op->schur) {
    SchurPrec* P = new SchurPrec;
    if (int rc = schur_build(op, P)) {
      delete P;
      return rc;
    }
    op->schur = P;
  }
  SchurPrec* P = static_cast<SchurPrec*>(op->schur);
  if (int rc = schur_reserve(P, nrhs, sizeof(double))) return rc;
  *out = P;
  return 0;
}

// Workspace of CG mass solves, cached on the space.
struct MassWork {
  int nrhs = 0, nb = 0;
  double *r = nullptr, *p = nullptr, *q = nullptr, *pa = nullptr, *pb = nullptr, *sums = nullptr;
  CgState* st = nullptr;
  CgState* host = nullptr;
  std::vector<void*> pool;
};

// Diagonal (rowsum = false) or row sums (true) of the mass of a space with a
// periodic axis: Kronecker products of the 1-D diagonals or row sums of the
// assembled 1-D masses with their wrap, times the component's metric.
std::vector<double> periodic_diag_host(const gym_space* sp, bool rowsum) {
  const gym_mesh* m = sp->mesh;
  const SpaceDesc& s = sp->desc;
  std::vector<double> out(s.ndofs);
  for (int c = 0; c < s.ncomp; ++c) {
    const CompDesc& cd = s.comp[c];
    std::vector<double> f[3];
    for (int a = 0; a < 3; ++a) {
      if (a >= s.dim) {
        f[a].assign(1, 1.0);
        continue;
      }
      std::vector<double> dg, rs;
      mass1d_diag_rowsum(s.r, (int)m->nel[a], (cd.nodal_mask >> a) & 1, (int)cd.start[a], (int)cd.count[a],
                         (s.periodic >> a) & 1, dg, rs);
      f[a] = rowsum ? rs : dg;
    }
    const double sc = metric_const(s.kind, c, m);
    int64_t idx = cd.offset;
    for (int64_t k = 0; k < cd.count[2]; ++k)
      for (int64_t j = 0; j < cd.count[1]; ++j)
        for (int64_t i = 0; i < cd.count[0]; ++i) out[idx++] = sc * f[0][i] * f[1][j] * f[2][k];
  }
  return out;
}

// Diagonal of M_k on an affine box (Kronecker product of 1-D diagonals);
// on curved cells it is the diagonal of the box with the same spacing,
// which only serves as the Jacobi preconditioner.
std::vector<double> mass_diag_host(const gym_space* sp) {
  const gym_mesh* m = sp->mesh;
  const SpaceDesc& s = sp->desc;
  if (s.periodic) return periodic_diag_host(sp, false);
  std::vector<Diag1D> D;
  for (int a = 0; a < 3; ++a) D.push_back(diag1d(s.r, a < m->dim ? m->nel[a] : 1));
  std::vector<double> out(s.ndofs);
  for (int c = 0; c < s.ncomp; ++c) {
    const CompDesc& cd = s.comp[c];
    const double sc = metric_const(s.kind, c, m);
    int64_t idx = cd.offset;
    for (int64_t k = 0; k < cd.count[2]; ++k)
      for (int64_t j = 0; j < cd.count[1]; ++j)
        for (int64_t i = 0; i < cd.count[0]; ++i) {
          int64_t p[3] = {cd.start[0] + i, cd.start[1] + j, cd.start[2] + k};
          double v = sc;
          for (int a = 0; a < m->dim; ++a) v *= (cd.nodal_mask >> a & 1) ? D[a].dn[p[a]] : D[a].de[p[a]];
          out[idx++] = v;
        }
  }
  return out;
}

// Lumped mass of an affine space: the row sums of its mass matrix without
// boundary conditions, at the kept unknowns (Kronecker product of 1-D row
// sums times the constant metric of the component).
LumpedTables lumped_tables_host(const gym_space* sp) {
  const gym_mesh* m = sp->mesh;
  LumpedTables t;
  for (int a = 0; a < 3; ++a) rowsum1d(sp->desc.r, a < m->dim ? m->nel[a] : 1, t.rn[a], t.re[a]);
  for (int c = 0; c < 3; ++c) t.sc[c] = c < sp->desc.ncomp ? metric_const(sp->desc.kind, c, m) : 0.0;
  return t;
}

// Row sums of the mass matrix without boundary conditions on curved cells:
// the natural-BC space's mass (the curved kernel, FP64) applied to ones on the
// device, then restricted to the unknowns `sp` keeps.  Empty on failure.
std::vector<double> curved_rowsums(const gym_space* sp) {
  const SpaceDesc& s = sp->desc;
  std::vector<double> out;
  gym_space* full = nullptr;
  if (gym_space_create(sp->ctx, sp->mesh, s.kind, s.r, GYM_BC_NATURAL, &full)) return out;
  const SpaceDesc& f = full->desc;
  const std::vector<double> ones(f.ndofs, 1.0);
  std::vector<double> rs(f.ndofs);
  void* d = nullptr;
  bool ok = hipMalloc(&d, sizeof(double) * 2 * f.ndofs) == hipSuccess;
  double* x = static_cast<double*>(d);
  ok = ok && hipMemcpy(x, ones.data(), sizeof(double) * f.ndofs, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && launch_mass_apply(full, GYM_F64, 1, x, x + f.ndofs, nullptr) == 0;
  ok = ok && hipMemcpy(rs.data(), x + f.ndofs, sizeof(double) * f.ndofs, hipMemcpyDeviceToHost) == hipSuccess;
  if (d) (void)hipFree(d);
  if (!ok) (void)hipGetLastError();
  if (ok) {
    out.resize(s.ndofs);
    for (int c = 0; c < s.ncomp; ++c) {
      const CompDesc& cd = s.comp[c];
      const CompDesc& fd = f.comp[c];
      int64_t idx = cd.offset;
      for (int64_t k = 0; k < cd.count[2]; ++k)
        for (int64_t j = 0; j < cd.count[1]; ++j)
          for (int64_t i = 0; i < cd.count[0]; ++i) {
            const int64_t p[3] = {cd.start[0] + i - fd.start[0], cd.start[1] + j - fd.start[1],
                                  cd.start[2] + k - fd.start[2]};
            out[idx++] = rs[fd.offset + p[0] + fd.count[0] * (p[1] + fd.count[1] * p[2])];
          }
    }
  }
  gym_space_destroy(full);
  return out;
}

std::vector<double> lumped_diag_host(const gym_space* sp, bool curved_exact) {
  const gym_mesh* m = sp->mesh;
  const SpaceDesc& s = sp->desc;
  if (s.periodic) return periodic_diag_host(sp, true);
  if (m->curved && curved_exact) return curved_rowsums(sp);
  const LumpedTables t = lumped_tables_host(sp);
  std::vector<double> out(s.ndofs);
  for (int c = 0; c < s.ncomp; ++c) {
    const CompDesc& cd = s.comp[c];
    int64_t idx = cd.offset;
    for (int64_t k = 0; k < cd.count[2]; ++k)
      for (int64_t j = 0; j < cd.count[1]; ++j)
        for (int64_t i = 0; i < cd.count[0]; ++i) {
          int64_t p[3] = {cd.start[0] + i, cd.start[1] + j, cd.start[2] + k};
          double v = t.sc[c];
          for (int a = 0; a < m->dim; ++a) v *= (cd.nodal_mask >> a & 1) ? t.rn[a][p[a]] : t.re[a][p[a]];
          out[idx++] = v;
        }
  }
  return out;
}

int ensure_mass_work(gym_space* sp, int nrhs, MassWork** out) {
  if (!sp->work.empty() && sp->work_nrhs == nrhs) {
    *out = (MassWork*)sp->work[0];
    return 0;
  }
  if (!sp->work.empty()) {
    MassWork* old = (MassWork*)sp->work[0];
    for (void* p : old->pool) (void)hipFree(p);
    if (old->host) (void)hipHostFree(old->host);
    delete old;
    sp->work.clear();
  }
  const long long n = sp->desc.ndofs;
  MassWork* w = new MassWork;
  sp->work.push_back(w);
  sp->work_nrhs = nrhs;
  w->nrhs = nrhs;
  w->nb = vec_grid(n, sp->ctx->ncu);
  double** vecs[3] = {&w->r, &w->p, &w->q};
  for (double** v : vecs) {
    void* p;
    if (int rc = dalloc(&p, sizeof(double) * n * nrhs)) return rc;
    w->pool.push_back(p);
    *v = (double*)p;
  }
  void* p;
  if (int rc = dalloc(&p, sizeof(double) * (2 * w->nb * nrhs + 2 * nrhs))) return rc;
  w->pool.push_back(p);
  w->pa = (double*)p;
  w->pb = w->pa + w->nb * nrhs;
  w->sums = w->pb + w->nb * nrhs;
  if (int rc = dalloc(&p, sizeof(CgState) * 2 * nrhs)) return rc;
  w->pool.push_back(p);
  w->st = (CgState*)p;
  GYM_HIP(hipHostMalloc((void**)&w->host, sizeof(CgState) * 2 * nrhs, hipHostMallocDefault));
  if (!sp->d_diag) {
    std::vector<double> d = mass_diag_host(sp);
    for (double& v : d) v = 1.0 / v;
    if (int rc = dalloc((void**)&sp->d_diag, sizeof(double) * n)) return rc;
    GYM_HIP(hipMemcpy(sp->d_diag, d.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  }
  *out = w;
  return 0;
}

}  // namespace gym

using namespace gym;

extern "C" {

const char* gym_last_error(void) { return g_err.c_str(); }

int gym_create(gym_ctx** out, int device) {
  if (!out) return fail(GYM_E_ARG, "out is NULL");
  int n = 0;
  GYM_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(GYM_E_ARG, "no HIP device " + std::to_string(device));
  GYM_HIP(hipSetDevice(device));
  gym_ctx* c = new gym_ctx;
  c->device = device;
  GYM_HIP(hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device));
  if (int rc = upload_tables()) {
    delete c;
    return rc;
  }
  if (int rc = noalloc_init(device)) {
    delete c;
    return rc;
  }
  *out = c;
  return GYM_OK;
}

int gym_destroy(gym_ctx* ctx) {
  delete ctx;
  return GYM_OK;
}

int gym_ctx_set(gym_ctx* ctx, int option, int value) {
  if (!ctx) return fail(GYM_E_ARG, "NULL context");
  if (option == GYM_OPT_MASS_FORM && (value == 0 || value == 1)) {
    ctx->mass_form = value;
    return GYM_OK;
  }
  if (option == GYM_OPT_TILE && value >= 0 && value <= 2) {
    ctx->tile = value;
    return GYM_OK;
  }
  if (option == GYM_OPT_CURVED_KERNEL && (value == 0 || value == 1)) {
    ctx->curved_kernel = value;
    return GYM_OK;
  }
  return fail(GYM_E_ARG, "unknown option or value");
}

int gym_mesh_create(gym_ctx* ctx, int dim, const int64_t nel[3], const double* vertices, const double lo[3],
                    const double hi[3], gym_mesh** out) {
  if (!ctx || !out || !nel) return fail(GYM_E_ARG, "NULL argument");
  if (dim != 2 && dim != 3) return fail(GYM_E_ARG, "dim must be 2 or 3");
  gym_mesh* m = new gym_mesh;
  m->ctx = ctx;
  m->dim = dim;
  int64_t nv = 1;
  for (int a = 0; a < 3; ++a) {
    m->nel[a] = a < dim ? nel[a] : 1;
    if (m->nel[a] < 1 || m->nel[a] > (1 << 20)) {
      delete m;
      return fail(GYM_E_ARG, "nel out of range");
    }
    m->lo[a] = lo ? lo[a] : 0.0;
    m->hi[a] = hi ? hi[a] : 1.0;
    if (a < dim && !(m->hi[a] > m->lo[a])) {
      delete m;
      return fail(GYM_E_ARG, "hi must exceed lo");
    }
    m->h[a] = a < dim ? (m->hi[a] - m->lo[a]) / m->nel[a] : 1.0;
    if (a < dim) nv *= m->nel[a] + 1;
  }
  if (vertices) {
    m->curved = true;
    m->vertices.assign(vertices, vertices + nv * dim);
    if (int rc = check_mesh_jacobians(m)) {
      delete m;
      return rc;
    }
    // 16 doubles of zero padding: the matrix-core Hodge kernel reads vertex
    // rows in 128-byte pieces that may run past the last vertex
    if (int rc = dalloc((void**)&m->d_vertices, sizeof(double) * (nv * dim + 16))) {
      delete m;
      return rc;
    }
    hipError_t e = hipMemcpy(m->d_vertices, vertices, sizeof(double) * nv * dim, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->d_vertices + nv * dim, 0, sizeof(double) * 16);
    if (e != hipSuccess) {
      (void)hipFree(m->d_vertices);
      delete m;
      return hip_fail(e, "hipMemcpy vertices");
    }
  }
  *out = m;
  return GYM_OK;
}

int gym_mesh_structured(gym_ctx* ctx, int dim, const int64_t nel[3], const double lo[3], const double hi[3],
                        double perturb_frac, uint64_t seed, gym_mesh** out) {
  if (!ctx || !out || !nel) return fail(GYM_E_ARG, "NULL argument");
  if (dim != 2 && dim != 3) return fail(GYM_E_ARG, "dim must be 2 or 3");
  if (!(perturb_frac >= 0.0 && perturb_frac < 0.5)) return fail(GYM_E_ARG, "perturb_frac must be in [0, 0.5)");
  if (perturb_frac == 0.0) return gym_mesh_create(ctx, dim, nel, nullptr, lo, hi, out);
  int64_t n[3] = {1, 1, 1};
  double L[3] = {0, 0, 0}, H[3] = {1, 1, 1};
  int64_t nv = 1;
  for (int a = 0; a < dim; ++a) {
    n[a] = nel[a];
    if (n[a] < 1 || n[a] > (1 << 20)) return fail(GYM_E_ARG, "nel out of range");
    L[a] = lo ? lo[a] : 0.0;
    H[a] = hi ? hi[a] : 1.0;
    if (!(H[a] > L[a])) return fail(GYM_E_ARG, "hi must exceed lo");
    nv *= n[a] + 1;
  }
  std::vector<double> v;
  try {
    v.resize((size_t)nv * dim);
  } catch (const std::bad_alloc&) {
    return fail(GYM_E_OOM, "host vertex array");
  }
  // SplitMix64 word w of stream `seed`, mapped to [0, 1) with 53 bits
  auto uniform = [seed](uint64_t w) {
    uint64_t z = seed + (w + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
  };
  for (int64_t k = 0; k < (dim == 3 ? n[2] + 1 : 1); ++k)
    for (int64_t j = 0; j <= n[1]; ++j)
      for (int64_t i = 0; i <= n[0]; ++i) {
        const int64_t vid = i + (n[0] + 1) * (j + (n[1] + 1) * k);
        const int64_t idx[3] = {i, j, k};
        for (int a = 0; a < dim; ++a) {
          double x = L[a] + ((H[a] - L[a]) * (double)idx[a]) / (double)n[a];
          if (idx[a] > 0 && idx[a] < n[a]) {
            const double h = (H[a] - L[a]) / (double)n[a];
            x += (2.0 * uniform((uint64_t)(dim * vid + a)) - 1.0) * (perturb_frac * h);
          }
          v[(size_t)vid * dim + a] = x;
        }
      }
  return gym_mesh_create(ctx, dim, n, v.data(), L, H, out);
}

int gym_mesh_vertices(const gym_mesh* m, double* out) {
  if (!m || !out) return fail(GYM_E_ARG, "NULL argument");
  const int d = m->dim;
  if (m->curved) {
    std::copy(m->vertices.begin(), m->vertices.end(), out);
    return GYM_OK;
  }
  const int64_t nx = m->nel[0], ny = m->nel[1], nz = d == 3 ? m->nel[2] : 0;
  for (int64_t k = 0; k <= nz; ++k)
    for (int64_t j = 0; j <= ny; ++j)
      for (int64_t i = 0; i <= nx; ++i) {
        const int64_t idx[3] = {i, j, k};
        const int64_t vid = i + (nx + 1) * (j + (ny + 1) * k);
        for (int a = 0; a < d; ++a)
          out[vid * d + a] = m->lo[a] + ((m->hi[a] - m->lo[a]) * (double)idx[a]) / (double)m->nel[a];
      }
  return GYM_OK;
}

int gym_mesh_set_periodic(gym_mesh* m, int mask) {
  if (!m) return fail(GYM_E_ARG, "NULL argument");
  if (mask < 0 || mask >= (1 << m->dim)) return fail(GYM_E_ARG, "periodic mask has bits beyond the mesh dimension");
  if (mask && m->curved) return fail(GYM_E_UNSUPPORTED, "periodic axes need an affine box");
  m->periodic = mask;
  return GYM_OK;
}

int gym_mesh_destroy(gym_mesh* m) {
  if (!m) return GYM_OK;
  if (m->d_vertices) (void)hipFree(m->d_vertices);
  for (auto& per_prec : m->qd)
    for (void* q : per_prec)
      if (q) (void)hipFree(q);
  delete m;
  return GYM_OK;
}

int gym_space_create(gym_ctx* ctx, const gym_mesh* mesh, int kind, int degree, int bc, gym_space** out) {
  if (!ctx || !mesh || !out) return fail(GYM_E_ARG, "NULL argument");
  if (kind < GYM_H1 || kind > GYM_L2) return fail(GYM_E_ARG, "bad space kind");
  if (degree < 1 || degree > kMaxR) return fail(GYM_E_ARG, "degree must be 1..4");
  if (bc != GYM_BC_NATURAL && bc != GYM_BC_ESSENTIAL) return fail(GYM_E_ARG, "bad bc");
  gym_space* s = new gym_space;
  s->ctx = ctx;
  s->mesh = mesh;
  s->desc = make_space_desc(kind, mesh->dim, mesh->nel, degree, bc, mesh->periodic);
  *out = s;
  return GYM_OK;
}

int64_t gym_space_ndofs(const gym_space* s) { return s ? s->desc.ndofs : -1; }

int gym_space_layout(const gym_space* s, gym_layout* out) {
  if (!s || !out) return fail(GYM_E_ARG, "NULL argument");
  const SpaceDesc& d = s->desc;
  gym_layout L{};
  L.kind = d.kind;
  L.dim = d.dim;
  L.degree = d.r;
  L.bc = d.bc;
  L.ncomp = d.ncomp;
  for (int a = 0; a < 3; ++a) L.m[a] = a < d.dim ? d.m[a] : 1;
  for (int c = 0; c < 3; ++c) {
    if (c < d.ncomp) {
      L.nodal_mask[c] = d.comp[c].nodal_mask;
      L.offset[c] = d.comp[c].offset;
      for (int a = 0; a < 3; ++a) {
        L.start[c][a] = a < d.dim ? d.comp[c].start[a] : 0;
        L.count[c][a] = a < d.dim ? d.comp[c].count[a] : 1;
      }
    } else {
      L.offset[c] = d.ndofs;
      for (int a = 0; a < 3; ++a) L.count[c][a] = 0;
    }
  }
  L.ndofs = d.ndofs;
  *out = L;
  return GYM_OK;
}

int gym_space_destroy(gym_space* s) {
  if (!s) return GYM_OK;
  if (s->d_diag) (void)hipFree(s->d_diag);
  if (s->band_mem) (void)hipFree(s->band_mem);
  delete static_cast<SpaiParams*>(s->band);
  if (!s->work.empty()) {
    MassWork* w = (MassWork*)s->work[0];
    for (void* p : w->pool) (void)hipFree(p);
    if (w->host) (void)hipHostFree(w->host);
    delete w;
  }
  delete s;
  return GYM_OK;
}

int gym_d_apply(const gym_space* from, const gym_space* to, int transpose, const double* x, double* y,
                void* stream) {
  return d_apply_n(from, to, transpose, 1, x, y, (hipStream_t)stream);
}

}  // extern "C"

namespace gym {

int d_apply_n(const gym_space* from, const gym_space* to, int transpose, int nrhs, const double* x, double* y,
              hipStream_t stream) {
  if (!from || !to || !x || !y || nrhs < 1) return fail(GYM_E_ARG, "NULL argument or nrhs < 1");
  if (from->mesh != to->mesh || from->desc.r != to->desc.r)
    return fail(GYM_E_ARG, "spaces on different meshes or degrees");
  const int dim = from->desc.dim;
  int op = -1;
  int fk = from->desc.kind, tk = to->desc.kind;
  if (fk == GYM_H1 && tk == GYM_HCURL) op = 0;
  else if (fk == GYM_HCURL && tk == (dim == 3 ? GYM_HDIV : GYM_L2)) op = 1;
  else if (fk == GYM_HDIV && tk == GYM_L2) op = 2;
  if (op < 0) return fail(GYM_E_ARG, "spaces are not consecutive in the de Rham complex");
  IncParams p{};
  p.x = x;
  p.y = y;
  const gym_space* src = transpose ? to : from;
  const gym_space* dst = transpose ? from : to;
  p.in = to_dev(src->desc, 0);
  p.out = to_dev(dst->desc, 0);
  p.in_ncomp = src->desc.ncomp;
  p.out_ncomp = dst->desc.ncomp;
  p.dim = dim;
  p.op = op;
  p.transpose = transpose ? 1 : 0;
  p.periodic = from->desc.periodic;
  p.nout = dst->desc.ndofs;
  p.nrhs = nrhs;
  p.in_stride = src->desc.ndofs;
  p.out_stride = dst->desc.ndofs;
  int rc = launch_incidence(p, stream);
  if (rc) return fail(GYM_E_HIP, "incidence launch failed");
  return GYM_OK;
}

}  // namespace gym

extern "C" {

int gym_mass_apply(const gym_space* space, int prec, int nrhs, const void* x, void* y, void* stream) {
  if (!space || !x || !y || nrhs < 1) return fail(GYM_E_ARG, "bad argument");
  if (prec != GYM_F64 && prec != GYM_F32 && prec != GYM_BF16) return fail(GYM_E_ARG, "unknown precision");
  return launch_mass_apply(space, prec, nrhs, x, y, (hipStream_t)stream);
}

int gym_op_create(gym_ctx* ctx, int problem, const gym_mesh* mesh, int degree, gym_op** out) {
  if (!ctx || !mesh || !out) return fail(GYM_E_ARG, "NULL argument");
  if (degree < 1 || degree > kMaxR) return fail(GYM_E_ARG, "degree must be 1..4");
  if (problem != GYM_MIXED_POISSON && problem != GYM_HODGE1) return fail(GYM_E_ARG, "unknown problem");
  if (problem == GYM_HODGE1 && mesh->dim != 3) return fail(GYM_E_UNSUPPORTED, "Hodge problem is 3-D only");
  if (mesh->periodic)
    return fail(GYM_E_UNSUPPORTED, "periodic meshes serve the time stepping and its eigenmodes, not the operators");
  gym_op* op = new gym_op;
  op->ctx = ctx;
  op->mesh = mesh;
  op->problem = problem;
  op->r = degree;
  if (problem == GYM_MIXED_POISSON) {
    op->sa = make_space_desc(GYM_HDIV, mesh->dim, mesh->nel, degree, GYM_BC_NATURAL);
    op->sb = make_space_desc(GYM_L2, mesh->dim, mesh->nel, degree, GYM_BC_NATURAL);
  } else {
    op->sa = make_space_desc(GYM_H1, mesh->dim, mesh->nel, degree, GYM_BC_ESSENTIAL);
    op->sb = make_space_desc(GYM_HCURL, mesh->dim, mesh->nel, degree, GYM_BC_ESSENTIAL);
  }
  op->na = op->sa.ndofs;
  op->nb = op->sb.ndofs;
  if (mesh->curved && mesh->dim == 3) {
    // the FP64 Gauss-point metrics now rather than inside the first apply
    const void* q;
    if (int rc = mesh_qdata(mesh, degree, 0, &q)) {
      delete op;
      return rc;
    }
  }
  std::vector<double> d = precond_diag_host(op);
  for (double& v : d) v = 1.0 / v;
  if (int rc = dalloc((void**)&op->d_prec, sizeof(double) * d.size())) {
    delete op;
    return rc;
  }
  hipError_t e = hipMemcpy(op->d_prec, d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(op->d_prec);
    delete op;
    return hip_fail(e, "hipMemcpy preconditioner");
  }
  *out = op;
  return GYM_OK;
}

int64_t gym_op_ndofs(const gym_op* op) { return op ? op->na + op->nb : -1; }

int gym_op_block_sizes(const gym_op* op, int64_t n[2]) {
  if (!op || !n) return fail(GYM_E_ARG, "NULL argument");
  n[0] = op->na;
  n[1] = op->nb;
  return GYM_OK;
}

static void free_work(gym_op* op) {
  if (op->work.empty()) return;
  OpWork* w = (OpWork*)op->work[0];
  for (void* p : w->pool) (void)hipFree(p);
  if (w->m64.host) (void)hipHostFree(w->m64.host);
  if (w->m32.host) (void)hipHostFree(w->m32.host);
  delete w;
  op->work.clear();
  op->work_nrhs = 0;
}

int gym_op_destroy(gym_op* op) {
  if (!op) return GYM_OK;
  free_work(op);
  if (op->schur) {
    schur_free(static_cast<SchurPrec*>(op->schur));
    delete static_cast<SchurPrec*>(op->schur);
  }
  if (op->mfma) {
    MfmaState* st = static_cast<MfmaState*>(op->mfma);
    if (st->frag) (void)hipFree(st->frag);
    if (st->yel) (void)hipFree(st->yel);
    delete st;
  }
  if (op->hc_halo) (void)hipFree(op->hc_halo);
  if (op->d_prec) (void)hipFree(op->d_prec);
  delete op;
  return GYM_OK;
}

int gym_op_apply(const gym_op* op, int prec, int nrhs, const void* x, void* y, void* stream) {
  if (!op || !x || !y || nrhs < 1) return fail(GYM_E_ARG, "bad argument");
  if (prec != GYM_F64 && prec != GYM_F32 && prec != GYM_BF16) return fail(GYM_E_ARG, "unknown precision");
  return launch_op_apply(op, prec, nrhs, x, y, (hipStream_t)stream);
}

int gym_op_precond_apply(gym_op* op, int precond, int nrhs, const double* y, double* z, void* stream) {
  if (!op || !y || !z || nrhs < 1) return fail(GYM_E_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  const long long n = op->na + op->nb;
  const int nb = vec_grid(n, op->ctx->ncu);
  if (precond == GYM_PRECOND_JACOBI) {
    for (int r = 0; r < nrhs; ++r) launch_axpy_diag(z + n * r, 0.0, 1.0, op->d_prec, y + n * r, n, nb, s);
    GYM_HIP(hipGetLastError());
    return GYM_OK;
  }
  if (precond != GYM_PRECOND_SCHUR) return fail(GYM_E_ARG, "unknown preconditioner");
  SchurPrec* P;
  if (int rc = ensure_schur(op, nrhs, &P)) return rc;
  if (launch_schur_apply<double>(*P, y, z, nrhs, nb, s)) return fail(GYM_E_HIP, "preconditioner launch");
  return GYM_OK;
}

int gym_op_precond_diag(const gym_op* op, double* diag, void* stream) {
  if (!op || !diag) return fail(GYM_E_ARG, "NULL argument");
  std::vector<double> d = precond_diag_host(op);
  GYM_HIP(hipMemcpyAsync(diag, d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice, (hipStream_t)stream));
  GYM_HIP(hipStreamSynchronize((hipStream_t)stream));
  return GYM_OK;
}

int gym_rhs_manufactured(const gym_op* op, int nmodes, const int* modes, const double* coeffs, double* b,
                         void* stream) {
  if (!op || !b || (nmodes > 0 && (!modes || !coeffs))) return fail(GYM_E_ARG, "bad argument");
  const gym_mesh* m = op->mesh;
  if (m->curved) return fail(GYM_E_UNSUPPORTED, "manufactured loads need an affine mesh");
  const int dim = m->dim, r = op->r, q = r + 2;
  const double pi = 3.14159265358979323846;
  Tables1D t = make_tables(r, q);
  // 1-D load factors: L[a][type][p] = int_axis g(x) b_p(x) dx over the
  // reference coordinate (h folded in by the caller), for g = sin or cos.
  auto load1d = [&](int a, bool nodal, bool use_cos, int k) {
    int64_t nel = m->nel[a], mm = r * nel;
    std::vector<double> out(nodal ? mm + 1 : mm, 0.0);
    for (int64_t e = 0; e < nel; ++e)
      for (int s = 0; s < q; ++s) {
        double x = m->lo[a] + m->h[a] * (e + t.gx[s]);
        double g = use_cos ? std::cos(k * pi * x) : std::sin(k * pi * x);
        double wg = t.gw[s] * g;
        if (nodal)
          for (int i = 0; i <= r; ++i) out[r * e + i] += wg * t.phi[s * (r + 1) + i];
        else
          for (int j = 0; j < r; ++j) out[r * e + j] += wg * t.edge[s * r + j];
      }
    return out;
  };
  std::vector<double> h(op->na + op->nb, 0.0);
  const SpaceDesc& sd = op->sb;
  double det = 1.0;
  for (int a = 0; a < dim; ++a) det *= m->h[a];
  for (int md = 0; md < nmodes; ++md) {
    const int* k = modes + md * dim;
    double k2 = 0;
    for (int a = 0; a < dim; ++a) k2 += double(k[a]) * k[a];
    for (int c = 0; c < sd.ncomp; ++c) {
      const CompDesc& cd = sd.comp[c];
      double coef;
      std::vector<double> L[3];
      if (op->problem == GYM_MIXED_POISSON) {
        // f = c pi^2 |k|^2 prod sin; L2 basis: F_i = int f b_i (reference cell)
        coef = -coeffs[md] * pi * pi * k2;  // the load enters as -F
        for (int a = 0; a < dim; ++a) L[a] = load1d(a, false, false, k[a]);
      } else {
        // f_c = c_c pi^2 |k|^2 cos(k_c pi x_c) prod_{b != c} sin(k_b pi x_b);
        // HCURL basis (covariant): F_i = det/h_c * prod_a int g_a b_a
        coef = coeffs[md * 3 + c] * pi * pi * k2 * det / m->h[c];
        for (int a = 0; a < dim; ++a) L[a] = load1d(a, (cd.nodal_mask >> a) & 1, a == c, k[a]);
      }
      int64_t idx = op->na + cd.offset;
      for (int64_t kk = 0; kk < cd.count[2]; ++kk)
        for (int64_t jj = 0; jj < cd.count[1]; ++jj)
          for (int64_t ii = 0; ii < cd.count[0]; ++ii) {
            double v = coef * L[0][cd.start[0] + ii] * L[1][cd.start[1] + jj];
            if (dim == 3) v *= L[2][cd.start[2] + kk];
            h[idx++] += v;
          }
    }
  }
  GYM_HIP(hipMemcpyAsync(b, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, (hipStream_t)stream));
  GYM_HIP(hipStreamSynchronize((hipStream_t)stream));
  return GYM_OK;
}

void gym_solve_opts_default(gym_solve_opts* o) {
  if (!o) return;
  o->method = GYM_MINRES;
  o->mode = GYM_MODE_F64;
  o->rtol = 1e-10;
  o->maxit = 20000;
  o->inner_rtol = 1e-4;
  o->max_outer = 30;
  o->check_every = 25;
  o->timing = 0;
  o->precond = GYM_PRECOND_JACOBI;
}

static int ensure_work(gym_op* op, int nrhs, OpWork** out) {
  long long n = op->na + op->nb;
  if (!op->work.empty() && op->work_nrhs == nrhs) {
    *out = (OpWork*)op->work[0];
    return 0;
  }
  free_work(op);
  OpWork* w = new OpWork;
  op->work.push_back(w);
  op->work_nrhs = nrhs;
  w->n = n;
  w->nrhs = nrhs;
  w->nb = vec_grid(n, op->ctx->ncu);
  if (int rc = alloc_minres<double>(w->pool, w->m64, n, nrhs)) return rc;
  void* p;
  if (int rc = dalloc(&p, sizeof(double) * n * nrhs * 3)) return rc;
  w->pool.push_back(p);
  w->tmp = (double*)p;
  w->r64 = w->tmp + n * nrhs;
  w->d64 = w->r64 + n * nrhs;
  if (int rc = dalloc(&p, sizeof(double) * (w->nb * nrhs + 4 * nrhs))) return rc;
  w->pool.push_back(p);
  w->part = (double*)p;
  w->sums = w->part + w->nb * nrhs;
  w->scale = w->sums + 2 * nrhs;
  *out = w;
  return 0;
}

static int ensure_work32(gym_op* op, OpWork* w) {
  if (w->r32) return 0;
  if (int rc = alloc_minres<float>(w->pool, w->m32, w->n, w->nrhs)) return rc;
  void* p;
  if (int rc = dalloc(&p, sizeof(float) * w->n * w->nrhs * 2)) return rc;
  w->pool.push_back(p);
  w->r32 = (float*)p;
  w->x32 = w->r32 + w->n * w->nrhs;
  return 0;
}

// FP64 mode of gym_solve on the workspace w (the operator's pool, or the
// static scratch array of gym_solve_noalloc): preconditioned MINRES, then the
// true FP64 residual; restarts on the residual while the preconditioned
// estimate was optimistic.  Allocates no device memory.
static int minres_f64(gym_op* op, const gym_solve_opts& opts, int nrhs, const double* b, double* x, OpWork& w,
                      int npa, const double* dinv, ApplyTimer& timer, hipStream_t s, int* iters, int* status,
                      std::vector<double>& rel, const PrecFn<double>* ext = nullptr) {
  const long long n = w.n;
  auto apply = [&](const double* in, double* out, const MrStep& m) {
    if (int rc = timer.begin(s)) return rc;
    if (int rc = launch_op_apply(op, GYM_F64, nrhs, in, out, s, &m, w.matrix_core)) return rc;
    return timer.end(s);
  };
  double tol = opts.rtol;
  int total = 0, flag = 0;
  const double* rhs = b;
  double* sol = x;
  *status = GYM_OK;
  for (int attempt = 0; attempt < 6; ++attempt) {
    int it = 0;
    if (int rc = run_minres<double>(apply, n, nrhs, w.nb, npa, rhs, sol, dinv, tol, opts.maxit - total,
                                    opts.check_every, w.m64, s, &it, &flag, ext))
      return rc;
    total += it;
    if (flag < 0) {
      *status = fail(GYM_E_BREAKDOWN, "MINRES breakdown (NaN or indefinite preconditioner)");
      break;
    }
    if (sol != x) launch_add(sol, x, n * nrhs, w.nb, s);
    if (int rc = relres_f64(op, nrhs, b, x, w.tmp, w.part, w.sums, w.nb, s, rel, nullptr, w.matrix_core)) return rc;
    double worst = *std::max_element(rel.begin(), rel.end());
    if (worst <= opts.rtol) break;
    if (total >= opts.maxit) {
      *status = GYM_W_NOT_CONVERGED;
      break;
    }
    // the preconditioned estimate was optimistic: restart on the true
    // residual, A d = b - A x (zero for right-hand sides already within
    // rtol), with the tolerance that brings the worst one below rtol
    launch_sub(b, w.tmp, w.r64, n * nrhs, w.nb, s);
    for (int r = 0; r < nrhs; ++r)
      if (rel[r] <= opts.rtol) launch_fill(w.r64 + n * r, 0.0, n, w.nb, s);
    tol = std::min(0.5, 0.3 * opts.rtol / worst);
    rhs = w.r64;
    sol = w.d64;
  }
  *iters = total;
  return 0;
}

int gym_solve(gym_op* op, const gym_solve_opts* opts_in, int nrhs, const double* b, double* x,
              gym_solve_info* info, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  if (!op || !b || !x || nrhs < 1) return fail(GYM_E_ARG, "bad argument");
  gym_solve_opts opts;
  if (opts_in) opts = *opts_in;
  else gym_solve_opts_default(&opts);
  gym_solve_info inf{};
  hipStream_t s = (hipStream_t)stream;
  if (opts.method != GYM_MINRES) return fail(GYM_E_UNSUPPORTED, "block operators are indefinite: use MINRES");
  if (opts.precond != GYM_PRECOND_JACOBI && opts.precond != GYM_PRECOND_NONE && opts.precond != GYM_PRECOND_SCHUR)
    return fail(GYM_E_ARG, "unknown preconditioner");
  OpWork* w;
  if (int rc = ensure_work(op, nrhs, &w)) return rc;
  SchurPrec* schur = nullptr;
  if (opts.precond == GYM_PRECOND_SCHUR)
    if (int rc = ensure_schur(op, nrhs, &schur)) return rc;
  const PrecFn<double> ext64 = [&](const double* in, double* out, const MinresState* gate) {
    return launch_schur_apply<double>(*schur, in, out, nrhs, w->nb, s, gate)
               ? fail(GYM_E_HIP, "preconditioner launch")
               : 0;
  };
  const PrecFn<float> ext32 = [&](const float* in, float* out, const MinresState* gate) {
    return launch_schur_apply<float>(*schur, in, out, nrhs, w->nb, s, gate) ? fail(GYM_E_HIP, "preconditioner launch")
                                                                            : 0;
  };
  const long long n = w->n;
  const double* dinv = op->d_prec;
  if (opts.precond == GYM_PRECOND_NONE) {
    if (!w->ones) {
      void* p;
      if (int rc = dalloc(&p, sizeof(double) * n)) return rc;
      w->pool.push_back(p);
      w->ones = (double*)p;
      launch_fill(w->ones, 1.0, n, w->nb, s);
    }
    dinv = w->ones;
  }
  std::vector<double> rel;
  int status = GYM_OK;
  ApplyTimer timer;
  timer.period = opts.timing > 0 ? opts.timing : 0;
  if (opts.mode == GYM_MODE_F64) {
    int npa = 0;
    if (int rc = op_workgroups(op, GYM_F64, nrhs, &npa)) return rc;
    if (int rc = ensure_partials(w->pool, w->m64, npa, w->nb, nrhs)) return rc;
    if (int rc = minres_f64(op, opts, nrhs, b, x, *w, npa, schur ? nullptr : dinv, timer, s, &inf.iters, &status,
                            rel, schur ? &ext64 : nullptr))
      return rc;
  } else if (opts.mode == GYM_MODE_IR_F32 || opts.mode == GYM_MODE_IR_BF16) {
    if (int rc = ensure_work32(op, w)) return rc;
    const int prec = opts.mode == GYM_MODE_IR_BF16 ? GYM_BF16 : GYM_F32;
    auto apply32 = [&](const float* in, float* out, const MrStep& m) {
      if (int rc = timer.begin(s)) return rc;
      if (int rc = launch_op_apply(op, prec, nrhs, in, out, s, &m)) return rc;
      return timer.end(s);
    };
    int npa = 0;
    if (int rc = op_workgroups(op, prec, nrhs, &npa)) return rc;
    if (int rc = ensure_partials(w->pool, w->m32, npa, w->nb, nrhs)) return rc;
    GYM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n * nrhs, s));
    int total = 0, outer = 0;
    std::vector<double> rn;
    if (int rc = relres_f64(op, nrhs, b, x, w->tmp, w->part, w->sums, w->nb, s, rel, &rn)) return rc;
    status = GYM_W_NOT_CONVERGED;
    for (outer = 0; outer < opts.max_outer; ++outer) {
      double worst = *std::max_element(rel.begin(), rel.end());
      if (worst <= opts.rtol) {
        status = GYM_OK;
        break;
      }
      // r64 = b - A x (tmp holds A x); scale each rhs to unit norm in FP32
      launch_sub(b, w->tmp, w->r64, n * nrhs, w->nb, s);
      std::vector<double> sc(2 * nrhs);
      for (int r = 0; r < nrhs; ++r) {
        sc[r] = rn[r] > 0 ? 1.0 / rn[r] : 0.0;
        sc[nrhs + r] = rn[r];
      }
      GYM_HIP(hipMemcpyAsync(w->scale, sc.data(), sizeof(double) * 2 * nrhs, hipMemcpyHostToDevice, s));
      launch_to_f32_scaled(w->r64, w->r32, n, nrhs, w->nb, w->scale, s);
      int it = 0, flag = 0;
      if (int rc = run_minres<float>(apply32, n, nrhs, w->nb, npa, w->r32, w->x32, schur ? nullptr : dinv,
                                     opts.inner_rtol, opts.maxit, opts.check_every, w->m32, s, &it, &flag,
                                     schur ? &ext32 : nullptr))
        return rc;
      total += it;
      if (flag < 0) {
        status = fail(GYM_E_BREAKDOWN, "inner MINRES breakdown");
        break;
      }
      launch_axpy_f32(w->x32, x, n, nrhs, w->nb, w->scale + nrhs, s);
      if (int rc = relres_f64(op, nrhs, b, x, w->tmp, w->part, w->sums, w->nb, s, rel, &rn)) return rc;
    }
    inf.iters = total;
    inf.outer_iters = outer;
  } else {
    return fail(GYM_E_ARG, "unknown solve mode");
  }
  if (rel.empty())
    if (int rc = relres_f64(op, nrhs, b, x, w->tmp, w->part, w->sums, w->nb, s, rel)) return rc;
  inf.rel_res = *std::max_element(rel.begin(), rel.end());
  if (status == GYM_OK && inf.rel_res > opts.rtol) status = GYM_W_NOT_CONVERGED;
  GYM_HIP(hipStreamSynchronize(s));
  if (int rc = timer.collect(&inf.applies, &inf.apply_ms)) return rc;
  inf.status = status;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

}  // extern "C"

namespace gym {

// FP64 solve on caller-provided device memory `base` of `bytes` bytes (the
// static scratch array of gym_solve_noalloc): the workspace of gym_solve's
// FP64 mode is carved from it, so nothing is allocated on the device.
int solve_f64_on(gym_op* op, const gym_solve_opts* opts_in, int nrhs, const double* b, double* x,
                 gym_solve_info* info, hipStream_t s, void* base, size_t bytes, MinresState* host_states,
                 int max_rhs) {
  auto t0 = std::chrono::steady_clock::now();
  if (!op || !b || !x || nrhs < 1) return fail(GYM_E_ARG, "bad argument");
  if (nrhs > max_rhs) return fail(GYM_E_ARG, "nrhs exceeds " + std::to_string(max_rhs));
  if (!base) return fail(GYM_E_HIP, "scratch array not set up on this device");
  gym_solve_opts opts;
  if (opts_in) opts = *opts_in;
  else gym_solve_opts_default(&opts);
  if (opts.method != GYM_MINRES) return fail(GYM_E_UNSUPPORTED, "block operators are indefinite: use MINRES");
  if (opts.mode != GYM_MODE_F64) return fail(GYM_E_UNSUPPORTED, "the allocation-free solve runs in FP64 mode only");
  if (opts.precond == GYM_PRECOND_SCHUR)
    return fail(GYM_E_UNSUPPORTED, "the allocation-free solve takes the diagonal preconditioners only");
  if (opts.precond != GYM_PRECOND_JACOBI && opts.precond != GYM_PRECOND_NONE)
    return fail(GYM_E_ARG, "unknown preconditioner");
  const long long n = op->na + op->nb;
  int npa = 0;
  if (int rc = op_workgroups(op, GYM_F64, nrhs, &npa, false)) return rc;
  OpWork w;
  w.matrix_core = false;
  w.n = n;
  w.nrhs = nrhs;
  w.nb = vec_grid(n, op->ctx->ncu);
  // carve: 256-byte aligned pieces, in doubles
  char* p = static_cast<char*>(base);
  size_t used = 0;
  bool fits = true;
  auto take = [&](long long count) -> double* {
    const size_t sz = ((size_t)count * sizeof(double) + 255) & ~(size_t)255;
    if (used + sz > bytes) {
      fits = false;
      return nullptr;
    }
    double* q = reinterpret_cast<double*>(p + used);
    used += sz;
    return q;
  };
  const long long nv = n * nrhs;
  double** vecs[8] = {&w.m64.r1, &w.m64.r2, &w.m64.y, &w.m64.z, &w.m64.zp, &w.m64.w, &w.m64.w1, &w.m64.w2};
  for (double** v : vecs) *v = take(nv);
  w.tmp = take(nv);
  w.r64 = take(nv);
  w.d64 = take(nv);
  w.ones = opts.precond == GYM_PRECOND_NONE ? take(n) : nullptr;
  w.m64.pa = take((long long)npa * nrhs);
  for (int k = 0; k < 2; ++k) {
    w.m64.pb[k] = take((long long)w.nb * nrhs);
    w.m64.pc[k] = take((long long)w.nb * nrhs);
    w.m64.alfa[k] = take(nrhs);
  }
  w.m64.npa_cap = npa;
  w.part = take((long long)w.nb * nrhs);
  w.sums = take(4LL * nrhs);
  w.scale = w.sums + 2 * nrhs;
  w.m64.st = reinterpret_cast<MinresState*>(take((long long)(sizeof(MinresState) * 2 * nrhs + 7) / 8));
  if (!fits)
    return fail(GYM_E_ARG, "problem too large for the allocation-free solve: needs more than " +
                               std::to_string(bytes) + " bytes of scratch (" + std::to_string(n) + " unknowns x " +
                               std::to_string(nrhs) + " rhs)");
  w.m64.host = host_states;
  const double* dinv = op->d_prec;
  if (w.ones) {
    launch_fill(w.ones, 1.0, n, w.nb, s);
    dinv = w.ones;
  }
  ApplyTimer timer;  // no HIP events here: timing is off
  gym_solve_info inf{};
  std::vector<double> rel;
  int status = GYM_OK;
  int rc = minres_f64(op, opts, nrhs, b, x, w, npa, dinv, timer, s, &inf.iters, &status, rel);
  w.m64.host = nullptr;  // not ours to free
  if (rc) return rc;
  inf.rel_res = rel.empty() ? 0.0 : *std::max_element(rel.begin(), rel.end());
  if (status == GYM_OK && inf.rel_res > opts.rtol) status = GYM_W_NOT_CONVERGED;
  GYM_HIP(hipStreamSynchronize(s));
  inf.status = status;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

}  // namespace gym

extern "C" {

int gym_mass_solve(const gym_space* space_c, const gym_solve_opts* opts_in, int nrhs, const double* b, double* x,
                   gym_solve_info* info, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  if (!space_c || !b || !x || nrhs < 1) return fail(GYM_E_ARG, "bad argument");
  gym_space* space = const_cast<gym_space*>(space_c);  // workspace cache only
  gym_solve_opts opts;
  if (opts_in) opts = *opts_in;
  else gym_solve_opts_default(&opts);
  if (opts.mode != GYM_MODE_F64) return fail(GYM_E_UNSUPPORTED, "mass solves run in FP64");
  hipStream_t s = (hipStream_t)stream;
  const long long n = space->desc.ndofs;
  MassWork* w;
  if (int rc = ensure_mass_work(space, nrhs, &w)) return rc;
  auto apply = [&](const double* in, double* out) { return launch_mass_apply(space, GYM_F64, nrhs, in, out, s); };
  CgVecs<double> V{b, x, w->r, w->p, w->q};
  cg_launch_init<double>(V, space->d_diag, n, nrhs, w->nb, w->pa, w->st, opts.rtol, s);
  int it = 0;
  const int every = opts.check_every < 1 ? 1 : opts.check_every;
  gym_solve_info inf{};
  int flag = 1;
  std::vector<double> h(2 * nrhs);
  for (int attempt = 0; attempt < 6; ++attempt) {
    bool all_done = false;
    while (it < opts.maxit && !all_done) {
      CgState* cur = w->st + (it & 1) * nrhs;
      CgState* next = w->st + ((it + 1) & 1) * nrhs;
      if (int rc = apply(V.p, V.q)) return rc;
      cg_launch_iter_tail<double>(V, space->d_diag, n, nrhs, w->nb, cur, next, w->pa, w->pb, s);
      ++it;
      if (it % every == 0 || it == opts.maxit) {
        GYM_HIP(hipMemcpyAsync(w->host, next, sizeof(CgState) * nrhs, hipMemcpyDeviceToHost, s));
        GYM_HIP(hipStreamSynchronize(s));
        all_done = true;
        for (int r = 0; r < nrhs; ++r) all_done = all_done && w->host[r].done;
      }
    }
    GYM_HIP(hipGetLastError());
    // true relative residual ||b - M x|| / ||b|| (q is scratch here: the next
    // iteration overwrites it with M p)
    if (int rc = apply(x, w->q)) return rc;
    launch_norm2(w->q, b, n, nrhs, w->nb, 1, w->pa, w->sums, s);
    launch_norm2(b, nullptr, n, nrhs, w->nb, 0, w->pa, w->sums + nrhs, s);
    GYM_HIP(hipMemcpyAsync(h.data(), w->sums, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
    GYM_HIP(hipStreamSynchronize(s));
    inf.rel_res = 0;
    flag = 1;
    for (int r = 0; r < nrhs; ++r) {
      double bn = std::sqrt(h[nrhs + r]);
      double rel = bn > 0 ? std::sqrt(h[r]) / bn : std::sqrt(h[r]);
      inf.rel_res = std::max(inf.rel_res, rel);
      if (w->host[r].flag < 0) flag = -1;
    }
    if (flag < 0 || inf.rel_res <= opts.rtol || it >= opts.maxit) break;
    // the preconditioned criterion was optimistic: tighten, resume (the
    // latest state is in slot it & 1)
    CgState* latest = w->st + (it & 1) * nrhs;
    GYM_HIP(hipMemcpyAsync(w->host, latest, sizeof(CgState) * nrhs, hipMemcpyDeviceToHost, s));
    GYM_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) {
      w->host[r].tol *= 0.1;
      w->host[r].done = 0;
      w->host[r].flag = 0;
    }
    GYM_HIP(hipMemcpyAsync(latest, w->host, sizeof(CgState) * nrhs, hipMemcpyHostToDevice, s));
  }
  inf.iters = it;
  inf.status = flag < 0 ? GYM_E_BREAKDOWN : (inf.rel_res <= opts.rtol ? GYM_OK : GYM_W_NOT_CONVERGED);
  if (flag < 0) fail(GYM_E_BREAKDOWN, "CG breakdown (NaN or non-positive curvature)");
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return inf.status;
}

}  // extern "C"
