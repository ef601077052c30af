// Generalized Yee time stepping (paper section 3; declared in include/gym.h).
//
// State (a, e), both in Lambda^1 with tangential components zero on the
// boundary.  One Strang step is a half step of the shear map
// a <- a - tau Q1 e, a full step of e <- e + tau P2 a, another half step in a
// (eqs. shearMaps, strangSplit).  The second half step of one step and the
// first of the next act on the same e, so n steps are
//   a -= tau/2 Q1 e;  n times { e += tau P2 a;  a -= tau Q1 e }  with the last
//   a-update halved,
// one Q1 and one P2 application per step.  P2 a = c^2 C^T M2~ C a runs as
// incidence, mass apply (or lumped scaling), transposed incidence; Q1 e as a
// CG mass solve (exact) or a diagonal scaling (lumped).  With both masses
// lumped the whole step is one stencil kernel (yee.hip), a ping-ponging
// between the caller's vector and a work vector.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "gym_internal.hpp"
#include "eig.hpp"
#include "krylov.hpp"
#include "spai.hpp"
#include "spai_op.hpp"
#include "yee.hpp"

using namespace gym;

struct gym_maxwell {
  gym_ctx* ctx = nullptr;
  const gym_mesh* mesh = nullptr;
  gym_maxwell_opts o{};
  gym_space* s1 = nullptr;  // Lambda^1, perfect conductor
  gym_space* s2 = nullptr;  // Lambda^2 (= C Lambda^1), no boundary condition
  long long n1 = 0, n2 = 0;
  int nb1 = 0, nb2 = 0;
  double* mem = nullptr;
  double *q1d = nullptr, *m2d = nullptr;  // lumped: 1 / rowsum(M1), rowsum(M2)
  double *q = nullptr, *t = nullptr;      // n1: Q1 e, C^T M2~ C a
  double *b = nullptr, *mb = nullptr;     // n2: C a, M2~ C a
  double *part = nullptr, *sums = nullptr;
  SpaiParams spai{};   // SPAI Q1: its 1-D factors
  double* spai_mem = nullptr;
  SpaiOpQ1 spai_op;    // SPAI-OP Q1 (set by gym_maxwell_spai_op)
  bool fused = false;  // both masses lumped: one stencil kernel per step
  YeeParams yp{};      // its fixed parameters (1-D row sums in w)
};

namespace {

// Lumped masses: one positive row sum per unknown (on curved cells they come
// from a device apply, which may fail; high-order curved rows need not sum
// positive).
int check_rowsums(const std::vector<double>& d, long long n) {
  if ((long long)d.size() != n) return fail(GYM_E_HIP, "lumped masses: the row sums could not be formed");
  for (double v : d)
    if (!(v > 0)) return fail(GYM_E_UNSUPPORTED, "lumped masses: a row sum of the mass matrix is not positive");
  return 0;
}

// q = Q1 e
bool sparse_q1(const gym_maxwell* mx) {
  return mx->o.q1 == GYM_Q1_SPAI_DIAG || mx->o.q1 == GYM_Q1_SPAI || mx->o.q1 == GYM_Q1_SPAI_OP;
}

// q = Q1 e for the sparse approximate inverses
void apply_sparse_q1(gym_maxwell* mx, const double* e, double* q, hipStream_t s) {
  if (mx->o.q1 == GYM_Q1_SPAI_OP) launch_spai_op_apply(mx->spai_op, e, q, mx->ctx->ncu, s);
  else launch_spai_apply(mx->spai, e, q, mx->nb1, s);
}

int apply_q1(gym_maxwell* mx, const double* e, double* q, hipStream_t s, int* warn) {
  if (sparse_q1(mx)) {
    apply_sparse_q1(mx, e, q, s);
    return 0;
  }
  if (mx->o.q1 == GYM_Q1_LUMPED) {
    launch_axpy_diag(q, 0.0, 1.0, mx->q1d, e, mx->n1, mx->nb1, s);
    return 0;
  }
  gym_solve_opts so;
  gym_solve_opts_default(&so);
  so.method = GYM_CG;
  so.rtol = mx->o.cg_rtol;
  so.maxit = mx->o.cg_maxit;
  gym_solve_info info{};
  int rc = gym_mass_solve(mx->s1, &so, 1, e, q, &info, s);
  if (rc == GYM_W_NOT_CONVERGED) {
    *warn = 1;
    return 0;
  }
  return rc;
}

// t = C^T M2~ C a (without c^2)
int apply_p2(gym_maxwell* mx, const double* a, hipStream_t s) {
  if (int rc = gym_d_apply(mx->s1, mx->s2, 0, a, mx->b, s)) return rc;
  if (mx->o.m2 == GYM_M2_LUMPED) {
    launch_axpy_diag(mx->mb, 0.0, 1.0, mx->m2d, mx->b, mx->n2, mx->nb2, s);
  } else if (int rc = gym_mass_apply(mx->s2, GYM_F64, 1, mx->b, mx->mb, s)) {
    return rc;
  }
  return gym_d_apply(mx->s1, mx->s2, 1, mx->mb, mx->t, s);
}

// y = C^T M2~ C x for ncol contiguous columns, in one launch per stage
// (b, mb: n2 x ncol work).
int apply_p2_n(gym_maxwell* mx, const double* x, double* y, int ncol, double* b, double* mb, hipStream_t s) {
  if (int rc = d_apply_n(mx->s1, mx->s2, 0, ncol, x, b, s)) return rc;
  if (mx->o.m2 == GYM_M2_LUMPED) {
    for (int j = 0; j < ncol; ++j)
      launch_axpy_diag(mb + mx->n2 * j, 0.0, 1.0, mx->m2d, b + mx->n2 * j, mx->n2, mx->nb2, s);
  } else if (int rc = gym_mass_apply(mx->s2, GYM_F64, ncol, b, mb, s)) {
    return rc;
  }
  return d_apply_n(mx->s1, mx->s2, 1, ncol, mb, y, s);
}

}  // namespace

extern "C" {

void gym_maxwell_opts_default(gym_maxwell_opts* o) {
  o->q1 = GYM_Q1_EXACT;
  o->m2 = GYM_M2_EXACT;
  o->c = 1.0;
  o->cg_rtol = 1e-14;
  o->cg_maxit = 1000;
}

int gym_maxwell_create(gym_ctx* ctx, const gym_mesh* mesh, int degree, const gym_maxwell_opts* opts,
                       gym_maxwell** out) {
  if (!ctx || !mesh || !out) return fail(GYM_E_ARG, "NULL argument");
  gym_maxwell_opts o;
  if (opts) o = *opts;
  else gym_maxwell_opts_default(&o);
  if (mesh->dim != 3 && !(mesh->dim == 2 && mesh->periodic == 3))
    return fail(GYM_E_ARG, "time stepping is 3-D, or 2-D on a doubly periodic mesh");
  if (degree < 1 || degree > 4) return fail(GYM_E_ARG, "degree must be 1..4");
  if ((o.q1 != GYM_Q1_EXACT && o.q1 != GYM_Q1_LUMPED && o.q1 != GYM_Q1_SPAI_DIAG && o.q1 != GYM_Q1_SPAI) ||
      (o.m2 != GYM_M2_EXACT && o.m2 != GYM_M2_LUMPED) ||
      !(o.c > 0) || !(o.cg_rtol > 0) || o.cg_maxit < 1)
    return fail(GYM_E_ARG, "bad time-stepping options");
  if (mesh->curved && (o.q1 == GYM_Q1_SPAI_DIAG || o.q1 == GYM_Q1_SPAI))
    return fail(GYM_E_UNSUPPORTED, "the SPAI needs an affine mesh");
  if (mesh->curved) {
    // the Gauss-point metrics of the mass applies, before the first step
    const void* qd;
    if (int rc = mesh_qdata(mesh, degree, 0, &qd)) return rc;
  }
  gym_maxwell* mx = new gym_maxwell;
  mx->ctx = ctx;
  mx->mesh = mesh;
  mx->o = o;
  int rc = gym_space_create(ctx, mesh, GYM_HCURL, degree, GYM_BC_ESSENTIAL, &mx->s1);
  // Lambda^2 = C Lambda^1: H(div) in 3-D, the scalar L2 space in 2-D
  if (!rc) rc = gym_space_create(ctx, mesh, mesh->dim == 3 ? GYM_HDIV : GYM_L2, degree, GYM_BC_NATURAL, &mx->s2);
  if (rc) {
    gym_maxwell_destroy(mx);
    return rc;
  }
  mx->n1 = gym_space_ndofs(mx->s1);
  mx->n2 = gym_space_ndofs(mx->s2);
  mx->nb1 = vec_grid(mx->n1, ctx->ncu);
  mx->nb2 = vec_grid(mx->n2, ctx->ncu);
  const bool lumped = o.q1 == GYM_Q1_LUMPED && o.m2 == GYM_M2_LUMPED;
  LumpedTables tab1, tab2;
  long long npos = 1, nw = 0;
  if (lumped) {
    tab1 = lumped_tables_host(mx->s1);
    tab2 = lumped_tables_host(mx->s2);
    for (int a = 0; a < 3; ++a) {
      npos *= (long long)tab1.rn[a].size();
      nw += (long long)(tab1.rn[a].size() + tab1.re[a].size());
    }
  }
  // one thread per lattice position, indexed in 32 bits (the stencil kernel
  // is written for the 3-D perfect conductor)
  mx->fused = lumped && npos < (1LL << 31) - 256 && mesh->dim == 3 && !mesh->periodic && !mesh->curved;
  const size_t total = 3 * (size_t)mx->n1 + 3 * (size_t)mx->n2 + (size_t)mx->nb1 + 4 + (mx->fused ? nw : 0);
  if (hipMalloc(&mx->mem, sizeof(double) * total) != hipSuccess) {
    (void)hipGetLastError();
    gym_maxwell_destroy(mx);
    return fail(GYM_E_OOM, "time stepping: device allocation failed");
  }
  double* p = mx->mem;
  mx->q1d = p, p += mx->n1;
  mx->q = p, p += mx->n1;
  mx->t = p, p += mx->n1;
  mx->m2d = p, p += mx->n2;
  mx->b = p, p += mx->n2;
  mx->mb = p, p += mx->n2;
  mx->part = p, p += mx->nb1;
  mx->sums = p, p += 4;
  if (mx->fused) {
    YeeParams& y = mx->yp;
    std::vector<double> w;
    for (int a = 0; a < 3; ++a) {
      y.wn[a] = (int)w.size();
      w.insert(w.end(), tab1.rn[a].begin(), tab1.rn[a].end());
      y.we[a] = (int)w.size();
      w.insert(w.end(), tab1.re[a].begin(), tab1.re[a].end());
      y.len[a] = (int)tab1.rn[a].size();
      y.q1s[a] = tab1.sc[a];
      y.m2s[a] = tab2.sc[a];
    }
    y.w = p;
    y.npos = (unsigned)npos;
    const SpaceDesc& d = mx->s1->desc;
    for (int c = 0; c < 3; ++c) {
      y.s1.c[c].offset = d.comp[c].offset;
      for (int a = 0; a < 3; ++a) {
        y.s1.c[c].start[a] = (int)d.comp[c].start[a];
        y.s1.c[c].count[a] = (int)d.comp[c].count[a];
      }
    }
    if (hipMemcpy(p, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice) != hipSuccess) {
      gym_maxwell_destroy(mx);
      return fail(GYM_E_HIP, "time stepping: upload failed");
    }
  }
  if (o.q1 == GYM_Q1_LUMPED) {
    std::vector<double> d = lumped_diag_host(mx->s1);
    if (int rc2 = check_rowsums(d, mx->n1)) {
      gym_maxwell_destroy(mx);
      return rc2;
    }
    for (double& v : d) v = 1.0 / v;
    if (hipMemcpy(mx->q1d, d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice) != hipSuccess) {
      gym_maxwell_destroy(mx);
      return fail(GYM_E_HIP, "time stepping: upload failed");
    }
  }
  if (o.q1 == GYM_Q1_SPAI_DIAG || o.q1 == GYM_Q1_SPAI) {
    if (int rc2 = build_spai_q1(mx->s1, o.q1 == GYM_Q1_SPAI ? 1 : 0, &mx->spai, &mx->spai_mem)) {
      gym_maxwell_destroy(mx);
      return rc2;
    }
  }
  if (o.m2 == GYM_M2_LUMPED) {
    std::vector<double> d = lumped_diag_host(mx->s2);
    if (int rc2 = check_rowsums(d, mx->n2)) {
      gym_maxwell_destroy(mx);
      return rc2;
    }
    if (hipMemcpy(mx->m2d, d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice) != hipSuccess) {
      gym_maxwell_destroy(mx);
      return fail(GYM_E_HIP, "time stepping: upload failed");
    }
  }
  *out = mx;
  return GYM_OK;
}

int64_t gym_maxwell_ndofs(const gym_maxwell* mx) { return mx ? mx->n1 : 0; }

int gym_maxwell_step(gym_maxwell* mx, double tau, int nsteps, double* a, double* e, void* stream) {
  if (!mx || !a || !e || !(tau > 0) || nsteps < 0) return fail(GYM_E_ARG, "bad argument");
  if (nsteps == 0) return GYM_OK;
  hipStream_t s = (hipStream_t)stream;
  const double c2 = mx->o.c * mx->o.c;
  if (mx->fused) {
    // a lives in buf[(nsteps - k) & 1] after k steps, so in the caller's
    // vector at the end
    double* buf[2] = {a, mx->t};
    YeeParams p = mx->yp;
    p.e = e;
    p.te = tau * c2;
    p.a_in = a;
    p.a_out = buf[nsteps & 1];
    p.ha = 0.5 * tau;
    if (launch_yee(p, true, mx->ctx->ncu, s)) return fail(GYM_E_HIP, "time stepping: kernel launch failed");
    for (int k = 0; k < nsteps; ++k) {
      p.a_in = buf[(nsteps - k) & 1];
      p.a_out = buf[(nsteps - k - 1) & 1];
      p.ha = (k == nsteps - 1) ? 0.5 * tau : tau;
      if (launch_yee(p, false, mx->ctx->ncu, s)) return fail(GYM_E_HIP, "time stepping: kernel launch failed");
    }
    GYM_HIP(hipGetLastError());
    return GYM_OK;
  }
  int warn = 0;
  if (int rc = apply_q1(mx, e, mx->q, s, &warn)) return rc;
  launch_axpy_diag(a, 1.0, -0.5 * tau, nullptr, mx->q, mx->n1, mx->nb1, s);
  for (int k = 0; k < nsteps; ++k) {
    if (int rc = apply_p2(mx, a, s)) return rc;
    launch_axpy_diag(e, 1.0, tau * c2, nullptr, mx->t, mx->n1, mx->nb1, s);
    if (int rc = apply_q1(mx, e, mx->q, s, &warn)) return rc;
    const double h = (k == nsteps - 1) ? 0.5 * tau : tau;
    launch_axpy_diag(a, 1.0, -h, nullptr, mx->q, mx->n1, mx->nb1, s);
  }
  GYM_HIP(hipGetLastError());
  return warn ? GYM_W_NOT_CONVERGED : GYM_OK;
}

int gym_maxwell_energy(gym_maxwell* mx, const double* a, const double* e, double* H, void* stream) {
  if (!mx || !a || !e || !H) return fail(GYM_E_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  int warn = 0;
  if (int rc = apply_q1(mx, e, mx->q, s, &warn)) return rc;
  if (int rc = apply_p2(mx, a, s)) return rc;
  launch_norm2(e, mx->q, mx->n1, 1, mx->nb1, 2, mx->part, mx->sums, s);
  launch_norm2(a, mx->t, mx->n1, 1, mx->nb1, 2, mx->part, mx->sums + 1, s);
  double h[2];
  GYM_HIP(hipMemcpyAsync(h, mx->sums, sizeof(h), hipMemcpyDeviceToHost, s));
  GYM_HIP(hipStreamSynchronize(s));
  *H = 0.5 * h[0] + 0.5 * mx->o.c * mx->o.c * h[1];
  return warn ? GYM_W_NOT_CONVERGED : GYM_OK;
}

void gym_eig_opts_default(gym_eig_opts* o) {
  o->nev = 4;
  o->largest = 0;
  o->block = 0;
  o->tol = 1e-8;
  o->maxit = 3000;
  o->grad_shift = 4.0;
  o->seed = 1;
}

int gym_maxwell_eigs(gym_maxwell* mx, const gym_eig_opts* opts, double* omega2, double* vecs, gym_eig_info* info,
                     void* stream) {
  if (!mx || !omega2) return fail(GYM_E_ARG, "NULL argument");
  gym_eig_opts o;
  if (opts) o = *opts;
  else gym_eig_opts_default(&o);
  const int k = o.block > 0 ? o.block : std::min(o.nev + 2, kEigMaxCols / 3);
  if (o.nev < 1 || k < o.nev || 3 * k > kEigMaxCols || !(o.tol > 0) || o.maxit < 1 || !(o.grad_shift > 0) ||
      (o.largest != 0 && o.largest != 1))
    return fail(GYM_E_ARG, "bad eigen-solver options (1 <= nev <= block <= 8)");
  hipStream_t s = (hipStream_t)stream;
  const long long n1 = mx->n1;
  if (n1 < 3LL * k) return fail(GYM_E_ARG, "eigen-solver: fewer unknowns than the search space needs");
  const double c2 = mx->o.c * mx->o.c;
  const bool lumped = mx->o.q1 == GYM_Q1_LUMPED;
  const bool spai_q1 = sparse_q1(mx);
  gym_space* s0 = nullptr;  // Lambda^0 with the conductor's boundary values removed
  if (int rc = gym_space_create(mx->ctx, mx->mesh, GYM_H1, mx->s1->desc.r, GYM_BC_ESSENTIAL, &s0)) return rc;
  const long long n0 = gym_space_ndofs(s0);
  const int nb1 = mx->nb1;
  const int nb0 = vec_grid(std::max(1LL, n0), mx->ctx->ncu);
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
  auto cleanup = [&] {
    for (void* p : pool) (void)hipFree(p);
    gym_space_destroy(s0);
  };
  double* X = alloc(n1 * k);
  double* bx = alloc(n1 * k);
  double* gp = alloc(n1 * k);
  double* bgp = alloc(n1 * k);
  double* g0 = alloc(std::max(1LL, n0) * k);
  double* phi = alloc(std::max(1LL, n0) * k);
  double* b2 = alloc(mx->n2 * k);   // C x, then M2~ C x, for the columns of an A apply
  double* mb2 = alloc(mx->n2 * k);
  double* dB = alloc(n1);    // lumped: the row sums of M1 (B itself)
  double* dT = alloc(n1);    // their inverses (the preconditioner)
  double* d0i = alloc(std::max(1LL, n0));  // inverse diagonal of M0 (the gradient shift's X)
  double* gw = alloc(eig_gram_work(nb1));
  double* cgw = spai_q1 ? alloc(3 * n1 * k) : nullptr;  // CG work of B = Q1^-1
  // On a mesh periodic along every axis, ker P2 holds besides the gradients
  // the harmonic fields: the interpolants of the constant fields (one per
  // axis; edge values proportional to the GLL sub-edge lengths).
  const int dimm = mx->mesh->dim;
  const int nh = mx->mesh->periodic == (1 << dimm) - 1 ? dimm : 0;
  double* H = nh ? alloc(n1 * nh) : nullptr;
  double* BH = nh ? alloc(n1 * nh) : nullptr;
  if (!X || !bx || !gp || !bgp || !g0 || !phi || !b2 || !mb2 || !dB || !dT || !d0i || !gw || (spai_q1 && !cgw) || (nh && (!H || !BH))) {
    cleanup();
    return fail(GYM_E_OOM, "eigen-solver: device allocation failed");
  }
  {
    // B itself when Q1 is lumped; otherwise only the preconditioner T
    std::vector<double> d = lumped_diag_host(mx->s1, lumped), di(d.size());
    if (int rc2 = check_rowsums(d, n1)) {
      cleanup();
      return rc2;
    }
    for (size_t i = 0; i < d.size(); ++i) di[i] = 1.0 / d[i];
    std::vector<double> d0 = mass_diag_host(s0);
    for (double& v : d0) v = 1.0 / v;
    if (hipMemcpy(dB, d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dT, di.data(), sizeof(double) * di.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (n0 > 0 && hipMemcpy(d0i, d0.data(), sizeof(double) * n0, hipMemcpyHostToDevice) != hipSuccess)) {
      cleanup();
      return fail(GYM_E_HIP, "eigen-solver: upload failed");
    }
  }
  auto colp = [](double* b, long long n, int j) { return b + (long long)j * n; };
  int warn = 0;
  EigOperators ops;
  // B = Q1^-1 for a SPAI Q1: CG on Q1 (symmetric positive definite, close to
  // M1^-1, so well conditioned), every column to relative residual 1e-13
  auto spai_inverse = [&](const double* x, double* y, int ncol) -> int {
    double* r = cgw;
    double* p = cgw + n1 * ncol;
    double* q = cgw + 2 * n1 * ncol;
    const long long nc = n1 * ncol;
    if (hipMemcpyAsync(r, x, sizeof(double) * nc, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(p, x, sizeof(double) * nc, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemsetAsync(y, 0, sizeof(double) * nc, s) != hipSuccess)
      return hip_fail(hipGetLastError(), "SPAI inverse");
    std::vector<double> G((size_t)ncol * ncol), rr(ncol), rr0(ncol);
    if (eig_gram(r, ncol, r, ncol, n1, G.data(), gw, nb1, s)) return hip_fail(hipGetLastError(), "SPAI inverse");
    for (int j = 0; j < ncol; ++j) rr[j] = rr0[j] = G[(size_t)j * ncol + j];
    for (int it = 0; it < 2000; ++it) {
      bool done = true;
      for (int j = 0; j < ncol; ++j)
        if (rr[j] > 1e-26 * rr0[j]) done = false;
      if (done) return 0;
      for (int j = 0; j < ncol; ++j) apply_sparse_q1(mx, colp(p, n1, j), colp(q, n1, j), s);
      if (eig_gram(p, ncol, q, ncol, n1, G.data(), gw, nb1, s)) return hip_fail(hipGetLastError(), "SPAI inverse");
      for (int j = 0; j < ncol; ++j) {
        const double pq = G[(size_t)j * ncol + j];
        if (!(pq > 0)) {
          if (rr[j] == 0.0) continue;
          return fail(GYM_E_BREAKDOWN, "eigen-solver: the SPAI Q1 is not positive definite");
        }
        const double al = rr[j] / pq;
        launch_axpy_diag(colp(y, n1, j), 1.0, al, nullptr, colp(p, n1, j), n1, nb1, s);
        launch_axpy_diag(colp(r, n1, j), 1.0, -al, nullptr, colp(q, n1, j), n1, nb1, s);
      }
      if (eig_gram(r, ncol, r, ncol, n1, G.data(), gw, nb1, s)) return hip_fail(hipGetLastError(), "SPAI inverse");
      for (int j = 0; j < ncol; ++j) {
        const double rn = G[(size_t)j * ncol + j];
        const double be = rr[j] > 0 ? rn / rr[j] : 0.0;
        rr[j] = rn;
        launch_axpy_diag(colp(p, n1, j), be, 1.0, nullptr, colp(r, n1, j), n1, nb1, s);
      }
    }
    warn = 1;
    return 0;
  };
  // B = Q1^-1: M1, its row sums when lumped, or the inverse of a SPAI
  ops.B = [&](const double* x, double* y, int ncol) -> int {
    if (spai_q1) return spai_inverse(x, y, ncol);
    if (!lumped) return gym_mass_apply(mx->s1, GYM_F64, ncol, x, y, s);
    launch_diag_cols(y, dB, x, n1, ncol, nb1, s);
    return 0;
  };
  // T: Q1 itself for a SPAI (it approximates B^-1 = Q1 exactly); otherwise
  // the inverse row sums of M1
  ops.T = [&](const double* x, double* y, int ncol) -> int {
    if (spai_q1) {
      for (int j = 0; j < ncol; ++j) apply_sparse_q1(mx, colp(const_cast<double*>(x), n1, j), colp(y, n1, j), s);
      return 0;
    }
    launch_diag_cols(y, dT, x, n1, ncol, nb1, s);
    return 0;
  };
  // A = c^2 (C^T M2~ C + s B G D0^-1 G^T B), D0 the diagonal of M0: P2 plus
  // a multiple of a gradient-space operator.  For any SPD X in place of
  // D0^-1 the term vanishes on fields with G^T B v = 0 and maps gradients to
  // B times gradients, so it lifts the gradients (the kernel of P2) above the
  // wanted modes and leaves every other eigenpair of (P2, B) alone; the
  // diagonal makes it a handful of launches instead of a mass solve.
  ops.A = [&](const double* x, double* y, int ncol) -> int {
    if (int rc = apply_p2_n(mx, x, y, ncol, b2, mb2, s)) return rc;
    if (o.largest) {  // -P2: its lowest pairs are the largest of P2
      launch_axpy_diag(y, 0.0, -c2, nullptr, y, n1 * ncol, nb1, s);
      return 0;
    }
    if (int rc = ops.B(x, bx, ncol)) return rc;
    if (int rc = d_apply_n(s0, mx->s1, 1, ncol, bx, g0, s)) return rc;
    launch_diag_cols(phi, d0i, g0, n0, ncol, nb0, s);
    if (int rc = d_apply_n(s0, mx->s1, 0, ncol, phi, gp, s)) return rc;
    if (int rc = ops.B(gp, bgp, ncol)) return rc;
    launch_axpy_diag(y, c2, c2 * o.grad_shift, nullptr, bgp, n1 * ncol, nb1, s);
    return 0;
  };
  // harmonic lift: A += c^2 s B H (H^T B H)^-1 H^T B, which moves the
  // harmonic fields (P2 h = 0) to omega^2 = s c^2 and, as every other
  // eigenvector of (P2, B) is B-orthogonal to them, leaves the rest alone
  std::vector<double> ghi((size_t)nh * nh);
  if (nh) {
    const SpaceDesc& d1 = mx->s1->desc;
    const std::vector<double> xi = gll_nodes(d1.r);
    std::vector<double> h((size_t)n1 * nh, 0.0);
    for (int a = 0; a < nh; ++a) {
      const CompDesc& cd = d1.comp[a];
      int64_t idx = cd.offset;
      for (int64_t kk = 0; kk < cd.count[2]; ++kk)
        for (int64_t j = 0; j < cd.count[1]; ++j)
          for (int64_t i = 0; i < cd.count[0]; ++i) {
            const int64_t p[3] = {cd.start[0] + i, cd.start[1] + j, cd.start[2] + kk};
            const int loc = (int)(p[a] % d1.r);
            h[(size_t)a * n1 + idx++] = xi[loc + 1] - xi[loc];
          }
    }
    std::vector<double> gh((size_t)nh * nh);
    int rc0 = hipMemcpy(H, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice) != hipSuccess
                  ? hip_fail(hipGetLastError(), "eigen-solver upload")
                  : ops.B(H, BH, nh);
    if (!rc0 && eig_gram(H, nh, BH, nh, n1, gh.data(), gw, nb1, s)) rc0 = hip_fail(hipGetLastError(), "eigen-solver gram");
    if (!rc0) {
      // (H^T B H)^-1 of at most 3 x 3, by Gauss-Jordan
      std::vector<double> a = gh;
      for (int i = 0; i < nh; ++i) ghi[(size_t)i * nh + i] = 1.0;
      for (int c = 0; c < nh; ++c) {
        const double piv = a[(size_t)c * nh + c];
        for (int j = 0; j < nh; ++j) {
          a[(size_t)c * nh + j] /= piv;
          ghi[(size_t)c * nh + j] /= piv;
        }
        for (int r2 = 0; r2 < nh; ++r2) {
          if (r2 == c) continue;
          const double f = a[(size_t)r2 * nh + c];
          for (int j = 0; j < nh; ++j) {
            a[(size_t)r2 * nh + j] -= f * a[(size_t)c * nh + j];
            ghi[(size_t)r2 * nh + j] -= f * ghi[(size_t)c * nh + j];
          }
        }
      }
    }
    if (rc0) {
      cleanup();
      return rc0;
    }
  }
  const std::function<int(const double*, double*, int)> base_a = ops.A;
  if (nh && !o.largest) {
    ops.A = [&, base_a](const double* x, double* y, int ncol) -> int {
      if (int rc = base_a(x, y, ncol)) return rc;
      std::vector<double> cf((size_t)nh * ncol);
      if (eig_gram(BH, nh, x, ncol, n1, cf.data(), gw, nb1, s)) return hip_fail(hipGetLastError(), "eigen-solver gram");
      for (int j = 0; j < ncol; ++j)
        for (int a = 0; a < nh; ++a) {
          double w = 0.0;
          for (int b = 0; b < nh; ++b) w += ghi[(size_t)a * nh + b] * cf[(size_t)b * ncol + j];
          launch_axpy_diag(colp(y, n1, j), 1.0, c2 * o.grad_shift * w, nullptr, BH + (long long)a * n1, n1, nb1, s);
        }
      return 0;
    };
  }
  launch_rhs_normal(X, 0, n1 * k, o.seed, vec_grid(n1 * k, mx->ctx->ncu), s);
  std::vector<double> lam(k);
  EigResult er;
  int rc = lobpcg(ops, n1, k, o.nev, o.tol, o.maxit, X, lam.data(), &er, mx->ctx->ncu, s);
  int ngrad = 0;
  if (rc >= 0 && !o.largest) {
    // a wanted pair with G^T B x != 0 is a gradient the shift did not lift far enough
    if (int r2 = ops.B(X, bx, k)) rc = r2;
    for (int j = 0; j < k && rc >= 0; ++j)
      if (int r2 = gym_d_apply(s0, mx->s1, 1, colp(bx, n1, j), colp(g0, n0, j), s)) rc = r2;
    std::vector<double> gg((size_t)k * k), bb((size_t)k * k);
    if (rc >= 0 && (eig_gram(g0, k, g0, k, n0, gg.data(), gw, nb1, s) || eig_gram(bx, k, bx, k, n1, bb.data(), gw, nb1, s)))
      rc = hip_fail(hipGetLastError(), "eigen-solver check");
    for (int j = 0; j < o.nev && rc >= 0; ++j)
      if (std::sqrt(gg[(size_t)j * k + j]) > 1e-4 * std::sqrt(bb[(size_t)j * k + j])) ++ngrad;
  }
  if (rc >= 0) {
    for (int j = 0; j < o.nev; ++j) omega2[j] = o.largest ? -lam[j] : lam[j];
    if (vecs && hipMemcpyAsync(vecs, X, sizeof(double) * n1 * o.nev, hipMemcpyDeviceToDevice, s) != hipSuccess)
      rc = hip_fail(hipGetLastError(), "eigen-solver copy");
    if (hipStreamSynchronize(s) != hipSuccess) rc = hip_fail(hipGetLastError(), "eigen-solver sync");
  }
  if (info) {
    info->iters = er.iters;
    info->converged = er.converged;
    info->max_resid = er.max_resid;
    info->gradient_modes = ngrad;
  }
  cleanup();
  if (rc < 0) return rc;
  if (ngrad) return fail(GYM_W_NOT_CONVERGED, "eigen-solver: a wanted pair is a gradient; raise grad_shift");
  return (rc == 1 || warn) ? GYM_W_NOT_CONVERGED : GYM_OK;
}

int gym_maxwell_spai_op(gym_maxwell* mx, int nprobe, const double* probes, double lambda, double rtol, int maxit,
                        int* iters, double* rel_res, void* stream) {
  if (!mx || nprobe < 0 || (nprobe > 0 && !probes) || !(lambda >= 0) || !(rtol > 0) || maxit < 1)
    return fail(GYM_E_ARG, "bad SPAI-OP arguments");
  if (mx->mesh->curved) return fail(GYM_E_UNSUPPORTED, "SPAI-OP needs an affine mesh");
  hipStream_t s = (hipStream_t)stream;
  const long long n1 = mx->n1;
  const double c2 = mx->o.c * mx->o.c;
  double* W = nullptr;
  if (hipMalloc(&W, sizeof(double) * 2 * std::max(1, nprobe) * n1) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GYM_E_OOM, "SPAI-OP: device allocation failed");
  }
  double* MW = W + (long long)std::max(1, nprobe) * n1;
  // the probing vectors P2 v_k and M1 P2 v_k
  for (int k = 0; k < nprobe; ++k) {
    if (int rc = apply_p2(mx, probes + (long long)k * n1, s)) {
      (void)hipFree(W);
      return rc;
    }
    launch_axpy_diag(W + (long long)k * n1, 0.0, c2, nullptr, mx->t, n1, mx->nb1, s);
  }
  if (nprobe > 0) {
    if (int rc = gym_mass_apply(mx->s1, GYM_F64, nprobe, W, MW, s)) {
      (void)hipFree(W);
      return rc;
    }
  }
  SpaiOpQ1 Q;
  int it = 0;
  double rel = 0.0;
  int rc = spai_op_build(mx->s1, W, MW, nprobe, lambda, rtol, maxit, mx->ctx->ncu, s, &Q, &it, &rel);
  (void)hipStreamSynchronize(s);
  (void)hipFree(W);
  if (iters) *iters = it;
  if (rel_res) *rel_res = rel;
  if (rc < 0) return rc;
  spai_op_free(&mx->spai_op);
  mx->spai_op = Q;
  mx->o.q1 = GYM_Q1_SPAI_OP;
  // the one-kernel stepping exists for lumped Q1 only: from now on the steps
  // apply SPAI-OP Q1 (and the lumped M2~ still, if that was chosen)
  mx->fused = false;
  return rc;
}

int gym_maxwell_destroy(gym_maxwell* mx) {
  if (!mx) return GYM_OK;
  if (mx->mem) (void)hipFree(mx->mem);
  if (mx->spai_mem) (void)hipFree(mx->spai_mem);
  spai_op_free(&mx->spai_op);
  if (mx->s1) gym_space_destroy(mx->s1);
  if (mx->s2) gym_space_destroy(mx->s2);
  delete mx;
  return GYM_OK;
}

}  // extern "C"
