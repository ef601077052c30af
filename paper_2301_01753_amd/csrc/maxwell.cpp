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

#include <cmath>
#include <vector>

#include "gym_internal.hpp"
#include "krylov.hpp"
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
  bool fused = false;  // both masses lumped: one stencil kernel per step
  YeeParams yp{};      // its fixed parameters (1-D row sums in w)
};

namespace {

// q = Q1 e
int apply_q1(gym_maxwell* mx, const double* e, double* q, hipStream_t s, int* warn) {
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
  if (mesh->dim != 3) return fail(GYM_E_ARG, "time stepping is 3-D");
  if (degree < 1 || degree > 4) return fail(GYM_E_ARG, "degree must be 1..4");
  if ((o.q1 != GYM_Q1_EXACT && o.q1 != GYM_Q1_LUMPED) || (o.m2 != GYM_M2_EXACT && o.m2 != GYM_M2_LUMPED) ||
      !(o.c > 0) || !(o.cg_rtol > 0) || o.cg_maxit < 1)
    return fail(GYM_E_ARG, "bad time-stepping options");
  if (mesh->curved && (o.q1 == GYM_Q1_LUMPED || o.m2 == GYM_M2_LUMPED))
    return fail(GYM_E_UNSUPPORTED, "lumped masses need an affine mesh");
  gym_maxwell* mx = new gym_maxwell;
  mx->ctx = ctx;
  mx->mesh = mesh;
  mx->o = o;
  int rc = gym_space_create(ctx, mesh, GYM_HCURL, degree, GYM_BC_ESSENTIAL, &mx->s1);
  if (!rc) rc = gym_space_create(ctx, mesh, GYM_HDIV, degree, GYM_BC_NATURAL, &mx->s2);
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
  // one thread per lattice position, indexed in 32 bits
  mx->fused = lumped && npos < (1LL << 31) - 256;
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
    for (double& v : d) v = 1.0 / v;
    if (hipMemcpy(mx->q1d, d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice) != hipSuccess) {
      gym_maxwell_destroy(mx);
      return fail(GYM_E_HIP, "time stepping: upload failed");
    }
  }
  if (o.m2 == GYM_M2_LUMPED) {
    std::vector<double> d = lumped_diag_host(mx->s2);
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

int gym_maxwell_destroy(gym_maxwell* mx) {
  if (!mx) return GYM_OK;
  if (mx->mem) (void)hipFree(mx->mem);
  if (mx->s1) gym_space_destroy(mx->s1);
  if (mx->s2) gym_space_destroy(mx->s2);
  delete mx;
  return GYM_OK;
}

}  // extern "C"
