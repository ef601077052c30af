// Shared host code of the operator kernels: table construction and the
// problem dispatch across the per-problem translation units.
#include <hip/hip_runtime.h>

#include "gym_internal.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace gym {

void fill_tables(TabSet<double>* hd, TabSet<double>* hl, TabSet<float>* hf, TabSet<float>* hb) {
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
    // bf16-rounded copy (only the Kronecker matrices are read in BF16 mode)
    TabSet<float>& b = hb[r - 1];
    b = f;
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) b.mn[i][j] = round_bf16(f.mn[i][j]);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) b.me[i][j] = round_bf16(f.me[i][j]);
  }
}


int upload_tables() {
  if (int rc = upload_tables_hodge()) return rc;
  if (int rc = upload_tables_poisson()) return rc;
  if (int rc = upload_tables_hodge_mr()) return rc;
  if (int rc = upload_tables_poisson_mr()) return rc;
  return upload_tables_mass();
}

int launch_op_batch(int prob, int dim, int r, OpParams* plist_host, int* bstart_host, int nreq, OpParams* plist_dev,
                    int* bstart_dev, int ncu, hipStream_t s) {
  if (dim != 3) return -2;
  if (nreq > 0 && plist_host[0].fused) {
    if (prob == PROB_HODGE)
      return launch_hodge_batch_mr(r, plist_host, bstart_host, nreq, plist_dev, bstart_dev, ncu, s);
    if (prob == PROB_POISSON)
      return launch_poisson_batch_mr(r, plist_host, bstart_host, nreq, plist_dev, bstart_dev, ncu, s);
    return -2;
  }
  if (prob == PROB_HODGE) return launch_hodge_batch(r, plist_host, bstart_host, nreq, plist_dev, bstart_dev, ncu, s);
  if (prob == PROB_POISSON)
    return launch_poisson_batch(r, plist_host, bstart_host, nreq, plist_dev, bstart_dev, ncu, s);
  return -2;
}

int launch_operator(int prob, int dim, int r, int prec, const OpParams& p, int nrhs, int ncu, hipStream_t s) {
  if (p.fused) {
    if (prob == PROB_HODGE) return launch_hodge_mr(dim, r, prec, p, nrhs, ncu, s);
    if (prob == PROB_POISSON) return launch_poisson_mr(dim, r, prec, p, nrhs, ncu, s);
    return -2;
  }
  if (prob == PROB_HODGE) return launch_hodge(dim, r, prec, p, nrhs, ncu, s);
  if (prob == PROB_POISSON) return launch_poisson(dim, r, prec, p, nrhs, ncu, s);
  return launch_mass(prob, dim, r, prec, p, nrhs, ncu, s);
}

}  // namespace gym
