// Host-side 1-D tables and space descriptors.
//
// The 1-D complex on [0,1] (degree r): nodal functions are the Lagrange
// polynomials on the Gauss-Lobatto-Legendre nodes; edge functions are
// e_j = -sum_{k<=j} phi_k', the histopolants dual to the sub-intervals
// [xi_j, xi_{j+1}] (integral degrees of freedom, the integral-normalised form
// of the Whitney duality of the paper's eq. WhitneyFormDefn).  With them the
// 1-D derivative is the +-1 incidence phi_i' = e_{i-1} - e_i, which is what
// makes G, C, D integer in every dimension.
#include <cmath>
#include <stdexcept>

#include "gym_internal.hpp"

namespace gym {

namespace {

// Legendre P_n and P_n' at x in [-1, 1] by the three-term recurrence.
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  p = p1;
  // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n); interior points only
  dp = n * (p0 - x * p1) / (1.0 - x * x);
}

}  // namespace

void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < q; ++i) {
    double t = std::cos(pi * (i + 0.75) / (q + 0.5));  // Chebyshev-like guess
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(q, t, p, dp);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p, dp;
    legendre(q, t, p, dp);
    // map from [-1, 1] to [0, 1]; weights halve
    x[q - 1 - i] = 0.5 * (t + 1.0);
    w[q - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);
  }
}

std::vector<double> gll_nodes(int r) {
  // Interior nodes are the roots of P_r'.  Newton with P_r'' from the
  // Legendre equation (1 - x^2) P'' = 2 x P' - r (r + 1) P.
  std::vector<double> out(r + 1);
  out[0] = 0.0;
  out[r] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int i = 1; i < r; ++i) {
    double t = -std::cos(pi * i / r);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(r, t, p, dp);
      double d2 = (2.0 * t * dp - r * (r + 1.0) * p) / (1.0 - t * t);
      double dt = dp / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    out[i] = 0.5 * (t + 1.0);
  }
  return out;
}

Tables1D make_tables(int r, int q) {
  if (r < 1 || r > 8 || q < 1 || q > 12) throw std::invalid_argument("table size");
  Tables1D t;
  t.r = r;
  t.q = q;
  t.nodes = gll_nodes(r);
  gauss_rule(q, t.gx, t.gw);
  t.phi.assign(q * (r + 1), 0.0);
  t.edge.assign(q * r, 0.0);
  for (int s = 0; s < q; ++s) {
    double x = t.gx[s];
    std::vector<double> val(r + 1), der(r + 1);
    for (int i = 0; i <= r; ++i) {
      double v = 1.0, d = 0.0;
      // product rule: d/dx prod_k (x - x_k)/(x_i - x_k)
      for (int k = 0; k <= r; ++k) {
        if (k == i) continue;
        double f = 1.0 / (t.nodes[i] - t.nodes[k]);
        d = d * (x - t.nodes[k]) * f + v * f;
        v = v * (x - t.nodes[k]) * f;
      }
      val[i] = v;
      der[i] = d;
    }
    double acc = 0.0;
    for (int i = 0; i <= r; ++i) t.phi[s * (r + 1) + i] = val[i];
    for (int j = 0; j < r; ++j) {
      acc -= der[j];
      t.edge[s * r + j] = acc;
    }
  }
  return t;
}

SpaceDesc make_space_desc(int kind, int dim, const int64_t nel[3], int r, int bc, int periodic) {
  SpaceDesc s;
  s.kind = kind;
  s.dim = dim;
  s.r = r;
  s.bc = bc;
  s.periodic = periodic & ((1 << dim) - 1);
  for (int a = 0; a < 3; ++a) s.m[a] = a < dim ? r * nel[a] : 1;
  int full = (1 << dim) - 1;
  if (kind == GYM_H1 || kind == GYM_L2) {
    s.ncomp = 1;
    s.comp[0].nodal_mask = kind == GYM_H1 ? full : 0;
  } else {
    s.ncomp = dim;
    for (int c = 0; c < dim; ++c)
      s.comp[c].nodal_mask = kind == GYM_HCURL ? (full & ~(1 << c)) : (1 << c);
  }
  int64_t off = 0;
  for (int c = 0; c < s.ncomp; ++c) {
    CompDesc& cd = s.comp[c];
    int64_t cnt = 1;
    for (int a = 0; a < 3; ++a) {
      if (a >= dim) {
        cd.start[a] = 0;
        cd.count[a] = 1;
      } else if (s.periodic >> a & 1) {  // m_a positions, the last wrapping onto the first
        cd.start[a] = 0;
        cd.count[a] = s.m[a];
      } else if (cd.nodal_mask >> a & 1) {
        if (bc == GYM_BC_ESSENTIAL) {
          cd.start[a] = 1;
          cd.count[a] = s.m[a] - 1;
        } else {
          cd.start[a] = 0;
          cd.count[a] = s.m[a] + 1;
        }
      } else {
        cd.start[a] = 0;
        cd.count[a] = s.m[a];
      }
      cnt *= cd.count[a];
    }
    cd.offset = off;
    off += cnt;
  }
  s.ndofs = off;
  return s;
}

void element_masses_1d(int r, std::vector<double>& mn, std::vector<double>& me) {
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

}  // namespace gym
