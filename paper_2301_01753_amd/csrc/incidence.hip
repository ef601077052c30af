// Incidence apply: y = d x or d^T x for the integer matrices G, C, D of the
// discrete de Rham complex (paper section 2, eq. discreteDeRham).
//
// One thread per output entry.  Each output component has at most six +-1
// terms (input component, lattice shift); the host sorts them by input
// index, so every entry is summed from +0.0 in ascending input order.  With
// +-1 coefficients the products are exact, hence the result is bit-identical
// to an ascending-order CSR sum of the same matrix (and independent of the
// launch shape).  On a periodic axis the shifted position wraps around; the
// terms are then summed in the same fixed order, which for the entries whose
// stencil wraps is not the ascending one (exact on integer data all the same).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "gym_internal.hpp"
#include "kernels.hpp"

namespace gym {

struct Term {
  int comp;
  int shift[3];
  int sign;
};

struct IncTerms {
  int nterm[3];
  Term t[3][6];
};

__global__ void __launch_bounds__(256) incidence_kernel(const IncParams p, const IncTerms terms) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.nout) return;
  const double* x = p.x + p.in_stride * blockIdx.y;  // right-hand side blockIdx.y
  int c = 0;
  while (c + 1 < p.out_ncomp && i >= p.out.c[c + 1].offset) ++c;
  const DevComp& oc = p.out.c[c];
  long long loc = i - oc.offset;
  int pos[3];
  pos[0] = (int)(loc % oc.count[0]) + oc.start[0];
  long long rest = loc / oc.count[0];
  pos[1] = (int)(rest % oc.count[1]) + oc.start[1];
  pos[2] = (int)(rest / oc.count[1]) + oc.start[2];
  double acc = 0.0;
  for (int k = 0; k < terms.nterm[c]; ++k) {
    const Term& t = terms.t[c][k];
    const DevComp& ic = p.in.c[t.comp];
    int g0 = pos[0] + t.shift[0] - ic.start[0];
    int g1 = pos[1] + t.shift[1] - ic.start[1];
    int g2 = pos[2] + t.shift[2] - ic.start[2];
    // periodic axes: a shift of +-1 past either end re-enters at the other
    if (p.periodic & 1) g0 = g0 < 0 ? g0 + ic.count[0] : (g0 >= ic.count[0] ? g0 - ic.count[0] : g0);
    if (p.periodic & 2) g1 = g1 < 0 ? g1 + ic.count[1] : (g1 >= ic.count[1] ? g1 - ic.count[1] : g1);
    if (p.periodic & 4) g2 = g2 < 0 ? g2 + ic.count[2] : (g2 >= ic.count[2] ? g2 - ic.count[2] : g2);
    if (g0 < 0 || g0 >= ic.count[0] || g1 < 0 || g1 >= ic.count[1] || g2 < 0 || g2 >= ic.count[2]) continue;
    double v = x[ic.offset + g0 + (long long)ic.count[0] * (g1 + (long long)ic.count[1] * g2)];
    if (t.sign > 0) acc += v;
    else acc -= v;
  }
  p.y[p.out_stride * blockIdx.y + i] = acc;
}

namespace {

// Forward stencils of d (output component -> terms on the input space).
std::vector<Term> forward_terms(int op, int dim, int c) {
  auto unit = [](int a, int s) {
    Term t{};
    t.shift[a] = s;
    return t;
  };
  std::vector<Term> out;
  auto add = [&](int comp, int axis, int s, int sign) {
    Term t = axis >= 0 ? unit(axis, s) : Term{};
    t.comp = comp;
    t.sign = sign;
    out.push_back(t);
  };
  if (op == 0) {  // (G u)_c(p) = u(p + e_c) - u(p)
    add(0, c, 1, +1);
    add(0, -1, 0, -1);
  } else if (op == 1) {
    if (dim == 3) {  // b_c(p) = a_c2(p + e_c1) - a_c2(p) - a_c1(p + e_c2) + a_c1(p)
      int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      add(c2, c1, 1, +1);
      add(c2, -1, 0, -1);
      add(c1, c2, 1, -1);
      add(c1, -1, 0, +1);
    } else {  // b(p) = a_y(p + e_x) - a_y(p) - a_x(p + e_y) + a_x(p)
      add(1, 0, 1, +1);
      add(1, -1, 0, -1);
      add(0, 1, 1, -1);
      add(0, -1, 0, +1);
    }
  } else {  // (D b)(p) = sum_a b_a(p + e_a) - b_a(p)
    for (int a = 0; a < dim; ++a) {
      add(a, a, 1, +1);
      add(a, -1, 0, -1);
    }
  }
  return out;
}

}  // namespace

int launch_incidence(const IncParams& p, hipStream_t s) {
  IncTerms terms{};
  // Transposes: output component k of d^T gathers the forward terms that
  // read input component k, with the shift negated.
  int n_fwd_out = p.transpose ? p.in_ncomp : p.out_ncomp;
  for (int c = 0; c < p.out_ncomp; ++c) {
    std::vector<Term> list;
    if (!p.transpose) {
      list = forward_terms(p.op, p.dim, c);
    } else {
      for (int j = 0; j < n_fwd_out; ++j) {
        for (Term t : forward_terms(p.op, p.dim, j)) {
          if (t.comp != c) continue;
          Term u{};
          u.comp = j;
          for (int a = 0; a < 3; ++a) u.shift[a] = -t.shift[a];
          u.sign = t.sign;
          list.push_back(u);
        }
      }
    }
    // ascending input index: component block, then lattice order (a shift
    // is zero or a single +-1 along one axis, so its sign decides)
    std::sort(list.begin(), list.end(), [](const Term& a, const Term& b) {
      if (a.comp != b.comp) return a.comp < b.comp;
      int sa = a.shift[0] + a.shift[1] + a.shift[2];
      int sb = b.shift[0] + b.shift[1] + b.shift[2];
      return sa < sb;
    });
    if (list.size() > 6) return -2;
    terms.nterm[c] = (int)list.size();
    for (size_t k = 0; k < list.size(); ++k) terms.t[c][k] = list[k];
  }
  if (p.nout == 0 || p.nrhs < 1) return 0;
  long long blocks = (p.nout + 255) / 256;
  hipLaunchKernelGGL(incidence_kernel, dim3((unsigned)blocks, (unsigned)p.nrhs), dim3(256), 0, s, p, terms);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gym
