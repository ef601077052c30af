// Build step: writes the 1-D contraction tables of degrees 1..4 (Gauss rule
// q = r + 1) as C++ constants, from the same make_tables() the library uses
// at run time, so that the kernels that include the result see the very same
// values as compile-time literals (no scalar-memory loads of table entries in
// their inner loops).  Hex-float output: exact.
#include <cstdio>
#include <vector>

#include "../gym_internal.hpp"

using gym::Tables1D;

static void emit(FILE* f, const char* name, const std::vector<double>& v, int rows, int cols, int cap_r,
                 int cap_c, bool weighted, const std::vector<double>& w) {
  std::fprintf(f, "  static constexpr double %s[%d][%d] = {\n", name, cap_r, cap_c);
  for (int s = 0; s < cap_r; ++s) {
    std::fprintf(f, "      {");
    for (int i = 0; i < cap_c; ++i) {
      double x = 0.0;
      if (s < rows && i < cols) x = v[s * cols + i] * (weighted ? w[s] : 1.0);
      std::fprintf(f, "%s%a", i ? ", " : "", x);
    }
    std::fprintf(f, "},\n");
  }
  std::fprintf(f, "  };\n");
}

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: gen_tables OUT.hpp\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "w");
  if (!f) return 1;
  std::fprintf(f,
               "// Generated at build time by csrc/gen/gen_tables.cpp from make_tables(): do not edit.\n"
               "// Rows: Gauss points t (q = r + 1); columns: nodal (r + 1) or edge (r) functions;\n"
               "// the *w tables carry the Gauss weight of their row.\n"
               "#pragma once\n\nnamespace gym {\nnamespace ctabs {\n\ntemplate <int R>\nstruct Tab;\n\n");
  for (int r = 1; r <= gym::kMaxR; ++r) {
    const Tables1D t = gym::make_tables(r, r + 1);
    std::fprintf(f, "template <>\nstruct Tab<%d> {\n", r);
    emit(f, "phi", t.phi, r + 1, r + 1, r + 1, r + 1, false, t.gw);
    emit(f, "phiw", t.phi, r + 1, r + 1, r + 1, r + 1, true, t.gw);
    emit(f, "edge", t.edge, r + 1, r, r + 1, r, false, t.gw);
    emit(f, "edgew", t.edge, r + 1, r, r + 1, r, true, t.gw);
    std::fprintf(f, "  static constexpr double gx[%d] = {", r + 1);
    for (int s = 0; s <= r; ++s) std::fprintf(f, "%s%a", s ? ", " : "", t.gx[s]);
    std::fprintf(f, "};  // Gauss points on [0, 1]\n");
    std::fprintf(f, "};\n\n");
  }
  std::fprintf(f, "}  // namespace ctabs\n}  // namespace gym\n");
  return std::fclose(f) == 0 ? 0 : 1;
}
