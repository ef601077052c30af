// Sparse approximate inverse Q1 of the Lambda^1 mass matrix on affine,
// axis-aligned meshes (paper section 5), as used by the time stepping.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

struct gym_space;

namespace gym {

// One component block of Q1 (a component of Lambda^1 couples to no other on
// axis-aligned cells):
//   y = scale (Q_x (x) Q_y (x) Q_z + Q_x^T (x) Q_y^T (x) Q_z^T) x,
// the symmetrised Kronecker product of 1-D banded factors.  band[t][a]:
// count[a] rows of 2w + 1 entries, row i holding (Q_a)_{i, i+k} (t = 0) or
// (Q_a^T)_{i, i+k} (t = 1) at k + w, k = -w..w, zero outside the matrix.
struct SpaiComp {
  long long offset;  // first unknown of the block
  int count[3];      // kept lattice positions per axis
  int w;             // half bandwidth of the 1-D factors
  int wrap;          // bit a: axis a is periodic (row i, offset k couples i and (i + k) mod count)
  double scale;
  const double* band[2][3];
};
struct SpaiParams {
  SpaiComp c[3];   // unused components: offset = n
  long long n;     // unknowns of the space
  int terms;       // 2: the symmetrised pair of Kronecker terms; 1: the first only
  double* tmp[2];  // two n-vectors of scratch for the axis passes of the apply
};

// Builds Q1 = (Q + Q^T) / 2, Q the column-wise least-squares SPAI of M1 with
// the diagonal pattern (pattern 0) or the pattern of M1 (pattern 1).  On an
// axis-aligned box M1's block of component c is s_c M_x (x) M_y (x) M_z
// (1-D assembled masses, edge along c and nodal along the other axes,
// restricted to the kept positions), both patterns are Kronecker products
// of 1-D patterns, and each column's normal equations are the Kronecker
// product of 1-D normal equations: so Q's block is (1/s_c) Q_x (x) Q_y (x) Q_z
// with Q_a the 1-D SPAI of M_a.  The bands and the apply's scratch go to one
// device allocation, returned in *mem (the caller frees it).
int build_spai_q1(const gym_space* s1, int pattern, SpaiParams* out, double** mem);
// The mass matrix of an affine space as one Kronecker term of assembled 1-D
// masses (scale: the component's metric constant), applied by the same band
// passes; used for spaces with a periodic axis.  Same ownership as above.
int build_band_mass(const gym_space* sp, SpaiParams* out, double** mem);
// 1-D diagonals and row sums of the assembled masses of a space along axis a
// (nodal or edge, with the space's wrap), for Jacobi and lumped masses.
void mass1d_diag_rowsum(int r, int nel, bool nodal, int start, int count, bool periodic, std::vector<double>& diag,
                        std::vector<double>& rowsum);
// y = Q1 x, as six 1-D band passes (three per Kronecker term) through the
// scratch in p; x and y must not overlap, and applies sharing p must not
// run concurrently.
void launch_spai_apply(const SpaiParams& p, const double* x, double* y, int nb, hipStream_t s);

// Assembled 1-D mass of nel elements of degree r on the reference element,
// nodal (r nel + 1 positions) or edge (r nel), restricted to [start, start +
// count): row-major band of half width r, A[i][k + r] = A_{i, i+k}.
// periodic: positions wrap modulo count (= r nel); an entry coupling i and j
// sits in row i at the raw offset k = j - i of its element (|k| <= r), so
// that entries which wrap onto the same column (count <= 2r) are kept apart
// and summed by the apply.
std::vector<double> mass1d_band(int r, int nel, bool nodal, int start, int count, bool periodic = false);

}  // namespace gym
