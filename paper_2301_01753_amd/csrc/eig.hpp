// Block kernels and the LOBPCG driver of the generalized eigen-solver
// (paper section 3: the spectrum of K~ = Q1 P2 sets the CFL bound; the
// lowest modes of the exact operator are the paper's dispersion tests).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <vector>

namespace gym {

// Blocks of column vectors: column j of an n x m block U is U + j n.
// G (p x q, row-major, host) = U^T V, summed in a fixed order (per-block
// partials, then one pass over the partials).  p, q <= kEigMaxCols.
constexpr int kEigMaxCols = 24;
int eig_gram(const double* U, int p, const double* V, int q, long long n, double* G_host, double* work, int nb,
             hipStream_t s);
// Y (n x q) = U (n x m) C (m x q); C row-major on the device, m, q <= kEigMaxCols.
void eig_combine(const double* U, int m, const double* C_dev, int q, long long n, double* Y, int nb, hipStream_t s);
// Column j of X (n x k) scaled by f[j] (device array).
void eig_scale(double* X, const double* f_dev, int k, long long n, int nb, hipStream_t s);
// Two Gram matrices G1 = U1^T V1 and G2 = U2^T V2 with one host
// synchronisation (same summation order as eig_gram).
int eig_gram2(const double* U1, int p1, const double* V1, int q1, double* G1_host, const double* U2, int p2,
              const double* V2, int q2, double* G2_host, long long n, double* work, int nb, hipStream_t s);
// Partial-sum slots eig_gram and eig_gram2 need in `work`.
long long eig_gram_work(int nb);
// Workgroups of the block kernels for n rows: one per 256 rows, at most 4 per
// CU (short blocks, k <= 8 columns of a few 10^5 rows, leave the GPU idle
// unless the rows are spread over every CU; on long ones more workgroups only
// lengthen the serial sum over their Gram partials).
int eig_grid(long long n, int ncu);

// Generalized symmetric-definite eigenproblem A x = lambda B x, lowest k
// eigenpairs, by LOBPCG (Knyazev 2001) with Rayleigh-Ritz on [X, W, P].  The
// operators act on blocks of columns (device pointers, ncol columns of
// length n); T is the preconditioner applied to the residuals (may be empty).
struct EigOperators {
  std::function<int(const double* x, double* y, int ncol)> A, B, T;
};
struct EigResult {
  int iters = 0;
  int converged = 0;       // leading eigenpairs with relative residual <= tol
  double max_resid = 0.0;  // over the first nev pairs
};
// X: n x k device block, the initial guess on entry, the eigenvectors on exit
// (B-orthonormal).  lam: k host values, ascending.  Returns 0, a negative
// status on error, or 1 when the iteration cap was reached first.
int lobpcg(const EigOperators& ops, long long n, int k, int nev, double tol, int maxit, double* X, double* lam,
           EigResult* res, int ncu, hipStream_t s);

// Eigenvalues (ascending, w) and eigenvectors (columns of V, m x m row-major)
// of the symmetric m x m row-major matrix H by cyclic Jacobi rotations.
void jacobi_eig(std::vector<double> H, int m, std::vector<double>& w, std::vector<double>& V);
// The same for a symmetric tridiagonal matrix (diagonal d, off-diagonal e,
// e[i] coupling rows i and i + 1) by implicit-shift QL.
void tridiag_eig(std::vector<double> d, std::vector<double> e, int n, std::vector<double>& w, std::vector<double>& V);

}  // namespace gym
