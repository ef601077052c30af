// LOBPCG for the lowest eigenpairs of A x = lambda B x (Knyazev, SIAM J. Sci.
// Comput. 23 (2001)), A symmetric, B symmetric positive definite.
//
// The search space is S = [X, W, P]: the current Ritz vectors X, the
// preconditioned residuals W = T (A X - B X Lambda), B-orthogonalised
// against X, and the previous search direction P; converged columns get no
// new directions (soft locking).  A S and B S are kept alongside S (one A and one B application
// per iteration, on W), so the Rayleigh-Ritz step only needs the Gram
// matrices S^T A S and S^T B S.  W and P are scaled to unit B-norm first; if
// S^T B S is still too ill-conditioned for its Cholesky factor, P is dropped
// for that iteration.  The small projected problem (at most 24 x 24) is
// reduced with the Cholesky factor to a standard symmetric one and solved by
// cyclic Jacobi rotations on the host; every vector operation runs on the
// device.
#include "eig.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

#include "gym_internal.hpp"
#include "krylov.hpp"

namespace gym {

// Eigenvalues (ascending, w) and orthonormal eigenvectors (columns of V,
// n x n row-major) of the symmetric tridiagonal matrix with diagonal d and
// off-diagonal e (e[i] couples rows i and i + 1) by the QL iteration with
// implicit Wilkinson shifts (Bowdler, Martin, Reinsch & Wilkinson 1968),
// accumulating the plane rotations.
void tridiag_eig(std::vector<double> d, std::vector<double> e, int n, std::vector<double>& w, std::vector<double>& V) {
  std::vector<double> Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  e.resize(n, 0.0);
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 64; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 2.2e-16 * dd) break;
      }
      if (m == l) break;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool deflated = false;
      for (int i = m - 1; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          f = Z[(size_t)k * n + i + 1];
          Z[(size_t)k * n + i + 1] = s * Z[(size_t)k * n + i] + c * f;
          Z[(size_t)k * n + i] = c * Z[(size_t)k * n + i] - s * f;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] < d[b]; });
  w.resize(n);
  V.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    w[j] = d[ord[j]];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Z[(size_t)i * n + ord[j]];
  }
}

// Eigenvalues (ascending) and eigenvectors (columns of V, row-major) of the
// symmetric m x m matrix H by cyclic Jacobi rotations.
void jacobi_eig(std::vector<double> H, int m, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        tot += h(i, j) * h(i, j);
        if (i != j) off += h(i, j) * h(i, j);
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        if (h(p, q) == 0.0) continue;
        const double theta = (h(q, q) - h(p, p)) / (2.0 * h(p, q));
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {  // H <- H J (columns p, q)
          const double hp = h(k, p), hq = h(k, q);
          h(k, p) = c * hp - s * hq;
          h(k, q) = s * hp + c * hq;
        }
        for (int k = 0; k < m; ++k) {  // H <- J^T H (rows p, q)
          const double hp = h(p, k), hq = h(q, k);
          h(p, k) = c * hp - s * hq;
          h(q, k) = s * hp + c * hq;
        }
        for (int k = 0; k < m; ++k) {  // V <- V J
          const double vp = V[(size_t)k * m + p], vq = V[(size_t)k * m + q];
          V[(size_t)k * m + p] = c * vp - s * vq;
          V[(size_t)k * m + q] = s * vp + c * vq;
        }
      }
  }
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return h(a, a) < h(b, b); });
  std::vector<double> Vs((size_t)m * m);
  w.resize(m);
  for (int j = 0; j < m; ++j) {
    w[j] = h(order[j], order[j]);
    for (int i = 0; i < m; ++i) Vs[(size_t)i * m + j] = V[(size_t)i * m + order[j]];
  }
  V.swap(Vs);
}

namespace {

// Cholesky factor L (lower, row-major m x m) of G; false if a pivot is not
// positive or falls below rel times the largest diagonal entry.
bool cholesky(const std::vector<double>& G, int m, std::vector<double>& L, double rel) {
  L.assign((size_t)m * m, 0.0);
  double dmax = 0.0;
  for (int i = 0; i < m; ++i) dmax = std::max(dmax, G[(size_t)i * m + i]);
  for (int j = 0; j < m; ++j) {
    double d = G[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
    if (!(d > rel * dmax)) return false;
    const double ljj = std::sqrt(d);
    L[(size_t)j * m + j] = ljj;
    for (int i = j + 1; i < m; ++i) {
      double v = G[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
      L[(size_t)i * m + j] = v / ljj;
    }
  }
  return true;
}

// Rayleigh-Ritz on the m columns with Gram matrices GA = S^T A S, GB = S^T B S:
// the k lowest Ritz values and the coefficients C (m x k, row-major) of their
// vectors.  False if GB is not safely positive definite.
bool rayleigh_ritz(std::vector<double> GA, std::vector<double> GB, int m, int k, std::vector<double>& lam,
                   std::vector<double>& C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) {
      const double a = 0.5 * (GA[(size_t)i * m + j] + GA[(size_t)j * m + i]);
      const double b = 0.5 * (GB[(size_t)i * m + j] + GB[(size_t)j * m + i]);
      GA[(size_t)i * m + j] = GA[(size_t)j * m + i] = a;
      GB[(size_t)i * m + j] = GB[(size_t)j * m + i] = b;
    }
  std::vector<double> L;
  if (!cholesky(GB, m, L, 1e-13)) return false;
  // H = L^-1 GA L^-T: Z = L^-1 GA (columns), H = L^-1 Z^T
  std::vector<double> Z((size_t)m * m), H((size_t)m * m);
  auto lsolve = [&](const std::vector<double>& R, std::vector<double>& O) {  // O = L^-1 R
    for (int c = 0; c < m; ++c)
      for (int i = 0; i < m; ++i) {
        double v = R[(size_t)i * m + c];
        for (int j = 0; j < i; ++j) v -= L[(size_t)i * m + j] * O[(size_t)j * m + c];
        O[(size_t)i * m + c] = v / L[(size_t)i * m + i];
      }
  };
  lsolve(GA, Z);
  std::vector<double> Zt((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Zt[(size_t)i * m + j] = Z[(size_t)j * m + i];
  lsolve(Zt, H);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) H[(size_t)i * m + j] = H[(size_t)j * m + i] = 0.5 * (H[(size_t)i * m + j] + H[(size_t)j * m + i]);
  std::vector<double> w, Y;
  jacobi_eig(H, m, w, Y);
  lam.assign(w.begin(), w.begin() + k);
  // C = L^-T Y[:, :k]: back substitution with L^T
  C.assign((size_t)m * k, 0.0);
  for (int c = 0; c < k; ++c)
    for (int i = m - 1; i >= 0; --i) {
      double v = Y[(size_t)i * m + c];
      for (int j = i + 1; j < m; ++j) v -= L[(size_t)j * m + i] * C[(size_t)j * k + c];
      C[(size_t)i * k + c] = v / L[(size_t)i * m + i];
    }
  return true;
}

}  // namespace

int lobpcg(const EigOperators& ops, long long n, int k, int nev, double tol, int maxit, double* X, double* lam_out,
           EigResult* res, int ncu, hipStream_t s) {
  if (k < 1 || 3 * k > kEigMaxCols || nev < 1 || nev > k || n < 3 * k) return GYM_E_ARG;
  const int nb = eig_grid(n, ncu);
  const long long nk = n * k;
  // S, AS, BS (3k columns each), the residual, new X / AX / BX, new P / AP / BP
  std::vector<double*> bufs;
  auto alloc = [&](long long cnt) -> double* {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(double) * cnt) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    bufs.push_back((double*)p);
    return (double*)p;
  };
  auto release = [&] {
    for (double* p : bufs) (void)hipFree(p);
  };
  double* S = alloc(3 * nk);
  double* AS = alloc(3 * nk);
  double* BS = alloc(3 * nk);
  double* R = alloc(nk);
  double* NX = alloc(3 * nk);
  double* NP = alloc(3 * nk);
  double* gw = alloc(eig_gram_work(nb));
  double* cdev = alloc(kEigMaxCols * kEigMaxCols + kEigMaxCols);
  if (!S || !AS || !BS || !R || !NX || !NP || !gw || !cdev) {
    release();
    return fail(GYM_E_OOM, "eigen-solver: device allocation failed");
  }
  double* fdev = cdev + kEigMaxCols * kEigMaxCols;
  auto col = [&](double* base, int j) { return base + (long long)j * n; };
  // Small host arrays go over asynchronously from a ring of pinned slots; a
  // slot is written again only after a stream synchronisation (every Gram
  // matrix brings one; otherwise the ring waits for its oldest copy).
  constexpr int kRing = 16;
  constexpr size_t kSlot = (size_t)kEigMaxCols * kEigMaxCols + kEigMaxCols;
  double* ring = nullptr;
  if (hipHostMalloc((void**)&ring, sizeof(double) * kRing * kSlot) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(GYM_E_OOM, "eigen-solver: pinned staging allocation failed");
  }
  int ring_pos = 0, since_sync = 0;
  auto upload = [&](const std::vector<double>& v, double* dst) {
    if (v.size() > kSlot) return -1;
    if (since_sync == kRing) {
      if (hipStreamSynchronize(s) != hipSuccess) return -1;
      since_sync = 0;
    }
    double* h = ring + (size_t)ring_pos * kSlot;
    std::copy(v.begin(), v.end(), h);
    ring_pos = (ring_pos + 1) % kRing;
    ++since_sync;
    return hipMemcpyAsync(dst, h, sizeof(double) * v.size(), hipMemcpyHostToDevice, s) == hipSuccess ? 0 : -1;
  };
  auto gram = [&](const double* U, int p, const double* V, int q, double* G) {
    const int rc = eig_gram(U, p, V, q, n, G, gw, nb, s);
    since_sync = 0;
    return rc;
  };
  auto gram2 = [&](const double* U1, int p1, const double* V1, int q1, double* G1, const double* U2, int p2,
                   const double* V2, int q2, double* G2) {
    const int rc = eig_gram2(U1, p1, V1, q1, G1, U2, p2, V2, q2, G2, n, gw, nb, s);
    since_sync = 0;
    return rc;
  };
  auto copy = [&](double* dst, const double* src, long long cnt) {
    return hipMemcpyAsync(dst, src, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s) == hipSuccess ? 0 : -1;
  };
  // columns of (U, AU, BU) scaled to unit B-norm
  // the nc columns of (U, AU, BU) scaled to unit B-norm
  auto normalize = [&](double* U, double* AU, double* BU, int nc) -> int {
    std::vector<double> G((size_t)nc * nc);
    if (gram(U, nc, BU, nc, G.data())) return -1;
    std::vector<double> f(nc);
    for (int j = 0; j < nc; ++j) {
      const double d = G[(size_t)j * nc + j];
      f[j] = d > 0 ? 1.0 / std::sqrt(d) : 0.0;
    }
    if (upload(f, fdev)) return -1;
    eig_scale(U, fdev, nc, n, nb, s);
    if (AU) eig_scale(AU, fdev, nc, n, nb, s);
    eig_scale(BU, fdev, nc, n, nb, s);
    return 0;
  };
  int status = 0;
  std::vector<double> lam(k, 0.0), C;
  int np = 0;  // P present
  res->iters = 0;
  res->converged = 0;
  res->max_resid = 0.0;
  do {
    // X: copy in, B X, unit B-norm, A X, Rayleigh-Ritz on X alone
    if (copy(S, X, nk)) { status = -1; break; }
    if ((status = ops.B(S, BS, k))) break;
    if (normalize(S, nullptr, BS, k)) { status = -1; break; }
    if ((status = ops.A(S, AS, k))) break;
    {
      std::vector<double> GA((size_t)k * k), GB((size_t)k * k);
      if (gram2(S, k, AS, k, GA.data(), S, k, BS, k, GB.data())) {
        status = -1;
        break;
      }
      if (!rayleigh_ritz(GA, GB, k, k, lam, C)) {
        status = fail(GYM_E_BREAKDOWN, "eigen-solver: initial block is rank deficient");
        break;
      }
      if (upload(C, cdev)) { status = -1; break; }
      eig_combine(S, k, cdev, k, n, col(NX, 0), nb, s);
      eig_combine(AS, k, cdev, k, n, col(NX, k), nb, s);
      eig_combine(BS, k, cdev, k, n, col(NX, 2 * k), nb, s);
      if (copy(S, col(NX, 0), nk) || copy(AS, col(NX, k), nk) || copy(BS, col(NX, 2 * k), nk)) { status = -1; break; }
    }
    status = 1;  // not converged unless the loop says so
    std::vector<int> prev_act;
    // A X, B X (and A P, B P) are carried as linear combinations, whose
    // rounding drifts from the true products over hundreds of iterations;
    // they are recomputed every kRefresh iterations and before convergence
    // is accepted.
    constexpr int kRefresh = 16;
    bool fresh = true;
    auto refresh = [&]() -> int {
      if (int rc = ops.A(S, AS, k)) return rc;
      if (int rc = ops.B(S, BS, k)) return rc;
      const int kp = (int)prev_act.size();
      if (np && kp > 0) {
        if (int rc = ops.A(col(S, k + kp), col(AS, k + kp), kp)) return rc;
        if (int rc = ops.B(col(S, k + kp), col(BS, k + kp), kp)) return rc;
      }
      fresh = true;
      return 0;
    };
    std::vector<double> rel(k);
    for (int it = 0; it < maxit; ++it) {
      res->iters = it;
      if (it > 0 && it % kRefresh == 0 && !fresh) {
        if (int rc = refresh()) { status = rc; break; }
      }
      for (int pass = 0; pass < 2; ++pass) {
        // residuals A X - B X Lambda of all k columns and their relative norms
        {
          std::vector<double> Cr((size_t)2 * k * k, 0.0);  // [AX; BX] -> R: identity over -Lambda
          for (int j = 0; j < k; ++j) {
            Cr[(size_t)j * k + j] = 1.0;
            Cr[(size_t)(k + j) * k + j] = -lam[j];
          }
          // AX and BX are not adjacent in memory: stage them side by side in NP
          if (copy(col(NP, 0), AS, nk) || copy(col(NP, k), BS, nk) || upload(Cr, cdev)) { status = -1; break; }
          eig_combine(NP, 2 * k, cdev, k, n, R, nb, s);
        }
        std::vector<double> GR((size_t)k * k), GX((size_t)k * k);
        if (gram2(R, k, R, k, GR.data(), BS, k, BS, k, GX.data())) {
          status = -1;
          break;
        }
        for (int j = 0; j < k; ++j) {
          const double rn = std::sqrt(std::max(0.0, GR[(size_t)j * k + j]));
          const double bn = std::sqrt(std::max(0.0, GX[(size_t)j * k + j]));
          rel[j] = rn / (std::max(std::fabs(lam[j]), 1e-300) * std::max(bn, 1e-300));
        }
        double worst = 0.0;
        int conv = 0;
        for (int j = 0; j < nev; ++j) {
          worst = std::max(worst, rel[j]);
          if (rel[j] <= tol && conv == j) conv = j + 1;
        }
        res->converged = conv;
        res->max_resid = worst;
        if (conv < nev || fresh) break;
        if (int rc = refresh()) { status = rc; break; }  // converged on carried products: confirm
      }
      if (status != 1) break;
      if (res->converged == nev) {
        status = 0;
        break;
      }
      // soft locking: only the columns still above tol get search directions
      std::vector<int> act;
      for (int j = 0; j < k; ++j)
        if (rel[j] > tol) act.push_back(j);
      const int ka = (int)act.size();
      if (act != prev_act) np = 0;  // P belongs to the previous active set
      // W = T R over the active columns, B W, B-orthogonal to X, unit B-norm, A W
      double* W = col(S, k);
      {
        std::vector<double> Ca((size_t)k * ka, 0.0);  // R -> its active columns
        for (int a = 0; a < ka; ++a) Ca[(size_t)act[a] * ka + a] = 1.0;
        if (upload(Ca, cdev)) { status = -1; break; }
        eig_combine(R, k, cdev, ka, n, col(NX, 0), nb, s);
      }
      if (ops.T) {
        if (int rc = ops.T(col(NX, 0), W, ka)) { status = rc; break; }
      } else if (copy(W, col(NX, 0), n * ka)) {
        status = -1;
        break;
      }
      if (int rc = ops.B(W, col(BS, k), ka)) { status = rc; break; }
      // W -= X (X^T B W) and the same for B W (X is B-orthonormal): a
      // converging residual is otherwise nearly in the span of X
      {
        std::vector<double> GXW((size_t)k * ka);
        if (gram(S, k, col(BS, k), ka, GXW.data())) { status = -1; break; }
        std::vector<double> Co((size_t)(k + ka) * ka, 0.0);  // [X W] -> W - X GXW
        for (int i = 0; i < k; ++i)
          for (int j = 0; j < ka; ++j) Co[(size_t)i * ka + j] = -GXW[(size_t)i * ka + j];
        for (int j = 0; j < ka; ++j) Co[(size_t)(k + j) * ka + j] = 1.0;
        if (upload(Co, cdev)) { status = -1; break; }
        eig_combine(S, k + ka, cdev, ka, n, col(NX, 0), nb, s);
        eig_combine(BS, k + ka, cdev, ka, n, col(NX, ka), nb, s);
        if (copy(W, col(NX, 0), n * ka) || copy(col(BS, k), col(NX, ka), n * ka)) { status = -1; break; }
      }
      if (normalize(W, nullptr, col(BS, k), ka)) { status = -1; break; }
      if (int rc = ops.A(W, col(AS, k), ka)) { status = rc; break; }
      // Rayleigh-Ritz on [X W P], dropping P if the basis is too ill-conditioned
      int m = np ? k + 2 * ka : k + ka;
      bool ok = false;
      while (!ok) {
        std::vector<double> GA((size_t)m * m), GB((size_t)m * m);
        if (gram2(S, m, AS, m, GA.data(), S, m, BS, m, GB.data())) break;
        ok = rayleigh_ritz(GA, GB, m, k, lam, C);
        if (!ok) {
          if (m == k + 2 * ka) m = k + ka;
          else break;
        }
      }
      if (!ok) {
        status = fail(GYM_E_BREAKDOWN, "eigen-solver: search space lost rank");
        break;
      }
      // new X, A X, B X; new P = the [W P] part of the combination, active columns
      if (upload(C, cdev)) { status = -1; break; }
      eig_combine(S, m, cdev, k, n, col(NX, 0), nb, s);
      eig_combine(AS, m, cdev, k, n, col(NX, k), nb, s);
      eig_combine(BS, m, cdev, k, n, col(NX, 2 * k), nb, s);
      std::vector<double> Cp((size_t)(m - k) * ka);
      for (int i = k; i < m; ++i)
        for (int a = 0; a < ka; ++a) Cp[(size_t)(i - k) * ka + a] = C[(size_t)i * k + act[a]];
      if (upload(Cp, cdev)) { status = -1; break; }
      eig_combine(col(S, k), m - k, cdev, ka, n, col(NP, 0), nb, s);
      eig_combine(col(AS, k), m - k, cdev, ka, n, col(NP, ka), nb, s);
      eig_combine(col(BS, k), m - k, cdev, ka, n, col(NP, 2 * ka), nb, s);
      const long long nka = n * ka;
      if (copy(S, col(NX, 0), nk) || copy(AS, col(NX, k), nk) || copy(BS, col(NX, 2 * k), nk) ||
          copy(col(S, k + ka), col(NP, 0), nka) || copy(col(AS, k + ka), col(NP, ka), nka) ||
          copy(col(BS, k + ka), col(NP, 2 * ka), nka)) {
        status = -1;
        break;
      }
      if (normalize(col(S, k + ka), col(AS, k + ka), col(BS, k + ka), ka)) { status = -1; break; }
      np = 1;
      prev_act = act;
      fresh = false;
      res->iters = it + 1;
    }
  } while (false);
  if (status >= 0) {
    if (copy(X, S, nk) || hipStreamSynchronize(s) != hipSuccess) status = -1;
    for (int j = 0; j < k; ++j) lam_out[j] = lam[j];
  }
  if (status == -1) status = hip_fail(hipGetLastError(), "eigen-solver");
  (void)hipStreamSynchronize(s);
  (void)hipHostFree(ring);
  release();
  return status;
}

}  // namespace gym
