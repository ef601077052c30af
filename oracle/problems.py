"""Block operators, manufactured solutions and solves (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper poses Maxwell's equations; the two elliptic problems here are
built only from its objects (G, C, D and the masses M_p of section 2) and
are readings of the workloads, not statements of the paper:

Mixed Poisson (H(div) x L2, sigma = -grad u, div sigma = f, u = 0 on the
boundary imposed naturally):
    [ M2      -D^T M3 ] [s]   [  0 ]
    [ -M3 D      0    ] [p] = [ -F ],   F_i = int f Lambda^d_i.

Hodge Laplacian on 1-forms (sigma in H1_0, u in H0(curl), the mixed form of
-Delta u = f; C^T M2 C is the paper's curl-of-curl P2 / c^2 of section 3):
    [ -M0     G^T M1    ] [sigma]   [ 0 ]
    [ M1 G    C^T M2 C  ] [  u  ] = [ F ].

Both matrices are symmetric indefinite.  The diagonal preconditioner is
block Jacobi: diag(M2 + D^T M3 D), diag(M3) for Poisson and
diag(M0 + G^T M1 G), diag(M1 + C^T M2 C) for Hodge (a reading; the paper uses
only a diagonal preconditioner, for its Sylvester PCG).

Manufactured fields (reading of "random Fourier coefficients, 8 modes"):
modes (a, b, c) in {1, 2}^3.  Poisson: u = sum c_m sin(a pi x) sin(b pi y)
sin(c pi z).  Hodge: u = sum (c^x_m cos sin sin, c^y_m sin cos sin,
c^z_m sin sin cos).  Each mode has f = pi^2 (a^2 + b^2 + c^2) x mode.

Pins: tests/test_oracle_problems.py (exact polynomial solutions reproduced
to round-off, convergence rates, residuals of MINRES against spsolve).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assembly, incidence
from .lattice import Space


class MixedPoisson:
    def __init__(self, mesh, r):
        self.mesh = mesh
        self.r = r
        self.sdiv = Space("HDIV", mesh.nel, r, "natural")
        self.sl2 = Space("L2", mesh.nel, r, "natural")
        self.M2 = assembly.mass_matrix(self.sdiv, mesh)
        self.M3 = assembly.mass_matrix(self.sl2, mesh)
        self.D = incidence.divergence(self.sdiv, self.sl2).astype(np.float64)
        B = -(self.M3 @ self.D)
        self.A = sp.bmat([[self.M2, B.T], [B, None]], format="csr")
        self.n = (self.sdiv.ndofs, self.sl2.ndofs)

    def precond_diag(self):
        d1 = (self.M2 + self.D.T @ self.M3 @ self.D).diagonal()
        d2 = self.M3.diagonal()
        return np.concatenate([d1, d2])

    def rhs(self, f):
        F = assembly.load_vector(self.sl2, self.mesh, f)
        return np.concatenate([np.zeros(self.sdiv.ndofs), -F])

    def split(self, x):
        return x[:self.n[0]], x[self.n[0]:]


class Hodge1:
    def __init__(self, mesh, r):
        self.mesh = mesh
        self.r = r
        d = mesh.dim
        self.s0 = Space("H1", mesh.nel, r, "essential")
        self.s1 = Space("HCURL", mesh.nel, r, "essential")
        self.s2 = Space("HDIV" if d == 3 else "L2", mesh.nel, r, "natural")
        self.M0 = assembly.mass_matrix(self.s0, mesh)
        self.M1 = assembly.mass_matrix(self.s1, mesh)
        self.M2 = assembly.mass_matrix(self.s2, mesh)
        self.G = incidence.gradient(self.s0, self.s1).astype(np.float64)
        self.C = incidence.curl(self.s1, self.s2).astype(np.float64)
        self.P2 = (self.C.T @ self.M2 @ self.C).tocsr()
        B = self.M1 @ self.G
        self.A = sp.bmat([[-self.M0, B.T], [B, self.P2]], format="csr")
        self.n = (self.s0.ndofs, self.s1.ndofs)

    def precond_diag(self):
        d1 = (self.M0 + self.G.T @ self.M1 @ self.G).diagonal()
        d2 = (self.M1 + self.P2).diagonal()
        return np.concatenate([d1, d2])

    def rhs(self, f):
        F = assembly.load_vector(self.s1, self.mesh, f)
        return np.concatenate([np.zeros(self.s0.ndofs), F])

    def split(self, x):
        return x[:self.n[0]], x[self.n[0]:]


def modes_3d():
    """The 8 wave-number triples (a, b, c) in {1, 2}^3, a fastest."""
    return [(a, b, c) for c in (1, 2) for b in (1, 2) for a in (1, 2)]


def poisson_fields(coeffs, modes):
    """(u, sigma, f) callables for u = sum c_m prod sin(k_i pi x_i)."""
    modes = [np.asarray(m, float) for m in modes]
    coeffs = np.asarray(coeffs, float)
    pi = np.pi

    def u(x):
        out = np.zeros(x.shape[0])
        for cm, k in zip(coeffs, modes):
            out += cm * np.prod(np.sin(k[None, :] * pi * x), axis=1)
        return out

    def sigma(x):
        d = x.shape[1]
        out = np.zeros_like(x)
        for cm, k in zip(coeffs, modes):
            s = np.sin(k[None, :] * pi * x)
            c = np.cos(k[None, :] * pi * x)
            for a in range(d):
                term = k[a] * pi * c[:, a]
                for b in range(d):
                    if b != a:
                        term = term * s[:, b]
                out[:, a] -= cm * term
        return out

    def f(x):
        out = np.zeros(x.shape[0])
        for cm, k in zip(coeffs, modes):
            out += cm * pi ** 2 * np.sum(k ** 2) * np.prod(np.sin(k[None, :] * pi * x), axis=1)
        return out

    return u, sigma, f


def hodge_fields(coeffs, modes):
    """(u, sigma = -div u, f = -Delta u) for the 3-D vector Fourier field.

    coeffs has shape (len(modes), 3); component a of mode k is
    c_a cos(k_a pi x_a) prod_{b != a} sin(k_b pi x_b)."""
    modes = [np.asarray(m, float) for m in modes]
    coeffs = np.asarray(coeffs, float).reshape(len(modes), -1)
    pi = np.pi

    def u(x):
        d = x.shape[1]
        out = np.zeros_like(x)
        for cm, k in zip(coeffs, modes):
            s = np.sin(k[None, :] * pi * x)
            c = np.cos(k[None, :] * pi * x)
            for a in range(d):
                term = cm[a] * c[:, a]
                for b in range(d):
                    if b != a:
                        term = term * s[:, b]
                out[:, a] += term
        return out

    def sigma(x):
        d = x.shape[1]
        out = np.zeros(x.shape[0])
        for cm, k in zip(coeffs, modes):
            s = np.sin(k[None, :] * pi * x)
            for a in range(d):
                # d/dx_a of c_a cos(k_a pi x_a) ... = -c_a k_a pi sin(...) prod sin
                out += cm[a] * k[a] * pi * np.prod(s, axis=1)
        return out

    def f(x):
        d = x.shape[1]
        out = np.zeros_like(x)
        for cm, k in zip(coeffs, modes):
            s = np.sin(k[None, :] * pi * x)
            c = np.cos(k[None, :] * pi * x)
            lam = pi ** 2 * np.sum(k ** 2)
            for a in range(d):
                term = cm[a] * lam * c[:, a]
                for b in range(d):
                    if b != a:
                        term = term * s[:, b]
                out[:, a] += term
        return out

    return u, sigma, f


def solve_direct(A, b):
    """SuperLU solve of the assembled block system."""
    return spla.spsolve(A.tocsc(), b)


def solve_minres(A, b, diag, rtol=1e-13, maxiter=100000):
    """Preconditioned MINRES (SciPy) with the block-Jacobi diagonal."""
    Minv = sp.diags(1.0 / diag)
    x, info = spla.minres(A, b, M=Minv, rtol=rtol, maxiter=maxiter)
    return x, info


def mass_cg(M, b, rtol=1e-14, maxiter=10000):
    """CG on M x = b with a Jacobi preconditioner (the exact-FEEC mass solve)."""
    Minv = sp.diags(1.0 / M.diagonal())
    x, info = spla.cg(M, b, M=Minv, rtol=rtol, maxiter=maxiter)
    return x, info


def schur_preconditioner(P):
    """Block preconditioner of the mixed Poisson system (a reading: the paper
    preconditions only with a diagonal, section 5.1).  With A's blocks M2 and
    B = -M3 D, the preconditioner is diag(diag(M2), S), S = B diag(M2)^-1 B^T
    = M3 D diag(M2)^-1 D^T M3: the Schur complement of the system whose flux
    block is replaced by its diagonal.  Returns (apply, S, d): apply(y) =
    [y_s / d; S^-1 y_p] by a sparse direct solve, d = diag(M2)."""
    d = P.M2.diagonal().copy()
    B = -(P.M3 @ P.D)
    S = (B @ sp.diags(1.0 / d) @ B.T).tocsc()
    lu = spla.splu(S)
    ns = d.size

    def apply(y):
        y = np.asarray(y, dtype=float)
        return np.concatenate([y[:ns] / d, lu.solve(y[ns:])])

    return apply, S, d


def solve_minres_prec(A, b, apply, rtol=1e-13, maxiter=100000):
    """SciPy MINRES with a preconditioner given as a function z = M^-1 y;
    returns (x, info, iterations)."""
    n = A.shape[0]
    M = spla.LinearOperator((n, n), matvec=apply, dtype=float)
    its = [0]

    def cb(_):
        its[0] += 1

    x, info = spla.minres(A, b, M=M, rtol=rtol, maxiter=maxiter, callback=cb)
    return x, info, its[0]
