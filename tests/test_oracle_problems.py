"""Pins of the oracle's block systems and solves: exact polynomial solutions,
convergence rates, MINRES against a direct solve, manufactured fields."""
import numpy as np
import pytest

import synth
from oracle import assembly, problems
from oracle.lattice import Mesh, Space


def test_hodge_reproduces_polynomial_solution():
    # u = (y(1-y)z(1-z), x(1-x)z(1-z), x(1-x)y(1-y)) lies in Q_2^- Lambda^1 with
    # zero tangential trace, sigma = -div u = 0 and f = -Delta u.  Galerkin plus
    # uniqueness: the discrete solution is the de Rham projection of u.
    nel = (3, 2, 3)
    mesh = Mesh(synth.uniform_vertices(nel))
    P = problems.Hodge1(mesh, 2)
    b = lambda t: t * (1 - t)
    x, y, z = (lambda X: X[:, 0]), (lambda X: X[:, 1]), (lambda X: X[:, 2])
    u = lambda X: np.stack([b(y(X)) * b(z(X)), b(x(X)) * b(z(X)), b(x(X)) * b(y(X))], 1)
    f = lambda X: 2 * np.stack([b(y(X)) + b(z(X)), b(x(X)) + b(z(X)), b(x(X)) + b(y(X))], 1)
    sol = problems.solve_direct(P.A, P.rhs(f))
    sig, uh = P.split(sol)
    assert np.abs(sig).max() < 1e-12
    assert np.abs(uh - assembly.de_rham(P.s1, mesh, u)).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_mixed_poisson_reproduces_polynomial_solution(dim):
    # u = prod x_i (1 - x_i): sigma = -grad u is in Q_3^- (H(div)), u in Q_3^- L2.
    nel = (2, 3) if dim == 2 else (2, 2, 2)
    mesh = Mesh(synth.uniform_vertices(nel))
    P = problems.MixedPoisson(mesh, 3)
    b = lambda t: t * (1 - t)
    db = lambda t: 1 - 2 * t

    def u(X):
        return np.prod(b(X), axis=1)

    def sigma(X):
        out = np.zeros_like(X)
        for a in range(dim):
            term = -db(X[:, a])
            for c in range(dim):
                if c != a:
                    term = term * b(X[:, c])
            out[:, a] = term
        return out

    def f(X):
        out = np.zeros(X.shape[0])
        for a in range(dim):
            term = 2.0 * np.ones(X.shape[0])
            for c in range(dim):
                if c != a:
                    term = term * b(X[:, c])
            out += term
        return out

    sol = problems.solve_direct(P.A, P.rhs(f))
    s, p = P.split(sol)
    assert np.abs(s - assembly.de_rham(P.sdiv, mesh, sigma)).max() < 1e-12
    assert np.abs(p - assembly.de_rham(P.sl2, mesh, u)).max() < 1e-12


def _poisson2d_errors(N, r):
    mesh = Mesh(synth.uniform_vertices((N, N)))
    P = problems.MixedPoisson(mesh, r)
    u, sig, f = problems.poisson_fields([1.0], [(1, 1)])
    s, p = P.split(problems.solve_direct(P.A, P.rhs(f)))
    eu = assembly.l2_error(P.sl2, mesh, p, u)
    es = assembly.l2_error(P.sdiv, mesh, s, sig)
    return eu[0] / eu[1], es[0] / es[1]


@pytest.mark.parametrize("r", [1, 2])
def test_mixed_poisson_rates_2d(r):
    # Optimal O(h^r) L2 rates for both fields on uniform meshes.
    e1 = _poisson2d_errors(8, r)
    e2 = _poisson2d_errors(16, r)
    for a, b in zip(e1, e2):
        assert np.log2(a / b) > r - 0.15


def test_hodge_rate_3d():
    errs = []
    for N in (2, 4):
        mesh = Mesh(synth.uniform_vertices((N, N, N)))
        P = problems.Hodge1(mesh, 2)
        c = synth.fourier_coeffs(0, 8, 3)
        u, sig, f = problems.hodge_fields(c[:1], synth.modes_3d()[:1])
        _, uh = P.split(problems.solve_direct(P.A, P.rhs(f)))
        e = assembly.l2_error(P.s1, mesh, uh, u)
        errs.append(e[0] / e[1])
    assert np.log2(errs[0] / errs[1]) > 2 - 0.3


def test_manufactured_fields_are_consistent():
    # f = -Delta u, sigma = -grad u (Poisson) and sigma = -div u (Hodge), by
    # central differences at random points.
    rng = np.random.default_rng(1)
    X = rng.uniform(0.1, 0.9, (20, 3))
    h = 1e-4
    c = synth.fourier_coeffs(4, 8, 1)[:, 0]
    u, sig, f = problems.poisson_fields(c, synth.modes_3d())
    lap = sum((u(X + h * np.eye(3)[a]) - 2 * u(X) + u(X - h * np.eye(3)[a])) / h ** 2 for a in range(3))
    assert np.abs(-lap - f(X)).max() < 1e-4 * np.abs(f(X)).max()
    g = np.stack([(u(X + h * np.eye(3)[a]) - u(X - h * np.eye(3)[a])) / (2 * h) for a in range(3)], 1)
    assert np.abs(-g - sig(X)).max() < 1e-6 * np.abs(sig(X)).max()
    c3 = synth.fourier_coeffs(5, 8, 3)
    u, sig, f = problems.hodge_fields(c3, synth.modes_3d())
    div = sum((u(X + h * np.eye(3)[a])[:, a] - u(X - h * np.eye(3)[a])[:, a]) / (2 * h) for a in range(3))
    assert np.abs(-div - sig(X)).max() < 1e-6 * np.abs(sig(X)).max()
    lap = sum((u(X + h * np.eye(3)[a]) - 2 * u(X) + u(X - h * np.eye(3)[a])) / h ** 2 for a in range(3))
    assert np.abs(-lap - f(X)).max() < 1e-4 * np.abs(f(X)).max()
    # essential trace: tangential components vanish on the boundary
    B = rng.uniform(0, 1, (10, 3))
    B[:, 0] = 0.0
    assert np.abs(u(B)[:, 1:]).max() < 1e-14


@pytest.mark.parametrize("which", ["poisson", "hodge"])
def test_minres_matches_direct(which):
    nel = (3, 3, 2)
    mesh = Mesh(synth.perturbed_vertices(nel, 0.15, seed=7))
    P = problems.MixedPoisson(mesh, 2) if which == "poisson" else problems.Hodge1(mesh, 2)
    b = synth.random_vector(P.A.shape[0], seed=3)
    xd = problems.solve_direct(P.A, b)
    xm, info = problems.solve_minres(P.A, b, P.precond_diag(), rtol=1e-13)
    assert info == 0
    assert np.linalg.norm(xm - xd) / np.linalg.norm(xd) < 1e-9


def test_block_operator_symmetric():
    nel = (2, 2, 2)
    mesh = Mesh(synth.perturbed_vertices(nel, 0.15, seed=9))
    for P in (problems.MixedPoisson(mesh, 2), problems.Hodge1(mesh, 2)):
        A = P.A.toarray()
        assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
        assert np.all(P.precond_diag() > 0)


def test_mass_cg_solves():
    nel = (3, 3, 3)
    mesh = Mesh(synth.perturbed_vertices(nel, 0.15, seed=4))
    s1 = Space("HCURL", nel, 2)
    M = assembly.mass_matrix(s1, mesh)
    b = synth.random_vector(s1.ndofs, seed=1)
    x, info = problems.mass_cg(M, b)
    assert info == 0
    assert np.linalg.norm(M @ x - b) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("which,nel,r,perturb", [("hodge", (6, 7, 5), 2, 0.0), ("hodge", (5, 6, 6), 1, 0.15),
                                                 ("poisson", (6, 5, 7), 2, 0.15), ("poisson", (5, 5, 6), 3, 0.0)])
def test_patch_rows_equal_global_rows(which, nel, r, perturb):
    # The full-size GPU tests sample rows of the global operator from an
    # oracle patch; on meshes small enough to assemble whole, those rows must
    # equal the global ones exactly (up to summation order), at the domain's
    # corners (boundary conditions) and inside.
    from patch_rows import origins, patch_rows
    verts = synth.perturbed_vertices(nel, perturb, seed=8) if perturb else synth.uniform_vertices(nel)
    P = problems.Hodge1(Mesh(verts), r) if which == "hodge" else problems.MixedPoisson(Mesh(verts), r)
    A = P.A.tocsr()
    x = synth.random_vector(A.shape[0], seed=13)
    y = A @ x
    for origin, mid in origins(nel, np.random.default_rng(3)):
        Ap, gmap, rows = patch_rows(which, verts, nel, r, origin, mid)
        yp = (Ap @ x[gmap])[rows]
        assert len(rows) > 0
        assert np.abs(yp - y[gmap[rows]]).max() <= 1e-13 * np.abs(y).max()
