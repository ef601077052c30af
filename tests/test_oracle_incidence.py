"""Pins of the oracle's incidence matrices: the complex, its cohomology,
the paper's finite-difference stencils and Stokes' theorem."""
import numpy as np
import pytest

import synth
from oracle import assembly, incidence, lattice
from oracle.lattice import Mesh, Space


def spaces3(nel, r, bc):
    return [Space(k, nel, r, bc) for k in ("H1", "HCURL", "HDIV", "L2")]


@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("bc", ["natural", "essential"])
def test_d_squared_is_zero(r, bc):
    # Section 2: CG = 0 and DC = 0, exactly as integer matrices.
    s0, s1, s2, s3 = spaces3((2, 3, 2), r, bc)
    G = incidence.gradient(s0, s1).astype(np.int64)
    C = incidence.curl(s1, s2).astype(np.int64)
    D = incidence.divergence(s2, s3).astype(np.int64)
    assert (C @ G).count_nonzero() == 0
    assert (D @ C).count_nonzero() == 0
    assert set(np.unique(G.data)) <= {-1, 1}
    assert set(np.unique(C.data)) <= {-1, 1}


def test_d_squared_is_zero_2d():
    s0 = Space("H1", (3, 4), 2)
    s1 = Space("HCURL", (3, 4), 2)
    s2 = Space("L2", (3, 4), 2)
    G = incidence.gradient(s0, s1).astype(np.int64)
    C = incidence.curl(s1, s2).astype(np.int64)
    assert (C @ G).count_nonzero() == 0


@pytest.mark.parametrize("bc,chi", [("natural", 1), ("essential", -1)])
def test_euler_characteristic(bc, chi):
    for r in (1, 2, 3):
        s = spaces3((2, 3, 4), r, bc)
        assert s[0].ndofs - s[1].ndofs + s[2].ndofs - s[3].ndofs == chi


@pytest.mark.parametrize("bc", ["natural", "essential"])
def test_exactness_by_rank(bc):
    # The cube has trivial cohomology: im d = ker d at every interior slot.
    s0, s1, s2, s3 = spaces3((2, 2, 1), 2, bc)
    G = incidence.gradient(s0, s1).toarray().astype(float)
    C = incidence.curl(s1, s2).toarray().astype(float)
    D = incidence.divergence(s2, s3).toarray().astype(float)
    rk = np.linalg.matrix_rank
    rG, rC, rD = rk(G), rk(C), rk(D)
    if bc == "natural":
        assert rG == s0.ndofs - 1           # ker G = constants
        assert rD == s3.ndofs               # D onto
    else:
        assert rG == s0.ndofs               # no constants with zero trace
        assert rD == s3.ndofs - 1           # image has zero mean
    assert s1.ndofs - rC == rG              # ker C = im G
    assert s2.ndofs - rD == rC              # ker D = im C


def test_curl_is_the_papers_finite_difference():
    # Section 4.2, eq. (dIsFiniteDiff): for Whitney forms with average-value
    # DoFs, b_face = (1/dx)(a_right - a_left) - (1/dy)(a_top - a_bottom) on a
    # z-normal face.  Average DoFs are integral DoFs divided by |sigma|.
    nel = (3, 4, 2)
    hi = (1.5, 2.0, 0.8)
    dx, dy, dz = (hi[a] / nel[a] for a in range(3))
    mesh = Mesh(synth.uniform_vertices(nel, hi=hi))
    s1 = Space("HCURL", nel, 1)
    s2 = Space("HDIV", nel, 1)
    C = incidence.curl(s1, s2).toarray().astype(float)
    D1 = lattice.cell_measures(s1, mesh)
    D2 = lattice.cell_measures(s2, mesh)
    Cp = C * D1[None, :] / D2[:, None]
    p = np.array([1, 2, 1])
    row = Cp[s2.index(2, p)]
    ex = lambda c, q: s1.index(c, np.asarray(q))
    expect = np.zeros(s1.ndofs)
    expect[ex(1, p + [1, 0, 0])] += 1 / dx   # a_y on the right edge
    expect[ex(1, p)] -= 1 / dx               # a_y on the left edge
    expect[ex(0, p + [0, 1, 0])] -= 1 / dy   # a_x on the top edge
    expect[ex(0, p)] += 1 / dy               # a_x on the bottom edge
    assert np.abs(row - expect).max() < 1e-13
    # eq. (dTIsFiniteDiff): the transpose on a z-edge mixes x- and y-normal faces
    # adjoining it with +-1/dx and +-1/dy.
    CpT = Cp.T
    e = s1.index(2, np.array([1, 1, 0]))
    nz = CpT[e][CpT[e] != 0]
    assert sorted(np.round(np.abs(nz), 12)) == sorted(np.round([1 / dx, 1 / dx, 1 / dy, 1 / dy], 12))


def _smooth_scalar(x):
    return np.sin(1.3 * x[:, 0] + 0.4) * np.cos(0.7 * x[:, 1]) * np.exp(0.5 * x[:, 2])


def _smooth_vector(x):
    return np.stack([np.sin(x[:, 1] + 2 * x[:, 2]), np.cos(x[:, 0] * x[:, 2]), x[:, 0] ** 2 * np.sin(x[:, 1])], 1)


def _curl(f, x, h=1e-5):
    def d(i, j):  # d f_i / d x_j, central difference
        e = np.zeros(3); e[j] = h
        return (f(x + e)[:, i] - f(x - e)[:, i]) / (2 * h)
    return np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)], 1)


def test_commuting_identity_gradient_on_perturbed_mesh():
    # eq. (eqnCommute): d R^0 = R^1 d, here by the fundamental theorem of calculus.
    nel = (3, 2, 2)
    mesh = Mesh(synth.perturbed_vertices(nel, 0.15, seed=3))
    for r in (1, 2):
        s0, s1 = Space("H1", nel, r), Space("HCURL", nel, r)
        G = incidence.gradient(s0, s1)
        def grad(x):
            a = 1.3 * x[:, 0] + 0.4
            b, e = 0.7 * x[:, 1], np.exp(0.5 * x[:, 2])
            return np.stack([1.3 * np.cos(a) * np.cos(b) * e, -0.7 * np.sin(a) * np.sin(b) * e,
                             0.5 * np.sin(a) * np.cos(b) * e], 1)
        lhs = incidence.apply_ordered(G, assembly.de_rham(s0, mesh, _smooth_scalar))
        rhs = assembly.de_rham(s1, mesh, grad, qr=10)
        assert np.abs(lhs - rhs).max() < 1e-13


def test_commuting_identity_curl_and_div():
    # Stokes on faces and Gauss on cells, on a perturbed mesh.
    nel = (2, 2, 3)
    mesh = Mesh(synth.perturbed_vertices(nel, 0.15, seed=5))
    r = 2
    s1, s2, s3 = Space("HCURL", nel, r), Space("HDIV", nel, r), Space("L2", nel, r)
    C = incidence.curl(s1, s2)
    D = incidence.divergence(s2, s3)
    lhs = incidence.apply_ordered(C, assembly.de_rham(s1, mesh, _smooth_vector, qr=12))
    rhs = assembly.de_rham(s2, mesh, lambda x: _curl(_smooth_vector, x), qr=12)
    assert np.abs(lhs - rhs).max() < 1e-7
    B = lambda x: np.stack([x[:, 0] * np.sin(x[:, 1]), np.cos(x[:, 2] + x[:, 0]), x[:, 1] * x[:, 2] ** 2], 1)
    divB = lambda x: np.sin(x[:, 1]) + 2 * x[:, 1] * x[:, 2]
    lhs = incidence.apply_ordered(D, assembly.de_rham(s2, mesh, B, qr=12))
    rhs = assembly.de_rham(s3, mesh, divB, qr=12)
    assert np.abs(lhs - rhs).max() < 1e-11


def test_ordered_apply_on_integers_is_exact():
    s0, s1, s2, s3 = spaces3((3, 2, 2), 2, "natural")
    G = incidence.gradient(s0, s1)
    C = incidence.curl(s1, s2)
    rng = np.random.default_rng(0)
    u = rng.integers(-2 ** 40, 2 ** 40, s0.ndofs).astype(np.float64)
    g = incidence.apply_ordered(G, u)
    assert np.array_equal(g, (G.astype(np.int64) @ u.astype(np.int64)).astype(np.float64))
    assert np.all(incidence.apply_ordered(C, g) == 0.0)
