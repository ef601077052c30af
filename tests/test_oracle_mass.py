"""Pins of the oracle's mass matrices: the paper's Whitney entries, closed-form
integrals of polynomial fields, positivity, and the paper's torus spectra."""
import numpy as np
import pytest
import scipy.linalg as sl

import synth
from conftest import golden
from oracle import assembly, incidence, lattice
from oracle.lattice import Mesh, Space


def _paper_scaled(space, mesh):
    M = assembly.mass_matrix(space, mesh).toarray()
    D = lattice.cell_measures(space, mesh)
    return D[:, None] * M * D[None, :]


def test_whitney_masses_uniform_cube():
    # Section 4.3, eq. (whitMassMatrices), interior rows, in units of Delta_V.
    nel = (4, 4, 4)
    hi = (1.0, 2.0, 3.0)
    mesh = Mesh(synth.uniform_vertices(nel, hi=hi))
    dV = np.prod(np.asarray(hi) / np.asarray(nel))
    P1 = _paper_scaled(Space("HCURL", nel, 1), mesh) / dV
    P2 = _paper_scaled(Space("HDIV", nel, 1), mesh) / dV
    s1, s2 = Space("HCURL", nel, 1), Space("HDIV", nel, 1)
    for c in range(3):
        pos = np.array([1, 2, 2])
        row = P1[s1.index(c, pos)]
        vals = sorted(set(np.round(row[np.abs(row) > 1e-14], 13)))
        expect = sorted(golden(k)[0] for k in ("whitney_m1_cell", "whitney_m1_face", "whitney_m1_diag"))
        assert np.allclose(vals, expect, atol=1e-12)
        assert abs(row.sum() - golden("whitney_row_sum")[0]) < 1e-12
        # counts: 1 diagonal, 4 face neighbours, 4 cell-diagonal neighbours
        assert np.sum(np.isclose(row, 1 / 9)) == 4 and np.sum(np.isclose(row, 1 / 36)) == 4
        row = P2[s2.index(c, np.array([2, 1, 2]))]
        vals = sorted(set(np.round(row[np.abs(row) > 1e-14], 13)))
        expect = sorted(golden(k)[0] for k in ("whitney_m2_cell", "whitney_m2_diag"))
        assert np.allclose(vals, expect, atol=1e-12)
        assert abs(row.sum() - 1.0) < 1e-12


def test_rectangle_whitney_entries():
    # Section 7.2: per cell 1/3 on the diagonal and 1/6 for the parallel pair;
    # assembled interior row {1/6, 2/3, 1/6} Delta_V.
    nel = (1, 1)
    mesh = Mesh(synth.uniform_vertices(nel, hi=(0.5, 0.25)))
    s1 = Space("HCURL", nel, 1)
    P = _paper_scaled(s1, mesh) / (0.5 * 0.25)
    assert np.allclose(np.diag(P), golden("rect_m1_cell_diag")[0], atol=1e-12)
    assert abs(P[0, 1] - golden("rect_m1_cell_off")[0]) < 1e-12
    assert abs(P[0, 2]) < 1e-14   # x-edge vs y-edge: orthogonal
    nel = (4, 4)
    mesh = Mesh(synth.uniform_vertices(nel))
    s1 = Space("HCURL", nel, 1)
    P = _paper_scaled(s1, mesh) * 16
    row = P[s1.index(0, np.array([1, 2]))]
    assert sorted(np.round(row[np.abs(row) > 1e-14], 12)) == sorted(np.round([1 / 6, 2 / 3, 1 / 6], 12))


BOX = ((2, 3, 2), (1.0, 2.0, 3.0))


@pytest.mark.parametrize("kind,field,value", [
    ("H1", lambda x: x[:, 0] * x[:, 1] * x[:, 2], 8.0),
    ("HCURL", lambda x: np.stack([x[:, 1], x[:, 2], x[:, 0]], 1), 28.0),
    ("HDIV", lambda x: np.stack([x[:, 0], x[:, 1], x[:, 2]], 1), 28.0),
    ("L2", lambda x: np.ones(x.shape[0]), 6.0),
])
@pytest.mark.parametrize("r", [1, 2])
def test_polynomial_norms_closed_form(kind, field, value, r):
    # x^T M x = int |u|^2 for u in the space; exact integrals over [0,1]x[0,2]x[0,3].
    nel, hi = BOX
    mesh = Mesh(synth.uniform_vertices(nel, hi=hi))
    s = Space(kind, nel, r)
    x = assembly.de_rham(s, mesh, field)
    M = assembly.mass_matrix(s, mesh)
    assert abs(x @ (M @ x) - value) < 1e-11 * value


def test_polynomial_cross_term_degree2():
    nel, hi = BOX
    mesh = Mesh(synth.uniform_vertices(nel, hi=hi))
    s = Space("H1", nel, 2)
    u = assembly.de_rham(s, mesh, lambda x: x[:, 0] ** 2)
    v = assembly.de_rham(s, mesh, lambda x: x[:, 1])
    M = assembly.mass_matrix(s, mesh)
    assert abs(u @ (M @ v) - 2.0) < 1e-12        # int x^2 y = (1/3)(2)(3)


@pytest.mark.parametrize("kind", ["H1", "HCURL", "HDIV", "L2"])
def test_spd_on_perturbed_mesh(kind):
    nel = (2, 2, 2)
    mesh = Mesh(synth.perturbed_vertices(nel, 0.15, seed=11))
    M = assembly.mass_matrix(Space(kind, nel, 2), mesh).toarray()
    assert np.abs(M - M.T).max() < 1e-14 * np.abs(M).max()
    sl.cholesky(M)


def test_volume_of_perturbed_cube():
    # Boundary vertices slide in their faces, so the domain stays the unit cube.
    nel = (3, 3, 3)
    mesh = Mesh(synth.perturbed_vertices(nel, 0.15, seed=2))
    s = Space("H1", nel, 1)
    one = np.ones(s.ndofs)
    assert abs(one @ (assembly.mass_matrix(s, mesh) @ one) - 1.0) < 1e-13


def _torus_spectrum(nel, hi):
    mesh = Mesh(synth.uniform_vertices(nel, hi=hi))
    s1 = Space("HCURL", nel, 1, periodic=True)
    s2 = Space("L2", nel, 1, periodic=True)
    M1 = assembly.mass_matrix(s1, mesh).toarray()
    M2 = assembly.mass_matrix(s2, mesh).toarray()
    C = incidence.curl(s1, s2).toarray().astype(float)
    ev = sl.eigh(C.T @ M2 @ C, M1, eigvals_only=True)
    return ev[ev > 1e-8 * ev.max()]


def test_exact_feec_frequency_20x20():
    # Section 7.5: omega = 1.0041 for K = M1^{-1} C^T M2 C on the 20x20 torus.
    nz = _torus_spectrum((20, 20), (2 * np.pi, 2 * np.pi))
    val, tol = golden("omega_20x20")
    assert abs(np.sqrt(nz[0]) - val) < tol
    # closed form of the Whitney dispersion relation for the fundamental mode
    h = 2 * np.pi / 20
    assert abs(nz[0] - 6 / h ** 2 * (1 - np.cos(h)) / (2 + np.cos(h))) < 1e-10


@pytest.mark.slow
def test_torus_20x80_spectrum():
    # Section 7.3: 1599 non-kernel modes; modes 797-801 at 137.9-138.3.
    nz = _torus_spectrum((20, 80), (5.0, 20.0))
    assert len(nz) == int(golden("torus_nonkernel_modes")[0])
    lo, tlo = golden("torus_mode797_lo")
    hi, thi = golden("torus_mode801_hi")
    assert abs(nz[796] - lo) < tlo and abs(nz[800] - hi) < thi
