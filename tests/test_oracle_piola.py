"""Pins of the oracle's full-Jacobian pull-backs (paper section 2, definition of
M_p, with the covariant / contravariant Piola maps of 1- and 2-forms).

On an affine but sheared mesh (vertices A X with a non-normal A) a constant
physical field c lies in every space Q_r^- Lambda^k: its pull-back to the
reference cell is constant (J^T c for a 1-form, det J J^-1 c for a 2-form,
det J c for a 3-form).  The de Rham map integrates c over the mapped lattice
cells (tangents J e_a, normals J e_b x J e_c, volumes det J: an evaluation path
of its own), so x = R(c) represents c exactly and

    x^T M x = int |c|^2 dx = |c|^2 |det A| (volume of the sheared unit box),
    F . x   = int f . c dx  for the load vector F of the constant f = c.

Neither identity holds if a metric is transposed (J^-T J^-1 instead of
J^-1 J^-T, J J^T instead of J^T J) or a pull-back uses J instead of J^T: for a
non-normal J those differ.  The last test plants exactly those mistakes in a
copy of the oracle's metric and checks that the pins catch them.
"""
import numpy as np
import pytest

from oracle import assembly
from oracle.lattice import Mesh, Space

# non-symmetric, non-normal shear (A A^T != A^T A), det A > 0
A3 = np.array([[1.00, 0.35, -0.20],
               [0.10, 0.90, 0.25],
               [-0.15, 0.30, 1.10]])
A2 = np.array([[1.00, 0.40],
               [-0.15, 0.85]])
OFFSET = {3: np.array([0.3, -0.2, 0.1]), 2: np.array([0.3, -0.2])}
C3 = np.array([0.7, -1.3, 0.4])
C2 = np.array([0.7, -1.3])
SCALAR = 1.7


def sheared_mesh(nel):
    d = len(nel)
    A = A3 if d == 3 else A2
    axes = [np.arange(n + 1) / n for n in nel]
    X = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    V = np.einsum("ij,...j->...i", A, X) + OFFSET[d]
    return Mesh(np.ascontiguousarray(V)), abs(np.linalg.det(A))


def _field(kind, d):
    if kind in ("H1", "L2"):
        return (lambda x: np.full(x.shape[0], SCALAR)), SCALAR ** 2
    c = C3 if d == 3 else C2
    return (lambda x: np.broadcast_to(c, x.shape).copy()), float(c @ c)


CASES = [(kind, r, nel) for nel in ((2, 3, 2), (3, 2)) for kind in ("H1", "HCURL", "HDIV", "L2")
         for r in (1, 2, 3)]


@pytest.mark.parametrize("kind,r,nel", CASES)
def test_constant_field_energy(kind, r, nel):
    mesh, vol = sheared_mesh(nel)
    s = Space(kind, nel, r)
    f, c2 = _field(kind, len(nel))
    x = assembly.de_rham(s, mesh, f)
    M = assembly.mass_matrix(s, mesh)
    assert abs(x @ (M @ x) - c2 * vol) < 1e-12 * c2 * vol


@pytest.mark.parametrize("kind,r,nel", CASES)
def test_constant_field_load_vector(kind, r, nel):
    mesh, vol = sheared_mesh(nel)
    s = Space(kind, nel, r)
    f, c2 = _field(kind, len(nel))
    x = assembly.de_rham(s, mesh, f)
    F = assembly.load_vector(s, mesh, f)
    assert abs(F @ x - c2 * vol) < 1e-12 * c2 * vol


def _planted_metric(kind, J):
    # transposed metrics: the mistakes the pins above must catch
    det = np.linalg.det(J)
    inv = np.linalg.inv(J)
    if kind == "HCURL":
        return det[..., None, None] * np.einsum("...ia,...ib->...ab", inv, inv)
    if kind == "HDIV":
        return np.einsum("...ai,...bi->...ab", J, J) / det[..., None, None]
    return assembly.metric(kind, J)


def _planted_pullback(kind, J, f):
    det = np.linalg.det(J)
    inv = np.linalg.inv(J)
    if kind == "HCURL":
        return det[..., None] * np.einsum("...ia,...i->...a", inv, f)
    if kind == "HDIV":
        return np.einsum("...ai,...i->...a", J, f)
    return assembly._phys_pullback(kind, J, f)


@pytest.mark.parametrize("kind", ["HCURL", "HDIV"])
def test_pins_catch_transposed_metrics(kind, monkeypatch):
    nel = (2, 2, 2)
    mesh, vol = sheared_mesh(nel)
    s = Space(kind, nel, 1)
    f, c2 = _field(kind, 3)
    x = assembly.de_rham(s, mesh, f)
    monkeypatch.setattr(assembly, "metric", _planted_metric)
    M = assembly.mass_matrix(s, mesh)
    assert abs(x @ (M @ x) - c2 * vol) > 1e-3 * c2 * vol
    monkeypatch.setattr(assembly, "_phys_pullback", _planted_pullback)
    F = assembly.load_vector(s, mesh, f)
    assert abs(F @ x - c2 * vol) > 1e-3 * c2 * vol
