"""Pins of the oracle's sparse approximate inverses (oracle/spai.py).

The paper prints, for its 20 x 20 periodic Whitney mesh (section 7.5), the
lowest frequency of Q1 C^T M2 C with Q1 the symmetrised SPAI of M1: 1.1499
for the diagonal pattern S(1) and 0.9634 for the pattern S(M1).  Besides
these printed values: the S(1) entries against their closed form
M_ll / ||M e_l||^2, each column's least-squares optimality (normal equations
on its pattern), and the symmetry of the result.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import synth
from conftest import golden
from oracle import assembly, incidence, spai
from oracle.lattice import Mesh, Space


def _torus(nel=(20, 20), hi=(2 * np.pi, 2 * np.pi)):
    mesh = Mesh(synth.uniform_vertices(nel, hi=hi))
    s1 = Space("HCURL", nel, 1, periodic=True)
    s2 = Space("L2", nel, 1, periodic=True)
    M1 = assembly.mass_matrix(s1, mesh)
    M2 = assembly.mass_matrix(s2, mesh)
    C = incidence.curl(s1, s2).astype(float)
    return M1, (C.T @ M2 @ C).toarray()


def _lowest_omega(Q, P2):
    w = np.sort(np.linalg.eigvals(Q.toarray() @ P2).real)
    return np.sqrt(w[w > 1e-8 * w.max()][0])


@pytest.mark.parametrize("pattern,key", [("diag", "spai_diag_omega_20x20"), ("m", "spai_m1_omega_20x20")])
def test_spai_dispersion_20x20(pattern, key):
    M1, P2 = _torus()
    val, tol = golden(key)
    assert abs(_lowest_omega(spai.spai(M1, pattern), P2) - val) < tol


def test_spai_diag_closed_form():
    # S(1): q_l minimises || q M e_l - e_l ||, so q_l = M_ll / ||M e_l||^2
    mesh = Mesh(synth.uniform_vertices((3, 2, 4), hi=(1.0, 0.7, 1.2)))
    M = assembly.mass_matrix(Space("HCURL", (3, 2, 4), 2, "essential"), mesh).toarray()
    Q = spai.spai(M, "diag").toarray()
    assert np.allclose(np.diag(Q), np.diag(M) / (M ** 2).sum(axis=0), rtol=1e-13)
    assert np.abs(Q - np.diag(np.diag(Q))).max() == 0.0


def test_spai_columns_are_least_squares_optimal():
    # S(M): M[:, I]^T (M[:, I] q_l - e_l) = 0 on each column's pattern I
    mesh = Mesh(synth.perturbed_vertices((2, 3, 2), 0.1, seed=4))
    M = spai.structural(assembly.mass_matrix(Space("HCURL", (2, 3, 2), 1, "essential"), mesh)).tocsc()
    Q = spai.spai_unsymmetrised(M, "m").tocsc()
    Md = M.toarray()
    for l in range(M.shape[0]):
        I = M.indices[M.indptr[l]:M.indptr[l + 1]]
        q = Q[:, l].toarray().ravel()
        assert set(np.nonzero(q)[0]) <= set(I)
        e = np.zeros(M.shape[0])
        e[l] = 1.0
        g = Md[:, I].T @ (Md @ q - e)
        assert np.abs(g).max() < 1e-12 * np.abs(Md).max() ** 2
    S = spai.spai(M, "m").toarray()
    assert np.array_equal(S, S.T)
    assert np.allclose(S, 0.5 * (Q + Q.T).toarray(), rtol=1e-12, atol=1e-12 * np.abs(S).max())
