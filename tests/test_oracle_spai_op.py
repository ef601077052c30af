"""Pins of the oracle's SPAI-OP (oracle/spai_op.py) against the paper's statements.

On the paper's 20 x 20 periodic Whitney mesh (sections 5 and 7.5):
  * lambda = 0: PCG reaches machine precision in 2 iterations, and the
    solution is the column-wise SPAI (already symmetric on this grid);
  * one probe P2 v (v the lowest mode of M1^-1 P2), lambda = 5e5, started
    from the column-wise SPAI: O(10^2) PCG iterations, the probed-mode
    residual ||Q1 P2 v - omega^2 v|| / omega^2 below 1e-4, the Frobenius fit
    within 8% of SPAI's, and the probed frequency 1.00412.
On a 3-D box with a perfect conductor (where the column-wise SPAI is not
symmetric): the lambda = 0 solution is symmetric and fits M1^-1 at least as
well as the symmetrised column-wise SPAI (it is the optimal symmetric one).
"""
import numpy as np
import pytest
import scipy.linalg as sl

import synth
from conftest import golden
from oracle import assembly, incidence, spai, spai_op
from oracle.lattice import Mesh, Space


@pytest.fixture(scope="module")
def torus():
    nel, hi = (20, 20), (2 * np.pi, 2 * np.pi)
    mesh = Mesh(synth.uniform_vertices(nel, hi=hi))
    s1 = Space("HCURL", nel, 1, periodic=True)
    s2 = Space("L2", nel, 1, periodic=True)
    M1 = assembly.mass_matrix(s1, mesh).tocsr()
    M2 = assembly.mass_matrix(s2, mesh)
    C = incidence.curl(s1, s2).astype(float)
    P2 = (C.T @ M2 @ C).tocsr()
    w, V = sl.eigh(P2.toarray(), M1.toarray())
    k = np.nonzero(w > 1e-9 * w.max())[0][0]
    return M1, P2, V[:, k], w[k]


def _fro(M1, Q):
    return np.linalg.norm(M1 @ Q.toarray() - np.eye(M1.shape[0]))


def test_lambda0_two_iterations_and_column_spai(torus):
    M1, _, _, _ = torus
    Q, its, rel = spai_op.SpaiOp(M1).solve(rtol=1e-14)
    assert its <= golden("spai_op_lam0_pcg_iters")[0] and rel <= 1e-14
    Qc = spai.spai(M1, "m")
    assert abs(Q - Qc).max() <= 1e-11 * abs(Qc).max()


def test_single_probe_dispersion(torus):
    M1, P2, v, om2 = torus
    S = spai_op.SpaiOp(M1, W=(P2 @ v)[:, None], lam=5e5)
    Qc = spai.spai(M1, "m")
    Q, its, rel = S.solve(q0=np.asarray(Qc[S.ir, S.ic]).ravel(), rtol=1e-6)
    assert 10 <= its <= 1000  # O(10^2)
    assert abs(Q - Q.T).max() <= 1e-6 * abs(Q).max()  # symmetric to the solver tolerance
    resid = np.linalg.norm(Q @ (P2 @ v) - om2 * v) / (om2 * np.linalg.norm(v))
    assert resid < golden("spai_op_probe_resid")[0]
    assert _fro(M1, Q) / _fro(M1, Qc) <= golden("spai_op_fro_ratio")[0]
    ev = np.linalg.eigvals(Q.toarray() @ P2.toarray()).real
    ev = ev[ev > 1e-9 * ev.max()]
    omega_hat = np.sqrt(ev[np.argmin(np.abs(ev - om2))])
    val, tol = golden("spai_op_omega_20x20")
    assert abs(omega_hat - val) < tol


def test_lambda0_is_the_optimal_symmetric_fit():
    nel = (4, 3, 4)
    mesh = Mesh(synth.uniform_vertices(nel, hi=(1.0, 1.2, 0.9)))
    M1 = assembly.mass_matrix(Space("HCURL", nel, 1, "essential"), mesh).tocsr()
    Q, its, rel = spai_op.SpaiOp(M1).solve(rtol=1e-14)
    assert rel <= 1e-13
    assert abs(Q - Q.T).max() <= 1e-13 * abs(Q).max()
    Qc = spai.spai(M1, "m")
    # near the conductor the column-wise solution is not symmetric, and the
    # symmetric optimum fits strictly better than its symmetrisation
    Qu = spai.spai_unsymmetrised(M1, "m")
    assert abs(Qu - Qu.T).max() > 1e-3 * abs(Qu).max()
    assert _fro(M1, Q) < _fro(M1, Qc)
