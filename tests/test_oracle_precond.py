"""The mixed Poisson block preconditioner diag(diag(M2), S),
S = M3 D diag(M2)^-1 D^T M3 (oracle.problems.schur_preconditioner), pinned to
what the algebra of saddle-point systems fixes:

* Murphy, Golub & Wathen (2000): for [[F, B^T], [B, 0]] preconditioned by
  diag(F, B F^-1 B^T) the preconditioned matrix has exactly the eigenvalues
  1 and (1 +- sqrt 5) / 2.  With F = diag(M2) and B = -M3 D this holds to
  round-off; a wrong S (a dropped M3, a transposed D, the full M2 in place of
  its diagonal) breaks it.
* For the true system (F = M2) the eigenvalues of P^-1 A then lie in intervals
  fixed by the spectrum of diag(M2)^-1 M2, which is mesh-independent, so the
  extreme eigenvalues and the MINRES iteration count do not grow under
  refinement (unlike block Jacobi, whose count grows like 1/h).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

import synth
from oracle import problems
from oracle.lattice import Mesh


def _problem(nel, r):
    return problems.MixedPoisson(Mesh(synth.uniform_vertices(nel)), r)


def test_three_eigenvalues_with_diagonal_flux_block():
    P = _problem((2, 3, 2), 2)
    apply, S, d = problems.schur_preconditioner(P)
    ns = d.size
    B = -(P.M3 @ P.D)
    Ahat = sp.bmat([[sp.diags(d), B.T], [B, None]]).toarray()
    Pm = sla.block_diag(np.diag(d), S.toarray())
    lam = sla.eigh(Ahat, Pm, eigvals_only=True)
    phi = (1 + np.sqrt(5)) / 2
    targets = np.array([1.0, phi, 1 - phi])
    dist = np.min(np.abs(lam[:, None] - targets[None, :]), axis=1)
    assert dist.max() < 1e-9, dist.max()
    # all three occur: 1 with multiplicity ns - np, the golden pair np times each
    np_ = S.shape[0]
    assert np.sum(np.abs(lam - 1) < 1e-9) == ns - np_
    assert np.sum(np.abs(lam - phi) < 1e-9) == np_ and np.sum(np.abs(lam - 1 + phi) < 1e-9) == np_


def test_apply_is_the_inverse_of_the_block_preconditioner():
    P = _problem((3, 2, 2), 3)
    apply, S, d = problems.schur_preconditioner(P)
    y = synth.random_vector(P.A.shape[0], seed=4)
    z = apply(y)
    ns = d.size
    assert np.allclose(d * z[:ns], y[:ns], rtol=1e-13, atol=0)
    assert np.allclose(S @ z[ns:], y[ns:], rtol=1e-10, atol=1e-12 * np.abs(y).max())


def test_mesh_independent_spectrum_and_iterations():
    # degree 2, N = 2, 3, 4: every eigenvalue of P^-1 A stays in fixed
    # intervals (measured: [-0.82, -0.56] and [0.49, 1.96], approaching their
    # limits from inside), and the MINRES count settles near 45, while block
    # Jacobi's count grows with N
    r = 2
    its, jac = [], []
    for N in (2, 3, 4):
        P = _problem((N, N, N), r)
        apply, S, d = problems.schur_preconditioner(P)
        Pm = sla.block_diag(np.diag(d), S.toarray())
        lam = sla.eigh(P.A.toarray(), Pm, eigvals_only=True)
        neg, pos = lam[lam < 0], lam[lam > 0]
        assert neg.min() > -1.0 and neg.max() < -0.5, (N, neg.min(), neg.max())
        assert pos.min() > 0.45 and pos.max() < 2.1, (N, pos.min(), pos.max())
        b = synth.random_vector(P.A.shape[0], seed=5)
        x, info, it = problems.solve_minres_prec(P.A, b, apply, rtol=1e-10)
        assert info == 0
        # SciPy stops on the preconditioned residual estimate; the true one follows within its conditioning
        assert np.linalg.norm(P.A @ x - b) < 1e-7 * np.linalg.norm(b)
        its.append(it)
        n = [0]
        import scipy.sparse.linalg as spla
        spla.minres(P.A, b, M=sp.diags(1.0 / P.precond_diag()), rtol=1e-10,
                    callback=lambda _: n.__setitem__(0, n[0] + 1))
        jac.append(n[0])
    assert max(its) < 50 and its[2] - its[1] <= 3, its
    assert jac[2] > 1.5 * jac[0], jac
