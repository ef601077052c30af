"""Sparse approximate inverses of a mass matrix (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper section 5 (eqs. FrobeniusDecomp, NormalEqSolve).  Q approximates M^-1
column by column: for column l, with the allowed rows I_l given by a sparsity
pattern S, q_l(I_l) minimises || M[:, I_l] q - e_l ||_2, i.e. the Frobenius
norm || M Q - 1 ||_F splits into one small least-squares problem per column.
Each is solved here as a dense least-squares problem on the rows where
M[:, I_l] is nonzero.  The result is then made symmetric, Q <- (Q + Q^T) / 2,
as section 5 does, so that it can serve as the Q1 of a symplectic scheme.

Patterns: 'diag' is S(1), one entry per column; 'm' is S(M), the sparsity of
M itself (its structural nonzeros: see :func:`structural`).

Pins (tests/test_oracle_spai.py): on the paper's 20 x 20 periodic Whitney mesh
the lowest non-kernel frequency of Q P2 against the printed 1.1499 (S(1)) and
0.9634 (S(M1)); the S(1) entries against their closed form M_ll / ||M e_l||^2;
each column's least-squares optimality (its normal equations); symmetry.
"""
import numpy as np
import scipy.sparse as sp


def structural(M, rel=1e-14):
    """M without the entries below rel times its largest: quadrature in
    floating point leaves roundoff (1e-17 and less) where the exact mass matrix
    has zeros, e.g. between the components of a 1-form on box cells; the
    pattern S(M) is that of the exact matrix."""
    M = sp.csr_matrix(M, copy=True)
    M.data[np.abs(M.data) <= rel * np.abs(M.data).max()] = 0.0
    M.eliminate_zeros()
    return M


def spai(M, pattern="m"):
    """Symmetrised column-wise SPAI of the sparse matrix M with pattern
    'diag' (S(1)) or 'm' (S(M))."""
    if pattern not in ("diag", "m"):
        raise ValueError("pattern: 'diag' or 'm'")
    M = sp.csc_matrix(structural(M))
    M.sort_indices()
    n = M.shape[0]
    rows, cols, vals = [], [], []
    for l in range(n):
        I = np.array([l]) if pattern == "diag" else M.indices[M.indptr[l]:M.indptr[l + 1]]
        sub = M[:, I].tocsr()
        R = np.unique(sub.nonzero()[0])  # rows where M[:, I] is nonzero
        A = sub[R].toarray()
        e = (R == l).astype(np.float64)
        q = np.linalg.lstsq(A, e, rcond=None)[0]
        rows += list(I)
        cols += [l] * len(I)
        vals += list(q)
    Q = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return (0.5 * (Q + Q.T)).tocsr()


def spai_unsymmetrised(M, pattern="m"):
    """The column-wise least-squares solution before symmetrisation (for the
    optimality pins)."""
    M = sp.csc_matrix(structural(M))
    M.sort_indices()
    n = M.shape[0]
    rows, cols, vals = [], [], []
    for l in range(n):
        I = np.array([l]) if pattern == "diag" else M.indices[M.indptr[l]:M.indptr[l + 1]]
        A = M[:, I].toarray()
        e = np.zeros(n)
        e[l] = 1.0
        q = np.linalg.lstsq(A, e, rcond=None)[0]
        rows += list(I)
        cols += [l] * len(I)
        vals += list(q)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
