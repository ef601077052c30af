"""Integer incidence matrices G, C, D of the discrete de Rham complex (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper section 2, eq. (discreteDeRham): the exterior derivative is represented
by the gradient G (N1 x N0), curl C (N2 x N1) and divergence D (N3 x N2) with
CG = 0 and DC = 0.  With integral degrees of freedom (Stokes' theorem on each
lattice cell) the entries are exactly +-1:
  (G u)_c(p)      = u(p + e_c) - u(p)
  (C a)_c(p)      = a_{c2}(p + e_{c1}) - a_{c2}(p) - a_{c1}(p + e_{c2}) + a_{c1}(p)
                    with (c1, c2) the cyclic successors of c     (3-D)
  (C a)(p)        = a_y(p + e_x) - a_y(p) - a_x(p + e_y) + a_x(p) (2-D, into L2)
  (D b)(p)        = sum_c b_c(p + e_c) - b_c(p)
Values outside the kept positions (essential boundary) are zero, so the
matrices are the corresponding sub-matrices.  In the paper's average-value
normalisation the same curl is the finite difference of eqs. (dIsFiniteDiff)
and (dTIsFiniteDiff) with entries +-1/Delta (a diagonal rescaling).

The apply contract used for bit-exact comparison: y_i is accumulated in FP64
from +0.0 over the row's entries in ascending column order.

Pins: tests/test_oracle_incidence.py (CG = 0, DC = 0, exactness by integer
rank, Euler characteristic, the paper's finite-difference stencils, Stokes /
commuting identity against quadrature).
"""
import numpy as np
import scipy.sparse as sp


def _build(out_space, in_space, terms_fn):
    rows, cols, vals = [], [], []
    for c in range(len(out_space.comps)):
        pos = out_space.positions(c)
        ridx = out_space.index(c, pos)
        for in_c, shift, sign in terms_fn(c):
            q = pos + np.asarray(shift)[None, :]
            cidx = in_space.index(in_c, q)
            keep = cidx >= 0
            rows.append(ridx[keep])
            cols.append(cidx[keep])
            vals.append(np.full(int(keep.sum()), sign, dtype=np.int8))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals).astype(np.int64)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(out_space.ndofs, in_space.ndofs)).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A.astype(np.int8)


def _unit(dim, a):
    e = np.zeros(dim, dtype=np.int64)
    e[a] = 1
    return e


def gradient(h1, hcurl):
    """G: H1 -> HCURL."""
    d = h1.dim
    z = np.zeros(d, dtype=np.int64)
    return _build(hcurl, h1, lambda c: [(0, _unit(d, c), 1), (0, z, -1)])


def curl(hcurl, target):
    """C: HCURL -> HDIV (3-D) or HCURL -> L2 (2-D)."""
    d = hcurl.dim
    z = np.zeros(d, dtype=np.int64)
    if d == 3:
        def terms(c):
            c1, c2 = (c + 1) % 3, (c + 2) % 3
            return [(c2, _unit(3, c1), 1), (c2, z, -1), (c1, _unit(3, c2), -1), (c1, z, 1)]
    elif d == 2:
        def terms(c):
            return [(1, _unit(2, 0), 1), (1, z, -1), (0, _unit(2, 1), -1), (0, z, 1)]
    else:
        raise ValueError("curl needs d = 2 or 3")
    return _build(target, hcurl, terms)


def divergence(hdiv, l2):
    """D: HDIV -> L2."""
    d = hdiv.dim
    z = np.zeros(d, dtype=np.int64)
    def terms(c):
        out = []
        for a in range(d):
            out += [(a, _unit(d, a), 1), (a, z, -1)]
        return out
    return _build(l2, hdiv, terms)


def transpose(A):
    """Integer transpose with sorted column indices."""
    T = A.T.tocsr()
    T.sort_indices()
    return T


def apply_ordered(A, x):
    """y = A x with each row summed from +0.0 in ascending column order (FP64)."""
    A = A.tocsr()
    A.sort_indices()
    x = np.asarray(x, dtype=np.float64)
    nnz_row = np.diff(A.indptr)
    y = np.zeros(A.shape[0], dtype=np.float64)
    kmax = int(nnz_row.max()) if nnz_row.size else 0
    for k in range(kmax):
        has = nnz_row > k
        j = A.indptr[:-1][has] + k
        y[has] = y[has] + A.data[j].astype(np.float64) * x[A.indices[j]]
    return y
