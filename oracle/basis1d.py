"""One-dimensional building blocks of the tensor-product spaces (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

On the reference interval [0, 1] with nodes 0 = xi_0 < ... < xi_r = 1:
  * nodal functions phi_i: Lagrange polynomials on the nodes (degree r);
  * edge functions e_j, j = 0..r-1: e_j = -sum_{k<=j} phi_k'.  They satisfy
    int_{xi_i}^{xi_{i+1}} e_j = delta_ij (integral duality, the 1-D case of
    the paper's eq. (WhitneyFormDefn) with integral normalisation) and
    phi_i' = e_{i-1} - e_i, i.e. the 1-D derivative is the +-1 incidence.
For r = 1 this is phi = (1 - x, x), e_0 = 1: the lowest-order Whitney pair
of the paper's section 4.1.

The nodes are Gauss-Lobatto-Legendre points (a reading: the paper fixes no
node placement above r = 1).  Quadrature is Gauss-Legendre.

Pins: tests/test_oracle_basis.py (duality, partition of unity, derivative
identity, r = 1 closed forms, quadrature exactness).
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gll_nodes(r):
    """GLL nodes on [0, 1] for degree r >= 1 (r + 1 points, endpoints included)."""
    if r < 1:
        raise ValueError("degree must be >= 1")
    if r == 1:
        x = np.array([-1.0, 1.0])
    else:
        c = np.zeros(r + 1)
        c[r] = 1.0
        inner = np.sort(_leg.legroots(_leg.legder(c)))
        x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def gauss(q):
    """Gauss-Legendre rule with q points on [0, 1]: (points, weights)."""
    x, w = _leg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def nodal_values(r, x):
    """phi_i(x) for the GLL nodes of degree r: array (len(x), r + 1)."""
    nodes = gll_nodes(r)
    x = np.asarray(x, dtype=np.float64)
    out = np.ones((x.size, r + 1))
    for i in range(r + 1):
        for k in range(r + 1):
            if k != i:
                out[:, i] *= (x - nodes[k]) / (nodes[i] - nodes[k])
    return out


def nodal_derivatives(r, x):
    """phi_i'(x): array (len(x), r + 1), by the product rule."""
    nodes = gll_nodes(r)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((x.size, r + 1))
    for i in range(r + 1):
        denom = 1.0
        for k in range(r + 1):
            if k != i:
                denom *= nodes[i] - nodes[k]
        for skip in range(r + 1):
            if skip == i:
                continue
            term = np.ones(x.size)
            for k in range(r + 1):
                if k != i and k != skip:
                    term *= x - nodes[k]
            out[:, i] += term
        out[:, i] /= denom
    return out


def edge_values(r, x):
    """e_j(x) = -sum_{k<=j} phi_k'(x): array (len(x), r)."""
    d = nodal_derivatives(r, x)
    return -np.cumsum(d, axis=1)[:, :r]


def table(kind, r, x):
    """Basis table for one axis: 'n' (nodal, r+1 functions) or 'e' (edge, r)."""
    if kind == "n":
        return nodal_values(r, x)
    if kind == "e":
        return edge_values(r, x)
    raise ValueError(kind)
