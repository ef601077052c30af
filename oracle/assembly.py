"""Mass matrices, load vectors, de Rham map and L2 errors by naive quadrature (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Mass matrices follow the paper's section 2 definition
(M_p)_ij = int (Lambda_i, Lambda_j)_p dx, computed element by element with a
tensor Gauss rule of q = r + 1 points per axis (a reading: the paper fixes no
rule; this one is exact on affine cells) and the pull-backs of each kind:
  H1    w detJ phi_i phi_j
  HCURL w detJ w_i^T J^{-1} J^{-T} w_j     (covariant)
  HDIV  w w_i^T J^T J w_j / detJ          (contravariant)
  L2    w w_i w_j / detJ
with J = dx/dxi of the cell's multilinear map.  Local matrices are added into
a global COO matrix (duplicates summed by SciPy), rows/columns of dropped
boundary positions removed.

Load vectors F_i = int f . Lambda_i use q_f = r + 2 points per axis (reading).
The de Rham map R^k integrates a smooth field over each lattice k-cell (the
degrees of freedom of the paper's eq. WhitneyFormDefn, integral-normalised).

Pins: tests/test_oracle_mass.py (Whitney closed forms of eq.
whitMassMatrices, 2-D rectangle entries, row sums, polynomial exactness,
SPD), tests/test_oracle_derham.py (reproduction, commuting identity).
"""
import numpy as np
import scipy.sparse as sp

from . import basis1d
from .lattice import tensor_grid, tensor_weights


def _det_inv(J):
    d = J.shape[-1]
    det = np.linalg.det(J)
    inv = np.linalg.inv(J)
    return det, inv


def metric(kind, J):
    """Pointwise inner-product matrix G with (u, v)_p dx = uhat^T G vhat dxi."""
    det, inv = _det_inv(J)
    d = J.shape[-1]
    eye = np.broadcast_to(np.eye(d), J.shape)
    if kind == "H1":
        return det[..., None, None] * eye
    if kind == "HCURL":
        return det[..., None, None] * np.einsum("...ai,...bi->...ab", inv, inv)
    if kind == "HDIV":
        return np.einsum("...ia,...ib->...ab", J, J) / det[..., None, None]
    if kind == "L2":
        return eye / det[..., None, None]
    raise ValueError(kind)


def local_mass(space, mesh, elems=None, q=None):
    """Local mass matrices (E, L, L) for the given element rows (default: all)."""
    q = space.r + 1 if q is None else q
    d = space.dim
    xi1, w1 = basis1d.gauss(q)
    xi = tensor_grid(xi1, d)
    w = tensor_weights(w1, d)
    B = space.local_basis(xi1)                         # (Q, L, d)
    _, J = mesh.geometry(xi)                           # (E, Q, d, d)
    if elems is not None:
        J = J[elems]
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("non-positive Jacobian determinant at a quadrature point")
    G = metric(space.kind, J) * w[None, :, None, None]
    out = np.empty((J.shape[0], B.shape[1], B.shape[1]))
    chunk = 1024
    for s in range(0, J.shape[0], chunk):
        T = np.einsum("eqab,qjb->eqaj", G[s:s + chunk], B)
        out[s:s + chunk] = np.einsum("qia,eqaj->eij", B, T)
    return out


def mass_matrix(space, mesh, q=None):
    """Global sparse SPD mass matrix of ``space`` on ``mesh`` (CSR, FP64)."""
    Ml = local_mass(space, mesh, q=q)
    dofs = space.element_dofs(mesh.element_multi_index())
    E, L = dofs.shape
    rows = np.repeat(dofs, L, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, L)).reshape(-1)
    vals = Ml.reshape(-1)
    keep = (rows >= 0) & (cols >= 0)
    M = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])),
                      shape=(space.ndofs, space.ndofs)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return M


def _phys_pullback(kind, J, f):
    """Weight vector g with f . Lambda_i detJ = g . what_i (reference proxy)."""
    det, inv = _det_inv(J)
    if kind == "H1":
        return det[..., None] * f
    if kind == "HCURL":
        return det[..., None] * np.einsum("...ai,...i->...a", inv, f)
    if kind == "HDIV":
        return np.einsum("...ia,...i->...a", J, f)
    if kind == "L2":
        return f
    raise ValueError(kind)


def load_vector(space, mesh, f, q=None):
    """F_i = int f . Lambda_i dx; f(x) maps (P, d) points to (P, d) (or (P,) scalar)."""
    q = space.r + 2 if q is None else q
    d = space.dim
    xi1, w1 = basis1d.gauss(q)
    xi = tensor_grid(xi1, d)
    w = tensor_weights(w1, d)
    B = space.local_basis(xi1)
    x, J = mesh.geometry(xi)
    E, Q = x.shape[:2]
    fv = np.asarray(f(x.reshape(-1, d)), dtype=np.float64)
    if fv.ndim == 1:
        fv = np.stack([fv] + [np.zeros_like(fv)] * (d - 1), axis=-1)
    fv = fv.reshape(E, Q, d)
    g = _phys_pullback(space.kind, J, fv) * w[None, :, None]
    Fl = np.einsum("eqa,qla->el", g, B)
    dofs = space.element_dofs(mesh.element_multi_index())
    keep = dofs >= 0
    F = np.zeros(space.ndofs)
    np.add.at(F, dofs[keep], Fl[keep])
    return F


def map_points(mesh, elem, xi):
    """Multilinear map and Jacobian at per-point (element, reference point) pairs."""
    d = mesh.dim
    elem = np.asarray(elem, dtype=np.int64)
    xi = np.asarray(xi, float)
    P = xi.shape[0]
    x = np.zeros((P, d))
    J = np.zeros((P, d, d))
    import itertools
    for bits in itertools.product((0, 1), repeat=d):
        bits = bits[::-1]
        sel = tuple(elem[:, a] + bits[a] for a in range(d))
        X = mesh.vertices[sel]                           # (P, d)
        val = np.ones(P)
        for a in range(d):
            val = val * (xi[:, a] if bits[a] else 1.0 - xi[:, a])
        x += val[:, None] * X
        for a in range(d):
            g = np.ones(P)
            for b in range(d):
                if b == a:
                    g = g * (1.0 if bits[b] else -1.0)
                else:
                    g = g * (xi[:, b] if bits[b] else 1.0 - xi[:, b])
            J[:, :, a] += g[:, None] * X
    return x, J


def de_rham(space, mesh, f, qr=8):
    """R^k f: integral of the smooth field f over every lattice k-cell.

    f maps (P, d) points to (P, d) vectors (or (P,) for scalar kinds).  The
    cell is a sub-box of one element in reference coordinates; its integral
    uses a tensor Gauss rule of qr points per integrated axis.
    """
    d = space.dim
    r = space.r
    nodes = basis1d.gll_nodes(r)
    g1, gw = basis1d.gauss(qr)
    out = np.zeros(space.ndofs)
    for c, comp in enumerate(space.comps):
        pos = space.positions(c)                          # (P, d)
        P = pos.shape[0]
        eaxes = [a for a in range(d) if comp[a] == "e"]
        k = len(eaxes)
        if k:
            sub = tensor_grid(g1, k)
            subw = tensor_weights(gw, k)
        else:
            sub = np.zeros((1, 0))
            subw = np.ones(1)
        S = sub.shape[0]
        elem = np.empty((P, d), dtype=np.int64)
        loc = np.empty((P, d), dtype=np.int64)
        for a in range(d):
            p = np.mod(pos[:, a], space.m[a]) if space.periodic else pos[:, a]
            e = np.minimum(p // r, space.nel[a] - 1)
            elem[:, a] = e
            loc[:, a] = p - r * e
        xi = np.zeros((P, S, d))
        jac_len = np.ones((P, S))
        for a in range(d):
            if comp[a] == "n":
                xi[:, :, a] = nodes[loc[:, a]][:, None]
            else:
                j = eaxes.index(a)
                lo = nodes[loc[:, a]]
                hi = nodes[loc[:, a] + 1]
                xi[:, :, a] = lo[:, None] + (hi - lo)[:, None] * sub[None, :, j]
                jac_len *= (hi - lo)[:, None]
        x, J = map_points(mesh, np.repeat(elem, S, axis=0), xi.reshape(-1, d))
        x = x.reshape(P, S, d)
        J = J.reshape(P, S, d, d)
        fv = np.asarray(f(x.reshape(-1, d)), dtype=np.float64)
        if space.kind in ("H1", "L2"):
            fv = fv.reshape(P, S)
            if space.kind == "H1":
                integrand = fv
            else:
                integrand = fv * np.linalg.det(J)
        else:
            fv = fv.reshape(P, S, d)
            if space.kind == "HCURL":
                integrand = np.einsum("psi,psi->ps", fv, J[:, :, :, c])
            else:  # HDIV: flux through the cell normal to axis c
                if d == 3:
                    c1, c2 = (c + 1) % 3, (c + 2) % 3
                    n = np.cross(J[:, :, :, c1], J[:, :, :, c2])
                else:
                    t = J[:, :, :, 1 - c]
                    n = np.stack([t[..., 1], -t[..., 0]], -1) if c == 0 else \
                        np.stack([-t[..., 1], t[..., 0]], -1)
                integrand = np.einsum("psi,psi->ps", fv, n)
        out[space.offsets[c]:space.offsets[c + 1]] = (integrand * subw[None, :] * jac_len).sum(1)
    return out


def evaluate(space, mesh, coeffs, xi1):
    """Physical field of ``coeffs`` at the tensor grid of xi1 in every element.

    Returns x (E, Q, d) and values (E, Q, d) (scalar kinds in slot 0)."""
    d = space.dim
    xi = tensor_grid(xi1, d)
    B = space.local_basis(xi1)
    x, J = mesh.geometry(xi)
    dofs = space.element_dofs(mesh.element_multi_index())
    cl = np.where(dofs >= 0, np.asarray(coeffs)[np.maximum(dofs, 0)], 0.0)
    ref = np.einsum("el,qla->eqa", cl, B)
    det, inv = _det_inv(J)
    if space.kind == "H1":
        val = ref
    elif space.kind == "HCURL":
        val = np.einsum("eqai,eqa->eqi", inv, ref)
    elif space.kind == "HDIV":
        val = np.einsum("eqia,eqa->eqi", J, ref) / det[..., None]
    else:
        val = ref / det[..., None]
    return x, val


def l2_error(space, mesh, coeffs, exact, q=None):
    """(||u_h - u||_L2, ||u||_L2) with a Gauss rule of r + 3 points per axis."""
    q = space.r + 3 if q is None else q
    d = space.dim
    xi1, w1 = basis1d.gauss(q)
    w = tensor_weights(w1, d)
    x, val = evaluate(space, mesh, coeffs, xi1)
    _, J = mesh.geometry(tensor_grid(xi1, d))
    det = np.linalg.det(J)
    E, Q = x.shape[:2]
    ev = np.asarray(exact(x.reshape(-1, d)), dtype=np.float64)
    if space.kind in ("H1", "L2"):
        ev = ev.reshape(E, Q)
        diff = (val[..., 0] - ev) ** 2
        nrm = ev ** 2
    else:
        ev = ev.reshape(E, Q, d)
        diff = ((val - ev) ** 2).sum(-1)
        nrm = (ev ** 2).sum(-1)
    wd = w[None, :] * det
    return float(np.sqrt((diff * wd).sum())), float(np.sqrt((nrm * wd).sum()))
