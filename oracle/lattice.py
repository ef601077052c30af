"""Structured mesh geometry and the tensor-product spaces Q_r^- Lambda^k (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Mesh: N_1 x ... x N_d cells with vertex coordinates given by the caller
(uniform box, or the seeded perturbation from ``synth``).  Each cell is the
image of [0,1]^d under the multilinear map of its 2^d corners, so a perturbed
hexahedron is non-affine.

Spaces (paper section 2: p-forms spanned by a locally supported basis; the
paper's cubical example is Q_1^- Lambda^p of section 4.1):
  kind H1    (k = 0)   one component, nodal in every axis
  kind HCURL (k = 1)   component c is edge along axis c, nodal elsewhere
  kind HDIV  (k = d-1) component c is nodal along axis c, edge elsewhere
                       (a 2-form proxy in 3-D, the rotated 1-form in 2-D)
  kind L2    (k = d)   one component, edge in every axis
Per axis the lattice has m = r*N cells; 1-D nodal positions are 0..m, edge
positions 0..m-1.  A degree of freedom is the integral of the form over one
k-cell of this lattice.  Global numbering ("canonical"): component blocks in
axis order, inside a block lexicographic with axis 0 fastest, over the kept
positions.  Essential boundary conditions drop nodal positions 0 and m
(zero trace); periodic axes identify position m with 0.
"""
import itertools

import numpy as np

KINDS = ("H1", "HCURL", "HDIV", "L2")


def components(kind, dim):
    """Per component, the per-axis 1-D type: 'n' nodal or 'e' edge."""
    if kind == "H1":
        return [tuple("n" * dim)]
    if kind == "L2":
        return [tuple("e" * dim)]
    comps = []
    for c in range(dim):
        if kind == "HCURL":
            comps.append(tuple("e" if a == c else "n" for a in range(dim)))
        elif kind == "HDIV":
            comps.append(tuple("n" if a == c else "e" for a in range(dim)))
        else:
            raise ValueError(kind)
    return comps


class Mesh:
    """Structured mesh: ``vertices`` has shape (N_1+1, ..., N_d+1, d)."""

    def __init__(self, vertices):
        v = np.asarray(vertices, dtype=np.float64)
        self.dim = v.shape[-1]
        if v.ndim != self.dim + 1:
            raise ValueError("vertex array must be (N+1)^d x d")
        self.vertices = v
        self.nel = tuple(s - 1 for s in v.shape[:-1])
        self.nelem = int(np.prod(self.nel))

    @staticmethod
    def uniform(nel, lo=None, hi=None):
        dim = len(nel)
        lo = np.zeros(dim) if lo is None else np.asarray(lo, float)
        hi = np.ones(dim) if hi is None else np.asarray(hi, float)
        axes = [lo[a] + (hi[a] - lo[a]) * np.arange(nel[a] + 1) / nel[a] for a in range(dim)]
        grid = np.meshgrid(*axes, indexing="ij")
        return Mesh(np.stack(grid, axis=-1))

    def element_multi_index(self):
        """(E, d) element indices, axis 0 fastest (canonical element order)."""
        ranges = [np.arange(n) for n in self.nel]
        g = np.meshgrid(*ranges, indexing="ij")
        return np.stack([x.reshape(-1, order="F") for x in g], axis=-1)

    def corners(self):
        """(E, 2^d, d) corner coordinates; corner c has bits (c_0, ..., c_{d-1})."""
        idx = self.element_multi_index()
        out = []
        for bits in itertools.product((0, 1), repeat=self.dim):
            bits = bits[::-1]  # corner order: axis 0 bit fastest
            sel = tuple(idx[:, a] + bits[a] for a in range(self.dim))
            out.append(self.vertices[sel])
        return np.stack(out, axis=1)

    def geometry(self, xi):
        """Map and Jacobian at reference points xi (Q, d).

        Returns x (E, Q, d) and J (E, Q, d, d) with J[..., i, a] = dx_i / dxi_a.
        """
        d = self.dim
        xi = np.asarray(xi, float)
        Q = xi.shape[0]
        nshape = []
        dshape = []
        for bits in itertools.product((0, 1), repeat=d):
            bits = bits[::-1]
            val = np.ones(Q)
            grads = []
            for a in range(d):
                f = xi[:, a] if bits[a] else 1.0 - xi[:, a]
                val = val * f
            for a in range(d):
                g = np.ones(Q)
                for b in range(d):
                    if b == a:
                        g = g * (1.0 if bits[b] else -1.0)
                    else:
                        g = g * (xi[:, b] if bits[b] else 1.0 - xi[:, b])
                grads.append(g)
            nshape.append(val)
            dshape.append(np.stack(grads, axis=-1))
        N = np.stack(nshape, axis=1)          # (Q, 2^d)
        dN = np.stack(dshape, axis=1)         # (Q, 2^d, d)
        X = self.corners()                    # (E, 2^d, d)
        x = np.einsum("qc,eci->eqi", N, X)
        J = np.einsum("qca,eci->eqia", dN, X)
        return x, J


def tensor_grid(pts, dim):
    """All d-tuples of a 1-D point list, axis 0 fastest: (len^d, d)."""
    g = np.meshgrid(*([pts] * dim), indexing="ij")
    return np.stack([x.reshape(-1, order="F") for x in g], axis=-1)


def tensor_weights(w, dim):
    g = np.meshgrid(*([w] * dim), indexing="ij")
    out = np.ones(g[0].shape)
    for x in g:
        out = out * x
    return out.reshape(-1, order="F")


class Space:
    """Q_r^- Lambda^k on a structured lattice with canonical numbering."""

    def __init__(self, kind, nel, r, bc="natural", periodic=False):
        if kind not in KINDS:
            raise ValueError(kind)
        if bc not in ("natural", "essential"):
            raise ValueError(bc)
        self.kind = kind
        self.dim = len(nel)
        self.nel = tuple(int(n) for n in nel)
        self.r = int(r)
        self.bc = bc
        self.periodic = bool(periodic)
        self.m = tuple(self.r * n for n in self.nel)
        self.comps = components(kind, self.dim)
        self.ranges = []   # per comp, per axis: (first kept position, count)
        self.counts = []
        for comp in self.comps:
            rr = [self._axis_range(t, a) for a, t in enumerate(comp)]
            self.ranges.append(rr)
            self.counts.append(int(np.prod([c for _, c in rr])))
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.ndofs = int(self.offsets[-1])

    def _axis_range(self, t, a):
        m = self.m[a]
        if t == "e" or self.periodic:
            return (0, m)
        if self.bc == "essential":
            return (1, m - 1)
        return (0, m + 1)

    def index(self, c, pos):
        """Global index of component c at lattice positions pos (..., d); -1 if dropped."""
        pos = np.asarray(pos, dtype=np.int64)
        idx = np.zeros(pos.shape[:-1], dtype=np.int64)
        ok = np.ones(pos.shape[:-1], dtype=bool)
        stride = 1
        for a in range(self.dim):
            p = pos[..., a]
            if self.periodic:
                p = np.mod(p, self.m[a])
            start, cnt = self.ranges[c][a]
            loc = p - start
            ok &= (loc >= 0) & (loc < cnt)
            idx += np.where(ok, loc, 0) * stride
            stride *= cnt
        return np.where(ok, idx + self.offsets[c], -1)

    def positions(self, c):
        """Lattice positions (count_c, d) of component c in canonical order."""
        rr = self.ranges[c]
        axes = [np.arange(s, s + n) for s, n in rr]
        g = np.meshgrid(*axes, indexing="ij")
        return np.stack([x.reshape(-1, order="F") for x in g], axis=-1)

    def local_layout(self):
        """Per component the per-axis local counts (r+1 nodal, r edge)."""
        return [tuple(self.r + 1 if t == "n" else self.r for t in comp) for comp in self.comps]

    def element_dofs(self, mesh_elems):
        """Global indices (E, L) of each element's local basis, local order:
        component blocks, then lexicographic local multi-index, axis 0 fastest."""
        cols = []
        for c, loc in enumerate(self.local_layout()):
            for lidx in itertools.product(*[range(n) for n in loc[::-1]]):
                lidx = lidx[::-1]
                pos = mesh_elems * self.r + np.asarray(lidx)[None, :]
                cols.append(self.index(c, pos))
        return np.stack(cols, axis=1)

    def local_basis(self, xi_1d):
        """Reference proxy values on the tensor grid of xi_1d.

        Returns B (Q, L, d): B[q, l, :] is the reference vector proxy of local
        function l (scalar kinds use slot 0)."""
        from . import basis1d
        d = self.dim
        Q1 = len(xi_1d)
        tabs = {t: basis1d.table(t, self.r, xi_1d) for t in ("n", "e")}
        pts = [np.arange(Q1)] * d
        qg = np.meshgrid(*pts, indexing="ij")
        qidx = np.stack([x.reshape(-1, order="F") for x in qg], axis=-1)  # (Q, d)
        blocks = []
        for c, comp in enumerate(self.comps):
            loc = [self.r + 1 if t == "n" else self.r for t in comp]
            for lidx in itertools.product(*[range(n) for n in loc[::-1]]):
                lidx = lidx[::-1]
                val = np.ones(qidx.shape[0])
                for a in range(d):
                    val = val * tabs[comp[a]][qidx[:, a], lidx[a]]
                vec = np.zeros((qidx.shape[0], d))
                slot = 0 if self.kind in ("H1", "L2") else c
                vec[:, slot] = val
                blocks.append(vec)
        return np.stack(blocks, axis=1)


def cell_measures(space, mesh):
    """|sigma| for every degree of freedom on a uniform axis-aligned mesh.

    The paper normalises Whitney forms by average value (eq. WhitneyFormDefn);
    with integral DoFs the two normalisations differ by D = diag(|sigma|):
    coefficients a_paper = a / |sigma|, masses M_paper = D M D.
    """
    h = []
    for a in range(space.dim):
        v = mesh.vertices
        sl = [0] * space.dim
        sl_hi = [0] * space.dim
        sl_hi[a] = 1
        h.append(float(v[tuple(sl_hi)][a] - v[tuple(sl)][a]))
    out = np.zeros(space.ndofs)
    from . import basis1d
    nodes = basis1d.gll_nodes(space.r)
    for c, comp in enumerate(space.comps):
        pos = space.positions(c)
        meas = np.ones(pos.shape[0])
        for a, t in enumerate(comp):
            if t == "e":
                loc = np.mod(pos[:, a], space.r)
                meas *= h[a] * (nodes[loc + 1] - nodes[loc])
        out[space.offsets[c]:space.offsets[c + 1]] = meas
    return out
