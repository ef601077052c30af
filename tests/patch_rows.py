"""Rows of the global block operators from an oracle patch (test helper).

One row of either block operator couples only unknowns of the elements that
contain its own unknown: every product in it (M1 G, G^T M1 G, C^T M2 C,
M3 D, D^T M3 D) stays inside one element, because incidence maps the
unknowns of an element's closure to unknowns of the same closure.  The oracle
assembled on a (2H+1)^3 element patch of the mesh (same vertices), with the
patch's own boundary conditions, therefore reproduces exactly the global rows
of the unknowns on the closure of any patch element at least one element
away from the patch boundary, or on the domain boundary where the patch
boundary coincides with it.
"""
import numpy as np

from oracle import problems
from oracle.lattice import Mesh, Space

H = 2  # patch = 2H+1 elements per axis


def global_spaces(which, nel, r):
    if which == "hodge":
        return [Space("H1", nel, r, "essential"), Space("HCURL", nel, r, "essential")]
    return [Space("HDIV", nel, r, "natural"), Space("L2", nel, r, "natural")]


def patch_problem(which, verts, r):
    mesh = Mesh(verts)
    P = problems.Hodge1(mesh, r) if which == "hodge" else problems.MixedPoisson(mesh, r)
    spaces = [P.s0, P.s1] if which == "hodge" else [P.sdiv, P.sl2]
    return P, spaces


def patch_rows(which, verts, nel, r, origin, mid):
    """Oracle patch operator and the maps patch unknown -> global unknown.

    Returns (A_patch, gmap, rows): gmap[k] = global index of patch unknown k;
    rows = patch unknowns on the closure of element `mid` (patch-local)."""
    sl = tuple(slice(o, o + 2 * H + 2) for o in origin)
    P, pspaces = patch_problem(which, verts[sl], r)
    gspaces = global_spaces(which, nel, r)
    goff = [0, gspaces[0].ndofs]
    poff = [0, pspaces[0].ndofs]
    gmap = np.empty(P.A.shape[0], dtype=np.int64)
    rows = []
    shift = np.array([r * o for o in origin])
    for b in range(2):
        ps, gs = pspaces[b], gspaces[b]
        for c in range(len(ps.comps)):
            pos = ps.positions(c)
            gi = gs.index(c, pos + shift)
            assert (gi >= 0).all()
            k0 = poff[b] + ps.offsets[c]
            gmap[k0:k0 + len(pos)] = goff[b] + gi
            inside = np.all((pos >= r * np.array(mid)) & (pos <= r * (np.array(mid) + 1)), axis=1)
            rows.append(k0 + np.nonzero(inside)[0])
    return P.A.tocsr(), gmap, np.concatenate(rows)


def origins(nel, rng):
    """Patch origins (low corner, interior, high corner) and the sampled
    element inside each patch (patch-local)."""
    lo = ((0, 0, 0), (0, 0, 0))
    hi = (tuple(n - (2 * H + 1) for n in nel), (2 * H, 2 * H, 2 * H))
    mid = tuple(int(rng.integers(0, n - (2 * H + 1) + 1)) for n in nel)
    return [lo, (mid, (H, H, H)), hi]
