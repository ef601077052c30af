"""Generalized Yee time stepping (oracle): shear maps composed by Strang splitting.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper section 3.  The discrete Maxwell system is Hamiltonian in the canonical
pair (a, e) (a: vector potential, e: M1-weighted electric field, both in
Lambda^1).  The mass matrices enter only the Hamiltonian (eq.
discTildeHamilSystem), here in units eps0 = 1, mu0 = 1 / c^2:

    H~(a, e) = 1/2 e^T Q1 e + 1/2 a^T P2 a,    P2 = c^2 C^T M~2 C,

with Q1 a symmetric approximation of M1^-1 and M~2 one of M2.  Each part
generates an exact shear map (eq. shearMaps):

    Phi^e_tau : a <- a - tau Q1 e,        Phi^a_tau : e <- e + tau P2 a,

composed here by Strang splitting Phi_tau = Phi^e_{tau/2} o Phi^a_tau o
Phi^e_{tau/2} (eq. strangSplit), applied literally, one step after another.

Choices of Q1 and M~2 (section 3 "Stability"; section 4.3 for the lumped
ones; section 5 for the sparse approximate inverses): 'exact' (Q1 = M1^-1
applied by a sparse LU solve; M~2 = M2), 'lumped' (the inverse row sums of
M1; the row sums of M2), and for Q1 only 'spai_diag' / 'spai' (the
symmetrised SPAI of M1 with the diagonal pattern S(1) or the pattern S(M1),
oracle/spai.py) or an explicit symmetric matrix (SPAI-OP, oracle/spai_op.py).  Row sums are
taken over the mass matrix of the space without boundary conditions and then
restricted to the kept unknowns: section 4.3 lumps rows that sum to the cell
volume, which the rows next to a perfect conductor only do before the
boundary unknowns are removed.

Stability (Proposition Stability): with Q1 and M~2 SPD the one-step map is
stable iff tau <= 2 / omega_max, omega_max^2 the largest eigenvalue of
K~ = Q1 P2.  Yee (section 4): Whitney forms (r = 1), lumped masses and
Strang splitting reproduce the Yee leapfrog; :func:`yee_fdtd` is that
leapfrog written directly as finite differences of cell-averaged fields.

Boundary: perfect conductor (tangential E = 0): a, e in H0(curl)
(essential), b = C a in H(div) (natural).  Or, with periodic=True, the torus
of sections 7.3 and 7.5: every axis periodic, no boundary; in 2-D the second
space is the scalar L2 space and C the 2-D curl.  Row sums are then those of
the periodic mass matrix itself.

Pins (tests/test_oracle_maxwell.py): equivalence with the hand-written Yee
finite differences; the one-step Jacobian against the paper's printed block
form; its spectrum on / off the unit circle at 0.9 / 1.1 tau_CFL and the
closed form of its eigenvalues; the lumped curl-of-curl spectrum against the
finite-difference symbol, and the exact (Whitney) one against the tensor
product of 1-D generalized eigenvalues; bounded energy; the phase rate of a
propagated eigenmode against 2 arcsin(tau omega / 2) / tau.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assembly, incidence, spai
from .lattice import Space


def _kept_row_sums(space, mesh):
    """Row sums of the mass matrix of `space` without boundary conditions,
    at the unknowns `space` keeps (its canonical order)."""
    if space.periodic:  # no boundary: the space's own rows
        return np.asarray(assembly.mass_matrix(space, mesh).sum(axis=1)).ravel()
    full = Space(space.kind, space.nel, space.r, "natural")
    rs = np.asarray(assembly.mass_matrix(full, mesh).sum(axis=1)).ravel()
    out = np.empty(space.ndofs)
    for c in range(len(space.comps)):
        pos = space.positions(c)
        out[space.index(c, pos)] = rs[full.index(c, pos)]
    return out


class Gym:
    """Generalized Yee method on a structured hexahedral mesh."""

    def __init__(self, mesh, r, q1="exact", m2="exact", c=1.0, periodic=False):
        given = sp.issparse(q1) or isinstance(q1, np.ndarray)
        if (not given and q1 not in ("exact", "lumped", "spai_diag", "spai")) or m2 not in ("exact", "lumped"):
            raise ValueError("q1: 'exact', 'lumped', 'spai_diag', 'spai' or a matrix; m2: 'exact' or 'lumped'")
        self.mesh, self.r, self.c = mesh, r, float(c)
        self.q1_kind, self.m2_kind = ("given" if given else q1), m2
        self.s1 = Space("HCURL", mesh.nel, r, "essential", periodic=periodic)
        self.s2 = Space("HDIV" if len(mesh.nel) == 3 else "L2", mesh.nel, r, "natural", periodic=periodic)
        self.M1 = assembly.mass_matrix(self.s1, mesh).tocsc()
        self.M2 = assembly.mass_matrix(self.s2, mesh).tocsr()
        self.C = incidence.curl(self.s1, self.s2).astype(np.float64).tocsr()
        self.rs1 = _kept_row_sums(self.s1, mesh)
        self.rs2 = _kept_row_sums(self.s2, mesh)
        M2t = self.M2 if m2 == "exact" else sp.diags(self.rs2)
        self.P2 = (self.c ** 2 * (self.C.T @ M2t @ self.C)).tocsr()
        self._lu = spla.splu(self.M1) if self.q1_kind == "exact" else None
        self.Q1 = None
        if given:  # an explicit symmetric Q1 (e.g. SPAI-OP, oracle/spai_op.py)
            self.Q1 = sp.csr_matrix(q1)
        elif q1.startswith("spai"):
            self.Q1 = spai.spai(self.M1, "diag" if q1 == "spai_diag" else "m")
        self.n = self.s1.ndofs

    def q1(self, e):
        """Q1 e: M1^-1 e (exact), e / rowsum(M1) (lumped) or the SPAI times e."""
        if self._lu is not None:
            return self._lu.solve(e)
        if self.Q1 is not None:
            return self.Q1 @ e
        return e / self.rs1

    def p2(self, a):
        return self.P2 @ a

    def strang(self, a, e, tau, nsteps):
        """nsteps Strang steps, each Phi^e_{tau/2}, then Phi^a_tau, then Phi^e_{tau/2}."""
        a, e = a.copy(), e.copy()
        for _ in range(nsteps):
            a = a - 0.5 * tau * self.q1(e)
            e = e + tau * self.p2(a)
            a = a - 0.5 * tau * self.q1(e)
        return a, e

    def energy(self, a, e):
        """H~ = 1/2 e^T Q1 e + 1/2 a^T P2 a."""
        return 0.5 * e @ self.q1(e) + 0.5 * a @ self.p2(a)

    def q1_dense(self):
        if self._lu is not None:
            return np.linalg.inv(self.M1.toarray())
        if self.Q1 is not None:
            return self.Q1.toarray()
        return np.diag(1.0 / self.rs1)

    def jacobian(self, tau):
        """One Strang step as a dense matrix on (a, e): the product of the
        three shear maps' Jacobians."""
        n = self.n
        I = np.eye(n)
        Q = self.q1_dense()
        P = self.P2.toarray()
        Je = np.block([[I, -0.5 * tau * Q], [np.zeros((n, n)), I]])
        Ja = np.block([[I, np.zeros((n, n))], [tau * P, I]])
        return Je @ Ja @ Je

    def omega2(self):
        """Eigenvalues omega^2 of K~ = Q1 P2 (ascending): P2 v = omega^2 Q1^-1 v."""
        if self._lu is not None:
            return sla.eigh(self.P2.toarray(), self.M1.toarray(), eigvals_only=True)
        if self.Q1 is not None:
            # Q1 P2 is similar to Q1^1/2 P2 Q1^1/2 when Q1 is positive definite
            wq, V = np.linalg.eigh(self.Q1.toarray())
            if wq.min() <= 0:
                raise ValueError("the SPAI is not positive definite")
            Qh = (V * np.sqrt(wq)) @ V.T
            return np.linalg.eigvalsh(Qh @ self.P2.toarray() @ Qh)
        d = 1.0 / np.sqrt(self.rs1)
        return np.linalg.eigvalsh(d[:, None] * self.P2.toarray() * d[None, :])

    def tau_cfl(self):
        return 2.0 / np.sqrt(self.omega2()[-1])

    def lowest_modes(self, k):
        """The k smallest eigenvalues omega^2 of K~ = Q1 P2 outside its kernel
        (the gradients), ascending (dense generalized eigenproblem)."""
        w = self.omega2()
        return np.sort(w[w > 1e-9 * w[-1]])[:k]

    def eigenmode(self, k):
        """k-th smallest non-kernel mode (omega^2, v) of the exact operator
        M1^-1 P2 (generalized symmetric eigenproblem, dense)."""
        w, V = sla.eigh(self.P2.toarray(), self.M1.toarray())
        tol = 1e-9 * w[-1]
        nz = np.nonzero(w > tol)[0]
        return w[nz[k]], V[:, nz[k]]


def yee_fdtd(nel, h, c, tau, E, B, nsteps):
    """Yee's leapfrog on cell-averaged fields, written as finite differences.

    E = (Ex, Ey, Ez) on edges: Ex[i, j, k] at (i + 1/2, j, k), shape
    (N0, N1+1, N2+1), etc.  B = (Bx, By, Bz) on faces: Bx[i, j, k] at
    (i, j + 1/2, k + 1/2), shape (N0+1, N1, N2), etc.  Tangential E on the
    boundary stays zero (perfect conductor).  Each step: B -= tau/2 curl E,
    E += tau c^2 curl B, B -= tau/2 curl E (the Strang composition; the two
    half steps between consecutive steps form the usual leapfrog)."""
    hx, hy, hz = h
    Ex, Ey, Ez = [x.copy() for x in E]
    Bx, By, Bz = [x.copy() for x in B]

    def faraday(s):
        Bx[...] -= s * ((Ez[:, 1:, :] - Ez[:, :-1, :]) / hy - (Ey[:, :, 1:] - Ey[:, :, :-1]) / hz)
        By[...] -= s * ((Ex[:, :, 1:] - Ex[:, :, :-1]) / hz - (Ez[1:, :, :] - Ez[:-1, :, :]) / hx)
        Bz[...] -= s * ((Ey[1:, :, :] - Ey[:-1, :, :]) / hx - (Ex[:, 1:, :] - Ex[:, :-1, :]) / hy)

    def ampere(s):
        Ex[:, 1:-1, 1:-1] += s * ((Bz[:, 1:, 1:-1] - Bz[:, :-1, 1:-1]) / hy - (By[:, 1:-1, 1:] - By[:, 1:-1, :-1]) / hz)
        Ey[1:-1, :, 1:-1] += s * ((Bx[1:-1, :, 1:] - Bx[1:-1, :, :-1]) / hz - (Bz[1:, :, 1:-1] - Bz[:-1, :, 1:-1]) / hx)
        Ez[1:-1, 1:-1, :] += s * ((By[1:, 1:-1, :] - By[:-1, 1:-1, :]) / hx - (Bx[1:-1, 1:, :] - Bx[1:-1, :-1, :]) / hy)

    for _ in range(nsteps):
        faraday(0.5 * tau)
        ampere(tau * c * c)
        faraday(0.5 * tau)
    return (Ex, Ey, Ez), (Bx, By, Bz)
