"""Operator-probed sparse approximate inverse, SPAI-OP (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper section 5 (eqs. SPAIOPobjective, symmetricOptimality, ThatDefinition,
SPAIOPSylvester, SPAIOPcoefficient, diagonalPreconditioner).  A symmetric Q1
supported on a symmetric pattern S minimises

    || M1 Q1 - 1 ||_F^2 + lambda sum_k || (M1 Q1 - 1) W_k ||^2,   W = P2 V,

V the probed modes.  Stationarity over the shared entries (Q1)_ij = (Q1)_ji
gives, with U = M1^2, T = 1 + lambda W W^T and R = M1 T + T M1, the
generalized Sylvester equations

    (U Q1 T + T Q1 U)_ij = R_ij    for (i, j) in S,

a symmetric positive semidefinite system A q = r in the n_q entries of S.
It is solved matrix-free by conjugate gradients with the diagonal of A as
preconditioner and a small Tikhonov shift eps, as the paper does: A q is
formed by assembling Q1 from q, computing U Q1 T + T Q1 U with T applied as
its identity and rank-n_probe parts, and reading the result on S.

Pins (tests/test_oracle_spai_op.py), on the paper's 20 x 20 periodic Whitney
mesh: lambda = 0 converges to machine precision in 2 PCG iterations and
reproduces the column-wise SPAI (the paper states both); with the single
probe P2 v of the lowest mode and lambda = 5e5 the probed frequency is the
printed 1.00412, the probed-mode residual is below 1e-4 and the Frobenius
fit stays within 8% of SPAI's (all three printed).
"""
import numpy as np
import scipy.sparse as sp

from .spai import structural


class SpaiOp:
    """The Sylvester system of SPAI-OP for M1 on the pattern S(M1)."""

    def __init__(self, M1, W=None, lam=0.0, eps=None):
        self.M = structural(M1)  # the exact zeros of M1 are not in S
        self.n = self.M.shape[0]
        self.U = (self.M @ self.M).tocsr()
        pat = sp.coo_matrix(self.M)
        self.ir, self.ic = pat.row.copy(), pat.col.copy()  # the entries of S
        self.nq = len(self.ir)
        self.lam = float(lam)
        self.W = np.zeros((self.n, 0)) if W is None else np.asarray(W, dtype=np.float64).reshape(self.n, -1)
        dU = self.U.diagonal()
        dT = 1.0 + self.lam * (self.W ** 2).sum(axis=1)
        self.eps = 1e-12 * dU.max() if eps is None else float(eps)
        self.prec = dU[self.ir] * dT[self.ic] + dT[self.ir] * dU[self.ic] + self.eps
        MW = self.M @ self.W
        # R = M T + T M on S: 2 M + lambda (M W W^T + W W^T M)
        self.r = (2.0 * np.asarray(self.M[self.ir, self.ic]).ravel()
                  + self.lam * ((MW[self.ir] * self.W[self.ic]).sum(axis=1)
                                + (self.W[self.ir] * MW[self.ic]).sum(axis=1)))

    def assemble(self, q):
        return sp.csr_matrix((q, (self.ir, self.ic)), shape=(self.n, self.n))

    def apply(self, q):
        """A q = (U Q T + T Q U) on S, plus eps q."""
        Q = self.assemble(q)
        UQ = (self.U @ Q).tocsr()
        QU = (Q @ self.U).tocsr()
        out = np.asarray(UQ[self.ir, self.ic]).ravel() + np.asarray(QU[self.ir, self.ic]).ravel()
        if self.lam != 0.0 and self.W.shape[1]:
            X = self.U @ (Q @ self.W)                # U Q W      (n x n_probe)
            Y = ((self.W.T @ Q) @ self.U).T          # (W^T Q U)^T (n x n_probe)
            out += self.lam * ((X[self.ir] * self.W[self.ic]).sum(axis=1)
                               + (self.W[self.ir] * Y[self.ic]).sum(axis=1))
        return out + self.eps * q

    def solve(self, q0=None, rtol=1e-14, maxit=5000):
        """Jacobi-preconditioned CG from q0 (zero by default).  Returns the
        symmetric Q1, the iteration count and the final relative residual."""
        q = np.zeros(self.nq) if q0 is None else np.array(q0, dtype=np.float64)
        res = self.r - self.apply(q)
        bn = np.linalg.norm(self.r)
        z = res / self.prec
        p = z.copy()
        rz = res @ z
        it = 0
        rel = np.linalg.norm(res) / bn
        while rel > rtol and it < maxit:
            Ap = self.apply(p)
            a = rz / (p @ Ap)
            q += a * p
            res -= a * Ap
            it += 1
            rel = np.linalg.norm(res) / bn
            z = res / self.prec
            rz_new = res @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        return self.assemble(q), it, rel
