"""Pins of the oracle's generalized Yee time stepping (oracle/maxwell.py).

Each pin checks the oracle against something other than itself: the Yee
leapfrog written directly as finite differences (paper section 4), the
one-step Jacobian printed in section 3 and its eigenvalue pairs (eq.
eigenvaluePairs), the stability threshold tau_CFL = 2 / omega_max
(Proposition Stability), the finite-difference dispersion symbol of the
lumped Whitney curl-of-curl, and the exact harmonic motion of one eigenmode.
"""
import numpy as np
import pytest

import synth
from conftest import golden
from oracle import maxwell
from oracle.lattice import Mesh


def _mesh(nel, hi):
    return Mesh(synth.uniform_vertices(nel, hi=hi))


def _yee_arrays(G, e, b):
    """Cell averages of the GYM state: E = (Delta_edge / Delta_V) e on edges
    (e is M1-weighted: E_line = Q1 e = Delta_edge^2 / Delta_V e for lumped
    Whitney forms), B = b / area on faces."""
    N = G.mesh.nel
    h = [G.mesh.vertices[(1, 0, 0)][0] - G.mesh.vertices[(0, 0, 0)][0],
         G.mesh.vertices[(0, 1, 0)][1] - G.mesh.vertices[(0, 0, 0)][1],
         G.mesh.vertices[(0, 0, 1)][2] - G.mesh.vertices[(0, 0, 0)][2]]
    dv = h[0] * h[1] * h[2]
    E, B = [], []
    for c in range(3):
        shape = [N[a] + (0 if a == c else 1) for a in range(3)]
        arr = np.zeros(shape)
        pos = G.s1.positions(c)
        arr[tuple(pos.T)] = e[G.s1.index(c, pos)] * h[c] / dv
        E.append(arr)
        shape = [N[a] + (1 if a == c else 0) for a in range(3)]
        arr = np.zeros(shape)
        pos = G.s2.positions(c)
        area = dv / h[c]
        arr[tuple(pos.T)] = b[G.s2.index(c, pos)] / area
        B.append(arr)
    return E, B, h


@pytest.mark.parametrize("nsteps", [1, 5])
def test_lumped_whitney_gym_is_the_yee_leapfrog(nsteps):
    # Section 4: Whitney forms, lumped masses and Strang splitting reproduce
    # Yee's updates (the paper reports agreement below 1e-15 after one step).
    G = maxwell.Gym(_mesh((4, 3, 5), (1.0, 0.9, 1.3)), 1, q1="lumped", m2="lumped", c=1.3)
    a0 = synth.random_vector(G.n, seed=1)
    e0 = synth.random_vector(G.n, seed=2)
    tau = 0.5 * G.tau_cfl()
    a1, e1 = G.strang(a0, e0, tau, nsteps)
    E0, B0, h = _yee_arrays(G, e0, G.C @ a0)
    E1, B1 = maxwell.yee_fdtd(G.mesh.nel, h, G.c, tau, E0, B0, nsteps)
    Eg, Bg, _ = _yee_arrays(G, e1, G.C @ a1)
    for x, y in zip(list(E1) + list(B1), list(Eg) + list(Bg)):
        assert np.abs(x - y).max() <= 1e-14 * np.abs(x).max()
    num = np.sqrt(sum(((x - y) ** 2).sum() for x, y in zip(E1, Eg)))
    assert num <= 1e-15 * nsteps * np.sqrt(sum((x ** 2).sum() for x in E1))


@pytest.mark.parametrize("q1", ["exact", "lumped"])
def test_jacobian_is_the_printed_block_form(q1):
    # Section 3: J = [[1 - tau^2/2 K, tau^3/4 K Q1 - tau Q1], [tau P2, 1 - tau^2/2 P2 Q1]]
    G = maxwell.Gym(_mesh((2, 3, 2), (1.0, 1.0, 1.0)), 1, q1=q1, m2="exact")
    tau = 0.37 * G.tau_cfl()
    Q = G.q1_dense()
    P = G.P2.toarray()
    K = Q @ P
    I = np.eye(G.n)
    J = np.block([[I - 0.5 * tau ** 2 * K, 0.25 * tau ** 3 * K @ Q - tau * Q],
                  [tau * P, I - 0.5 * tau ** 2 * P @ Q]])
    assert np.abs(G.jacobian(tau) - J).max() <= 1e-12 * np.abs(J).max()


@pytest.mark.parametrize("q1,nel,r", [("exact", (2, 3, 2), 1), ("lumped", (2, 3, 2), 1), ("exact", (2, 2, 2), 2)])
def test_cfl_threshold(q1, nel, r):
    # Proposition Stability: all eigenvalues on the unit circle iff tau <= 2 / omega_max;
    # they come in reciprocal pairs either way (symplecticity).
    G = maxwell.Gym(_mesh(nel, (1.0, 1.0, 1.0)), r, q1=q1, m2="exact")
    tcfl = G.tau_cfl()
    lam = np.linalg.eigvals(G.jacobian(0.9 * tcfl))
    assert np.abs(np.abs(lam) - 1).max() < 1e-7
    lam = np.linalg.eigvals(G.jacobian(1.1 * tcfl))
    assert np.abs(lam).max() > 1.1
    big = np.sort(np.abs(lam))
    assert np.allclose(big * big[::-1], 1.0, atol=1e-7)


def test_strang_eigenvalue_pairs():
    # eq. eigenvaluePairs: each omega^2 of K gives lambda = 1 - z/2 +- sqrt(z (z - 4)) / 2, z = tau^2 omega^2
    G = maxwell.Gym(_mesh((2, 2, 3), (1.0, 1.0, 1.0)), 1, q1="exact", m2="exact")
    tau = 0.8 * G.tau_cfl()
    z = tau ** 2 * G.omega2()
    pred = np.concatenate([1 - z / 2 + 0.5 * np.sqrt(z * (z - 4) + 0j), 1 - z / 2 - 0.5 * np.sqrt(z * (z - 4) + 0j)])
    lam = np.linalg.eigvals(G.jacobian(tau))
    key = lambda v: np.round(np.angle(v), 9)
    assert np.allclose(np.sort_complex(lam[np.argsort(key(lam))]), np.sort_complex(pred[np.argsort(key(pred))]),
                       atol=1e-8)


def test_lumped_spectrum_is_the_yee_dispersion_symbol():
    # Lumped Whitney forms on a perfect-conductor box: the non-zero omega^2 are
    # c^2 sum_a (2 / h_a)^2 sin^2(pi n_a / (2 N_a)), with two polarisations
    # when n_x, n_y, n_z > 0, one when exactly one of them is zero.
    nel, hi, c = (3, 4, 2), (1.2, 1.0, 0.7), 0.8
    G = maxwell.Gym(_mesh(nel, hi), 1, q1="lumped", m2="lumped", c=c)
    w2 = G.omega2()
    nonzero = np.sort(w2[w2 > 1e-9 * w2[-1]])
    h = [hi[a] / nel[a] for a in range(3)]
    pred = []
    for nx in range(nel[0]):
        for ny in range(nel[1]):
            for nz in range(nel[2]):
                n = (nx, ny, nz)
                pos = sum(1 for v in n if v > 0)
                mult = 2 if pos == 3 else (1 if pos == 2 else 0)
                val = c * c * sum((2 / h[a]) ** 2 * np.sin(np.pi * n[a] / (2 * nel[a])) ** 2 for a in range(3))
                pred += [val] * mult
    pred = np.sort(pred)
    assert len(pred) == len(nonzero)
    assert np.allclose(nonzero, pred, rtol=1e-12)


def whitney_spectrum(nel, hi, c):
    """Non-kernel omega^2 of M1^-1 P2 for Whitney forms with exact masses on
    a uniform perfect-conductor box: on a tensor lattice the curl-of-curl
    separates into 1-D problems, and the 1-D nodal stiffness (1/h)[2, -1]
    against the 1-D mass (h/6)[4, 1] has the eigenvalues
    (6/h^2)(1 - cos t)/(2 + cos t), t = pi n / N.  Multiplicity: two
    polarisations when n_x, n_y, n_z > 0, one when exactly one is zero."""
    h = [hi[a] / nel[a] for a in range(3)]
    lam = [[(6 / h[a] ** 2) * (1 - np.cos(np.pi * n / nel[a])) / (2 + np.cos(np.pi * n / nel[a]))
            for n in range(nel[a])] for a in range(3)]
    out = []
    for nx in range(nel[0]):
        for ny in range(nel[1]):
            for nz in range(nel[2]):
                pos = (nx > 0) + (ny > 0) + (nz > 0)
                mult = 2 if pos == 3 else (1 if pos == 2 else 0)
                out += [c * c * (lam[0][nx] + lam[1][ny] + lam[2][nz])] * mult
    return np.sort(out)


@pytest.mark.parametrize("nel,hi", [((3, 4, 2), (1.2, 1.0, 0.7)), ((3, 3, 3), (1.0, 1.0, 1.0))])
def test_exact_whitney_spectrum_closed_form(nel, hi):
    # The exact-FEEC operator K = M1^-1 P2 (section 3) on a box: every
    # non-kernel eigenvalue of the dense generalized problem against the
    # closed form, with multiplicities.
    c = 0.8
    G = maxwell.Gym(_mesh(nel, hi), 1, q1="exact", m2="exact", c=c)
    pred = whitney_spectrum(nel, hi, c)
    got = G.lowest_modes(10 ** 6)
    assert len(got) == len(pred)
    assert np.allclose(got, pred, rtol=1e-12)


def test_energy_is_bounded():
    # Symplectic Strang splitting: the modified energy oscillates without drift.
    G = maxwell.Gym(_mesh((3, 3, 3), (1.0, 1.0, 1.0)), 2, q1="exact", m2="exact")
    tau = 0.3 * G.tau_cfl()
    a = synth.random_vector(G.n, seed=3)
    e = synth.random_vector(G.n, seed=4)
    H0 = G.energy(a, e)
    dev = []
    for _ in range(40):
        a, e = G.strang(a, e, tau, 25)
        dev.append(G.energy(a, e) / H0 - 1)
    dev = np.abs(np.array(dev))
    assert dev.max() < (0.3 * 2) ** 2
    assert dev[20:].max() < 1.5 * dev[:20].max() + 1e-12


def test_eigenmode_phase_rate():
    # A mode of M1^-1 P2 started as (a, e) = (0, M1 v) stays in its invariant
    # plane: <e(n), e(0)> / |e(0)|^2 = cos(n theta), cos(theta) = 1 - tau^2 omega^2 / 2,
    # i.e. numerical frequency 2 arcsin(tau omega / 2) / tau.
    G = maxwell.Gym(_mesh((3, 2, 3), (1.0, 1.0, 1.0)), 2, q1="exact", m2="exact")
    w2, v = G.eigenmode(0)
    tau = 0.3 * G.tau_cfl()
    theta = 2 * np.arcsin(tau * np.sqrt(w2) / 2)
    e0 = G.M1 @ v
    a, e = np.zeros(G.n), e0.copy()
    for n in range(1, 61):
        a, e = G.strang(a, e, tau, 1)
        assert abs(e @ e0 / (e0 @ e0) - np.cos(n * theta)) < 1e-10


@pytest.mark.parametrize("q1,key", [("exact", "omega_20x20"), ("spai_diag", "spai_diag_omega_20x20"),
                                    ("spai", "spai_m1_omega_20x20")])
def test_periodic_torus_frequencies(q1, key):
    # Section 7.5: the lowest non-kernel frequency of Q1 P2 on the 20 x 20
    # periodic Whitney mesh, for exact Q1 and the two SPAI patterns, through
    # the Gym class on periodic spaces (2-D: Lambda^2 is L2, C the 2-D curl)
    G = maxwell.Gym(Mesh(synth.uniform_vertices((20, 20), hi=(2 * np.pi, 2 * np.pi))), 1, q1=q1, periodic=True)
    val, tol = golden(key)
    w = G.lowest_modes(1)
    assert abs(np.sqrt(w[0]) - val) < tol


def test_periodic_gym_kernel_holds_the_harmonic_fields():
    # on the torus ker P2 is the gradients plus one constant field per axis:
    # dim ker = (n0 - 1) + 2 in 2-D (n0: periodic nodal unknowns)
    nel = (5, 4)
    G = maxwell.Gym(Mesh(synth.uniform_vertices(nel)), 2, periodic=True)
    w = G.omega2()
    n0 = (2 * 5) * (2 * 4)
    assert int(np.sum(w < 1e-9 * w.max())) == (n0 - 1) + 2
