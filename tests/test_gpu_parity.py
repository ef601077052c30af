"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Incidence must match bit for bit (ascending-order sums of +-1 terms).
Floating-point applies are compared element by element with a relative
tolerance of 1e-13 of the output's max norm in FP64: both sides evaluate the
same Gauss-point sums, so they differ only by summation order (O(10) roundings
of terms bounded by the output scale).  FP32 contractions: 2e-5.
"""
import numpy as np
import pytest

import synth
from oracle import assembly, incidence, problems
from oracle.lattice import Mesh, Space

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    from paper_2301_01753_amd import gym
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = gym.gym_create(0)
    yield gym, ctx
    gym.gym_destroy(ctx)


DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _mesh(gym, ctx, nel, hi=None):
    return gym.gym_mesh_create(ctx, len(nel), nel, hi=hi)


KINDS = {"H1": 0, "HCURL": 1, "HDIV": 2, "L2": 3}


# ---- incidence: bit-exact ----------------------------------------------------
INC_CASES = [
    ((3, 4, 2), 1, "natural"), ((3, 4, 2), 2, "essential"), ((2, 3, 5), 3, "natural"),
    ((5, 2, 3), 4, "essential"), ((1, 1, 1), 1, "natural"), ((7, 3, 2), 2, "natural"),
]


@pytest.mark.parametrize("nel,r,bc", INC_CASES)
def test_incidence_bit_exact_3d(g, nel, r, bc):
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    bcc = 1 if bc == "essential" else 0
    chain = ["H1", "HCURL", "HDIV", "L2"]
    fns = [incidence.gradient, incidence.curl, incidence.divergence]
    for k in range(3):
        so = [Space(chain[k], nel, r, bc), Space(chain[k + 1], nel, r, bc)]
        sg = [gym.gym_space_create(ctx, mesh, KINDS[chain[k]], r, bcc),
              gym.gym_space_create(ctx, mesh, KINDS[chain[k + 1]], r, bcc)]
        assert gym.gym_space_ndofs(sg[0]) == so[0].ndofs
        assert gym.gym_space_ndofs(sg[1]) == so[1].ndofs
        A = fns[k](so[0], so[1])
        for tr in (0, 1):
            nin = so[1].ndofs if tr else so[0].ndofs
            x = synth.random_vector(nin, seed=10 + k + 3 * tr)
            y = torch.full((so[0].ndofs if tr else so[1].ndofs,), np.nan, dtype=torch.float64, device=DEV)
            gym.gym_d_apply(sg[0], sg[1], tr, _t(x), y)
            torch.cuda.synchronize()
            ref = incidence.apply_ordered(incidence.transpose(A) if tr else A, x)
            got = y.cpu().numpy()
            assert np.array_equal(got, ref), f"k={k} tr={tr}: {np.abs(got - ref).max()}"
        for s in sg:
            gym.gym_space_destroy(s)
    gym.gym_mesh_destroy(mesh)


def test_incidence_complex_exact_on_integers(g):
    # C (G x) and D (C y) vanish exactly for integer data below 2^50.
    gym, ctx = g
    nel, r = (4, 3, 5), 2
    mesh = _mesh(gym, ctx, nel)
    s = [gym.gym_space_create(ctx, mesh, k, r, 0) for k in range(4)]
    n = [gym.gym_space_ndofs(t) for t in s]
    rng = np.random.default_rng(0)
    u = _t(rng.integers(-2 ** 40, 2 ** 40, n[0]).astype(np.float64))
    a = _t(rng.integers(-2 ** 40, 2 ** 40, n[1]).astype(np.float64))
    gu = torch.empty(n[1], dtype=torch.float64, device=DEV)
    cgu = torch.empty(n[2], dtype=torch.float64, device=DEV)
    ca = torch.empty(n[2], dtype=torch.float64, device=DEV)
    dca = torch.empty(n[3], dtype=torch.float64, device=DEV)
    gym.gym_d_apply(s[0], s[1], 0, u, gu)
    gym.gym_d_apply(s[1], s[2], 0, gu, cgu)
    gym.gym_d_apply(s[1], s[2], 0, a, ca)
    gym.gym_d_apply(s[2], s[3], 0, ca, dca)
    torch.cuda.synchronize()
    assert torch.all(cgu == 0) and torch.all(dca == 0)


@pytest.mark.parametrize("r", [1, 3])
def test_incidence_bit_exact_2d(g, r):
    gym, ctx = g
    nel = (5, 3)
    mesh = _mesh(gym, ctx, nel)
    pairs = [("H1", "HCURL", incidence.gradient), ("HCURL", "L2", incidence.curl), ("HDIV", "L2", incidence.divergence)]
    for a, b, fn in pairs:
        so = [Space(a, nel, r), Space(b, nel, r)]
        sg = [gym.gym_space_create(ctx, mesh, KINDS[a], r, 0), gym.gym_space_create(ctx, mesh, KINDS[b], r, 0)]
        A = fn(*so)
        for tr in (0, 1):
            x = synth.random_vector(A.shape[0] if tr else A.shape[1], seed=5)
            y = torch.empty(A.shape[1] if tr else A.shape[0], dtype=torch.float64, device=DEV)
            gym.gym_d_apply(sg[0], sg[1], tr, _t(x), y)
            torch.cuda.synchronize()
            ref = incidence.apply_ordered(incidence.transpose(A) if tr else A, x)
            assert np.array_equal(y.cpu().numpy(), ref)


# ---- mass apply ----------------------------------------------------------------
MASS_CASES = [
    ("H1", (9, 10, 3), 1, "natural"), ("HCURL", (9, 3, 10), 2, "essential"), ("HDIV", (4, 7, 5), 3, "natural"),
    ("L2", (5, 4, 3), 4, "natural"), ("HCURL", (4, 5, 7), 4, "natural"), ("H1", (7, 5, 4), 3, "essential"),
    ("HDIV", (17, 9, 2), 1, "natural"), ("L2", (9, 2, 9), 2, "natural"),
]


def _rel(got, ref):
    return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)


FORMS = [(0, 1), (0, 2), (1, 1), (1, 2)]   # (mass form, tile option)


@pytest.fixture(params=FORMS, ids=["kron-large", "kron-small", "gauss-large", "gauss-small"])
def form(request, g):
    gym, ctx = g
    gym.gym_ctx_set(ctx, gym.GYM_OPT_MASS_FORM, request.param[0])
    gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, request.param[1])
    yield request.param
    gym.gym_ctx_set(ctx, gym.GYM_OPT_MASS_FORM, 0)
    gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, 0)


@pytest.mark.parametrize("kind,nel,r,bc", MASS_CASES)
def test_mass_apply_3d(g, form, kind, nel, r, bc):
    gym, ctx = g
    hi = (1.0, 1.7, 0.6)
    mesh = _mesh(gym, ctx, nel, hi=hi)
    sp = gym.gym_space_create(ctx, mesh, KINDS[kind], r, 1 if bc == "essential" else 0)
    so = Space(kind, nel, r, bc)
    M = assembly.mass_matrix(so, Mesh(synth.uniform_vertices(nel, hi=hi)))
    x = synth.random_vector(so.ndofs, seed=r, nrhs=2)
    y = torch.empty(2 * so.ndofs, dtype=torch.float64, device=DEV)
    gym.gym_mass_apply(sp, gym.GYM_F64, 2, _t(x), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().reshape(2, -1)
    for k in range(2):
        ref = M @ x.reshape(2, -1)[k]
        assert _rel(got[k], ref) < 1e-13
    # FP32 contractions
    x32 = torch.tensor(x, dtype=torch.float32, device=DEV)
    y32 = torch.empty(2 * so.ndofs, dtype=torch.float32, device=DEV)
    gym.gym_mass_apply(sp, gym.GYM_F32, 2, x32, y32)
    torch.cuda.synchronize()
    ref = M @ x.reshape(2, -1)[1]
    assert _rel(y32.cpu().numpy().reshape(2, -1)[1].astype(np.float64), ref) < 2e-5


@pytest.mark.parametrize("kind", ["H1", "HCURL", "HDIV", "L2"])
@pytest.mark.parametrize("r", [1, 2, 4])
def test_mass_apply_2d(g, form, kind, r):
    gym, ctx = g
    nel = (19, 6)
    mesh = _mesh(gym, ctx, nel, hi=(2.0, 0.5))
    sp = gym.gym_space_create(ctx, mesh, KINDS[kind], r, 0)
    so = Space(kind, nel, r)
    M = assembly.mass_matrix(so, Mesh(synth.uniform_vertices(nel, hi=(2.0, 0.5))))
    x = synth.random_vector(so.ndofs, seed=7)
    y = torch.empty(so.ndofs, dtype=torch.float64, device=DEV)
    gym.gym_mass_apply(sp, gym.GYM_F64, 1, _t(x), y)
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), M @ x) < 1e-13


# ---- block operators -------------------------------------------------------------
OP_CASES = [
    ("poisson", (11, 10), 1), ("poisson", (6, 17), 2), ("poisson", (5, 4), 4),
    ("poisson", (9, 9, 5), 1), ("poisson", (7, 3, 6), 2), ("poisson", (5, 7, 3), 3), ("poisson", (4, 5, 4), 4),
    ("hodge", (9, 10, 4), 1), ("hodge", (9, 4, 5), 2), ("hodge", (5, 7, 3), 3), ("hodge", (4, 3, 5), 4),
    ("hodge", (1, 1, 1), 2), ("poisson", (1, 1, 1), 3),
]


def _oracle_problem(which, nel, r):
    mesh = Mesh(synth.uniform_vertices(nel))
    return problems.MixedPoisson(mesh, r) if which == "poisson" else problems.Hodge1(mesh, r)


@pytest.mark.parametrize("which,nel,r", OP_CASES)
def test_operator_apply(g, form, which, nel, r):
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem(which, nel, r)
    n = gym.gym_op_ndofs(op)
    assert n == P.A.shape[0]
    assert gym.gym_op_block_sizes(op) == P.n
    x = synth.random_vector(n, seed=3, nrhs=2)
    y = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    gym.gym_op_apply(op, gym.GYM_F64, 2, _t(x), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().reshape(2, -1)
    for k in range(2):
        ref = P.A @ x.reshape(2, -1)[k]
        assert _rel(got[k], ref) < 1e-13, f"rhs {k}"
    # FP32 contractions on FP32 vectors
    y32 = torch.empty(2 * n, dtype=torch.float32, device=DEV)
    gym.gym_op_apply(op, gym.GYM_F32, 2, torch.tensor(x, dtype=torch.float32, device=DEV), y32)
    torch.cuda.synchronize()
    ref = P.A @ x.reshape(2, -1)[0]
    assert _rel(y32.cpu().numpy().reshape(2, -1)[0].astype(np.float64), ref) < 5e-5
    # preconditioner diagonal
    d = torch.empty(n, dtype=torch.float64, device=DEV)
    gym.gym_op_precond_diag(op, d)
    assert _rel(d.cpu().numpy(), P.precond_diag()) < 1e-13
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


@pytest.mark.parametrize("which,nel,r", [("poisson", (6, 5, 4), 2), ("hodge", (5, 4, 6), 2),
                                         ("poisson", (16, 16), 1), ("hodge", (3, 3, 3), 3)])
def test_manufactured_load_vector(g, which, nel, r):
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem(which, nel, r)
    dim = len(nel)
    modes = synth.modes_3d() if dim == 3 else synth.modes_2d()
    if which == "poisson":
        c = synth.fourier_coeffs(0, len(modes), 1)
        _, _, f = problems.poisson_fields(c[:, 0], modes)
    else:
        c = synth.fourier_coeffs(0, len(modes), 3)
        _, _, f = problems.hodge_fields(c, modes)
    b = torch.empty(P.A.shape[0], dtype=torch.float64, device=DEV)
    gym.gym_rhs_manufactured(op, modes, c, b)
    ref = P.rhs(f)
    assert _rel(b.cpu().numpy(), ref) < 1e-12
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


# ---- solves ----------------------------------------------------------------------
SOLVE_CASES = [("poisson", (16, 16), 1), ("poisson", (5, 6, 4), 2), ("hodge", (4, 5, 4), 2),
               ("hodge", (3, 3, 3), 3), ("poisson", (3, 3, 2), 4)]


@pytest.mark.parametrize("which,nel,r", SOLVE_CASES)
def test_solve_fp64_matches_direct(g, which, nel, r):
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem(which, nel, r)
    n = P.A.shape[0]
    b = synth.random_vector(n, seed=11, nrhs=2)
    x = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.rtol = 1e-13
    info = gym.gym_solve(op, opts, 2, _t(b), x)
    got = x.cpu().numpy().reshape(2, -1)
    for k in range(2):
        ref = problems.solve_direct(P.A, b.reshape(2, -1)[k])
        err = np.linalg.norm(got[k] - ref) / np.linalg.norm(ref)
        assert err < 1e-10, f"rhs {k}: rel err {err}, iters {info.iters}, rel_res {info.rel_res}"
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


@pytest.mark.parametrize("maxit", [1, 7, 30])
@pytest.mark.parametrize("which,nel,r", [("hodge", (4, 3, 5), 2), ("poisson", (5, 4, 3), 1)])
def test_solve_iteration_cap_matches_minres_iterate(g, which, nel, r, maxit):
    # Stopped by the iteration cap, the solve returns the k-th preconditioned
    # MINRES iterate (the pending step is completed without another apply):
    # SciPy's Paige-Saunders MINRES with the same diagonal, k iterations.
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem(which, nel, r)
    n = P.A.shape[0]
    b = synth.random_vector(n, seed=21, nrhs=2)
    x = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.rtol = 1e-14
    opts.maxit = maxit
    opts.check_every = 4
    info = gym.gym_solve(op, opts, 2, _t(b), x)
    assert info.iters == maxit and info.status == gym.GYM_W_NOT_CONVERGED
    got = x.cpu().numpy().reshape(2, -1)
    for k in range(2):
        ref, _ = problems.solve_minres(P.A, b.reshape(2, -1)[k], P.precond_diag(), rtol=1e-300, maxiter=maxit)
        err = np.linalg.norm(got[k] - ref) / np.linalg.norm(ref)
        assert err < 1e-10, f"rhs {k}: {maxit} iterations, rel diff {err}"
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


def test_solve_converged_rhs_is_left_alone(g):
    # Three right-hand sides in one launch; the zero one is converged at the
    # start and must stay exactly zero while the others iterate.
    gym, ctx = g
    nel, r = (4, 4, 3), 2
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem("hodge", nel, r)
    n = P.A.shape[0]
    b = np.concatenate([synth.random_vector(n, seed=5), np.zeros(n), synth.random_vector(n, seed=6)])
    x = torch.full((3 * n,), 7.0, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.rtol = 1e-12
    info = gym.gym_solve(op, opts, 3, _t(b), x)
    got = x.cpu().numpy().reshape(3, -1)
    assert info.status == 0
    assert np.all(got[1] == 0.0)
    for k in (0, 2):
        ref = problems.solve_direct(P.A, b.reshape(3, -1)[k])
        assert np.linalg.norm(got[k] - ref) / np.linalg.norm(ref) < 1e-9
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


@pytest.mark.parametrize("which,nel,r", [("poisson", (5, 6, 4), 2), ("hodge", (4, 5, 4), 2)])
def test_solve_mixed_precision_refinement(g, which, nel, r):
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem(which, nel, r)
    n = P.A.shape[0]
    b = synth.random_vector(n, seed=12)
    x = torch.empty(n, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.mode = gym.GYM_MODE_IR_F32
    opts.rtol = 1e-12
    opts.inner_rtol = 1e-4
    info = gym.gym_solve(op, opts, 1, _t(b), x)
    ref = problems.solve_direct(P.A, b)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert info.status == 0 and info.outer_iters >= 1
    assert err < 1e-8, f"rel err {err}, outer {info.outer_iters}, iters {info.iters}"
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


def test_hodge_polynomial_solution_on_gpu(g):
    # u in Q_2^- Lambda^1 with zero tangential trace is reproduced exactly.
    gym, ctx = g
    nel, r = (4, 3, 5), 2
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem("hodge", nel, r)
    bb = lambda t: t * (1 - t)
    u = lambda X: np.stack([bb(X[:, 1]) * bb(X[:, 2]), bb(X[:, 0]) * bb(X[:, 2]), bb(X[:, 0]) * bb(X[:, 1])], 1)
    f = lambda X: 2 * np.stack([bb(X[:, 1]) + bb(X[:, 2]), bb(X[:, 0]) + bb(X[:, 2]), bb(X[:, 0]) + bb(X[:, 1])], 1)
    rhs = P.rhs(f)
    x = torch.empty(rhs.size, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.rtol = 1e-13
    gym.gym_solve(op, opts, 1, _t(rhs), x)
    sig, uh = P.split(x.cpu().numpy())
    mesh_o = Mesh(synth.uniform_vertices(nel))
    assert np.abs(uh - assembly.de_rham(P.s1, mesh_o, u)).max() < 1e-10
    assert np.abs(sig).max() < 1e-10
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


def test_errors_are_reported(g):
    gym, ctx = g
    with pytest.raises(gym.GymError):
        gym.gym_mesh_create(ctx, 4, (2, 2, 2))
    mesh = _mesh(gym, ctx, (2, 2, 2))
    with pytest.raises(gym.GymError):
        gym.gym_space_create(ctx, mesh, 0, 9, 0)
    s0 = gym.gym_space_create(ctx, mesh, 0, 1, 0)
    s2 = gym.gym_space_create(ctx, mesh, 2, 1, 0)
    x = torch.zeros(100, dtype=torch.float64, device=DEV)
    with pytest.raises(gym.GymError):
        gym.gym_d_apply(s0, s2, 0, x, x)   # not consecutive in the complex
    bad = synth.uniform_vertices((2, 2, 2))
    bad[1, 1, 1] = [2.0, 2.0, 2.0]          # folds the cells
    with pytest.raises(gym.GymError):
        gym.gym_mesh_create(ctx, 3, (2, 2, 2), vertices=bad)


# ---- curved (perturbed, non-affine) cells -----------------------------------------
CURVED_MASS = [("H1", (5, 4, 6), 1), ("HCURL", (4, 5, 3), 2), ("HDIV", (3, 4, 5), 3), ("L2", (4, 3, 4), 2),
               ("HCURL", (3, 3, 4), 3), ("HDIV", (6, 5, 4), 1), ("H1", (3, 4, 3), 4)]


@pytest.mark.parametrize("tile", [1, 2], ids=["large", "small"])
@pytest.mark.parametrize("kind,nel,r", CURVED_MASS)
def test_mass_apply_curved(g, tile, kind, nel, r):
    gym, ctx = g
    gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, tile)
    verts = synth.perturbed_vertices(nel, 0.15, seed=21)
    mesh = gym.gym_mesh_create(ctx, 3, nel, vertices=verts)
    sp = gym.gym_space_create(ctx, mesh, KINDS[kind], r, 0)
    so = Space(kind, nel, r)
    M = assembly.mass_matrix(so, Mesh(verts))
    x = synth.random_vector(so.ndofs, seed=4, nrhs=2)
    y = torch.empty(2 * so.ndofs, dtype=torch.float64, device=DEV)
    gym.gym_mass_apply(sp, gym.GYM_F64, 2, _t(x), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().reshape(2, -1)
    for k in range(2):
        assert _rel(got[k], M @ x.reshape(2, -1)[k]) < 1e-13
    gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, 0)
    gym.gym_space_destroy(sp)
    gym.gym_mesh_destroy(mesh)


CURVED_OPS = [("hodge", (5, 4, 4), 1), ("hodge", (4, 5, 3), 2), ("hodge", (3, 3, 4), 3),
              ("poisson", (5, 4, 4), 1), ("poisson", (4, 3, 5), 2), ("poisson", (3, 4, 3), 4)]


@pytest.mark.parametrize("tile", [1, 2], ids=["large", "small"])
@pytest.mark.parametrize("which,nel,r", CURVED_OPS)
def test_operator_apply_curved(g, tile, which, nel, r):
    gym, ctx = g
    gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, tile)
    verts = synth.perturbed_vertices(nel, 0.15, seed=8)
    mesh = gym.gym_mesh_create(ctx, 3, nel, vertices=verts)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    mo = Mesh(verts)
    P = problems.MixedPoisson(mo, r) if which == "poisson" else problems.Hodge1(mo, r)
    n = gym.gym_op_ndofs(op)
    x = synth.random_vector(n, seed=6, nrhs=2)
    y = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    gym.gym_op_apply(op, gym.GYM_F64, 2, _t(x), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().reshape(2, -1)
    for k in range(2):
        assert _rel(got[k], P.A @ x.reshape(2, -1)[k]) < 1e-13, f"rhs {k}"
    y32 = torch.empty(2 * n, dtype=torch.float32, device=DEV)
    gym.gym_op_apply(op, gym.GYM_F32, 2, torch.tensor(x, dtype=torch.float32, device=DEV), y32)
    torch.cuda.synchronize()
    assert _rel(y32.cpu().numpy().reshape(2, -1)[1].astype(np.float64), P.A @ x.reshape(2, -1)[1]) < 5e-5
    gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, 0)
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


@pytest.mark.parametrize("mode", ["f64", "ir_f32"])
def test_solve_curved_hodge(g, mode):
    gym, ctx = g
    nel, r = (3, 4, 3), 3
    verts = synth.perturbed_vertices(nel, 0.15, seed=0)
    mesh = gym.gym_mesh_create(ctx, 3, nel, vertices=verts)
    op = gym.gym_op_create(ctx, gym.GYM_HODGE1, mesh, r)
    P = problems.Hodge1(Mesh(verts), r)
    n = P.A.shape[0]
    nrhs = 3
    b = synth.random_vector(n, seed=31, nrhs=nrhs)
    x = torch.empty(nrhs * n, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.rtol = 1e-13 if mode == "f64" else 1e-12
    if mode == "ir_f32":
        opts.mode = gym.GYM_MODE_IR_F32
    info = gym.gym_solve(op, opts, nrhs, _t(b), x)
    got = x.cpu().numpy().reshape(nrhs, -1)
    tol = 1e-10 if mode == "f64" else 1e-8
    for k in range(nrhs):
        ref = problems.solve_direct(P.A, b.reshape(nrhs, -1)[k])
        err = np.linalg.norm(got[k] - ref) / np.linalg.norm(ref)
        assert err < tol, f"rhs {k}: {err} (iters {info.iters}, outer {info.outer_iters})"
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


# Whole-CU tiles run 512, 768 or 1024 threads per workgroup depending on the
# problem, degree and form; the fused MINRES step sums partials over the
# workgroup, so every width is exercised in a solve (automatic tiling would
# pick small tiles on these meshes).
WIDE_CASES = [("poisson", (5, 4, 6), 1, 0.0, "f64"),    # 512 threads
              ("hodge", (4, 5, 3), 2, 0.0, "f64"),      # Kronecker, 1024
              ("hodge", (3, 4, 3), 3, 0.0, "f64"),      # Kronecker Hodge r = 3, 768
              ("hodge", (4, 3, 4), 2, 0.15, "f64"),     # curved, 768
              ("hodge", (4, 5, 3), 2, 0.0, "ir_f32")]   # FP32 Kronecker r = 2, 768


@pytest.mark.parametrize("which,nel,r,perturb,mode", WIDE_CASES)
def test_solve_whole_cu_tiles(g, which, nel, r, perturb, mode):
    gym, ctx = g
    verts = synth.perturbed_vertices(nel, perturb, seed=2) if perturb else None
    mesh = gym.gym_mesh_create(ctx, 3, nel, vertices=verts)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    vo = verts if perturb else synth.uniform_vertices(nel)
    P = problems.Hodge1(Mesh(vo), r) if which == "hodge" else problems.MixedPoisson(Mesh(vo), r)
    n = P.A.shape[0]
    b = synth.random_vector(n, seed=41, nrhs=2)
    x = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.rtol = 1e-13 if mode == "f64" else 1e-12
    if mode == "ir_f32":
        opts.mode = gym.GYM_MODE_IR_F32
    gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, 1)
    try:
        info = gym.gym_solve(op, opts, 2, _t(b), x)
    finally:
        gym.gym_ctx_set(ctx, gym.GYM_OPT_TILE, 0)
    got = x.cpu().numpy().reshape(2, -1)
    tol = 1e-10 if mode == "f64" else 1e-8
    for k in range(2):
        ref = problems.solve_direct(P.A, b.reshape(2, -1)[k])
        err = np.linalg.norm(got[k] - ref) / np.linalg.norm(ref)
        assert err < tol, f"rhs {k}: {err} (iters {info.iters})"
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


@pytest.mark.parametrize("curved", [False, True], ids=["affine", "curved"])
def test_mass_solve_and_exact_feec_operator(g, curved):
    # K a = M1^{-1} C^T M2 C a, the exact-FEEC curl-of-curl of section 3,
    # composed from incidence, mass apply and the CG mass solve.
    import scipy.sparse.linalg as spla
    gym, ctx = g
    nel, r = (4, 3, 5), 2
    verts = synth.perturbed_vertices(nel, 0.15, seed=3) if curved else synth.uniform_vertices(nel)
    mesh = gym.gym_mesh_create(ctx, 3, nel, vertices=verts if curved else None)
    s1 = gym.gym_space_create(ctx, mesh, gym.GYM_HCURL, r, 0)
    s2 = gym.gym_space_create(ctx, mesh, gym.GYM_HDIV, r, 0)
    o1, o2 = Space("HCURL", nel, r), Space("HDIV", nel, r)
    mo = Mesh(verts)
    M1 = assembly.mass_matrix(o1, mo).tocsc()
    M2 = assembly.mass_matrix(o2, mo)
    C = incidence.curl(o1, o2).astype(np.float64)
    opts = gym.gym_solve_opts_default()
    opts.rtol = 1e-13
    b = synth.random_vector(o1.ndofs, seed=2, nrhs=2)
    x = torch.empty(2 * o1.ndofs, dtype=torch.float64, device=DEV)
    info = gym.gym_mass_solve(s1, opts, 2, _t(b), x)
    assert info.status == 0 and info.rel_res < 1e-13
    for k in range(2):
        ref = spla.spsolve(M1, b.reshape(2, -1)[k])
        assert np.linalg.norm(x.cpu().numpy().reshape(2, -1)[k] - ref) / np.linalg.norm(ref) < 1e-11
    a = _t(synth.random_vector(o1.ndofs, seed=9))
    ca = torch.empty(o2.ndofs, dtype=torch.float64, device=DEV)
    mca = torch.empty_like(ca)
    p2a = torch.empty_like(a)
    ka = torch.empty_like(a)
    gym.gym_d_apply(s1, s2, 0, a, ca)
    gym.gym_mass_apply(s2, gym.GYM_F64, 1, ca, mca)
    gym.gym_d_apply(s1, s2, 1, mca, p2a)
    gym.gym_mass_solve(s1, opts, 1, p2a, ka)
    an = a.cpu().numpy()
    ref = spla.spsolve(M1, C.T @ (M2 @ (C @ an)))
    assert np.linalg.norm(ka.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-10
    for s in (s1, s2):
        gym.gym_space_destroy(s)
    gym.gym_mesh_destroy(mesh)


# ---- BF16 contraction operands (FP32 accumulate), inside FP64 refinement ----------
@pytest.mark.parametrize("which,nel,r", [("poisson", (4, 5, 3), 4), ("hodge", (5, 4, 4), 2), ("poisson", (9, 7), 2),
                                         ("hodge", (3, 4, 3), 3)])
def test_operator_apply_bf16(g, which, nel, r):
    # every contraction operand is rounded to bf16 (8 significant bits), so
    # the apply differs from FP64 by a few bf16 ulps of the output scale:
    # well above FP32 round-off, well below 5e-2
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem(which, nel, r)
    n = P.A.shape[0]
    x = synth.random_vector(n, seed=13)
    y = torch.empty(n, dtype=torch.float32, device=DEV)
    gym.gym_op_apply(op, gym.GYM_BF16, 1, torch.tensor(x, dtype=torch.float32, device=DEV), y)
    torch.cuda.synchronize()
    err = _rel(y.cpu().numpy().astype(np.float64), P.A @ x)
    assert 1e-5 < err < 5e-2, err
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


@pytest.mark.parametrize("nel,r", [((4, 5, 3), 4), ((3, 2, 4), 3), ((5, 3, 3), 4)])
def test_poisson_bf16_matrix_core_apply_error_bound(g, nel, r):
    # Mixed Poisson at degree >= 3 applies each element operator
    # A_e = [[M2_e, B_e^T], [B_e, 0]], B_e = -M3_e D_e, as one bf16 product with
    # FP32 accumulation, then sums at most two element results per unknown in
    # FP32.  Entries of A_e and of x are rounded to bf16 (unit round-off
    # u = 2^-8), so per output row
    #   |y - A x|_i <= (2 u + u^2 + 2 * 2^-24 K) (sum_e P_e^T |A_e| |P_e x|)_i,
    # K the element row length.  Checked row by row with the oracle's element
    # matrices (x rounded to FP32 first, as the caller passes it).
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON, mesh, r)
    P = _oracle_problem("poisson", nel, r)
    n = P.A.shape[0]
    x32 = synth.random_vector(n, seed=13).astype(np.float32)
    y = torch.empty(n, dtype=torch.float32, device=DEV)
    gym.gym_op_apply(op, gym.GYM_BF16, 1, torch.tensor(x32, device=DEV), y)
    torch.cuda.synchronize()
    x = x32.astype(np.float64)
    M = P.mesh
    m2 = assembly.local_mass(P.sdiv, M)
    m3 = assembly.local_mass(P.sl2, M)
    ei = M.element_multi_index()
    dd = P.sdiv.element_dofs(ei)
    dc = P.sl2.element_dofs(ei)
    D = P.D.tocsr()
    bound_vec = np.zeros(n)
    ns = P.sdiv.ndofs
    for e in range(dd.shape[0]):
        Be = -m3[e] @ D[dc[e]][:, dd[e]].toarray()
        xs, xp = np.abs(x[dd[e]]), np.abs(x[ns + dc[e]])
        bound_vec[dd[e]] += np.abs(m2[e]) @ xs + np.abs(Be.T) @ xp
        bound_vec[ns + dc[e]] += np.abs(Be) @ xs
    K = 3 * (r + 1) * r * r + r ** 3
    u = 2.0 ** -8
    tol = (2 * u + u * u + 2 * 2.0 ** -24 * K) * bound_vec + 1e-30
    err = np.abs(y.cpu().numpy().astype(np.float64) - P.A @ x)
    ratio = (err / tol).max()
    print(f"nel={nel} r={r}: max |y - Ax| / bound = {ratio:.3f}, rel err {_rel(y.cpu().numpy(), P.A @ x):.2e}",
          flush=True)
    assert ratio <= 1.0
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


@pytest.mark.parametrize("which,nel,r", [("poisson", (4, 4, 3), 3), ("hodge", (4, 3, 4), 2)])
def test_solve_mixed_precision_bf16(g, which, nel, r):
    gym, ctx = g
    mesh = _mesh(gym, ctx, nel)
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON if which == "poisson" else gym.GYM_HODGE1, mesh, r)
    P = _oracle_problem(which, nel, r)
    n = P.A.shape[0]
    b = synth.random_vector(n, seed=17, nrhs=2)
    x = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    opts = gym.gym_solve_opts_default()
    opts.mode = gym.GYM_MODE_IR_BF16
    opts.rtol = 1e-12
    opts.inner_rtol = 1e-2
    opts.max_outer = 60
    info = gym.gym_solve(op, opts, 2, _t(b), x)
    assert info.status == 0, (info.rel_res, info.outer_iters)
    got = x.cpu().numpy().reshape(2, -1)
    for k in range(2):
        ref = problems.solve_direct(P.A, b.reshape(2, -1)[k])
        err = np.linalg.norm(got[k] - ref) / np.linalg.norm(ref)
        assert err < 1e-8, (k, err, info.outer_iters, info.iters)
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)
