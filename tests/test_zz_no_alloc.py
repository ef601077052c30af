"""gym_solve_noalloc (the FP64 solve whose workspace is a static device array)
against gym_solve on the same operator and right-hand sides, through the C
ABI: two calls in a row, the second on a smaller problem, each must give
gym_solve's solution (same kernels, same order: bit for bit) and its status;
and a problem larger than the array is refused with GYM_E_ARG."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def g():
    from paper_2301_01753_amd import gym
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = gym.gym_create(0)
    yield gym, ctx
    gym.gym_destroy(ctx)


def _solve_both(gym, ctx, problem, nel, r, nrhs, seed, precond):
    mesh = gym.gym_mesh_create(ctx, 3, nel)
    op = gym.gym_op_create(ctx, problem, mesh, r)
    n = gym.gym_op_ndofs(op)
    b = torch.tensor(synth.random_vector(n, seed=seed, nrhs=nrhs), device=DEV)
    o = gym.gym_solve_opts_default()
    o.rtol = 1e-10
    o.precond = precond
    x_ref = torch.empty_like(b)
    x_na = torch.full_like(b, float("nan"))
    i_ref = gym.gym_solve(op, o, nrhs, b, x_ref)
    i_na = gym.gym_solve_noalloc(op, o, nrhs, b, x_na)
    torch.cuda.synchronize()
    out = (x_ref.cpu().numpy(), x_na.cpu().numpy(), i_ref, i_na)
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)
    return out


def test_noalloc_solve_matches_gym_solve_twice(g):
    gym, ctx = g
    cases = [(gym.GYM_HODGE1, (6, 5, 4), 2, 2, 3, gym.GYM_PRECOND_JACOBI),
             (gym.GYM_MIXED_POISSON, (3, 4, 2), 1, 1, 4, gym.GYM_PRECOND_NONE)]
    for problem, nel, r, nrhs, seed, pre in cases:
        xr, xn, ir, ina = _solve_both(gym, ctx, problem, nel, r, nrhs, seed, pre)
        print(f"nel={nel} r={r} nrhs={nrhs}: {ir.iters} / {ina.iters} iterations, "
              f"rel_res {ir.rel_res:.2e} / {ina.rel_res:.2e}", flush=True)
        assert ina.status == ir.status == gym.GYM_OK
        assert ina.iters == ir.iters
        assert np.array_equal(xn, xr)
        assert ina.rel_res == ir.rel_res <= 1e-10


def test_noalloc_solve_refuses_oversize(g):
    gym, ctx = g
    # 1,012,095 unknowns x 2 rhs: about 180 MB of workspace
    mesh = gym.gym_mesh_create(ctx, 3, (32, 32, 32))
    op = gym.gym_op_create(ctx, gym.GYM_HODGE1, mesh, 2)
    n = gym.gym_op_ndofs(op)
    b = torch.zeros(2 * n, dtype=torch.float64, device=DEV)
    x = torch.empty_like(b)
    o = gym.gym_solve_opts_default()
    with pytest.raises(gym.GymError) as e:
        gym.gym_solve_noalloc(op, o, 2, b, x)
    assert e.value.status == gym.GYM_E_ARG and "too large" in str(e.value)
    o.mode = gym.GYM_MODE_IR_F32
    with pytest.raises(gym.GymError) as e:
        gym.gym_solve_noalloc(op, o, 1, b, x)
    assert e.value.status == gym.GYM_E_UNSUPPORTED
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)
