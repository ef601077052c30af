"""Thin ctypes binding of the gym C ABI (include/gym.h).

Argument marshalling only: every call goes straight to ``lib/libgym.so``,
whose HIP kernels do all the work.  Functions carry the C names; device
vectors are passed as torch tensors (their ``data_ptr()``) and streams as
``torch.cuda.Stream`` objects or raw handles.  There is no fallback: if the
library is missing, :func:`lib` raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libgym.so")

GYM_OK = 0
GYM_W_NOT_CONVERGED = 1
GYM_E_ARG = -1
GYM_E_OOM = -2
GYM_E_HIP = -3
GYM_E_INVALID_MESH = -4
GYM_E_BREAKDOWN = -5
GYM_E_UNSUPPORTED = -6

GYM_H1, GYM_HCURL, GYM_HDIV, GYM_L2 = 0, 1, 2, 3
GYM_BC_NATURAL, GYM_BC_ESSENTIAL = 0, 1
GYM_F64, GYM_F32, GYM_BF16 = 0, 1, 2
GYM_MIXED_POISSON, GYM_HODGE1 = 0, 1
GYM_MINRES, GYM_CG = 0, 1
GYM_MODE_F64, GYM_MODE_IR_F32, GYM_MODE_IR_BF16 = 0, 1, 2
GYM_PRECOND_JACOBI, GYM_PRECOND_NONE, GYM_PRECOND_SCHUR = 0, 1, 2
GYM_Q1_EXACT, GYM_Q1_LUMPED, GYM_Q1_SPAI_DIAG, GYM_Q1_SPAI, GYM_Q1_SPAI_OP = 0, 1, 2, 3, 4
GYM_M2_EXACT, GYM_M2_LUMPED = 0, 1

KIND = {"H1": GYM_H1, "HCURL": GYM_HCURL, "HDIV": GYM_HDIV, "L2": GYM_L2}


class GymError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gym status {status}: {msg}")
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("mode", ctypes.c_int), ("rtol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("check_every", ctypes.c_int), ("timing", ctypes.c_int), ("precond", ctypes.c_int)]


class Layout(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dim", ctypes.c_int), ("degree", ctypes.c_int), ("bc", ctypes.c_int),
                ("ncomp", ctypes.c_int), ("nodal_mask", ctypes.c_int * 3), ("m", ctypes.c_int64 * 3),
                ("start", (ctypes.c_int64 * 3) * 3), ("count", (ctypes.c_int64 * 3) * 3),
                ("offset", ctypes.c_int64 * 3), ("ndofs", ctypes.c_int64)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("seconds", ctypes.c_double), ("applies", ctypes.c_int),
                ("apply_ms", ctypes.c_double)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("mem_budget", ctypes.c_int64), ("max_slots", ctypes.c_int),
                ("rtol", ctypes.c_double), ("maxit", ctypes.c_int), ("precond", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int), ("nel", ctypes.c_int), ("degree", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("rhs", ctypes.POINTER(ctypes.c_double)),
                ("want_solution", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("latency_s", ctypes.c_double), ("ndofs", ctypes.c_int64)]


class MaxwellOpts(ctypes.Structure):
    _fields_ = [("q1", ctypes.c_int), ("m2", ctypes.c_int), ("c", ctypes.c_double), ("cg_rtol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int)]


class EigOpts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int), ("largest", ctypes.c_int), ("block", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("grad_shift", ctypes.c_double), ("seed", ctypes.c_uint64)]


class EigInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("max_resid", ctypes.c_double),
                ("gradient_modes", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
# name -> (restype, argtypes); the full exported surface of include/gym.h
SIGNATURES = {
    "gym_create": (_I, [ctypes.POINTER(_P), _I]),
    "gym_destroy": (_I, [_P]),
    "gym_last_error": (ctypes.c_char_p, []),
    "gym_ctx_set": (_I, [_P, _I, _I]),
    "gym_mesh_create": (_I, [_P, _I, ctypes.POINTER(_I64), _P, _P, _P, ctypes.POINTER(_P)]),
    "gym_mesh_structured": (_I, [_P, _I, ctypes.POINTER(_I64), _P, _P, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.POINTER(_P)]),
    "gym_mesh_vertices": (_I, [_P, _P]),
    "gym_mesh_set_periodic": (_I, [_P, _I]),
    "gym_mesh_destroy": (_I, [_P]),
    "gym_space_create": (_I, [_P, _P, _I, _I, _I, ctypes.POINTER(_P)]),
    "gym_space_ndofs": (_I64, [_P]),
    "gym_space_destroy": (_I, [_P]),
    "gym_space_layout": (_I, [_P, ctypes.POINTER(Layout)]),
    "gym_d_apply": (_I, [_P, _P, _I, _P, _P, _P]),
    "gym_mass_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "gym_op_create": (_I, [_P, _I, _P, _I, ctypes.POINTER(_P)]),
    "gym_op_ndofs": (_I64, [_P]),
    "gym_op_block_sizes": (_I, [_P, ctypes.POINTER(_I64)]),
    "gym_op_destroy": (_I, [_P]),
    "gym_op_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "gym_op_precond_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "gym_op_precond_diag": (_I, [_P, _P, _P]),
    "gym_rhs_manufactured": (_I, [_P, _I, _P, _P, _P, _P]),
    "gym_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "gym_solve": (_I, [_P, ctypes.POINTER(SolveOpts), _I, _P, _P, ctypes.POINTER(SolveInfo), _P]),
    "gym_solve_noalloc": (_I, [_P, ctypes.POINTER(SolveOpts), _I, _P, _P, ctypes.POINTER(SolveInfo), _P]),
    "gym_mass_solve": (_I, [_P, ctypes.POINTER(SolveOpts), _I, _P, _P, ctypes.POINTER(SolveInfo), _P]),
    "gym_serve_start": (_I, [ctypes.POINTER(ServeOpts), ctypes.POINTER(_P)]),
    "gym_serve_submit": (_I, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "gym_serve_poll": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(Result), _P]),
    "gym_serve_stop": (_I, [_P]),
    "gym_maxwell_opts_default": (None, [ctypes.POINTER(MaxwellOpts)]),
    "gym_maxwell_create": (_I, [_P, _P, _I, ctypes.POINTER(MaxwellOpts), ctypes.POINTER(_P)]),
    "gym_maxwell_ndofs": (_I64, [_P]),
    "gym_maxwell_step": (_I, [_P, ctypes.c_double, _I, _P, _P, _P]),
    "gym_maxwell_energy": (_I, [_P, _P, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "gym_maxwell_destroy": (_I, [_P]),
    "gym_maxwell_spai_op": (_I, [_P, _I, _P, ctypes.c_double, ctypes.c_double, _I, ctypes.POINTER(_I),
                                ctypes.POINTER(ctypes.c_double), _P]),
    "gym_eig_opts_default": (None, [ctypes.POINTER(EigOpts)]),
    "gym_maxwell_eigs": (_I, [_P, ctypes.POINTER(EigOpts), ctypes.POINTER(ctypes.c_double), _P,
                             ctypes.POINTER(EigInfo), _P]),
}

_lib = None


def lib():
    """Load libgym.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2301_01753_amd.build")
        # torch ships its own HIP runtime under the same soname as the one
        # libgym links.  Loaded first, torch's copy serves both; loaded after
        # libgym it would start a second runtime that finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, ok=(GYM_OK,)):
    if status not in ok:
        msg = lib().gym_last_error().decode()
        raise GymError(status, msg)
    return status


def _ptr(t):
    """Device pointer of a torch tensor (or an int / None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ---- thin wrappers, one per C entry point ----------------------------------
def gym_create(device=0):
    h = _P()
    _check(lib().gym_create(ctypes.byref(h), device))
    return h


def gym_destroy(ctx):
    _check(lib().gym_destroy(ctx))


GYM_OPT_MASS_FORM, GYM_OPT_TILE, GYM_OPT_CURVED_KERNEL = 0, 1, 2


def gym_ctx_set(ctx, option, value):
    _check(lib().gym_ctx_set(ctx, option, value))


def gym_mesh_create(ctx, dim, nel, vertices=None, lo=None, hi=None):
    def pad3(v, fill):
        v = list(v)[:3]
        return v + [fill] * (3 - len(v))
    n = (_I64 * 3)(*pad3(nel, 1))
    lo_a = (ctypes.c_double * 3)(*pad3(lo if lo is not None else [0.0] * 3, 0.0))
    hi_a = (ctypes.c_double * 3)(*pad3(hi if hi is not None else [1.0] * 3, 1.0))
    vp = None
    if vertices is not None and dim in (2, 3):
        v = np.ascontiguousarray(np.asarray(vertices, dtype=np.float64))
        # vertex (i, j, k) at ((k*(ny+1) + j)*(nx+1) + i)*dim: axis 0 fastest
        v = np.ascontiguousarray(np.transpose(v, list(range(dim))[::-1] + [dim]))
        vp = v.ctypes.data_as(_P)
    h = _P()
    _check(lib().gym_mesh_create(ctx, dim, n, vp, ctypes.cast(lo_a, _P), ctypes.cast(hi_a, _P), ctypes.byref(h)))
    return h


def gym_mesh_structured(ctx, dim, nel, perturb_frac=0.0, seed=0, lo=None, hi=None):
    """Box mesh with the library's seeded vertex perturbation (gym.h)."""
    def pad3(v, fill):
        v = list(v)[:3]
        return v + [fill] * (3 - len(v))
    n = (_I64 * 3)(*pad3(nel, 1))
    lo_a = (ctypes.c_double * 3)(*pad3(lo if lo is not None else [0.0] * 3, 0.0))
    hi_a = (ctypes.c_double * 3)(*pad3(hi if hi is not None else [1.0] * 3, 1.0))
    h = _P()
    _check(lib().gym_mesh_structured(ctx, dim, n, ctypes.cast(lo_a, _P), ctypes.cast(hi_a, _P), float(perturb_frac),
                                     ctypes.c_uint64(seed), ctypes.byref(h)))
    return h


def gym_mesh_set_periodic(mesh, mask):
    """Axes in mask (bit a: axis a) become periodic (gym.h)."""
    _check(lib().gym_mesh_set_periodic(mesh, int(mask)))


def gym_mesh_vertices(mesh, nel):
    """Vertex coordinates as an array (N_1+1, ..., N_d+1, d), axis 0 first
    (the layout synth.uniform_vertices returns)."""
    dim = len(nel)
    shape = [int(n) + 1 for n in nel][::-1] + [dim]
    v = np.empty(shape, dtype=np.float64)
    _check(lib().gym_mesh_vertices(mesh, v.ctypes.data_as(_P)))
    return np.ascontiguousarray(np.transpose(v, list(range(dim))[::-1] + [dim]))


def gym_mesh_destroy(mesh):
    _check(lib().gym_mesh_destroy(mesh))


def gym_space_create(ctx, mesh, kind, degree, bc=GYM_BC_NATURAL):
    if isinstance(kind, str):
        kind = KIND[kind]
    h = _P()
    _check(lib().gym_space_create(ctx, mesh, kind, degree, bc, ctypes.byref(h)))
    return h


def gym_space_ndofs(space):
    return int(lib().gym_space_ndofs(space))


def gym_space_layout(space):
    L = Layout()
    _check(lib().gym_space_layout(space, ctypes.byref(L)))
    return L


def gym_space_destroy(space):
    _check(lib().gym_space_destroy(space))


def gym_d_apply(src, dst, transpose, x, y, stream=None):
    _check(lib().gym_d_apply(src, dst, int(transpose), _ptr(x), _ptr(y), _stream(stream)))


def gym_mass_apply(space, prec, nrhs, x, y, stream=None):
    _check(lib().gym_mass_apply(space, prec, nrhs, _ptr(x), _ptr(y), _stream(stream)))


def gym_op_create(ctx, problem, mesh, degree):
    h = _P()
    _check(lib().gym_op_create(ctx, problem, mesh, degree, ctypes.byref(h)))
    return h


def gym_op_ndofs(op):
    return int(lib().gym_op_ndofs(op))


def gym_op_block_sizes(op):
    n = (_I64 * 2)()
    _check(lib().gym_op_block_sizes(op, n))
    return int(n[0]), int(n[1])


def gym_op_destroy(op):
    _check(lib().gym_op_destroy(op))


def gym_op_apply(op, prec, nrhs, x, y, stream=None):
    _check(lib().gym_op_apply(op, prec, nrhs, _ptr(x), _ptr(y), _stream(stream)))


def gym_op_precond_apply(op, precond, nrhs, y, z, stream=None):
    _check(lib().gym_op_precond_apply(op, precond, nrhs, _ptr(y), _ptr(z), _stream(stream)))


def gym_op_precond_diag(op, diag, stream=None):
    _check(lib().gym_op_precond_diag(op, _ptr(diag), _stream(stream)))


def gym_rhs_manufactured(op, modes, coeffs, b, stream=None):
    m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    _check(lib().gym_rhs_manufactured(op, int(m.shape[0]), m.ctypes.data_as(_P), c.ctypes.data_as(_P),
                                      _ptr(b), _stream(stream)))


def gym_solve_opts_default():
    o = SolveOpts()
    lib().gym_solve_opts_default(ctypes.byref(o))
    return o


def gym_solve(op, opts, nrhs, b, x, stream=None):
    info = SolveInfo()
    st = lib().gym_solve(op, ctypes.byref(opts), nrhs, _ptr(b), _ptr(x), ctypes.byref(info), _stream(stream))
    _check(st, ok=(GYM_OK, GYM_W_NOT_CONVERGED))
    return info


def gym_solve_noalloc(op, opts, nrhs, b, x, stream=None):
    info = SolveInfo()
    st = lib().gym_solve_noalloc(op, ctypes.byref(opts), nrhs, _ptr(b), _ptr(x), ctypes.byref(info),
                                 _stream(stream))
    _check(st, ok=(GYM_OK, GYM_W_NOT_CONVERGED))
    return info


def gym_mass_solve(space, opts, nrhs, b, x, stream=None):
    info = SolveInfo()
    st = lib().gym_mass_solve(space, ctypes.byref(opts), nrhs, _ptr(b), _ptr(x), ctypes.byref(info),
                              _stream(stream))
    _check(st, ok=(GYM_OK, GYM_W_NOT_CONVERGED))
    return info


def gym_maxwell_opts_default():
    o = MaxwellOpts()
    lib().gym_maxwell_opts_default(ctypes.byref(o))
    return o


def gym_maxwell_create(ctx, mesh, degree, opts=None):
    h = _P()
    _check(lib().gym_maxwell_create(ctx, mesh, degree, ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(h)))
    return h


def gym_maxwell_ndofs(mx):
    return int(lib().gym_maxwell_ndofs(mx))


def gym_maxwell_step(mx, tau, nsteps, a, e, stream=None):
    st = lib().gym_maxwell_step(mx, float(tau), int(nsteps), _ptr(a), _ptr(e), _stream(stream))
    _check(st, ok=(GYM_OK, GYM_W_NOT_CONVERGED))
    return st


def gym_maxwell_energy(mx, a, e, stream=None):
    h = ctypes.c_double()
    st = lib().gym_maxwell_energy(mx, _ptr(a), _ptr(e), ctypes.byref(h), _stream(stream))
    _check(st, ok=(GYM_OK, GYM_W_NOT_CONVERGED))
    return h.value


def gym_maxwell_destroy(mx):
    _check(lib().gym_maxwell_destroy(mx))


def gym_maxwell_spai_op(mx, probes, lam, rtol=1e-12, maxit=5000, stream=None):
    """Replace Q1 by SPAI-OP with the modes `probes` (device tensor of
    nprobe x ndofs doubles, or None); returns (iterations, rel_res, status)."""
    n = gym_maxwell_ndofs(mx)
    npb = 0 if probes is None else probes.numel() // n
    it = ctypes.c_int()
    rel = ctypes.c_double()
    st = lib().gym_maxwell_spai_op(mx, npb, _ptr(probes), float(lam), float(rtol), int(maxit), ctypes.byref(it),
                                   ctypes.byref(rel), _stream(stream))
    _check(st, ok=(GYM_OK, GYM_W_NOT_CONVERGED))
    return it.value, rel.value, st


def gym_eig_opts_default():
    o = EigOpts()
    lib().gym_eig_opts_default(ctypes.byref(o))
    return o


def gym_maxwell_eigs(mx, opts=None, vecs=None, stream=None):
    """Lowest non-kernel (or, with opts.largest, the largest) omega^2 of Q1 P2:
    returns (omega2 numpy array, EigInfo, status); `vecs`, if given, is a device
    tensor of nev x ndofs doubles."""
    o = opts if opts is not None else gym_eig_opts_default()
    w = np.zeros(o.nev, dtype=np.float64)
    info = EigInfo()
    st = lib().gym_maxwell_eigs(mx, ctypes.byref(o), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                _ptr(vecs) if vecs is not None else None, ctypes.byref(info), _stream(stream))
    _check(st, ok=(GYM_OK, GYM_W_NOT_CONVERGED))
    return w, info, st


def gym_serve_start(opts):
    h = _P()
    _check(lib().gym_serve_start(ctypes.byref(opts), ctypes.byref(h)))
    return h


def gym_serve_submit(srv, req):
    rid = ctypes.c_uint64()
    _check(lib().gym_serve_submit(srv, ctypes.byref(req), ctypes.byref(rid)))
    return int(rid.value)


def gym_serve_poll(srv, rid, x_host=None):
    res = Result()
    xp = None if x_host is None else x_host.ctypes.data_as(_P)
    st = lib().gym_serve_poll(srv, rid, ctypes.byref(res), xp)
    _check(st, ok=(0, 2))
    return st, res


def gym_serve_stop(srv):
    _check(lib().gym_serve_stop(srv))
