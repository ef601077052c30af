"""Benchmark of the matrix-free FEEC hot path on one MI355X.

Headline workload: the unit cube, 96^3 hexahedra with seeded vertex
perturbations (+-15% of h per coordinate, multilinear cells, so every cell has
its own Jacobian field), degree-3 Hodge Laplacian on 1-forms (sigma in H1_0,
u in H0(curl)), 8 right-hand sides per apply, FP64.  758.5 M unknowns per
apply (94.8 M per right-hand side).

A step is one FP64 operator apply y = A x of all 8 right-hand sides: per
cell, the sum-factorised contractions of the four mass terms (M0, M1 twice,
M2; the gradient and curl through the nodal-derivative tables) with the
Gauss-point metrics of the curved cells, the x and y contractions on the
matrix cores; the deterministic sums over shared positions (LDS within a
tile, a second kernel across tiles).  x is resident in HBM before the timed
region.

value = 8 x ndofs / (median HIP-event time of one apply), GDoF/s; the wall
time of the K timed applies gives ms_per_step.  Also reported (extras): the
FP32 apply of the same workload with its error against FP64; the 64^3
degree-4 mixed Poisson workload: applies per precision and whole solves to
relative residual 1e-8 in FP64 and in FP32 / bf16-operand refinement, each
with its error against the FP64 solution; the 32^3 degree-2 Hodge solves; the
serving loop; the time-stepping, eigen-solver and SPAI-OP rates.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "operator-apply GDoF/s and solves/s to 1e-8 rel. err: FP64 vs mixed vs batched"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6        # 256 CU x 64 FP64 FMA lanes x 2 x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3

HEAD_N, HEAD_R, HEAD_PERTURB, HEAD_NRHS = 96, 3, 0.15, 8


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def comp_flops(n, q):
    """Sum-factorised flops of one component: 3 forward contractions
    (coefficients -> Gauss points), 3 transposed ones, per element."""
    nx, ny, nz = n
    fwd = 2 * (q * ny * nz * nx + q * q * nz * ny + q ** 3 * nz)
    bwd = 2 * (q * q * nz * q + q * ny * nz * q + nx * ny * nz * q)
    return fwd + bwd


def kron_comp_flops(n):
    """Flops of one component in the Kronecker form M_x (x) M_y (x) M_z:
    three 1-D element-matrix contractions."""
    nx, ny, nz = n
    return 2 * nx * ny * nz * (nx + ny + nz)


def algorithmic_flops_per_element(problem, r, kron=False, metric=False):
    """Flops per element and right-hand side of one operator apply (no halo
    recomputation): the Gauss-point sum factorisation (q = r + 1), or the
    Kronecker form that the kernel evaluates on affine cells.  metric: add the
    pointwise metric at the q^3 Gauss points of curved cells, 1 flop per point
    for a scalar mass and 15 (symmetric 3x3 times a 3-vector) for a vector
    mass."""
    q, N, E = r + 1, r + 1, r
    f = kron_comp_flops if kron else (lambda n: comp_flops(n, q))
    h1 = f((N, N, N))
    hcurl = sum(f(tuple(E if a == c else N for a in range(3))) for c in range(3))
    hdiv = sum(f(tuple(N if a == c else E for a in range(3))) for c in range(3))
    l2 = f((E, E, E))
    pts = q ** 3 if metric else 0
    if problem == "hodge":
        return h1 + 2 * hcurl + hdiv + pts * (1 + 15 + 15 + 15)   # M0 sigma, M1 u, M1 G sigma, M2 C u
    return hdiv + 2 * l2 + pts * (15 + 1 + 1)                     # M2 s, M3 p, M3 D s


def cpu_baseline(N, r, nrhs, reps=20):
    """The CPU oracle on a bounded sample of the headline workload: the same
    perturbed-mesh recipe at N^3 cells, degree r, assembled by naive
    quadrature (not timed in the rate), then the median of `reps` sparse
    applies to nrhs right-hand sides, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import problems
    from oracle.lattice import Mesh

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        P = problems.Hodge1(Mesh(synth.perturbed_vertices_counter((N, N, N), HEAD_PERTURB, 0)), r)
        t_asm = time.perf_counter() - t0
        n = P.A.shape[0]
        X = np.asarray(synth.random_vector(n, seed=3, nrhs=nrhs).reshape(nrhs, n).T, order="F")
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            P.A @ X
            ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    return {
        "value": nrhs * n / t / 1e9,
        "unit": "GDoF/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"SciPy CSR apply of the assembled {N}^3 perturbed (15%) degree-{r} Hodge operator "
                   f"({n} DoFs, {P.A.nnz} nonzeros) to {nrhs} right-hand sides, median of {reps}: "
                   f"{t * 1e3:.2f} ms; assembly {t_asm:.1f} s not counted; 1 thread of {os.cpu_count()} host cores"),
    }


def event_times(fn, reps, warmup):
    """Run fn() warmup + reps times on the current stream; returns (per-call
    HIP-event ms list, wall seconds of the timed calls)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [a.elapsed_time(b) for a, b in ev], wall


def median(v):
    v = sorted(v)
    k = len(v)
    return 0.5 * (v[(k - 1) // 2] + v[k // 2])


def apply_rates(gym, op, n, nrhs, precs, reps, warmup, seed):
    """Median apply time per contraction precision and the relative error of
    each lower-precision apply against the FP64 apply of the same vector."""
    import torch
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    x = torch.randn(nrhs * n, dtype=torch.float64, device="cuda:0", generator=gen)
    y64 = torch.empty_like(x)
    out = {}
    for name, prec in precs:
        xi = x if prec == gym.GYM_F64 else x.float()
        yi = y64 if prec == gym.GYM_F64 else torch.empty_like(xi)
        ms, wall = event_times(lambda: gym.gym_op_apply(op, prec, nrhs, xi, yi), reps, warmup)
        t = median(ms)
        e = {"median_us": t * 1e3, "gdof_s": nrhs * n / t / 1e6, "applies": reps}
        if prec != gym.GYM_F64:
            e["rel_err_vs_f64_apply"] = float(torch.linalg.norm(yi.double() - y64) / torch.linalg.norm(y64))
        out[name] = e
        del yi
    del x, y64
    return out


def poisson64_solves(gym, ctx, rtol, modes, reps):
    """64^3 degree-4 mixed Poisson (67.3 M unknowns): whole solves from x = 0
    to relative residual `rtol` (true FP64 residual) in FP64 and in
    mixed-precision refinement, MINRES with the block preconditioner
    diag(diag(M2), M3 D diag(M2)^-1 D^T M3); each result's relative error
    against the FP64 solution.  Also the apply rates per precision and the
    preconditioner's own time."""
    import torch
    import synth
    mesh = gym.gym_mesh_create(ctx, 3, (64, 64, 64))
    op = gym.gym_op_create(ctx, gym.GYM_MIXED_POISSON, mesh, 4)
    n = gym.gym_op_ndofs(op)
    res = {"ndofs": n, "apply": apply_rates(gym, op, n, 1, (("f64", gym.GYM_F64), ("f32", gym.GYM_F32),
                                                            ("bf16", gym.GYM_BF16)), 50, 3, 11)}
    b = torch.empty(n, dtype=torch.float64, device="cuda:0")
    gym.gym_rhs_manufactured(op, synth.modes_3d(), synth.fourier_coeffs(0, 8, 1), b)
    zt = torch.empty_like(b)
    gym.gym_op_precond_apply(op, gym.GYM_PRECOND_SCHUR, 1, b, zt)  # set-up (host eigenproblems), not timed
    ms, _ = event_times(lambda: gym.gym_op_precond_apply(op, gym.GYM_PRECOND_SCHUR, 1, b, zt), 10, 1)
    res["schur_precond_apply_us"] = median(ms) * 1e3
    del zt
    x64 = None
    for name, mode, inner in modes:
        o = gym.gym_solve_opts_default()
        o.mode = mode
        o.rtol = rtol
        o.maxit = 200000
        o.inner_rtol = inner
        o.max_outer = 60
        o.check_every = 10
        o.precond = gym.GYM_PRECOND_SCHUR
        x = torch.empty_like(b)
        walls, infos = [], []
        for k in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            inf = gym.gym_solve(op, o, 1, b, x)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            infos.append(inf)
            log(f"  poisson 64^3 r4 {name} solve {k}: {inf.iters} it, {inf.outer_iters} outer, "
                f"rel_res {inf.rel_res:.2e}, {walls[-1]:.2f} s")
        e = {"solves_per_s": reps / sum(walls), "seconds_per_solve": sum(walls) / reps,
             "iters": infos[-1].iters, "outer_iters": infos[-1].outer_iters, "rel_res": infos[-1].rel_res,
             "status": infos[-1].status}
        if mode != gym.GYM_MODE_F64:
            e["inner_rtol"] = inner
        if x64 is None:
            x64 = x.clone()
        else:
            e["rel_err_vs_fp64_solve"] = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        res[name] = e
    f64 = res[modes[0][0]]["solves_per_s"]
    for name, _, _ in modes[1:]:
        res[name]["speedup_vs_fp64"] = res[name]["solves_per_s"] / f64
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)
    del b, x, x64
    torch.cuda.empty_cache()
    return res


def hodge32_solves(gym, ctx, steps, rtol):
    """32^3 degree-2 Hodge (1.01 M unknowns, manufactured 8-mode field): FP64
    solves to `rtol`, 8 right-hand sides per solve, and IR-FP32."""
    import torch
    import synth
    mesh = gym.gym_mesh_create(ctx, 3, (32, 32, 32))
    op = gym.gym_op_create(ctx, gym.GYM_HODGE1, mesh, 2)
    n = gym.gym_op_ndofs(op)
    b = torch.empty(n, dtype=torch.float64, device="cuda:0")
    gym.gym_rhs_manufactured(op, synth.modes_3d(), synth.fourier_coeffs(0, 8, 3), b)
    res = {"ndofs": n}

    def run(mode, nrhs, bv, k):
        o = gym.gym_solve_opts_default()
        o.rtol, o.mode, o.timing = rtol, mode, 16
        x = torch.empty_like(bv)
        gym.gym_solve(op, o, nrhs, bv, x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, ap, ms = 0, 0, 0.0
        for _ in range(k):
            inf = gym.gym_solve(op, o, nrhs, bv, x)
            its, ap, ms = its + inf.iters, ap + inf.applies, ms + inf.apply_ms
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return {"solves_per_s": nrhs * k / wall, "iters_per_solve": its / k, "rel_res": inf.rel_res,
                "gdof_s_in_solve": nrhs * n * its / wall / 1e9,
                "apply_us": ms / max(ap, 1) * 1e3}, x

    res["f64"], x64 = run(gym.GYM_MODE_F64, 1, b, steps)
    res["ir_f32"], x32 = run(gym.GYM_MODE_IR_F32, 1, b, max(1, steps // 2))
    res["ir_f32"]["rel_err_vs_fp64_solve"] = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
    B = torch.empty(8 * n, dtype=torch.float64, device="cuda:0")
    for k in range(8):
        gym.gym_rhs_manufactured(op, synth.modes_3d(), synth.fourier_coeffs(k, 8, 3), B[k * n:(k + 1) * n])
    res["f64_8rhs"], _ = run(gym.GYM_MODE_F64, 8, B, max(1, steps // 4))
    res["f64_8rhs"]["speedup_vs_fp64"] = res["f64_8rhs"]["solves_per_s"] / res["f64"]["solves_per_s"]
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)
    return res


def serving(gym, nreq, seed, max_slots, qps=None, budget=32 << 30, precond=None):
    """Run `nreq` mixed-Poisson requests (N ~ U{8..48}, r ~ U{1,2,3}, seeded
    N(0,1) right-hand sides) through the serving loop.  qps=None submits
    everything at t = 0; otherwise arrivals are a Poisson process."""
    import numpy as np
    rng = np.random.default_rng(seed)
    reqs = [(int(rng.integers(8, 49)), int(rng.integers(1, 4)), 1000 + k) for k in range(nreq)]
    gaps = rng.exponential(1.0 / qps, nreq) if qps else np.zeros(nreq)
    if precond is None:
        precond = gym.GYM_PRECOND_SCHUR
    o = gym.ServeOpts(device=0, mem_budget=budget, max_slots=max_slots, rtol=1e-8, maxit=100000, precond=precond)
    srv = gym.gym_serve_start(o)
    t0 = time.perf_counter()
    due = t0 + np.cumsum(gaps)
    ids, done = {}, {}
    k = 0
    last_log = t0
    while len(done) < nreq:
        now = time.perf_counter()
        while k < nreq and due[k] <= now:
            nel, r, sd = reqs[k]
            ids[gym.gym_serve_submit(srv, gym.Request(problem=0, nel=nel, degree=r, seed=sd, rhs=None,
                                                      want_solution=0))] = k
            k += 1
        for rid in [i for i in ids if i not in done]:
            st, res = gym.gym_serve_poll(srv, rid)
            if st == 0:
                done[rid] = res
        if now - last_log > 10:
            log(f"  serving: {len(done)}/{nreq} done")
            last_log = now
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    gym.gym_serve_stop(srv)
    lat = np.array([r.latency_s for r in done.values()])
    dof_it = sum(r.ndofs * r.iters for r in done.values())
    bad = sum(1 for r in done.values() if r.status != 0)
    its = np.array([r.iters for r in done.values()])
    return {"requests": nreq, "max_slots": max_slots, "qps": qps, "solves_per_s": nreq / wall,
            "precond": {gym.GYM_PRECOND_SCHUR: "block (Schur)", gym.GYM_PRECOND_JACOBI: "Jacobi"}[precond],
            "median_iters": float(np.median(its)), "max_iters": int(its.max()),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "gdof_s": dof_it / wall / 1e9, "wall_s": wall, "not_converged": bad,
            "mean_ndofs": float(np.mean([r.ndofs for r in done.values()]))}


def profile_workload(gym, ctx, which, applies):
    """For kernel traces and HBM counters: a plain copy of known size (it
    calibrates FETCH_SIZE / WRITE_SIZE per byte), then `applies` operator
    applies of the workload per contraction precision, no timing of its own."""
    import torch
    dev = torch.device("cuda:0")
    # calibration: 256 MiB and 2 GiB moved by a blit copy and by an
    # elementwise kernel (plain vector loads and stores, like the operator's)
    for words in (32 << 20, 256 << 20):
        src = torch.empty(words, dtype=torch.float64, device=dev).normal_()
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"profile-workload: calibration copies of {words * 8} bytes done")
        del src, dst
    if which == "poisson_r4_64cube":
        N, r, perturb, nrhs, prob = 64, 4, 0.0, 1, gym.GYM_MIXED_POISSON
        precs = (("f64", gym.GYM_F64), ("f32", gym.GYM_F32), ("bf16", gym.GYM_BF16))
    elif which == "hodge_r2_64cube":
        N, r, perturb, nrhs, prob = 64, 2, 0.0, 1, gym.GYM_HODGE1
        precs = (("f64", gym.GYM_F64), ("f32", gym.GYM_F32))
    else:
        N, r, perturb, nrhs, prob = 96, 3, 0.15, 8, gym.GYM_HODGE1
        precs = (("f64", gym.GYM_F64), ("f32", gym.GYM_F32))
    mesh = workload_mesh(gym, ctx, N, perturb)
    op = gym.gym_op_create(ctx, prob, mesh, r)
    n = gym.gym_op_ndofs(op)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    x = torch.randn(nrhs * n, dtype=torch.float64, device=dev, generator=gen)
    for name, prec in precs:
        xi = x if prec == gym.GYM_F64 else x.float()
        yi = torch.empty_like(xi)
        for k in range(applies):
            gym.gym_op_apply(op, prec, nrhs, xi, yi)
            torch.cuda.synchronize()
            log(f"profile-workload {which}: {name} apply {k + 1}/{applies} done")
        del xi, yi
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)


def workload_mesh(gym, ctx, N, perturb):
    """N^3 unit-cube mesh; perturb > 0: the library's seeded perturbed mesh
    (SplitMix64 offsets, seed 0)."""
    return gym.gym_mesh_structured(ctx, 3, (N, N, N), perturb, 0)


def maxwell_rates(gym, ctx, N, r, q1, steps):
    """Strang steps per second of the generalized Yee time stepping on an
    N^3 unit box (perfect conductor), lumped, exact or SPAI (pattern S(M1))
    Q1, exact M2~ unless Q1 is lumped (then both lumped: Yee's method for
    r = 1)."""
    import torch
    mesh = gym.gym_mesh_create(ctx, 3, (N, N, N))
    o = gym.gym_maxwell_opts_default()
    lumped = q1 == "lumped"
    o.q1 = {"lumped": gym.GYM_Q1_LUMPED, "exact": gym.GYM_Q1_EXACT, "spai": gym.GYM_Q1_SPAI}[q1]
    o.m2 = gym.GYM_M2_LUMPED if lumped else gym.GYM_M2_EXACT
    mx = gym.gym_maxwell_create(ctx, mesh, r, o)
    n = gym.gym_maxwell_ndofs(mx)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(21)
    a = torch.randn(n, dtype=torch.float64, device="cuda:0", generator=gen)
    e = torch.randn(n, dtype=torch.float64, device="cuda:0", generator=gen)
    # a step well inside the stability bound (2 / omega_max <= h / (c sqrt(3)) for Whitney; r^2 finer)
    tau = 0.25 / (N * r * r)
    gym.gym_maxwell_step(mx, tau, 2, a, e)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gym.gym_maxwell_step(mx, tau, steps, a, e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gym.gym_maxwell_destroy(mx)
    gym.gym_mesh_destroy(mesh)
    out = {"ndofs": n, "steps": steps, "steps_per_s": steps / wall, "gdof_steps_s": n * steps / wall / 1e9}
    if lumped:
        # one stencil kernel per step reads a and e and writes both: 32 B per unknown
        out["kernel"] = "yee_kernel (fused lumped Strang step)"
        out["algorithmic_gb_s"] = 32.0 * n * steps / wall / 1e9
        out["hbm_frac"] = out["algorithmic_gb_s"] / PEAK_HBM_GBS
    return out


def eig_rates(gym, ctx, N, r, nev, block):
    """Lowest non-kernel eigenpairs of the exact (Q1 = M1^-1) time-stepping
    operator on an N^3 unit box: wall time, LOBPCG iterations, and the
    relative deviation from the closed-form Whitney spectrum (r = 1)."""
    import numpy as np
    import torch
    mesh = gym.gym_mesh_create(ctx, 3, (N, N, N))
    mx = gym.gym_maxwell_create(ctx, mesh, r, gym.gym_maxwell_opts_default())
    o = gym.gym_eig_opts_default()
    o.nev, o.block, o.tol = nev, block, 1e-10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, info, st = gym.gym_maxwell_eigs(mx, o)
    wall = time.perf_counter() - t0
    out = {"ndofs": gym.gym_maxwell_ndofs(mx), "nev": nev, "block": block, "seconds": wall, "iters": info.iters,
           "max_resid": info.max_resid, "status": st, "omega2": [float(v) for v in w]}
    if r == 1:
        h = 1.0 / N
        lam = [(6 / h ** 2) * (1 - np.cos(np.pi * n / N)) / (2 + np.cos(np.pi * n / N)) for n in range(N)]
        ref = sorted(lam[a] + lam[b] + lam[c] for a in range(N) for b in range(N) for c in range(N)
                     if (a > 0) + (b > 0) + (c > 0) >= 2 for _ in range(2 if min(a, b, c) > 0 else 1))[:nev]
        out["max_rel_dev_closed_form"] = float(max(abs(x - y) / y for x, y in zip(w, ref)))
    gym.gym_maxwell_destroy(mx)
    gym.gym_mesh_destroy(mesh)
    return out


def spai_op_rates(gym, ctx, nel, hi, r, lam, steps):
    """SPAI-OP on an nel box with extents hi (perfect conductor, exact M2~):
    the lowest exact mode v (LOBPCG, not timed) is the probe P2 v; times the
    matrix-free Sylvester PCG that builds Q1 and the Strang steps with that
    Q1.  (The probed frequency itself is checked by the GPU tests: an
    eigen-solve on a SPAI Q1 takes B = Q1^-1 by an inner CG and is slow.)"""
    import torch
    mesh = gym.gym_mesh_create(ctx, 3, nel, hi=hi)
    mx = gym.gym_maxwell_create(ctx, mesh, r, gym.gym_maxwell_opts_default())
    n = gym.gym_maxwell_ndofs(mx)
    e = gym.gym_eig_opts_default()
    e.nev, e.tol = 1, 1e-10
    v = torch.empty(n, dtype=torch.float64, device="cuda:0")
    gym.gym_maxwell_eigs(mx, e, v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, rel, st = gym.gym_maxwell_spai_op(mx, v, lam, rtol=1e-10, maxit=20000)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(22)
    a = torch.randn(n, dtype=torch.float64, device="cuda:0", generator=gen)
    f = torch.randn(n, dtype=torch.float64, device="cuda:0", generator=gen)
    tau = 0.25 / (max(nel) * r * r)
    gym.gym_maxwell_step(mx, tau, 2, a, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gym.gym_maxwell_step(mx, tau, steps, a, f)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gym.gym_maxwell_destroy(mx)
    gym.gym_mesh_destroy(mesh)
    return {"ndofs": n, "lambda": lam, "probes": 1, "pcg_iters": it, "pcg_rel_res": rel, "status": st,
            "build_seconds": build, "pcg_iters_per_s": it / build, "steps": steps, "steps_per_s": steps / wall}


def cfl_rate(gym, ctx, N):
    """omega_max of Yee's method (Whitney forms, lumped masses) on an N^3 unit
    box by the largest-pair solver, tau_CFL = 2 / omega_max, and the relative
    deviation from the closed form (the Yee symbol at n = N - 1 on every axis)."""
    import numpy as np
    import torch
    mesh = gym.gym_mesh_create(ctx, 3, (N, N, N))
    o = gym.gym_maxwell_opts_default()
    o.q1, o.m2 = gym.GYM_Q1_LUMPED, gym.GYM_M2_LUMPED
    mx = gym.gym_maxwell_create(ctx, mesh, 1, o)
    e = gym.gym_eig_opts_default()
    e.nev, e.largest, e.block, e.tol = 2, 1, 4, 1e-10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, info, st = gym.gym_maxwell_eigs(mx, e)
    wall = time.perf_counter() - t0
    ref = 3 * (2 * N) ** 2 * np.sin(np.pi * (N - 1) / (2 * N)) ** 2
    out = {"ndofs": gym.gym_maxwell_ndofs(mx), "seconds": wall, "iters": info.iters, "status": st,
           "omega_max2": float(w[0]), "tau_cfl": float(2 / np.sqrt(w[0])),
           "rel_dev_closed_form": float(abs(w[0] - ref) / ref)}
    gym.gym_maxwell_destroy(mx)
    gym.gym_mesh_destroy(mesh)
    return out


# Sources of the operator kernel: the HBM traffic recorded under profiles/
# (rocprofv3 FETCH_SIZE / WRITE_SIZE runs) is reported only while these are
# unchanged since the counters were taken.
KERNEL_SOURCES = ("paper_2301_01753_amd/csrc/hodge_mfma.hip", "paper_2301_01753_amd/csrc/hodge_mfma.hpp",
                  "paper_2301_01753_amd/csrc/kernels.hpp", "paper_2301_01753_amd/csrc/geom.hpp",
                  "paper_2301_01753_amd/csrc/gen/gen_tables.cpp", "paper_2301_01753_amd/csrc/tables.cpp")
TRAFFIC_FILE = "profiles/op_kernel_hodge_r3_96cube_perturbed_traffic.txt"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) of the operator
    kernel on this workload, or None when not measured for the current sources."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k] = v
    if kv.get("source_hash") != kernel_source_hash() or kv.get("workload") != workload:
        return None
    return float(kv["fetch_bytes"]) + float(kv["write_bytes"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60, help="timed applies (>= 50 for the median)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--no-solves", action="store_true", help="skip the 64^3 degree-4 Poisson solves")
    ap.add_argument("--profile-apply", type=int, default=0,
                    help="counter runs: copy calibration + this many MINRES steps of the 32^3 degree-2 Hodge "
                         "workload, no JSON")
    ap.add_argument("--profile-workload", choices=("poisson_r4_64cube", "hodge_r3_96cube_perturbed_8rhs",
                                                   "hodge_r2_64cube"),
                    help="counter/trace runs: copy calibration + K operator applies per precision of that "
                         "workload, no JSON")
    ap.add_argument("--profile-spai-q1", action="store_true",
                    help="only the SPAI-Q1 time stepping (128^3 degree 1, 32^3 degree 2), for a kernel trace")
    ap.add_argument("--profile-spai-op", action="store_true",
                    help="only the SPAI-OP builds (degree 1 and 2) and stepping, for a kernel trace")
    ap.add_argument("--profile-maxwell", action="store_true",
                    help="profiling runs: only the lumped time-stepping rates (Yee 128^3, degree 2 on 32^3), no JSON")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests in the serving sample (0 skips it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(DESIGN.md describes how the operator would shard).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2301_01753_amd import gym

    dev = torch.device("cuda:0")
    ctx = gym.gym_create(0)
    if args.profile_spai_q1:
        for N, deg, steps in ((128, 1, 200), (32, 2, 500)):
            log(f"SPAI-Q1 time stepping {N}^3 degree {deg}: {maxwell_rates(gym, ctx, N, deg, 'spai', steps)}")
        gym.gym_destroy(ctx)
        return
    if args.profile_spai_op:
        for nel, deg in (((24, 20, 16), 1), ((12, 10, 8), 2)):
            log(f"SPAI-OP {nel} degree {deg}: {spai_op_rates(gym, ctx, nel, (1.0, 1.3, 0.8), deg, 5e5, 500)}")
        gym.gym_destroy(ctx)
        return
    if args.profile_workload:
        profile_workload(gym, ctx, args.profile_workload, args.steps)
        gym.gym_destroy(ctx)
        return
    if args.profile_maxwell:
        for N, deg in ((128, 1), (32, 2)):
            log(f"lumped time stepping {N}^3 degree {deg}: {maxwell_rates(gym, ctx, N, deg, 'lumped', 2000)}")
        gym.gym_destroy(ctx)
        return
    if args.profile_apply:
        import synth
        mesh = gym.gym_mesh_create(ctx, 3, (32, 32, 32))
        op = gym.gym_op_create(ctx, gym.GYM_HODGE1, mesh, 2)
        n = gym.gym_op_ndofs(op)
        b = torch.empty(n, dtype=torch.float64, device=dev)
        gym.gym_rhs_manufactured(op, synth.modes_3d(), synth.fourier_coeffs(0, 8, 3), b)
        src = torch.empty(32 << 20, dtype=torch.float64, device=dev).normal_()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        xv = torch.empty_like(b)
        o = gym.gym_solve_opts_default()
        o.maxit = args.profile_apply
        gym.gym_solve(op, o, 1, b, xv)
        torch.cuda.synchronize()
        log(f"profile-apply: copy of {src.numel() * 8} bytes x3, {args.profile_apply} MINRES steps")
        return

    # ---- headline: perturbed 96^3 degree-3 Hodge, 8 rhs, FP64 apply ----
    N, r, nrhs = HEAD_N, HEAD_R, HEAD_NRHS
    t0 = time.perf_counter()
    mesh = gym.gym_mesh_structured(ctx, 3, (N, N, N), HEAD_PERTURB, 0)
    op = gym.gym_op_create(ctx, gym.GYM_HODGE1, mesh, r)
    n = gym.gym_op_ndofs(op)
    log(f"workload: perturbed {N}^3 degree {r} Hodge, {n} DoFs x {nrhs} rhs (setup {time.perf_counter() - t0:.1f} s)")
    gen = torch.Generator(device=dev)
    gen.manual_seed(12)
    x = torch.randn(nrhs * n, dtype=torch.float64, device=dev, generator=gen)
    y = torch.empty_like(x)
    ms, wall = event_times(lambda: gym.gym_op_apply(op, gym.GYM_F64, nrhs, x, y), args.steps, args.warmup)
    t_med = median(ms) / 1e3
    value = nrhs * n / t_med / 1e9
    log(f"FP64 apply: median {t_med * 1e3:.3f} ms over {args.steps} applies ({min(ms):.3f} .. {max(ms):.3f} ms), "
        f"wall {wall / args.steps * 1e3:.3f} ms per apply")
    nel3 = N ** 3
    flops = algorithmic_flops_per_element("hodge", r, metric=True) * nel3 * nrhs
    # bytes: the vectors in and out once, and the cell vertices once (the
    # kernel computes the Piola metrics at the Gauss points from them)
    qbytes = 3 * 8.0 * (N + 1) ** 3
    bytes_ = 16.0 * n * nrhs + qbytes
    roof = {"bound": "alu", "achieved": flops / t_med / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic("hodge_r3_96cube_perturbed_8rhs_f64")
    roof["kernel"] = ("hodge_mfma_kernel<16, 2> + hodge_mfma_fixup (one apply: the matrix-core element kernel "
                      "and its tile-boundary sums)")
    roof["avg_launch_us"] = sum(ms) / len(ms) * 1e3
    roof["median_launch_us"] = t_med * 1e6
    roof["algorithmic_flops"] = flops
    roof["algorithmic_bytes"] = bytes_
    roof["arithmetic_intensity"] = flops / bytes_
    roof["achieved_hbm_gb_s"] = bytes_ / t_med / 1e9
    roof["hbm_frac"] = roof["achieved_hbm_gb_s"] / PEAK_HBM_GBS
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"unit cube {N}^3 hex, seeded vertex perturbation 15% of h (SplitMix64, seed 0), "
                         f"degree-{r} Hodge Laplacian on 1-forms (H1_0 x H0(curl)), {nrhs} N(0,1) right-hand "
                         f"sides, FP64 matrix-free operator apply"),
            "ndofs_per_rhs": n,
            "nrhs": nrhs,
            "parallelism": "single GPU",
        },
        "apply_median_ms": t_med * 1e3,
        "roofline": roof,
    }
    extras = {}
    if not args.no_extras:
        log("FP32 apply of the headline workload ...")
        del y
        extras["hodge_r3_96cube_perturbed_8rhs_f32"] = apply_rates(
            gym, op, n, nrhs, (("f64", gym.GYM_F64), ("f32", gym.GYM_F32)), 20, 2, 12)
    del x
    gym.gym_op_destroy(op)
    gym.gym_mesh_destroy(mesh)
    torch.cuda.empty_cache()

    if not args.no_extras:
        if not args.no_solves:
            log("64^3 degree-4 mixed Poisson: applies and solves to 1e-8 ...")
            extras["poisson_r4_64cube"] = poisson64_solves(
                gym, ctx, 1e-8, (("f64", gym.GYM_MODE_F64, 0.0), ("ir_f32", gym.GYM_MODE_IR_F32, 1e-2),
                                 ("ir_bf16", gym.GYM_MODE_IR_BF16, 1e-2)), 3)
        log("32^3 degree-2 Hodge solves ...")
        extras["hodge_r2_32cube"] = hodge32_solves(gym, ctx, 4, 1e-10)
        if args.serve_requests > 0:
            nreq = args.serve_requests
            log(f"serving {nreq} requests (batched) ...")
            batched = serving(gym, nreq, 7, max_slots=32)
            log("serving (one at a time) ...")
            single = serving(gym, nreq, 7, max_slots=1)
            sweep = {}
            for f in (0.5, 1.0, 2.0):
                log(f"serving (Poisson arrivals at {f} x the batched rate) ...")
                sweep[f"{f}x"] = serving(gym, nreq, 7, max_slots=32, qps=f * batched["solves_per_s"])
            extras["serving"] = {
                "workload": f"{nreq} mixed Poisson solves, N ~ U{{8..48}}^3 hex, degree ~ U{{1,2,3}}, "
                            "N(0,1) rhs (seeded), rel. residual 1e-8, block preconditioner",
                "batched": batched, "one_at_a_time": single, "poisson_arrivals": sweep,
                "speedup_batched_vs_one_at_a_time": batched["solves_per_s"] / single["solves_per_s"],
            }
        log("generalized Yee time stepping ...")
        extras["gym_time_stepping"] = {
            "yee_r1_128cube_lumped": maxwell_rates(gym, ctx, 128, 1, "lumped", 2000),
            "r2_32cube_lumped": maxwell_rates(gym, ctx, 32, 2, "lumped", 2000),
            "r2_32cube_exact_q1_cg": maxwell_rates(gym, ctx, 32, 2, "exact", 20),
            "r1_128cube_spai_q1": maxwell_rates(gym, ctx, 128, 1, "spai", 200),
            "r2_32cube_spai_q1": maxwell_rates(gym, ctx, 32, 2, "spai", 500),
        }
        log("SPAI-OP ...")
        extras["gym_spai_op"] = {"r1_24x20x16_box": spai_op_rates(gym, ctx, (24, 20, 16), (1.0, 1.3, 0.8), 1, 5e5, 500)}
        log("eigenmodes ...")
        extras["gym_eigenmodes"] = {
            "whitney_24cube_lowest5": eig_rates(gym, ctx, 24, 1, 5, 7),
            "yee_128cube_omega_max": cfl_rate(gym, ctx, 128),
        }
        out["extras"] = extras

    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(7, r, nrhs)

    gym.gym_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
