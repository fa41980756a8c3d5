#!/usr/bin/env python3
"""Throughput of the hp-multigrid preconditioned skeleton solve on one MI355X.

Headline workload (the largest single-GPU configuration): 3D generalized
Stokes on the unit cube, 4^3 Kuhn cubes (six tetrahedra each) refined three
times (32^3 cubes, 196,608 tetrahedra, 4 levels), order k = 3, beta = 1,
nu = 1, gamma = eps^-1 = 1e3, f = uniform[-1,1) per data point (seed 0);
edge-patch relaxation and smoothing, m_p = m_h = 2, variable V-cycle.
A step is inner solve #1 of the AL-Uzawa iteration: A^eps lambda = g from
lambda = 0 by flexible CG preconditioned by MG_hp to relative residual 1e-8,
every operation in the HIP library, the condensed load g already resident
in HBM.  `value` is the all-FP64 solve; `mixed` stores the V-cycle's
operators in FP32 (FP64 vectors, accumulation and Krylov; same 1e-8 on the
FP64 operator), with its relative difference from the FP64 solution.  The
same cube at k = 2 and the 2D workloads (256x256 Stokes, the lid-driven
cavity, Alg. 3, the batch gradient) are reported as sub-objects.

Prints one JSON line (metric, value = skeleton DOFs solved per second,
roofline of the dominant kernel from live HIP-event timing, the V-cycle
against the compulsory bytes of its operators, and the CPU oracle timed on
the host's cores on a bounded sample).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_MFMA_TFS = 78.6
KCLASS3 = {0: "order-k edge-patch Gauss-Seidel, one colour (k_patch_gs3)",
           1: "order-k skeleton apply S_K x_K (k_cell_apply3 + k_face_gather3)",
           2: "lowest-order edge-patch Gauss-Seidel phases (k_patch_gs3_lo)",
           3: "MG_hp"}
KCLASS = {0: "order-k vertex-patch Gauss-Seidel, one colour phase (k_patch_gs_fused; "
             "k_patch_relax_wave for the first phase from zero)",
          1: "order-k cell apply S_K x_K (k_cell_apply: the residual and Krylov applies)",
          2: "lowest-order smoothing phases on launched levels (k_patch_gs_fused on streamed levels, "
             "k_gs_records on the others)"}
# Class 4: MG_h on the coarse levels -- at the V-cycle's entry level the
# operator tabulated at assembly (one dense GEMV), else the single-workgroup
# kernel.
COARSE_CLASS = "coarse MG_h: tabulated operator (k_gemv_rows) / single-workgroup kernel (k_coarse_cycle)"
# The 2D line reports the order-k cell apply (every Krylov apply and every
# V-cycle residual read all cell blocks) and the colour phase.
ROOF_CLASS = 1

def _oracle_worker(args):
    """One CPU process of the baseline: the 3D oracle on the sample mesh,
    setup untimed, then `reps` inner solves #1 timed."""
    k, reps, seed = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import solver3d
    with threadpool_limits(1):
        c, t = synth.kuhn_cube(1)
        S = solver3d.Setup3(c, t, 2, k, 1.0, 1.0, 1e3)
        f = synth.source_uniform(seed, 1, S.lv.n_cells, (k + 2) ** 3, dim=3)[0]
        g = S.prob.rhs(f)
        t0 = time.perf_counter()
        for _ in range(reps):
            _, its, _ = S.inner(g, atol=0.0)
        dt = time.perf_counter() - t0
    return S.Aeps.shape[0], its, dt


def cpu_baseline(k, reps, workers):
    """The CPU oracle, untuned, on a bounded sample of the headline workload,
    on `workers` host cores at once (one process each, one thread each):
    the unit cube as one Kuhn cube refined twice (384 tetrahedra, 3 levels),
    same k, beta, nu, gamma, smoothing and f recipe; each process times
    `reps` inner solves #1 (setup excluded).  The value is the sum of the
    processes' rates.  Runs before the GPU is touched (forked workers)."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, [(k, reps, 0)] * workers)
    wall = time.perf_counter() - t0
    n, its = res[0][0], res[0][1]
    rate = sum(n * reps / dt for _, _, dt in res)
    return {"value": rate, "unit": "skeleton DOFs/s", "cores": workers, "kind": "oracle",
            "sample": f"unit cube, one Kuhn cube refined twice (384 tets, 3 levels), k={k}, N_skel={n}, "
                      f"inner solve #1 ({its} its) x{reps} in each of {workers} single-thread processes "
                      f"(numpy/scipy), setup excluded; sum of the processes' rates",
            "seconds_per_process": [round(dt, 2) for _, _, dt in res], "wall_s": round(wall, 1)}


def oseen_workload(hd, synth, torch, np, steps, re, k=3, n_refine=5):
    """Lid-driven cavity: 128x128 squares (32768 cells, 6 levels), k = 3,
    beta = 0, nu = 1/Re, eps^-1 = 1e2 nu, lid uhat = (1,0) on the top side,
    body force sum_{a,b=1..3} c_ab sin(a pi x) sin(b pi y) (c ~ U[-1,1),
    seed 2); a Stokes solve then `steps` Picard steps, each AL-Uzawa with
    FGMRES(50) preconditioned by the FP32-storage V-cycle.  Timed: the
    solves (each step's re-assembly reported separately).  Then the adjoint
    of the last Picard step's Oseen system (its wind fixed) for the kinetic
    energy J = sum_{K,q} w_q |K| |u(x_q)|^2: a context holding A^T (assembled,
    timed apart) and one adjoint solve giving dJ/df and dJ/dnu."""
    c, t = synth.kuhn_square(4)
    nu = 1.0 / re
    s = hd.Solver(c, t, n_refine, k, 0.0, nu, 1e2 * nu, oseen=1, vcycle_precision=1)
    X = s.data_points().cpu().numpy()
    coef = synth.uniform_pm1(2, 0, (2, 3, 3))
    f = np.zeros(X.shape)
    for i in range(2):
        for a in range(3):
            for b in range(3):
                f[..., i] += coef[i, a, b] * np.sin((a + 1) * np.pi * X[..., 0]) * np.sin((b + 1) * np.pi * X[..., 1])
    f = torch.as_tensor(f, device="cuda")
    s.set_dirichlet_velocity(torch.as_tensor(synth.lid_velocity(s.boundary_facets().cpu().numpy()), device="cuda"))
    t_solve = t_asm = 0.0
    its, dus, x0, u_prev, w_last = [], [], None, None, None
    for n in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w_last = u_prev
        s.set_wind(None if u_prev is None else u_prev)
        s.assemble()
        torch.cuda.synchronize()
        t_asm += time.perf_counter() - t0
        t0 = time.perf_counter()
        u, p, state, info, st = s.solve(f, x0=x0)
        torch.cuda.synchronize()
        t_solve += time.perf_counter() - t0
        its.append(info["its"])
        if u_prev is not None:
            dus.append(float((u - u_prev).abs().max()))
        u_prev, x0 = u, state[:s.n_skel]
    adj = None
    if w_last is not None:
        sa = hd.Solver(c, t, n_refine, k, 0.0, nu, 1e2 * nu, oseen=1, vcycle_precision=1, transpose=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sa.set_wind(w_last)
        sa.set_dirichlet(s.dirichlet_data())
        sa.assemble()
        torch.cuda.synchronize()
        t_aasm = time.perf_counter() - t0
        gu = 2.0 * s.data_weights()[..., None] * u_prev
        t0 = time.perf_counter()
        gf, gnu, _, ainfo, ast = sa.solve_adjoint(f, state, gu)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        adj = {"value": s.n_skel / t_adj, "unit": "skeleton DOFs/s", "status": ast, "solve_s": t_adj,
               "assemble_s": t_aasm, "fgmres_its_per_uzawa_step": ainfo["its"],
               "grad_norms": {"f": float(gf.norm()), "nu": float(gnu.norm())},
               "functional": "kinetic energy sum w_q |K| |u(x_q)|^2 at the last Picard step, wind fixed"}
        sa.close()
    out = {"workload": f"lid-driven cavity, 128x128 structured triangulation ({s.n_cells} cells, {s.levels} "
                       f"levels), k={k}, Re={re:g}, beta=0, eps^-1=1e2 nu; Stokes solve + {steps} Picard steps",
           "n_skel": s.n_skel, "value": s.n_skel * (steps + 1) / t_solve, "unit": "skeleton DOFs/s",
           "solve_s": t_solve, "assemble_s_total": t_asm, "fgmres_its_per_uzawa_step": its,
           "picard_max_du": dus, "adjoint_last_step": adj,
           "precision": "V-cycle operators FP32, FGMRES(50) and everything else FP64"}
    s.close()
    return out


def lid_solver(hd, synth, torch, k, n_refine, beta, nu, **kw):
    """A context on the paper's cavity: the unit square from 2x2 Kuhn
    squares (level n_refine + 1), lid u = (4x(1-x), 0) on y = 1 (its facet
    L^2 projection), no-slip elsewhere, (nu eps)^-1 = 1e6, two AL-Uzawa
    steps per linear solve (Sec. 5 settings)."""
    c, t = synth.kuhn_square(2)
    s = hd.Solver(c, t, n_refine, k, beta, nu, 1e6 * nu, uzawa_max=2, uzawa_tol=-1.0, **kw)
    ends = s.boundary_facets().cpu().numpy()
    lid = synth.lid_coefficients(ends, k, lambda x: 4.0 * x * (1.0 - x))
    s.set_dirichlet(torch.as_tensor(lid, device="cuda"))
    return s


def alg3_workload(hd, synth, torch, np, re, k=3, n_refine=6):
    """Alg. 3 on the paper's lid-driven cavity (Sec. 5.2.2): level 7
    (128x128), k = 3, beta = 0, nu = 1/Re, f = 0, (nu eps)^-1 = 1e6, two
    AL-Uzawa steps per linear solve, m_p = m_h = 1.  A Stokes solve, Picard
    steps until ||u_n - u_{n-1}||_0 < 1e-4, then Newton steps until
    ||u_n - u_{n-1}||_0 <= max(1e-8 ||u_n||_0, 1e-10), every inner solve by
    FGMRES(50) with the FP64 V-cycle to rel. res. 1e-8.  Reports the
    average FGMRES iterations per inner solve in each phase (the quantity
    the paper tabulates) and the wall time of the whole iteration
    (re-assemblies included)."""
    nu = 1.0 / re
    s = lid_solver(hd, synth, torch, k, n_refine, 0.0, nu, oseen=1)
    f = torch.zeros((s.n_cells, s.n_q, 2), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = hd.picard_newton(s, f, eps_picard=1e-4, newton_rtol=1e-8, newton_atol=1e-10)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res = {"workload": f"lid-driven cavity (lid 4x(1-x), f = 0), level {n_refine + 1} ({s.n_cells} cells), "
                       f"k={k}, Re={re:g}, beta=0, (nu eps)^-1=1e6, two Uzawa steps, m=1; Alg. 3: Picard "
                       f"to 1e-4, then Newton to 1e-8",
           "n_skel": s.n_skel, "wall_s": wall, "steps": [o["kind"] for o in out],
           "du": [o["du"] for o in out], "status": [o["status"] for o in out]}
    for kind in ("picard", "newton"):
        its = [i for o in out if o["kind"] == kind for i in o["info"]["its"]]
        res[f"avg_fgmres_its_{kind}"] = float(np.mean(its)) if its else None
        res[f"solve_s_{kind}"] = float(sum(o["info"]["t_solve"] for o in out if o["kind"] == kind))
    s.close()
    return res


def step_solver(hd, synth, torch, k, n_refine, beta, nu, **kw):
    """A context on the paper's backward-facing step (Sec. 5.3): 15 squares
    of side 0.5 (level n_refine + 1), inflow (16 (1-y)(y-0.5), 0) on x = 0,
    do-nothing outflow on x = 4, no-slip elsewhere, (nu eps)^-1 = 1e6, two
    AL-Uzawa steps, vertex patches (kw may choose others)."""
    c, t, out = synth.step_domain(1)
    s = hd.Solver(c, t, n_refine, k, beta, nu, 1e6 * nu, uzawa_max=2, uzawa_tol=-1.0, outflow=out, **kw)
    ends = s.boundary_facets().cpu().numpy()
    s.set_dirichlet_full(torch.as_tensor(synth.boundary_coefficients(ends, k, synth.step_inflow), device="cuda"))
    return s


def step_tables(hd, synth, torch, np):
    """The paper's step runs beside tab:stokesBack (k = 0..3, levels 4-7,
    beta in {0, 1e3}, m in {1, 2}, variable V- and W-cycle) and
    tab:nsBack2D (Alg. 3, k = 0..3, nu in {1, 1e-2, 1e-3}, m = 1).  One
    JSON line per case; a breakdown of the flexible CG is reported as
    "NA" (status -6)."""
    for k in range(4):
        for level in range(4, 8):
            for cyc in (1, 2):
                for beta in (0.0, 1e3):
                    for m in (1, 2):
                        kw = dict(cycle=cyc, m_relax=m, m_smooth=m)
                        if cyc == 2:
                            kw["vcycle_growth"] = 1
                        s = step_solver(hd, synth, torch, k, level - 1, beta, 1.0, **kw)
                        s.assemble()
                        f = torch.zeros((s.n_cells, s.n_q, 2), dtype=torch.float64, device="cuda")
                        try:
                            u, p, state, info, st = s.solve(f)
                            its, status = info["its"], st
                        except hd.HdgmgError as e:
                            its, status = None, e.status
                        print(json.dumps({"table": "stokesBack", "d": 2, "k": k, "level": level,
                                          "cycle": "V" if cyc == 1 else "W", "beta": beta, "m": m,
                                          "pcg_its": its, "status": status}), flush=True)
                        s.close()
    for k in range(4):
        for level in (range(4, 8) if k < 2 else range(3, 7)):
            for nu in (1.0, 1e-2, 1e-3):
                s = step_solver(hd, synth, torch, k, level - 1, 0.0, nu, oseen=1)
                f = torch.zeros((s.n_cells, s.n_q, 2), dtype=torch.float64, device="cuda")
                t0 = time.perf_counter()
                try:
                    out = hd.picard_newton(s, f, eps_picard=1e-4, newton_rtol=1e-8, newton_atol=1e-10,
                                           max_picard=30, max_newton=10 if k > 0 else 0)
                    rec = {"steps": [o["kind"] for o in out], "status": max(o["status"] for o in out)}
                    for kind in ("picard", "newton"):
                        its = [i for o in out if o["kind"] == kind for i in o["info"]["its"]]
                        rec[f"avg_pgm_its_{kind}"] = float(np.mean(its)) if its else None
                except hd.HdgmgError as e:
                    rec = {"status": e.status}
                rec.update({"table": "nsBack2D", "k": k, "level": level, "nu": nu,
                            "wall_s": time.perf_counter() - t0})
                print(json.dumps(rec), flush=True)
                s.close()


def paper_tables(hd, synth, torch, np):
    """The paper's cavity runs beside its tables: PCG counts of the Stokes
    cavity (Sec. 5.2.1; k = 0..3, levels 4-7, beta in {0, 1e3}, m in {1, 2},
    variable V- and W-cycle) and average PGM counts of Alg. 3 on the
    Navier-Stokes cavity (Sec. 5.2.2; k = 2, 3, levels 5-8, nu in {1, 1e-2,
    1e-3}, m = 1).  One JSON line per case."""
    for k in range(4):
        for level in range(4, 8):
            for cyc in (1, 2):
                for beta in (0.0, 1e3):
                    for m in (1, 2):
                        kw = dict(cycle=cyc, m_relax=m, m_smooth=m)
                        if cyc == 2:
                            kw["vcycle_growth"] = 1
                        s = lid_solver(hd, synth, torch, k, level - 1, beta, 1.0, **kw)
                        s.assemble()
                        f = torch.zeros((s.n_cells, s.n_q, 2), dtype=torch.float64, device="cuda")
                        try:
                            u, p, state, info, st = s.solve(f)
                            its, status = info["its"], st
                        except hd.HdgmgError as e:
                            its, status = None, e.status
                        print(json.dumps({"table": "stokesLid", "d": 2, "k": k, "level": level,
                                          "cycle": "V" if cyc == 1 else "W", "beta": beta, "m": m,
                                          "pcg_its": its, "status": status}), flush=True)
                        s.close()
    for k in (2, 3):
        for level in range(5, 9):
            for nu in (1.0, 1e-2, 1e-3):
                s = lid_solver(hd, synth, torch, k, level - 1, 0.0, nu, oseen=1)
                f = torch.zeros((s.n_cells, s.n_q, 2), dtype=torch.float64, device="cuda")
                t0 = time.perf_counter()
                out = hd.picard_newton(s, f, eps_picard=1e-4, newton_rtol=1e-8, newton_atol=1e-10)
                rec = {"table": "nsLid2D", "k": k, "level": level, "nu": nu, "wall_s": time.perf_counter() - t0,
                       "steps": [o["kind"] for o in out], "status": max(o["status"] for o in out)}
                for kind in ("picard", "newton"):
                    its = [i for o in out if o["kind"] == kind for i in o["info"]["its"]]
                    rec[f"avg_pgm_its_{kind}"] = float(np.mean(its)) if its else None
                print(json.dumps(rec), flush=True)
                s.close()


def adjoint_workload(hd, synth, torch, np, nrhs):
    """Batch gradient: 128x128 squares (32768 cells), k = 2, beta = 1,
    eps^-1 = 1e2, per-cell nu = exp(0.5 Z) (Z ~ N(0,1), seed 3); sources
    f_i ~ U[-1,1) (seeds 100..), target u_t ~ U[-1,1) (seed 4); loss
    sum_i sum_{K,q} w_q |K| |u_i - u_t|^2; forward solves and adjoint
    solves (gradients w.r.t. f_i and nu) with the FP32-storage V-cycle.
    Timed: forward + backward of the autograd function, on one context and
    on a pool of four contexts with a HIP stream each (the batch spread over
    them), each after one untimed pass; `value` is the pool's."""
    c, t = synth.kuhn_square(4)
    nr, k = 5, 2
    n_cells = 32 * 4 ** nr
    nu = np.exp(0.5 * synth.normal(3, 0, n_cells))
    s = hd.Solver(c, t, nr, k, 1.0, nu, 1e2, vcycle_precision=1)
    s.assemble()
    # the same problem on four contexts, one HIP stream each: the batch's
    # solves run concurrently (their lowest-order levels are latency-bound)
    pool = hd.solver_pool(4, c, t, nr, k, 1.0, nu, 1e2, vcycle_precision=1)
    nq = s.n_q
    F = torch.as_tensor(np.stack([synth.source_uniform(100 + i, 1, n_cells, nq)[0] for i in range(nrhs)]),
                        device="cuda").requires_grad_(True)
    ut = torch.as_tensor(synth.source_uniform(4, 1, n_cells, nq)[0], device="cuda")
    nu_t = torch.as_tensor(nu, device="cuda").requires_grad_(True)
    W = s.data_weights()

    def run(solver):
        F.grad = None
        nu_t.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = hd.stokes_solve(solver, F, nu_t)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        J = (W[None, :, :, None] * (u - ut[None]) ** 2).sum()
        t0 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        return t_f, time.perf_counter() - t0

    run(s)  # untimed: graph capture and first-call buffers of every context
    run(pool)
    t1_fwd, t1_bwd = run(s)
    t_fwd, t_bwd = run(pool)
    out = {"workload": f"batch gradient, 128x128 structured triangulation ({n_cells} cells), k={k}, beta=1, "
                       f"eps^-1=1e2, log-normal per-cell nu, {nrhs} sources; forward + adjoint solves",
           "n_skel": s.n_skel, "value": 2 * nrhs * s.n_skel / (t_fwd + t_bwd), "unit": "skeleton DOFs/s",
           "streams": len(pool), "forward_s": t_fwd, "backward_s": t_bwd,
           "value_one_stream": 2 * nrhs * s.n_skel / (t1_fwd + t1_bwd),
           "forward_s_one_stream": t1_fwd, "backward_s_one_stream": t1_bwd,
           "grad_norms": {"f": float(F.grad.norm()), "nu": float(nu_t.grad.norm())},
           "precision": "V-cycle operators FP32, flexible CG and everything else FP64"}
    for p_ in pool:
        p_.close()
    s.close()
    return out


def copy_bandwidth(torch, reps=5):
    """Read + write bandwidth of a plain 1 GiB device copy (HIP events)."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * src.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def sweep(hd, synth, torch, np, c, t, a):
    """Config sweeps (one JSON line per case, printed as it finishes).
    Stokes: 256x256 (7 levels), k in 1..4, beta in {0, 1, 1e3}, nu = 1,
    gamma in {1, 1e2, 1e4}, FP64 and FP32-storage V-cycles; source seeded
    uniform[-1,1) plus the gradient of the trig polynomial; inner solve #1
    to rel. res. 1e-8 (atol 0), best of two after one warm-up.  Cavity:
    128x128, k = 3, Re in {1, 10, 100, 1000}, a Stokes solve + 10 Picard
    steps (oseen_workload)."""
    rows = []
    for k in (1, 2, 3, 4):
        for beta in (0.0, 1.0, 1e3):
            for gamma in (1.0, 1e2, 1e4):
                for prec in (0, 1):
                    t0 = time.perf_counter()
                    s = hd.Solver(c, t, a.n_refine, k, beta, 1.0, gamma, atol=0.0, vcycle_precision=prec)
                    s.assemble()
                    torch.cuda.synchronize()
                    t_asm = time.perf_counter() - t0
                    X = s.data_points().cpu().numpy()
                    f = synth.source_uniform(0, 1, s.n_cells, s.n_q)[0] + synth.trig_gradient(X, 1)
                    g = s.rhs(torch.as_tensor(f, device="cuda"))
                    x = torch.empty_like(g)
                    s.inner_solve(g, x)
                    best = None
                    for _ in range(2):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        _, its, rel, st = s.inner_solve(g, x)
                        torch.cuda.synchronize()
                        dt = time.perf_counter() - t0
                        best = dt if best is None else min(best, dt)
                    row = {"case": "stokes 256x256", "k": k, "beta": beta, "gamma": gamma,
                           "vcycle": "fp64" if prec == 0 else "fp32", "n_skel": s.n_skel, "iterations": its,
                           "status": st, "rel_res": rel, "ms": 1e3 * best, "dofs_per_s": s.n_skel / best,
                           "setup_assemble_s": t_asm}
                    print(json.dumps(row), flush=True)
                    rows.append(row)
                    s.close()
    for re_ in (1.0, 10.0, 100.0, 1000.0):
        o = oseen_workload(hd, synth, torch, np, 10, re_)
        its = [i for step in o["fgmres_its_per_uzawa_step"] for i in step]
        row = {"case": "cavity 128x128 k=3", "Re": re_, "value": o["value"], "solve_s": o["solve_s"],
               "assemble_s_total": o["assemble_s_total"], "avg_fgmres_its": float(np.mean(its)),
               "uzawa_steps": [len(step) for step in o["fgmres_its_per_uzawa_step"]],
               "picard_max_du": o["picard_max_du"]}
        print(json.dumps(row), flush=True)
        rows.append(row)
    print(json.dumps({"sweep_cases": len(rows)}), flush=True)


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs of `bench.py --profile-run` (the same kernel and
# workload), each scaled by what the counter reads for a copy kernel of
# known size (FETCH_SIZE counts 0.500 of the bytes read, WRITE_SIZE 1.000 of
# those written on this part); the summary, with its commands, is in
# COUNTER_SOURCE.  Retake them whenever the kernel changes.
COUNTER_TRAFFIC = {("order-k edge-patch Gauss-Seidel, one colour (k_patch_gs3)", 3): 7.369e9 + 0.027e9}
COUNTER_SOURCE = "profiles/k_patch_gs3_fp64_k3_32cube.md"


def progress(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def stokes3d(hd, synth, torch, np, k, prec, steps, warmup, tsteps, x_ref=None):
    """The cube workload at order k and V-cycle storage `prec`: setup,
    assembly, inner solve #1 timed `steps` times after `warmup`, then
    `tsteps` more with the live per-kernel timers."""
    progress(f"cube k={k} precision {prec}: setup and assembly")
    c, t = synth.kuhn_cube(4)
    t0 = time.perf_counter()
    s = hd.Solver(c, t, 3, k, 1.0, 1.0, 1e3, atol=0.0, m_relax=2, m_smooth=2, vcycle_precision=prec)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    s.assemble()
    torch.cuda.synchronize()
    t_assemble = time.perf_counter() - t0
    f = torch.as_tensor(synth.source_uniform(0, 1, s.n_cells, s.n_q, dim=3)[0], device="cuda")
    g = s.rhs(f)
    del f
    x = torch.empty_like(g)
    for _ in range(warmup):
        s.inner_solve(g, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_all = []
    for _ in range(steps):
        _, its, rel, st = s.inner_solve(g, x)
        its_all.append(its)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    progress(f"cube k={k} precision {prec}: {steps} solves in {T:.2f} s, iterations {its_all}")
    xh = x.cpu().numpy()
    err = None if x_ref is None else float(np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref))
    for cls in range(4):
        s.timer(cls, True)
    torch.cuda.synchronize()
    for _ in range(tsteps):
        s.inner_solve(g, x)
    torch.cuda.synchronize()
    tm = {cls: s.timer_read(cls) for cls in range(4)}
    for cls in range(4):
        s.timer(cls, False)
    out = dict(T=T, its=its_all, tm=tm, t_setup=t_setup, t_assemble=t_assemble, n_skel=s.n_skel,
               n_cells=s.n_cells, levels=s.levels, rel=rel, status=st, x=xh, err_vs_fp64=err,
               vc_design=s.query(12), vc_compulsory=s.query(13))
    s.close()
    del g, x
    torch.cuda.empty_cache()
    return out


def classes3(tm):
    return {KCLASS3[c_]: {"ms": tm[c_][0], "launches": tm[c_][1], "GB": tm[c_][2] / 1e9,
                          "avg_us": 1e3 * tm[c_][0] / max(tm[c_][1], 1)} for c_ in range(4)}


def vcycle3(m):
    ms, n, _ = m["tm"][3]
    avg = ms / max(n, 1) * 1e-3
    return {"avg_ms": 1e3 * avg, "compulsory_GB": m["vc_compulsory"] / 1e9,
            "compulsory_GB_per_s": m["vc_compulsory"] / avg / 1e9,
            "frac_of_hbm_peak": m["vc_compulsory"] / avg / 1e9 / PEAK_HBM_GBS,
            "implementation_GB": m["vc_design"] / 1e9, "implementation_GB_per_s": m["vc_design"] / avg / 1e9,
            "model": "compulsory = every stored operator read once per use in packed symmetric form (cell "
                     "blocks, edge-patch inverses, CR blocks, coarsest inverse) + vectors + transfers; "
                     "implementation = what the launches move (per edge patch and patch cell the coupling "
                     "of its two patch faces to its two far faces, a quarter of S_K, so S_K is read 1.5 "
                     "times per sweep; full patch inverses)"}


def stokes2d_line(hd, synth, torch, np, a):
    """The 256x256 generalized Stokes workload of the triangular path (k = 2,
    beta = 1, gamma = 1e2, 7 levels, vertex patches, m_p = m_h = 1): FP64,
    FP32-storage and FP16-storage V-cycles, with kernel classes and the
    V-cycle against its compulsory bytes."""
    c, t = synth.kuhn_square(4)

    def measure(prec, x_ref=None):
        t0 = time.perf_counter()
        s = hd.Solver(c, t, 6, 2, 1.0, 1.0, 1e2, atol=0.0, vcycle_precision=prec)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        s.assemble()
        torch.cuda.synchronize()
        t_assemble = time.perf_counter() - t0
        X = s.data_points().cpu().numpy()
        f = synth.source_uniform(0, 1, s.n_cells, s.n_q)[0] + synth.trig_gradient(X, 1)
        g = s.rhs(torch.as_tensor(f, device="cuda"))
        x = torch.empty_like(g)
        s.inner_solve(g, x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its_all = []
        for _ in range(a.steps2d):
            _, its, rel, st = s.inner_solve(g, x)
            its_all.append(its)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        xh = x.cpu().numpy()
        for cls in range(5):
            s.timer(cls, True)
        for _ in range(a.steps2d):
            s.inner_solve(g, x)
        torch.cuda.synchronize()
        tm = {cls: s.timer_read(cls) for cls in range(5)}
        for cls in range(5):
            s.timer(cls, False)
        s.timer(3, True)
        for _ in range(a.steps2d):
            s.inner_solve(g, x)
        torch.cuda.synchronize()
        vc = s.timer_read(3)
        s.timer(3, False)
        out = dict(T=T, its=its_all, tm=tm, n_skel=s.n_skel, n_cells=s.n_cells, vc=vc,
                   vc_design=s.query(12), vc_compulsory=s.query(13), t_setup=t_setup, t_assemble=t_assemble,
                   err=None if x_ref is None else float(np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)), x=xh)
        s.close()
        return out

    m64 = measure(0)
    progress("2D FP64 done")
    m32 = measure(1, m64["x"])
    m16 = measure(2, m64["x"])
    progress("2D mixed done")

    def classes(tm_):
        return {KCLASS.get(c_, "MG_hp"): {"ms": tm_[c_][0], "launches": tm_[c_][1], "GB": tm_[c_][2] / 1e9}
                for c_ in range(4)} | {COARSE_CLASS: {"ms": tm_[4][0], "launches": tm_[4][1], "GB": tm_[4][2] / 1e9}}

    def vcyc(m):
        ms, n, _ = m["vc"]
        avg = ms / max(n, 1) * 1e-3
        return {"avg_ms": 1e3 * avg, "compulsory_GB": m["vc_compulsory"] / 1e9,
                "compulsory_GB_per_s": m["vc_compulsory"] / avg / 1e9,
                "frac_of_hbm_peak": m["vc_compulsory"] / avg / 1e9 / PEAK_HBM_GBS,
                "implementation_GB": m["vc_design"] / 1e9,
                "implementation_GB_per_s": m["vc_design"] / avg / 1e9,
                "timing": "HIP events around each graph replay of MG_hp"}

    ms, n_l, by = m64["tm"][ROOF_CLASS]
    n = m64["n_skel"]
    return {"workload": f"2D generalized Stokes, 256x256 structured triangulation ({m64['n_cells']} cells, 7 levels), "
                        f"k=2, beta=1, nu=1, gamma=1e2; inner solve #1 to rel.res 1e-8",
            "n_skel": n, "value": n * a.steps2d / m64["T"], "unit": "skeleton DOFs/s",
            "ms_per_step": 1e3 * m64["T"] / a.steps2d, "iterations": m64["its"],
            "vcycle": vcyc(m64), "kernel_classes": classes(m64["tm"]),
            "cell_apply": {"avg_us": 1e3 * ms / n_l, "algorithmic_bytes_per_launch": by / n_l,
                           "GB_per_s": by / n_l / (ms / n_l * 1e-3) / 1e9},
            "colour_phase": {"avg_us": 1e3 * m64["tm"][0][0] / max(m64["tm"][0][1], 1),
                             "algorithmic_bytes_per_launch": m64["tm"][0][2] / max(m64["tm"][0][1], 1),
                             "GB_per_s": m64["tm"][0][2] / max(m64["tm"][0][0] * 1e-3, 1e-30) / 1e9,
                             "kernel": KCLASS[0]},
            "setup_s": m64["t_setup"], "assemble_s": m64["t_assemble"],
            "mixed": {"value": n * a.steps2d / m32["T"], "iterations": m32["its"],
                      "rel_diff_vs_fp64_solution": m32["err"], "vcycle": vcyc(m32),
                      "precision": "V-cycle operators FP32; vectors, accumulation and FCG FP64"},
            "mixed_fp16": {"value": n * a.steps2d / m16["T"], "iterations": m16["its"],
                           "rel_diff_vs_fp64_solution": m16["err"], "vcycle": vcyc(m16),
                           "precision": "order-k cell blocks and patch inverses FP16 (scaled), other "
                                        "V-cycle operators FP32; vectors, accumulation and FCG FP64"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k", type=int, default=3, help="order of the headline cube workload (2 or 3)")
    ap.add_argument("--steps2d", type=int, default=5)
    ap.add_argument("--timer-steps", type=int, default=1)
    ap.add_argument("--cpu-reps", type=int, default=2)
    ap.add_argument("--cpu-workers", type=int, default=0, help="0: min(16, host cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the triangular-mesh workloads")
    ap.add_argument("--no-oseen", action="store_true", help="skip the lid-driven cavity Picard workload")
    ap.add_argument("--picard-steps", type=int, default=10)
    ap.add_argument("--re", type=float, default=100.0)
    ap.add_argument("--alg3-re", type=float, default=1000.0, help="Reynolds number of the Alg. 3 cavity")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the batch-gradient workload")
    ap.add_argument("--adjoint-rhs", type=int, default=16)
    ap.add_argument("--n-refine", type=int, default=6)
    ap.add_argument("--sweep", action="store_true",
                    help="parameter sweeps instead of the bench line: the 256x256 generalized Stokes "
                         "workload over k, beta, gamma and V-cycle precision, and the cavity over Re; "
                         "one JSON line per case, then a summary line")
    ap.add_argument("--tables", choices=["cavity", "step"], default=None,
                    help="the paper's Stokes and Navier-Stokes cavity or step runs (one JSON line per case)")
    ap.add_argument("--profile-solves", type=int, default=2)
    ap.add_argument("--profile-prec", type=int, default=0, choices=[0, 1, 2, 3],
                    help="vcycle_precision of the profile run (2: triangles only; 3: tetrahedra only)")
    ap.add_argument("--profile-dim", type=int, default=3, choices=[2, 3],
                    help="--profile-run on the tetrahedral cube (3) or the 256x256 triangle workload (2)")
    ap.add_argument("--profile-run", action="store_true",
                    help="counter-collection run: a 1 GiB device copy (calibration of the HBM "
                         "counters) then two FP64 inner solves of the cube workload; prints a summary only")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {a.gpus} is not supported "
              "(a context holds the whole mesh; sharding across GPUs is not implemented).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    cpu = None
    if not (a.no_cpu_baseline or a.sweep or a.profile_run or a.tables):
        # before anything touches the GPU: the workers are forked
        workers = a.cpu_workers or min(16, os.cpu_count() or 1)
        progress(f"CPU oracle baseline on {workers} processes")
        cpu = cpu_baseline(a.k, a.cpu_reps, workers)
    import torch
    import paper_2303_06762_amd as hd
    import synth

    torch.cuda.set_device(0)
    c, t = synth.kuhn_square(4)
    if a.sweep:
        sweep(hd, synth, torch, np, c, t, a)
        return
    if a.tables:
        (paper_tables if a.tables == "cavity" else step_tables)(hd, synth, torch, np)
        return
    if a.profile_run:
        # calibration: an elementwise kernel reading exactly 1 GiB and
        # writing exactly 1 GiB
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        if a.profile_dim == 2:
            # the triangle workload of the 2D line: 256x256, k = 2, gamma = 1e2
            s = hd.Solver(c, t, a.n_refine, 2, 1.0, 1.0, 1e2, atol=0.0, vcycle_precision=a.profile_prec)
        else:
            c3, t3 = synth.kuhn_cube(4)
            s = hd.Solver(c3, t3, 3, a.k, 1.0, 1.0, 1e3, atol=0.0, m_relax=2, m_smooth=2,
                          vcycle_precision=a.profile_prec)
        s.assemble()
        g = torch.ones(s.n_skel, dtype=torch.float64, device="cuda")
        x = torch.empty_like(g)
        for _ in range(a.profile_solves):
            _, its, rel, st = s.inner_solve(g, x)
        torch.cuda.synchronize()
        out = {"profile_run": True, "n_skel": s.n_skel, "iterations": its}
        if a.profile_dim == 2:
            # per level: lowest-order unknowns and nonzeros of the transfer
            # into it (the counter summaries price the launches with these)
            out["levels"] = [{"level": l, "n_lo": s.query(9, l),
                              "transfer_nnz": s.query(14, l) if l else 0}
                             for l in range(s.query(3))]
        print(json.dumps(out))
        return

    # mixed storage: FP32 cell blocks (AL term apart, FP64) and lowest-order
    # operators; the order-k edge-patch inverses FP64 at k = 3 (precision 3;
    # all-FP32 storage does not converge there at this size) and FP32 at k = 2
    mixed_prec = {2: 1, 3: 3}
    m64 = stokes3d(hd, synth, torch, np, a.k, 0, a.steps, a.warmup, a.timer_steps)
    m32 = stokes3d(hd, synth, torch, np, a.k, mixed_prec[a.k], a.steps, a.warmup, a.timer_steps, m64["x"])
    k_other = 2 if a.k == 3 else 3
    o64 = stokes3d(hd, synth, torch, np, k_other, 0, 1, 1, a.timer_steps)
    o32 = stokes3d(hd, synth, torch, np, k_other, mixed_prec[k_other], 1, 1, 0, o64["x"])
    tm = m64["tm"]
    by_time = max((0, 1, 2), key=lambda c_: tm[c_][0])
    ms, n_l, by = tm[by_time]
    achieved = (by / n_l) / (ms / n_l * 1e-3) / 1e9
    copy_gbs = copy_bandwidth(torch)
    n_skel = m64["n_skel"]
    wl = (f"3D generalized Stokes, unit cube, 4^3 Kuhn cubes refined 3 times (32^3 cubes, {m64['n_cells']} "
          f"tetrahedra, {m64['levels']} levels), k={a.k}, beta=1, nu=1, gamma=1e3, edge patches, m_p=m_h=2; "
          f"inner solve #1 to rel.res 1e-8")
    out = {
        "metric": "skeleton DOFs solved/s to rel.res 1e-8 (FP64 vs mixed); V-cycle HBM GB/s",
        "value": n_skel * a.steps / m64["T"],
        "unit": "skeleton DOFs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * m64["T"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl, "n_skel": n_skel, "iterations": m64["its"], "status": m64["status"],
                   "precision": "FP64 operators, vectors and Krylov"},
        "mixed": {"value": n_skel * a.steps / m32["T"], "unit": "skeleton DOFs/s",
                  "ms_per_step": 1e3 * m32["T"] / a.steps, "iterations": m32["its"],
                  "rel_diff_vs_fp64_solution": m32["err_vs_fp64"],
                  "precision": ("V-cycle operators stored FP32 (cell blocks without their AL term, which is "
                                "applied apart in FP64; CR levels, transfers, coarsest inverse)"
                                + (", order-k edge-patch inverses FP64" if mixed_prec[a.k] == 3
                                   else ", edge-patch inverses FP32")
                                + "; vectors, accumulation and the flexible CG FP64; same rel.res 1e-8 on the "
                                  "FP64 operator"),
                  "vcycle": vcycle3(m32), "kernel_classes": classes3(m32["tm"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": COUNTER_TRAFFIC.get((KCLASS3[by_time], a.k)),
                     "traffic_source": COUNTER_SOURCE if (KCLASS3[by_time], a.k) in COUNTER_TRAFFIC else None,
                     "kernel": KCLASS3[by_time], "launches": n_l, "avg_us": 1e3 * ms / n_l,
                     "algorithmic_bytes_per_launch": by / n_l,
                     "bytes_model": "per colour phase (block Gauss-Seidel in the direct form x_s = "
                                    "A_ss^-1 (b_s - A_sr x_r)): for each edge patch its inverse and, for each "
                                    "patch cell, the coupling of its patch faces to its far faces in S_K, each "
                                    "entry read once in the stored (FP64, full) layout, plus the patch's "
                                    "vectors; the first phase from zero: inverses and vectors only",
                     "copy_GB_per_s": copy_gbs},
        "vcycle": vcycle3(m64),
        "kernel_classes": classes3(tm),
        "setup_s": m64["t_setup"], "assemble_s": m64["t_assemble"],
        f"k{k_other}": {"workload": wl.replace(f"k={a.k}", f"k={k_other}"), "n_skel": o64["n_skel"],
                        "value": o64["n_skel"] / o64["T"], "iterations": o64["its"],
                        "mixed_value": o32["n_skel"] / o32["T"], "mixed_iterations": o32["its"],
                        "mixed_precision": "as the headline's mixed entry" + (
                            " but with FP32 edge-patch inverses" if mixed_prec[k_other] == 1
                            else " with FP64 order-k edge-patch inverses"),
                        "mixed_rel_diff_vs_fp64_solution": o32["err_vs_fp64"],
                        "vcycle": vcycle3(o64), "kernel_classes": classes3(o64["tm"]),
                        "assemble_s": o64["t_assemble"]},
    }
    del m64, m32, o64, o32
    if not a.no_2d:
        out["stokes2d"] = stokes2d_line(hd, synth, torch, np, a)
        if not a.no_oseen:
            out["oseen"] = oseen_workload(hd, synth, torch, np, a.picard_steps, a.re)
            progress("cavity Picard done")
            out["alg3"] = alg3_workload(hd, synth, torch, np, a.alg3_re)
            progress("Alg. 3 done")
        if not a.no_adjoint:
            out["adjoint"] = adjoint_workload(hd, synth, torch, np, a.adjoint_rhs)
            progress("batch gradient done")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
