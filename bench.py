#!/usr/bin/env python3
"""Throughput of the hp-multigrid preconditioned skeleton solve on one MI355X.

Workload: 2D generalized Stokes on the unit square, 4x4 structured coarse
mesh refined 6 times (256x256 squares, 131072 triangles, 7 levels), order
k = 2, beta = 1, nu = 1, gamma = eps^-1 = 1e2; f = uniform[-1,1) per data
point (seed 0) plus the gradient of a seeded trigonometric polynomial.
A step is inner solve #1 of the AL-Uzawa iteration: A^eps lambda = g from
lambda = 0 by flexible CG preconditioned by MG_hp (variable V-cycle,
m_p = m_h = 1) to relative residual 1e-8, every operation in the HIP
library, the condensed load g already resident in HBM.

Prints one JSON line (metric, value = skeleton DOFs solved per second,
roofline of the dominant kernel from live HIP-event timing, the V-cycle's
achieved bandwidth, and the CPU oracle timed on a bounded sample).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KCLASS = {0: "order-k vertex-patch Gauss-Seidel colour phase (k_gs)",
          1: "order-k skeleton apply (k_apply)",
          2: "lowest-order patch Gauss-Seidel phases (k_gs, all CR levels)"}


def cpu_baseline(k, beta, gamma, reps):
    """The CPU oracle, untuned, on a bounded sample of the same workload:
    32x32 squares (2048 cells, 4 levels), same k, beta, nu, gamma and f
    recipe; inner solve #1 timed `reps` times (setup excluded)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import solver
    with threadpool_limits(1):
        c, t = synth.kuhn_square(4)
        S = solver.Setup(c, t, 3, k, 1.0, beta, gamma)
        nq = (k + 2) ** 2
        X = np.array([e.xq for e in S.prob.elems])
        f = synth.source_uniform(0, 1, S.lv.n_cells, nq)[0] + synth.trig_gradient(X, 1)
        g = S.prob.rhs(f)
        t0 = time.perf_counter()
        for _ in range(reps):
            _, its, _ = S.inner(g, atol=0.0)
        dt = time.perf_counter() - t0
    n = S.Aeps.shape[0]
    return {"value": n * reps / dt, "unit": "skeleton DOFs/s", "cores": 1, "kind": "oracle",
            "sample": f"32x32 squares (2048 cells, 4 levels), k={k}, N_skel={n}, inner solve #1 "
                      f"({its} its) x{reps}, numpy/scipy single thread, setup excluded",
            "seconds": round(dt, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--n-refine", type=int, default=6)
    ap.add_argument("--beta", type=float, default=1.0)
    ap.add_argument("--gamma", type=float, default=1e2)
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {a.gpus} is not supported "
              "(see the sharding notes in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2303_06762_amd as hd
    import synth

    torch.cuda.set_device(0)
    c, t = synth.kuhn_square(4)
    t0 = time.perf_counter()
    s = hd.Solver(c, t, a.n_refine, a.k, a.beta, 1.0, a.gamma, atol=0.0)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    s.assemble()
    torch.cuda.synchronize()
    t_assemble = time.perf_counter() - t0
    X = s.data_points().cpu().numpy()
    f = synth.source_uniform(0, 1, s.n_cells, s.n_q)[0] + synth.trig_gradient(X, 1)
    f_dev = torch.as_tensor(f, device="cuda")
    g = s.rhs(f_dev)
    x = torch.empty_like(g)
    for _ in range(a.warmup):
        s.inner_solve(g, x)
    # timed region: K inner solves, nothing else
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_all = []
    for _ in range(a.steps):
        _, its, rel, st = s.inner_solve(g, x)
        its_all.append(its)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    value = s.n_skel * a.steps / T
    # same work again with live per-kernel event timers
    for cls in range(4):
        s.timer(cls, True)
    torch.cuda.synchronize()
    for _ in range(a.steps):
        s.inner_solve(g, x)
    torch.cuda.synchronize()
    tm = {cls: s.timer_read(cls) for cls in range(4)}
    for cls in range(4):
        s.timer(cls, False)
    dom = max((0, 1, 2), key=lambda c_: tm[c_][0])
    ms, n_l, by = tm[dom]
    achieved = (by / n_l) / (ms / n_l * 1e-3) / 1e9
    vc_ms, vc_n, vc_b = tm[3]
    out = {
        "metric": "skeleton DOFs solved/s to rel.res 1e-8 (FP64 vs mixed); V-cycle HBM GB/s",
        "value": value,
        "unit": "skeleton DOFs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * T / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D generalized Stokes, {4 << a.n_refine}x{4 << a.n_refine} structured "
                               f"triangulation ({s.n_cells} cells, {s.levels} levels), k={a.k}, "
                               f"beta={a.beta:g}, nu=1, gamma={a.gamma:g}; inner solve #1 to rel.res 1e-8",
                   "n_skel": s.n_skel, "iterations": its_all, "precision": "fp64 (V-cycle fp64)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": KCLASS[dom], "launches": n_l, "avg_us": 1e3 * ms / n_l,
                     "algorithmic_bytes_per_launch": by / n_l},
        "vcycle": {"avg_ms": vc_ms / max(vc_n, 1), "algorithmic_GB": vc_b / max(vc_n, 1) / 1e9,
                   "GB_per_s": (vc_b / max(vc_n, 1)) / (vc_ms / max(vc_n, 1) * 1e-3) / 1e9},
        "kernel_classes": {KCLASS.get(c_, "MG_hp"): {"ms": tm[c_][0], "launches": tm[c_][1],
                                                      "GB": tm[c_][2] / 1e9} for c_ in range(4)},
        "setup_s": t_setup, "assemble_s": t_assemble,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.k, a.beta, a.gamma, a.cpu_reps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
