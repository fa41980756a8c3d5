"""GPU parity of the damped block Jacobi smoother (opts.smoother = 1, eq.
bjac) and of the additive MG_hp (opts.additive = 1, Remark 3.4) against the
oracle, on triangles and tetrahedra, through the C ABI.

FP64 bars: one MG_hp application within 1e-10 relative of the oracle's;
inner solves with iteration counts within +-1, the true residual of the
GPU iterate within the stopping tolerance 1e-8, and the two iterates within
1e-8 of each other (the solves stop at relative residual 1e-8, and the
Jacobi variants' longer Krylov recurrences carry the two sides' different
rounding further than the default preconditioner's).
"""
import numpy as np
import pytest

import synth
from oracle import solver, solver3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


SM = {0: "gs", 1: "jacobi"}

CASES2 = [  # (name, n, n_refine, k, beta, gamma, smoother, additive[, patch_relax, patch_smooth])
    ("k2_edge_smooth", 2, 2, 2, 1.0, 1e2, 0, 0, 1, 2),
    ("k1_edge_all", 2, 2, 1, 1.0, 1e4, 0, 0, 2, 2),
    ("k2_jacobi", 2, 2, 2, 1.0, 1e2, 1, 0),
    ("k0_jacobi", 2, 2, 0, 1.0, 1e4, 1, 0),
    ("k1_additive", 2, 2, 1, 1.0, 1e2, 0, 1),
    ("k3_jacobi_additive", 2, 2, 3, 0.0, 1e4, 1, 1),
    # 2048 cells: large enough that Gauss-Seidel would take the record and
    # single-workgroup forms; Jacobi runs launch by launch on every level
    ("k1_jacobi_2048", 2, 4, 1, 1.0, 1e2, 1, 0),
]


@pytest.mark.parametrize("case", CASES2, ids=[c[0] for c in CASES2])
def test_triangles(case):
    import paper_2303_06762_amd as hd
    name, n, nr, k, beta, gamma, sm, add = case[:8]
    pr, ps = case[8:] if len(case) > 8 else (0, 0)
    _note(f"smoother parity 2D {name}")
    c, t = synth.kuhn_square(n)
    P2 = {0: "vertex", 1: "vertex", 2: "edge"}
    O = solver.Setup(c, t, nr, k, 1.0, beta, gamma, smoother=SM[sm], additive=bool(add), patch_relax=P2[pr],
                     patch_smooth=P2[ps])
    s = hd.Solver(c, t, nr, k, beta, 1.0, gamma, smoother=sm, additive=add, patch_relax=pr, patch_smooth=ps)
    s.assemble()
    x = synth.uniform_pm1(1, 0, (s.n_skel,))
    assert rel(host(s.precondition(dev(x))), O.prec(x)) <= 1e-10
    b = synth.uniform_pm1(2, 0, (s.n_skel,))
    xg, its, rr, st = s.inner_solve(dev(b))
    xo, its_o, _ = O.inner(b)
    assert st == 0
    assert abs(its - its_o) <= 1, (its, its_o)
    assert np.linalg.norm(host(s.apply(xg)) - b) <= 1e-8 * np.linalg.norm(b)
    assert rel(host(xg), xo) <= 1e-8
    _note(f"  its {its} (oracle {its_o})")
    s.close()


PATCH = {0: "edge", 1: "vertex", 2: "edge"}

CASES3 = [  # (name, k, beta, gamma, smoother, additive, patch_relax, patch_smooth)
    ("k2_jacobi", 2, 1.0, 1e3, 1, 0, 0, 0),
    ("k1_additive", 1, 1.0, 1e3, 0, 1, 0, 0),
    ("k0_jacobi", 0, 1.0, 1e2, 1, 0, 0, 0),
    # vertex-patch relaxation with edge-patch smoothing (the paper's choice
    # for long domains), and vertex patches on every level
    ("k2_vertex_relax", 2, 1.0, 1e3, 0, 0, 1, 2),
    ("k1_vertex_all", 1, 0.0, 1e2, 0, 0, 1, 1),
    ("k3_vertex_relax_jacobi", 3, 1.0, 1e3, 1, 0, 1, 0),
]


@pytest.mark.parametrize("case", CASES3, ids=[c[0] for c in CASES3])
def test_tetrahedra(case):
    import paper_2303_06762_amd as hd
    name, k, beta, gamma, sm, add, pr, ps = case
    _note(f"smoother parity 3D {name}")
    c, t = synth.kuhn_cube(1)
    O = solver3d.Setup3(c, t, 1, k, 1.0, beta, gamma, smoother=SM[sm], additive=bool(add),
                        patch_relax=PATCH[pr], patch_smooth=PATCH[ps])
    s = hd.Solver(c, t, 1, k, beta, 1.0, gamma, m_relax=2, m_smooth=2, smoother=sm, additive=add,
                  patch_relax=pr, patch_smooth=ps)
    s.assemble()
    x = synth.uniform_pm1(1, 0, (s.n_skel,))
    assert rel(host(s.precondition(dev(x))), O.prec(x)) <= 1e-10
    b = synth.uniform_pm1(2, 0, (s.n_skel,))
    xg, its, rr, st = s.inner_solve(dev(b))
    xo, its_o, _ = O.inner(b)
    assert st == 0
    assert abs(its - its_o) <= 1, (its, its_o)
    assert np.linalg.norm(host(s.apply(xg)) - b) <= 1e-8 * np.linalg.norm(b)
    assert rel(host(xg), xo) <= 1e-8
    _note(f"  its {its} (oracle {its_o})")
    s.close()


def test_invalid_patch_options_are_refused():
    import paper_2303_06762_amd as hd
    c, t = synth.kuhn_square(2)
    with pytest.raises(hd.HdgmgError) as e:
        hd.Solver(c, t, 1, 1, 1.0, 1.0, 1e2, patch_relax=3)
    assert e.value.status == -1
    with pytest.raises(hd.HdgmgError) as e:
        hd.Solver(c, t, 1, 1, 1.0, 1.0, 1e2, smoother=2)
    assert e.value.status == -1
