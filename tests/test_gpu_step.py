"""GPU parity on non-square domains with do-nothing outflow and an inflow
(Sec. 5.3), through the C ABI (hdgmg_mesh.outflow, hdgmg_set_dirichlet_full).

FP64 bars as for the square: cell blocks, load, apply and one MG_hp
application within 1e-10 of the oracle's; inner and AL-Uzawa solves with
counts within +-1 and iterates within 1e-9 (with the edge-patch smoother,
whose longer recurrences carry rounding further: 1e-8 for an inner solve,
the solve tolerance, 1e-7 for the chained AL-Uzawa solves); the Poiseuille flow of the
channel reproduced (k = 2, 3); on the step the outflow flux equals the
inflow's 1/3 and every cell is divergence free to the Uzawa tolerance.
"""
import numpy as np
import pytest

import synth
from oracle import solver

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _inflow_lv(lv, k):
    D = np.zeros((lv.n_facets, 2, k + 1))
    bnd = np.where(lv.int_id < 0)[0]
    D[bnd] = synth.boundary_coefficients(lv.coords[lv.edges[bnd]], k, synth.step_inflow)
    return D


def gpu(step, n_refine, k, nu=1.0, beta=0.0, gamma=1e3, **kw):
    import paper_2303_06762_amd as hd
    c, t, out = synth.step_domain(1, step=step)
    s = hd.Solver(c, t, n_refine, k, beta, nu, gamma, outflow=out, **kw)
    ends = host(s.boundary_facets())
    s.set_dirichlet_full(dev(synth.boundary_coefficients(ends, k, synth.step_inflow)))
    s.assemble()
    return s


@pytest.mark.parametrize("k", [2, 3])
def test_channel_poiseuille(k):
    nu = 0.7
    _note(f"channel Poiseuille k={k}")
    s = gpu(False, 2, k, nu=nu, uzawa_tol=1e-13, uzawa_max=64, rtol=1e-12, atol=0.0)
    f = np.zeros((s.n_cells, s.n_q, 2))
    u, p, state, info, st = s.solve(dev(f))
    assert st == 0
    X = host(s.data_points())
    ue = np.stack([16 * (1 - X[..., 1]) * (X[..., 1] - 0.5), 0 * X[..., 0]], axis=-1)
    assert np.abs(host(u) - ue).max() <= 1e-9
    assert np.abs(host(p) - 32 * nu * (4.0 - X[..., 0])).max() <= 1e-7
    s.close()


CASES = [  # (name, n_refine, k, beta, gamma[, patch_relax, patch_smooth])
    ("k0", 2, 0, 1.0, 1e2),
    ("k1", 2, 1, 0.0, 1e3),
    ("k2", 1, 2, 1e3, 1e2),
    ("k2_J3", 2, 2, 0.0, 1e3),
    # the paper's step setting: vertex-patch relaxation, edge-patch smoothing
    ("k2_J3_edge_smooth", 2, 2, 0.0, 1e3, 1, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_step_matches_oracle(case):
    name, nr, k, beta, gamma = case[:5]
    pr, ps = case[5:] if len(case) > 5 else (0, 0)
    _note(f"step parity {name}")
    c, t, out = synth.step_domain(1)
    P2 = {0: "vertex", 1: "vertex", 2: "edge"}
    O = solver.Setup(c, t, nr, k, 1.0, beta, gamma, outflow=out, dirichlet=lambda lv: _inflow_lv(lv, k),
                     patch_relax=P2[pr], patch_smooth=P2[ps])
    s = gpu(True, nr, k, beta=beta, gamma=gamma, patch_relax=pr, patch_smooth=ps)
    assert s.n_skel == O.Aeps.shape[0]
    lv = O.lv
    S = host(s.export(0))
    for K in range(0, lv.n_cells, max(1, lv.n_cells // 16)):
        e = O.prob.elems[K]
        assert rel(S[K], e.S + O.eps_inv / e.area * np.outer(e.d, e.d)) <= 1e-10
    f = synth.source_uniform(3, 1, s.n_cells, s.n_q)[0]
    x = synth.uniform_pm1(1, 0, (s.n_skel,))
    assert rel(host(s.apply(dev(x))), O.Aeps @ x) <= 1e-10
    assert rel(host(s.precondition(dev(x))), O.prec(x)) <= 1e-10
    b = synth.uniform_pm1(2, 0, (s.n_skel,))
    xg, its, rr, st = s.inner_solve(dev(b))
    xo, its_o, _ = O.inner(b)
    assert st == 0 and abs(its - its_o) <= 1, (its, its_o)
    # the edge-patch smoother's longer recurrences carry the two sides'
    # rounding further: its iterates agree to the solve tolerance
    bar = 1e-8 if (pr, ps) != (0, 0) else 1e-9
    assert np.linalg.norm(host(s.apply(xg)) - b) <= 1e-8 * np.linalg.norm(b)
    assert rel(host(xg), xo) <= bar
    # full solve with the inflow: the load carries the lift of the
    # prescribed values, the Uzawa loop their flux
    u, p, state, info, st = s.solve(dev(f))
    ref = O.solve(f)
    # beta = 1e3 with eps^-1 = 1e2 contracts slowly (Lemma 3.1): both sides
    # stop at the 50-step cap, the library saying so
    assert st == (1 if len(ref["its"]) == 50 else 0)
    assert len(info["its"]) == len(ref["its"])
    assert all(abs(a - b_) <= 1 for a, b_ in zip(info["its"], ref["its"])), (info["its"], ref["its"])
    # (the full solve chains one inner solve per Uzawa step)
    fbar = 1e-9 if (pr, ps) == (0, 0) else 1e-7
    lam = host(state)[:s.n_skel]
    assert rel(lam, ref["lam"]) <= fbar
    assert rel(host(state)[s.n_skel:], ref["p0"]) <= 10 * fbar
    uo, po, _, _ = O.prob.recover(ref["lam"], ref["p0"], f)
    assert rel(host(u), uo) <= fbar
    assert rel(host(p), po) <= 10 * fbar
    # mass: every cell divergence free with the inflow flux, so the outflow
    # flux is the inflow's 1/3
    # (checked where the Uzawa loop converged)
    if st == 0:
        D = O.prob.matrix_D()
        assert np.abs(D @ lam + O.prob.flux_b()).max() <= 1e-8
        m = k + 1
        flux = 0.0
        for E in np.where(lv.outflow)[0]:
            K, i = lv.facet_cells[E, 0], lv.facet_local[E, 0]
            flux += lv.sigma[K, i] * lv.length[E] * lam[(lv.int_id[E] * 2) * m]
        assert abs(flux - 1.0 / 3.0) <= 1e-7
    _note(f"  its {info['its']} (oracle {ref['its']})")
    s.close()


def test_step_level5_properties():
    # the paper's step at level 5 (15 coarse squares refined four times,
    # 7680 cells), k = 2, (nu eps)^-1 = 1e6 with two Uzawa steps: the
    # solves converge in a bounded count and the flow leaves through the
    # do-nothing boundary with the inflow's flux
    _note("step level 5 k=2")
    s = gpu(True, 4, 2, gamma=1e6, uzawa_max=2, uzawa_tol=-1.0)
    f = np.zeros((s.n_cells, s.n_q, 2))
    u, p, state, info, st = s.solve(dev(f))
    assert st == 0 and max(info["its"]) <= 40, info["its"]
    U = host(u)
    X = host(s.data_points())
    W = host(s.data_weights())
    # the velocity is divergence free with no flux through the walls, so
    # every vertical section x = c > 0.5 carries the inflow's 1/3 and
    # int_{x > 0.5} u_x = 3.5 / 3 (the data rule integrates u_x exactly)
    inner = X[..., 0] > 0.5
    q = np.sum((W * U[..., 0])[inner]) / 3.5
    assert abs(q - 1.0 / 3.0) <= 1e-6, q
    s.close()


def test_step_oseen_matches_oracle():
    # an Oseen system on the step (the wind a discrete Stokes velocity of
    # the step, the inflow data, do-nothing outflow): blocks, MG_hp and the
    # AL-Uzawa + FGMRES solve as the oracle's
    import paper_2303_06762_amd as hd
    from oracle import hdg, mesh, oseen
    k, nu, nr = 2, 0.05, 2
    c, t, out = synth.step_domain(1)
    levels = mesh.hierarchy(c, t, nr, out)
    lv = levels[-1]
    nq = (k + 2) ** 2
    D = _inflow_lv(lv, k)
    pr0 = oseen.OseenProblem(lv, k, 1.0, 0.0, 1e2, None, D)
    f0 = np.zeros((lv.n_cells, nq, 2))
    lam0, p00 = pr0.solve_direct(f0)
    winds = oseen.state_wind(pr0, lam0, p00, f0)
    wq = np.array([winds[K](pr0.elems[K].xq) for K in range(lv.n_cells)])
    _note("step oseen k=2")
    S = oseen.OseenSetup(levels, k, nu, 0.0, 1e2, winds, D)
    s = hd.Solver(c, t, nr, k, 0.0, nu, 1e2, oseen=1, outflow=out)
    ends = host(s.boundary_facets())
    s.set_dirichlet_full(dev(synth.boundary_coefficients(ends, k, synth.step_inflow)))
    s.set_wind(dev(wq))
    s.assemble()
    ref_b = np.array([e.S + S.eps_inv / e.area * np.outer(e.d, e.d) for e in S.prob.elems])
    assert rel(host(s.export(0)), ref_b) <= 1e-10
    r = synth.uniform_pm1(11, 0, (s.n_skel,))
    assert rel(host(s.precondition(dev(r))), S.prec(r)) <= 1e-10
    f = synth.source_uniform(7, 1, lv.n_cells, nq)[0]
    u, p, state, info, st = s.solve(dev(f))
    ref = S.solve(f)
    assert st == 0
    assert all(abs(a - b_) <= 1 for a, b_ in zip(info["its"], ref["its"])), (info["its"], ref["its"])
    assert rel(host(state)[:s.n_skel], ref["lam"]) <= 1e-9
    uo, _, _, _ = S.prob.recover(ref["lam"], ref["p0"], f)
    assert rel(host(u), uo) <= 1e-9
    s.close()


def test_channel_navier_stokes_poiseuille():
    # Alg. 3 in the library on the channel: the Poiseuille flow solves the
    # Navier-Stokes equations with p = 32 nu (4 - x), reproduced at k = 2
    # (the do-nothing facets' convection term on both sides)
    import paper_2303_06762_amd as hd
    nu, k = 0.05, 2
    _note("channel Navier-Stokes Poiseuille k=2")
    c, t, out = synth.step_domain(1, step=False)
    # (the Uzawa stop sits above the rounding floor of the pressure update,
    # about 1e-12 with inner solves to rel. res. 1e-12)
    s = hd.Solver(c, t, 2, k, 0.0, nu, 1e2, oseen=1, outflow=out, uzawa_tol=1e-12, uzawa_max=64, rtol=1e-12,
                  atol=0.0)
    ends = host(s.boundary_facets())
    s.set_dirichlet_full(dev(synth.boundary_coefficients(ends, k, synth.step_inflow)))
    f = np.zeros((s.n_cells, s.n_q, 2))
    res = hd.picard_newton(s, dev(f), eps_picard=1e-3, newton_rtol=1e-12, newton_atol=1e-13, max_newton=6)
    assert res[-1]["kind"] == "newton" and all(o["status"] == 0 for o in res)
    X = host(s.data_points())
    u, p = host(res[-1]["u"]), host(res[-1]["p"])
    assert np.abs(u[..., 0] - 16 * (1 - X[..., 1]) * (X[..., 1] - 0.5)).max() <= 1e-8
    assert np.abs(u[..., 1]).max() <= 1e-8
    assert np.abs(p - 32 * nu * (4.0 - X[..., 0])).max() <= 1e-6
    s.close()


def test_step_alg3_matches_oracle():
    # Alg. 3 on the step (level 3, k = 2, nu = 1e-2): the step kinds, every
    # step's velocity and inner counts as the oracle's Alg. 3
    import paper_2303_06762_amd as hd
    from oracle import mesh, oseen
    k, nu, nr, gamma = 2, 1e-2, 2, 1e2
    c, t, out = synth.step_domain(1)
    levels = mesh.hierarchy(c, t, nr, out)
    lv = levels[-1]
    D = _inflow_lv(lv, k)
    f = np.zeros((lv.n_cells, (k + 2) ** 2, 2))
    _note("step alg3 k=2 nu=1e-2")
    ref = oseen.picard_newton(levels, k, nu, 0.0, gamma, f, D, eps_picard=1e-3, max_picard=30, max_newton=6)
    s = hd.Solver(c, t, nr, k, 0.0, nu, gamma, oseen=1, outflow=out)
    ends = host(s.boundary_facets())
    s.set_dirichlet_full(dev(synth.boundary_coefficients(ends, k, synth.step_inflow)))
    res = hd.picard_newton(s, dev(f), eps_picard=1e-3, max_picard=30, max_newton=6)
    assert [o["kind"] for o in res] == [r["kind"] for r in ref]
    for o_, r_ in zip(res, ref):
        assert o_["status"] == 0
        assert rel(host(o_["u"]), r_["u"]) < 1e-7
        for a, b_ in zip(o_["info"]["its"], r_["its"]):
            assert abs(a - b_) <= 1, (o_["info"]["its"], r_["its"])
    _note(f"  {len(res)} steps")
    s.close()
