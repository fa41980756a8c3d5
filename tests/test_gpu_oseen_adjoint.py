"""GPU parity of the adjoint of the Oseen system (opts.oseen = 1,
opts.transpose = 1) against the oracle's transposed system and dense
adjoint.

A forward context solves the Picard-linearised system at a fixed wind; an
adjoint context with the same wind assembles the transposed system and
runs hdgmg_solve_adjoint.  FP64 bars: the transposed order-k and
lowest-order blocks and one MG_hp application of A^T within 1e-10
relative of the oracle's transposed hierarchy; the misfit within 1e-8;
dJ/df and dJ/dnu within 1e-6 of the largest entry of the oracle's dense
adjoint; adjoint inner iteration counts within +-1 of the oracle's FGMRES
on the transposed system.  Mixed precision: the gradients within 1e-6 and
iteration counts at most the oracle's + 2.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint, hdg, mesh, oseen

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
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {
    # name: (n, n_refine, k, beta, wind scale, solver kwargs)
    "k1": (2, 2, 1, 1.0, 20.0, {}),
    "k2": (2, 2, 2, 1.0, 20.0, {}),
    "k3_beta0": (2, 2, 3, 0.0, 20.0, {}),
    "k0": (4, 1, 0, 1.0, 20.0, {}),
    "k2_stream_per_level": (2, 2, 2, 1.0, 20.0, dict(stream_dofs=0, coarse_dofs=0)),
    "k2_mixed": (2, 2, 2, 1.0, 20.0, dict(vcycle_precision=1)),
}

_ORACLE = {}


def oracle_case(name):
    if name in _ORACLE:
        return _ORACLE[name]
    n, nr, k, beta, scale, kw = CASES[name]
    c, t = synth.kuhn_square(n)
    levels = mesh.hierarchy(c, t, nr)
    lv = levels[-1]
    nq = (k + 2) ** 2
    nu = 0.1 * np.exp(0.5 * synth.normal(3, 0, lv.n_cells))
    # wind: a discrete Stokes velocity, scaled
    pr0 = hdg.Problem(lv, k, 1.0, 1.0, 1e2)
    f0 = synth.source_uniform(100, 1, lv.n_cells, nq)[0]
    lam0, p00 = pr0.solve_direct(f0)
    winds = [(lambda X, w=w: scale * w(X)) for w in oseen.state_wind(pr0, lam0, p00, f0)]
    wq = np.array([winds[K](pr0.elems[K].xq) for K in range(lv.n_cells)])
    f = synth.source_uniform(7, 1, lv.n_cells, nq)[0]
    ut = synth.source_uniform(4, 1, lv.n_cells, nq)[0]
    Sa = oseen.OseenSetup(levels, k, nu, beta, 1e2, winds, transpose=True)
    fwd = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds)
    J, gf, gnu, _ = adjoint.gradients(fwd, f, ut, prob_adj=Sa.prob)
    _ORACLE[name] = dict(c=c, t=t, levels=levels, nu=nu, wq=wq, f=f, ut=ut, Sa=Sa, fwd=fwd, J=J, gf=gf, gnu=gnu)
    return _ORACLE[name]


def gpu_solver(name, transpose):
    import paper_2303_06762_amd as hd
    n, nr, k, beta, scale, kw = CASES[name]
    o = oracle_case(name)
    s = hd.Solver(o["c"], o["t"], nr, k, beta, o["nu"], 1e2, oseen=1, transpose=transpose, **kw)
    s.set_wind(dev(o["wq"]))
    s.assemble()
    return s


@pytest.mark.parametrize("name", [n for n in CASES if "mixed" not in n])
def test_transposed_blocks_and_preconditioner(name):
    o = oracle_case(name)
    _note(f"oseen adjoint blocks {name}")
    s = gpu_solver(name, 1)
    Sa = o["Sa"]
    blocks = host(s.export(0))
    ref = np.array([e.S + Sa.eps_inv / e.area * np.outer(e.d, e.d) for e in Sa.prob.elems])
    assert rel(blocks, ref) < 1e-10
    # transposes of the forward blocks
    fb = np.array([e.S + Sa.eps_inv / e.area * np.outer(e.d, e.d) for e in o["fwd"].elems])
    assert rel(blocks, np.transpose(fb, (0, 2, 1))) < 1e-10
    beta = CASES[name][3]
    for l in range(len(o["levels"])):
        Bl = host(s.export(1, l))
        pr = oseen.OseenProblem(o["levels"][l], 0, Sa.hier.nus[l], beta, 1e2)
        B = pr._assemble(list(Bl)).toarray()
        assert rel(B, Sa.hier.A[l].toarray()) < 1e-10, l
    r = synth.uniform_pm1(11, 0, s.n_skel)
    z = host(s.precondition(dev(r)))
    assert rel(z, Sa.prec(r)) < 1e-10
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_oseen_adjoint_matches_dense_adjoint(name):
    o = oracle_case(name)
    mixed = "mixed" in name
    _note(f"oseen adjoint gradients {name}")
    sf = gpu_solver(name, 0)
    u, p, state, info, st = sf.solve(dev(o["f"]))
    assert st == 0, info
    uh = host(u)
    J1 = adjoint.misfit(o["fwd"], uh, o["ut"])
    assert abs(J1 - o["J"]) <= 1e-8 * abs(o["J"])
    gu = adjoint.misfit_grad(o["fwd"], uh, o["ut"])
    # the forward context refuses the adjoint of its nonsymmetric system
    import paper_2303_06762_amd as hd
    with pytest.raises(hd.HdgmgError):
        sf.solve_adjoint(dev(o["f"]), state, dev(gu))
    sa = gpu_solver(name, 1)
    gf, gnu, ast, ainfo, st = sa.solve_adjoint(dev(o["f"]), state, dev(gu))
    assert st == 0, ainfo
    gf1, gnu1 = host(gf), host(gnu)
    assert np.abs(gf1 - o["gf"]).max() <= 1e-6 * np.abs(o["gf"]).max(), np.abs(gf1 - o["gf"]).max()
    assert np.abs(gnu1 - o["gnu"]).max() <= 1e-6 * np.abs(o["gnu"]).max(), np.abs(gnu1 - o["gnu"]).max()
    # iteration counts of the transposed solve against the oracle's method
    W = adjoint.weights(o["fwd"])
    ref = o["Sa"].solve(gu / W[:, :, None])
    its_o, its_g = ref["its"], ainfo["its"]
    _note(f"  adjoint its gpu {its_g} oracle {its_o}")
    n = min(len(its_o), len(its_g))
    assert n >= 1 and abs(len(its_o) - len(its_g)) <= 1
    for a, b in zip(its_g[:n], its_o[:n]):
        assert (a <= b + 2) if mixed else abs(a - b) <= 1, (its_g, its_o)
    sf.close()
    sa.close()


@pytest.mark.parametrize("with_wind", [False, True])
def test_adjoint_with_lid_data(with_wind):
    # tangential Dirichlet data on the top side: the forward solve carries
    # the lid, the adjoint has homogeneous data, dJ/dnu keeps the lid in the
    # forward state's lifting
    import paper_2303_06762_amd as hd
    name = "k2"
    n, nr, k, beta, scale, kw = CASES[name]
    o = oracle_case(name)
    lv = o["levels"][-1]
    lid = oseen.lid_dirichlet(lv, k)
    bd = dev(np.array([lid[E] for E in np.where(lv.int_id < 0)[0]]))
    winds = None
    if with_wind:
        pr0 = hdg.Problem(lv, k, 1.0, 1.0, 1e2)
        f0 = synth.source_uniform(100, 1, lv.n_cells, (k + 2) ** 2)[0]
        lam0, p00 = pr0.solve_direct(f0)
        winds = [(lambda X, w=w: scale * w(X)) for w in oseen.state_wind(pr0, lam0, p00, f0)]
    fwd = oseen.OseenProblem(lv, k, o["nu"], beta, 1e2, winds, lid)
    adj = oseen.OseenProblem(lv, k, o["nu"], beta, 1e2, winds, transpose=True)
    J0, gf0, gnu0, _ = adjoint.gradients(fwd, o["f"], o["ut"], prob_adj=adj)
    _note(f"lid adjoint wind={with_wind}")

    def make(transpose):
        s = hd.Solver(o["c"], o["t"], nr, k, beta, o["nu"], 1e2, oseen=1 if with_wind else 0,
                      transpose=transpose, **kw)
        if with_wind:
            s.set_wind(dev(o["wq"]))
        s.set_dirichlet(bd)
        s.assemble()
        return s

    sf = make(0)
    u, p, state, info, st = sf.solve(dev(o["f"]))
    assert st == 0, info
    uh = host(u)
    assert abs(adjoint.misfit(fwd, uh, o["ut"]) - J0) <= 1e-8 * abs(J0)
    gu = adjoint.misfit_grad(fwd, uh, o["ut"])
    sa = make(1) if with_wind else sf
    gf, gnu, ast, ainfo, st = sa.solve_adjoint(dev(o["f"]), state, dev(gu))
    assert st == 0, ainfo
    gf1, gnu1 = host(gf), host(gnu)
    assert np.abs(gf1 - gf0).max() <= 1e-6 * np.abs(gf0).max(), np.abs(gf1 - gf0).max()
    assert np.abs(gnu1 - gnu0).max() <= 1e-6 * np.abs(gnu0).max(), np.abs(gnu1 - gnu0).max()
    # the forward context still solves with its lid afterwards
    u2, _, _, _, st = sf.solve(dev(o["f"]))
    assert st == 0 and np.abs(host(u2) - uh).max() <= 1e-12 * np.abs(uh).max()
    sf.close()
    if with_wind:
        sa.close()
