"""GPU parity of the adjoint solve (hdgmg_solve_adjoint) and its autograd
wrapper against the oracle's dense adjoint.

Bars: the misfit within 1e-8 relative, dJ/df and dJ/dnu within 1e-6 of the
largest entry (both sides solve to relative residual 1e-8 / Uzawa 1e-10;
the oracle's reference is the direct solve).  At the 128x128 size, where
the oracle's direct solve is too slow, two identities that hold at any size
are checked instead: the transpose identity <gu, du(df)> = <gf, df> and, for
beta = 0, Euler's identity sum_K nu_K dJ/dnu_K = -<gu, u>.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint, hdg, mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def jittered_square(n, seed, amp=0.2):
    c, t = synth.kuhn_square(n)
    h = 1.0 / n
    inner = (c[:, 0] > 0) & (c[:, 0] < 1) & (c[:, 1] > 0) & (c[:, 1] < 1)
    d = synth.uniform_pm1(seed, 7, c.shape) * amp * h
    c = c.copy()
    c[inner] += d[inner]
    return c, t


CASES = {
    # name: (mesh, n_refine, k, beta, gamma, solver kwargs)
    "k2_lognormal": (lambda: synth.kuhn_square(4), 1, 2, 1.0, 1e2, {}),
    "k1_beta0_jittered": (lambda: jittered_square(4, 5), 1, 1, 0.0, 1e2, {}),
    "k3_stream": (lambda: synth.kuhn_square(2), 2, 3, 1.0, 1e2, dict(stream_dofs=0)),
    "k2_mixed": (lambda: synth.kuhn_square(4), 1, 2, 1.0, 1e2, dict(vcycle_precision=1, stream_dofs=0)),
}


def lognormal_nu(n_cells, seed=3):
    return np.exp(0.5 * synth.normal(seed, 0, n_cells))


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_dense_adjoint(name):
    import paper_2303_06762_amd as hd
    mk, nr, k, beta, gamma, kw = CASES[name]
    c, t = mk()
    lv = mesh.hierarchy(c, t, nr)[-1]
    nu = lognormal_nu(lv.n_cells)
    nq = (k + 2) ** 2
    f = synth.source_uniform(100, 1, lv.n_cells, nq)[0]
    ut = synth.source_uniform(4, 1, lv.n_cells, nq)[0]
    prob = hdg.Problem(lv, k, nu, beta, gamma)
    J0, gf0, gnu0, _ = adjoint.gradients(prob, f, ut)
    _note(f"adjoint case {name}: {lv.n_cells} cells, k={k}")
    s = hd.Solver(c, t, nr, k, beta, nu, gamma, **kw)
    s.assemble()
    u, p, state, info, st = s.solve(dev(f))
    assert st == 0, info
    uh = host(u)
    J1 = adjoint.misfit(prob, uh, ut)
    assert abs(J1 - J0) <= 1e-8 * abs(J0)
    gu = adjoint.misfit_grad(prob, uh, ut)
    gf, gnu, ast, ainfo, st = s.solve_adjoint(dev(f), state, dev(gu))
    assert st == 0, ainfo
    gf1, gnu1 = host(gf), host(gnu)
    assert np.abs(gf1 - gf0).max() <= 1e-6 * np.abs(gf0).max(), np.abs(gf1 - gf0).max()
    assert np.abs(gnu1 - gnu0).max() <= 1e-6 * np.abs(gnu0).max(), np.abs(gnu1 - gnu0).max()
    # gnu accumulates: a second call adds the same gradient again
    gf2, gnu2, _, _, st = s.solve_adjoint(dev(f), state, dev(gu), gnu=gnu)
    assert np.abs(host(gnu2) - 2 * gnu1).max() <= 1e-9 * np.abs(gnu1).max()
    s.close()


def test_autograd_batch_matches_oracle():
    import paper_2303_06762_amd as hd
    c, t = synth.kuhn_square(4)
    nr, k, beta, gamma = 1, 2, 1.0, 1e2
    lv = mesh.hierarchy(c, t, nr)[-1]
    nu = lognormal_nu(lv.n_cells)
    nq = (k + 2) ** 2
    nrhs = 3
    F = synth.source_uniform(100, nrhs, lv.n_cells, nq)
    ut = synth.source_uniform(4, 1, lv.n_cells, nq)[0]
    prob = hdg.Problem(lv, k, nu, beta, gamma)
    W = adjoint.weights(prob)
    Jo, gfo, gnuo = 0.0, [], np.zeros(lv.n_cells)
    for i in range(nrhs):
        J_, gf_, gnu_, _ = adjoint.gradients(prob, F[i], ut)
        Jo += J_
        gfo.append(gf_)
        gnuo += gnu_
    gfo = np.array(gfo)
    _note("autograd batch: 3 sources, 128 cells, k=2")
    s = hd.Solver(c, t, nr, k, beta, nu, gamma)
    s.assemble()
    Wg = host(s.data_weights())
    assert np.abs(Wg - W).max() <= 1e-14 * np.abs(W).max()
    f_t = dev(F).requires_grad_(True)
    nu_t = dev(nu).requires_grad_(True)
    u = hd.stokes_solve(s, f_t, nu_t)
    J = (dev(W)[None, :, :, None] * (u - dev(ut)[None]) ** 2).sum()
    J.backward()
    assert abs(J.item() - Jo) <= 1e-8 * abs(Jo)
    assert np.abs(host(f_t.grad) - gfo).max() <= 1e-6 * np.abs(gfo).max()
    assert np.abs(host(nu_t.grad) - gnuo).max() <= 1e-6 * np.abs(gnuo).max()
    s.close()


@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_adjoint_identities_at_128x128(beta):
    # 128x128 squares (32768 cells, 6 levels), k = 2, gamma = 1e2,
    # log-normal per-cell viscosity: the batch-gradient workload's size.
    import paper_2303_06762_amd as hd
    c, t = synth.kuhn_square(4)
    nr, k, gamma = 5, 2, 1e2
    n_cells = 16 * 2 * 4 ** nr
    nu = lognormal_nu(n_cells)
    _note(f"adjoint identities 128x128 beta={beta}")
    s = hd.Solver(c, t, nr, k, beta, nu, gamma)
    s.assemble()
    nq = s.n_q
    f = dev(synth.source_uniform(100, 1, n_cells, nq)[0])
    ut = dev(synth.source_uniform(4, 1, n_cells, nq)[0])
    u, _, state, info, st = s.solve(f)
    assert st == 0
    # any gu defines a linear functional <gu, u> for which both identities hold
    gu = 2.0 * (u - ut)
    gf, gnu, _, ainfo, st = s.solve_adjoint(f, state, gu)
    assert st == 0
    df = dev(synth.source_uniform(51, 1, n_cells, nq)[0])
    du, _, _, _, st = s.solve(df)
    assert st == 0
    lhs, rhs = float((gu * du).sum()), float((gf * df).sum())
    assert abs(lhs - rhs) <= 1e-7 * (gu.abs() * du.abs()).sum().item()
    if beta == 0.0:
        e_lhs = float((dev(nu) * gnu).sum())
        e_rhs = -float((gu * u).sum())
        assert abs(e_lhs - e_rhs) <= 1e-6 * abs(e_rhs)
    s.close()


def test_stream_pool_batch_matches_single_solver():
    # the batch spread over four contexts on four HIP streams (solves
    # running concurrently) gives the single context's results
    import paper_2303_06762_amd as hd
    c, t = synth.kuhn_square(4)
    nr, k, beta, gamma = 1, 2, 1.0, 1e2
    n_cells = 32 * 4 ** nr
    nu = lognormal_nu(n_cells)
    nq = (k + 2) ** 2
    nrhs = 6
    F = synth.source_uniform(100, nrhs, n_cells, nq)
    ut = dev(synth.source_uniform(4, 1, n_cells, nq)[0])
    _note("stream pool: 6 sources over 4 streams")
    s = hd.Solver(c, t, nr, k, beta, nu, gamma)
    s.assemble()
    W = s.data_weights()
    pool = hd.solver_pool(4, c, t, nr, k, beta, nu, gamma)
    res = []
    for solver in (s, pool):
        f_t = dev(F).requires_grad_(True)
        nu_t = dev(nu).requires_grad_(True)
        u = hd.stokes_solve(solver, f_t, nu_t)
        J = (W[None, :, :, None] * (u - ut[None]) ** 2).sum()
        J.backward()
        res.append((host(u), J.item(), host(f_t.grad), host(nu_t.grad)))
    (u0, J0, gf0, gn0), (u1, J1, gf1, gn1) = res
    assert np.abs(u1 - u0).max() <= 1e-12 * np.abs(u0).max()
    assert abs(J1 - J0) <= 1e-12 * abs(J0)
    assert np.abs(gf1 - gf0).max() <= 1e-12 * np.abs(gf0).max()
    assert np.abs(gn1 - gn0).max() <= 1e-12 * np.abs(gn0).max()
    for p_ in pool:
        p_.close()
    s.close()


def test_native_batch_calls():
    # hdgmg_solve_batch / hdgmg_solve_adjoint_batch over three contexts
    # against one context's single solves; a context given twice is refused
    import paper_2303_06762_amd as hd
    c, t = synth.kuhn_square(4)
    nr, k, beta, gamma = 1, 2, 1.0, 1e2
    n_cells = 32 * 4 ** nr
    nu = lognormal_nu(n_cells)
    nq = (k + 2) ** 2
    F = dev(synth.source_uniform(200, 5, n_cells, nq))
    GU = dev(synth.source_uniform(300, 5, n_cells, nq))
    _note("native batch: 5 sources over 3 contexts")
    s = hd.Solver(c, t, nr, k, beta, nu, gamma)
    s.assemble()
    pool = hd.solver_pool(3, c, t, nr, k, beta, nu, gamma)
    U, P, S, infos = hd.solve_batch(pool, F)
    gf_b, gnu_b = hd.solve_adjoint_batch(pool, F, S, GU)
    gnu1 = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
    for i in range(5):
        u, p, st_, info, st = s.solve(F[i])
        assert st == 0 and infos[i]["its"] == info["its"]
        assert (U[i] - u).abs().max().item() <= 1e-12 * u.abs().max().item()
        assert (P[i] - p).abs().max().item() <= 1e-12 * p.abs().max().item()
        gf, _, _, _, st = s.solve_adjoint(F[i], st_, GU[i], gnu=gnu1)
        assert st == 0
        assert (gf_b[i] - gf).abs().max().item() <= 1e-12 * gf.abs().max().item()
    assert (gnu_b - gnu1).abs().max().item() <= 1e-12 * gnu1.abs().max().item()
    with pytest.raises(hd.HdgmgError) as e:
        hd.solve_batch([pool[0], pool[1], pool[0]], F)
    assert e.value.status == -1
    for p_ in pool:
        p_.close()
    s.close()


def test_nrhs_entry_points():
    # hdgmg_solve and hdgmg_solve_adjoint with nrhs = 3 on one context
    # against three single-source calls; the viscosity gradient of the
    # nrhs call is the sum of the single calls'
    import paper_2303_06762_amd as hd
    c, t = synth.kuhn_square(4)
    nr, k, beta, gamma = 1, 2, 1.0, 1e2
    n_cells = 32 * 4 ** nr
    nu = lognormal_nu(n_cells)
    nq = (k + 2) ** 2
    F = dev(synth.source_uniform(210, 3, n_cells, nq))
    GU = dev(synth.source_uniform(310, 3, n_cells, nq))
    _note("nrhs entry points: 3 sources on one context")
    s = hd.Solver(c, t, nr, k, beta, nu, gamma)
    s.assemble()
    U, P, S, infos, st = s.solve_many(F)
    assert st == 0
    GF, GNU, ADJ, ainfos, st = s.solve_adjoint_many(F, S, GU)
    assert st == 0
    gnu1 = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
    for i in range(3):
        u, p, st_, info, st = s.solve(F[i])
        assert st == 0 and infos[i]["its"] == info["its"]
        assert (U[i] - u).abs().max().item() <= 1e-12 * u.abs().max().item()
        assert (P[i] - p).abs().max().item() <= 1e-12 * p.abs().max().item()
        assert (S[i] - st_).abs().max().item() <= 1e-12 * st_.abs().max().item()
        gf, _, adj, ainfo, st = s.solve_adjoint(F[i], st_, GU[i], gnu=gnu1)
        assert st == 0 and ainfos[i]["its"] == ainfo["its"]
        assert (GF[i] - gf).abs().max().item() <= 1e-12 * gf.abs().max().item()
        assert (ADJ[i] - adj).abs().max().item() <= 1e-12 * adj.abs().max().item()
    assert (GNU - gnu1).abs().max().item() <= 1e-12 * gnu1.abs().max().item()
    s.close()
