"""Pins of the oracle's Oseen / Picard path (Sec. 4).

Checked against: the upwind energy identity of the convection form (a
closed form), the optimal convergence order on manufactured solutions
with a strong wind and with tangential boundary data, exact flux
reproduction of the RT0 wind projection, the defining properties of the
harmonic transfers, FGMRES against a dense solve, and the method's solve
against the direct one.
"""
import numpy as np
import pytest

import synth
from oracle import hdg, mesh, oseen, quad
from tests import manufactured as mf


def stokes_state(lv, k, seed=100, nu=1.0, beta=1.0):
    pr = hdg.Problem(lv, k, nu, beta, 1e2)
    f = synth.source_uniform(seed, 1, lv.n_cells, (k + 2) ** 2)[0]
    lam, p0 = pr.solve_direct(f)
    return pr, f, lam, p0


@pytest.mark.parametrize("k", [0, 1, 2])
def test_upwind_energy_identity(k):
    # For a pointwise divergence-free, normal-continuous wind vanishing in
    # normal direction on the boundary, and any normal-continuous (u, uhat):
    #   sum_K c_K(w; u, u) = 1/2 sum_K <|w.n_K|, (t(u_K) - uhat)^2>_{dK},
    # point by point of the facet rule (the upwind switch is pointwise, so
    # the right side is summed over the same Gauss points; the volume rule
    # is exact).
    c, t = synth.kuhn_square(2)
    lv = mesh.hierarchy(c, t, 1)[-1]
    pr, f, lam, p0 = stokes_state(lv, k)
    winds = oseen.state_wind(pr, lam, p0, f)
    rng = np.random.default_rng(1)
    lam_u = rng.standard_normal(pr.n_dof)
    lhs = rhs = 0.0
    s, om = quad.gauss_legendre01(oseen.convection_points(k))
    phi = hdg.facet_basis(k, s)
    for K, e in enumerate(pr.elems):
        C = oseen.convection_matrix(e, winds[K])
        z = e.E @ pr.local(lam_u, K)
        if e.Zh.shape[1] > 0:
            z = z + e.Zh @ rng.standard_normal(e.Zh.shape[1])
        lhs += z @ C @ z
        a = z[:e.na]
        for fl in range(3):
            E = lv.cell_facets[K, fl]
            X0, X1 = lv.coords[lv.edges[E, 0]], lv.coords[lv.edges[E, 1]]
            xl = X0[None, :] + s[:, None] * (X1 - X0)[None, :]
            Pv, _, _ = e.rt.eval(xl)
            ut = (Pv @ lv.tangent[E]) @ a
            uh = phi @ z[e.na + fl * e.m:e.na + (fl + 1) * e.m]
            wn = winds[K](xl) @ (lv.sigma[K, fl] * lv.normal[E])
            rhs += 0.5 * lv.length[E] * np.sum(om * np.abs(wn) * (ut - uh) ** 2)
    assert rhs > 0
    assert abs(lhs - rhs) <= 1e-10 * rhs, (lhs, rhs)


def _oseen_errors(n, k, nu, wind_scale, cavity):
    c, t = synth.kuhn_square(n)
    lv = mesh.Level(c, t)
    vel = mf.cavity_velocity if cavity else mf.velocity
    grad = mf.cavity_grad_velocity if cavity else mf.grad_velocity
    winds = [(lambda X: wind_scale * vel(X)) for _ in range(lv.n_cells)]
    dirichlet = None
    if cavity:
        dirichlet = np.zeros((lv.n_facets, k + 1))
        s, om = quad.gauss_legendre01(k + 4)
        phi = hdg.facet_basis(k, s)
        for E in np.where(lv.int_id < 0)[0]:
            X0, X1 = lv.coords[lv.edges[E, 0]], lv.coords[lv.edges[E, 1]]
            xl = X0[None, :] + s[:, None] * (X1 - X0)[None, :]
            dirichlet[E] = (om * (vel(xl) @ lv.tangent[E])) @ phi
    pr = oseen.OseenProblem(lv, k, nu, 0.0, 1.0, winds, dirichlet)
    if cavity:
        f = np.array([mf.cavity_source(e.xq, nu, 0.0, wind_scale) for e in pr.elems])
    else:
        f = np.array([mf.source(e.xq, nu, 0.0) +
                      wind_scale * np.einsum("qij,qj->qi", mf.grad_velocity(e.xq), mf.velocity(e.xq))
                      for e in pr.elems])
    lam, p0 = pr.solve_direct(f)
    eu = eL = 0.0
    for K, e in enumerate(pr.elems):
        vs = np.sort(lv.cells[K])
        X, w = quad.data_points(lv.coords[vs], k + 4)
        w = w * lv.area[K]
        u, p, L, _ = e.recover(pr.local(lam, K), p0[K], f[K], X)
        eu += np.sum(w * np.sum((u - vel(X)) ** 2, axis=1))
        eL += np.sum(w * np.sum((L + nu * grad(X)) ** 2, axis=(1, 2)))
    return np.sqrt(eu), np.sqrt(eL)


@pytest.mark.parametrize("k,cavity", [(1, False), (2, False), (1, True), (2, True)])
def test_oseen_convergence_order(k, cavity):
    # Sec. 4 scheme with a wind 20 times the solution at nu = 0.05 (the cell
    # Peclet number reaches ~2 on the coarsest mesh); optimal order k+1 in
    # u_h and L_h
    e = [_oseen_errors(n, k, 0.05, 20.0, cavity) for n in (4, 8, 16)]
    for comp in range(2):
        rates = [np.log2(e[i][comp] / e[i + 1][comp]) for i in range(2)]
        assert rates[-1] > k + 1 - 0.3, (comp, rates, e)


def test_manufactured_cavity_source_matches_finite_differences():
    X = np.array([[0.31, 0.62], [0.77, 0.12]])
    h = 1e-4
    nu, beta, ws = 1.3, 0.4, 7.0
    lap = np.zeros((2, 2))
    for d in range(2):
        ed = np.zeros(2)
        ed[d] = h
        lap += (mf.cavity_velocity(X + ed) - 2 * mf.cavity_velocity(X) + mf.cavity_velocity(X - ed)) / h ** 2
    G = np.zeros((2, 2, 2))
    for d in range(2):
        ed = np.zeros(2)
        ed[d] = h
        G[:, :, d] = (mf.cavity_velocity(X + ed) - mf.cavity_velocity(X - ed)) / (2 * h)
    assert np.abs(G - mf.cavity_grad_velocity(X)).max() < 1e-7
    u = mf.cavity_velocity(X)
    gp = np.stack([(mf.pressure(X + [h, 0]) - mf.pressure(X - [h, 0])) / (2 * h),
                   (mf.pressure(X + [0, h]) - mf.pressure(X - [0, h])) / (2 * h)], axis=1)
    ref = -nu * lap + beta * u + ws * np.einsum("pij,pj->pi", G, u) + gp
    assert np.abs(ref - mf.cavity_source(X, nu, beta, ws)).max() < 1e-6
    assert np.abs(G[:, 0, 0] + G[:, 1, 1]).max() < 1e-9
    # u.n = 0 on the boundary, u_x = -g(x) on top, 0 on the other sides
    s = np.linspace(0, 1, 7)
    top = np.stack([s, np.ones_like(s)], axis=1)
    assert np.allclose(mf.cavity_velocity(top)[:, 1], 0) and np.allclose(mf.cavity_velocity(top)[:, 0], -mf.g0(s))
    for side in (np.stack([s, 0 * s], 1), np.stack([0 * s, s], 1), np.stack([1 + 0 * s, s], 1)):
        assert np.allclose(mf.cavity_velocity(side), 0)


def test_rt0_flux_projection_and_coarsening():
    c, t = synth.kuhn_square(2)
    levels = mesh.hierarchy(c, t, 2)
    wc = np.array([0.7, -1.3])
    const = [(lambda X: np.tile(wc, (len(X), 1))) for _ in range(levels[-1].n_cells)]
    flux = oseen.facet_fluxes(levels[-1], const)
    for l in range(len(levels) - 1, 0, -1):
        flux = oseen.coarsen_fluxes(levels[l - 1], levels[l], flux)
        lv = levels[l - 1]
        # exact on unknown-carrying facets; no flux through Dirichlet facets
        dof = lv.int_id >= 0
        assert np.abs(flux[dof] - (lv.length * (lv.normal @ wc))[dof]).max() < 1e-13
        assert np.all(flux[~dof] == 0.0)
    # a discrete divergence-free wind stays divergence-free on every level
    lv = levels[-1]
    pr, f, lam, p0 = stokes_state(lv, 2)
    flux = oseen.facet_fluxes(lv, oseen.state_wind(pr, lam, p0, f))
    for l in range(len(levels) - 1, -1, -1):
        L = levels[l]
        net = np.array([sum(L.sigma[K, i] * flux[L.cell_facets[K, i]] for i in range(3))
                        for K in range(L.n_cells)])
        assert np.abs(net).max() < 1e-12 * np.abs(flux).max()
        bd = L.int_id < 0
        assert np.abs(flux[bd]).max() < 1e-12 * np.abs(flux).max()
        # the RT0 field of these fluxes reproduces them
        w0 = oseen.rt0_winds(L, flux)
        assert np.abs(oseen.facet_fluxes(L, w0) - flux).max() < 1e-12 * np.abs(flux).max()
        if l > 0:
            flux = oseen.coarsen_fluxes(levels[l - 1], L, flux)


def test_nonsymmetric_transfers_are_harmonic():
    # prolongation: (A P d)_T = 0; restriction: R A E_T = 0 (T = fine
    # unknowns strictly inside coarse cells)
    from oracle import mg
    c, t = synth.kuhn_square(2)
    levels = mesh.hierarchy(c, t, 2)
    lv = levels[-1]
    pr, f, lam, p0 = stokes_state(lv, 1)
    flux = 1e4 * oseen.facet_fluxes(lv, oseen.state_wind(pr, lam, p0, f))
    H = oseen.OseenHierarchy(levels, 0.1, 1.0, 1e2, flux)
    A = H.A[-1].toarray()
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()      # really nonsymmetric
    td = mg.interior_dofs(levels[-2], levels[-1])
    P, R = H.P[-1].toarray(), H.R[-1].toarray()
    assert np.abs((A @ P)[td]).max() < 1e-11 * np.abs(A).max()
    assert np.abs(R @ A[:, td]).max() < 1e-11 * np.abs(A).max()


def test_fgmres_matches_dense_solve():
    rng = np.random.default_rng(4)
    n = 30
    A = np.eye(n) * 12 + rng.standard_normal((n, n))   # spectrum in a disc about 12 of radius ~sqrt(n)
    b = rng.standard_normal(n)
    ref = np.linalg.solve(A, b)
    x, its, hist = oseen.fgmres(A, b, lambda r: r, rtol=1e-12, atol=0.0, restart=50)
    assert its <= n and np.abs(x - ref).max() < 1e-9 * np.abs(ref).max()
    x, its, hist = oseen.fgmres(A, b, lambda r: r, rtol=1e-10, atol=0.0, restart=7, max_it=2000)
    assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)
    # a preconditioner changing from call to call (flexible)
    cnt = [0]

    def prec(r):
        cnt[0] += 1
        return r / (3.0 + (cnt[0] % 3))
    x, its, hist = oseen.fgmres(A, b, prec, rtol=1e-10, atol=0.0, restart=50)
    assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 2])
def test_oseen_method_reaches_direct_solution(k):
    c, t = synth.kuhn_square(2)
    levels = mesh.hierarchy(c, t, 2)
    lv = levels[-1]
    pr, f, lam, p0 = stokes_state(lv, k)
    winds = [(lambda X, w=w: 20.0 * w(X)) for w in oseen.state_wind(pr, lam, p0, f)]
    S = oseen.OseenSetup(levels, k, 0.1, 1.0, 1e2, winds, oseen.lid_dirichlet(lv, k))
    lam_d, p_d = S.prob.solve_direct(f)
    r = S.solve(f)
    assert np.linalg.norm(r["lam"] - lam_d) <= 1e-7 * np.linalg.norm(lam_d)
    assert max(r["its"]) < 60


def test_picard_lid_cavity_contracts():
    # Re = 10 lid-driven cavity, k = 1: Picard steps contract
    c, t = synth.kuhn_square(2)
    levels = mesh.hierarchy(c, t, 2)
    k = 1
    lv = levels[-1]
    f = np.zeros((lv.n_cells, (k + 2) ** 2, 2))
    steps = oseen.picard(levels, k, 0.1, 0.0, 1e1, f, 4, oseen.lid_dirichlet(lv, k), direct=True)
    d = [np.abs(steps[i + 1]["u"] - steps[i]["u"]).max() for i in range(len(steps) - 1)]
    assert d[-1] < 0.5 * d[0] and d[-1] < d[-2]
