"""Pins of the oracle's Newton linearisation (Sec. 4.2, Alg. 3).

The Newton term C_h(du; u_prev, v) is checked against the independently
coded Picard form: for a frozen upwind switch C_h(w; u, v) is linear in the
wind, so the difference quotient of the Picard matrix in the wind, applied
to the transported state, is the Newton matrix applied to the wind's
increment -- exactly, up to rounding.  The Newton right-hand side equals
the Picard form of the previous state (bilinearity).  On a small cavity the
Newton steps converge quadratically to a fixed point of the Picard map,
and the method (AL-Uzawa + FGMRES + MG_hp with Picard-type lowest-order
levels) reaches the direct solve of each Newton system.
"""
import numpy as np
import pytest

import synth
from oracle import hdg, mesh, oseen


def rt_field(e, coef):
    return lambda X: np.einsum("pai,a->pi", e.rt.eval(X)[0], coef)


@pytest.mark.parametrize("k", [0, 1, 3])
def test_newton_matrix_is_the_wind_derivative_of_the_picard_form(k):
    c, t = synth.kuhn_square(2)
    lv = mesh.hierarchy(c, t, 1)[-1]
    pr = hdg.Problem(lv, k, 0.1, 1.0, 1e2)
    # cells with three interior facets (on boundary facets the Newton term
    # is left out: the increment's normal trace vanishes there)
    inner = [K for K in range(lv.n_cells) if all(lv.int_id[lv.cell_facets[K]] >= 0)]
    assert len(inner) >= 3
    for K in inner[:3]:
        e = pr.elems[K]
        z = synth.uniform_pm1(30 + K, 0, e.nz)        # transported local state
        dw = synth.uniform_pm1(60 + K, 0, e.na)       # wind increment
        w = rt_field(e, z[:e.na])                     # wind = the state's velocity
        h = 1e-6
        wp = lambda X, w=w, d=rt_field(e, dw): w(X) + h * d(X)
        C0 = oseen.convection_matrix(e, w)
        C1 = oseen.convection_matrix(e, wp)
        fd = (C1 - C0) @ z / h
        N = oseen.newton_matrix(e, w, z)
        dz = np.zeros(e.nz)
        dz[:e.na] = dw
        assert np.abs(fd - N @ dz).max() <= 1e-7 * np.abs(N @ dz).max(), K
        # Newton load = Picard form of the state itself (bilinearity)
        assert np.abs(C0 @ z - N @ z).max() <= 1e-12 * np.abs(C0 @ z).max()
        # the Newton term is not a multiple of the Picard one
        assert np.abs(N - C0).max() >= 1e-2 * np.abs(C0).max()


def cavity(k, n=2, n_refine=2, nu=0.05):
    c, t = synth.kuhn_square(n)
    levels = mesh.hierarchy(c, t, n_refine)
    lv = levels[-1]
    nq = (k + 2) ** 2
    f = 0.5 * synth.source_uniform(7, 1, lv.n_cells, nq)[0]
    return levels, lv, nu, f, oseen.lid_dirichlet(lv, k)


def test_newton_converges_quadratically_to_a_picard_fixed_point():
    k = 2
    levels, lv, nu, f, lid = cavity(k)
    steps = oseen.picard_newton(levels, k, nu, 0.0, 1e2, f, lid, eps_picard=1e-3, direct=True,
                                newton_rtol=1e-13, newton_atol=1e-14, max_newton=8)
    kinds = [s["kind"] for s in steps]
    assert kinds[0] == "stokes" and "picard" in kinds and kinds[-1] == "newton"
    dn = [s["du"] for s in steps if s["kind"] == "newton"]
    dp = [s["du"] for s in steps if s["kind"] == "picard"]
    # Picard contracts linearly; Newton's updates square (until round-off)
    assert dp[-1] < 1e-3
    assert len(dn) >= 3
    # (measured: Picard 1.7e-2, 1.7e-3, 1.5e-4; Newton 1.1e-5, 4.7e-11, 3.6e-15)
    assert dn[1] <= 10.0 * dn[0] ** 2 and dn[1] <= 1e-4 * dn[0]
    for a, b in zip(dn, dn[1:]):
        if a > 1e-9:
            assert b <= 50.0 * a * a + 1e-12, dn
    assert dn[-1] <= 1e-11, dn
    # the limit is a fixed point of the Picard map: one Picard step with
    # the limit as its wind returns it
    last = steps[-1]
    prob = last["prob"]
    w = oseen.state_wind(prob, last["lam"], last["p0"], f)
    pp = oseen.OseenProblem(lv, k, nu, 0.0, 1e2, w, lid)
    lam, p0 = pp.solve_direct(f)
    u, _, _, _ = pp.recover(lam, p0, f)
    assert oseen.l2_diff(pp, u, last["u"]) <= 1e-10 * oseen.l2_diff(pp, u, 0 * u)


def test_method_solves_the_newton_systems():
    k = 1
    levels, lv, nu, f, lid = cavity(k)
    ref = oseen.picard_newton(levels, k, nu, 0.0, 1e2, f, lid, eps_picard=1e-3, direct=True, max_newton=2)
    # the first Newton system, built from the direct Picard state before it
    i = [s["kind"] for s in ref].index("newton")
    prev = ref[i - 1]
    w = oseen.state_wind(prev["prob"], prev["lam"], prev["p0"], f)
    zs = oseen.local_states(prev["prob"], prev["lam"], f)
    S = oseen.OseenSetup(levels, k, nu, 0.0, 1e2, w, lid, newton_z=zs)
    r = S.solve(f, lam0=prev["lam"])
    lam_d, p_d = S.prob.solve_direct(f)
    assert np.abs(r["lam"] - lam_d).max() <= 1e-7 * np.abs(lam_d).max()
    assert np.abs(r["lam"] - ref[i]["lam"]).max() <= 1e-7 * np.abs(lam_d).max()
    assert max(r["its"]) <= 60, r["its"]


def test_navier_stokes_convergence_order():
    # Sec. 5.1.2: Alg. 3 (direct linear solves) on the manufactured solution
    # with the convection (u . grad) u in the source converges at order k+1
    # in the velocity, as for the generalized Stokes problem
    from tests import manufactured as mf
    k, nu = 1, 0.05
    errs = []
    for n in (4, 8):
        c, t = synth.kuhn_square(n)
        levels = mesh.hierarchy(c, t, 0)
        lv = levels[-1]
        pr = hdg.Problem(lv, k, nu, 0.0, 1.0)
        X = np.array([e.xq for e in pr.elems])
        f = mf.ns_source(X, nu)
        steps = oseen.picard_newton(levels, k, nu, 0.0, 1e2, f, None, eps_picard=1e-3, direct=True,
                                    newton_rtol=1e-12, newton_atol=1e-14, max_newton=6)
        assert steps[-1]["kind"] == "newton"
        u = steps[-1]["u"]
        w = np.array([e.wq for e in pr.elems])
        errs.append(np.sqrt(np.sum(w[..., None] * (u - mf.velocity(X)) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > k + 1 - 0.3, errs


def test_pseudo_time_picard_reaches_the_steady_solution():
    # Sec. 5.2.2: backward-Euler pseudo-time steps in the Picard phase; at
    # their fixed point the mass terms cancel, so Alg. 3 ends at the same
    # discrete steady solution as without them
    k = 2
    levels, lv, nu, f, lid = cavity(k)
    kw = dict(eps_picard=1e-3, direct=True, newton_rtol=1e-13, newton_atol=1e-14, max_newton=8)
    ref = oseen.picard_newton(levels, k, nu, 0.0, 1e2, f, lid, **kw)
    pt = oseen.picard_newton(levels, k, nu, 0.0, 1e2, f, lid, dt_inv=2.0, **kw)
    assert pt[-1]["kind"] == "newton"
    prob = pt[-1]["prob"]
    un = oseen.l2_diff(prob, ref[-1]["u"], 0 * ref[-1]["u"])
    assert oseen.l2_diff(prob, pt[-1]["u"], ref[-1]["u"]) <= 1e-10 * un
    # the pseudo-time steps differ from plain Picard steps (the mass term acts)
    assert oseen.l2_diff(prob, pt[1]["u"], ref[1]["u"]) > 1e-3 * un
