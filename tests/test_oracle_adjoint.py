"""Pins of the oracle's adjoint gradients.

The adjoint formulas are not in the paper; they follow from its discrete
problem (stWeak) by the envelope theorem.  Every pin here checks them
against something that does not use them: central finite differences of
the misfit through fresh forward solves, the exact scaling of the
generalized Stokes solution in nu when beta = 0, and the method's own
solve (AL-Uzawa + flexible CG + MG_hp).
"""
import numpy as np
import pytest

import synth
from oracle import adjoint, hdg, mesh, solver


def small_case(k, beta, n=2, n_refine=1, seed=3):
    c, t = synth.kuhn_square(n)
    lv = mesh.hierarchy(c, t, n_refine)[-1]
    nu = np.exp(0.5 * synth.normal(seed, 0, lv.n_cells))
    nq = (k + 2) ** 2
    f = synth.source_uniform(100, 1, lv.n_cells, nq)[0]
    ut = synth.source_uniform(4, 1, lv.n_cells, nq)[0]
    return c, t, lv, nu, f, ut


@pytest.mark.parametrize("k,beta", [(1, 1.0), (2, 0.0)])
def test_grad_nu_matches_central_differences(k, beta):
    c, t, lv, nu, f, ut = small_case(k, beta)
    prob = hdg.Problem(lv, k, nu, beta, 1e2)
    J, gf, gnu, _ = adjoint.gradients(prob, f, ut)
    h = 1e-4  # relative step: rounding (~1e-16 J / h) and truncation (~h^2) both << tolerance
    for K in (0, 5, lv.n_cells - 1):
        e = np.zeros(lv.n_cells)
        e[K] = h * nu[K]
        Jp = adjoint.misfit_of(lv, k, nu + e, beta, 1e2, f, ut)
        Jm = adjoint.misfit_of(lv, k, nu - e, beta, 1e2, f, ut)
        fd = (Jp - Jm) / (2 * e[K])
        assert abs(fd - gnu[K]) <= 1e-6 * np.abs(gnu).max(), (K, fd, gnu[K])


def test_grad_f_matches_central_differences():
    k, beta = 1, 1.0
    c, t, lv, nu, f, ut = small_case(k, beta)
    prob = hdg.Problem(lv, k, nu, beta, 1e2)
    J, gf, gnu, _ = adjoint.gradients(prob, f, ut)
    rng = np.random.default_rng(0)
    h = 1e-4  # J is quadratic in f: central differences are exact up to rounding
    for _ in range(6):
        K, q, i = rng.integers(lv.n_cells), rng.integers(f.shape[1]), rng.integers(2)
        fp, fm = f.copy(), f.copy()
        fp[K, q, i] += h
        fm[K, q, i] -= h
        fd = (adjoint.misfit_of(lv, k, nu, beta, 1e2, fp, ut) -
              adjoint.misfit_of(lv, k, nu, beta, 1e2, fm, ut)) / (2 * h)
        assert abs(fd - gf[K, q, i]) <= 1e-8 * np.abs(gf).max() + 1e-12


def test_grad_nu_scaling_identity_beta0():
    # beta = 0: u_h(s nu) = u_h(nu) / s, so sum_K nu_K dJ/dnu_K = dJ/ds at
    # s = 1 = -sum gu . u_h (Euler's identity for the homogeneous map).
    k = 2
    c, t, lv, nu, f, ut = small_case(k, 0.0)
    prob = hdg.Problem(lv, k, nu, 0.0, 1e2)
    J, gf, gnu, _ = adjoint.gradients(prob, f, ut)
    lam, p0 = prob.solve_direct(f)
    u = adjoint.velocity(prob, lam, p0, f)
    gu = adjoint.misfit_grad(prob, u, ut)
    lhs = float(nu @ gnu)
    rhs = -float(np.sum(gu * u))
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs)


def test_grad_f_is_linear_response_transpose():
    # For the linear source-to-velocity map B: <gu, B df> = <gf, df> for
    # any df (gf = B^T gu); brute force on random directions.
    k, beta = 1, 1.0
    c, t, lv, nu, f, ut = small_case(k, beta)
    prob = hdg.Problem(lv, k, nu, beta, 1e2)
    J, gf, gnu, _ = adjoint.gradients(prob, f, ut)
    lam, p0 = prob.solve_direct(f)
    gu = adjoint.misfit_grad(prob, adjoint.velocity(prob, lam, p0, f), ut)
    for s in range(3):
        df = synth.source_uniform(50 + s, 1, lv.n_cells, f.shape[1])[0]
        l2, p2 = prob.solve_direct(df)
        du = adjoint.velocity(prob, l2, p2, df)
        assert abs(np.sum(gu * du) - np.sum(gf * df)) <= 1e-10 * np.abs(gf).sum()


def test_method_adjoint_reaches_dense_adjoint():
    k, beta = 2, 1.0
    c, t = synth.kuhn_square(2)
    S = solver.Setup(c, t, 2, k, np.exp(0.5 * synth.normal(3, 0, 8 * 16)), beta, 1e2)
    lv = S.lv
    nq = (k + 2) ** 2
    f = synth.source_uniform(100, 1, lv.n_cells, nq)[0]
    ut = synth.source_uniform(4, 1, lv.n_cells, nq)[0]

    def method(fq):
        r = S.solve(fq)
        return r["lam"], r["p0"]

    J0, gf0, gnu0, _ = adjoint.gradients(S.prob, f, ut)
    J1, gf1, gnu1, _ = adjoint.gradients(S.prob, f, ut, solve=method)
    assert abs(J1 - J0) <= 1e-8 * abs(J0)
    assert np.abs(gf1 - gf0).max() <= 1e-7 * np.abs(gf0).max()
    assert np.abs(gnu1 - gnu0).max() <= 1e-7 * np.abs(gnu0).max()


# ---------------------------------------------------------------- Oseen
# The Picard-linearised system at a fixed wind is nonsymmetric; its adjoint
# is the transposed system (oracle.oseen, transpose=True).  The pins below
# check the transposed condensation against the forward one and the
# gradients against finite differences, the linear-response identity and
# the method's FGMRES solve of the transposed system.
from oracle import oseen  # noqa: E402

_OSEEN = {}


def oseen_case(k, n=2, n_refine=1, scale=20.0, beta=1.0):
    key = (k, n, n_refine, scale, beta)
    if key in _OSEEN:
        return _OSEEN[key]
    c, t = synth.kuhn_square(n)
    levels = mesh.hierarchy(c, t, n_refine)
    lv = levels[-1]
    nq = (k + 2) ** 2
    nu = 0.1 * np.exp(0.5 * synth.normal(3, 0, lv.n_cells))
    pr0 = hdg.Problem(lv, k, 1.0, 1.0, 1e2)
    f0 = synth.source_uniform(100, 1, lv.n_cells, nq)[0]
    lam0, p00 = pr0.solve_direct(f0)
    winds = [(lambda X, w=w: scale * w(X)) for w in oseen.state_wind(pr0, lam0, p00, f0)]
    f = synth.source_uniform(7, 1, lv.n_cells, nq)[0]
    ut = synth.source_uniform(4, 1, lv.n_cells, nq)[0]
    _OSEEN[key] = (levels, lv, nu, beta, winds, f, ut)
    return _OSEEN[key]


def oseen_misfit(lv, k, nu, beta, winds, f, ut):
    pr = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds)
    lam, p0 = pr.solve_direct(f)
    return adjoint.misfit(pr, adjoint.velocity(pr, lam, p0, f), ut)


def oseen_gradients(k, **kw):
    levels, lv, nu, beta, winds, f, ut = oseen_case(k, **kw)
    fwd = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds)
    adj = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds, transpose=True)
    return fwd, adj, adjoint.gradients(fwd, f, ut, prob_adj=adj)


@pytest.mark.parametrize("k", [0, 2])
def test_oseen_transposed_condensation(k):
    # Condensation commutes with transposition: each cell block of the
    # transposed system is the transpose of the forward block, and both are
    # far from symmetric (the wind is strong).
    levels, lv, nu, beta, winds, f, ut = oseen_case(k)
    fwd = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds)
    adj = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds, transpose=True)
    for ef, ea in zip(fwd.elems, adj.elems):
        assert np.abs(ea.S - ef.S.T).max() <= 1e-12 * np.abs(ef.S).max()
    A, At = fwd.matrix_Aeps().toarray(), adj.matrix_Aeps().toarray()
    assert np.abs(At - A.T).max() <= 1e-12 * np.abs(A).max()
    A0 = fwd.matrix_A().toarray()  # without the (symmetric) AL term
    assert np.abs(A - A.T).max() >= 1e-3 * np.abs(A0).max()


@pytest.mark.parametrize("k", [1, 2])
def test_oseen_grad_nu_matches_central_differences(k):
    levels, lv, nu, beta, winds, f, ut = oseen_case(k)
    _, _, (J, gf, gnu, _) = oseen_gradients(k)
    h = 1e-4
    for K in (0, 7, lv.n_cells - 1):
        e = np.zeros(lv.n_cells)
        e[K] = h * nu[K]
        fd = (oseen_misfit(lv, k, nu + e, beta, winds, f, ut) -
              oseen_misfit(lv, k, nu - e, beta, winds, f, ut)) / (2 * e[K])
        assert abs(fd - gnu[K]) <= 1e-6 * np.abs(gnu).max(), (K, fd, gnu[K])


def test_oseen_grad_f_matches_central_differences_and_needs_the_transpose():
    k = 1
    levels, lv, nu, beta, winds, f, ut = oseen_case(k)
    fwd, adj, (J, gf, gnu, _) = oseen_gradients(k)
    # the forward system's own solve in place of the transposed one gives a
    # visibly different gradient: the pin below can tell them apart
    _, gf_wrong, _, _ = adjoint.gradients(fwd, f, ut)
    assert np.abs(gf_wrong - gf).max() >= 1e-2 * np.abs(gf).max()
    rng = np.random.default_rng(1)
    h = 1e-4  # J is quadratic in f: central differences are exact up to rounding
    for _ in range(6):
        K, q, i = rng.integers(lv.n_cells), rng.integers(f.shape[1]), rng.integers(2)
        fp, fm = f.copy(), f.copy()
        fp[K, q, i] += h
        fm[K, q, i] -= h
        fd = (oseen_misfit(lv, k, nu, beta, winds, fp, ut) -
              oseen_misfit(lv, k, nu, beta, winds, fm, ut)) / (2 * h)
        assert abs(fd - gf[K, q, i]) <= 1e-8 * np.abs(gf).max() + 1e-12


def test_oseen_grad_f_is_linear_response_transpose():
    k = 2
    levels, lv, nu, beta, winds, f, ut = oseen_case(k)
    fwd, adj, (J, gf, gnu, _) = oseen_gradients(k)
    lam, p0 = fwd.solve_direct(f)
    gu = adjoint.misfit_grad(fwd, adjoint.velocity(fwd, lam, p0, f), ut)
    for s in range(3):
        df = synth.source_uniform(50 + s, 1, lv.n_cells, f.shape[1])[0]
        l2, p2 = fwd.solve_direct(df)
        du = adjoint.velocity(fwd, l2, p2, df)
        assert abs(np.sum(gu * du) - np.sum(gf * df)) <= 1e-10 * np.abs(gf).sum()


def test_oseen_method_adjoint_reaches_dense_adjoint():
    # the method on the transposed system: AL-Uzawa + FGMRES preconditioned
    # by MG_hp built from the transposed blocks (patch factors, harmonic
    # transfers and lowest-order wind blocks all of A^T)
    k = 2
    levels, lv, nu, beta, winds, f, ut = oseen_case(k, n_refine=2)
    fwd, adj, (J0, gf0, gnu0, _) = oseen_gradients(k, n_refine=2)
    Sf = oseen.OseenSetup(levels, k, nu, beta, 1e2, winds)
    Sa = oseen.OseenSetup(levels, k, nu, beta, 1e2, winds, transpose=True)

    def method(S):
        def run(fq):
            r = S.solve(fq)
            run.its = r["its"]
            return r["lam"], r["p0"]
        return run

    sa = method(Sa)
    J1, gf1, gnu1, _ = adjoint.gradients(Sf.prob, f, ut, solve=method(Sf), prob_adj=Sa.prob, solve_adj=sa)
    assert abs(J1 - J0) <= 1e-8 * abs(J0)
    assert np.abs(gf1 - gf0).max() <= 1e-7 * np.abs(gf0).max()
    assert np.abs(gnu1 - gnu0).max() <= 1e-7 * np.abs(gnu0).max()
    assert max(sa.its) <= 60, sa.its


@pytest.mark.parametrize("with_wind", [False, True])
def test_lid_data_gradients_match_central_differences(with_wind):
    # Tangential Dirichlet data on the top side (the cavity's lid): the
    # adjoint keeps homogeneous data, the forward lifting keeps the lid.
    k = 1
    levels, lv, nu, beta, winds, f, ut = oseen_case(k)
    winds = winds if with_wind else None
    lid = oseen.lid_dirichlet(lv, k)
    fwd = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds, lid)
    adj = oseen.OseenProblem(lv, k, nu, beta, 1e2, winds, transpose=True)
    J, gf, gnu, (lam_a, _) = adjoint.gradients(fwd, f, ut, prob_adj=adj)

    def Jof(nu_, f_):
        pr = oseen.OseenProblem(lv, k, nu_, beta, 1e2, winds, lid)
        lam, p0 = pr.solve_direct(f_)
        return adjoint.misfit(pr, adjoint.velocity(pr, lam, p0, f_), ut)

    h = 1e-4
    for K in (0, 9, lv.n_cells - 1):
        e = np.zeros(lv.n_cells)
        e[K] = h * nu[K]
        fd = (Jof(nu + e, f) - Jof(nu - e, f)) / (2 * e[K])
        assert abs(fd - gnu[K]) <= 1e-6 * np.abs(gnu).max(), (K, fd, gnu[K])
    rng = np.random.default_rng(2)
    for _ in range(4):
        K, q, i = rng.integers(lv.n_cells), rng.integers(f.shape[1]), rng.integers(2)
        fp, fm = f.copy(), f.copy()
        fp[K, q, i] += h
        fm[K, q, i] -= h
        fd = (Jof(nu, fp) - Jof(nu, fm)) / (2 * h)
        assert abs(fd - gf[K, q, i]) <= 1e-8 * np.abs(gf).max() + 1e-12
    # dropping the lid from the forward lifting in dJ/dnu is detectable
    lam, p0 = fwd.solve_direct(f)
    f_a = adjoint.misfit_grad(fwd, adjoint.velocity(fwd, lam, p0, f), ut) / adjoint.weights(fwd)[:, :, None]
    gnu_nolid = np.array([adjoint.grad_nu_cell(e, hdg.Problem.local(fwd, lam, K), f[K], adj.local(lam_a, K),
                                               f_a[K], adj.elems[K])
                          for K, e in enumerate(fwd.elems)])
    assert np.abs(gnu_nolid - gnu).max() >= 1e-2 * np.abs(gnu).max()
