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
