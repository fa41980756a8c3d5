"""Pins of the oracle on non-square domains with do-nothing outflow and an
inflow (Sec. 5.3): the backward-facing step and a straight channel.

Do-nothing facets carry skeleton unknowns (both components); the inflow
prescribes normal and tangential data, whose flux enters the divergence
constraint and the AL-Uzawa loop.  Closed forms: in the channel
[0, 4] x [0.5, 1] with the parabolic inflow the Stokes solution is the
Poiseuille flow u = (16 (1-y)(y-0.5), 0), p = 32 nu (4 - x) (the do-nothing
condition nu du/dn - p n = 0 holds at x = 4), which the scheme reproduces
for k >= 2 (u quadratic, p linear); on the step every cell is divergence
free and the outflow flux equals the inflow flux 16 int_{0.5}^{1} (1-y)(y-0.5)
dy = 1/3.
"""
import numpy as np
import pytest

import synth
from oracle import mesh, oseen, solver, quad


def _inflow(lv, k):
    D = np.zeros((lv.n_facets, 2, k + 1))
    bnd = np.where(lv.int_id < 0)[0]
    ends = lv.coords[lv.edges[bnd]]
    D[bnd] = synth.boundary_coefficients(ends, k, synth.step_inflow)
    return D


def _setup(step, n_refine, k, nu=1.0, beta=0.0, gamma=1e3, **kw):
    c, t, out = synth.step_domain(1, step=step)
    return solver.Setup(c, t, n_refine, k, nu, beta, gamma, outflow=out,
                        dirichlet=lambda lv: _inflow(lv, k), **kw)


def test_step_mesh_and_do_nothing_facets():
    c, t, out = synth.step_domain(1)
    assert len(t) == 30 and len(out) == 2
    levels = mesh.hierarchy(c, t, 2, out)
    for l, lv in enumerate(levels):
        assert lv.n_cells == 30 * 4 ** l
        assert lv.outflow.sum() == 2 * 2 ** l
        # do-nothing facets lie on x = 4 and carry unknowns
        assert np.allclose(lv.midpoint[lv.outflow, 0], 4.0)
        assert np.all(lv.int_id[lv.outflow] >= 0)
        area = lv.area.sum()
        assert abs(area - (4.0 * 0.5 + 3.5 * 0.5)) < 1e-12


@pytest.mark.parametrize("k", [2, 3])
def test_poiseuille_reproduced_in_the_channel(k):
    nu = 0.7
    S = _setup(False, 1, k, nu=nu)
    lv = S.lv
    f = np.zeros((lv.n_cells, (k + 2) ** 2, 2))
    lam, p0 = S.prob.solve_direct(f)
    u, p, L, dv = S.prob.recover(lam, p0, f)
    X = np.array([e.xq for e in S.prob.elems])
    ue = np.stack([16 * (1 - X[..., 1]) * (X[..., 1] - 0.5), 0 * X[..., 0]], axis=-1)
    assert np.abs(u - ue).max() <= 1e-10
    assert np.abs(p - 32 * nu * (4.0 - X[..., 0])).max() <= 1e-9
    G = np.zeros(X.shape[:-1] + (2, 2))
    G[..., 0, 1] = 16.0 * (1.5 - 2.0 * X[..., 1])
    assert np.abs(L + nu * G).max() <= 1e-9
    # the method (AL-Uzawa + flexible CG + MG_hp) reaches it too
    r = S.solve(f, rtol=1e-12, atol=0.0, uzawa_tol=1e-13)
    u2, p2, _, _ = S.prob.recover(r["lam"], r["p0"], f)
    assert np.abs(u2 - ue).max() <= 1e-9
    assert np.abs(p2 - 32 * nu * (4.0 - X[..., 0])).max() <= 1e-7


@pytest.mark.parametrize("k", [0, 1, 2])
def test_step_mass_conservation(k):
    S = _setup(True, 1, k, beta=1.0)
    lv = S.lv
    f = np.zeros((lv.n_cells, (k + 2) ** 2, 2))
    lam, p0 = S.prob.solve_direct(f)
    # cellwise divergence zero (with the inflow flux) and outflow flux 1/3
    D = S.prob.matrix_D()
    assert np.abs(D @ lam + S.prob.flux_b()).max() <= 1e-12
    m = k + 1
    out = 0.0
    for E in np.where(lv.outflow)[0]:
        K, i = lv.facet_cells[E, 0], lv.facet_local[E, 0]
        out += lv.sigma[K, i] * lv.length[E] * lam[(lv.int_id[E] * 2 + 0) * m]
    assert abs(out - 1.0 / 3.0) <= 1e-12
    # R2 = R1
    r = S.solve(f, rtol=1e-12, atol=0.0, uzawa_tol=1e-13)
    assert np.abs(r["lam"] - lam).max() <= 1e-7 * np.abs(lam).max()
    assert np.abs(r["p0"] - p0).max() <= 1e-6 * np.abs(p0).max()


@pytest.mark.parametrize("k", [2, 3])
def test_navier_stokes_poiseuille_in_the_channel(k):
    # the Poiseuille flow also solves the Navier-Stokes equations ((u.grad)u
    # = 0) with p = 32 nu (4 - x); the scheme reproduces it only if the
    # convection form leaves the do-nothing condition (nu grad u - p I) n = 0
    # on the outflow (the total-flux form would impose p = 32 nu (4 - x) -
    # u_x^2 there, which no linear pressure meets)
    nu = 0.05
    c, t, out = synth.step_domain(1, step=False)
    levels = mesh.hierarchy(c, t, 1, out)
    lv = levels[-1]
    D = np.zeros((lv.n_facets, 2, k + 1))
    bnd = np.where(lv.int_id < 0)[0]
    D[bnd] = synth.boundary_coefficients(lv.coords[lv.edges[bnd]], k, synth.step_inflow)
    f = np.zeros((lv.n_cells, (k + 2) ** 2, 2))
    steps = oseen.picard_newton(levels, k, nu, 0.0, 1e2, f, D, eps_picard=1e-3, direct=True, newton_rtol=1e-13,
                                newton_atol=1e-14, max_newton=6)
    last = steps[-1]
    assert last["kind"] == "newton" and last["du"] <= 1e-10
    u, p, _, _ = last["prob"].recover(last["lam"], last["p0"], f)
    X = np.array([e.xq for e in last["prob"].elems])
    assert np.abs(u[..., 0] - 16 * (1 - X[..., 1]) * (X[..., 1] - 0.5)).max() <= 1e-9
    assert np.abs(u[..., 1]).max() <= 1e-9
    assert np.abs(p - 32 * nu * (4.0 - X[..., 0])).max() <= 1e-8


def test_navier_stokes_on_the_step_converges():
    # Alg. 3 with direct linear solves on the step (level 3, k = 2) at
    # nu = 1e-2 and 1e-3: Picard contracts and Newton converges
    # quadratically (the outflow condition keeps the energy of the
    # linearisations bounded)
    k = 2
    c, t, out = synth.step_domain(1)
    levels = mesh.hierarchy(c, t, 2, out)
    lv = levels[-1]
    D = np.zeros((lv.n_facets, 2, k + 1))
    bnd = np.where(lv.int_id < 0)[0]
    D[bnd] = synth.boundary_coefficients(lv.coords[lv.edges[bnd]], k, synth.step_inflow)
    f = np.zeros((lv.n_cells, (k + 2) ** 2, 2))
    for nu in (1e-2, 1e-3):
        steps = oseen.picard_newton(levels, k, nu, 0.0, 1e6 * nu, f, D, eps_picard=1e-4, direct=True,
                                    max_picard=30, max_newton=10)
        dn = [s["du"] for s in steps if s["kind"] == "newton"]
        assert dn and dn[-1] <= 1e-8, (nu, dn)
