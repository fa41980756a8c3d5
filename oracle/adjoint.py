"""Adjoint of the generalized Stokes solve (test infrastructure only).

Not in the paper; derived from its discrete problem.  The scheme (stWeak)
with the lifting eliminated is the symmetric saddle point

    nu (Lift(u, uhat), Lift(v, vhat)) + beta (u, v) - (p, div v) - (q, div u)
        = (f, v),

the source entering only through (f, v) evaluated with the data rule:
sum_{K,q} w_q |K| f(x_q) . v(x_q).  For the velocity misfit

    J = sum_{K,q} w_q |K| |u_h(x_q) - u_target(x_q)|^2

the adjoint state is the solution of the same system whose load is the
functional v -> sum_{K,q} gu_{K,q} . v(x_q) with gu = dJ/du_h(x_q)
= 2 w_q |K| (u_h - u_target); that is the forward solve with the source
values gu / (w_q |K|).  Then
    dJ/df_{K,q} = w_q |K| u_adj(x_q),
    dJ/dnu_K    = -(Lift(u, uhat), Lift(u_adj, uhat_adj))_K
(the only nu-dependent term of the system is the nu-weighted lifting
energy; the augmented-Lagrangian weight is a fixed number and multiplies
div u_h, which vanishes at the discrete solution).

Oseen (Picard-linearised) systems at a fixed wind: the convection form makes
the saddle point nonsymmetric, so the adjoint state solves the transposed
system (convection transposed per cell, Stokes part and constraint
unchanged) with the same load functional.  The two formulas above keep
their form, with the adjoint's local fields recovered by the transposed
local solve: dJ/dnu_K = -(Lift(z), Lift(z_adj))_K still holds because the
convection form does not depend on nu.

Inhomogeneous tangential Dirichlet data (the lid of the cavity) enter the
forward load and the forward local fields only: the adjoint state has
homogeneous data (its test space is the forward's), so prob_adj is then the
same system without the boundary values, while the forward state's lifting
in dJ/dnu keeps them.
"""
import numpy as np

from . import hdg


def weights(prob):
    """w_q |K| per cell and data point [n_cells, n_q]."""
    return np.array([e.wq for e in prob.elems])


def misfit(prob, u_qp, ut_qp):
    """J for u_qp, ut_qp [n_cells, n_q, 2]."""
    return float(np.sum(weights(prob)[:, :, None] * (u_qp - ut_qp) ** 2))


def misfit_grad(prob, u_qp, ut_qp):
    """dJ/du at the data points."""
    return 2.0 * weights(prob)[:, :, None] * (u_qp - ut_qp)


def lift_coefficients(e, z):
    """Lift(z) per component (i, j) in the cell's P^k basis: M^-1 R_ij z."""
    Minv = np.linalg.inv(e.M)
    return np.array([[Minv @ (e.R[i, j] @ z) for j in range(2)] for i in range(2)])


def grad_nu_cell(e, lam_u, f_u, lam_a, f_a, e_adj=None):
    """-(Lift(z_u), Lift(z_a))_K for the local states recovered from the
    skeleton values and sources of the forward and adjoint solves (e_adj:
    the cell of the transposed system when it differs from e)."""
    z_u, _ = e.recover_z(lam_u, f_u)
    z_a, _ = (e_adj or e).recover_z(lam_a, f_a)
    Lu = lift_coefficients(e, z_u)
    La = lift_coefficients(e, z_a)
    s = 0.0
    for i in range(2):
        for j in range(2):
            s += Lu[i, j] @ e.M @ La[i, j]
    return -s


def velocity(prob, lam, p0, f_qp):
    u, _, _, _ = prob.recover(lam, p0, f_qp)
    return u


def gradients(prob, f_qp, ut_qp, solve=None, prob_adj=None, solve_adj=None):
    """(J, dJ/df [n_cells, n_q, 2], dJ/dnu [n_cells], adjoint (lam, p0)).

    solve(f_qp) -> (lam, p0) defaults to the direct solve of the condensed
    saddle point (the dense adjoint); the method's solve can be passed in.
    prob_adj / solve_adj: the transposed system with homogeneous boundary
    data and its solve, for nonsymmetric (Oseen) problems or inhomogeneous
    Dirichlet data; by default the forward ones."""
    solve = solve or prob.solve_direct
    pa = prob_adj or prob
    solve_adj = solve_adj or (pa.solve_direct if prob_adj is not None else solve)
    lam, p0 = solve(f_qp)
    u = velocity(prob, lam, p0, f_qp)
    J = misfit(prob, u, ut_qp)
    W = weights(prob)
    gu = misfit_grad(prob, u, ut_qp)
    f_adj = gu / W[:, :, None]
    lam_a, p0_a = solve_adj(f_adj)
    u_a = velocity(pa, lam_a, p0_a, f_adj)
    gf = W[:, :, None] * u_a
    gnu = np.array([grad_nu_cell(e, prob.local(lam, K), f_qp[K], pa.local(lam_a, K), f_adj[K],
                                 pa.elems[K] if prob_adj is not None else None)
                    for K, e in enumerate(prob.elems)])
    return J, gf, gnu, (lam_a, p0_a)


def misfit_of(lv, k, nu, beta, gamma, f_qp, ut_qp):
    """J by a fresh direct solve (for finite differences)."""
    prob = hdg.Problem(lv, k, nu, beta, gamma)
    lam, p0 = prob.solve_direct(f_qp)
    return misfit(prob, velocity(prob, lam, p0, f_qp), ut_qp)
