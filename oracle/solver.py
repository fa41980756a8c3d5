"""End-to-end oracle drivers (test infrastructure only).

R1: the discrete solution by a direct solve of the condensed saddle point.
R2: the method: AL-Uzawa outer loop (stOpEq-ALU), flexible CG inner solve
    (x0 = 0 for every Uzawa step), preconditioned by MG_hp (Alg. 2) whose
    auxiliary solver is MG_h (Alg. 1) on the lowest-order CR-equivalent
    operators of all levels (k0-stOptEq-ALU).
"""
import numpy as np

from . import mesh, hdg, mg, krylov, oseen


class Setup:
    def __init__(self, coords, cells, n_refine, k, nu, beta, gamma,
                 m_p=1, m_h=1, q=1, growth=2, harmonic=True, smoother="gs", additive=False,
                 outflow=None, dirichlet=None, patch_relax="vertex", patch_smooth="vertex"):
        """outflow: do-nothing facets of the coarsest mesh (vertex pairs);
        dirichlet: boundary data on the finest level as in
        oseen.OseenProblem (a callable lv -> array is evaluated there)."""
        self.levels = mesh.hierarchy(coords, cells, n_refine, outflow)
        self.lv = self.levels[-1]
        self.k = k
        if callable(dirichlet):
            dirichlet = dirichlet(self.lv)
        if dirichlet is not None or outflow is not None:
            self.prob = oseen.OseenProblem(self.lv, k, nu, beta, gamma, None, dirichlet)
        else:
            self.prob = hdg.Problem(self.lv, k, nu, beta, gamma)
        self.Aeps = self.prob.matrix_Aeps().tocsr()
        self.D = self.prob.matrix_D().tocsr()
        self.eps_inv = self.prob.eps_inv
        self.hier = mg.Hierarchy(self.levels, self.prob.nu_c, beta, self.eps_inv,
                                 harmonic=harmonic, smoother=smoother, patch=patch_smooth)
        self.prec = mg.HPMG(self.Aeps, self.lv, k, self.hier, m_p, m_h, q, growth, smoother, additive,
                            patch_relax)

    def inner(self, b, rtol=1e-8, atol=1e-10, max_it=500):
        return krylov.fcg(self.Aeps, b, self.prec, rtol, atol, max_it)

    def solve(self, f_qp, rtol=1e-8, atol=1e-10, max_it=500, uzawa_max=50, uzawa_tol=1e-10):
        g = self.prob.rhs(f_qp)
        lam, p0, log = krylov.uzawa(self.Aeps, self.D, self.lv.area, g, self.eps_inv,
                                    lambda b: self.inner(b, rtol, atol, max_it),
                                    uzawa_max, uzawa_tol, self.prob.constraint_rhs())
        return dict(g=g, lam=lam, p0=p0, its=[l[0] for l in log], hist=[l[1] for l in log])
