"""Oseen / Picard linearisation of the Navier-Stokes scheme (Sec. 4), the
oracle's version (test infrastructure only: nothing in the product path
imports it).

* Convection (the trilinear form C_h of Sec. 4.1) for a wind w, trial
  (u, uhat) and test (v, vhat):
      - sum_ij (u_i w_j, d_j v_i)_K
      + < (w.n_K) t(u_up), t(v) - vhat >_{dK},
  t(.) the tangential component in the facet frame; the upwind value is
  the cell's own trace t(u) where w.n_K > 0 and the facet unknown uhat where
  w.n_K < 0 (the switch is taken on the wind, which keeps the Picard form
  linear; where w.n_K = 0 the term vanishes).  The normal part of u_up does
  not enter since it multiplies a tangential quantity.
* Picard (nsWeak with f' = f): the wind is the previous velocity u_h^(n-1).
* Condensation with a nonsymmetric element matrix H: the same elimination as
  in the Stokes case, with the test-side coupling E^T H Zh in place of the
  transpose of the trial-side one.
* Lowest-order operators of MG_h: the generic condensation at k = 0 with the
  wind replaced by its RT0 projection (the field with the same facet fluxes);
  on coarser levels a coarse facet's flux is the sum of its two halves'.
  Prolongation uses A (harmonic extension A_TT^-1 A_T.); restriction is the
  transpose of the same construction built with A^T, i.e.
  r_c = I^T (r - A_.T A_TT^-1 r_T), which equals the Stokes case's
  transpose when A is symmetric.
* Inner solve: FGMRES(restart) with right preconditioning and modified
  Gram-Schmidt, stopping at ||r|| <= max(rtol ||r_0||, atol) on the Arnoldi
  residual; x_0 = the latest skeleton iterate.
* Tangential Dirichlet data on boundary facets (the lid of the cavity):
  uhat . t_F prescribed per boundary facet and mode; moved to the load.
* Newton linearisation (Sec. 4.2): the Jacobian adds to the Picard form the
  term C_h(du; u_prev, v) -- the previous velocity transported by the
  increment's flux -- with the upwind switch frozen on u_prev.n_K (taken
  point by point; where it vanishes the facet term is dropped, as in the
  Picard form).  Solving for u_n = u_prev + du directly, the right-hand side
  is f plus the functional C_h(u_prev; u_prev, v), which by bilinearity (for
  the frozen switch) equals the Picard matrix applied to the previous local
  state.  The lowest-order levels of MG_h keep the Picard operators of the
  RT0-projected wind.
* Transposed (adjoint) systems, transpose=True: every cell's convection
  matrix enters transposed (the Stokes part is symmetric), on the order-k
  level and on every lowest-order level.  Static condensation commutes with
  transposition, so the condensed operator, the patch blocks and the
  harmonic transfers built from it are those of A^T; the AL weight and the
  divergence constraint are symmetric and unchanged.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import hdg, quad, mg, cr, krylov


# ------------------------------------------------------------- convection
def convection_points(k):
    """Points per direction of the convection rules: the volume integrand
    (u in RT_k, w in RT_k, grad v) and the facet integrand (w.n, t(u),
    t(v)) have degree 3k+2 for a discrete wind, so the Stroud rule and the
    Gauss-Legendre rule with ceil((3k+3)/2) points are exact; the upwind
    switch is taken point by point at the facet Gauss points."""
    return (3 * k + 4) // 2


def convection_matrix(e, wind):
    """C [nz, nz] (row: test, column: trial) of cell e for the wind callable
    wind(X [np,2]) -> [np,2] (the wind restricted to this cell)."""
    lv, K, k, m = e.lv, e.K, e.k, e.m
    na, nz = e.na, e.nz
    C = np.zeros((nz, nz))
    nc = convection_points(k)
    vs = np.sort(lv.cells[K])
    X, w = quad.data_points(lv.coords[vs], nc)
    wq = w * e.area
    val, grd, _ = e.rt.eval(X)         # val [q, a, i], grd [q, a, i, j] = d_j u_a,i
    W = wind(X)
    # - sum_ij (u_i w_j, d_j v_i): trial a (u_a,i), test b (w . grad v_b,i)
    wgrad = np.einsum("qj,qbij->qbi", W, grd)
    C[:na, :na] -= np.einsum("q,qbi,qai->ba", wq, wgrad, val)
    s, om = quad.gauss_legendre01(nc)
    phi = hdg.facet_basis(k, s)
    for f in range(3):
        E = lv.cell_facets[K, f]
        X0 = lv.coords[lv.edges[E, 0]]
        X1 = lv.coords[lv.edges[E, 1]]
        L = lv.length[E]
        t = lv.tangent[E]
        nK = lv.sigma[K, f] * lv.normal[E]
        xl = X0[None, :] + s[:, None] * (X1 - X0)[None, :]
        Pv, _, _ = e.rt.eval(xl)
        ut = Pv @ t                                  # [l, a]
        wn = wind(xl) @ nK                           # [l]
        for l in range(len(s)):
            if wn[l] == 0.0:
                continue
            test = np.zeros(nz)
            test[:na] = ut[l]
            test[na + f * m:na + (f + 1) * m] = -phi[l]
            trial = np.zeros(nz)
            if wn[l] > 0:
                trial[:na] = ut[l]
            else:
                trial[na + f * m:na + (f + 1) * m] = phi[l]
            C += (L * om[l] * wn[l]) * np.outer(test, trial)
        if getattr(lv, "outflow", None) is not None and lv.outflow[E]:
            # do-nothing facet: + <(w.n) u, vhat> (tangential: the facet
            # unknown's test; normal: the cell's normal trace), so that the
            # natural condition is (nu grad u - p I) n = 0 rather than the
            # total-flux condition (with - (w.n) u) that the conservative
            # volume form leaves on a one-sided facet
            un = Pv @ nK
            for l in range(len(s)):
                tt = np.zeros(nz)
                tt[na + f * m:na + (f + 1) * m] = phi[l]
                tn = np.zeros(nz)
                tn[:na] = un[l]
                tr_t = np.zeros(nz)
                tr_t[:na] = ut[l]
                tr_n = np.zeros(nz)
                tr_n[:na] = un[l]
                C += (L * om[l] * wn[l]) * (np.outer(tt, tr_t) + np.outer(tn, tr_n))
    return C


def newton_matrix(e, wind, z_prev):
    """N [nz, nz] (row: test, column: trial) of the Newton term
    C_h(du; u_prev, v) for the increment du (trial: RT coefficients only),
    the previous velocity wind(X) (u_prev in this cell) and its local state
    z_prev (RT coefficients, then tangential facet traces; the upwind value
    on a facet is the cell's trace t(u_prev) where u_prev.n_K > 0 and the
    facet unknown uhat_prev where u_prev.n_K < 0)."""
    lv, K, k, m = e.lv, e.K, e.k, e.m
    na, nz = e.na, e.nz
    N = np.zeros((nz, nz))
    nc = convection_points(k)
    vs = np.sort(lv.cells[K])
    X, w = quad.data_points(lv.coords[vs], nc)
    wq = w * e.area
    val, grd, _ = e.rt.eval(X)
    U = wind(X)
    # - sum_ij (u_prev,i du_j, d_j v_i): trial a (du = u_a), test b
    N[:na, :na] -= np.einsum("q,qi,qaj,qbij->ba", wq, U, val, grd)
    s, om = quad.gauss_legendre01(nc)
    phi = hdg.facet_basis(k, s)
    for f in range(3):
        E = lv.cell_facets[K, f]
        if lv.int_id[E] < 0:
            # boundary facet: the increment's normal trace vanishes there
            # (and u_prev.n_K is zero up to rounding, so no switch is taken)
            continue
        X0 = lv.coords[lv.edges[E, 0]]
        X1 = lv.coords[lv.edges[E, 1]]
        L = lv.length[E]
        t = lv.tangent[E]
        nK = lv.sigma[K, f] * lv.normal[E]
        xl = X0[None, :] + s[:, None] * (X1 - X0)[None, :]
        Pv, _, _ = e.rt.eval(xl)
        ut = Pv @ t                                  # [l, a]
        un = Pv @ nK                                 # [l, a]: du.n_K per trial
        wn = wind(xl) @ nK
        for l in range(len(s)):
            if wn[l] == 0.0:
                continue
            if wn[l] > 0:
                up = ut[l] @ z_prev[:na]
            else:
                up = phi[l] @ z_prev[na + f * m:na + (f + 1) * m]
            test = np.zeros(nz)
            test[:na] = ut[l]
            test[na + f * m:na + (f + 1) * m] = -phi[l]
            trial = np.zeros(nz)
            trial[:na] = un[l]
            N += (L * om[l] * up) * np.outer(test, trial)
        if getattr(lv, "outflow", None) is not None and lv.outflow[E]:
            # derivative of the do-nothing facet term in its first argument:
            # <(du.n) u_prev, v^>
            a_prev = z_prev[:na]
            for l in range(len(s)):
                upt = ut[l] @ a_prev
                upn = un[l] @ a_prev
                tt = np.zeros(nz)
                tt[na + f * m:na + (f + 1) * m] = phi[l]
                tn = np.zeros(nz)
                tn[:na] = un[l]
                trial = np.zeros(nz)
                trial[:na] = un[l]
                N += (L * om[l]) * (upt * np.outer(tt, trial) + upn * np.outer(tn, trial))
    return N


class OseenElement:
    """A cell of the Picard-linearised scheme: the Stokes element's forms
    plus the convection matrix, condensed without assuming symmetry.
    Fz_extra: an additional local load (both interior and facet rows), the
    Newton right-hand side."""

    def __init__(self, base, C, Fz_extra=None):
        self.base = base
        self.Fz_extra = Fz_extra
        self.H = base.H + C
        E, Zh, H = base.E, base.Zh, self.H
        HE = H @ E
        S = E.T @ HE
        self.Kyy = None
        if Zh.shape[1] > 0:
            self.Kyy = Zh.T @ H @ Zh
            self.EHZ = E.T @ H @ Zh
            S = S - self.EHZ @ np.linalg.solve(self.Kyy, Zh.T @ HE)
        self.S = S
        for name in ("lv", "K", "k", "m", "area", "d", "wq", "xq", "na", "nz", "E", "Zh", "Dm", "W",
                     "M", "R", "P", "rt", "mean_psi", "nu"):
            setattr(self, name, getattr(base, name))

    def load_z(self, f_q):
        Fz = self.base.load_z(f_q)
        return Fz if self.Fz_extra is None else Fz + self.Fz_extra

    def load(self, f_q):
        Fz = self.load_z(f_q)
        g = self.E.T @ Fz
        if self.Kyy is not None:
            g = g - self.EHZ @ np.linalg.solve(self.Kyy, self.Zh.T @ Fz)
        return g

    def recover_z(self, lam, f_q):
        Fz = self.load_z(f_q)
        z = self.E @ lam
        if self.Kyy is not None:
            z = z + self.Zh @ np.linalg.solve(self.Kyy, self.Zh.T @ (Fz - self.H @ z))
        return z, Fz

    def recover(self, lam, p0, f_q, X=None):
        z, Fz = self.recover_z(lam, f_q)
        a = z[:self.na]
        r = (self.H @ z - Fz)[:self.na]
        G = self.Dm @ self.W
        pi, *_ = np.linalg.lstsq(G.T, self.W.T @ r, rcond=None)
        X = self.xq if X is None else X
        val, grd, div = self.rt.eval(X)
        psi, _ = self.P.eval(X)
        u = np.einsum("pai,a->pi", val, a)
        p = p0 + (psi[:, 1:] - self.mean_psi[None, 1:]) @ pi
        Minv = np.linalg.inv(self.M)
        Lift = np.zeros((len(X), 2, 2))
        for i in range(2):
            for j in range(2):
                Lift[:, i, j] = psi @ (Minv @ (self.R[i, j] @ z))
        return u, p, -self.nu * Lift, div @ a


def zero_wind(X):
    return np.zeros((len(X), 2))


class OseenProblem(hdg.Problem):
    """Condensed Picard-linearised system on one level.  winds: one callable
    per cell (None: no convection).  dirichlet: [n_facets, k+1] tangential
    coefficients on the Dirichlet boundary facets, or [n_facets, 2, k+1]
    normal and tangential ones (an inflow); None: homogeneous.  Prescribed
    normal values change the cells' divergence by their flux (flux_b), which
    the AL-Uzawa loop and the direct solve carry.  transpose: the
    transposed system (convection matrices transposed per cell)."""

    def __init__(self, lv, k, nu, beta, gamma, winds=None, dirichlet=None, transpose=False, newton_z=None):
        super().__init__(lv, k, nu, beta, gamma)
        if winds is not None:
            def cell(e, K):
                C = convection_matrix(e, winds[K])
                if newton_z is not None:
                    # Jacobian C + N, load C z_prev (= C_h(u_prev; u_prev, .))
                    Nm = newton_matrix(e, winds[K], newton_z[K])
                    return OseenElement(e, C + Nm, C @ newton_z[K])
                return OseenElement(e, C.T.copy() if transpose else C)
            self.elems = [cell(e, K) for K, e in enumerate(self.elems)]
        self.dirichlet = dirichlet

    def boundary_local(self, K):
        """Local skeleton vector holding only the prescribed boundary values."""
        out = np.zeros(6 * self.m)
        if self.dirichlet is None:
            return out
        lv = self.lv
        full = np.ndim(self.dirichlet) == 3
        for f in range(3):
            E = lv.cell_facets[K, f]
            if lv.int_id[E] < 0:
                for j in range(self.m):
                    if full:
                        out[hdg.lam_index(self.k, f, 0, j)] = self.dirichlet[E, 0, j]
                        out[hdg.lam_index(self.k, f, 1, j)] = self.dirichlet[E, 1, j]
                    else:
                        out[hdg.lam_index(self.k, f, 1, j)] = self.dirichlet[E, j]
        return out

    def flux_b(self):
        """Per cell |K| div of the prescribed boundary values: d . (boundary
        part of the local skeleton vector), [n_cells]."""
        return np.array([e.d @ self.boundary_local(K) for K, e in enumerate(self.elems)])

    def constraint_rhs(self):
        return self.flux_b()

    def rhs(self, f_qp):
        g = np.zeros(self.n_dof)
        for K, e in enumerate(self.elems):
            gk = e.load(f_qp[K]) - e.S @ self.boundary_local(K)
            idx = self.gidx[K]
            keep = idx >= 0
            np.add.at(g, idx[keep], gk[keep])
        return g

    def local(self, lam, K):
        return super().local(lam, K) + self.boundary_local(K)


# ------------------------------------------------------------- winds
def state_wind(prob, lam, p0, f_qp):
    """Per-cell callables of the velocity u_h of a solved state."""
    def make(K):
        e = prob.elems[K]
        lk = prob.local(lam, K)
        return lambda X: e.recover(lk, p0[K], f_qp[K], X)[0]
    return [make(K) for K in range(prob.lv.n_cells)]


def facet_fluxes(lv, winds, n_gauss=8):
    """int_F w . n_F over every unknown-carrying facet (from the first
    adjacent cell); zero on Dirichlet boundary facets (the coarse-level
    winds of the preconditioner carry no flux through them)."""
    s, om = quad.gauss_legendre01(n_gauss)
    flux = np.zeros(lv.n_facets)
    for E in range(lv.n_facets):
        if lv.int_id[E] < 0:
            continue
        K = lv.facet_cells[E, 0]
        X0, X1 = lv.coords[lv.edges[E, 0]], lv.coords[lv.edges[E, 1]]
        xl = X0[None, :] + s[:, None] * (X1 - X0)[None, :]
        flux[E] = lv.length[E] * om @ (winds[K](xl) @ lv.normal[E])
    return flux


def coarsen_fluxes(lc, lf, flux_f):
    """Coarse facet flux = sum of the fluxes through its two halves (the
    half from coarse vertex a to the midpoint vertex of coarse facet E,
    which refinement numbers n_vertices(coarse) + E)."""
    nvc = len(lc.coords)
    flux_c = np.zeros(lc.n_facets)
    for F in range(lf.n_facets):
        a, b = lf.edges[F]
        if a < nvc <= b:
            E = b - nvc
            flux_c[E] += flux_f[F] * (lf.normal[F] @ lc.normal[E])
    return flux_c


def rt0_winds(lv, flux):
    """Per-cell callables of the RT0 field with the given facet fluxes."""
    def make(K):
        sig = np.array([lv.sigma[K, f] * flux[lv.cell_facets[K, f]] for f in range(3)])
        return lambda X: np.einsum("pia,i->pa", cr.rt0_basis(lv, K, X), sig)
    return [make(K) for K in range(lv.n_cells)]


# ------------------------------------------------------------- MG_h blocks
class OseenHierarchy(mg.Hierarchy):
    """Lowest-order levels with the convection of the RT0-projected wind
    (flux: facet fluxes of the wind on the finest level; None: Stokes)."""

    def __init__(self, levels, nu_fine, beta, eps_inv, flux=None, harmonic=True, transpose=False, smoother="gs",
                 patch="vertex"):
        self.levels = levels
        J = len(levels)
        nus = [None] * J
        nus[-1] = np.broadcast_to(np.asarray(nu_fine, float), (levels[-1].n_cells,)).copy()
        for l in range(J - 1, 0, -1):
            nus[l - 1] = nus[l].reshape(-1, 4).mean(axis=1)
        self.nus = nus
        fluxes = [None] * J
        if flux is not None:
            fluxes[-1] = flux
            for l in range(J - 1, 0, -1):
                fluxes[l - 1] = coarsen_fluxes(levels[l - 1], levels[l], fluxes[l])
        self.fluxes = fluxes
        self.A = []
        for l, lv in enumerate(levels):
            winds = None if flux is None else rt0_winds(lv, fluxes[l])
            pr = OseenProblem(lv, 0, nus[l], beta, eps_inv, winds, transpose=transpose)
            self.A.append(pr.matrix_Aeps().tocsr())
        self.smooth = [None] + [mg.PatchGS(self.A[l], levels[l], 1, smoother, patch) for l in range(1, J)]
        self.P, self.R = [None], [None]
        for l in range(1, J):
            Iavg = mg.averaging(levels[l - 1], levels[l])
            if harmonic:
                td = mg.interior_dofs(levels[l - 1], levels[l])
                Pl = mg.stabilised_transfer(self.A[l], Iavg, td)
                Rl = mg.stabilised_transfer(self.A[l].T.tocsr(), Iavg, td).T.tocsr()
            else:
                Pl, Rl = Iavg, Iavg.T.tocsr()
            self.P.append(Pl)
            self.R.append(Rl)
        self.coarse = np.linalg.inv(self.A[0].toarray())

    def mg_h(self, l, g, u0, m_l, q=1, growth=2):
        if l == 0:
            return self.coarse @ g
        u = u0.copy()
        for _ in range(m_l):
            self.smooth[l].forward(u, g)
        r = g - self.A[l] @ u
        rc = self.R[l] @ r
        du = np.zeros(len(rc))
        for _ in range(q):
            du = self.mg_h(l - 1, rc, du, growth * m_l, q, growth)
        u = u + self.P[l] @ du
        for _ in range(m_l):
            self.smooth[l].backward(u, g)
        return u


# ------------------------------------------------------------- FGMRES
def fgmres(A, b, prec, rtol=1e-8, atol=1e-10, max_it=500, x0=None, restart=50):
    """Flexible GMRES(restart), right preconditioning, modified Gram-Schmidt.
    Returns (x, iterations, Arnoldi residual history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    beta = np.linalg.norm(r)
    hist = [beta]
    tol = max(rtol * beta, atol)
    its = 0
    while beta > tol and its < max_it:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j_end = 0
        for j in range(restart):
            z = prec(V[j])
            Z.append(z)
            w = A @ z
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            for i in range(j):
                h0 = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = h0
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]))
            if hist[-1] <= tol or its >= max_it:
                break
        y = np.zeros(j_end)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_end] @ y[i + 1:]) / H[i, i]
        for i in range(j_end):
            x = x + y[i] * Z[i]
        if hist[-1] <= tol:
            break
        r = b - A @ x
        beta = np.linalg.norm(r)
    return x, its, hist


# ------------------------------------------------------------- drivers
class OseenSetup:
    """R2 for one Picard step: AL-Uzawa with FGMRES inner solves (x_0 = the
    latest skeleton iterate) preconditioned by MG_hp with the lowest-order
    Oseen hierarchy."""

    def __init__(self, levels, k, nu, beta, gamma, winds=None, dirichlet=None, m_p=1, m_h=1,
                 q=1, growth=2, restart=50, transpose=False, newton_z=None, smoother="gs", additive=False,
                 patch_relax="vertex", patch_smooth="vertex"):
        self.levels = levels
        self.lv = levels[-1]
        self.k = k
        self.prob = OseenProblem(self.lv, k, nu, beta, gamma, winds, dirichlet, transpose, newton_z)
        self.Aeps = self.prob.matrix_Aeps().tocsr()
        self.D = self.prob.matrix_D().tocsr()
        self.eps_inv = self.prob.eps_inv
        flux = None if winds is None else facet_fluxes(self.lv, winds)
        self.hier = OseenHierarchy(levels, self.prob.nu_c, beta, self.eps_inv, flux,
                                   transpose=transpose, smoother=smoother, patch=patch_smooth)
        self.prec = mg.HPMG(self.Aeps, self.lv, k, self.hier, m_p, m_h, q, growth, smoother, additive, patch_relax)
        self.restart = restart

    def solve(self, f_qp, lam0=None, rtol=1e-8, atol=1e-10, max_it=500, uzawa_max=50,
              uzawa_tol=1e-10, p_init=None):
        """p_init: the initial pressure of the AL-Uzawa loop (zero for the
        Picard form; the previous pressure for a Newton step, which makes
        the loop on (u_n, p_n) the paper's loop on the increments from
        zero).  uzawa_tol < 0: exactly uzawa_max steps."""
        g = self.prob.rhs(f_qp)
        p = np.zeros(self.lv.n_cells) if p_init is None else p_init.copy()
        lam = np.zeros(self.prob.n_dof) if lam0 is None else lam0.copy()
        log = []
        area = self.lv.area
        fb = self.prob.flux_b()
        # the AL term of the prescribed flux: A^eps lam = g + D^T p - eps^-1 D^T (flux_b / |K|)
        g = g - self.eps_inv * (self.D.T @ (fb / area))
        for n in range(uzawa_max):
            b = g + self.D.T @ p
            lam, its, hist = fgmres(self.Aeps, b, self.prec, rtol, atol, max_it, lam, self.restart)
            log.append((its, hist))
            dp = -self.eps_inv * (self.D @ lam + fb) / area
            p = p + dp
            dn = np.sqrt(np.sum(area * dp ** 2))
            pn = np.sqrt(np.sum(area * p ** 2))
            if dn <= uzawa_tol * max(1.0, pn):
                break
        return dict(g=g, lam=lam, p0=p, its=[l[0] for l in log], hist=[l[1] for l in log])


def lid_dirichlet(lv, k, top=1.0):
    """uhat = (1, 0) on the facets of the top side y = top: the facet L^2
    projection of a constant is its mode-0 coefficient (1, 0) . t_F."""
    D = np.zeros((lv.n_facets, k + 1))
    for E in range(lv.n_facets):
        if lv.int_id[E] < 0:
            a, b = lv.coords[lv.edges[E]]
            if abs(a[1] - top) < 1e-12 and abs(b[1] - top) < 1e-12:
                D[E, 0] = lv.tangent[E, 0]
    return D


def picard(levels, k, nu, beta, gamma, f_qp, n_steps, dirichlet=None, direct=False, **kw):
    """Stokes solve then n_steps Picard steps (wind = previous velocity).
    Returns the list of per-step dicts (lam, p0, its, u at the data points)."""
    out = []
    winds = None
    lam = None
    for n in range(n_steps + 1):
        S = OseenSetup(levels, k, nu, beta, gamma, winds, dirichlet, **kw)
        if direct:
            lam_d, p_d = S.prob.solve_direct(f_qp)
            r = dict(lam=lam_d, p0=p_d, its=[])
        else:
            r = S.solve(f_qp, lam0=lam)
        u, _, _, _ = S.prob.recover(r["lam"], r["p0"], f_qp)
        r["u"] = u
        r["setup"] = S
        out.append(r)
        winds = state_wind(S.prob, r["lam"], r["p0"], f_qp)
        lam = r["lam"]
    return out


def local_states(prob, lam, f_qp):
    """Per-cell local state z (RT coefficients, tangential facet traces) of
    a solved skeleton vector (boundary values included)."""
    return [e.recover_z(prob.local(lam, K), f_qp[K])[0] for K, e in enumerate(prob.elems)]


def l2_diff(prob, u1, u2):
    W = np.array([e.wq for e in prob.elems])
    return float(np.sqrt(np.sum(W[:, :, None] * (u1 - u2) ** 2)))


def picard_newton(levels, k, nu, beta, gamma, f_qp, dirichlet=None, eps_picard=1e-4, newton_rtol=1e-8,
                  newton_atol=1e-10, max_picard=50, max_newton=20, direct=False, solve_kw=None, dt_inv=0.0,
                  **kw):
    """Alg. 3: a Stokes solve, Picard steps until ||u_n - u_{n-1}||_0 <
    eps_picard, then Newton steps until ||u_n - u_{n-1}||_0 <=
    max(newton_rtol ||u_n||_0, newton_atol); every step starts from the
    previous skeleton vector, a Newton step's AL-Uzawa loop from the
    previous pressure.  dt_inv > 0: the Stokes and Picard steps are
    backward-Euler pseudo-time steps (Sec. 5.2.2), (u_n - u_{n-1}) dt_inv
    added to the equation: beta + dt_inv in the operator, f + dt_inv
    u_{n-1} as the load (u_{-1} = 0).  solve_kw: options of
    OseenSetup.solve.  Returns the per-step dicts (kind, lam, p0, u, its,
    du)."""
    out = []
    solve_kw = solve_kw or {}
    winds = zs = lam = u_prev = p_prev = None
    kind = "stokes"
    n_p = n_n = 0
    while True:
        nz_ = zs if kind == "newton" else None
        pt = dt_inv > 0.0 and kind != "newton"
        beta_s = beta + dt_inv if pt else beta
        f_s = f_qp + dt_inv * u_prev if pt and u_prev is not None else f_qp
        if direct:
            prob = OseenProblem(levels[-1], k, nu, beta_s, gamma, winds, dirichlet, newton_z=nz_)
            lam_d, p_d = prob.solve_direct(f_s)
            r = dict(lam=lam_d, p0=p_d, its=[])
            S = None
        else:
            S = OseenSetup(levels, k, nu, beta_s, gamma, winds, dirichlet, newton_z=nz_, **kw)
            prob = S.prob
            r = S.solve(f_s, lam0=lam, p_init=p_prev if kind == "newton" else None, **solve_kw)
        u, _, _, _ = prob.recover(r["lam"], r["p0"], f_s)
        du = None if u_prev is None else l2_diff(prob, u, u_prev)
        r.update(kind=kind, u=u, du=du, setup=S, prob=prob)
        out.append(r)
        unorm = l2_diff(prob, u, 0.0 * u)
        if kind == "newton":
            n_n += 1
            if du <= max(newton_rtol * unorm, newton_atol) or n_n >= max_newton:
                break
        else:
            if kind == "picard":
                n_p += 1
            if kind == "picard" and (du < eps_picard or n_p >= max_picard):
                kind = "newton"
            elif kind == "stokes":
                kind = "picard"
        # the next linearisation at this step's fields (recovered with the
        # load this step solved with)
        winds = state_wind(prob, r["lam"], r["p0"], f_s)
        zs = local_states(prob, r["lam"], f_s)
        lam, u_prev, p_prev = r["lam"], u, r["p0"]
    return out
