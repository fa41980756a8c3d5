"""hp-multigrid preconditioner (oracle; test infrastructure only).

* Vertex-patch subspaces (Sec. 3.4.2): the patch of vertex s holds every
  unknown on the interior facets containing s.  Block Gauss-Seidel visits
  the patches colour by colour (canonical colouring of the vertex graph,
  mesh.Level.vertex_colours) and does x_s += (A_ss)^-1 (b - A x)_s; the
  transposed sweep visits the colours in reverse order.  Patches of one
  colour share no cell, so their order within a colour does not matter.
* Intergrid transfer (avgOpt, div-transfer, harmonic-ex): I averages the
  coarse CR field at fine facet midpoints (the mean of the two sides on a
  coarse facet); the stabilised transfer is (id - P^T) I with P^T the
  A^eps-orthogonal projection onto the fine unknowns strictly inside coarse
  cells; restriction is its transpose.
* MG_h (Alg. 1) with an exact coarsest solve, q = 1 (V) or 2 (W), and
  m(l-1) = growth * m(l); MG_hp (Alg. 2) with the natural inclusion of the
  lowest-order space (mode 0 of every facet component) and its transpose.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cr


class PatchGS:
    """Vertex-patch block Gauss-Seidel on a level with m modes per component
    (patch="edge": one facet per patch, mesh.Level.facet_patches);
    with smoother="jacobi" the damped block Jacobi smoother (eq. bjac)
    instead: x += s sum_s E_s (A_ss)^-1 E_s^T (b - A x), every patch from
    the same residual, s = 1 / (number of colours) (within one colour the
    patch projections are A-orthogonal, so their sum is a projection and
    the sum over all patches is bounded by the colour count); it is its own
    transpose."""

    def __init__(self, A, lv, m, smoother="gs", patch="vertex"):
        self.A = A.tocsr()
        self.jacobi = smoother == "jacobi"
        if patch == "edge":
            # edge (facet) patches: one facet's unknowns per patch
            fp, fcol = lv.facet_patches()
            col = fcol
            vf = fp
        else:
            col = lv.vertex_colours()
            vf = lv.vertex_facets()
        self.colours = []
        for c in range(int(col.max()) + 1):
            pats = []
            for v in np.where(col == c)[0]:
                fs = vf[v]
                if not fs:
                    continue
                d = np.array([(lv.int_id[f] * 2 + cc) * m + j
                              for f in fs for cc in range(2) for j in range(m)])
                rows = self.A[d]
                Ass = rows[:, d].toarray()
                pats.append((d, rows, np.linalg.inv(Ass)))
            self.colours.append(pats)
        self.damp = 1.0 / len(self.colours)

    def _jacobi(self, x, b):
        r = b - self.A @ x
        dx = np.zeros_like(x)
        for pats in self.colours:
            for d, rows, Ainv in pats:
                dx[d] += Ainv @ r[d]
        x += self.damp * dx

    def forward(self, x, b):
        if self.jacobi:
            return self._jacobi(x, b)
        for pats in self.colours:
            for d, rows, Ainv in pats:
                x[d] += Ainv @ (b[d] - rows @ x)

    def backward(self, x, b):
        if self.jacobi:
            return self._jacobi(x, b)
        for pats in reversed(self.colours):
            for d, rows, Ainv in pats:
                x[d] += Ainv @ (b[d] - rows @ x)


def averaging(lc, lf):
    """Sparse I_{l-1}^l from coarse level lc to fine level lf (2-DOF facets)."""
    rows, cols, vals = [], [], []

    def cr_value_weights(T, x):
        """Coarse CR field on cell T at x, as weights on coarse DOFs:
        list of (dof, 2-vector)."""
        V = lc.coords[lc.cells[T]]
        # barycentric coordinates
        Mb = np.array([[V[0, 0], V[1, 0], V[2, 0]], [V[0, 1], V[1, 1], V[2, 1]], [1, 1, 1]])
        lam = np.linalg.solve(Mb, np.array([x[0], x[1], 1.0]))
        out = []
        for i, E in enumerate(lc.cell_facets[T]):
            ei = lc.int_id[E]
            if ei < 0:
                continue
            phi = 1.0 - 2.0 * lam[i]
            out.append((2 * ei + 0, phi * lc.normal[E]))
            out.append((2 * ei + 1, phi * lc.tangent[E]))
        return out, lam

    for F in np.where(lf.dof)[0]:
        fi = lf.int_id[F]
        x = lf.midpoint[F]
        Kf = lf.facet_cells[F, 0]
        T = lf.parent[Kf]
        w, lam = cr_value_weights(T, x)
        if lam.min() < -1e-12:
            raise AssertionError("midpoint outside parent")
        if lam.min() < 1e-12:
            i0 = int(np.argmin(lam))
            E = lc.cell_facets[T, i0]
            if lc.interior[E]:
                # the mean of the two sides on a coarse interior facet
                a, b = lc.facet_cells[E]
                T2 = b if a == T else a
                w2, _ = cr_value_weights(T2, x)
                w = [(d, 0.5 * v) for d, v in w] + [(d, 0.5 * v) for d, v in w2]
            else:
                # a fine do-nothing facet on a coarse one: the one side
                assert lc.outflow[E], "fine dof facet on a coarse Dirichlet facet"
        for d, v in w:
            rows += [2 * fi, 2 * fi + 1]
            cols += [d, d]
            vals += [v @ lf.normal[F], v @ lf.tangent[F]]
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * lf.n_int, 2 * lc.n_int))


def interior_dofs(lc, lf):
    """Fine DOFs on fine facets whose midpoints lie strictly inside a coarse
    cell."""
    out = []
    for F in np.where(lf.interior)[0]:
        x = lf.midpoint[F]
        T = lf.parent[lf.facet_cells[F, 0]]
        V = lc.coords[lc.cells[T]]
        Mb = np.array([[V[0, 0], V[1, 0], V[2, 0]], [V[0, 1], V[1, 1], V[2, 1]], [1, 1, 1]])
        lam = np.linalg.solve(Mb, np.array([x[0], x[1], 1.0]))
        if lam.min() > 1e-12:
            fi = lf.int_id[F]
            out += [2 * fi, 2 * fi + 1]
    return np.array(sorted(out))


def stabilised_transfer(Af, Iavg, tdofs):
    """(id - P^T) I with P^T = E_T (E_T^T A E_T)^-1 E_T^T A."""
    n = Af.shape[0]
    ATT = Af[tdofs][:, tdofs].tocsc()
    AI = (Af @ Iavg).tocsr()[tdofs].toarray()
    corr = spla.splu(ATT).solve(AI)
    Pcorr = np.zeros((n, Iavg.shape[1]))
    Pcorr[tdofs] = corr
    return sp.csr_matrix(Iavg.toarray() - Pcorr)


class Hierarchy:
    """Lowest-order levels 1..J with transfers and smoothers."""

    def __init__(self, levels, nu_fine, beta, eps_inv, harmonic=True, smoother="gs", patch="vertex"):
        self.levels = levels
        J = len(levels)
        nus = [None] * J
        nus[-1] = np.broadcast_to(np.asarray(nu_fine, float), (levels[-1].n_cells,)).copy()
        for l in range(J - 1, 0, -1):
            # coarse viscosity: mean over the four children
            nus[l - 1] = nus[l].reshape(-1, 4).mean(axis=1)
        self.nus = nus
        self.A = [cr.assemble(lv, nus[l], beta, eps_inv) for l, lv in enumerate(levels)]
        self.smooth = [None] + [PatchGS(self.A[l], levels[l], 1, smoother, patch) for l in range(1, J)]
        self.P = [None]
        for l in range(1, J):
            Iavg = averaging(levels[l - 1], levels[l])
            if harmonic:
                Pl = stabilised_transfer(self.A[l], Iavg, interior_dofs(levels[l - 1], levels[l]))
            else:
                Pl = Iavg
            self.P.append(Pl)
        self.coarse = np.linalg.inv(self.A[0].toarray())

    def mg_h(self, l, g, u0, m_l, q=1, growth=2):
        """Alg. 1 on level index l (0 = coarsest)."""
        if l == 0:
            return self.coarse @ g
        u = u0.copy()
        for _ in range(m_l):
            self.smooth[l].forward(u, g)
        r = g - self.A[l] @ u
        rc = self.P[l].T @ r
        du = np.zeros(len(rc))
        for _ in range(q):
            du = self.mg_h(l - 1, rc, du, growth * m_l, q, growth)
        u = u + self.P[l] @ du
        for _ in range(m_l):
            self.smooth[l].backward(u, g)
        return u


class HPMG:
    """Alg. 2 with zero initial guess: the preconditioner z = MG_hp(r).

    additive=True: the additive (parallel) counterpart of Remark 3.4 -- the
    relaxation (m_p forward then m_p transposed sweeps from zero on r) plus
    the lowest-order correction Pi_0^k MG_h(Pi_k^0 r), both from the same r."""

    def __init__(self, Ak, lv, k, hier, m_p=1, m_h=1, q=1, growth=2, smoother="gs", additive=False,
                 patch="vertex"):
        self.Ak, self.k, self.hier = Ak.tocsr(), k, hier
        self.m_p, self.m_h, self.q, self.growth = m_p, m_h, q, growth
        self.additive = additive
        m = k + 1
        self.mode0 = np.array([(f * 2 + c) * m for f in range(lv.n_int) for c in range(2)])
        self.relax = PatchGS(self.Ak, lv, m, smoother, patch) if k > 0 else None

    def __call__(self, g):
        J = len(self.hier.levels) - 1
        if self.k == 0:
            return self.hier.mg_h(J, g, np.zeros_like(g), self.m_h, self.q, self.growth)
        if self.additive:
            x = np.zeros_like(g)
            for _ in range(self.m_p):
                self.relax.forward(x, g)
            for _ in range(self.m_p):
                self.relax.backward(x, g)
            x[self.mode0] += self.hier.mg_h(J, g[self.mode0], np.zeros(len(self.mode0)), self.m_h,
                                            self.q, self.growth)
            return x
        x = np.zeros_like(g)
        for _ in range(self.m_p):
            self.relax.forward(x, g)
        r = g - self.Ak @ x
        d0 = self.hier.mg_h(J, r[self.mode0], np.zeros(len(self.mode0)), self.m_h,
                            self.q, self.growth)
        x[self.mode0] += d0
        for _ in range(self.m_p):
            self.relax.backward(x, g)
        return x
