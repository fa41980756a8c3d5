"""hp-multigrid preconditioner on tetrahedral meshes (oracle; test
infrastructure only).

* Edge-patch subspaces (Sec. 3.4.2, the edge-patch smoother the paper uses
  in three dimensions): the patch of edge e holds every unknown on the
  interior faces containing e.  Block Gauss-Seidel visits the patches
  colour by colour (mesh3d.Level3.edge_colours: greedy in edge order, edges
  of one colour share no cell) and does x_s += (A_ss)^-1 (b - A x)_s; the
  transposed sweep visits the colours in reverse order.
* Intergrid transfer (avgOpt, div-transfer, harmonic-ex): I evaluates the
  coarse CR field at the centroids of the fine faces (the mean of the two
  sides on a coarse face) and splits it in the fine face frame; the
  stabilised transfer is (id - P^T) I with P^T the A^eps-orthogonal
  projection onto the fine unknowns strictly inside coarse cells;
  restriction is its transpose.
* MG_h (Alg. 1) with an exact coarsest solve, MG_hp (Alg. 2) with the
  natural inclusion of the lowest-order space (mode 0 of every face
  component) and its transpose.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cr3d


class EdgePatchGS:
    """Edge-patch block Gauss-Seidel on a level with m modes per component;
    smoother="jacobi": the damped block Jacobi smoother (eq. bjac) with
    damping 1 / (number of colours), as mg.PatchGS; patch="vertex": vertex
    patches (every interior face containing the vertex, greedy vertex
    colouring) instead of edge patches."""

    def __init__(self, A, lv, m, smoother="gs", patch="edge"):
        self.A = A.tocsr()
        self.jacobi = smoother == "jacobi"
        if patch == "vertex":
            pats_of = lv.vertex_patches()
            col = lv.vertex_colours(pats_of)
        else:
            pats_of = lv.edge_patches()
            col = lv.edge_colours(pats_of)
        self.colours = []
        for c in range(int(col.max()) + 1):
            pats = []
            for e in np.where(col == c)[0]:
                fs = pats_of[e]
                d = np.array([(lv.int_id[f] * 3 + cc) * m + j
                              for f in fs for cc in range(3) for j in range(m)])
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


def _bary(lc, T, x):
    V = lc.coords[lc.cells[T]]
    Mb = np.vstack([V.T, np.ones(4)])
    return np.linalg.solve(Mb, np.array([x[0], x[1], x[2], 1.0]))


def averaging(lc, lf):
    """Sparse I_{l-1}^l from coarse level lc to fine level lf (3 unknowns per
    interior face)."""
    rows, cols, vals = [], [], []

    def cr_value_weights(T, x):
        lam = _bary(lc, T, x)
        out = []
        for i, E in enumerate(lc.cell_facets[T]):
            ei = lc.int_id[E]
            if ei < 0:
                continue
            phi = 1.0 - 3.0 * lam[i]
            out.append((3 * ei + 0, phi * lc.normal[E]))
            out.append((3 * ei + 1, phi * lc.t1[E]))
            out.append((3 * ei + 2, phi * lc.t2[E]))
        return out, lam

    for F in np.where(lf.interior)[0]:
        fi = lf.int_id[F]
        x = lf.centroid[F]
        T = lf.parent[lf.facet_cells[F, 0]]
        w, lam = cr_value_weights(T, x)
        if lam.min() < -1e-12:
            raise AssertionError("centroid outside parent")
        if lam.min() < 1e-12:
            i0 = int(np.argmin(lam))
            E = lc.cell_facets[T, i0]
            assert lc.interior[E], "fine interior face on a coarse boundary face"
            a, b = lc.facet_cells[E]
            T2 = b if a == T else a
            w2, _ = cr_value_weights(T2, x)
            w = [(d, 0.5 * v) for d, v in w] + [(d, 0.5 * v) for d, v in w2]
        for d, v in w:
            rows += [3 * fi, 3 * fi + 1, 3 * fi + 2]
            cols += [d, d, d]
            vals += [v @ lf.normal[F], v @ lf.t1[F], v @ lf.t2[F]]
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * lf.n_int, 3 * lc.n_int))


def interior_dofs(lc, lf):
    """Fine unknowns on fine faces whose centroids lie strictly inside a
    coarse cell."""
    out = []
    for F in np.where(lf.interior)[0]:
        T = lf.parent[lf.facet_cells[F, 0]]
        if _bary(lc, T, lf.centroid[F]).min() > 1e-12:
            fi = lf.int_id[F]
            out += [3 * fi, 3 * fi + 1, 3 * fi + 2]
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


class Hierarchy3:
    """Lowest-order levels 1..J on tetrahedra with transfers and smoothers."""

    def __init__(self, levels, nu_fine, beta, eps_inv, harmonic=True, smoother="gs", patch="edge"):
        self.levels = levels
        J = len(levels)
        nus = [None] * J
        nus[-1] = np.broadcast_to(np.asarray(nu_fine, float), (levels[-1].n_cells,)).copy()
        for l in range(J - 1, 0, -1):
            nus[l - 1] = nus[l].reshape(-1, 8).mean(axis=1)
        self.nus = nus
        self.A = [cr3d.assemble(lv, nus[l], beta, eps_inv) for l, lv in enumerate(levels)]
        self.smooth = [None] + [EdgePatchGS(self.A[l], levels[l], 1, smoother, patch) for l in range(1, J)]
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


class HPMG3:
    """Alg. 2 with zero initial guess on tetrahedra: z = MG_hp(r)."""

    def __init__(self, Ak, lv, k, hier, m_p=2, m_h=2, q=1, growth=2, smoother="gs", additive=False,
                 patch="edge"):
        self.Ak, self.k, self.hier = Ak.tocsr(), k, hier
        self.m_p, self.m_h, self.q, self.growth = m_p, m_h, q, growth
        self.additive = additive
        mF = (k + 1) * (k + 2) // 2
        self.mode0 = np.array([(f * 3 + c) * mF for f in range(lv.n_int) for c in range(3)])
        self.relax = EdgePatchGS(self.Ak, lv, mF, smoother, patch) if k > 0 else None

    def __call__(self, g):
        J = len(self.hier.levels) - 1
        if self.k == 0:
            return self.hier.mg_h(J, g, np.zeros_like(g), self.m_h, self.q, self.growth)
        if self.additive:
            # additive counterpart (Remark 3.4), as mg.HPMG
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
        d0 = self.hier.mg_h(J, r[self.mode0], np.zeros(len(self.mode0)), self.m_h, self.q, self.growth)
        x[self.mode0] += d0
        for _ in range(self.m_p):
            self.relax.backward(x, g)
        return x
