"""Local solver, static condensation and the condensed skeleton system of the
H(div)-HDG scheme (oracle; test infrastructure only).

Scheme (stWeak), Sec. 3.2: find (L_h, u_h, uhat_h, p_h) in
[P^k]^{2x2} x RT_k,0 x tangential-P^k_0 x P^k_0 with
  (nu^-1 L, G) + (grad u, G) - <tng(u - uhat), G n> = 0
  -(L, grad v) + <L n, tng(v - vhat)> + (beta u, v) - (p, div v) = (f, v)
  (div u, q) = 0.
The first equation gives L = -nu Lift(u, uhat) with Lift the P^k projection
defined by it; the second then reads
  nu (Lift(u,uhat), Lift(v,vhat)) + beta (u, v) - (p, div v) = (f, v).
Per cell the local unknowns (interior RT_k part and the mean-free pressure)
are eliminated (Sec. 3.2, the global/local split of Sec. 2): for given
skeleton data (normal trace of u and tangential trace uhat, each in P^k per
facet) the interior part minimises the cell energy
  1/2 [nu |Lift|^2 + beta |u|^2] - (f, u)
over RT_k fields with those normal traces and div u in P^0.  The Hessian of
the minimum in the skeleton data is the cell block S_K of A_{k,h}
(stOptForm); its gradient at zero data gives the load g_K.

Skeleton coefficients: per interior facet F, component c in {n, t} (global
frame n_F, t_F) and mode j of the facet basis
phi_j(s) = sqrt(2j+1) P_j(2s-1), orthonormal for (1/|F|) int_F:
  u.n_F = sum_j c^n_j phi_j,   uhat.t_F = sum_j c^t_j phi_j.
Global index: (int_id(F) * 2 + c) * (k+1) + j.  Cell-local index:
(i * 2 + c) * (k+1) + j for local facet i.

This module uses a monomial basis of RT_k = [P^k]^2 + x Ptilde^k in scaled
coordinates and eliminates the interior by the null-space method (SVD);
the HIP library uses a different basis and a different elimination, so that
agreement of the two is evidence about the condensed operator itself.
"""
import numpy as np
from numpy.polynomial import legendre
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import quad


def exponents(k):
    """Exponents (a, b) of the monomials of P^k, by degree."""
    return [(d - b, b) for d in range(k + 1) for b in range(d + 1)]


def facet_basis(k, s):
    """phi_j(s) = sqrt(2j+1) P_j(2s-1), j = 0..k; returns [len(s), k+1]."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros((len(s), k + 1))
    for j in range(k + 1):
        c = np.zeros(j + 1)
        c[j] = 1.0
        out[:, j] = np.sqrt(2 * j + 1) * legendre.legval(2 * s - 1, c)
    return out


class Monomials:
    """Scalar P^k monomials xi^alpha in xi = (x - xc)/h."""

    def __init__(self, k, xc, h):
        self.k, self.xc, self.h = k, np.asarray(xc, float), float(h)
        self.exps = exponents(k)
        self.n = len(self.exps)

    def eval(self, X):
        xi = (np.asarray(X, float) - self.xc) / self.h
        v = np.zeros((len(xi), self.n))
        g = np.zeros((len(xi), self.n, 2))
        for r, (a, b) in enumerate(self.exps):
            v[:, r] = xi[:, 0] ** a * xi[:, 1] ** b
            if a > 0:
                g[:, r, 0] = a * xi[:, 0] ** (a - 1) * xi[:, 1] ** b / self.h
            if b > 0:
                g[:, r, 1] = b * xi[:, 0] ** a * xi[:, 1] ** (b - 1) / self.h
        return v, g


class RTMonomials:
    """Basis of RT_k(K): (m,0), (0,m) for monomials m of degree <= k, then
    xi * m for monomials of degree exactly k (xi = (x - xc)/h)."""

    def __init__(self, k, xc, h):
        self.P = Monomials(k, xc, h)
        self.k = k
        self.top = [r for r, (a, b) in enumerate(self.P.exps) if a + b == k]
        self.n = 2 * self.P.n + len(self.top)

    def eval(self, X):
        """values [np, n, 2], gradients [np, n, 2, 2] with [..., i, j] =
        d u_i / d x_j, divergence [np, n]."""
        X = np.asarray(X, float)
        pv, pg = self.P.eval(X)
        xi = (X - self.P.xc) / self.P.h
        npn, nP = len(X), self.P.n
        val = np.zeros((npn, self.n, 2))
        grd = np.zeros((npn, self.n, 2, 2))
        for r in range(nP):
            val[:, r, 0] = pv[:, r]
            grd[:, r, 0, :] = pg[:, r, :]
            val[:, nP + r, 1] = pv[:, r]
            grd[:, nP + r, 1, :] = pg[:, r, :]
        for t, r in enumerate(self.top):
            c = 2 * nP + t
            for i in range(2):
                val[:, c, i] = xi[:, i] * pv[:, r]
                for j in range(2):
                    grd[:, c, i, j] = xi[:, i] * pg[:, r, j] + \
                        (pv[:, r] / self.P.h if i == j else 0.0)
        div = grd[:, :, 0, 0] + grd[:, :, 1, 1]
        return val, grd, div


def lam_index(k, i, c, j):
    """Cell-local skeleton index of local facet i, component c (0=n, 1=t),
    mode j."""
    return (i * 2 + c) * (k + 1) + j


class Element:
    """Local matrices and condensation of one cell.

    Attributes after construction:
      S    condensed block [6(k+1), 6(k+1)] (A_{k,h} restricted to the cell)
      d    AL vector: d . lambda_K = |K| (div u)_K (sigma_{K,F} |F| on the
           mode-0 normal coefficient of each facet)
    """

    def __init__(self, lv, K, k, nu, beta):
        self.lv, self.K, self.k, self.nu, self.beta = lv, K, k, float(nu), float(beta)
        m = k + 1
        self.m = m
        V = lv.coords[lv.cells[K]]
        self.area = lv.area[K]
        xc = V.mean(axis=0)
        h = max(np.linalg.norm(V[a] - V[b]) for a, b in ((0, 1), (1, 2), (2, 0)))
        self.rt = RTMonomials(k, xc, h)
        self.P = Monomials(k, xc, h)
        na, nP = self.rt.n, self.P.n
        self.na, self.nP = na, nP
        nz = na + 3 * m
        self.nz = nz
        # volume quadrature: data rule on the sorted vertices (exact to 2k+3)
        vs = np.sort(lv.cells[K])
        self.xq, w = quad.data_points(lv.coords[vs], k + 2)
        self.wq = w * self.area
        Phi, dPhi, divPhi = self.rt.eval(self.xq)
        psi, _ = self.P.eval(self.xq)
        self.Phi_q = Phi
        wq = self.wq
        M = psi.T @ (wq[:, None] * psi)
        R = np.zeros((2, 2, nP, nz))
        for i in range(2):
            for j in range(2):
                R[i, j, :, :na] = np.einsum("q,qr,qa->ra", wq, psi, dPhi[:, :, i, j])
        s, om = quad.gauss_legendre01(k + 2)
        phi = facet_basis(k, s)
        T = np.zeros((3 * m, na))
        self.d = np.zeros(6 * m)
        for f in range(3):
            e = lv.cell_facets[K, f]
            X0 = lv.coords[lv.edges[e, 0]]
            X1 = lv.coords[lv.edges[e, 1]]
            L = lv.length[e]
            t = lv.tangent[e]
            n = lv.normal[e]
            nK = lv.sigma[K, f] * n
            xl = X0[None, :] + s[:, None] * (X1 - X0)[None, :]
            Pv, _, _ = self.rt.eval(xl)
            ps, _ = self.P.eval(xl)
            ut = Pv @ t
            un = Pv @ n
            for i in range(2):
                for j in range(2):
                    R[i, j, :, :na] -= np.einsum("l,lr,la->ra", L * om, ps, ut) * t[i] * nK[j]
                    R[i, j, :, na + f * m:na + (f + 1) * m] += \
                        np.einsum("l,lr,lm->rm", L * om, ps, phi) * t[i] * nK[j]
            T[f * m:(f + 1) * m, :] = np.einsum("l,lm,la->ma", om, phi, un)
            self.d[lam_index(k, f, 0, 0)] = lv.sigma[K, f] * L
        self.M, self.R, self.T = M, R, T
        Minv = np.linalg.inv(M)
        H = np.zeros((nz, nz))
        for i in range(2):
            for j in range(2):
                H += nu * R[i, j].T @ Minv @ R[i, j]
        H[:na, :na] += beta * np.einsum("q,qai,qbi->ab", wq, Phi, Phi)
        self.H = H
        # divergence constraint against the mean-free part of P^k
        mean = (wq @ psi) / self.area
        q_mf = psi[:, 1:] - mean[None, 1:]
        self.mean_psi = mean
        Dm = q_mf.T @ (wq[:, None] * divPhi)
        self.Dm = Dm
        # null-space elimination of the interior
        C = np.vstack([T, Dm])
        U, sv, Vt = np.linalg.svd(C)
        nc = C.shape[0]
        assert sv[-1] > 1e-12 * sv[0], "constraint matrix rank deficient"
        Z = Vt[nc:].T
        Cp = np.linalg.pinv(C)
        E = np.zeros((nz, 6 * m))
        for f in range(3):
            for j in range(m):
                E[:na, lam_index(k, f, 0, j)] = Cp[:, f * m + j]
                E[na + f * m + j, lam_index(k, f, 1, j)] = 1.0
        Zh = np.vstack([Z, np.zeros((3 * m, Z.shape[1]))])
        self.E, self.Zh = E, Zh
        HE = H @ E
        S = E.T @ HE
        if Zh.shape[1] > 0:
            self.Kyy = Zh.T @ H @ Zh
            self.X = np.linalg.solve(self.Kyy, Zh.T @ HE)
            S = S - HE.T @ Zh @ self.X
        else:
            self.Kyy = None
        self.S = 0.5 * (S + S.T)
        # interior bubbles (zero normal trace) for the pressure recovery
        _, st, Vtt = np.linalg.svd(T)
        self.W = Vtt[T.shape[0]:].T

    # -- loads and recovery ----------------------------------------------
    def load_z(self, f_q):
        """F_z: (f, u_a) for the RT basis by the data rule, zero on uhat."""
        Fz = np.zeros(self.nz)
        Fz[:self.na] = np.einsum("q,qai,qi->a", self.wq, self.Phi_q, f_q)
        return Fz

    def load(self, f_q):
        """Condensed load g_K for source values f_q [n_q, 2] at the data points."""
        Fz = self.load_z(f_q)
        g = self.E.T @ Fz
        if self.Kyy is not None:
            y = np.linalg.solve(self.Kyy, self.Zh.T @ Fz)
            g = g - (self.H @ self.E).T @ self.Zh @ y
        return g

    def recover_z(self, lam, f_q):
        Fz = self.load_z(f_q)
        z = self.E @ lam
        if self.Kyy is not None:
            y = np.linalg.solve(self.Kyy, self.Zh.T @ (Fz - self.H @ z))
            z = z + self.Zh @ y
        return z, Fz

    def recover(self, lam, p0, f_q, X=None):
        """Local recovery at points X (default: the data points).
        Returns (u [np,2], p [np], L [np,2,2], div u [np])."""
        z, Fz = self.recover_z(lam, f_q)
        a = z[:self.na]
        # mean-free pressure from the interior-bubble equations
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


class Problem:
    """Condensed skeleton system on one level (stOptForm, stALform).

    nu: scalar or per-cell array; gamma: the augmented-Lagrangian weight,
    eps^-1 = gamma * nu_ref with nu_ref = 1 (the paper's normalisation
    (nu eps)^-1 for unit viscosity)."""

    def __init__(self, lv, k, nu, beta, gamma):
        self.lv, self.k = lv, k
        self.m = k + 1
        nu_c = np.broadcast_to(np.asarray(nu, float), (lv.n_cells,))
        self.nu_c = nu_c
        self.beta = float(beta)
        self.eps_inv = float(gamma)
        self.elems = [Element(lv, K, k, nu_c[K], beta) for K in range(lv.n_cells)]
        self.n_dof = lv.n_int * 2 * self.m
        self.gidx = np.zeros((lv.n_cells, 6 * self.m), dtype=np.int64)
        for K in range(lv.n_cells):
            for f in range(3):
                fi = lv.int_id[lv.cell_facets[K, f]]
                for c in range(2):
                    for j in range(self.m):
                        li = lam_index(k, f, c, j)
                        self.gidx[K, li] = -1 if fi < 0 else (fi * 2 + c) * self.m + j

    def _assemble(self, blocks):
        rows, cols, vals = [], [], []
        for K, B in enumerate(blocks):
            g = self.gidx[K]
            keep = g >= 0
            gi = g[keep]
            Bk = B[np.ix_(keep, keep)]
            rows.append(np.repeat(gi, len(gi)))
            cols.append(np.tile(gi, len(gi)))
            vals.append(Bk.ravel())
        n = self.n_dof
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))

    def matrix_A(self):
        """A_{k,h} (no AL term)."""
        return self._assemble([e.S for e in self.elems])

    def matrix_Aeps(self):
        """A^eps = A + eps^-1 B*B with (B*B u, v) = (div u, div v)."""
        return self._assemble([e.S + self.eps_inv / e.area * np.outer(e.d, e.d)
                               for e in self.elems])

    def matrix_D(self):
        """D [n_cells, n_dof] with (D lambda)_K = |K| (div u)_K."""
        rows, cols, vals = [], [], []
        for K, e in enumerate(self.elems):
            g = self.gidx[K]
            keep = (g >= 0) & (e.d != 0)
            rows.append(np.full(keep.sum(), K))
            cols.append(g[keep])
            vals.append(e.d[keep])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.lv.n_cells, self.n_dof))

    def rhs(self, f_qp):
        """Global condensed load g for f_qp [n_cells, n_q, 2]."""
        g = np.zeros(self.n_dof)
        for K, e in enumerate(self.elems):
            gk = e.load(f_qp[K])
            idx = self.gidx[K]
            keep = idx >= 0
            np.add.at(g, idx[keep], gk[keep])
        return g

    def local(self, lam, K):
        idx = self.gidx[K]
        out = np.zeros(len(idx))
        keep = idx >= 0
        out[keep] = lam[idx[keep]]
        return out

    def recover(self, lam, p0, f_qp, points=None):
        """u, p, L, div u at the data points (or per-cell point lists)."""
        us, ps, Ls, ds = [], [], [], []
        for K, e in enumerate(self.elems):
            X = None if points is None else points[K]
            u, p, L, dv = e.recover(self.local(lam, K), p0[K], f_qp[K], X)
            us.append(u), ps.append(p), Ls.append(L), ds.append(dv)
        return np.array(us), np.array(ps), np.array(Ls), np.array(ds)

    def constraint_rhs(self):
        """-D lambda equals this per cell (the prescribed boundary flux; zero
        for homogeneous data)."""
        return np.zeros(self.lv.n_cells)

    def solve_direct(self, f_qp):
        """R1: the condensed saddle point [[A, -D^T, 0], [-D, 0, w], [0, w^T, 0]]
        with w_K = |K| (mean-free pressure), by sparse LU; with do-nothing
        facets the pressure is determined and [[A, -D^T], [-D, 0]] is
        solved.  Returns (lambda, p0 [n_cells])."""
        A = self.matrix_A()
        D = self.matrix_D()
        nK = self.lv.n_cells
        c = self.constraint_rhs()
        if getattr(self.lv, "outflow", None) is not None and self.lv.outflow.any():
            Kmat = sp.bmat([[A, -D.T], [-D, None]], format="csc")
            rhs = np.concatenate([self.rhs(f_qp), c])
        else:
            w = sp.csr_matrix(self.lv.area.reshape(-1, 1))
            Kmat = sp.bmat([[A, -D.T, None], [-D, None, w], [None, w.T, None]], format="csc")
            rhs = np.concatenate([self.rhs(f_qp), c, [0.0]])
        sol = spla.spsolve(Kmat, rhs)
        return sol[:self.n_dof], sol[self.n_dof:self.n_dof + nK]


def solve_uncondensed(lv, k, nu, beta, f_qp):
    """The scheme (stWeak) assembled without any elimination and solved by
    dense LU: unknowns L, RT_k coefficients per cell, full P^k pressure per
    cell, global normal and tangential facet coefficients, Lagrange
    multipliers tying each cell's normal traces to the facet coefficients,
    and one multiplier for the mean-free pressure.  Only for tiny meshes.
    Returns (c^n [n_int, k+1], c^t [n_int, k+1], per-cell objects)."""
    m = k + 1
    els = [Element(lv, K, k, nu, beta) for K in range(lv.n_cells)]
    e0 = els[0]
    na, nP = e0.na, e0.nP
    nK, nI = lv.n_cells, lv.n_int
    oL = 0
    oA = oL + nK * 4 * nP
    oP = oA + nK * na
    oN = oP + nK * nP
    oT = oN + nI * m
    oMu = oT + nI * m
    oTh = oMu + nK * 3 * m
    N = oTh + 1
    A = np.zeros((N, N))
    b = np.zeros(N)
    for K, e in enumerate(els):
        Lb = oL + K * 4 * nP
        Ab = oA + K * na
        Pb = oP + K * nP
        Mub = oMu + K * 3 * m
        # local z index -> global column (a part, then uhat per local facet)
        zcol = list(range(Ab, Ab + na))
        for f in range(3):
            fi = lv.int_id[lv.cell_facets[K, f]]
            for j in range(m):
                zcol.append(-1 if fi < 0 else oT + fi * m + j)
        zcol = np.array(zcol)
        psi_full = e.P.eval(e.xq)[0]
        _, _, divPhi = e.rt.eval(e.xq)
        Dfull = psi_full.T @ (e.wq[:, None] * divPhi)         # (div u_a, psi_r)
        for i in range(2):
            for j in range(2):
                rr = Lb + (i * 2 + j) * nP + np.arange(nP)
                # (1): nu^-1 M l_ij + R_ij z = 0
                A[np.ix_(rr, rr)] += e.M / e.nu
                for c in range(e.nz):
                    if zcol[c] >= 0:
                        A[rr, zcol[c]] += e.R[i, j][:, c]
                # (2): -sum_ij R_ij^T l_ij + ... in the z rows
                for c in range(e.nz):
                    if zcol[c] >= 0:
                        A[zcol[c], rr] -= e.R[i, j][:, c]
        massRT = np.einsum("q,qai,qbi->ab", e.wq, e.Phi_q, e.Phi_q)
        A[Ab:Ab + na, Ab:Ab + na] += beta * massRT
        A[Ab:Ab + na, Pb:Pb + nP] -= Dfull.T
        A[Ab:Ab + na, Mub:Mub + 3 * m] -= e.T.T
        b[Ab:Ab + na] += e.load_z(f_qp[K])[:na]
        # (3): (div u, psi_r) + theta int psi_r = 0
        A[Pb:Pb + nP, Ab:Ab + na] += Dfull
        A[Pb:Pb + nP, oTh] += e.wq @ psi_full
        A[oTh, Pb:Pb + nP] += e.wq @ psi_full
        # (4): T a - c^n = 0 ; multiplier force on c^n
        A[Mub:Mub + 3 * m, Ab:Ab + na] += e.T
        for f in range(3):
            fi = lv.int_id[lv.cell_facets[K, f]]
            if fi >= 0:
                for j in range(m):
                    A[Mub + f * m + j, oN + fi * m + j] -= 1.0
                    A[oN + fi * m + j, Mub + f * m + j] -= 1.0
    sol = np.linalg.solve(A, b)
    cn = sol[oN:oN + nI * m].reshape(nI, m)
    ct = sol[oT:oT + nI * m].reshape(nI, m)
    per_cell = []
    for K, e in enumerate(els):
        a = sol[oA + K * na:oA + (K + 1) * na]
        pc = sol[oP + K * nP:oP + (K + 1) * nP]
        per_cell.append((e, a, pc))
    return cn, ct, per_cell


def postprocess(e, lam, f_q, X=None):
    """Local post-processing (stPost) of one cell: u* in [P^{k+1}(K)]^2 with
    (grad u*_i, grad v)_K = (Lift_i., grad v)_K for all v in P^{k+1}(K) and
    (u*, w)_K = (u_h, w)_K for constant w; Lift(u, uhat) = -L_h / nu is the
    scheme's gradient approximation (the displayed right-hand side (L_h,
    grad v) drops the factor -1/nu of the mixed form nu^-1 L + grad u = 0).
    e: an Element (or OseenElement); returns u* at X (default: the data
    points) [np, 2]."""
    z, _ = e.recover_z(lam, f_q)
    k = e.k
    Minv = np.linalg.inv(e.M)
    coef = np.array([[Minv @ (e.R[i, j] @ z) for j in range(2)] for i in range(2)])   # [i, j, nP]
    Q = Monomials(k + 1, e.P.xc, e.P.h)
    lv, K = e.lv, e.K
    vs = np.sort(lv.cells[K])
    Xq, w = quad.data_points(lv.coords[vs], k + 3)   # exact to degree 2k+5
    w = w * e.area
    qv, qg = Q.eval(Xq)                              # [q, r], [q, r, j]
    psi, _ = e.P.eval(Xq)                            # P^k monomials of the lifting
    lift = np.einsum("ijr,qr->qij", coef, psi)
    uh = np.einsum("pai,a->pi", e.rt.eval(Xq)[0], z[:e.na])
    A = np.einsum("q,qrj,qsj->rs", w, qg, qg)
    mvec = w @ qv
    n = Q.n
    KKT = np.zeros((n + 1, n + 1))
    KKT[:n, :n] = A
    KKT[:n, n] = mvec
    KKT[n, :n] = mvec
    ustar_c = np.zeros((n, 2))
    for i in range(2):
        rhs = np.zeros(n + 1)
        rhs[:n] = np.einsum("q,qj,qrj->r", w, lift[:, i, :], qg)
        rhs[n] = w @ uh[:, i]
        ustar_c[:, i] = np.linalg.solve(KKT, rhs)[:n]
    X = e.xq if X is None else X
    return Q.eval(X)[0] @ ustar_c
