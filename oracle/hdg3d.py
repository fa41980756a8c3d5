"""Local solver, static condensation and the condensed skeleton system of the
H(div)-HDG scheme on tetrahedra (oracle; test infrastructure only).

The scheme (stWeak) of Sec. 3.2 in three dimensions: find (L_h, u_h, uhat_h,
p_h) in [P^k]^{3x3} x RT_k,0 x tangential-P^k_0 x P^k_0.  As in two
dimensions L = -nu Lift(u, uhat), with Lift the [P^k]^{3x3} function given
by (Lift, G) = (grad u, G) - <tng(u - uhat), G n_K> (tng(v) = v - (v.n) n),
and the interior of each cell minimises 1/2 [nu |Lift|^2 + beta |u|^2] -
(f, u) over RT_k fields with prescribed normal traces and div u in P^0; the
Hessian of that minimum in the skeleton data is the cell block S_K of
A_{k,h} (stOptForm) and its gradient at zero data the load g_K.

Skeleton coefficients: per interior face F, component c in {n, t1, t2}
(global face frame) and mode j of the face basis phi_j, orthonormal for the
normalised measure (1/|F|) int_F:
  u.n_F = sum_j c^n_j phi_j,   uhat = sum_j (c^t1_j t1_F + c^t2_j t2_F) phi_j.
Face basis: the Gram-Schmidt orthonormalisation (normalised measure on the
reference triangle {xi, eta >= 0, xi + eta <= 1}) of the monomials
xi^a eta^b ordered by total degree a+b, then by b; phi_0 = 1.  The affine
map of a face from its sorted vertices keeps the normalised inner product,
so the same polynomials in (xi, eta) are orthonormal on every face.
Global index: (int_id(F) * 3 + c) * m_F + j, m_F = (k+1)(k+2)/2.  Cell-local
index: (i * 3 + c) * m_F + j for local face i.

Monomial RT_k basis ([P^k]^3 + x Ptilde^k in scaled coordinates) and
null-space (SVD) elimination of the interior, as in the two-dimensional
module; the HIP library uses a different basis and elimination.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import quad


def exponents3(k):
    """Exponents (a, b, c) of the monomials of P^k in three variables."""
    out = []
    for d in range(k + 1):
        for c in range(d + 1):
            for b in range(d - c + 1):
                out.append((d - b - c, b, c))
    return out


def face_exponents(k):
    """(a, b) of xi^a eta^b ordered by degree, then by b."""
    return [(d - b, b) for d in range(k + 1) for b in range(d + 1)]


def face_basis_coeffs(k):
    """C [m_F, m_F] with phi = C @ monomials: Gram-Schmidt of the ordered
    monomials in the normalised L2 product on the reference triangle, i.e.
    phi_j = (m_j - sum_{i<j} (m_j, phi_i) phi_i) / |.| with positive leading
    coefficient.  Computed as the QR factorisation (positive diagonal) of
    the weighted monomial values at a rule exact to degree 2k+1, which is
    that Gram-Schmidt process (the Gram matrix of the monomials, with
    moments 2 a! b! / (a+b+2)!, is R^T R)."""
    ex = face_exponents(k)
    xi, w = quad.stroud_triangle(k + 1)
    V = np.stack([xi[:, 0] ** a * xi[:, 1] ** b for a, b in ex], axis=1)
    _, Rm = np.linalg.qr(np.sqrt(w)[:, None] * V)
    Rm = Rm * np.sign(np.diag(Rm))[:, None]
    return np.linalg.inv(Rm).T


def face_basis(k, xi, eta):
    """phi_j(xi, eta), j < m_F: [len(xi), m_F]."""
    C = face_basis_coeffs(k)
    ex = face_exponents(k)
    mono = np.stack([xi ** a * eta ** b for a, b in ex], axis=1)
    return mono @ C.T


class Monomials3:
    """Scalar P^k monomials xi^alpha in xi = (x - xc)/h."""

    def __init__(self, k, xc, h):
        self.k, self.xc, self.h = k, np.asarray(xc, float), float(h)
        self.exps = exponents3(k)
        self.n = len(self.exps)

    def eval(self, X):
        xi = (np.asarray(X, float) - self.xc) / self.h
        v = np.zeros((len(xi), self.n))
        g = np.zeros((len(xi), self.n, 3))
        for r, e in enumerate(self.exps):
            v[:, r] = xi[:, 0] ** e[0] * xi[:, 1] ** e[1] * xi[:, 2] ** e[2]
            for d in range(3):
                if e[d] > 0:
                    ee = list(e)
                    ee[d] -= 1
                    g[:, r, d] = e[d] * xi[:, 0] ** ee[0] * xi[:, 1] ** ee[1] * xi[:, 2] ** ee[2] / self.h
        return v, g


class RT3Monomials:
    """Basis of RT_k(K) in 3D: m e_i for monomials m of degree <= k and
    i = 0, 1, 2, then xi * m for monomials of degree exactly k."""

    def __init__(self, k, xc, h):
        self.P = Monomials3(k, xc, h)
        self.k = k
        self.top = [r for r, e in enumerate(self.P.exps) if sum(e) == k]
        self.n = 3 * self.P.n + len(self.top)

    def eval(self, X):
        """values [np, n, 3], gradients [np, n, 3, 3] ([..., i, j] = d u_i /
        d x_j), divergence [np, n]."""
        X = np.asarray(X, float)
        pv, pg = self.P.eval(X)
        xi = (X - self.P.xc) / self.P.h
        npn, nP = len(X), self.P.n
        val = np.zeros((npn, self.n, 3))
        grd = np.zeros((npn, self.n, 3, 3))
        for i in range(3):
            val[:, i * nP:(i + 1) * nP, i] = pv
            grd[:, i * nP:(i + 1) * nP, i, :] = pg
        for t, r in enumerate(self.top):
            c = 3 * nP + t
            for i in range(3):
                val[:, c, i] = xi[:, i] * pv[:, r]
                for j in range(3):
                    grd[:, c, i, j] = xi[:, i] * pg[:, r, j] + (pv[:, r] / self.P.h if i == j else 0.0)
        div = grd[:, :, 0, 0] + grd[:, :, 1, 1] + grd[:, :, 2, 2]
        return val, grd, div


def m_face(k):
    return (k + 1) * (k + 2) // 2


def lam_index(k, i, c, j):
    """Cell-local skeleton index of local face i, component c (0 = n,
    1 = t1, 2 = t2), mode j."""
    return (i * 3 + c) * m_face(k) + j


def face_points(lv, F, n):
    """Points of the Stroud rule (n per direction) on face F, their reference
    coordinates (xi, eta) and weights summing to 1."""
    xi, w = quad.stroud_triangle(n)
    X0, X1, X2 = (lv.coords[v] for v in lv.faces[F])
    pts = X0[None, :] + xi[:, :1] * (X1 - X0)[None, :] + xi[:, 1:2] * (X2 - X0)[None, :]
    return pts, xi[:, 0], xi[:, 1], w


class Element3:
    """Local matrices and condensation of one tetrahedron.

    S  condensed block [12 m_F, 12 m_F];  d  AL vector with
    d . lambda_K = |K| (div u)_K (sigma_{K,F} |F| on the mode-0 normal
    coefficient of each face)."""

    def __init__(self, lv, K, k, nu, beta):
        self.lv, self.K, self.k, self.nu, self.beta = lv, K, k, float(nu), float(beta)
        mF = m_face(k)
        self.mF = mF
        V = lv.coords[lv.cells[K]]
        self.area = lv.volume[K]          # |K| (named as in two dimensions)
        xc = V.mean(axis=0)
        h = max(np.linalg.norm(V[a] - V[b]) for a in range(4) for b in range(a + 1, 4))
        self.rt = RT3Monomials(k, xc, h)
        self.P = Monomials3(k, xc, h)
        na, nP = self.rt.n, self.P.n
        self.na, self.nP = na, nP
        nz = na + 4 * 2 * mF
        self.nz = nz
        vs = np.sort(lv.cells[K])
        self.xq, w = quad.tet_data_points(lv.coords[vs], k + 2)
        self.wq = w * self.area
        Phi, dPhi, divPhi = self.rt.eval(self.xq)
        psi, _ = self.P.eval(self.xq)
        self.Phi_q = Phi
        wq = self.wq
        M = psi.T @ (wq[:, None] * psi)
        R = np.zeros((3, 3, nP, nz))
        for i in range(3):
            for j in range(3):
                R[i, j, :, :na] = np.einsum("q,qr,qa->ra", wq, psi, dPhi[:, :, i, j])
        T = np.zeros((4 * mF, na))
        self.d = np.zeros(12 * mF)
        for f in range(4):
            F = lv.cell_facets[K, f]
            xl, s1, s2, om = face_points(lv, F, k + 2)
            A = lv.area_f[F]
            n = lv.normal[F]
            tt = (lv.t1[F], lv.t2[F])
            nK = lv.sigma[K, f] * n
            Pv, _, _ = self.rt.eval(xl)
            ps, _ = self.P.eval(xl)
            phi = face_basis(k, s1, s2)
            for c in range(2):
                t = tt[c]
                ut = Pv @ t
                off = na + (f * 2 + c) * mF
                lw = np.einsum("l,lr,la->ra", A * om, ps, ut)
                lp = np.einsum("l,lr,lm->rm", A * om, ps, phi)
                for i in range(3):
                    for j in range(3):
                        R[i, j, :, :na] -= lw * t[i] * nK[j]
                        R[i, j, :, off:off + mF] += lp * t[i] * nK[j]
            T[f * mF:(f + 1) * mF, :] = np.einsum("l,lm,la->ma", om, phi, Pv @ n)
            self.d[lam_index(k, f, 0, 0)] = lv.sigma[K, f] * A
        self.M, self.R, self.T = M, R, T
        Minv = np.linalg.inv(M)
        H = np.zeros((nz, nz))
        for i in range(3):
            for j in range(3):
                H += nu * R[i, j].T @ Minv @ R[i, j]
        H[:na, :na] += beta * np.einsum("q,qai,qbi->ab", wq, Phi, Phi)
        self.H = H
        mean = (wq @ psi) / self.area
        q_mf = psi[:, 1:] - mean[None, 1:]
        self.mean_psi = mean
        Dm = q_mf.T @ (wq[:, None] * divPhi)
        self.Dm = Dm
        C = np.vstack([T, Dm])
        U, sv, Vt = np.linalg.svd(C)
        nc = C.shape[0]
        assert sv[-1] > 1e-12 * sv[0], "constraint matrix rank deficient"
        Z = Vt[nc:].T
        Cp = np.linalg.pinv(C)
        E = np.zeros((nz, 12 * mF))
        for f in range(4):
            for j in range(mF):
                E[:na, lam_index(k, f, 0, j)] = Cp[:, f * mF + j]
                for c in range(2):
                    E[na + (f * 2 + c) * mF + j, lam_index(k, f, 1 + c, j)] = 1.0
        Zh = np.vstack([Z, np.zeros((8 * mF, Z.shape[1]))])
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
        _, st, Vtt = np.linalg.svd(T)
        self.W = Vtt[T.shape[0]:].T

    def load_z(self, f_q):
        Fz = np.zeros(self.nz)
        Fz[:self.na] = np.einsum("q,qai,qi->a", self.wq, self.Phi_q, f_q)
        return Fz

    def load(self, f_q):
        """Condensed load g_K for source values f_q [n_q, 3] at the data points."""
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
        """(u [np,3], p [np], L [np,3,3], div u [np]) at X (default: the data
        points)."""
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
        Lift = np.zeros((len(X), 3, 3))
        for i in range(3):
            for j in range(3):
                Lift[:, i, j] = psi @ (Minv @ (self.R[i, j] @ z))
        return u, p, -self.nu * Lift, div @ a


class Problem3:
    """Condensed skeleton system on one tetrahedral level (stOptForm,
    stALform); eps^-1 = gamma (unit reference viscosity)."""

    def __init__(self, lv, k, nu, beta, gamma):
        self.lv, self.k = lv, k
        self.mF = m_face(k)
        nu_c = np.broadcast_to(np.asarray(nu, float), (lv.n_cells,))
        self.nu_c = nu_c
        self.beta = float(beta)
        self.eps_inv = float(gamma)
        self.elems = [Element3(lv, K, k, nu_c[K], beta) for K in range(lv.n_cells)]
        self.n_dof = lv.n_int * 3 * self.mF
        self.gidx = np.zeros((lv.n_cells, 12 * self.mF), dtype=np.int64)
        for K in range(lv.n_cells):
            for f in range(4):
                fi = lv.int_id[lv.cell_facets[K, f]]
                for c in range(3):
                    for j in range(self.mF):
                        li = lam_index(k, f, c, j)
                        self.gidx[K, li] = -1 if fi < 0 else (fi * 3 + c) * self.mF + j

    def _assemble(self, blocks):
        rows, cols, vals = [], [], []
        for K, B in enumerate(blocks):
            g = self.gidx[K]
            keep = g >= 0
            gi = g[keep]
            rows.append(np.repeat(gi, len(gi)))
            cols.append(np.tile(gi, len(gi)))
            vals.append(B[np.ix_(keep, keep)].ravel())
        n = self.n_dof
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))

    def matrix_A(self):
        return self._assemble([e.S for e in self.elems])

    def matrix_Aeps(self):
        return self._assemble([e.S + self.eps_inv / e.area * np.outer(e.d, e.d) for e in self.elems])

    def matrix_D(self):
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
        us, ps, Ls, ds = [], [], [], []
        for K, e in enumerate(self.elems):
            X = None if points is None else points[K]
            u, p, L, dv = e.recover(self.local(lam, K), p0[K], f_qp[K], X)
            us.append(u), ps.append(p), Ls.append(L), ds.append(dv)
        return np.array(us), np.array(ps), np.array(Ls), np.array(ds)

    def solve_direct(self, f_qp):
        """R1: the condensed saddle point with the mean-free pressure
        multiplier, by sparse LU.  Returns (lambda, p0 [n_cells])."""
        A = self.matrix_A()
        D = self.matrix_D()
        w = sp.csr_matrix(self.lv.volume.reshape(-1, 1))
        nK = self.lv.n_cells
        Kmat = sp.bmat([[A, -D.T, None], [-D, None, w], [None, w.T, None]], format="csc")
        rhs = np.concatenate([self.rhs(f_qp), np.zeros(nK + 1)])
        sol = spla.spsolve(Kmat, rhs)
        return sol[:self.n_dof], sol[self.n_dof:self.n_dof + nK]


def solve_uncondensed(lv, k, nu, beta, f_qp):
    """The scheme (stWeak) on tetrahedra without any elimination, by dense
    LU: unknowns L, RT_k coefficients and full P^k pressure per cell, the
    global normal and tangential face coefficients, multipliers tying each
    cell's normal traces to the face coefficients, and one multiplier for
    the mean-free pressure.  Tiny meshes only.  Returns (c^n [n_int, m_F],
    c^t [n_int, 2, m_F], per-cell (element, a, pressure coefficients))."""
    mF = m_face(k)
    els = [Element3(lv, K, k, nu, beta) for K in range(lv.n_cells)]
    e0 = els[0]
    na, nP = e0.na, e0.nP
    nK, nI = lv.n_cells, lv.n_int
    oL = 0
    oA = oL + nK * 9 * nP
    oP = oA + nK * na
    oN = oP + nK * nP
    oT = oN + nI * mF
    oMu = oT + nI * 2 * mF
    oTh = oMu + nK * 4 * mF
    N = oTh + 1
    A = np.zeros((N, N))
    b = np.zeros(N)
    for K, e in enumerate(els):
        Lb = oL + K * 9 * nP
        Ab = oA + K * na
        Pb = oP + K * nP
        Mub = oMu + K * 4 * mF
        zcol = list(range(Ab, Ab + na))
        for f in range(4):
            fi = lv.int_id[lv.cell_facets[K, f]]
            for c in range(2):
                for j in range(mF):
                    zcol.append(-1 if fi < 0 else oT + (fi * 2 + c) * mF + j)
        zcol = np.array(zcol)
        psi_full = e.P.eval(e.xq)[0]
        _, _, divPhi = e.rt.eval(e.xq)
        Dfull = psi_full.T @ (e.wq[:, None] * divPhi)
        for i in range(3):
            for j in range(3):
                rr = Lb + (i * 3 + j) * nP + np.arange(nP)
                A[np.ix_(rr, rr)] += e.M / e.nu
                for c in range(e.nz):
                    if zcol[c] >= 0:
                        A[rr, zcol[c]] += e.R[i, j][:, c]
                        A[zcol[c], rr] -= e.R[i, j][:, c]
        massRT = np.einsum("q,qai,qbi->ab", e.wq, e.Phi_q, e.Phi_q)
        A[Ab:Ab + na, Ab:Ab + na] += beta * massRT
        A[Ab:Ab + na, Pb:Pb + nP] -= Dfull.T
        A[Ab:Ab + na, Mub:Mub + 4 * mF] -= e.T.T
        b[Ab:Ab + na] += e.load_z(f_qp[K])[:na]
        A[Pb:Pb + nP, Ab:Ab + na] += Dfull
        A[Pb:Pb + nP, oTh] += e.wq @ psi_full
        A[oTh, Pb:Pb + nP] += e.wq @ psi_full
        A[Mub:Mub + 4 * mF, Ab:Ab + na] += e.T
        for f in range(4):
            fi = lv.int_id[lv.cell_facets[K, f]]
            if fi >= 0:
                for j in range(mF):
                    A[Mub + f * mF + j, oN + fi * mF + j] -= 1.0
                    A[oN + fi * mF + j, Mub + f * mF + j] -= 1.0
    sol = np.linalg.solve(A, b)
    cn = sol[oN:oN + nI * mF].reshape(nI, mF)
    ct = sol[oT:oT + nI * 2 * mF].reshape(nI, 2, mF)
    per_cell = []
    for K, e in enumerate(els):
        per_cell.append((e, sol[oA + K * na:oA + (K + 1) * na], sol[oP + K * nP:oP + (K + 1) * nP]))
    return cn, ct, per_cell
