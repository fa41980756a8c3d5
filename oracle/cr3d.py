"""Lowest-order operators on tetrahedra (oracle; test infrastructure only).

Closed-form cell block of A^eps_{0,h} (k0-stOptForm, Sec. 3.4.1, in three
dimensions): with the Crouzeix-Raviart interpolant Pi^CR of (RT0 field,
tangential face constants) (RT0N1_2CR) and the RT0 interpolant Pi^RT
(CR_2RT0),
    nu (grad Pi^CR u, grad Pi^CR v) + beta (Pi^RT Pi^CR u, Pi^RT Pi^CR v)
    + eps^-1 (div Pi^CR u, div Pi^CR v).
On a tetrahedron the CR basis function of face i is 1 - 3 lambda_i, with
gradient |F_i| n_{K,i} / |K| (lambda_i the barycentric coordinate of the
vertex opposite F_i), and Pi^RT Pi^CR u is the RT0 field itself (Lemma 3.2),
whose basis function with unit outward flux through F_i is
(x - x_i) / (3|K|).  Local unknowns: (face i, component c) -> 3 i + c with
c = 0 the normal coefficient u.n_F and c = 1, 2 the tangential coefficients
of uhat in (t1_F, t2_F).
"""
import numpy as np
import scipy.sparse as sp

from . import quad


def rt0_basis(lv, K, X):
    """Values [np, 4, 3] of the RT0 basis with unit outward flux through local
    face i: (x - x_i) / (3|K|), x_i the vertex opposite face i."""
    V = lv.coords[lv.cells[K]]
    X = np.atleast_2d(X)
    return (X[:, None, :] - V[None, :, :]) / (3.0 * lv.volume[K])


def rt0_mass(lv, K):
    """M_ij = int_K psi_i . psi_j (Stroud rule exact to degree 3)."""
    V = lv.coords[lv.cells[K]]
    X, w = quad.tet_data_points(V, 2)
    P = rt0_basis(lv, K, X)
    return lv.volume[K] * np.einsum("q,qia,qja->ij", w, P, P)


def cell_block(lv, K, nu, beta, eps_inv):
    """Closed-form 12 x 12 block of A^eps_{0,h} on one tetrahedron."""
    fs = lv.cell_facets[K]
    sg = lv.sigma[K]
    vol = lv.volume[K]
    Af = lv.area_f[fs]
    nK = sg[:, None] * lv.normal[fs]
    frame = np.stack([lv.normal[fs], lv.t1[fs], lv.t2[fs]], axis=1)   # [4, 3, 3]
    grad = Af[:, None] * nK / vol
    Mrt = rt0_mass(lv, K)
    q = sg * Af
    A = np.zeros((12, 12))
    for i in range(4):
        for a in range(3):
            for j in range(4):
                for b in range(3):
                    A[3 * i + a, 3 * j + b] = nu * (frame[i, a] @ frame[j, b]) * (grad[i] @ grad[j]) * vol
    for i in range(4):
        for j in range(4):
            A[3 * i, 3 * j] += beta * q[i] * q[j] * Mrt[i, j] + eps_inv * q[i] * q[j] / vol
    return A


def assemble(lv, nu_cells, beta, eps_inv):
    """Global A^eps_{0,l} on interior-face unknowns 3 int_id + c."""
    rows, cols, vals = [], [], []
    for K in range(lv.n_cells):
        B = cell_block(lv, K, nu_cells[K], beta, eps_inv)
        g = np.array([3 * lv.int_id[f] + c if lv.int_id[f] >= 0 else -1
                      for f in lv.cell_facets[K] for c in range(3)])
        keep = g >= 0
        gi = g[keep]
        rows.append(np.repeat(gi, len(gi)))
        cols.append(np.tile(gi, len(gi)))
        vals.append(B[np.ix_(keep, keep)].ravel())
    n = 3 * lv.n_int
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def pi_cr(lv, lam0):
    """Pi^CR of a lowest-order skeleton vector: the Cartesian value
    U_F = c^n n_F + c^t1 t1_F + c^t2 t2_F at the centroid of each interior
    face; [n_int, 3]."""
    c = lam0.reshape(-1, 3)
    ints = np.where(lv.interior)[0]
    return c[:, :1] * lv.normal[ints] + c[:, 1:2] * lv.t1[ints] + c[:, 2:3] * lv.t2[ints]
