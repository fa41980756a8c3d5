"""Lowest-order operators (oracle; test infrastructure only).

* Closed-form cell block of A^eps_{0,h} (k0-stOptForm, Sec. 3.4.1): with the
  Crouzeix-Raviart interpolant Pi^CR of (RT0 field, tangential facet
  constants) (RT0N1_2CR) and the RT0 interpolant Pi^RT (CR_2RT0),
    nu (grad Pi^CR u, grad Pi^CR v) + beta (Pi^RT Pi^CR u, Pi^RT Pi^CR v)
    + eps^-1 (div Pi^CR u, div Pi^CR v).
  On a triangle, the CR basis function of facet i is 1 - 2 lambda_i with
  gradient |F_i| n_{K,i} / |K|, and Pi^RT Pi^CR u is the RT0 field itself
  (Lemma 3.2), whose basis function with unit outward flux through F_i is
  (x - x_i) / (2|K|).
* An independent solve of the pressure-robust CR scheme (equivCRstWeak) in
  Cartesian midpoint values, for the equivalence of Theorem 3.1.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import quad


def _frames(lv, K):
    fs = lv.cell_facets[K]
    return fs, lv.normal[fs], lv.tangent[fs], lv.length[fs], lv.sigma[K]


def rt0_basis(lv, K, X):
    """Values [np, 3, 2] of the RT0 basis with unit outward flux through local
    facet i: (x - x_i) / (2|K|), x_i the vertex opposite facet i."""
    V = lv.coords[lv.cells[K]]
    X = np.atleast_2d(X)
    return (X[:, None, :] - V[None, :, :]) / (2.0 * lv.area[K])


def rt0_mass(lv, K):
    """M_ij = int_K psi_i . psi_j, by the edge-midpoint rule (exact for
    quadratics on triangles)."""
    V = lv.coords[lv.cells[K]]
    mids = np.array([(V[1] + V[2]) / 2, (V[2] + V[0]) / 2, (V[0] + V[1]) / 2])
    P = rt0_basis(lv, K, mids)                      # [3 mids, 3, 2]
    return lv.area[K] / 3.0 * np.einsum("pia,pja->ij", P, P)


def cell_block(lv, K, nu, beta, eps_inv):
    """Closed-form 6x6 block on local DOFs (facet i, comp c) -> 2i + c, with
    c = 0 the normal coefficient u.n_F and c = 1 the tangential uhat.t_F."""
    fs, n, t, L, sg = _frames(lv, K)
    area = lv.area[K]
    nK = sg[:, None] * n
    frame = np.stack([n, t], axis=1)                 # [3, 2, 2] frame vectors
    A = np.zeros((6, 6))
    grad = L[:, None] * nK / area                    # grad of CR basis
    Mrt = rt0_mass(lv, K)
    q = sg * L                                       # flux of c^n = 1
    for i in range(3):
        for a in range(2):
            for j in range(3):
                for b in range(2):
                    A[2 * i + a, 2 * j + b] = nu * (frame[i, a] @ frame[j, b]) * \
                        (grad[i] @ grad[j]) * area
    for i in range(3):
        for j in range(3):
            A[2 * i, 2 * j] += beta * q[i] * q[j] * Mrt[i, j] + eps_inv * q[i] * q[j] / area
    return A


def assemble(lv, nu_cells, beta, eps_inv):
    """Global A^eps_{0,l} on interior-facet DOFs 2*int_id + c."""
    rows, cols, vals = [], [], []
    for K in range(lv.n_cells):
        B = cell_block(lv, K, nu_cells[K], beta, eps_inv)
        g = np.array([2 * lv.int_id[f] + c if lv.int_id[f] >= 0 else -1
                      for f in lv.cell_facets[K] for c in range(2)])
        keep = g >= 0
        gi = g[keep]
        rows.append(np.repeat(gi, len(gi)))
        cols.append(np.tile(gi, len(gi)))
        vals.append(B[np.ix_(keep, keep)].ravel())
    n = 2 * lv.n_int
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def pi_cr(lv, lam0):
    """Pi^CR of a lowest-order skeleton vector: Cartesian midpoint value
    U_F = c^n n_F + c^t t_F on each interior facet; [n_int, 2]."""
    c = lam0.reshape(-1, 2)
    ints = np.where(lv.interior)[0]
    return c[:, :1] * lv.normal[ints] + c[:, 1:] * lv.tangent[ints]


def rt0_field_from_skeleton(lv, lam0, K, X):
    """The RT0 part u of (u, uhat) evaluated at points X of cell K."""
    c = lam0.reshape(-1, 2)
    val = np.zeros((len(np.atleast_2d(X)), 2))
    P = rt0_basis(lv, K, X)
    for i, f in enumerate(lv.cell_facets[K]):
        fi = lv.int_id[f]
        if fi >= 0:
            val += lv.sigma[K, i] * lv.length[f] * c[fi, 0] * P[:, i, :]
    return val


def pi_rt_of_cr(lv, U, K, X):
    """Pi^RT of a CR field with midpoint values U [n_int, 2] (zero on the
    boundary), evaluated at points X of cell K: the RT0 field with fluxes
    int_F v . n_K = |F| U_F . n_K."""
    P = rt0_basis(lv, K, X)
    val = np.zeros((len(np.atleast_2d(X)), 2))
    for i, f in enumerate(lv.cell_facets[K]):
        fi = lv.int_id[f]
        if fi >= 0:
            nK = lv.sigma[K, i] * lv.normal[f]
            val += lv.length[f] * (U[fi] @ nK) * P[:, i, :]
    return val


def solve_pressure_robust_cr(lv, nu, beta, f_qp, nq):
    """The modified CR scheme (equivCRstWeak) in Cartesian midpoint unknowns
    and a P0 pressure, solved by sparse LU with a mean-zero multiplier.
    f_qp are source values at the data points of each cell (rule with nq
    points per direction).  Returns (U [n_int, 2], p [n_cells])."""
    nI, nK = lv.n_int, lv.n_cells
    nu_c = np.broadcast_to(np.asarray(nu, float), (nK,))
    NU = 2 * nI
    rows, cols, vals = [], [], []
    rhs = np.zeros(NU + nK + 1)

    def add(r, c, v):
        rows.append(r), cols.append(c), vals.append(v)

    for K in range(nK):
        fs = lv.cell_facets[K]
        area = lv.area[K]
        nK_ = lv.sigma[K][:, None] * lv.normal[fs]
        grad = lv.length[fs][:, None] * nK_ / area
        ids = lv.int_id[fs]
        Mrt = rt0_mass(lv, K)
        vs = np.sort(lv.cells[K])
        xq, w = quad.data_points(lv.coords[vs], nq)
        Pq = rt0_basis(lv, K, xq)
        load = np.einsum("q,qia,qa->i", w * area, Pq, f_qp[K])   # (f, psi_i)
        for i in range(3):
            if ids[i] < 0:
                continue
            for comp in range(2):
                r = 2 * ids[i] + comp
                for j in range(3):
                    if ids[j] < 0:
                        continue
                    # stiffness: nu grad phi_i . grad phi_j |K| per component
                    add(r, 2 * ids[j] + comp, nu_c[K] * (grad[i] @ grad[j]) * area)
                    # mass of Pi^RT: flux of component comp of facet j's value
                    for cj in range(2):
                        add(r, 2 * ids[j] + cj,
                            beta * lv.length[fs[i]] * nK_[i, comp] *
                            lv.length[fs[j]] * nK_[j, cj] * Mrt[i, j])
                # -(p, div v): div of CR field = sum_i |F_i| U_i . n_i / |K|
                add(r, NU + K, -lv.length[fs[i]] * nK_[i, comp])
                add(NU + K, r, -lv.length[fs[i]] * nK_[i, comp])
                rhs[r] += lv.length[fs[i]] * nK_[i, comp] * load[i]
        add(NU + K, NU + nK, area)
        add(NU + nK, NU + K, area)
    Kmat = sp.csc_matrix((vals, (rows, cols)), shape=(NU + nK + 1,) * 2)
    sol = spla.spsolve(Kmat, rhs)
    return sol[:NU].reshape(nI, 2), sol[NU:NU + nK]
