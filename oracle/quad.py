"""Quadrature rules (oracle; test infrastructure only).

Data rule on a triangle: Stroud conical product with n points per direction,
Gauss-Legendre in u and Gauss-Jacobi (weight 1-v) in v, mapped by
(u(1-v), v) onto the reference triangle; weights normalised to sum 1; points
ordered with u fastest.  With n = k+2 it is exact to degree 2k+3, enough for
every bilinear form of the order-k scheme, and the source f is given at its
points.  Facet rule: Gauss-Legendre on [0,1], weights summing to 1.
"""
import numpy as np
from scipy.special import roots_legendre, roots_jacobi


def gauss_legendre01(n):
    x, w = roots_legendre(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_jacobi01(n, alpha):
    """Nodes/weights for int_0^1 (1-v)^alpha f(v) dv."""
    x, w = roots_jacobi(n, alpha, 0.0)
    return 0.5 * (x + 1.0), w * 2.0 ** (-alpha - 1.0)


def stroud_triangle(n):
    """Reference points xi [n*n, 2] on {xi1,xi2 >= 0, xi1+xi2 <= 1} and
    weights [n*n] summing to 1 (u fastest)."""
    u, wu = gauss_legendre01(n)
    v, wv = gauss_jacobi01(n, 1.0)
    pts, wts = [], []
    for j in range(n):
        for i in range(n):
            pts.append((u[i] * (1.0 - v[j]), v[j]))
            wts.append(wu[i] * wv[j])
    wts = np.asarray(wts)
    return np.asarray(pts), wts / wts.sum()


def data_points(X_sorted, n):
    """Physical data points of a triangle whose vertices are given sorted by
    global index (rows of X_sorted), and weights summing to 1."""
    xi, w = stroud_triangle(n)
    X0, X1, X2 = X_sorted
    pts = X0[None, :] + xi[:, :1] * (X1 - X0)[None, :] + xi[:, 1:2] * (X2 - X0)[None, :]
    return pts, w


def stroud_tet(n):
    """Reference points xi [n^3, 3] on {xi >= 0, xi1+xi2+xi3 <= 1} and weights
    [n^3] summing to 1: Gauss-Legendre in u, Gauss-Jacobi with weight (1-v) in
    v and (1-w)^2 in w, mapped by (u(1-v)(1-w), v(1-w), w); u fastest, then v.
    Exact to degree 2n-1."""
    u, wu = gauss_legendre01(n)
    v, wv = gauss_jacobi01(n, 1.0)
    w, ww = gauss_jacobi01(n, 2.0)
    pts, wts = [], []
    for c in range(n):
        for b in range(n):
            for a in range(n):
                pts.append((u[a] * (1.0 - v[b]) * (1.0 - w[c]), v[b] * (1.0 - w[c]), w[c]))
                wts.append(wu[a] * wv[b] * ww[c])
    wts = np.asarray(wts)
    return np.asarray(pts), wts / wts.sum()


def tet_data_points(X_sorted, n):
    """Physical data points of a tetrahedron whose vertices are given sorted by
    global index (rows of X_sorted), and weights summing to 1."""
    xi, w = stroud_tet(n)
    X0, X1, X2, X3 = X_sorted
    pts = (X0[None, :] + xi[:, :1] * (X1 - X0)[None, :] + xi[:, 1:2] * (X2 - X0)[None, :]
           + xi[:, 2:3] * (X3 - X0)[None, :])
    return pts, w
