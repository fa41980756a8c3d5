"""Manufactured 2D solution of the generalized Stokes problem (Sec. 5.1):
u = curl(psi) with psi = g(x) g(y), g(t) = t^2 (1-t)^2, so
u_x = x^2 (x-1)^2 2y(1-y)(2y-1) = -g(x) g'(y), u_y = g'(x) g(y);
p = x(1-x)(1-y) - 1/12;  f = -nu Lap u + beta u + grad p."""
import numpy as np


def g0(t): return t ** 2 * (1 - t) ** 2
def g1(t): return 2 * t - 6 * t ** 2 + 4 * t ** 3
def g2(t): return 2 - 12 * t + 12 * t ** 2
def g3(t): return -12 + 24 * t


def velocity(X):
    x, y = X[..., 0], X[..., 1]
    return np.stack([-g0(x) * g1(y), g1(x) * g0(y)], axis=-1)


def grad_velocity(X):
    """[..., i, j] = d u_i / d x_j."""
    x, y = X[..., 0], X[..., 1]
    G = np.zeros(X.shape[:-1] + (2, 2))
    G[..., 0, 0] = -g1(x) * g1(y)
    G[..., 0, 1] = -g0(x) * g2(y)
    G[..., 1, 0] = g2(x) * g0(y)
    G[..., 1, 1] = g1(x) * g1(y)
    return G


def pressure(X):
    x, y = X[..., 0], X[..., 1]
    return x * (1 - x) * (1 - y) - 1.0 / 12.0


def source(X, nu, beta):
    x, y = X[..., 0], X[..., 1]
    lap_ux = -(g2(x) * g1(y) + g0(x) * g3(y))
    lap_uy = g3(x) * g0(y) + g1(x) * g2(y)
    u = velocity(X)
    gp = np.stack([(1 - 2 * x) * (1 - y), -x * (1 - x)], axis=-1)
    return -nu * np.stack([lap_ux, lap_uy], axis=-1) + beta * u + gp


def ns_source(X, nu):
    """Stationary Navier-Stokes (Sec. 5.1.2): -nu Lap u + (u . grad) u +
    grad p for the same u and p."""
    u = velocity(X)
    conv = np.einsum("...ij,...j->...i", grad_velocity(X), u)
    return source(X, nu, 0.0) + conv


# Cavity-type solution with a tangential boundary velocity on the top side:
# u = curl(psi), psi = g(x) h(y), h(y) = y^2 (1 - y), so u.n = 0 on the whole
# boundary, u = 0 on the left, right and bottom sides and u_x = -g(x) on top.
def h0(t): return t ** 2 - t ** 3
def h1(t): return 2 * t - 3 * t ** 2
def h2(t): return 2 - 6 * t
def h3(t): return -6.0 + 0 * t


def cavity_velocity(X):
    x, y = X[..., 0], X[..., 1]
    return np.stack([g0(x) * h1(y), -g1(x) * h0(y)], axis=-1)


def cavity_grad_velocity(X):
    """[..., i, j] = d u_i / d x_j."""
    x, y = X[..., 0], X[..., 1]
    G = np.zeros(X.shape[:-1] + (2, 2))
    G[..., 0, 0] = g1(x) * h1(y)
    G[..., 0, 1] = g0(x) * h2(y)
    G[..., 1, 0] = -g2(x) * h0(y)
    G[..., 1, 1] = -g1(x) * h1(y)
    return G


def cavity_source(X, nu, beta, wind_scale):
    """-nu Lap u + beta u + (w . grad) u + grad p with w = wind_scale * u
    and the pressure of `pressure`."""
    x, y = X[..., 0], X[..., 1]
    lap = np.stack([g2(x) * h1(y) + g0(x) * h3(y), -(g3(x) * h0(y) + g1(x) * h2(y))], axis=-1)
    u = cavity_velocity(X)
    G = cavity_grad_velocity(X)
    conv = wind_scale * np.einsum("...ij,...j->...i", G, u)
    gp = np.stack([(1 - 2 * x) * (1 - y), -x * (1 - x)], axis=-1)
    return -nu * lap + beta * u + conv + gp


# Manufactured 3D solution of Sec. 5.1: with g(t) = t^2 (1-t)^2,
# u = (g(x) g'(y) g'(z), g(y) g'(x) g'(z), -2 g(z) g'(x) g'(y)) (divergence
# free, zero on the boundary of the unit cube), p = x(1-x)(1-y)(1-z) - 1/24.
def velocity3(X):
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    return np.stack([g0(x) * g1(y) * g1(z), g0(y) * g1(x) * g1(z), -2 * g0(z) * g1(x) * g1(y)], axis=-1)


def grad_velocity3(X):
    """[..., i, j] = d u_i / d x_j."""
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    G = np.zeros(X.shape[:-1] + (3, 3))
    G[..., 0, 0] = g1(x) * g1(y) * g1(z)
    G[..., 0, 1] = g0(x) * g2(y) * g1(z)
    G[..., 0, 2] = g0(x) * g1(y) * g2(z)
    G[..., 1, 0] = g0(y) * g2(x) * g1(z)
    G[..., 1, 1] = g1(y) * g1(x) * g1(z)
    G[..., 1, 2] = g0(y) * g1(x) * g2(z)
    G[..., 2, 0] = -2 * g0(z) * g2(x) * g1(y)
    G[..., 2, 1] = -2 * g0(z) * g1(x) * g2(y)
    G[..., 2, 2] = -2 * g1(z) * g1(x) * g1(y)
    return G


def pressure3(X):
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    return x * (1 - x) * (1 - y) * (1 - z) - 1.0 / 24.0


def source3(X, nu, beta):
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    lap = np.stack([
        g2(x) * g1(y) * g1(z) + g0(x) * g3(y) * g1(z) + g0(x) * g1(y) * g3(z),
        g3(x) * g0(y) * g1(z) + g1(x) * g2(y) * g1(z) + g1(x) * g0(y) * g3(z),
        -2 * (g3(x) * g1(y) * g0(z) + g1(x) * g3(y) * g0(z) + g1(x) * g1(y) * g2(z))], axis=-1)
    gp = np.stack([(1 - 2 * x) * (1 - y) * (1 - z), -x * (1 - x) * (1 - z), -x * (1 - x) * (1 - y)], axis=-1)
    return -nu * lap + beta * velocity3(X) + gp
