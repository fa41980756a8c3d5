"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method: only a counter-based random
number generator, the coarse structured triangulation handed to the solver
as its input mesh, and the seeded data arrays built from the generator.

Random numbers (counter mode splitmix64, Steele, Lea & Flood 2014):
  key = seed*16 + stream;  x = (key << 32) + i;
  out = splitmix64-finaliser(x + 0x9E3779B97F4A7C15);
  uniform[0,1) = (out >> 11) * 2^-53;   uniform[-1,1) = 2u - 1.
Data arrays are indexed C-order [nrhs][n_cells][n_qp][dim], and element i of
that flat array takes counter i.
"""
import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLD = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, stream, idx):
    """Counter-mode splitmix64 outputs (uint64) for counters ``idx``."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = np.uint64(seed) * np.uint64(16) + np.uint64(stream)
    with np.errstate(over="ignore"):
        z = (key << np.uint64(32)) + idx + _GOLD
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, stream, n):
    """n uniforms in [0,1) from counters 0..n-1."""
    z = splitmix64(seed, stream, np.arange(n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed, stream, shape):
    """Uniforms in [-1,1) filling ``shape`` in C order."""
    n = int(np.prod(shape))
    return (2.0 * uniform01(seed, stream, n) - 1.0).reshape(shape)


def normal(seed, stream, n):
    """Standard normals by Box-Muller on (1-u1, u2); u1, u2 from streams
    ``stream`` and ``stream+1``."""
    u1 = 1.0 - uniform01(seed, stream, n)
    u2 = uniform01(seed, stream + 1, n)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def kuhn_square(n):
    """Structured triangulation of [0,1]^2 with n x n squares, each split along
    its (i,j)-(i+1,j+1) diagonal.

    Vertex (i,j) has index i + (n+1) j.  Square (i,j) (index i + n j) yields two
    triangles, in this order: (v_ij, v_i+1,j, v_i+1,j+1) then
    (v_ij, v_i,j+1, v_i+1,j+1).  Returns (coords [nv,2] float64,
    cells [nc,3] int32).
    """
    xs = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    cells = []
    for j in range(n):
        for i in range(n):
            v = lambda a, b: a + (n + 1) * b
            cells.append((v(i, j), v(i + 1, j), v(i + 1, j + 1)))
            cells.append((v(i, j), v(i, j + 1), v(i + 1, j + 1)))
    return coords, np.asarray(cells, dtype=np.int32)


def kuhn_cube(n):
    """Structured tetrahedral mesh of [0,1]^3 with n^3 cubes, each split into
    the six tetrahedra of its Kuhn (Freudenthal) subdivision.

    Vertex (i,j,l) has index i + (n+1) j + (n+1)^2 l.  Cube (i,j,l) (index
    i + n j + n^2 l) yields one tetrahedron per permutation (a,b,c) of the
    axes (0,1,2), in lexicographic order of the permutation: the vertex path
    base, base + e_a, base + e_a + e_b, base + (1,1,1).  Returns (coords
    [nv,3] float64, cells [nc,4] int32)."""
    xs = np.linspace(0.0, 1.0, n + 1)
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    cells = []
    for l in range(n):
        for j in range(n):
            for i in range(n):
                for p in perms:
                    pos = [i, j, l]
                    path = [tuple(pos)]
                    for ax in p:
                        pos[ax] += 1
                        path.append(tuple(pos))
                    cells.append([a + (n + 1) * b + (n + 1) ** 2 * c for a, b, c in path])
    return coords, np.asarray(cells, dtype=np.int32)


def lid_velocity(ends, top=1.0):
    """Boundary data of the lid-driven cavity: one constant velocity per
    boundary facet, (1, 0) on the facets whose two end points lie on the side
    y = top, zero elsewhere.  ends: array [n_boundary_facets][2][2]."""
    ends = np.asarray(ends)
    on = (np.abs(ends[:, 0, 1] - top) < 1e-12) & (np.abs(ends[:, 1, 1] - top) < 1e-12)
    g = np.zeros((ends.shape[0], 2))
    g[on, 0] = 1.0
    return g


def step_domain(n=1, length=4.0, step=True):
    """The backward-facing step ([0.5, L] x [0, 0.5]) u ([0, L] x [0.5, 1])
    of the paper's Sec. 5.3 (L = 4) from squares of side 0.5/n, each split
    along its (i,j)-(i+1,j+1) diagonal as in kuhn_square; vertices are the
    used grid points (i, j) in (j, i) lexicographic order.  step=False: the
    channel [0, L] x [0.5, 1] alone.  Returns (coords, cells, outflow):
    outflow lists the vertex pairs of the facets on x = L (the do-nothing
    boundary)."""
    h = 0.5 / n
    ni, nj = int(round(length / h)), 2 * n
    sq = [(i, j) for j in range(nj) for i in range(ni) if not ((i < n or not step) and j < n)]
    used = set()
    for i, j in sq:
        used |= {(i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1)}
    order = sorted(used, key=lambda v: (v[1], v[0]))
    idx = {v: a for a, v in enumerate(order)}
    coords = np.array([(i * h, j * h) for i, j in order], dtype=np.float64)
    cells = []
    for i, j in sq:
        cells.append((idx[i, j], idx[i + 1, j], idx[i + 1, j + 1]))
        cells.append((idx[i, j], idx[i, j + 1], idx[i + 1, j + 1]))
    outflow = [(idx[ni, j], idx[ni, j + 1]) for j in range(0 if step else n, nj)]
    return coords, np.asarray(cells, dtype=np.int32), outflow


def boundary_coefficients(ends, k, velocity):
    """Normal and tangential coefficients [n_facets][2][k+1] of a boundary
    velocity field: the facet L^2 projection of velocity(X) . n_F and
    . t_F onto the modes phi_j(s) = sqrt(2j+1) P_j(2s-1), s from the first
    end point to the second, t_F = (second - first)/|.|, n_F = (t_y, -t_x).
    velocity maps points [..., 2] to vectors [..., 2]; ends [nb][2][2]."""
    ends = np.asarray(ends, dtype=np.float64)
    xg, wg = np.polynomial.legendre.leggauss(k + 4)
    s, w = 0.5 * (xg + 1.0), 0.5 * wg
    phi = np.stack([np.sqrt(2 * j + 1) * np.polynomial.legendre.legval(2 * s - 1, np.eye(k + 1)[j])
                    for j in range(k + 1)])
    out = np.zeros((ends.shape[0], 2, k + 1))
    for i, (a, b) in enumerate(ends):
        t = (b - a) / np.hypot(*(b - a))
        nrm = np.array([t[1], -t[0]])
        X = a[None, :] + s[:, None] * (b - a)[None, :]
        u = velocity(X)
        out[i, 0] = phi @ (w * (u @ nrm))
        out[i, 1] = phi @ (w * (u @ t))
    return out


def step_inflow(X, x0=0.0):
    """The paper's inflow (16 (1 - y)(y - 0.5), 0) on x = x0 (zero elsewhere)."""
    X = np.asarray(X)
    on = np.abs(X[..., 0] - x0) < 1e-12
    u = np.zeros(X.shape)
    u[..., 0] = np.where(on, 16.0 * (1.0 - X[..., 1]) * (X[..., 1] - 0.5), 0.0)
    return u


def lid_coefficients(ends, k, profile, top=1.0):
    """Tangential boundary coefficients [n_boundary_facets][k+1] of the lid
    velocity (profile(x), 0) on the facets of the side y = top (zero
    elsewhere): the facet L^2 projection onto the modes
    phi_j(s) = sqrt(2j+1) P_j(2s-1), s running from the facet's first end
    point to its second (the tangent's direction); ends: [nb][2][2].  The
    lid of the paper's cavity is profile(x) = 4x(1-x)."""
    ends = np.asarray(ends, dtype=np.float64)
    out = np.zeros((ends.shape[0], k + 1))
    xg, wg = np.polynomial.legendre.leggauss(k + 4)
    s, w = 0.5 * (xg + 1.0), 0.5 * wg
    phi = np.stack([np.sqrt(2 * j + 1) * np.polynomial.legendre.legval(2 * s - 1, np.eye(k + 1)[j])
                    for j in range(k + 1)])
    for i, (a, b) in enumerate(ends):
        if abs(a[1] - top) >= 1e-12 or abs(b[1] - top) >= 1e-12:
            continue
        tx = (b[0] - a[0]) / np.hypot(*(b - a))
        x = a[0] + s * (b[0] - a[0])
        out[i] = phi @ (w * profile(x) * tx)
    return out


def source_uniform(seed, nrhs, n_cells, n_qp, dim=2, stream=0):
    """f at the data quadrature points, i.i.d. uniform[-1,1):
    array [nrhs][n_cells][n_qp][dim]."""
    return uniform_pm1(seed, stream, (nrhs, n_cells, n_qp, dim))


def trig_coefficients(seed, n_modes=4, stream=0):
    """Coefficients of phi(x) = sum_{m in {0..n-1}^2, m != 0}
    a_m cos(pi m.x + theta_m): a_m ~ U[-1,1), theta_m ~ U[0, 2pi).
    Returns (modes [M,2], a [M], theta [M])."""
    modes = np.array([(i, j) for j in range(n_modes) for i in range(n_modes)
                      if (i, j) != (0, 0)], dtype=np.float64)
    a = uniform_pm1(seed, stream, (len(modes),))
    theta = 2.0 * np.pi * uniform01(seed, stream + 1, len(modes))
    return modes, a, theta


def trig_gradient(X, seed, n_modes=4, stream=0):
    """Gradient at points X [..., 2] of the seeded trigonometric polynomial
    phi(x) = sum_m a_m cos(pi m.x + theta_m) of trig_coefficients."""
    modes, a, th = trig_coefficients(seed, n_modes, stream)
    arg = np.pi * np.tensordot(X, modes.T, axes=([-1], [0])) + th
    s = -np.sin(arg) * a
    return np.pi * np.tensordot(s, modes, axes=([-1], [0]))
