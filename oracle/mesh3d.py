"""Nested tetrahedral meshes and their skeleton (oracle; test infrastructure).

Conventions (Sec. 2 and Sec. 3.4.2 of the paper in three dimensions; the
numbering is ours):
* Local face i of a cell is the face opposite its i-th stored vertex.
* A face is the sorted vertex triple (v0 < v1 < v2); faces are numbered in
  lexicographic order of that triple.  Face frame:
  n_F = (x1 - x0) x (x2 - x0) / |.|, t1_F = (x1 - x0) / |.|,
  t2_F = n_F x t1_F.  A face point has reference coordinates (xi, eta) with
  x = x0 + xi (x1 - x0) + eta (x2 - x0).  sigma_{K,F} = n_{K,F} . n_F = +-1
  with n_{K,F} the outward normal.
* Interior faces (two adjacent cells) are numbered in face order; boundary
  faces carry no unknowns (homogeneous Dirichlet data).
* Edges are sorted vertex pairs numbered lexicographically.
* Refinement (Bey's red refinement): the midpoint of coarse edge e becomes
  vertex nv + e; cell c = (x0, x1, x2, x3) has the children
    8c+0 (x0, x01, x02, x03)   8c+1 (x01, x1, x12, x13)
    8c+2 (x02, x12, x2, x23)   8c+3 (x03, x13, x23, x3)
    8c+4 (x01, x02, x03, x13)  8c+5 (x01, x02, x12, x13)
    8c+6 (x02, x03, x13, x23)  8c+7 (x02, x12, x13, x23)
  with xab the midpoint of the edge (xa, xb).  On a Kuhn mesh (vertices in
  path order) the children are the Kuhn tetrahedra of the mesh of half the
  width, so the levels are nested Kuhn meshes.
"""
import numpy as np

# local face i is opposite stored vertex i: its other three stored vertices
FACE_VERTS = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))
EDGE_VERTS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


class Level3:
    """One tetrahedral mesh with its skeleton."""

    def __init__(self, coords, cells):
        self.dim = 3
        self.coords = np.asarray(coords, dtype=np.float64)
        self.cells = np.asarray(cells, dtype=np.int64)
        nc = len(self.cells)
        self.n_cells = nc
        self.n_vertices = len(self.coords)
        tri = np.zeros((nc, 4, 3), dtype=np.int64)
        for i, fv in enumerate(FACE_VERTS):
            tri[:, i, :] = np.sort(self.cells[:, fv], axis=1)
        faces, inv = np.unique(tri.reshape(-1, 3), axis=0, return_inverse=True)
        self.faces = faces
        self.cell_facets = inv.reshape(nc, 4)
        nf = len(faces)
        self.n_facets = nf
        cnt = np.bincount(self.cell_facets.ravel(), minlength=nf)
        assert cnt.max() <= 2, "non-conforming mesh"
        self.facet_cells = -np.ones((nf, 2), dtype=np.int64)
        self.facet_local = -np.ones((nf, 2), dtype=np.int64)
        fill = np.zeros(nf, dtype=np.int64)
        for K in range(nc):
            for i in range(4):
                f = self.cell_facets[K, i]
                self.facet_cells[f, fill[f]] = K
                self.facet_local[f, fill[f]] = i
                fill[f] += 1
        self.interior = cnt == 2
        self.int_id = -np.ones(nf, dtype=np.int64)
        self.int_id[self.interior] = np.arange(int(self.interior.sum()))
        self.n_int = int(self.interior.sum())
        X0 = self.coords[faces[:, 0]]
        X1 = self.coords[faces[:, 1]]
        X2 = self.coords[faces[:, 2]]
        cr = np.cross(X1 - X0, X2 - X0)
        self.area_f = 0.5 * np.linalg.norm(cr, axis=1)
        self.normal = cr / np.linalg.norm(cr, axis=1)[:, None]
        self.t1 = (X1 - X0) / np.linalg.norm(X1 - X0, axis=1)[:, None]
        self.t2 = np.cross(self.normal, self.t1)
        self.centroid = (X0 + X1 + X2) / 3.0
        V = self.coords[self.cells]
        self.volume = np.abs(np.einsum("ki,ki->k", np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]),
                                       V[:, 3] - V[:, 0])) / 6.0
        assert np.all(self.volume > 0), "degenerate cell"
        self.sigma = np.zeros((nc, 4))
        for i in range(4):
            f = self.cell_facets[:, i]
            out = self.centroid[f] - V[:, i]            # from the opposite vertex
            s = np.sign(np.einsum("kd,kd->k", out, self.normal[f]))
            assert np.all(s != 0)
            self.sigma[:, i] = s
        pairs = np.zeros((nc, 6, 2), dtype=np.int64)
        for e, (a, b) in enumerate(EDGE_VERTS):
            pairs[:, e, :] = np.sort(self.cells[:, [a, b]], axis=1)
        self.edges, einv = np.unique(pairs.reshape(-1, 2), axis=0, return_inverse=True)
        self.cell_edges = einv.reshape(nc, 6)
        self.n_edges = len(self.edges)

    def edge_patches(self):
        """For each edge, the interior faces containing it (sorted face ids)."""
        fe = {}
        for e, (a, b) in enumerate(self.edges):
            fe[(int(a), int(b))] = e
        out = [[] for _ in range(self.n_edges)]
        for F in np.where(self.interior)[0]:
            v = self.faces[F]
            for a, b in ((v[0], v[1]), (v[0], v[2]), (v[1], v[2])):
                out[fe[(int(a), int(b))]].append(int(F))
        return [sorted(x) for x in out]

    def edge_colours(self, patches):
        """Greedy colouring of the edges with a non-empty patch, in edge
        order: each takes the smallest colour not used by an earlier such
        edge sharing a cell with it (edges of one colour then lie in no
        common cell, so their patches are uncoupled).  Edges with an empty
        patch get -1."""
        cells_of = [[] for _ in range(self.n_edges)]
        for K in range(self.n_cells):
            for e in self.cell_edges[K]:
                cells_of[e].append(K)
        col = -np.ones(self.n_edges, dtype=np.int64)
        for e in range(self.n_edges):
            if not patches[e]:
                continue
            used = set()
            for K in cells_of[e]:
                for e2 in self.cell_edges[K]:
                    if col[e2] >= 0:
                        used.add(int(col[e2]))
            c = 0
            while c in used:
                c += 1
            col[e] = c
        return col


    def vertex_patches(self):
        """For each vertex, the interior faces containing it (sorted face ids)."""
        out = [[] for _ in range(len(self.coords))]
        for F in np.where(self.interior)[0]:
            for v in self.faces[F]:
                out[int(v)].append(int(F))
        return [sorted(x) for x in out]

    def vertex_colours(self, patches):
        """Greedy colouring of the vertices with a non-empty patch, in vertex
        order: each takes the smallest colour not used by an earlier such
        vertex sharing a cell with it.  Vertices with an empty patch get -1."""
        nv = len(self.coords)
        cells_of = [[] for _ in range(nv)]
        for K in range(self.n_cells):
            for v in self.cells[K]:
                cells_of[int(v)].append(K)
        col = -np.ones(nv, dtype=np.int64)
        for v in range(nv):
            if not patches[v]:
                continue
            used = {int(col[w]) for K in cells_of[v] for w in self.cells[K] if col[w] >= 0}
            c = 0
            while c in used:
                c += 1
            col[v] = c
        return col


def refine(coords, cells):
    """Bey's red refinement with the numbering above: (coords, cells, parent)."""
    lvl = Level3(coords, cells)
    nv = len(lvl.coords)
    mids = 0.5 * (lvl.coords[lvl.edges[:, 0]] + lvl.coords[lvl.edges[:, 1]])
    new = np.concatenate([lvl.coords, mids], axis=0)
    emap = {(int(a), int(b)): e for e, (a, b) in enumerate(lvl.edges)}
    out = np.zeros((8 * lvl.n_cells, 4), dtype=np.int64)
    for c in range(lvl.n_cells):
        x = [int(v) for v in lvl.cells[c]]

        def m(a, b):
            return nv + emap[(min(x[a], x[b]), max(x[a], x[b]))]

        out[8 * c + 0] = (x[0], m(0, 1), m(0, 2), m(0, 3))
        out[8 * c + 1] = (m(0, 1), x[1], m(1, 2), m(1, 3))
        out[8 * c + 2] = (m(0, 2), m(1, 2), x[2], m(2, 3))
        out[8 * c + 3] = (m(0, 3), m(1, 3), m(2, 3), x[3])
        out[8 * c + 4] = (m(0, 1), m(0, 2), m(0, 3), m(1, 3))
        out[8 * c + 5] = (m(0, 1), m(0, 2), m(1, 2), m(1, 3))
        out[8 * c + 6] = (m(0, 2), m(0, 3), m(1, 3), m(2, 3))
        out[8 * c + 7] = (m(0, 2), m(1, 2), m(1, 3), m(2, 3))
    parent = np.repeat(np.arange(lvl.n_cells), 8)
    return new, out, parent


def hierarchy(coords, cells, n_refine):
    """Levels T_1 (coarsest) .. T_J, J = n_refine + 1, with parent maps."""
    levels = [Level3(coords, cells)]
    parents = [None]
    c, t = np.asarray(coords, float), np.asarray(cells)
    for _ in range(n_refine):
        c, t, p = refine(c, t)
        levels.append(Level3(c, t))
        parents.append(p)
    for l, p in zip(levels, parents):
        l.parent = p
    return levels
