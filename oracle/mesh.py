"""Nested triangulations and skeleton topology (oracle; test infrastructure).

Conventions (Sec. 2 and Sec. 3.4.2 of the paper; the numbering is ours):
* Local facet i of a cell is the edge opposite its i-th stored vertex.
* A facet is the sorted vertex pair (v0 < v1); facets are numbered in
  lexicographic order of that pair.  Facet frame: t_F = (x_v1 - x_v0)/|.|,
  n_F = (t_y, -t_x); a facet point has parameter s in [0,1] from v0 to v1.
  sigma_{K,F} = n_{K,F} . n_F = +-1 with n_{K,F} the outward normal.
* Interior facets (two adjacent cells) and do-nothing (outflow) boundary
  facets carry the skeleton unknowns and are numbered together in facet
  order ("dof facets", int_id); the other boundary facets carry Dirichlet
  data (homogeneous unless given).  outflow: the coarsest mesh's do-nothing
  facets as vertex pairs; on refinement both halves of such a facet are
  do-nothing facets.
* Red refinement: the midpoint of coarse facet e becomes vertex nv + e; cell
  c = (a, b, c) has children 4c+0 = (a, m_ab, m_ca), 4c+1 = (m_ab, b, m_bc),
  4c+2 = (m_ca, m_bc, c), 4c+3 = (m_bc, m_ca, m_ab).
"""
import numpy as np


class Level:
    """One triangulation with its skeleton."""

    def __init__(self, coords, cells, outflow=None):
        self.coords = np.asarray(coords, dtype=np.float64)
        self.cells = np.asarray(cells, dtype=np.int64)
        nc = len(self.cells)
        self.n_cells = nc
        pairs = np.zeros((nc, 3, 2), dtype=np.int64)
        for i in range(3):
            a = self.cells[:, (i + 1) % 3]
            b = self.cells[:, (i + 2) % 3]
            pairs[:, i, 0] = np.minimum(a, b)
            pairs[:, i, 1] = np.maximum(a, b)
        edges, inv = np.unique(pairs.reshape(-1, 2), axis=0, return_inverse=True)
        self.edges = edges
        self.cell_facets = inv.reshape(nc, 3)
        ne = len(edges)
        self.n_facets = ne
        cnt = np.bincount(self.cell_facets.ravel(), minlength=ne)
        assert cnt.max() <= 2, "non-conforming mesh"
        self.facet_cells = -np.ones((ne, 2), dtype=np.int64)
        self.facet_local = -np.ones((ne, 2), dtype=np.int64)
        fill = np.zeros(ne, dtype=np.int64)
        for K in range(nc):
            for i in range(3):
                e = self.cell_facets[K, i]
                self.facet_cells[e, fill[e]] = K
                self.facet_local[e, fill[e]] = i
                fill[e] += 1
        self.interior = cnt == 2
        self.outflow = np.zeros(ne, dtype=bool)
        if outflow is not None and len(outflow):
            key = {(int(min(a, b)), int(max(a, b))) for a, b in outflow}
            for e in range(ne):
                if cnt[e] == 1 and (int(edges[e, 0]), int(edges[e, 1])) in key:
                    self.outflow[e] = True
            assert self.outflow.sum() == len(key), "outflow pairs must be boundary facets"
        self.dof = self.interior | self.outflow
        self.int_id = -np.ones(ne, dtype=np.int64)
        self.int_id[self.dof] = np.arange(int(self.dof.sum()))
        self.n_int = int(self.dof.sum())
        X0 = self.coords[edges[:, 0]]
        X1 = self.coords[edges[:, 1]]
        d = X1 - X0
        self.length = np.linalg.norm(d, axis=1)
        self.tangent = d / self.length[:, None]
        self.normal = np.stack([self.tangent[:, 1], -self.tangent[:, 0]], axis=1)
        self.midpoint = 0.5 * (X0 + X1)
        V = self.coords[self.cells]                     # [nc,3,2]
        e1 = V[:, 1] - V[:, 0]
        e2 = V[:, 2] - V[:, 0]
        self.area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        self.sigma = np.zeros((nc, 3))
        for i in range(3):
            f = self.cell_facets[:, i]
            out = self.midpoint[f] - V[:, i]            # from opposite vertex
            s = np.sign(np.einsum("kd,kd->k", out, self.normal[f]))
            assert np.all(s != 0)
            self.sigma[:, i] = s
        nv = len(self.coords)
        self.n_vertices = nv

    def vertex_facets(self):
        """For each vertex, the dof facets containing it (sorted)."""
        out = [[] for _ in range(self.n_vertices)]
        for e in range(self.n_facets):
            if self.dof[e]:
                out[self.edges[e, 0]].append(e)
                out[self.edges[e, 1]].append(e)
        return [sorted(x) for x in out]

    def facet_patches(self):
        """Edge (facet) patches of a triangulation: each dof facet alone (the
        unknowns interior to the union of its cells), greedily coloured in
        facet order so that facets of one colour lie in no common cell.
        Returns (patches [list of [facet]], colours [n_patches])."""
        pats, col = [], []
        colour_of = -np.ones(self.n_facets, dtype=np.int64)
        for e in range(self.n_facets):
            if not self.dof[e]:
                continue
            used = set()
            for K in self.facet_cells[e]:
                if K < 0:
                    continue
                for e2 in self.cell_facets[K]:
                    if colour_of[e2] >= 0:
                        used.add(int(colour_of[e2]))
            c = 0
            while c in used:
                c += 1
            colour_of[e] = c
            pats.append([e])
            col.append(c)
        return pats, np.array(col)

    def cell_neighbours(self):
        """nbr[K][i] = cell across local facet i of K, or -1 on the boundary."""
        nbr = -np.ones((self.n_cells, 3), dtype=np.int64)
        for K in range(self.n_cells):
            for i in range(3):
                e = self.cell_facets[K, i]
                a, b = self.facet_cells[e]
                nbr[K, i] = b if a == K else a
        return nbr

    def vertex_colours(self):
        """Canonical vertex colouring used to order the patch sweeps.

        Propagation: the stored vertices of cell 0 get colours 0,1,2; cells are
        visited breadth-first from cell 0 (neighbours across local facets
        0,1,2 in that order) and each uncoloured vertex of a visited cell takes
        the smallest colour in {0,1,2} unused by that cell's coloured vertices.
        If the result is not a proper colouring of the vertex graph (or misses
        a vertex), fall back to greedy colouring in vertex-index order
        (smallest colour unused by already coloured neighbours)."""
        col = -np.ones(self.n_vertices, dtype=np.int64)
        nbr = self.cell_neighbours()
        seen = np.zeros(self.n_cells, dtype=bool)
        queue = [0]
        seen[0] = True
        head = 0
        while head < len(queue):
            K = queue[head]
            head += 1
            vs = self.cells[K]
            for v in vs:
                if col[v] < 0:
                    used = {col[u] for u in vs if col[u] >= 0}
                    c = 0
                    while c in used:
                        c += 1
                    col[v] = c
            for i in range(3):
                J = nbr[K, i]
                if J >= 0 and not seen[J]:
                    seen[J] = True
                    queue.append(J)
        ok = np.all(col >= 0) and np.all(col <= 2) and \
            np.all(col[self.edges[:, 0]] != col[self.edges[:, 1]])
        if ok:
            return col
        adj = [set() for _ in range(self.n_vertices)]
        for a, b in self.edges:
            adj[a].add(b)
            adj[b].add(a)
        col = -np.ones(self.n_vertices, dtype=np.int64)
        for v in range(self.n_vertices):
            used = {col[u] for u in adj[v] if col[u] >= 0}
            c = 0
            while c in used:
                c += 1
            col[v] = c
        return col


def refine(coords, cells):
    """Red refinement with the canonical numbering above.  Returns
    (coords, cells, parent)."""
    lvl = Level(coords, cells)
    nv = len(lvl.coords)
    new = np.concatenate([lvl.coords, lvl.midpoint], axis=0)
    out = np.zeros((4 * lvl.n_cells, 3), dtype=np.int64)
    for c in range(lvl.n_cells):
        a, b, cc = lvl.cells[c]
        # facet opposite local vertex i: mid of the other two
        m_bc = nv + lvl.cell_facets[c, 0]
        m_ca = nv + lvl.cell_facets[c, 1]
        m_ab = nv + lvl.cell_facets[c, 2]
        out[4 * c + 0] = (a, m_ab, m_ca)
        out[4 * c + 1] = (m_ab, b, m_bc)
        out[4 * c + 2] = (m_ca, m_bc, cc)
        out[4 * c + 3] = (m_bc, m_ca, m_ab)
    parent = np.repeat(np.arange(lvl.n_cells), 4)
    return new, out, parent


def refine_pairs(lvl, pairs):
    """Both halves of each facet (a, b) of lvl after red refinement."""
    out = []
    nv = len(lvl.coords)
    for a, b in pairs:
        a, b = int(min(a, b)), int(max(a, b))
        e = int(np.where((lvl.edges[:, 0] == a) & (lvl.edges[:, 1] == b))[0][0])
        out += [(a, nv + e), (b, nv + e)]
    return out


def hierarchy(coords, cells, n_refine, outflow=None):
    """Levels T_1 (coarsest) .. T_J, J = n_refine + 1, with parent maps;
    outflow: do-nothing facets of the coarsest mesh (vertex pairs)."""
    levels = [Level(coords, cells, outflow)]
    parents = [None]
    c, t = np.asarray(coords, float), np.asarray(cells)
    pairs = list(outflow) if outflow is not None else []
    for _ in range(n_refine):
        pairs = refine_pairs(levels[-1], pairs)
        c, t, p = refine(c, t)
        levels.append(Level(c, t, pairs))
        parents.append(p)
    for l, p in zip(levels, parents):
        l.parent = p
    return levels
