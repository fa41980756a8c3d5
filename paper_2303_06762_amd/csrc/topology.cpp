// Host-side mesh hierarchy and skeleton topology.
#include "topology.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <set>
#include <tuple>

namespace hdgmg {

std::string build_level(Level& L) {
  const int nc = L.nc;
  // (v0, v1, cell, local facet) for all cell facets, sorted lexicographically
  std::vector<std::array<int, 4>> rec(3 * (size_t)nc);
  for (int c = 0; c < nc; ++c) {
    for (int i = 0; i < 3; ++i) {
      int a = L.cells[3 * c + (i + 1) % 3], b = L.cells[3 * c + (i + 2) % 3];
      if (a == b) return "cell with a repeated vertex";
      if (a < 0 || b < 0 || a >= L.nv || b >= L.nv) return "vertex index out of range";
      rec[3 * c + i] = {std::min(a, b), std::max(a, b), c, i};
    }
  }
  std::sort(rec.begin(), rec.end());
  L.cell_facets.assign(3 * (size_t)nc, -1);
  L.edges.clear();
  L.facet_cells.clear();
  L.facet_loc.clear();
  for (size_t r = 0; r < rec.size();) {
    size_t s = r;
    while (s < rec.size() && rec[s][0] == rec[r][0] && rec[s][1] == rec[r][1]) ++s;
    if (s - r > 2) return "facet shared by more than two cells";
    int f = (int)(L.edges.size() / 2);
    L.edges.push_back(rec[r][0]);
    L.edges.push_back(rec[r][1]);
    for (size_t t = r; t < r + 2; ++t) {
      if (t < s) {
        L.facet_cells.push_back(rec[t][2]);
        L.facet_loc.push_back(rec[t][3]);
        L.cell_facets[3 * rec[t][2] + rec[t][3]] = f;
      } else {
        L.facet_cells.push_back(-1);
        L.facet_loc.push_back(-1);
      }
    }
    r = s;
  }
  L.nf = (int)(L.edges.size() / 2);
  L.outflow.assign(L.nf, 0);
  for (const auto& pr : L.outflow_in) {
    const int a = std::min(pr.first, pr.second), b = std::max(pr.first, pr.second);
    // facets are sorted by their vertex pair: binary search
    int lo = 0, hi = L.nf - 1, hit = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) / 2;
      const int ea = L.edges[2 * mid], eb = L.edges[2 * mid + 1];
      if (ea == a && eb == b) {
        hit = mid;
        break;
      }
      if (ea < a || (ea == a && eb < b))
        lo = mid + 1;
      else
        hi = mid - 1;
    }
    if (hit < 0 || L.facet_cells[2 * hit + 1] >= 0) return "an outflow pair is not a boundary facet";
    L.outflow[hit] = 1;
  }
  L.int_id.assign(L.nf, -1);
  L.int_facet.clear();
  for (int f = 0; f < L.nf; ++f)
    if (L.facet_cells[2 * f + 1] >= 0 || L.outflow[f]) {
      L.int_id[f] = (int)L.int_facet.size();
      L.int_facet.push_back(f);
    }
  L.nint = (int)L.int_facet.size();
  L.tang.resize(2 * (size_t)L.nf);
  L.norm.resize(2 * (size_t)L.nf);
  L.len.resize(L.nf);
  for (int f = 0; f < L.nf; ++f) {
    const double* p0 = &L.X[2 * L.edges[2 * f]];
    const double* p1 = &L.X[2 * L.edges[2 * f + 1]];
    double dx = p1[0] - p0[0], dy = p1[1] - p0[1];
    double l = std::sqrt(dx * dx + dy * dy);
    if (!(l > 0)) return "zero-length facet";
    L.len[f] = l;
    L.tang[2 * f] = dx / l;
    L.tang[2 * f + 1] = dy / l;
    L.norm[2 * f] = dy / l;
    L.norm[2 * f + 1] = -dx / l;
  }
  L.area.resize(nc);
  L.sigma.resize(3 * (size_t)nc);
  L.cell_dofs.resize(3 * (size_t)nc);
  for (int c = 0; c < nc; ++c) {
    const double* a = &L.X[2 * L.cells[3 * c]];
    const double* b = &L.X[2 * L.cells[3 * c + 1]];
    const double* d = &L.X[2 * L.cells[3 * c + 2]];
    double det = (b[0] - a[0]) * (d[1] - a[1]) - (b[1] - a[1]) * (d[0] - a[0]);
    if (!(std::fabs(det) > 0)) return "zero-area cell";
    L.area[c] = 0.5 * std::fabs(det);
    for (int i = 0; i < 3; ++i) {
      int f = L.cell_facets[3 * c + i];
      const double* vi = &L.X[2 * L.cells[3 * c + i]];
      const double* p0 = &L.X[2 * L.edges[2 * f]];
      const double* p1 = &L.X[2 * L.edges[2 * f + 1]];
      // outward: from the opposite vertex towards the facet midpoint
      double mx = 0.5 * (p0[0] + p1[0]) - vi[0], my = 0.5 * (p0[1] + p1[1]) - vi[1];
      double s = mx * L.norm[2 * f] + my * L.norm[2 * f + 1];
      L.sigma[3 * c + i] = s > 0 ? 1 : -1;
      L.cell_dofs[3 * c + i] = L.int_id[f];
    }
  }
  return "";
}

void refine(const Level& C, Level& F) {
  F.nv = C.nv + C.nf;
  F.nc = 4 * C.nc;
  F.X.resize(2 * (size_t)F.nv);
  for (int v = 0; v < C.nv; ++v) {
    F.X[2 * v] = C.X[2 * v];
    F.X[2 * v + 1] = C.X[2 * v + 1];
  }
  for (int f = 0; f < C.nf; ++f) {
    const double* p0 = &C.X[2 * C.edges[2 * f]];
    const double* p1 = &C.X[2 * C.edges[2 * f + 1]];
    F.X[2 * (C.nv + f)] = 0.5 * (p0[0] + p1[0]);
    F.X[2 * (C.nv + f) + 1] = 0.5 * (p0[1] + p1[1]);
  }
  // both halves of a do-nothing facet are do-nothing facets
  F.outflow_in.clear();
  for (int f = 0; f < C.nf; ++f)
    if (!C.outflow.empty() && C.outflow[f]) {
      F.outflow_in.push_back({C.edges[2 * f], C.nv + f});
      F.outflow_in.push_back({C.edges[2 * f + 1], C.nv + f});
    }
  F.cells.resize(3 * (size_t)F.nc);
  F.parent.resize(F.nc);
  for (int c = 0; c < C.nc; ++c) {
    int a = C.cells[3 * c], b = C.cells[3 * c + 1], d = C.cells[3 * c + 2];
    int m_bc = C.nv + C.cell_facets[3 * c + 0];
    int m_da = C.nv + C.cell_facets[3 * c + 1];
    int m_ab = C.nv + C.cell_facets[3 * c + 2];
    const int ch[4][3] = {{a, m_ab, m_da}, {m_ab, b, m_bc}, {m_da, m_bc, d}, {m_bc, m_da, m_ab}};
    for (int q = 0; q < 4; ++q) {
      for (int i = 0; i < 3; ++i) F.cells[3 * (4 * c + q) + i] = ch[q][i];
      F.parent[4 * c + q] = c;
    }
  }
}

void build_patches(Level& L) {
  const int nv = L.nv, nc = L.nc;
  // vertex colouring: propagate a 3-colouring through the cells breadth-first
  // from cell 0, else greedy in vertex order
  std::vector<int> col(nv, -1);
  std::vector<char> seen(nc, 0);
  std::vector<int> queue;
  queue.reserve(nc);
  if (nc > 0) {
    queue.push_back(0);
    seen[0] = 1;
  }
  for (size_t h = 0; h < queue.size(); ++h) {
    int c = queue[h];
    for (int i = 0; i < 3; ++i) {
      int v = L.cells[3 * c + i];
      if (col[v] >= 0) continue;
      int used = 0;
      for (int j = 0; j < 3; ++j) {
        int u = L.cells[3 * c + j];
        if (col[u] >= 0) used |= 1 << col[u];
      }
      int cc = 0;
      while (used & (1 << cc)) ++cc;
      col[v] = cc;
    }
    for (int i = 0; i < 3; ++i) {
      int f = L.cell_facets[3 * c + i];
      int o = L.facet_cells[2 * f] == c ? L.facet_cells[2 * f + 1] : L.facet_cells[2 * f];
      if (o >= 0 && !seen[o]) {
        seen[o] = 1;
        queue.push_back(o);
      }
    }
  }
  bool ok = true;
  for (int v = 0; v < nv; ++v) ok = ok && col[v] >= 0 && col[v] <= 2;
  for (int f = 0; f < L.nf && ok; ++f) ok = col[L.edges[2 * f]] != col[L.edges[2 * f + 1]];
  if (!ok) {
    std::vector<std::vector<int>> adj(nv);
    for (int f = 0; f < L.nf; ++f) {
      adj[L.edges[2 * f]].push_back(L.edges[2 * f + 1]);
      adj[L.edges[2 * f + 1]].push_back(L.edges[2 * f]);
    }
    std::fill(col.begin(), col.end(), -1);
    for (int v = 0; v < nv; ++v) {
      std::set<int> used;
      for (int u : adj[v])
        if (col[u] >= 0) used.insert(col[u]);
      int cc = 0;
      while (used.count(cc)) ++cc;
      col[v] = cc;
    }
  }
  L.colour = col;
  L.ncol = 0;
  for (int v = 0; v < nv; ++v) L.ncol = std::max(L.ncol, col[v] + 1);
  std::vector<std::vector<int>> vfac(nv), vcell(nv);
  for (int i = 0; i < L.nint; ++i) {
    int f = L.int_facet[i];
    vfac[L.edges[2 * f]].push_back(i);
    vfac[L.edges[2 * f + 1]].push_back(i);
  }
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < 3; ++i) vcell[L.cells[3 * c + i]].push_back(c);
  L.colour_ptr.assign(1, 0);
  L.patch_vertex.clear();
  L.patch_facet_ptr.assign(1, 0);
  L.patch_facets.clear();
  L.patch_cell_ptr.assign(1, 0);
  L.patch_cells.clear();
  L.max_patch_facets = 0;
  for (int cc = 0; cc < L.ncol; ++cc) {
    for (int v = 0; v < nv; ++v) {
      if (col[v] != cc || vfac[v].empty()) continue;
      std::sort(vfac[v].begin(), vfac[v].end());
      std::sort(vcell[v].begin(), vcell[v].end());
      L.patch_vertex.push_back(v);
      for (int i : vfac[v]) L.patch_facets.push_back(i);
      L.patch_facet_ptr.push_back((int)L.patch_facets.size());
      for (int c : vcell[v]) L.patch_cells.push_back(c);
      L.patch_cell_ptr.push_back((int)L.patch_cells.size());
      L.max_patch_facets = std::max(L.max_patch_facets, (int)vfac[v].size());
    }
    L.colour_ptr.push_back((int)L.patch_vertex.size());
  }
}

void build_facet_patches(Level& L) {
  std::vector<int> col(L.nf, -1);
  int ncol = 0;
  for (int f = 0; f < L.nf; ++f) {
    if (L.int_id[f] < 0) continue;
    int used = 0;
    for (int s = 0; s < 2; ++s) {
      const int c = L.facet_cells[2 * f + s];
      if (c < 0) continue;
      for (int i = 0; i < 3; ++i) {
        const int cc = col[L.cell_facets[3 * c + i]];
        if (cc >= 0) used |= 1 << cc;
      }
    }
    int k = 0;
    while (used & (1 << k)) ++k;
    col[f] = k;
    ncol = std::max(ncol, k + 1);
  }
  L.ncol = ncol;
  L.colour_ptr.assign(1, 0);
  L.patch_vertex.clear();
  L.patch_facet_ptr.assign(1, 0);
  L.patch_facets.clear();
  L.patch_cell_ptr.assign(1, 0);
  L.patch_cells.clear();
  L.max_patch_facets = ncol > 0 ? 1 : 0;
  for (int k = 0; k < ncol; ++k) {
    for (int f = 0; f < L.nf; ++f) {
      if (col[f] != k) continue;
      L.patch_vertex.push_back(f);
      L.patch_facets.push_back(L.int_id[f]);
      L.patch_facet_ptr.push_back((int)L.patch_facets.size());
      int a = L.facet_cells[2 * f], b = L.facet_cells[2 * f + 1];
      if (b >= 0 && b < a) std::swap(a, b);
      L.patch_cells.push_back(a);
      if (b >= 0) L.patch_cells.push_back(b);
      L.patch_cell_ptr.push_back((int)L.patch_cells.size());
    }
    L.colour_ptr.push_back((int)L.patch_vertex.size());
  }
}

void build_averaging(const Level& C, const Level& F, Averaging& A) {
  // weights of the coarse CR midpoint vectors U_E = c^n_E n_E + c^t_E t_E
  // at the midpoint of each fine interior facet
  A.row_ptr.assign(1, 0);
  A.col.clear();
  A.val.clear();
  auto other_cell = [&](int E, int T) {
    int a = C.facet_cells[2 * E], b = C.facet_cells[2 * E + 1];
    return a == T ? b : a;
  };
  auto facet_opposite = [&](int T, int v) {
    for (int i = 0; i < 3; ++i)
      if (C.cells[3 * T + i] == v) return C.cell_facets[3 * T + i];
    return -1;
  };
  for (int fi = 0; fi < F.nint; ++fi) {
    int f = F.int_facet[fi];
    int a = F.edges[2 * f], b = F.edges[2 * f + 1];  // a < b
    std::map<int, double> w;                         // coarse facet -> weight
    if (a >= C.nv) {
      // both endpoints are coarse-facet midpoints: inside one coarse cell
      int E1 = a - C.nv, E2 = b - C.nv;
      w[E1] += 0.5;
      w[E2] += 0.5;
    } else {
      // half of coarse facet E: the mean of the two sides' CR fields at the
      // fine midpoint (one side on a do-nothing facet)
      int v = a, E = b - C.nv;
      int w_end = C.edges[2 * E] == v ? C.edges[2 * E + 1] : C.edges[2 * E];
      w[E] += 1.0;
      const int nside = C.facet_cells[2 * E + 1] >= 0 ? 2 : 1;
      for (int s = 0; s < nside; ++s) {
        int T = C.facet_cells[2 * E + s];
        w[facet_opposite(T, w_end)] += 0.5 / nside;
        w[facet_opposite(T, v)] -= 0.5 / nside;
      }
      (void)other_cell;
    }
    for (int comp = 0; comp < 2; ++comp) {
      const double* e = comp == 0 ? &F.norm[2 * f] : &F.tang[2 * f];
      for (auto& kv : w) {
        int E = kv.first;
        int ei = C.int_id[E];
        if (ei < 0 || kv.second == 0.0) continue;
        double wn = kv.second * (C.norm[2 * E] * e[0] + C.norm[2 * E + 1] * e[1]);
        double wt = kv.second * (C.tang[2 * E] * e[0] + C.tang[2 * E + 1] * e[1]);
        A.col.push_back(2 * ei);
        A.val.push_back(wn);
        A.col.push_back(2 * ei + 1);
        A.val.push_back(wt);
      }
      A.row_ptr.push_back((int)A.col.size());
    }
  }
  A.inner_facets.resize(3 * (size_t)C.nc);
  for (int T = 0; T < C.nc; ++T)
    for (int i = 0; i < 3; ++i) A.inner_facets[3 * T + i] = F.int_id[F.cell_facets[3 * (4 * T + 3) + i]];
}

}  // namespace hdgmg
