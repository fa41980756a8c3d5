// Host-side tetrahedral topology (see mesh3d.hpp).
#include "mesh3d.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

namespace hdgmg {

namespace {
constexpr int FACE_V[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
constexpr int EDGE_V[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

inline void sub3(const double* a, const double* b, double* c) {
  for (int i = 0; i < 3; ++i) c[i] = a[i] - b[i];
}
inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

int find_edge(const std::vector<int>& edges, int a, int b) {
  // edges sorted lexicographically as pairs
  int lo = 0, hi = (int)edges.size() / 2;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    int ea = edges[2 * mid], eb = edges[2 * mid + 1];
    if (ea < a || (ea == a && eb < b))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
}  // namespace

std::string build_level3(Level3& L) {
  const int nc = L.nc;
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < 4; ++i) {
      int v = L.cells[4 * c + i];
      if (v < 0 || v >= L.nv) return "cell vertex index out of range";
    }
  // faces: sorted triples, unique, lexicographic
  std::vector<std::array<int, 4>> tri((size_t)nc * 4);  // (v0, v1, v2, cell*4+i)
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < 4; ++i) {
      int v[3] = {L.cells[4 * c + FACE_V[i][0]], L.cells[4 * c + FACE_V[i][1]], L.cells[4 * c + FACE_V[i][2]]};
      std::sort(v, v + 3);
      if (v[0] == v[1] || v[1] == v[2]) return "repeated vertex in a cell";
      tri[(size_t)4 * c + i] = {v[0], v[1], v[2], 4 * c + i};
    }
  std::sort(tri.begin(), tri.end());
  L.faces.clear();
  L.cell_faces.assign((size_t)nc * 4, -1);
  for (size_t t = 0; t < tri.size(); ++t) {
    if (t == 0 || tri[t][0] != tri[t - 1][0] || tri[t][1] != tri[t - 1][1] || tri[t][2] != tri[t - 1][2]) {
      L.faces.push_back(tri[t][0]);
      L.faces.push_back(tri[t][1]);
      L.faces.push_back(tri[t][2]);
    }
    L.cell_faces[tri[t][3]] = (int)L.faces.size() / 3 - 1;
  }
  L.nf = (int)L.faces.size() / 3;
  L.face_cells.assign((size_t)L.nf * 2, -1);
  L.face_loc.assign((size_t)L.nf * 2, -1);
  std::vector<int> cnt(L.nf, 0);
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < 4; ++i) {
      int f = L.cell_faces[4 * c + i];
      if (cnt[f] >= 2) return "face shared by more than two cells";
      L.face_cells[2 * f + cnt[f]] = c;
      L.face_loc[2 * f + cnt[f]] = i;
      ++cnt[f];
    }
  L.int_id.assign(L.nf, -1);
  L.int_face.clear();
  for (int f = 0; f < L.nf; ++f)
    if (cnt[f] == 2) {
      L.int_id[f] = (int)L.int_face.size();
      L.int_face.push_back(f);
    }
  L.nint = (int)L.int_face.size();
  // face frames
  L.fn.assign((size_t)L.nf * 3, 0.0);
  L.ft1.assign((size_t)L.nf * 3, 0.0);
  L.ft2.assign((size_t)L.nf * 3, 0.0);
  L.farea.assign(L.nf, 0.0);
  for (int f = 0; f < L.nf; ++f) {
    const double* X0 = &L.X[3 * L.faces[3 * f]];
    const double* X1 = &L.X[3 * L.faces[3 * f + 1]];
    const double* X2 = &L.X[3 * L.faces[3 * f + 2]];
    double a[3], b[3], n[3];
    sub3(X1, X0, a);
    sub3(X2, X0, b);
    cross3(a, b, n);
    double nn = std::sqrt(dot3(n, n)), la = std::sqrt(dot3(a, a));
    if (!(nn > 0)) return "degenerate face";
    L.farea[f] = 0.5 * nn;
    for (int d = 0; d < 3; ++d) {
      L.fn[3 * f + d] = n[d] / nn;
      L.ft1[3 * f + d] = a[d] / la;
    }
    cross3(&L.fn[3 * f], &L.ft1[3 * f], &L.ft2[3 * f]);
  }
  // volumes and orientations
  L.vol.assign(nc, 0.0);
  L.sigma.assign((size_t)nc * 4, 0);
  for (int c = 0; c < nc; ++c) {
    const int* v = &L.cells[4 * c];
    double a[3], b[3], d[3], cr[3];
    sub3(&L.X[3 * v[1]], &L.X[3 * v[0]], a);
    sub3(&L.X[3 * v[2]], &L.X[3 * v[0]], b);
    sub3(&L.X[3 * v[3]], &L.X[3 * v[0]], d);
    cross3(a, b, cr);
    L.vol[c] = std::fabs(dot3(cr, d)) / 6.0;
    if (!(L.vol[c] > 0)) return "zero-volume cell";
    for (int i = 0; i < 4; ++i) {
      int f = L.cell_faces[4 * c + i];
      double cen[3] = {0, 0, 0};
      for (int j = 0; j < 3; ++j)
        for (int e = 0; e < 3; ++e) cen[e] += L.X[3 * L.faces[3 * f + j] + e] / 3.0;
      double out[3];
      sub3(cen, &L.X[3 * v[i]], out);
      double s = dot3(out, &L.fn[3 * f]);
      L.sigma[4 * c + i] = s > 0 ? 1 : -1;
    }
  }
  // edges
  std::vector<std::array<int, 3>> pr((size_t)nc * 6);
  for (int c = 0; c < nc; ++c)
    for (int e = 0; e < 6; ++e) {
      int a = L.cells[4 * c + EDGE_V[e][0]], b = L.cells[4 * c + EDGE_V[e][1]];
      pr[(size_t)6 * c + e] = {std::min(a, b), std::max(a, b), 6 * c + e};
    }
  std::sort(pr.begin(), pr.end());
  L.edges.clear();
  L.cell_edges.assign((size_t)nc * 6, -1);
  for (size_t t = 0; t < pr.size(); ++t) {
    if (t == 0 || pr[t][0] != pr[t - 1][0] || pr[t][1] != pr[t - 1][1]) {
      L.edges.push_back(pr[t][0]);
      L.edges.push_back(pr[t][1]);
    }
    L.cell_edges[pr[t][2]] = (int)L.edges.size() / 2 - 1;
  }
  L.ne = (int)L.edges.size() / 2;
  L.cell_dofs.assign((size_t)nc * 4, -1);
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < 4; ++i) L.cell_dofs[4 * c + i] = L.int_id[L.cell_faces[4 * c + i]];
  return "";
}

void refine3(const Level3& C, Level3& F) {
  F.nv = C.nv + C.ne;
  F.X.assign((size_t)F.nv * 3, 0.0);
  std::copy(C.X.begin(), C.X.end(), F.X.begin());
  for (int e = 0; e < C.ne; ++e)
    for (int d = 0; d < 3; ++d)
      F.X[3 * (C.nv + e) + d] = 0.5 * (C.X[3 * C.edges[2 * e] + d] + C.X[3 * C.edges[2 * e + 1] + d]);
  F.nc = 8 * C.nc;
  F.cells.assign((size_t)F.nc * 4, 0);
  F.parent.assign(F.nc, 0);
  for (int c = 0; c < C.nc; ++c) {
    const int* x = &C.cells[4 * c];
    auto m = [&](int a, int b) {
      return C.nv + find_edge(C.edges, std::min(x[a], x[b]), std::max(x[a], x[b]));
    };
    const int ch[8][4] = {{x[0], m(0, 1), m(0, 2), m(0, 3)}, {m(0, 1), x[1], m(1, 2), m(1, 3)},
                          {m(0, 2), m(1, 2), x[2], m(2, 3)}, {m(0, 3), m(1, 3), m(2, 3), x[3]},
                          {m(0, 1), m(0, 2), m(0, 3), m(1, 3)}, {m(0, 1), m(0, 2), m(1, 2), m(1, 3)},
                          {m(0, 2), m(0, 3), m(1, 3), m(2, 3)}, {m(0, 2), m(1, 2), m(1, 3), m(2, 3)}};
    for (int s = 0; s < 8; ++s) {
      for (int i = 0; i < 4; ++i) F.cells[4 * (8 * c + s) + i] = ch[s][i];
      F.parent[8 * c + s] = c;
    }
  }
}

void build_edge_patches(Level3& L) {
  // interior faces of each edge
  std::vector<std::vector<int>> ef(L.ne);
  for (int f = 0; f < L.nf; ++f) {
    if (L.int_id[f] < 0) continue;
    const int* v = &L.faces[3 * f];
    const int pairs[3][2] = {{v[0], v[1]}, {v[0], v[2]}, {v[1], v[2]}};
    for (auto& p : pairs) ef[find_edge(L.edges, p[0], p[1])].push_back(L.int_id[f]);
  }
  std::vector<std::vector<int>> ec(L.ne);
  for (int c = 0; c < L.nc; ++c)
    for (int e = 0; e < 6; ++e) ec[L.cell_edges[6 * c + e]].push_back(c);
  std::vector<int> col(L.ne, -1);
  int ncol = 0;
  for (int e = 0; e < L.ne; ++e) {
    if (ef[e].empty()) continue;
    std::vector<char> used(64, 0);
    for (int c : ec[e])
      for (int j = 0; j < 6; ++j) {
        int cc = col[L.cell_edges[6 * c + j]];
        if (cc >= 0) {
          if (cc >= (int)used.size()) used.resize(cc + 1, 0);
          used[cc] = 1;
        }
      }
    int k = 0;
    while (k < (int)used.size() && used[k]) ++k;
    col[e] = k;
    ncol = std::max(ncol, k + 1);
  }
  L.ncol = ncol;
  L.colour_ptr.assign(ncol + 1, 0);
  L.patch_edge.clear();
  for (int k = 0; k < ncol; ++k) {
    L.colour_ptr[k] = (int)L.patch_edge.size();
    for (int e = 0; e < L.ne; ++e)
      if (col[e] == k) L.patch_edge.push_back(e);
  }
  L.colour_ptr[ncol] = (int)L.patch_edge.size();
  L.pf_ptr.assign(1, 0);
  L.pc_ptr.assign(1, 0);
  L.pf.clear();
  L.pc.clear();
  L.max_patch_faces = L.max_patch_cells = 0;
  for (int e : L.patch_edge) {
    std::vector<int> fs = ef[e];
    std::sort(fs.begin(), fs.end());
    L.pf.insert(L.pf.end(), fs.begin(), fs.end());
    L.pf_ptr.push_back((int)L.pf.size());
    std::vector<int> cs = ec[e];
    std::sort(cs.begin(), cs.end());
    L.pc.insert(L.pc.end(), cs.begin(), cs.end());
    L.pc_ptr.push_back((int)L.pc.size());
    L.max_patch_faces = std::max(L.max_patch_faces, (int)fs.size());
    L.max_patch_cells = std::max(L.max_patch_cells, (int)cs.size());
  }
}

void build_vertex_patches(Level3& L) {
  std::vector<std::vector<int>> vf(L.nv), vc(L.nv);
  for (int f = 0; f < L.nf; ++f) {
    if (L.int_id[f] < 0) continue;
    for (int i = 0; i < 3; ++i) vf[L.faces[3 * f + i]].push_back(L.int_id[f]);
  }
  for (int c = 0; c < L.nc; ++c)
    for (int i = 0; i < 4; ++i) vc[L.cells[4 * c + i]].push_back(c);
  std::vector<int> col(L.nv, -1);
  int ncol = 0;
  for (int v = 0; v < L.nv; ++v) {
    if (vf[v].empty()) continue;
    std::vector<char> used(64, 0);
    for (int c : vc[v])
      for (int j = 0; j < 4; ++j) {
        const int cc = col[L.cells[4 * c + j]];
        if (cc >= 0) {
          if (cc >= (int)used.size()) used.resize(cc + 1, 0);
          used[cc] = 1;
        }
      }
    int k = 0;
    while (k < (int)used.size() && used[k]) ++k;
    col[v] = k;
    ncol = std::max(ncol, k + 1);
  }
  L.ncol = ncol;
  L.colour_ptr.assign(ncol + 1, 0);
  L.patch_edge.clear();
  for (int k = 0; k < ncol; ++k) {
    L.colour_ptr[k] = (int)L.patch_edge.size();
    for (int v = 0; v < L.nv; ++v)
      if (col[v] == k) L.patch_edge.push_back(v);
  }
  L.colour_ptr[ncol] = (int)L.patch_edge.size();
  L.pf_ptr.assign(1, 0);
  L.pc_ptr.assign(1, 0);
  L.pf.clear();
  L.pc.clear();
  L.max_patch_faces = L.max_patch_cells = 0;
  for (int v : L.patch_edge) {
    std::vector<int> fs = vf[v];
    std::sort(fs.begin(), fs.end());
    L.pf.insert(L.pf.end(), fs.begin(), fs.end());
    L.pf_ptr.push_back((int)L.pf.size());
    std::vector<int> cs = vc[v];
    std::sort(cs.begin(), cs.end());
    L.pc.insert(L.pc.end(), cs.begin(), cs.end());
    L.pc_ptr.push_back((int)L.pc.size());
    L.max_patch_faces = std::max(L.max_patch_faces, (int)fs.size());
    L.max_patch_cells = std::max(L.max_patch_cells, (int)cs.size());
  }
}

namespace {
// barycentric coordinates of x in cell T of level C
void bary(const Level3& C, int T, const double* x, double* lam) {
  const int* v = &C.cells[4 * T];
  double A[4][5];
  for (int r = 0; r < 3; ++r) {
    for (int j = 0; j < 4; ++j) A[r][j] = C.X[3 * v[j] + r];
    A[r][4] = x[r];
  }
  for (int j = 0; j < 4; ++j) A[3][j] = 1.0;
  A[3][4] = 1.0;
  for (int p = 0; p < 4; ++p) {
    int piv = p;
    for (int r = p + 1; r < 4; ++r)
      if (std::fabs(A[r][p]) > std::fabs(A[piv][p])) piv = r;
    if (piv != p)
      for (int j = 0; j < 5; ++j) std::swap(A[p][j], A[piv][j]);
    for (int r = 0; r < 4; ++r) {
      if (r == p) continue;
      double f = A[r][p] / A[p][p];
      for (int j = p; j < 5; ++j) A[r][j] -= f * A[p][j];
    }
  }
  for (int j = 0; j < 4; ++j) lam[j] = A[j][4] / A[j][j];
}
}  // namespace

void build_averaging3(const Level3& C, const Level3& F, Averaging3& A) {
  const int nrow = 3 * F.nint;
  std::vector<std::vector<std::pair<int, double>>> rows(nrow);
  A.inner.assign((size_t)C.nc * 8, -1);
  std::vector<int> ninner(C.nc, 0);
  for (int fi = 0; fi < F.nint; ++fi) {
    const int f = F.int_face[fi];
    double x[3] = {0, 0, 0};
    for (int j = 0; j < 3; ++j)
      for (int d = 0; d < 3; ++d) x[d] += F.X[3 * F.faces[3 * f + j] + d] / 3.0;
    const int T = F.parent[F.face_cells[2 * f]];
    double lam[4];
    bary(C, T, x, lam);
    int i0 = 0;
    for (int j = 1; j < 4; ++j)
      if (lam[j] < lam[i0]) i0 = j;
    // weights: contribution of each coarse unknown (3 E + c) to the
    // Cartesian value at x, accumulated per fine component
    std::vector<std::pair<int, std::array<double, 3>>> w;
    auto add_cell = [&](int cell, double scale) {
      double l[4];
      bary(C, cell, x, l);
      for (int i = 0; i < 4; ++i) {
        int E = C.cell_faces[4 * cell + i];
        int ei = C.int_id[E];
        if (ei < 0) continue;
        double phi = (1.0 - 3.0 * l[i]) * scale;
        const double* fr[3] = {&C.fn[3 * E], &C.ft1[3 * E], &C.ft2[3 * E]};
        for (int c = 0; c < 3; ++c) w.push_back({3 * ei + c, {phi * fr[c][0], phi * fr[c][1], phi * fr[c][2]}});
      }
    };
    if (lam[i0] > 1e-12) {
      add_cell(T, 1.0);
      A.inner[8 * T + ninner[T]++] = fi;
    } else {
      int E = C.cell_faces[4 * T + i0];
      int a = C.face_cells[2 * E], b = C.face_cells[2 * E + 1];
      int T2 = a == T ? b : a;
      add_cell(T, 0.5);
      if (T2 >= 0) add_cell(T2, 0.5);
    }
    const double* ff[3] = {&F.fn[3 * f], &F.ft1[3 * f], &F.ft2[3 * f]};
    for (int c = 0; c < 3; ++c) {
      auto& row = rows[3 * fi + c];
      for (auto& p : w) {
        double v = p.second[0] * ff[c][0] + p.second[1] * ff[c][1] + p.second[2] * ff[c][2];
        bool merged = false;
        for (auto& q : row)
          if (q.first == p.first) {
            q.second += v;
            merged = true;
            break;
          }
        if (!merged) row.push_back({p.first, v});
      }
    }
  }
  A.row_ptr.assign(nrow + 1, 0);
  A.col.clear();
  A.val.clear();
  for (int r = 0; r < nrow; ++r) {
    auto row = rows[r];
    std::sort(row.begin(), row.end());
    for (auto& p : row) {
      A.col.push_back(p.first);
      A.val.push_back(p.second);
    }
    A.row_ptr[r + 1] = (int)A.col.size();
  }
}

}  // namespace hdgmg
