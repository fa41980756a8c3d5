// Host-side numeric setup (quadrature tables, transfers, coarsest inverse).
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <map>
#include <thread>

namespace hdgmg {

namespace {
// Gauss-Legendre on [0,1] (ascending nodes, weights sum 1) by Newton on P_n.
void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double p0 = 1.0, p1 = t, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      p0 = 1.0;
      p1 = t;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2 * j - 1) * t * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    p0 = 1.0;
    p1 = t;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2 * j - 1) * t * p1 - (j - 1) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[n - 1 - i] = 0.5 * (t + 1.0);              // cos ordering is descending
    w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // (2 / ((1-t^2) P_n'^2)) / 2
  }
}

// Jacobi P_n^{(1,0)} and its derivative.
void jacobi10(int n, double t, double& pn, double& dpn) {
  const double a = 1.0, b = 0.0;
  double p0 = 1.0, p1 = (a + 1.0) + (a + b + 2.0) * (t - 1.0) / 2.0;
  if (n == 0) {
    pn = 1.0;
    dpn = 0.0;
    return;
  }
  for (int j = 2; j <= n; ++j) {
    double c1 = 2.0 * j * (j + a + b) * (2.0 * j + a + b - 2.0);
    double c2 = (2.0 * j + a + b - 1.0) * ((2.0 * j + a + b) * (2.0 * j + a + b - 2.0) * t + a * a - b * b);
    double c3 = 2.0 * (j + a - 1.0) * (j + b - 1.0) * (2.0 * j + a + b);
    double p2 = (c2 * p1 - c3 * p0) / c1;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  // (2n+a+b)(1-t^2) P_n' = n[(a-b) - (2n+a+b) t] P_n + 2(n+a)(n+b) P_{n-1}
  dpn = (n * ((a - b) - (2.0 * n + a + b) * t) * p1 + 2.0 * (n + a) * (n + b) * p0) /
        ((2.0 * n + a + b) * (1.0 - t * t));
}

// Gauss-Jacobi nodes/weights for int_0^1 (1-v) g(v) dv: roots of
// P_n^{(1,0)} bracketed on a grid, refined by bisection then Newton.
void gauss_jacobi10_01(int n, double* x, double* w) {
  const int G = 4000;
  int found = 0;
  double prev_t = -1.0 + 1e-12, pv, dv;
  jacobi10(n, prev_t, pv, dv);
  for (int i = 1; i <= G && found < n; ++i) {
    double t = -1.0 + 2.0 * i / G;
    if (i == G) t = 1.0 - 1e-12;
    double pc, dc;
    jacobi10(n, t, pc, dc);
    if ((pv < 0) != (pc < 0)) {
      double lo = prev_t, hi = t, plo = pv;
      for (int it = 0; it < 60; ++it) {
        double mid = 0.5 * (lo + hi), pm, dm;
        jacobi10(n, mid, pm, dm);
        if ((pm < 0) == (plo < 0)) {
          lo = mid;
          plo = pm;
        } else {
          hi = mid;
        }
      }
      double r = 0.5 * (lo + hi);
      for (int it = 0; it < 5; ++it) {
        double pr, dr;
        jacobi10(n, r, pr, dr);
        if (dr == 0) break;
        r -= pr / dr;
      }
      double pr, dr;
      jacobi10(n, r, pr, dr);
      x[found] = 0.5 * (r + 1.0);
      w[found] = (4.0 / ((1.0 - r * r) * dr * dr)) / 4.0;
      ++found;
    }
    prev_t = t;
    pv = pc;
  }
}

}  // namespace

QuadTables make_tables(int k) {
  QuadTables Q;
  std::memset(&Q, 0, sizeof(Q));
  Q.k = k;
  const int n = k + 2;
  Q.nq = n * n;
  Q.nfq = n;
  double u[NF_MAX], wu[NF_MAX], v[NF_MAX], wv[NF_MAX];
  gauss_legendre01(n, u, wu);
  gauss_jacobi10_01(n, v, wv);
  double tot = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int q = j * n + i;
      Q.xi[q][0] = u[i] * (1.0 - v[j]);
      Q.xi[q][1] = v[j];
      Q.wq[q] = wu[i] * wv[j];
      tot += Q.wq[q];
    }
  for (int q = 0; q < Q.nq; ++q) Q.wq[q] /= tot;
  for (int i = 0; i < n; ++i) {
    Q.s[i] = u[i];
    Q.ws[i] = wu[i];
  }
  return Q;
}

ConvTables make_conv_tables(int k) {
  ConvTables T;
  std::memset(&T, 0, sizeof(T));
  const int n = (3 * k + 4) / 2;
  T.n = n;
  T.nq = n * n;
  double u[NC_MAX], wu[NC_MAX], v[NC_MAX], wv[NC_MAX];
  gauss_legendre01(n, u, wu);
  gauss_jacobi10_01(n, v, wv);
  double tot = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int q = j * n + i;
      T.xi[q][0] = u[i] * (1.0 - v[j]);
      T.xi[q][1] = v[j];
      T.wq[q] = wu[i] * wv[j];
      tot += T.wq[q];
    }
  for (int q = 0; q < T.nq; ++q) T.wq[q] /= tot;
  for (int i = 0; i < n; ++i) {
    T.s[i] = u[i];
    T.ws[i] = wu[i];
  }
  return T;
}

// ------------------------------------------------------------ dense helpers
bool invert_spd(const std::vector<double>& A, int n, std::vector<double>& inv) {
  // Cholesky then column solves; inv column-major (symmetric anyway)
  std::vector<double> L(A);
  for (int j = 0; j < n; ++j) {
    double d = L[(size_t)j * n + j];
    for (int q = 0; q < j; ++q) d -= L[(size_t)j * n + q] * L[(size_t)j * n + q];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = L[(size_t)i * n + j];
      for (int q = 0; q < j; ++q) s -= L[(size_t)i * n + q] * L[(size_t)j * n + q];
      L[(size_t)i * n + j] = s / d;
    }
  }
  inv.assign((size_t)n * n, 0.0);
  std::vector<double> col(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = i == c ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) s -= L[(size_t)i * n + q] * col[q];
      col[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = col[i];
      for (int q = i + 1; q < n; ++q) s -= L[(size_t)q * n + i] * col[q];
      col[i] = s / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[(size_t)c * n + i] = col[i];
  }
  return true;
}

bool invert_general(const std::vector<double>& A, int n, std::vector<double>& inv) {
  std::vector<double> LU(A);
  std::vector<int> piv(n);
  for (int j = 0; j < n; ++j) {
    int pr = j;
    double best = std::fabs(LU[(size_t)j * n + j]);
    for (int i = j + 1; i < n; ++i)
      if (std::fabs(LU[(size_t)i * n + j]) > best) {
        best = std::fabs(LU[(size_t)i * n + j]);
        pr = i;
      }
    if (!(best > 0)) return false;
    piv[j] = pr;
    if (pr != j)
      for (int c = 0; c < n; ++c) std::swap(LU[(size_t)j * n + c], LU[(size_t)pr * n + c]);
    for (int i = j + 1; i < n; ++i) {
      double l = LU[(size_t)i * n + j] / LU[(size_t)j * n + j];
      LU[(size_t)i * n + j] = l;
      if (l != 0.0)
        for (int c = j + 1; c < n; ++c) LU[(size_t)i * n + c] -= l * LU[(size_t)j * n + c];
    }
  }
  inv.assign((size_t)n * n, 0.0);
  std::vector<double> col(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) col[i] = i == c ? 1.0 : 0.0;
    for (int j = 0; j < n; ++j)
      if (piv[j] != j) std::swap(col[j], col[piv[j]]);
    for (int i = 0; i < n; ++i)
      for (int q = 0; q < i; ++q) col[i] -= LU[(size_t)i * n + q] * col[q];
    for (int i = n - 1; i >= 0; --i) {
      double t = col[i];
      for (int q = i + 1; q < n; ++q) t -= LU[(size_t)i * n + q] * col[q];
      col[i] = t / LU[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[(size_t)c * n + i] = col[i];
  }
  return true;
}

void host_cr_blocks(const Level& L, const std::vector<double>& nu, double beta, double eps_inv,
                    std::vector<double>& B) {
  B.resize((size_t)L.nc * 36);
  for (int c = 0; c < L.nc; ++c) {
    CellGeom g;
    cell_geom(L.X.data(), L.cells.data() + 3 * c, g);
    cr_block(g, nu[c], beta, eps_inv, &B[(size_t)c * 36]);
  }
}


void level_viscosities(const std::vector<Level>& lv, const std::vector<double>& nu_fine,
                       std::vector<std::vector<double>>& nu) {
  const int J = (int)lv.size();
  nu.assign(J, {});
  nu[J - 1] = nu_fine;
  for (int l = J - 1; l > 0; --l) {
    nu[l - 1].assign(lv[l - 1].nc, 0.0);
    for (int c = 0; c < lv[l - 1].nc; ++c)
      nu[l - 1][c] = 0.25 * (nu[l][4 * c] + nu[l][4 * c + 1] + nu[l][4 * c + 2] + nu[l][4 * c + 3]);
  }
}

bool stabilised_transfer(const Level& Cl, const Level& Fl, const Averaging& Av, const std::vector<double>& B,
                         bool transpose, bool general, CSR& Pc) {
  const int nfd = 2 * Fl.nint;
  // rows of P in fixed-capacity slots (the averaging rows have <= 10 entries,
  // the corrected interior rows the coarse unknowns of a coarse cell and its
  // three neighbours)
  constexpr int CAP = 24;
  std::vector<int> pc((size_t)nfd * CAP), pn(nfd, 0);
  std::vector<double> pv((size_t)nfd * CAP);
  std::atomic<bool> overflow(false);
  auto add_to = [&](int r, int c, double v) {
    int* ci = &pc[(size_t)r * CAP];
    double* cv = &pv[(size_t)r * CAP];
    for (int e = 0; e < pn[r]; ++e)
      if (ci[e] == c) {
        cv[e] += v;
        return;
      }
    if (pn[r] == CAP) {
      overflow = true;
      return;
    }
    ci[pn[r]] = c;
    cv[pn[r]++] = v;
  };
  // P starts as the averaging I (duplicate columns merged)
  for (int r = 0; r < nfd; ++r)
    for (int q = Av.row_ptr[r]; q < Av.row_ptr[r + 1]; ++q) add_to(r, Av.col[q], Av.val[q]);
  // harmonic correction inside every coarse cell: rows of the interior fine
  // DOFs become I - A_TT^-1 (A I)_T (A I from the unmodified averaging rows).
  // Coarse cells own disjoint interior rows: ranges of them run in parallel.
  std::atomic<bool> failed(false);
  auto cells = [&](int T0, int T1) {
  std::vector<int> cols;
  std::vector<double> AI, ATT(36), inv;
  for (int T = T0; T < T1 && !failed; ++T) {
    int inner[3];
    for (int i = 0; i < 3; ++i) inner[i] = Av.inner_facets[3 * T + i];
    auto pos_of = [&](int fi) {
      for (int i = 0; i < 3; ++i)
        if (inner[i] == fi) return i;
      return -1;
    };
    std::fill(ATT.begin(), ATT.end(), 0.0);
    cols.clear();
    AI.clear();  // [column slot][6]
    auto slot = [&](int c) {
      for (size_t i = 0; i < cols.size(); ++i)
        if (cols[i] == c) return (int)i;
      cols.push_back(c);
      AI.resize(AI.size() + 6, 0.0);
      return (int)cols.size() - 1;
    };
    int sl[32];
    for (int ch = 0; ch < 4; ++ch) {
      int Kc = 4 * T + ch;
      const double* BK = &B[(size_t)Kc * 36];
      int p1s[3];
      for (int i1 = 0; i1 < 3; ++i1) {
        int f1 = Fl.cell_dofs[3 * Kc + i1];
        p1s[i1] = f1 >= 0 ? pos_of(f1) : -1;
      }
      for (int i2 = 0; i2 < 3; ++i2) {
        int f2 = Fl.cell_dofs[3 * Kc + i2];
        if (f2 < 0) continue;
        int p2 = pos_of(f2);
        for (int bb = 0; bb < 2; ++bb) {
          const int r = 2 * f2 + bb;
          const int q0 = Av.row_ptr[r], nq = std::min(Av.row_ptr[r + 1] - q0, 32);
          if (Av.row_ptr[r + 1] - q0 > 32) {
            failed = true;
            return;
          }
          for (int q = 0; q < nq; ++q) sl[q] = slot(Av.col[q0 + q]);
          for (int i1 = 0; i1 < 3; ++i1) {
            const int p1 = p1s[i1];
            if (p1 < 0) continue;
            for (int a = 0; a < 2; ++a) {
              double v = transpose ? BK[(2 * i2 + bb) * 6 + 2 * i1 + a] : BK[(2 * i1 + a) * 6 + 2 * i2 + bb];
              if (p2 >= 0) ATT[(2 * p1 + a) * 6 + 2 * p2 + bb] += v;
              for (int q = 0; q < nq; ++q) AI[(size_t)sl[q] * 6 + 2 * p1 + a] += v * Av.val[q0 + q];
            }
          }
        }
      }
    }
    if (!(general ? invert_general(ATT, 6, inv) : invert_spd(ATT, 6, inv))) {
      failed = true;
      return;
    }
    for (int a = 0; a < 6; ++a) {
      int fr = 2 * inner[a / 2] + a % 2;
      for (size_t j = 0; j < cols.size(); ++j) {
        double s = 0.0;
        for (int bb = 0; bb < 6; ++bb) s += inv[(size_t)bb * 6 + a] * AI[j * 6 + bb];
        if (s != 0.0) add_to(fr, cols[j], -s);
      }
    }
  }
  };
  const int nth = Cl.nc >= 2048 ? (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency())) : 1;
  if (nth <= 1) {
    cells(0, Cl.nc);
  } else {
    std::vector<std::thread> th;
    const int chunk = (Cl.nc + nth - 1) / nth;
    for (int i = 0; i < nth; ++i) th.emplace_back(cells, i * chunk, std::min(Cl.nc, (i + 1) * chunk));
    for (auto& t : th) t.join();
  }
  if (failed) return false;
  if (overflow) return false;
  Pc = CSR();
  Pc.n = nfd;
  Pc.rp.assign(1, 0);
  Pc.ci.reserve((size_t)nfd * 14);
  Pc.v.reserve((size_t)nfd * 14);
  std::vector<std::pair<int, double>> row;
  for (int r = 0; r < nfd; ++r) {
    row.clear();
    for (int e = 0; e < pn[r]; ++e) row.push_back({pc[(size_t)r * CAP + e], pv[(size_t)r * CAP + e]});
    std::sort(row.begin(), row.end());
    for (auto& kv : row) {
      if (kv.second == 0.0) continue;
      Pc.ci.push_back(kv.first);
      Pc.v.push_back(kv.second);
    }
    Pc.rp.push_back((int)Pc.ci.size());
  }
  return true;
}

void csr_transpose(const CSR& A, int ncols, CSR& T) {
  T = CSR();
  T.n = ncols;
  T.rp.assign(ncols + 1, 0);
  for (int c : A.ci) ++T.rp[c + 1];
  for (int c = 0; c < ncols; ++c) T.rp[c + 1] += T.rp[c];
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  std::vector<int> next(T.rp.begin(), T.rp.end() - 1);
  for (int r = 0; r < A.n; ++r)
    for (int q = A.rp[r]; q < A.rp[r + 1]; ++q) {
      const int at = next[A.ci[q]]++;
      T.ci[at] = r;
      T.v[at] = A.v[q];
    }
}

void assemble_csr(const Level& L, const std::vector<double>& B, CSR& A) {
  // a lowest-order unknown couples with the unknowns of the facets of its two
  // cells: at most 10 columns per row
  constexpr int CAP = 10;
  const int n = 2 * L.nint;
  std::vector<int> ci((size_t)n * CAP), cnt(n, 0);
  std::vector<double> cv((size_t)n * CAP);
  for (int c = 0; c < L.nc; ++c)
    for (int i1 = 0; i1 < 3; ++i1) {
      int f1 = L.cell_dofs[3 * c + i1];
      if (f1 < 0) continue;
      for (int i2 = 0; i2 < 3; ++i2) {
        int f2 = L.cell_dofs[3 * c + i2];
        if (f2 < 0) continue;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            const int r = 2 * f1 + a, col = 2 * f2 + b;
            const double v = B[(size_t)c * 36 + (2 * i1 + a) * 6 + 2 * i2 + b];
            int* rc = &ci[(size_t)r * CAP];
            double* rv = &cv[(size_t)r * CAP];
            int e = 0;
            while (e < cnt[r] && rc[e] != col) ++e;
            if (e == cnt[r]) {
              if (e == CAP) continue;  // cannot happen on a conforming triangulation
              rc[e] = col;
              rv[e] = 0.0;
              ++cnt[r];
            }
            rv[e] += v;
          }
      }
    }
  A = CSR();
  A.n = n;
  A.rp.assign(1, 0);
  std::vector<std::pair<int, double>> row;
  for (int r = 0; r < n; ++r) {
    row.clear();
    for (int e = 0; e < cnt[r]; ++e) row.push_back({ci[(size_t)r * CAP + e], cv[(size_t)r * CAP + e]});
    std::sort(row.begin(), row.end());
    for (auto& kv : row) {
      A.ci.push_back(kv.first);
      A.v.push_back(kv.second);
    }
    A.rp.push_back((int)A.ci.size());
  }
}

bool coarse_inverse(const Level& L0, const std::vector<double>& B, bool general, std::vector<double>& inv) {
  const int n = 2 * L0.nint;
  std::vector<double> A((size_t)n * n, 0.0);
  for (int c = 0; c < L0.nc; ++c)
    for (int i1 = 0; i1 < 3; ++i1) {
      int f1 = L0.cell_dofs[3 * c + i1];
      if (f1 < 0) continue;
      for (int i2 = 0; i2 < 3; ++i2) {
        int f2 = L0.cell_dofs[3 * c + i2];
        if (f2 < 0) continue;
        for (int a = 0; a < 2; ++a)
          for (int bb = 0; bb < 2; ++bb)
            A[(size_t)(2 * f1 + a) * n + 2 * f2 + bb] += B[(size_t)c * 36 + (2 * i1 + a) * 6 + 2 * i2 + bb];
      }
    }
  if (n == 0) {
    inv.clear();
    return true;
  }
  return general ? invert_general(A, n, inv) : invert_spd(A, n, inv);
}

}  // namespace hdgmg
