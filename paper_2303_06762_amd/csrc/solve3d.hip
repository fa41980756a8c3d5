// Host orchestration of the tetrahedral path: hierarchy and topology
// (mesh3d), assembly of the order-k cell blocks (tet.hip), the lowest-order
// CR-equivalent levels, harmonic-extension transfers and the coarsest
// inverse, MG_h (Alg. 1) with edge-patch block Gauss-Seidel, MG_hp (Alg. 2),
// flexible CG and the AL-Uzawa loop (stOpEq-ALU).
#include "solve3d.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "host_setup.hpp"
#include "kernels.hpp"
#include "mesh3d.hpp"
#include "tet.hpp"

namespace hdgmg {

namespace {

struct DevLev3 {
  int nc = 0, nint = 0, mF = 1, nK = 12;
  long ndof = 0;
  int *cells = nullptr, *cell_dofs = nullptr, *fcell = nullptr, *floc = nullptr;
  double *X = nullptr, *vol = nullptr, *cdiv = nullptr, *fdiv = nullptr, *nu = nullptr;
  double* S = nullptr;
  float* S32 = nullptr;
  int np = 0, ncol = 0, ns_max = 0;
  bool vertex = false;   // vertex patches (Gauss-Seidel by full residual + patch correction per colour)
  std::vector<int> colour_ptr, hns;
  int *pf_ptr = nullptr, *pf = nullptr, *pc_ptr = nullptr, *pc = nullptr;
  long* poff = nullptr;
  // lowest-order edge patches: one record per patch cell (cell, packed patch
  // faces / slots / sides / far faces, the far faces' interior numbers), in
  // patch-cell order
  int* prec = nullptr;
  long pinv_len = 0;
  double* pinv = nullptr;
  float* pinv32 = nullptr;
  std::vector<long> hpoff;
  // words each colour phase reads: cell-block entries, patch-inverse
  // entries, and vector words (FP64)
  std::vector<double> phase_S, phase_P, phase_V;
  // vector words of a phase from x = 0 (b read, x read and written on the
  // patch faces; no cell blocks or cell vectors)
  std::vector<double> phase_V0;
  double *u = nullptr, *g = nullptr, *r = nullptr, *yK = nullptr;
  // order-k level: the twelve mode-0 rows of every cell block ([nK][12][nc],
  // in the V-cycle's storage, FP32 without the AL term) and their products,
  // for the residual that MG_hp restricts to the lowest-order space
  double* S0 = nullptr;
  float* S0_32 = nullptr;
  double* y0K = nullptr;
};

struct DevTr3 {
  int nfine = 0, ncoarse = 0, Pw = 0, Rw = 0;
  int *Pci = nullptr, *Rci = nullptr;
  double *Pv = nullptr, *Rv = nullptr;
  float *Pv32 = nullptr, *Rv32 = nullptr;
};

}  // namespace

struct Ctx3 {
  int k = 0, J = 1;
  double beta = 0.0, eps_inv = 1.0;
  std::vector<double> nu_fine;
  hdgmg_opts opts;
  hipStream_t st = nullptr, own = nullptr;
  hdgmg_alloc_fn alloc_fn = nullptr;
  hdgmg_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  std::vector<void*> allocs;
  std::vector<Level3> lv;
  std::vector<Averaging3> av;
  TetTables* T = nullptr;
  DevLev3 K;
  std::vector<DevLev3> cr;
  std::vector<DevTr3> tr;
  double* coarse_inv = nullptr;
  // the coarsest inverse row by row (rows padded to ld0 words) for the
  // wavefront-per-row GEMV, in the V-cycle's storage precision
  double* coarse_rows = nullptr;
  float* coarse_rows32 = nullptr;
  int ld0 = 0;
  int n0 = 0;
  double *x = nullptr, *r = nullptr, *r_old = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double *b = nullptr, *gvec = nullptr, *lam = nullptr, *p0 = nullptr, *sc = nullptr, *part = nullptr;
  double *statebuf = nullptr, *gK = nullptr;
  int* status = nullptr;
  bool assembled = false;
  std::string err;
  struct Timer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    double bytes = 0.0;
  } timers[5];
  double apply_bytes = 0.0, vcycle_bytes = 0.0, vcycle_compulsory = 0.0;
};

namespace {

#define HIPC3(expr)                                                                 \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      c->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr; \
      return HDGMG_EHIP;                                                            \
    }                                                                               \
  } while (0)
#define TRY3(expr)                   \
  do {                               \
    hdgmg_status s_ = (expr);        \
    if (s_ != HDGMG_OK) return s_;   \
  } while (0)

void* raw_alloc(Ctx3* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (c->alloc_fn) return c->alloc_fn(bytes, c->alloc_ctx);
  void* v = nullptr;
  return hipMalloc(&v, bytes) == hipSuccess ? v : nullptr;
}
void raw_free(Ctx3* c, void* p) {
  if (!p) return;
  if (c->free_fn)
    c->free_fn(p, c->alloc_ctx);
  else
    (void)hipFree(p);
}

template <typename T>
hdgmg_status dalloc(Ctx3* c, T** p, size_t n) {
  void* v = raw_alloc(c, n * sizeof(T));
  if (!v) {
    c->err = "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed";
    return HDGMG_ENOMEM;
  }
  c->allocs.push_back(v);
  *p = static_cast<T*>(v);
  return HDGMG_OK;
}

template <typename T>
hdgmg_status upload(Ctx3* c, T** p, const std::vector<T>& h) {
  TRY3(dalloc(c, p, std::max<size_t>(h.size(), 1)));
  if (!h.empty()) HIPC3(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->st));
  return HDGMG_OK;
}

// ---- quadrature tables (host) ----------------------------------------------
// Gauss-Jacobi rule for int_0^1 (1-v)^alpha g(v) dv by the Golub-Welsch
// eigenvalue problem of the Jacobi matrix of the weight (1-t)^alpha on
// [-1, 1] (symmetric tridiagonal QL with implicit shifts).
void gauss_jacobi01(int n, double alpha, double* x, double* w) {
  std::vector<double> dg(n), off(n, 0.0), z((size_t)n * n, 0.0);
  const double a = alpha, b = 0.0;
  for (int i = 0; i < n; ++i) {
    const double s = 2.0 * i + a + b;
    dg[i] = (i == 0 && a + b == 0.0) ? (b - a) / (a + b + 2.0) : (b * b - a * a) / (s * (s + 2.0));
    if (i + 1 < n) {
      const double j = i + 1.0, t = 2.0 * j + a + b;
      off[i] = std::sqrt(4.0 * j * (j + a) * (j + b) * (j + a + b) / (t * t * (t + 1.0) * (t - 1.0)));
    }
    z[(size_t)i * n + i] = 1.0;
  }
  // tqli on (dg, off): eigenvalues in dg, eigenvectors in the rows of z
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 200; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(dg[m]) + std::fabs(dg[m + 1]);
        if (std::fabs(off[m]) <= 1e-17 * dd) break;
      }
      if (m == l) break;
      double g = (dg[l + 1] - dg[l]) / (2.0 * off[l]);
      double r = std::hypot(g, 1.0);
      g = dg[m] - dg[l] + off[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
      double s = 1.0, cc = 1.0, p = 0.0;
      int i = m - 1;
      for (; i >= l; --i) {
        double f = s * off[i], bb = cc * off[i];
        r = std::hypot(f, g);
        off[i + 1] = r;
        if (r == 0.0) {
          dg[i + 1] -= p;
          off[m] = 0.0;
          break;
        }
        s = f / r;
        cc = g / r;
        g = dg[i + 1] - p;
        r = (dg[i] - g) * s + 2.0 * cc * bb;
        p = s * r;
        dg[i + 1] = g + p;
        g = cc * r - bb;
        for (int kk = 0; kk < n; ++kk) {
          f = z[(size_t)(i + 1) * n + kk];
          z[(size_t)(i + 1) * n + kk] = s * z[(size_t)i * n + kk] + cc * f;
          z[(size_t)i * n + kk] = cc * z[(size_t)i * n + kk] - s * f;
        }
      }
      if (r == 0.0 && i >= l) continue;
      dg[l] -= p;
      off[l] = g;
      off[m] = 0.0;
    }
  }
  // weights: mu0 * (first component of the normalised eigenvector)^2
  std::vector<std::pair<double, double>> nw(n);
  double tot = 0.0;
  for (int i = 0; i < n; ++i) {
    const double v0 = z[(size_t)i * n + 0];
    nw[i] = {dg[i], v0 * v0};
    tot += v0 * v0;
  }
  std::sort(nw.begin(), nw.end());
  for (int i = 0; i < n; ++i) {
    x[i] = 0.5 * (nw[i].first + 1.0);
    w[i] = nw[i].second / tot;  // normalised; scaled by the caller
  }
}

void make_tet_tables(int k, TetTables& T) {
  std::memset(&T, 0, sizeof(T));
  const int n = k + 2;
  T.k = k;
  T.nq = n * n * n;
  T.nfq = n * n;
  double u[8], wu[8], v[8], wv[8], s[8], ws[8];
  gauss_jacobi01(n, 0.0, u, wu);
  gauss_jacobi01(n, 1.0, v, wv);
  gauss_jacobi01(n, 2.0, s, ws);
  double tot = 0.0;
  int q = 0;
  for (int c = 0; c < n; ++c)
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a, ++q) {
        T.xq[q][0] = u[a] * (1.0 - v[b]) * (1.0 - s[c]);
        T.xq[q][1] = v[b] * (1.0 - s[c]);
        T.xq[q][2] = s[c];
        T.wq[q] = wu[a] * wv[b] * ws[c];
        tot += T.wq[q];
      }
  for (q = 0; q < T.nq; ++q) T.wq[q] /= tot;
  tot = 0.0;
  q = 0;
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a, ++q) {
      T.xf[q][0] = u[a] * (1.0 - v[b]);
      T.xf[q][1] = v[b];
      T.wf[q] = wu[a] * wv[b];
      tot += T.wf[q];
    }
  for (q = 0; q < T.nfq; ++q) T.wf[q] /= tot;
  // face basis: modified Gram-Schmidt (two passes) of xi^a eta^b ordered by
  // degree, then b, in the discrete inner product of the face rule (exact
  // for the degree-2k products)
  const int mF = (k + 1) * (k + 2) / 2, nf = T.nfq;
  std::vector<double> B((size_t)mF * nf);
  int j = 0;
  for (int dgr = 0; dgr <= k; ++dgr)
    for (int bb = 0; bb <= dgr; ++bb, ++j) {
      const int aa = dgr - bb;
      for (int l = 0; l < nf; ++l) B[(size_t)j * nf + l] = std::pow(T.xf[l][0], aa) * std::pow(T.xf[l][1], bb);
    }
  for (int i = 0; i < mF; ++i) {
    double* bi = &B[(size_t)i * nf];
    for (int pass = 0; pass < 2; ++pass)
      for (int p = 0; p < i; ++p) {
        const double* bp = &B[(size_t)p * nf];
        double d = 0.0;
        for (int l = 0; l < nf; ++l) d += T.wf[l] * bi[l] * bp[l];
        for (int l = 0; l < nf; ++l) bi[l] -= d * bp[l];
      }
    double nn = 0.0;
    for (int l = 0; l < nf; ++l) nn += T.wf[l] * bi[l] * bi[l];
    nn = std::sqrt(nn);
    for (int l = 0; l < nf; ++l) bi[l] /= nn;
  }
  for (int l = 0; l < nf; ++l)
    for (int i = 0; i < mF; ++i) T.phif[l][i] = B[(size_t)i * nf + l];
}

// ---- lowest-order transfers (host) ------------------------------------------
void assemble_csr3(const Level3& L, const std::vector<double>& B, CSR& A) {
  const int n = 3 * L.nint;
  std::vector<std::vector<std::pair<int, double>>> rows(n);
  for (int c = 0; c < L.nc; ++c)
    for (int i = 0; i < 4; ++i) {
      const int di = L.cell_dofs[4 * c + i];
      if (di < 0) continue;
      for (int a = 0; a < 3; ++a)
        for (int j = 0; j < 4; ++j) {
          const int dj = L.cell_dofs[4 * c + j];
          if (dj < 0) continue;
          for (int bb = 0; bb < 3; ++bb) rows[3 * di + a].push_back({3 * dj + bb, B[(size_t)c * 144 + (3 * i + a) * 12 + 3 * j + bb]});
        }
    }
  A.n = n;
  A.rp.assign(n + 1, 0);
  A.ci.clear();
  A.v.clear();
  for (int r = 0; r < n; ++r) {
    auto& row = rows[r];
    std::sort(row.begin(), row.end());
    for (size_t t = 0; t < row.size(); ++t) {
      if (!A.ci.empty() && (int)A.rp[r] < (int)A.ci.size() && A.ci.back() == row[t].first) {
        A.v.back() += row[t].second;
      } else {
        A.ci.push_back(row[t].first);
        A.v.push_back(row[t].second);
      }
    }
    A.rp[r + 1] = (int)A.ci.size();
  }
}

// (id - E_T A_TT^-1 A_T.) I, rows of the fine unknowns inside each coarse cell
// corrected (harmonic-ex, div-transfer)
bool stabilised_transfer3(const Level3& C, const Level3& F, const Averaging3& Av, const CSR& Af, CSR& P) {
  const int nfr = 3 * F.nint;
  std::vector<std::vector<std::pair<int, double>>> rows(nfr);
  for (int r = 0; r < nfr; ++r)
    for (int t = Av.row_ptr[r]; t < Av.row_ptr[r + 1]; ++t) rows[r].push_back({Av.col[t], Av.val[t]});
  const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<char> ok(nth, 1);
  std::vector<std::thread> pool;
  for (int th = 0; th < nth; ++th)
    pool.emplace_back([&, th]() {
      std::vector<double> ATT(24 * 24), Lc(24 * 24);
      for (int T = th; T < C.nc; T += nth) {
        int tf[8], nt = 0;
        for (int q = 0; q < 8; ++q)
          if (Av.inner[8 * T + q] >= 0) tf[nt++] = Av.inner[8 * T + q];
        const int n = 3 * nt;
        if (n == 0) continue;
        std::vector<int> td(n);
        for (int q = 0; q < nt; ++q)
          for (int cc = 0; cc < 3; ++cc) td[3 * q + cc] = 3 * tf[q] + cc;
        // A_TT and the rows of A I on td
        std::vector<int> cols;
        std::vector<std::vector<std::pair<int, double>>> AI(n);
        for (int i = 0; i < n; ++i) {
          for (int j = 0; j < n; ++j) ATT[i * n + j] = 0.0;
          const int r = td[i];
          for (int t = Af.rp[r]; t < Af.rp[r + 1]; ++t) {
            const int cj = Af.ci[t];
            for (int j = 0; j < n; ++j)
              if (td[j] == cj) ATT[i * n + j] = Af.v[t];
            for (int u = Av.row_ptr[cj]; u < Av.row_ptr[cj + 1]; ++u) AI[i].push_back({Av.col[u], Af.v[t] * Av.val[u]});
          }
          for (auto& pr : AI[i]) cols.push_back(pr.first);
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        const int nc2 = (int)cols.size();
        std::vector<double> Bm((size_t)n * nc2, 0.0);
        for (int i = 0; i < n; ++i)
          for (auto& pr : AI[i]) {
            const int j = (int)(std::lower_bound(cols.begin(), cols.end(), pr.first) - cols.begin());
            Bm[(size_t)i * nc2 + j] += pr.second;
          }
        // Cholesky of A_TT and solve for all columns
        for (int j = 0; j < n; ++j) {
          double d = ATT[j * n + j];
          for (int q = 0; q < j; ++q) d -= Lc[j * n + q] * Lc[j * n + q];
          if (!(d > 0)) {
            ok[th] = 0;
            return;
          }
          Lc[j * n + j] = std::sqrt(d);
          for (int i = j + 1; i < n; ++i) {
            double s = ATT[i * n + j];
            for (int q = 0; q < j; ++q) s -= Lc[i * n + q] * Lc[j * n + q];
            Lc[i * n + j] = s / Lc[j * n + j];
          }
        }
        for (int cc = 0; cc < nc2; ++cc) {
          double y[24];
          for (int i = 0; i < n; ++i) {
            double s = Bm[(size_t)i * nc2 + cc];
            for (int q = 0; q < i; ++q) s -= Lc[i * n + q] * y[q];
            y[i] = s / Lc[i * n + i];
          }
          for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int q = i + 1; q < n; ++q) s -= Lc[q * n + i] * y[q];
            y[i] = s / Lc[i * n + i];
          }
          for (int i = 0; i < n; ++i) Bm[(size_t)i * nc2 + cc] = y[i];
        }
        for (int i = 0; i < n; ++i) {
          auto& row = rows[td[i]];
          for (int cc = 0; cc < nc2; ++cc) {
            const double v = -Bm[(size_t)i * nc2 + cc];
            bool merged = false;
            for (auto& pr : row)
              if (pr.first == cols[cc]) {
                pr.second += v;
                merged = true;
                break;
              }
            if (!merged) row.push_back({cols[cc], v});
          }
        }
      }
    });
  for (auto& t : pool) t.join();
  for (char o : ok)
    if (!o) return false;
  P.n = nfr;
  P.rp.assign(nfr + 1, 0);
  P.ci.clear();
  P.v.clear();
  for (int r = 0; r < nfr; ++r) {
    auto row = rows[r];
    std::sort(row.begin(), row.end());
    for (auto& pr : row) {
      P.ci.push_back(pr.first);
      P.v.push_back(pr.second);
    }
    P.rp[r + 1] = (int)P.ci.size();
  }
  return true;
}

void to_ell3(const CSR& A, int& w, std::vector<int>& ci, std::vector<double>& v) {
  w = 0;
  for (int r = 0; r < A.n; ++r) w = std::max(w, A.rp[r + 1] - A.rp[r]);
  ci.assign((size_t)std::max(w, 1) * A.n, 0);
  v.assign((size_t)std::max(w, 1) * A.n, 0.0);
  for (int r = 0; r < A.n; ++r)
    for (int t = A.rp[r]; t < A.rp[r + 1]; ++t) {
      ci[(size_t)(t - A.rp[r]) * A.n + r] = A.ci[t];
      v[(size_t)(t - A.rp[r]) * A.n + r] = A.v[t];
    }
}

// dense inverse of an SPD matrix (row-major in, column-major out): Cholesky,
// then the columns solved on host threads
bool invert_spd_par(const std::vector<double>& A, int n, std::vector<double>& inv) {
  std::vector<double> L(A);
  for (int j = 0; j < n; ++j) {
    double d = L[(size_t)j * n + j];
    for (int q = 0; q < j; ++q) d -= L[(size_t)j * n + q] * L[(size_t)j * n + q];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    L[(size_t)j * n + j] = d;
    const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto body = [&](int th) {
      for (int i = j + 1 + th; i < n; i += nth) {
        double s = L[(size_t)i * n + j];
        for (int q = 0; q < j; ++q) s -= L[(size_t)i * n + q] * L[(size_t)j * n + q];
        L[(size_t)i * n + j] = s / d;
      }
    };
    if (n - j > 256) {
      std::vector<std::thread> pool;
      for (int th = 0; th < nth; ++th) pool.emplace_back(body, th);
      for (auto& t : pool) t.join();
    } else {
      body(0);
      for (int th = 1; th < nth; ++th) body(th);
    }
  }
  inv.assign((size_t)n * n, 0.0);
  const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int th = 0; th < nth; ++th)
    pool.emplace_back([&, th]() {
      std::vector<double> col(n);
      for (int cc = th; cc < n; cc += nth) {
        for (int i = 0; i < n; ++i) {
          double s = i == cc ? 1.0 : 0.0;
          for (int q = 0; q < i; ++q) s -= L[(size_t)i * n + q] * col[q];
          col[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
          double s = col[i];
          for (int q = i + 1; q < n; ++q) s -= L[(size_t)q * n + i] * col[q];
          col[i] = s / L[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[(size_t)cc * n + i] = col[i];
      }
    });
  for (auto& t : pool) t.join();
  return true;
}

// ---- device levels ----------------------------------------------------------
hdgmg_status upload_level(Ctx3* c, const Level3& L, int mF, DevLev3& D) {
  D.nc = L.nc;
  D.nint = L.nint;
  D.mF = mF;
  D.nK = 12 * mF;
  D.ndof = (long)L.nint * 3 * mF;
  TRY3(upload(c, &D.X, L.X));
  TRY3(upload(c, &D.cells, L.cells));
  TRY3(upload(c, &D.cell_dofs, L.cell_dofs));
  std::vector<int> fcell(2 * (size_t)L.nint), floc(2 * (size_t)L.nint);
  std::vector<double> fdiv(2 * (size_t)L.nint), cdiv(4 * (size_t)L.nc);
  for (int fi = 0; fi < L.nint; ++fi) {
    const int f = L.int_face[fi];
    for (int s = 0; s < 2; ++s) {
      fcell[2 * fi + s] = L.face_cells[2 * f + s];
      floc[2 * fi + s] = L.face_loc[2 * f + s];
      fdiv[2 * fi + s] = L.sigma[4 * fcell[2 * fi + s] + floc[2 * fi + s]] * L.farea[f];
    }
  }
  for (int cc = 0; cc < L.nc; ++cc)
    for (int i = 0; i < 4; ++i) cdiv[4 * cc + i] = L.sigma[4 * cc + i] * L.farea[L.cell_faces[4 * cc + i]];
  TRY3(upload(c, &D.fcell, fcell));
  TRY3(upload(c, &D.floc, floc));
  TRY3(upload(c, &D.fdiv, fdiv));
  TRY3(upload(c, &D.cdiv, cdiv));
  TRY3(upload(c, &D.vol, L.vol));
  D.np = (int)L.patch_edge.size();
  D.ncol = L.ncol;
  D.colour_ptr = L.colour_ptr;
  TRY3(upload(c, &D.pf_ptr, L.pf_ptr));
  TRY3(upload(c, &D.pf, L.pf));
  TRY3(upload(c, &D.pc_ptr, L.pc_ptr));
  TRY3(upload(c, &D.pc, L.pc));
  if (mF == 1 && !D.vertex) {
    // records of the lowest-order colour phase (else the general kernel)
    const size_t npc = L.pc.size();
    std::vector<int> prec(4 * npc);
    bool ok = true;
    for (int p = 0; p < (int)L.pc_ptr.size() - 1 && ok; ++p) {
      const int f0 = L.pf_ptr[p], nf = L.pf_ptr[p + 1] - f0;
      if (nf < 1 || nf > 12 || L.pc_ptr[p + 1] - L.pc_ptr[p] > 12) ok = false;
      for (int j = L.pc_ptr[p]; j < L.pc_ptr[p + 1] && ok; ++j) {
        const int K = L.pc[j];
        int code = 15 << 4 | 15 << 8, cnt = 0, nfar = 0, dfar[2] = {0, 0};
        for (int i = 0; i < 4; ++i) {
          const int dof = L.cell_dofs[4 * K + i];
          if (dof < 0) continue;  // boundary face: x = 0 there
          int sl = -1;
          for (int q = 0; q < nf; ++q)
            if (L.pf[f0 + q] == dof) sl = q;
          if (sl < 0) {
            // an interior face outside the patch (not containing the edge)
            if (nfar == 2) {
              ok = false;
              break;
            }
            code |= i << (14 + 2 * nfar);
            dfar[nfar++] = dof;
            continue;
          }
          if (cnt == 2) {
            ok = false;
            break;
          }
          const int sd = fcell[2 * (size_t)dof] == K ? 0 : 1;
          code = (code & ~(3 << (2 * cnt)) & ~(15 << (4 + 4 * cnt))) | i << (2 * cnt) | sl << (4 + 4 * cnt) |
                 sd << (12 + cnt);
          ++cnt;
        }
        code |= nfar << 18;
        prec[4 * (size_t)j] = K;
        prec[4 * (size_t)j + 1] = code;
        prec[4 * (size_t)j + 2] = dfar[0];
        prec[4 * (size_t)j + 3] = dfar[1];
      }
    }
    if (ok && npc > 0) TRY3(upload(c, &D.prec, prec));
  }
  D.hpoff.assign(D.np + 1, 0);
  D.hns.assign(D.np, 0);
  D.ns_max = 0;
  for (int p = 0; p < D.np; ++p) {
    const long ns = (long)(L.pf_ptr[p + 1] - L.pf_ptr[p]) * 3 * mF;
    D.hns[p] = (int)ns;
    D.hpoff[p + 1] = D.hpoff[p] + ns * ns;
    D.ns_max = std::max<int>(D.ns_max, (int)ns);
  }
  D.pinv_len = D.hpoff[D.np];
  TRY3(upload(c, &D.poff, D.hpoff));
  TRY3(dalloc(c, &D.S, (size_t)std::max(L.nc, 1) * D.nK * D.nK));
  TRY3(dalloc(c, &D.pinv, (size_t)std::max<long>(D.pinv_len, 1)));
  TRY3(dalloc(c, &D.u, (size_t)std::max<long>(D.ndof, 1)));
  TRY3(dalloc(c, &D.g, (size_t)std::max<long>(D.ndof, 1)));
  TRY3(dalloc(c, &D.r, (size_t)std::max<long>(D.ndof, 1)));
  TRY3(dalloc(c, &D.yK, (size_t)std::max(L.nc, 1) * D.nK));
  // algorithmic bytes of a colour phase: per patch cell its two patch-face
  // row blocks of S_K, the patch inverse, and the vectors
  D.phase_S.assign(D.ncol, 0.0);
  D.phase_P.assign(D.ncol, 0.0);
  D.phase_V.assign(D.ncol, 0.0);
  D.phase_V0.assign(D.ncol, 0.0);
  for (int col = 0; col < D.ncol; ++col) {
    if (D.vertex) {
      // vertex patches: a full residual per colour, then the patch inverses
      D.phase_S[col] = (double)D.nc * D.nK * D.nK;
      D.phase_V[col] = 2.0 * D.nc * D.nK + 4.0 * D.ndof;
    }
    for (int p = L.colour_ptr[col]; p < L.colour_ptr[col + 1]; ++p) {
      const double ns = (double)(L.pf_ptr[p + 1] - L.pf_ptr[p]) * 3 * mF;
      const double ncl = L.pc_ptr[p + 1] - L.pc_ptr[p];
      D.phase_P[col] += ns * ns;
      D.phase_V0[col] += 3.0 * ns;
      if (D.vertex) {
        D.phase_V[col] += 3.0 * ns;
      } else {
        // direct form: per patch cell the rows of its patch faces times the
        // columns of its far faces (interior faces outside the patch)
        for (int j = L.pc_ptr[p]; j < L.pc_ptr[p + 1]; ++j) {
          const int K = L.pc[j];
          int npf = 0, nfar = 0;
          for (int i = 0; i < 4; ++i) {
            const int dof = L.cell_dofs[4 * K + i];
            if (dof < 0) continue;
            bool in = false;
            for (int q = L.pf_ptr[p]; q < L.pf_ptr[p + 1]; ++q) in = in || L.pf[q] == dof;
            if (in)
              ++npf;
            else
              ++nfar;
          }
          D.phase_S[col] += (double)npf * nfar * 9.0 * mF * mF;
        }
        D.phase_V[col] += ncl * D.nK + 3.0 * ns;
      }
    }
  }
  return HDGMG_OK;
}

template <typename TS>
Level3View<TS> view(const DevLev3& D, const TS* S) {
  Level3View<TS> v;
  v.nc = D.nc;
  v.nint = D.nint;
  v.mF = D.mF;
  v.nK = D.nK;
  v.cell_dofs = D.cell_dofs;
  v.fcell = D.fcell;
  v.floc = D.floc;
  v.S = S;
  v.al = 0.0;
  v.cdiv = D.cdiv;
  v.vol = D.vol;
  return v;
}

// the FP32 blocks hold A without its AL term, added apart in FP64
Level3View<float> view32(const Ctx3* c, const DevLev3& D) {
  Level3View<float> v = view<float>(D, D.S32);
  v.al = c->eps_inv;
  return v;
}

// vcycle_precision 1: every V-cycle operator stored FP32; 3: the same but the
// order-k edge-patch inverses kept FP64
bool f32(const Ctx3* c) { return c->opts.vcycle_precision >= 1; }
bool pinv64(const Ctx3* c, const DevLev3& D) { return c->opts.vcycle_precision == 3 && &D == &c->K; }

int kt_begin(Ctx3* c, int cls) {
  auto& T = c->timers[cls];
  if (!T.on) return -1;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1;
  }
  (void)hipEventRecord(a, c->st);
  T.ev.push_back({a, b});
  return (int)T.ev.size() - 1;
}
void kt_end(Ctx3* c, int cls, int id, double bytes) {
  if (id < 0) return;
  auto& T = c->timers[cls];
  (void)hipEventRecord(T.ev[id].second, c->st);
  T.bytes += bytes;
}
void kt_clear(Ctx3::Timer& T) {
  for (auto& e : T.ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  T.ev.clear();
  T.bytes = 0.0;
}

// y = alpha A x + b on a level (b may be null)
void level_apply(Ctx3* c, DevLev3& D, const double* x, double* y, double alpha, const double* b, bool vc) {
  if (vc && f32(c))
    launch_cell_apply3<float>(c->st, view32(c, D), x, D.yK);
  else
    launch_cell_apply3<double>(c->st, view<double>(D, D.S), x, D.yK);
  launch_face_gather3(c->st, D.nint, D.mF, D.nK, D.fcell, D.floc, D.yK, alpha, b, y);
}

void apply_k(Ctx3* c, const double* x, double* y, double alpha, const double* b, bool vc) {
  DevLev3& D = c->K;
  const int t = kt_begin(c, 1);
  level_apply(c, D, x, y, alpha, b, vc);
  kt_end(c, 1, t, (vc && f32(c) ? 4.0 : 8.0) * D.nc * (double)D.nK * D.nK + 8.0 * (2.0 * D.nc * D.nK + 2.0 * D.ndof));
}

double phase_bytes(const Ctx3* c, const DevLev3& D, int col) {
  const double bs = f32(c) ? 4.0 : 8.0, bp = f32(c) && !pinv64(c, D) ? 4.0 : 8.0;
  return D.phase_S[col] * bs + D.phase_P[col] * bp + D.phase_V[col] * 8.0;
}
// the same for an edge-patch phase from x = 0
double phase_bytes_zero(const Ctx3* c, const DevLev3& D, int col) {
  const double bp = f32(c) && !pinv64(c, D) ? 4.0 : 8.0;
  return D.phase_P[col] * bp + D.phase_V0[col] * 8.0;
}

// Damped block Jacobi sweep (eq. bjac): r = b - A x once, then every
// colour's patches add A_ss^-1 r_s / (number of colours)
void jacobi_sweep(Ctx3* c, DevLev3& D, double* x, const double* b, int cls) {
  level_apply(c, D, x, D.r, -1.0, b, true);
  const double damp = 1.0 / D.ncol;
  for (int col = 0; col < D.ncol; ++col) {
    const int p0 = D.colour_ptr[col], p1 = D.colour_ptr[col + 1];
    const int t = kt_begin(c, cls);
    if (f32(c) && !pinv64(c, D))
      launch_patch_correct<float>(c->st, D.pf_ptr, D.pf, D.poff, D.pinv32, 3 * D.mF, D.ns_max, p0, p1, D.r, x,
                                  damp);
    else
      launch_patch_correct<double>(c->st, D.pf_ptr, D.pf, D.poff, D.pinv, 3 * D.mF, D.ns_max, p0, p1, D.r, x,
                                   damp);
    kt_end(c, cls, t, phase_bytes(c, D, col));
  }
}

// x_zero: x = 0 at entry, so the first colour phase of an edge-patch
// Gauss-Seidel sweep forms its patch residuals from b alone
void sweep(Ctx3* c, DevLev3& D, double* x, const double* b, bool forward, int cls, bool x_zero = false) {
  if (c->opts.smoother == 1) {
    jacobi_sweep(c, D, x, b, cls);
    return;
  }
  if (D.vertex) {
    // vertex patches of one colour share no cell: the residual after the
    // previous colour, then every patch of the colour corrected at once
    for (int ci = 0; ci < D.ncol; ++ci) {
      const int col = forward ? ci : D.ncol - 1 - ci;
      const int p0 = D.colour_ptr[col], p1 = D.colour_ptr[col + 1];
      const int t = kt_begin(c, cls);
      level_apply(c, D, x, D.r, -1.0, b, true);
      if (f32(c) && !pinv64(c, D))
        launch_patch_correct<float>(c->st, D.pf_ptr, D.pf, D.poff, D.pinv32, 3 * D.mF, D.ns_max, p0, p1, D.r, x,
                                    1.0);
      else
        launch_patch_correct<double>(c->st, D.pf_ptr, D.pf, D.poff, D.pinv, 3 * D.mF, D.ns_max, p0, p1, D.r, x,
                                     1.0);
      kt_end(c, cls, t, phase_bytes(c, D, col));
    }
    return;
  }
  for (int ci = 0; ci < D.ncol; ++ci) {
    const int col = forward ? ci : D.ncol - 1 - ci;
    const int p0 = D.colour_ptr[col], p1 = D.colour_ptr[col + 1];
    const bool fz = x_zero && ci == 0;
    const int t = kt_begin(c, cls);
    if (D.prec && f32(c) && pinv64(c, D))
      launch_patch_gs3_lo<float, double>(c->st, view32(c, D), D.pf_ptr, D.pf, D.pc_ptr, D.prec, D.poff, D.pinv,
                                         p0, p1, x, b, fz);
    else if (D.prec && f32(c))
      launch_patch_gs3_lo<float, float>(c->st, view32(c, D), D.pf_ptr, D.pf, D.pc_ptr, D.prec, D.poff, D.pinv32,
                                        p0, p1, x, b, fz);
    else if (D.prec)
      launch_patch_gs3_lo<double, double>(c->st, view<double>(D, D.S), D.pf_ptr, D.pf, D.pc_ptr, D.prec, D.poff,
                                          D.pinv, p0, p1, x, b, fz);
    else if (f32(c) && pinv64(c, D))
      launch_patch_gs3<float, double>(c->st, view32(c, D), D.pf_ptr, D.pf, D.pc_ptr, D.pc, D.poff, D.pinv, p0,
                                      p1, x, b, fz);
    else if (f32(c))
      launch_patch_gs3<float, float>(c->st, view32(c, D), D.pf_ptr, D.pf, D.pc_ptr, D.pc, D.poff, D.pinv32, p0,
                                     p1, x, b, fz);
    else
      launch_patch_gs3<double, double>(c->st, view<double>(D, D.S), D.pf_ptr, D.pf, D.pc_ptr, D.pc, D.poff,
                                       D.pinv, p0, p1, x, b, fz);
    kt_end(c, cls, t, fz ? phase_bytes_zero(c, D, col) : phase_bytes(c, D, col));
  }
}

void ell(Ctx3* c, int n, int w, const int* ci, const double* v, const float* v32, const double* x, double* y,
         double beta_y, double* zero_out) {
  if (f32(c))
    launch_ell_spmv<float>(c->st, n, w, ci, v32, x, y, beta_y, zero_out);
  else
    launch_ell_spmv<double>(c->st, n, w, ci, v, x, y, beta_y, zero_out);
}

// Alg. 1 on lowest-order level l from the iterate in cr[l].u (zero when
// called from MG_hp), right-hand side cr[l].g
// u_zero: D.u = 0 at entry (the restriction or the caller cleared it)
void mg_h(Ctx3* c, int l, int m_l, bool u_zero) {
  DevLev3& D = c->cr[l];
  if (l == 0) {
    if (f32(c))
      launch_gemv_rows<float>(c->st, c->n0, c->ld0, c->coarse_rows32, D.g, D.u);
    else
      launch_gemv_rows<double>(c->st, c->n0, c->ld0, c->coarse_rows, D.g, D.u);
    return;
  }
  for (int s = 0; s < m_l; ++s) sweep(c, D, D.u, D.g, true, 2, u_zero && s == 0);
  level_apply(c, D, D.u, D.r, -1.0, D.g, true);
  DevTr3& T = c->tr[l];
  DevLev3& C = c->cr[l - 1];
  ell(c, T.ncoarse, T.Rw, T.Rci, T.Rv, T.Rv32, D.r, C.g, 0.0, C.u);
  for (int n = 0; n < c->opts.cycle; ++n) mg_h(c, l - 1, c->opts.vcycle_growth * m_l, n == 0);
  ell(c, T.nfine, T.Pw, T.Pci, T.Pv, T.Pv32, C.u, D.u, 1.0, nullptr);
  for (int s = 0; s < m_l; ++s) sweep(c, D, D.u, D.g, false, 2);
}

// Alg. 2 with zero initial guess: z = MG_hp(r)
void mg_hp(Ctx3* c, const double* r, double* z) {
  const int t = kt_begin(c, 3);
  DevLev3& KL = c->K;
  DevLev3& DJ = c->cr[c->J - 1];
  if (c->k == 0) {
    launch_copy(c->st, DJ.ndof, r, DJ.g);
    launch_fill(c->st, DJ.ndof, 0.0, DJ.u);
    mg_h(c, c->J - 1, c->opts.m_smooth, true);
    launch_copy(c->st, DJ.ndof, DJ.u, z);
  } else if (c->opts.additive) {
    // additive counterpart: relaxation and lowest-order correction of r
    launch_fill(c->st, KL.ndof, 0.0, z);
    for (int s = 0; s < c->opts.m_relax; ++s) sweep(c, KL, z, r, true, 0, s == 0);
    for (int s = 0; s < c->opts.m_relax; ++s) sweep(c, KL, z, r, false, 0);
    launch_mode0_extract3(c->st, KL.nint, KL.mF, r, DJ.g, DJ.u);
    mg_h(c, c->J - 1, c->opts.m_smooth, true);
    launch_mode0_add3(c->st, KL.nint, KL.mF, DJ.u, z);
  } else {
    launch_fill(c->st, KL.ndof, 0.0, z);
    for (int s = 0; s < c->opts.m_relax; ++s) sweep(c, KL, z, r, true, 0, s == 0);
    // Pi_k^0 (r - A z): only the mode-0 rows of A z
    if (f32(c))
      launch_mode0_residual3<float>(c->st, view32(c, KL), KL.S0_32, z, KL.y0K, r, DJ.g, DJ.u);
    else
      launch_mode0_residual3<double>(c->st, view<double>(KL, KL.S), KL.S0, z, KL.y0K, r, DJ.g, DJ.u);
    mg_h(c, c->J - 1, c->opts.m_smooth, true);
    launch_mode0_add3(c->st, KL.nint, KL.mF, DJ.u, z);
    for (int s = 0; s < c->opts.m_relax; ++s) sweep(c, KL, z, r, false, 0);
  }
  kt_end(c, 3, t, c->vcycle_bytes);
}

// flexible CG (Notay) for A^eps x = b from x = 0
hdgmg_status fcg3(Ctx3* c, double* sc, double* part, const double* b, double* x, int* its_out, double* rel_out) {
  const long n = c->K.ndof;
  const int NB = RED_BLOCKS;
  hipStream_t st = c->st;
  double hs[SC_N];
  launch_fill(st, n, 0.0, x);
  launch_copy(st, n, b, c->r);
  launch_dot(st, n, c->r, c->r, part, NB);
  launch_finalize(st, part, NB, 1, sc, SC_BB);
  HIPC3(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
  HIPC3(hipStreamSynchronize(st));
  const double r0 = std::sqrt(hs[SC_BB]);
  if (!std::isfinite(r0)) {
    c->err = "non-finite right-hand side";
    return HDGMG_ENONFINITE;
  }
  const double tol = std::max(c->opts.rtol * r0, c->opts.atol);
  if (its_out) *its_out = 0;
  if (rel_out) *rel_out = r0 > 0 ? 1.0 : 0.0;
  if (r0 <= tol) return HDGMG_OK;
  mg_hp(c, c->r, c->z);
  launch_dot(st, n, c->z, c->r, part, NB);
  launch_finalize(st, part, NB, 1, sc, SC_ZR);
  launch_copy(st, n, c->z, c->p);
  int it = 0;
  while (it < c->opts.max_it) {
    apply_k(c, c->p, c->q, 1.0, nullptr, false);
    launch_dot(st, n, c->p, c->q, part, NB);
    launch_finalize(st, part, NB, 1, sc, SC_PQ);
    launch_fcg_xr(st, n, x, c->r, c->r_old, c->p, c->q, sc, part, NB);
    launch_finalize(st, part, NB, 1, sc, SC_RR);
    HIPC3(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPC3(hipStreamSynchronize(st));
    ++it;
    // breakdown first: with z.r = 0 or p.Ap = 0 the step itself is 0/0
    if (hs[SC_PQ] <= 0.0 || hs[SC_ZR] <= 0.0) {
      c->err = "flexible CG breakdown (p.Ap <= 0 or z.r <= 0)";
      return HDGMG_EBREAKDOWN;
    }
    if (!std::isfinite(hs[SC_RR]) || !std::isfinite(hs[SC_PQ]) || !std::isfinite(hs[SC_ZR])) {
      c->err = "non-finite value in flexible CG";
      return HDGMG_ENONFINITE;
    }
    const double rn = std::sqrt(hs[SC_RR]);
    if (its_out) *its_out = it;
    if (rel_out) *rel_out = rn / r0;
    if (rn <= tol) return HDGMG_OK;
    mg_hp(c, c->r, c->z);
    launch_dot2(st, n, c->z, c->r, c->r_old, part, NB);
    launch_finalize(st, part, NB, 2, sc, SC_ZRN);
    launch_fcg_p(st, n, c->p, c->z, sc);
    launch_scalar_move(st, sc, SC_ZRN, SC_ZR);
  }
  c->err = "inner solve reached max_it";
  return HDGMG_NOT_CONVERGED;
}

hdgmg_status check_status(Ctx3* c, const char* what) {
  int h = 0;
  HIPC3(hipMemcpyAsync(&h, c->status, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPC3(hipStreamSynchronize(c->st));
  if (h) {
    c->err = std::string(what) + ": singular local system (status " + std::to_string(h) + ")";
    return HDGMG_ENONFINITE;
  }
  return HDGMG_OK;
}

TetCells tet_cells(Ctx3* c, const double* nu, int per_cell) {
  TetCells E;
  E.T = c->T;
  E.X = c->K.X;
  E.cells = c->K.cells;
  E.cell_dofs = c->K.cell_dofs;
  E.nu = nu;
  E.nu_per_cell = per_cell;
  E.beta = c->beta;
  E.eps_inv = c->eps_inv;
  E.k = c->k;
  E.nc = c->K.nc;
  return E;
}

// batched element kernel over all finest cells with a workspace of at most
// ~1 GiB
hdgmg_status element_pass(Ctx3* c, int mode, const double* f, const double* lam, const double* p0, double* S,
                          double* gK, double* u, double* p) {
  const long per = tet_ws_words(c->k, mode);
  const long maxb = std::max<long>(64, (1L << 27) / per);
  const int nb = (int)std::min<long>(maxb, c->K.nc);
  double* ws = nullptr;
  void* raw = raw_alloc(c, (size_t)nb * per * sizeof(double));
  if (!raw) {
    c->err = "element workspace allocation failed";
    return HDGMG_ENOMEM;
  }
  ws = static_cast<double*>(raw);
  HIPC3(hipMemsetAsync(c->status, 0, sizeof(int), c->st));
  TetCells E = tet_cells(c, c->K.nu, c->nu_fine.size() > 1);
  for (int c0 = 0; c0 < c->K.nc; c0 += nb)
    launch_tet_local(c->st, E, mode, c0, std::min(nb, c->K.nc - c0), ws, f, lam, p0, S, gK, u, p, c->status);
  hipError_t e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(c->st);
  raw_free(c, raw);
  if (e != hipSuccess || e2 != hipSuccess) {
    c->err = std::string("HIP error in the element kernel: ") + hipGetErrorString(e != hipSuccess ? e : e2);
    return HDGMG_EHIP;
  }
  return check_status(c, "element");
}

hdgmg_status patch_inverses(Ctx3* c, DevLev3& D) {
  if (D.np == 0) return HDGMG_OK;
  const long per = 2L * D.ns_max * D.ns_max;
  const int nb = (int)std::max<long>(1, std::min<long>(D.np, (1L << 27) / std::max<long>(per, 1)));
  void* raw = raw_alloc(c, (size_t)nb * per * sizeof(double));
  if (!raw) {
    c->err = "patch workspace allocation failed";
    return HDGMG_ENOMEM;
  }
  HIPC3(hipMemsetAsync(c->status, 0, sizeof(int), c->st));
  for (int p0 = 0; p0 < D.np; p0 += nb)
    launch_patch_inverse3(c->st, view<double>(D, D.S), D.pf_ptr, D.pf, D.pc_ptr, D.pc, D.poff, p0,
                          std::min(nb, D.np - p0), D.ns_max, static_cast<double*>(raw), D.pinv, c->status);
  hipError_t e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(c->st);
  raw_free(c, raw);
  if (e != hipSuccess || e2 != hipSuccess) {
    c->err = std::string("HIP error in the patch inverses: ") + hipGetErrorString(e != hipSuccess ? e : e2);
    return HDGMG_EHIP;
  }
  return check_status(c, "patch inverse");
}

hdgmg_status make_f32_level(Ctx3* c, DevLev3& D) {
  if (!D.S32) TRY3(dalloc(c, &D.S32, (size_t)std::max(D.nc, 1) * D.nK * D.nK));
  launch_f32_blocks_noal(c->st, D.nc, D.mF, D.S, D.cdiv, D.vol, c->eps_inv, D.S32);
  if (pinv64(c, D)) return HDGMG_OK;
  if (!D.pinv32) TRY3(dalloc(c, &D.pinv32, (size_t)std::max<long>(D.pinv_len, 1)));
  launch_f32_copy(c->st, D.pinv_len, D.pinv, D.pinv32);
  return HDGMG_OK;
}

}  // namespace

// ============================================================================
hdgmg_status d3_setup(const hdgmg_mesh* mesh, int k, double beta, const double* nu, int nu_len, double gamma,
                      const hdgmg_opts* opts, void* stream, hdgmg_alloc_fn alloc_fn, hdgmg_free_fn free_fn,
                      void* alloc_ctx, Ctx3** out, std::string& err) {
  *out = nullptr;
  if (k < 0 || k > K3MAX) {
    err = "tetrahedral meshes support 0 <= k <= 3";
    return HDGMG_EINVAL;
  }
  if (mesh->n_vertices < 4 || mesh->n_cells < 1 || mesh->n_refine < 0 || mesh->n_refine > 6) {
    err = "3D mesh must have >= 1 cell and 0 <= n_refine <= 6";
    return HDGMG_EMESH;
  }
  const long nfine = (long)mesh->n_cells << (3 * mesh->n_refine);
  if (nfine > (1L << 30)) {
    err = "refined mesh too large";
    return HDGMG_EMESH;
  }
  if (nu_len != 1 && nu_len != nfine) {
    err = "nu must have 1 or n_fine_cells entries";
    return HDGMG_EINVAL;
  }
  Ctx3* c = new Ctx3();
  hdgmg_default_opts(&c->opts);
  if (opts) c->opts = *opts;
  if (c->opts.vcycle_precision < 0 || c->opts.vcycle_precision > 3 || c->opts.vcycle_precision == 2) {
    err = "tetrahedral meshes: vcycle_precision must be 0 (FP64), 1 (FP32) or 3 (FP32, FP64 patch inverses)";
    delete c;
    return HDGMG_EINVAL;
  }
  if (c->opts.oseen || c->opts.transpose) {
    err = "the Oseen system is available on triangular meshes only";
    delete c;
    return HDGMG_EINVAL;
  }
  if (c->opts.smoother < 0 || c->opts.smoother > 1 || c->opts.additive < 0 || c->opts.additive > 1 ||
      c->opts.patch_relax < 0 || c->opts.patch_relax > 2 || c->opts.patch_smooth < 0 || c->opts.patch_smooth > 2) {
    err = "invalid smoother, additive or patch options";
    delete c;
    return HDGMG_EINVAL;
  }
  c->k = k;
  c->beta = beta;
  c->eps_inv = gamma;
  c->nu_fine.assign(nu, nu + nu_len);
  c->alloc_fn = alloc_fn;
  c->free_fn = free_fn;
  c->alloc_ctx = alloc_ctx;
  c->st = (hipStream_t)stream;
  if (!c->st) {
    if (hipStreamCreate(&c->own) != hipSuccess) {
      err = "hipStreamCreate failed";
      delete c;
      return HDGMG_EHIP;
    }
    c->st = c->own;
  }
  c->J = mesh->n_refine + 1;
  c->lv.resize(c->J);
  Level3& L0 = c->lv[0];
  L0.nv = mesh->n_vertices;
  L0.nc = mesh->n_cells;
  L0.X.assign(mesh->coords, mesh->coords + 3 * (size_t)L0.nv);
  L0.cells.assign(mesh->cells, mesh->cells + 4 * (size_t)L0.nc);
  std::string e = build_level3(L0);
  for (int l = 1; l < c->J && e.empty(); ++l) {
    refine3(c->lv[l - 1], c->lv[l]);
    e = build_level3(c->lv[l]);
  }
  if (!e.empty()) {
    err = "mesh: " + e;
    d3_destroy(c);
    return HDGMG_EMESH;
  }
  // patches: opts.patch_smooth on every level, opts.patch_relax on the
  // finest for the order-k relaxation (1 vertex, else edge)
  const bool vrelax = c->opts.patch_relax == 1, vsmooth = c->opts.patch_smooth == 1;
  auto patches = [&](Level3& L, bool vertex) {
    if (vertex) {
      build_vertex_patches(L);
      if (L.max_patch_faces > 48 || L.max_patch_cells > 32) {
        err = "mesh: a vertex lies in more than 48 faces or 32 cells";
        return false;
      }
    } else {
      build_edge_patches(L);
      if (L.max_patch_faces > 12 || L.max_patch_cells > 12) {
        err = "mesh: an edge lies in more than 12 faces or cells";
        return false;
      }
    }
    return true;
  };
  for (int l = 0; l < c->J; ++l)
    if (!patches(c->lv[l], l == c->J - 1 ? vrelax : vsmooth)) {
      d3_destroy(c);
      return HDGMG_EMESH;
    }
  c->av.resize(c->J);
  for (int l = 1; l < c->J; ++l) build_averaging3(c->lv[l - 1], c->lv[l], c->av[l]);
  *out = c;
  hdgmg_status s;
  auto fail = [&](hdgmg_status st) {
    err = c->err;
    d3_destroy(c);
    *out = nullptr;
    return st;
  };
  // device data
  TetTables Th;
  make_tet_tables(k, Th);
  if ((s = dalloc(c, &c->T, 1))) return fail(s);
  if (hipMemcpyAsync(c->T, &Th, sizeof(Th), hipMemcpyHostToDevice, c->st) != hipSuccess) {
    c->err = "table upload failed";
    return fail(HDGMG_EHIP);
  }
  Level3& LF = c->lv[c->J - 1];
  c->K.vertex = vrelax;
  if ((s = upload_level(c, LF, dims3(k).mF, c->K))) return fail(s);
  {
    std::vector<double> nuv(c->nu_fine);
    if ((s = upload(c, &c->K.nu, nuv))) return fail(s);
  }
  if (vrelax != vsmooth && !patches(LF, vsmooth)) {
    d3_destroy(c);
    *out = nullptr;
    return HDGMG_EMESH;
  }
  c->cr.resize(c->J);
  for (int l = 0; l < c->J; ++l) {
    c->cr[l].vertex = vsmooth;
    if ((s = upload_level(c, c->lv[l], 1, c->cr[l]))) return fail(s);
  }
  // per-level viscosities: the finest as given, coarser the mean of the eight children
  {
    std::vector<std::vector<double>> nus(c->J);
    nus[c->J - 1].assign(LF.nc, c->nu_fine[0]);
    if (c->nu_fine.size() > 1) nus[c->J - 1] = c->nu_fine;
    for (int l = c->J - 1; l > 0; --l) {
      nus[l - 1].assign(c->lv[l - 1].nc, 0.0);
      for (int cc = 0; cc < c->lv[l].nc; ++cc) nus[l - 1][c->lv[l].parent[cc]] += nus[l][cc] / 8.0;
    }
    for (int l = 0; l < c->J; ++l)
      if ((s = upload(c, &c->cr[l].nu, nus[l]))) return fail(s);
  }
  const long n = c->K.ndof, nc = LF.nc;
  for (double** v : {&c->x, &c->r, &c->r_old, &c->z, &c->p, &c->q, &c->b, &c->gvec, &c->lam})
    if ((s = dalloc(c, v, (size_t)std::max<long>(n, 1)))) return fail(s);
  if ((s = dalloc(c, &c->p0, (size_t)nc))) return fail(s);
  if ((s = dalloc(c, &c->sc, SC_N))) return fail(s);
  if ((s = dalloc(c, &c->part, 4 * RED_BLOCKS))) return fail(s);
  if ((s = dalloc(c, &c->gK, (size_t)nc * c->K.nK))) return fail(s);
  if ((s = dalloc(c, &c->statebuf, (size_t)(n + nc)))) return fail(s);
  if ((s = dalloc(c, &c->status, 1))) return fail(s);
  if (hipStreamSynchronize(c->st) != hipSuccess) {
    c->err = "upload failed";
    return fail(HDGMG_EHIP);
  }
  return HDGMG_OK;
}

void d3_destroy(Ctx3* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  for (auto& T : c->timers) kt_clear(T);
  for (void* p : c->allocs) raw_free(c, p);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

const char* d3_error(const Ctx3* c) { return c->err.c_str(); }

hdgmg_status d3_assemble(Ctx3* c) {
  c->assembled = false;
  // order-k cell blocks
  if (c->k > 0) TRY3(element_pass(c, TET_CONDENSE, nullptr, nullptr, nullptr, c->K.S, nullptr, nullptr, nullptr));
  // lowest-order levels: closed-form blocks (the order-0 level is the
  // order-k level itself when k = 0)
  std::vector<std::vector<double>> hostB(c->J);
  for (int l = 0; l < c->J; ++l) {
    DevLev3& D = c->cr[l];
    launch_cr_blocks3(c->st, D.X, D.cells, D.nc, D.nu, c->beta, c->eps_inv, D.S);
    hostB[l].resize((size_t)D.nc * 144);
    HIPC3(hipMemcpyAsync(hostB[l].data(), D.S, hostB[l].size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  }
  if (c->k == 0)
    HIPC3(hipMemcpyAsync(c->K.S, c->cr[c->J - 1].S, (size_t)c->K.nc * 144 * sizeof(double),
                         hipMemcpyDeviceToDevice, c->st));
  HIPC3(hipStreamSynchronize(c->st));
  // the host copies in dense row-major order (the device stores face row blocks)
  for (int l = 0; l < c->J; ++l) {
    std::vector<double> dense(hostB[l].size());
    for (size_t cc = 0; cc < hostB[l].size() / 144; ++cc)
      for (int r = 0; r < 12; ++r)
        for (int q = 0; q < 12; ++q) dense[cc * 144 + r * 12 + q] = hostB[l][cc * 144 + sblk(r, q, 3, 12)];
    hostB[l].swap(dense);
  }
  // patch inverses
  if (c->k > 0) TRY3(patch_inverses(c, c->K));
  for (int l = 1; l < c->J; ++l) TRY3(patch_inverses(c, c->cr[l]));
  // transfers
  c->tr.assign(c->J, DevTr3());
  double tr_bytes = 0.0;
  for (int l = 1; l < c->J; ++l) {
    CSR Af, P, R;
    assemble_csr3(c->lv[l], hostB[l], Af);
    if (!stabilised_transfer3(c->lv[l - 1], c->lv[l], c->av[l], Af, P)) {
      c->err = "singular interior block in the harmonic extension";
      return HDGMG_ENONFINITE;
    }
    csr_transpose(P, 3 * c->lv[l - 1].nint, R);
    DevTr3& T = c->tr[l];
    T.nfine = P.n;
    T.ncoarse = R.n;
    std::vector<int> ci;
    std::vector<double> v;
    to_ell3(P, T.Pw, ci, v);
    TRY3(upload(c, &T.Pci, ci));
    TRY3(upload(c, &T.Pv, v));
    tr_bytes += 12.0 * v.size();
    to_ell3(R, T.Rw, ci, v);
    TRY3(upload(c, &T.Rci, ci));
    TRY3(upload(c, &T.Rv, v));
    tr_bytes += 12.0 * v.size();
  }
  // coarsest inverse
  {
    CSR A0;
    assemble_csr3(c->lv[0], hostB[0], A0);
    const int n0 = A0.n;
    c->n0 = n0;
    std::vector<double> dense((size_t)n0 * n0, 0.0), inv;
    for (int r = 0; r < n0; ++r)
      for (int t = A0.rp[r]; t < A0.rp[r + 1]; ++t) dense[(size_t)r * n0 + A0.ci[t]] = A0.v[t];
    if (n0 > 0 && !invert_spd_par(dense, n0, inv)) {
      c->err = "coarsest operator not positive definite";
      return HDGMG_ENONFINITE;
    }
    if (!c->coarse_inv) TRY3(dalloc(c, &c->coarse_inv, (size_t)std::max(n0, 1) * std::max(n0, 1)));
    if (n0 > 0)
      HIPC3(hipMemcpyAsync(c->coarse_inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPC3(hipStreamSynchronize(c->st));
  }
  if (f32(c)) {
    if (c->k > 0) TRY3(make_f32_level(c, c->K));
    for (int l = 0; l < c->J; ++l) TRY3(make_f32_level(c, c->cr[l]));
    for (int l = 1; l < c->J; ++l) {
      DevTr3& T = c->tr[l];
      const long np_ = (long)std::max(T.Pw, 1) * T.nfine, nr_ = (long)std::max(T.Rw, 1) * T.ncoarse;
      if (!T.Pv32) TRY3(dalloc(c, &T.Pv32, (size_t)np_));
      if (!T.Rv32) TRY3(dalloc(c, &T.Rv32, (size_t)nr_));
      launch_f32_copy(c->st, np_, T.Pv, T.Pv32);
      launch_f32_copy(c->st, nr_, T.Rv, T.Rv32);
    }
    HIPC3(hipStreamSynchronize(c->st));
  }
  c->ld0 = (c->n0 + 3) / 4 * 4;
  if (f32(c)) {
    if (!c->coarse_rows32) TRY3(dalloc(c, &c->coarse_rows32, (size_t)std::max(c->n0, 1) * std::max(c->ld0, 4)));
    launch_transpose_to<float>(c->st, c->n0, c->ld0, c->coarse_inv, c->coarse_rows32);
  } else {
    if (!c->coarse_rows) TRY3(dalloc(c, &c->coarse_rows, (size_t)std::max(c->n0, 1) * std::max(c->ld0, 4)));
    launch_transpose_to<double>(c->st, c->n0, c->ld0, c->coarse_inv, c->coarse_rows);
  }
  HIPC3(hipGetLastError());
  if (c->k > 0) {
    DevLev3& D = c->K;
    const size_t n0r = (size_t)std::max(D.nc, 1) * 12 * D.nK;
    if (!D.y0K) TRY3(dalloc(c, &D.y0K, (size_t)std::max(D.nc, 1) * 12));
    if (f32(c)) {
      if (!D.S0_32) TRY3(dalloc(c, &D.S0_32, n0r));
      launch_pack_mode0_rows3<float>(c->st, D.nc, D.mF, D.S32, D.S0_32);
    } else {
      if (!D.S0) TRY3(dalloc(c, &D.S0, n0r));
      launch_pack_mode0_rows3<double>(c->st, D.nc, D.mF, D.S, D.S0);
    }
    HIPC3(hipGetLastError());
  }
  // algorithmic bytes of one V-cycle in the storage the preconditioner reads
  const double b = f32(c) ? 4.0 : 8.0;
  double vb = 0.0;
  auto level_sweep = [&](const DevLev3& D) {
    double s = 0.0;
    for (int col = 0; col < D.ncol; ++col) s += phase_bytes(c, D, col);
    return s;
  };
  auto level_res = [&](const DevLev3& D) { return b * D.nc * (double)D.nK * D.nK + 8.0 * 4.0 * D.ndof; };
  // the order-k residual: only its mode-0 rows (x_K gathered per cell, the
  // twelve rows' products written and read, b's and g0's mode-0 entries)
  auto res0 = [&](const DevLev3& D) {
    return b * D.nc * 12.0 * D.nK + 8.0 * (D.nc * (double)D.nK + 3.0 * D.nc * 12.0 + 3.0 * 3.0 * D.nint);
  };
  // the first edge-patch Gauss-Seidel phase of a level starts from zero
  auto zero_saving = [&](const DevLev3& D) {
    if (D.vertex || c->opts.smoother == 1 || D.ncol == 0) return 0.0;
    return phase_bytes(c, D, 0) - phase_bytes_zero(c, D, 0);
  };
  if (c->k > 0)
    vb += 2.0 * c->opts.m_relax * level_sweep(c->K) + (c->opts.additive ? 0.0 : res0(c->K)) - zero_saving(c->K);
  int m = c->opts.m_smooth;
  for (int l = c->J - 1; l >= 1; --l) {
    vb += 2.0 * m * level_sweep(c->cr[l]) + level_res(c->cr[l]) - zero_saving(c->cr[l]);
    m *= c->opts.vcycle_growth;
  }
  vb += tr_bytes * b / 8.0 + b * (double)c->n0 * c->n0;
  c->vcycle_bytes = vb;
  // compulsory bytes: every stored operator read once per use in packed
  // symmetric form (cell blocks nK(nK+1)/2 words, patch inverses
  // ns(ns+1)/2, the coarsest inverse n0(n0+1)/2), plus the vectors
  auto tri = [](double n) { return n * (n + 1.0) / 2.0; };
  auto sweep_c = [&](const DevLev3& D) {
    double pb = 0.0;
    for (int q = 0; q < D.np; ++q) pb += tri((double)D.hns[q]);
    return D.nc * tri(D.nK) * b + pb * (pinv64(c, D) ? 8.0 : b) + 3.0 * 8.0 * D.ndof;
  };
  auto res_c = [&](const DevLev3& D) { return D.nc * tri(D.nK) * b + 3.0 * 8.0 * D.ndof; };
  // the order-k residual enters MG_hp only through its mode-0 rows
  auto res0_c = [&](const DevLev3& D) { return D.nc * 12.0 * D.nK * b + 3.0 * 8.0 * 3.0 * D.nint; };
  double vc = 0.0;
  if (c->k > 0) vc += 2.0 * c->opts.m_relax * sweep_c(c->K) + (c->opts.additive ? 0.0 : res0_c(c->K));
  double vis = 1.0, ml = c->opts.m_smooth;
  for (int l = c->J - 1; l >= 1; --l) {
    vc += vis * (2.0 * ml * sweep_c(c->cr[l]) + res_c(c->cr[l]));
    vis *= c->opts.cycle;
    ml *= c->opts.vcycle_growth;
  }
  vc += tr_bytes * b / 8.0 + vis * tri((double)c->n0) * b;
  c->vcycle_compulsory = vc;
  c->assembled = true;
  return HDGMG_OK;
}

hdgmg_status d3_rhs(Ctx3* c, const double* f_qp, double* g) {
  if (!c->assembled) {
    c->err = "hdgmg_rhs before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  TRY3(element_pass(c, TET_LOAD, f_qp, nullptr, nullptr, nullptr, c->gK, nullptr, nullptr));
  DevLev3& D = c->K;
  launch_face_gather3(c->st, D.nint, D.mF, D.nK, D.fcell, D.floc, c->gK, 1.0, nullptr, g);
  HIPC3(hipGetLastError());
  HIPC3(hipStreamSynchronize(c->st));
  return HDGMG_OK;
}

hdgmg_status d3_apply(Ctx3* c, const double* x, double* y) {
  if (!c->assembled) {
    c->err = "hdgmg_apply before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  apply_k(c, x, y, 1.0, nullptr, false);
  HIPC3(hipGetLastError());
  HIPC3(hipStreamSynchronize(c->st));
  return HDGMG_OK;
}

hdgmg_status d3_precondition(Ctx3* c, const double* r, double* z) {
  if (!c->assembled) {
    c->err = "hdgmg_precondition before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  mg_hp(c, r, z);
  HIPC3(hipGetLastError());
  HIPC3(hipStreamSynchronize(c->st));
  return HDGMG_OK;
}

hdgmg_status d3_inner_solve(Ctx3* c, const double* b, double* x, int* its, double* rel_res, double* sc,
                            double* part) {
  if (!c->assembled) {
    c->err = "hdgmg_inner_solve before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  hdgmg_status s = fcg3(c, sc ? sc : c->sc, part ? part : c->part, b, x, its, rel_res);
  HIPC3(hipStreamSynchronize(c->st));
  return s;
}

hdgmg_status d3_recover(Ctx3* c, const double* f_qp, const double* state, double* u_qp, double* p_qp) {
  if (!c->assembled) {
    c->err = "hdgmg_recover before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  return element_pass(c, TET_RECOVER, f_qp, state, state + c->K.ndof, nullptr, nullptr, u_qp, p_qp);
}

hdgmg_status d3_solve(Ctx3* c, const double* f_qp, const double* x0, double* u_qp, double* p_qp, double* state,
                      hdgmg_info* info) {
  if (!c->assembled) {
    c->err = "hdgmg_solve before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = c->st;
  const DevLev3& KL = c->K;
  (void)x0;
  launch_fill(st, KL.nc, 0.0, c->p0);
  TRY3(d3_rhs(c, f_qp, c->gvec));
  hdgmg_status result = HDGMG_OK;
  for (int n = 0; n < c->opts.uzawa_max; ++n) {
    launch_uzawa_rhs3(st, KL.nint, KL.mF, c->gvec, KL.fdiv, KL.fcell, c->p0, c->b);
    int its = 0;
    double rel = 0.0;
    hdgmg_status s = fcg3(c, c->sc, c->part, c->b, c->lam, &its, &rel);
    if (s < 0) return s;
    if (s == HDGMG_NOT_CONVERGED) result = s;
    launch_uzawa_update3(st, KL.nc, KL.mF, KL.cell_dofs, KL.cdiv, KL.vol, c->lam, c->eps_inv, c->p0, c->part,
                         RED_BLOCKS);
    launch_finalize(st, c->part, RED_BLOCKS, 2, c->sc, SC_DP);
    double hs[SC_N];
    HIPC3(hipMemcpyAsync(hs, c->sc, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPC3(hipStreamSynchronize(st));
    const double dn = std::sqrt(hs[SC_DP]), pn = std::sqrt(hs[SC_PP]);
    if (info) {
      info->uzawa_steps = n + 1;
      info->its[n] = its;
      info->rel_res[n] = rel;
      info->dp_l2[n] = dn;
      info->div_l2 = dn / c->eps_inv;
    }
    if (dn <= c->opts.uzawa_tol * std::max(1.0, pn)) break;
    if (n == c->opts.uzawa_max - 1 && c->opts.uzawa_tol >= 0) {
      result = HDGMG_NOT_CONVERGED;
      c->err = "AL-Uzawa reached uzawa_max";
    }
  }
  double* stt = state ? state : c->statebuf;
  launch_copy(st, KL.ndof, c->lam, stt);
  launch_copy(st, KL.nc, c->p0, stt + KL.ndof);
  TRY3(d3_recover(c, f_qp, stt, u_qp, p_qp));
  HIPC3(hipStreamSynchronize(st));
  if (info) info->t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return result;
}

hdgmg_status d3_query(const Ctx3* c, int what, int level, int64_t* value) {
  const Level3& LF = c->lv[c->J - 1];
  switch (what) {
    case 0: *value = LF.nc; return HDGMG_OK;
    case 1: *value = (int64_t)(c->k + 2) * (c->k + 2) * (c->k + 2); return HDGMG_OK;
    case 2: *value = c->K.ndof; return HDGMG_OK;
    case 3: *value = c->J; return HDGMG_OK;
    case 4: {
      *value = 0;
      return HDGMG_OK;
    }
    case 5: *value = LF.nint; return HDGMG_OK;
    case 6: *value = c->k; return HDGMG_OK;
    case 7: *value = c->K.ncol; return HDGMG_OK;
    case 8:
    case 9:
      if (level < 0 || level >= c->J) return HDGMG_EINVAL;
      *value = what == 8 ? c->lv[level].nc : 3L * c->lv[level].nint;
      return HDGMG_OK;
    case 10: *value = LF.nf - LF.nint; return HDGMG_OK;
    case 11: *value = 3; return HDGMG_OK;
    case 12: *value = (int64_t)c->vcycle_bytes; return HDGMG_OK;
    case 13: *value = (int64_t)c->vcycle_compulsory; return HDGMG_OK;
    default: return HDGMG_EINVAL;
  }
}

hdgmg_status d3_export(const Ctx3* c, int what, int level, void* dst, size_t bytes) {
  Ctx3* cc = const_cast<Ctx3*>(c);
  if (!c->assembled && (what == 0 || what == 1)) {
    cc->err = "export before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  const void* src = nullptr;
  size_t n = 0;
  if (what == 0) {
    src = c->K.S;
    n = (size_t)c->K.nc * c->K.nK * c->K.nK * sizeof(double);
  } else if (what == 1) {
    if (level < 0 || level >= c->J) return HDGMG_EINVAL;
    src = c->cr[level].S;
    n = (size_t)c->cr[level].nc * 144 * sizeof(double);
  } else {
    cc->err = "export: only cell blocks (what 0, 1) on tetrahedral meshes";
    return HDGMG_EINVAL;
  }
  if (bytes < n) return HDGMG_EINVAL;
  // dense [nc][nK][nK] from the face-row-block storage
  const DevLev3& D = what == 0 ? c->K : c->cr[level];
  launch_blocks_to_dense(c->st, D.nc, 3 * D.mF, static_cast<const double*>(src), static_cast<double*>(dst));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) {
    cc->err = std::string("HIP error: ") + hipGetErrorString(e);
    return HDGMG_EHIP;
  }
  return HDGMG_OK;
}

hdgmg_status d3_kernel_timer(Ctx3* c, int cls, int enable) {
  if (cls < 0 || cls > 4) return HDGMG_EINVAL;
  HIPC3(hipStreamSynchronize(c->st));
  kt_clear(c->timers[cls]);
  c->timers[cls].on = enable != 0;
  return HDGMG_OK;
}

hdgmg_status d3_kernel_timer_read(Ctx3* c, int cls, double* total_ms, int64_t* launches, double* bytes) {
  if (cls < 0 || cls > 4) return HDGMG_EINVAL;
  HIPC3(hipStreamSynchronize(c->st));
  auto& T = c->timers[cls];
  double tot = 0.0;
  for (auto& e : T.ev) {
    float ms = 0.0f;
    HIPC3(hipEventElapsedTime(&ms, e.first, e.second));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)T.ev.size();
  if (bytes) *bytes = T.bytes;
  return HDGMG_OK;
}

}  // namespace hdgmg
