// Per-cell local solver of the H(div)-HDG scheme and the closed-form
// lowest-order cell block.  Callable from device kernels (one thread per
// cell) and from host code (transfer construction).
//
// Order-k cell (scheme stWeak, Sec. 3.2).  With Lift(u, uhat) the [P^k]^{2x2}
// function defined by (Lift, G) = (grad u, G) - <tng(u - uhat), G n_K>, the
// cell energy is 1/2 [nu |Lift|^2 + beta |u|^2] - (f, u).  For given skeleton
// data lambda = (c^n, c^t) the interior minimises it over u in RT_k(K) with
//   N a = c^n          (normal trace moments against the facet Legendre basis)
//   D a = 0            (div u orthogonal to mean-free P^k: div u in P^0)
// which is the saddle point
//   [H_aa N^T D^T] [a]   [F - H_at c^t]
//   [N    0   0  ] [mu] = [c^n        ]
//   [D    0   0  ] [pi]   [0          ]      (KKT, pivoted LU).
// By the envelope theorem the condensed block is
//   S = blockdiag(0, H_tt) - B^T KKT^-1 B,  B = [[0, -H_at], [I, 0], [0, 0]]
// (columns c^n, c^t), the load is g = B^T KKT^-1 [F; 0; 0], and the interior
// pressure is p^o = -sum_r pi_r (q_r - mean q_r)  (stationarity in the
// interior bubbles).  The AL term eps^-1 |K|^-1 d d^T of stALform is added
// to S, with d = sigma_{K,F} |F| on each mode-0 normal coefficient.
//
// Basis: monomials xi^alpha of the reference coordinates of the affine map
// from the cell's vertices sorted by global index; RT_k = [P^k]^2 +
// (x - x_0)/h * {degree-k monomials}.  Quadrature: the data rule (exact to
// degree 2k+3) and Gauss-Legendre with k+2 points on the facets.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace hdgmg {

#define HDI __host__ __device__ inline

constexpr int KMAX = 4;
constexpr int NQ_MAX = (KMAX + 2) * (KMAX + 2);
constexpr int NF_MAX = KMAX + 2;

// Reference quadrature tables, passed to kernels by value.
struct QuadTables {
  int k, nq, nfq;
  double xi[NQ_MAX][2];  // Stroud points on the reference triangle
  double wq[NQ_MAX];     // weights, sum 1
  double s[NF_MAX];      // Gauss-Legendre points on [0,1]
  double ws[NF_MAX];     // weights, sum 1
};

// Rules of the convection terms (Sec. 4.1) for a discrete wind in RT_k:
// the volume and facet integrands have degree 3k+2, so the Stroud rule and
// Gauss-Legendre with n = floor((3k+4)/2) points per direction are exact.
// The upwind switch is taken at the facet points.  Kept in device memory
// (passed by pointer).
constexpr int NC_MAX = (3 * KMAX + 4) / 2;
struct ConvTables {
  int n, nq;
  double xi[NC_MAX * NC_MAX][2];
  double wq[NC_MAX * NC_MAX];  // sum 1
  double s[NC_MAX];
  double ws[NC_MAX];           // sum 1
};

struct Dims {
  int k, m, nP, na, nz, nK, nN, nD, nkkt, ntop;
};

HDI Dims dims_of(int k) {
  Dims d;
  d.k = k;
  d.m = k + 1;
  d.nP = (k + 1) * (k + 2) / 2;
  d.ntop = k + 1;
  d.na = 2 * d.nP + d.ntop;
  d.nz = d.na + 3 * d.m;
  d.nK = 6 * d.m;
  d.nN = 3 * d.m;
  d.nD = d.nP - 1;
  d.nkkt = d.na + d.nN + d.nD;
  return d;
}

// Strided view into a workspace shared by a batch of cells (one cell per
// thread, element i of cell t at p[i * s + t]): coalesced across a wavefront.
struct WS {
  double* p;
  long s;
  HDI double& operator[](long i) const { return p[i * s]; }
};

// Monomials xi1^a xi2^b, ordered by degree d then by b = 0..d; values and
// reference derivatives.
HDI void monomials(int k, double x1, double x2, double* v, double* d1, double* d2) {
  double p1[KMAX + 2], p2[KMAX + 2];
  p1[0] = p2[0] = 1.0;
  for (int i = 1; i <= k; ++i) {
    p1[i] = p1[i - 1] * x1;
    p2[i] = p2[i - 1] * x2;
  }
  int r = 0;
  for (int d = 0; d <= k; ++d)
    for (int b = 0; b <= d; ++b, ++r) {
      int a = d - b;
      v[r] = p1[a] * p2[b];
      d1[r] = a > 0 ? a * p1[a - 1] * p2[b] : 0.0;
      d2[r] = b > 0 ? b * p1[a] * p2[b - 1] : 0.0;
    }
}

// Orthonormal facet functions sqrt(2j+1) P_j(2s-1), j = 0..k.
HDI void facet_legendre(int k, double s, double* phi) {
  double t = 2.0 * s - 1.0;
  double pm = 1.0, p = t;
  phi[0] = 1.0;
  if (k >= 1) phi[1] = sqrt(3.0) * t;
  for (int j = 2; j <= k; ++j) {
    double pn = ((2 * j - 1) * t * p - (j - 1) * pm) / j;
    pm = p;
    p = pn;
    phi[j] = sqrt(2.0 * j + 1.0) * pn;
  }
}

// Geometry of one cell.
struct CellGeom {
  double X[3][2];     // stored vertex order
  int vid[3];
  double Xs0[2];      // sorted-vertex map x = Xs0 + J xi
  double J[2][2], Ji[2][2];
  double area, h;
  // local facet i (opposite stored vertex i)
  double P0[3][2], P1[3][2];  // endpoints in global order (v0 < v1)
  double t[3][2], n[3][2], len[3];
  int sigma[3];
};

HDI void cell_geom(const double* Xall, const int* cell, CellGeom& g) {
  for (int i = 0; i < 3; ++i) {
    g.vid[i] = cell[i];
    g.X[i][0] = Xall[2 * cell[i]];
    g.X[i][1] = Xall[2 * cell[i] + 1];
  }
  int o[3] = {0, 1, 2};
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (g.vid[o[b]] < g.vid[o[a]]) {
        int t = o[a];
        o[a] = o[b];
        o[b] = t;
      }
  g.Xs0[0] = g.X[o[0]][0];
  g.Xs0[1] = g.X[o[0]][1];
  for (int r = 0; r < 2; ++r) {
    g.J[r][0] = g.X[o[1]][r] - g.Xs0[r];
    g.J[r][1] = g.X[o[2]][r] - g.Xs0[r];
  }
  double det = g.J[0][0] * g.J[1][1] - g.J[0][1] * g.J[1][0];
  g.Ji[0][0] = g.J[1][1] / det;
  g.Ji[0][1] = -g.J[0][1] / det;
  g.Ji[1][0] = -g.J[1][0] / det;
  g.Ji[1][1] = g.J[0][0] / det;
  g.area = 0.5 * fabs(det);
  g.h = sqrt(2.0 * g.area);
  for (int i = 0; i < 3; ++i) {
    int a = (i + 1) % 3, b = (i + 2) % 3;
    if (g.vid[b] < g.vid[a]) {
      int t = a;
      a = b;
      b = t;
    }
    double dx = g.X[b][0] - g.X[a][0], dy = g.X[b][1] - g.X[a][1];
    double l = sqrt(dx * dx + dy * dy);
    g.len[i] = l;
    g.P0[i][0] = g.X[a][0];
    g.P0[i][1] = g.X[a][1];
    g.P1[i][0] = g.X[b][0];
    g.P1[i][1] = g.X[b][1];
    g.t[i][0] = dx / l;
    g.t[i][1] = dy / l;
    g.n[i][0] = dy / l;
    g.n[i][1] = -dx / l;
    double mx = 0.5 * (g.X[a][0] + g.X[b][0]) - g.X[i][0];
    double my = 0.5 * (g.X[a][1] + g.X[b][1]) - g.X[i][1];
    g.sigma[i] = (mx * g.n[i][0] + my * g.n[i][1]) > 0 ? 1 : -1;
  }
}

// RT_k basis at a point: values u[a][i], gradients gr[a][i][j] = du_i/dx_j.
HDI void rt_basis(const Dims& D, const CellGeom& g, double x1, double x2, const double* xphys,
                  double* u, double* gr, double* mono) {
  double v[16], d1[16], d2[16];
  monomials(D.k, x1, x2, v, d1, d2);
  for (int r = 0; r < D.nP; ++r) mono[r] = v[r];
  for (int r = 0; r < D.nP; ++r) {
    double gx = d1[r] * g.Ji[0][0] + d2[r] * g.Ji[1][0];
    double gy = d1[r] * g.Ji[0][1] + d2[r] * g.Ji[1][1];
    int a0 = 2 * r, a1 = 2 * r + 1;
    u[2 * a0] = v[r];
    u[2 * a0 + 1] = 0.0;
    u[2 * a1] = 0.0;
    u[2 * a1 + 1] = v[r];
    gr[4 * a0 + 0] = gx;
    gr[4 * a0 + 1] = gy;
    gr[4 * a0 + 2] = 0.0;
    gr[4 * a0 + 3] = 0.0;
    gr[4 * a1 + 0] = 0.0;
    gr[4 * a1 + 1] = 0.0;
    gr[4 * a1 + 2] = gx;
    gr[4 * a1 + 3] = gy;
  }
  double y0 = (xphys[0] - g.Xs0[0]) / g.h, y1 = (xphys[1] - g.Xs0[1]) / g.h;
  for (int t = 0; t < D.ntop; ++t) {
    int r = D.nP - D.ntop + t;
    int a = 2 * D.nP + t;
    double gx = d1[r] * g.Ji[0][0] + d2[r] * g.Ji[1][0];
    double gy = d1[r] * g.Ji[0][1] + d2[r] * g.Ji[1][1];
    u[2 * a] = y0 * v[r];
    u[2 * a + 1] = y1 * v[r];
    gr[4 * a + 0] = v[r] / g.h + y0 * gx;
    gr[4 * a + 1] = y0 * gy;
    gr[4 * a + 2] = y1 * gx;
    gr[4 * a + 3] = v[r] / g.h + y1 * gy;
  }
}

// Workspace size (doubles per cell) for order k.
HDI long element_ws_size(int k) {
  Dims D = dims_of(k);
  long n = 0;
  n += D.nP * D.nP;             // M
  n += 4L * D.nP * D.nz;        // R
  n += (long)D.nP * D.nz;       // Y
  n += (long)D.nz * D.nz;       // H
  n += (long)D.nN * D.na;       // N
  n += (long)D.nP * D.na;       // Dr
  n += 2L * D.na;               // F (two loads for EL_GRADNU)
  n += (long)D.nkkt * D.nkkt;   // KKT
  n += D.nkkt;                  // pivots
  n += (long)D.nkkt * D.nK;     // right-hand sides / solutions
  n += D.nP;                    // means
  return n;
}

enum { EL_CONDENSE = 0, EL_LOAD = 1, EL_RECOVER = 2, EL_GRADNU = 3, EL_POSTPROCESS = 4 };

// The local solve of one cell.  Returns 0 on success, 1 if the KKT matrix
// is singular.  Inputs/outputs by mode:
//   EL_CONDENSE: out = S^eps [nK][nK] (row-major)
//   EL_LOAD:     f [nq][2] at the data points; out = g [nK]
//   EL_RECOVER:  f, lam [nK], p0; out = u [nq][2] then p [nq]
//   EL_POSTPROCESS: f, lam [nK]; out = u* [nq][2] at the data points, the
//                local post-processing (stPost): u* in [P^{k+1}]^2 with
//                (grad u*_i, grad v) = (Lift_i., grad v) for v in P^{k+1}
//                and the cell mean of u_h (Lift = -L_h / nu)
//   EL_GRADNU:   two local states, (f, lam) and (f2, lam2); out[0] =
//                -(Lift(z), Lift(z2))_K, the derivative with respect to this
//                cell's viscosity of the adjoint-weighted residual (the only
//                nu-dependent term of the element energy is nu ||Lift||^2)
// With a wind (CT and wc non-null; wc = the wind's coefficients in this
// cell's RT_k basis) the element matrix gains the Picard convection form of
// Sec. 4.1 (test v, trial u):
//   - sum_ij (u_i w_j, d_j v_i)_K + <(w.n_K) t(u_up), t(v) - vhat>_{dK},
// with u_up the cell's own trace where w.n_K > 0 and uhat where w.n_K < 0;
// the volume terms then use the convection rule and the source term the
// data rule.  H is nonsymmetric; rows are test functions, so the condensed
// rows of tangential unknowns read H_ta (rows), not H_at^T, and S is not
// symmetrised.  transpose: the cell of the transposed (adjoint) system, H
// replaced by H^T before the local solve (only the convection part is
// nonsymmetric); the condensed block is then S^T and the load, recovery and
// kept factors are those of the transposed local system.  EL_GRADNU ignores
// it: with a wind it recovers (f, lam) with the forward local system and
// (f2, lam2) with the transposed one (the forward and adjoint states).
HDI int element_local(const QuadTables& Q, const CellGeom& g, double nu, double beta,
                      double eps_inv, int mode, const double* f, const double* lam,
                      double p0, WS w, double* out, const double* f2 = nullptr,
                      const double* lam2 = nullptr, const ConvTables* CT = nullptr,
                      const double* wc = nullptr, const WS* fac = nullptr, bool transpose = false,
                      int oflags = 0) {
  const Dims D = dims_of(Q.k);
  const int nP = D.nP, na = D.na, nz = D.nz, m = D.m, nK = D.nK, nN = D.nN, nkkt = D.nkkt;
  long o = 0;
  WS M{w.p + o * w.s, w.s};
  o += nP * nP;
  WS R{w.p + o * w.s, w.s};
  o += 4L * nP * nz;
  WS Y{w.p + o * w.s, w.s};
  o += (long)nP * nz;
  WS H{w.p + o * w.s, w.s};
  o += (long)nz * nz;
  WS Nm{w.p + o * w.s, w.s};
  o += (long)nN * na;
  WS Dr{w.p + o * w.s, w.s};
  o += (long)nP * na;
  WS F{w.p + o * w.s, w.s};
  o += 2L * na;
  WS Kk{w.p + o * w.s, w.s};
  o += (long)nkkt * nkkt;
  WS piv{w.p + o * w.s, w.s};
  o += nkkt;
  WS Bx{w.p + o * w.s, w.s};
  o += (long)nkkt * nK;
  WS mean{w.p + o * w.s, w.s};

  for (long i = 0; i < (long)nP * nP; ++i) M[i] = 0.0;
  for (long i = 0; i < 4L * nP * nz; ++i) R[i] = 0.0;
  for (long i = 0; i < (long)nz * nz; ++i) H[i] = 0.0;
  for (long i = 0; i < (long)nN * na; ++i) Nm[i] = 0.0;
  for (long i = 0; i < (long)nP * na; ++i) Dr[i] = 0.0;
  for (int i = 0; i < 2 * na; ++i) F[i] = 0.0;
  for (int i = 0; i < nP; ++i) mean[i] = 0.0;

  double u[2 * 40], gr[4 * 40], mono[16];
  const bool conv = CT != nullptr && wc != nullptr;
  // ---- volume terms (the source term inline only with the data rule)
  const int nvq = conv ? CT->nq : Q.nq;
  for (int q = 0; q < nvq; ++q) {
    double x1 = conv ? CT->xi[q][0] : Q.xi[q][0], x2 = conv ? CT->xi[q][1] : Q.xi[q][1];
    double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2,
                    g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
    double wt = (conv ? CT->wq[q] : Q.wq[q]) * g.area;
    rt_basis(D, g, x1, x2, xp, u, gr, mono);
    for (int r = 0; r < nP; ++r) {
      mean[r] += wt * mono[r];
      for (int s = 0; s < nP; ++s) M[r * nP + s] += wt * mono[r] * mono[s];
    }
    for (int a = 0; a < na; ++a) {
      double dv = gr[4 * a + 0] + gr[4 * a + 3];
      for (int r = 0; r < nP; ++r) {
        double wm = wt * mono[r];
        for (int ij = 0; ij < 4; ++ij) R[((long)ij * nP + r) * nz + a] += wm * gr[4 * a + ij];
        Dr[(long)r * na + a] += wm * dv;
      }
      for (int b = 0; b <= a; ++b)
        H[(long)a * nz + b] += beta * wt * (u[2 * a] * u[2 * b] + u[2 * a + 1] * u[2 * b + 1]);
      if (!conv && mode != EL_CONDENSE) F[a] += wt * (f[2 * q] * u[2 * a] + f[2 * q + 1] * u[2 * a + 1]);
      if (!conv && mode == EL_GRADNU) F[na + a] += wt * (f2[2 * q] * u[2 * a] + f2[2 * q + 1] * u[2 * a + 1]);
    }
  }
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < a; ++b) H[(long)b * nz + a] = H[(long)a * nz + b];
  if (conv) {
    // source term with the data rule
    if (mode != EL_CONDENSE)
      for (int q = 0; q < Q.nq; ++q) {
        double x1 = Q.xi[q][0], x2 = Q.xi[q][1];
        double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2,
                        g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
        double wt = Q.wq[q] * g.area;
        rt_basis(D, g, x1, x2, xp, u, gr, mono);
        for (int a = 0; a < na; ++a) F[a] += wt * (f[2 * q] * u[2 * a] + f[2 * q + 1] * u[2 * a + 1]);
        if (mode == EL_GRADNU)
          for (int a = 0; a < na; ++a) F[na + a] += wt * (f2[2 * q] * u[2 * a] + f2[2 * q + 1] * u[2 * a + 1]);
      }
    // - sum_ij (u_i w_j, d_j v_i): H[test b][trial a]
    for (int q = 0; q < CT->nq; ++q) {
      double x1 = CT->xi[q][0], x2 = CT->xi[q][1];
      double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2,
                      g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
      double wt = CT->wq[q] * g.area;
      rt_basis(D, g, x1, x2, xp, u, gr, mono);
      double wx = 0.0, wy = 0.0;
      for (int c = 0; c < na; ++c) {
        wx += wc[c] * u[2 * c];
        wy += wc[c] * u[2 * c + 1];
      }
      for (int b = 0; b < na; ++b) {
        const double g0 = wt * (wx * gr[4 * b + 0] + wy * gr[4 * b + 1]);  // w . grad v_b,0
        const double g1 = wt * (wx * gr[4 * b + 2] + wy * gr[4 * b + 3]);  // w . grad v_b,1
        for (int a = 0; a < na; ++a) H[(long)b * nz + a] -= g0 * u[2 * a] + g1 * u[2 * a + 1];
      }
    }
  }
  for (int r = 0; r < nP; ++r) mean[r] /= g.area;
  // ---- facet terms
  double phi[KMAX + 1];
  for (int i = 0; i < 3; ++i) {
    const double* t = g.t[i];
    double nK_[2] = {g.sigma[i] * g.n[i][0], g.sigma[i] * g.n[i][1]};
    for (int l = 0; l < Q.nfq; ++l) {
      double s = Q.s[l];
      double xp[2] = {g.P0[i][0] + s * (g.P1[i][0] - g.P0[i][0]),
                      g.P0[i][1] + s * (g.P1[i][1] - g.P0[i][1])};
      double dx = xp[0] - g.Xs0[0], dy = xp[1] - g.Xs0[1];
      double x1 = g.Ji[0][0] * dx + g.Ji[0][1] * dy;
      double x2 = g.Ji[1][0] * dx + g.Ji[1][1] * dy;
      rt_basis(D, g, x1, x2, xp, u, gr, mono);
      facet_legendre(D.k, s, phi);
      double wl = Q.ws[l] * g.len[i];
      for (int r = 0; r < nP; ++r) {
        for (int ii = 0; ii < 2; ++ii)
          for (int jj = 0; jj < 2; ++jj) {
            double c = wl * mono[r] * t[ii] * nK_[jj];
            long row = ((long)(ii * 2 + jj) * nP + r) * nz;
            for (int a = 0; a < na; ++a) R[row + a] -= c * (u[2 * a] * t[0] + u[2 * a + 1] * t[1]);
            for (int j = 0; j < m; ++j) R[row + na + i * m + j] += c * phi[j];
          }
      }
      for (int j = 0; j < m; ++j)
        for (int a = 0; a < na; ++a)
          Nm[(long)(i * m + j) * na + a] +=
              Q.ws[l] * phi[j] * (u[2 * a] * g.n[i][0] + u[2 * a + 1] * g.n[i][1]);
    }
  }
  // ---- convection facet terms: <(w.n_K) t(u_up), t(v) - vhat>
  if (conv) {
    for (int i = 0; i < 3; ++i) {
      const double* t = g.t[i];
      double nK_[2] = {g.sigma[i] * g.n[i][0], g.sigma[i] * g.n[i][1]};
      for (int l = 0; l < CT->n; ++l) {
        double s = CT->s[l];
        double xp[2] = {g.P0[i][0] + s * (g.P1[i][0] - g.P0[i][0]),
                        g.P0[i][1] + s * (g.P1[i][1] - g.P0[i][1])};
        double dx = xp[0] - g.Xs0[0], dy = xp[1] - g.Xs0[1];
        double x1 = g.Ji[0][0] * dx + g.Ji[0][1] * dy;
        double x2 = g.Ji[1][0] * dx + g.Ji[1][1] * dy;
        rt_basis(D, g, x1, x2, xp, u, gr, mono);
        facet_legendre(D.k, s, phi);
        double wn = 0.0;
        for (int c = 0; c < na; ++c) wn += wc[c] * (u[2 * c] * nK_[0] + u[2 * c + 1] * nK_[1]);
        if (wn == 0.0) continue;
        const double cw = CT->ws[l] * g.len[i] * wn;
        // test rows: RT coefficients (v.t) and this facet's uhat modes (-phi)
        for (int b = 0; b < nz; ++b) {
          double tv;
          if (b < na)
            tv = u[2 * b] * t[0] + u[2 * b + 1] * t[1];
          else if (b >= na + i * m && b < na + (i + 1) * m)
            tv = -phi[b - na - i * m];
          else
            continue;
          tv *= cw;
          if (wn > 0.0) {
            for (int a = 0; a < na; ++a) H[(long)b * nz + a] += tv * (u[2 * a] * t[0] + u[2 * a + 1] * t[1]);
          } else {
            for (int j = 0; j < m; ++j) H[(long)b * nz + na + i * m + j] += tv * phi[j];
          }
        }
        if ((oflags >> i) & 1) {
          // do-nothing facet: + <(w.n_K) u, vhat>, the tangential part on the
          // facet unknowns' rows, the normal part on the cell's normal
          // trace, so that the natural condition is (nu grad u - p I) n = 0
          for (int a = 0; a < na; ++a) {
            const double ut = u[2 * a] * t[0] + u[2 * a + 1] * t[1];
            const double un = u[2 * a] * nK_[0] + u[2 * a + 1] * nK_[1];
            for (int j = 0; j < m; ++j) H[(long)(na + i * m + j) * nz + a] += cw * phi[j] * ut;
            for (int b = 0; b < na; ++b) H[(long)b * nz + a] += cw * (u[2 * b] * nK_[0] + u[2 * b + 1] * nK_[1]) * un;
          }
        }
      }
    }
  }
  if (conv && transpose && mode != EL_GRADNU)
    for (int a = 0; a < nz; ++a)
      for (int b = 0; b < a; ++b) {
        const double t = H[(long)a * nz + b];
        H[(long)a * nz + b] = H[(long)b * nz + a];
        H[(long)b * nz + a] = t;
      }
  // the second state of EL_GRADNU is solved with the transposed local system
  const bool tcol = conv && mode == EL_GRADNU;
  // ---- H += nu sum_ij R_ij^T M^-1 R_ij (Cholesky of M)
  for (int j = 0; j < nP; ++j) {
    double d = M[j * nP + j];
    for (int p = 0; p < j; ++p) d -= M[j * nP + p] * M[j * nP + p];
    if (!(d > 0)) return 1;
    d = sqrt(d);
    M[j * nP + j] = d;
    for (int i = j + 1; i < nP; ++i) {
      double s = M[i * nP + j];
      for (int p = 0; p < j; ++p) s -= M[i * nP + p] * M[j * nP + p];
      M[i * nP + j] = s / d;
    }
  }
  for (int ij = 0; ij < 4; ++ij) {
    // Y = L^-1 R_ij, then H += nu Y^T Y
    for (int c = 0; c < nz; ++c)
      for (int r = 0; r < nP; ++r) {
        double s = R[((long)ij * nP + r) * nz + c];
        for (int p = 0; p < r; ++p) s -= M[r * nP + p] * Y[(long)p * nz + c];
        Y[(long)r * nz + c] = s / M[r * nP + r];
      }
    for (int a = 0; a < nz; ++a)
      for (int b = 0; b <= a; ++b) {
        double s = 0.0;
        for (int r = 0; r < nP; ++r) s += Y[(long)r * nz + a] * Y[(long)r * nz + b];
        H[(long)a * nz + b] += nu * s;
        if (b != a) H[(long)b * nz + a] += nu * s;
      }
  }
  // ---- KKT matrix
  for (long i = 0; i < (long)nkkt * nkkt; ++i) Kk[i] = 0.0;
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < na; ++b) Kk[(long)a * nkkt + b] = H[(long)a * nz + b];
  for (int c = 0; c < nN; ++c)
    for (int a = 0; a < na; ++a) {
      Kk[(long)(na + c) * nkkt + a] = Nm[(long)c * na + a];
      Kk[(long)a * nkkt + na + c] = Nm[(long)c * na + a];
    }
  for (int r = 1; r < nP; ++r)
    for (int a = 0; a < na; ++a) {
      double dval = Dr[(long)r * na + a] - mean[r] * Dr[a];
      Kk[(long)(na + nN + r - 1) * nkkt + a] = dval;
      Kk[(long)a * nkkt + na + nN + r - 1] = dval;
    }
  // ---- LU with partial pivoting
  for (int j = 0; j < nkkt; ++j) {
    int pr = j;
    double best = fabs(Kk[(long)j * nkkt + j]);
    for (int i = j + 1; i < nkkt; ++i) {
      double v = fabs(Kk[(long)i * nkkt + j]);
      if (v > best) {
        best = v;
        pr = i;
      }
    }
    if (!(best > 0)) return 1;
    piv[j] = (double)pr;
    if (pr != j)
      for (int c = 0; c < nkkt; ++c) {
        double t = Kk[(long)j * nkkt + c];
        Kk[(long)j * nkkt + c] = Kk[(long)pr * nkkt + c];
        Kk[(long)pr * nkkt + c] = t;
      }
    double dj = Kk[(long)j * nkkt + j];
    for (int i = j + 1; i < nkkt; ++i) {
      double l = Kk[(long)i * nkkt + j] / dj;
      Kk[(long)i * nkkt + j] = l;
      if (l != 0.0)
        for (int c = j + 1; c < nkkt; ++c) Kk[(long)i * nkkt + c] -= l * Kk[(long)j * nkkt + c];
    }
  }
  // ---- factors kept for later loads and recoveries (element_cached)
  if (fac && mode == EL_CONDENSE) {
    const WS& Fo = *fac;
    long o2 = 0;
    for (long i = 0; i < (long)nkkt * nkkt; ++i) Fo[o2++] = Kk[i];
    for (int i = 0; i < nkkt; ++i) Fo[o2++] = piv[i];
    for (int t = 0; t < 3 * m; ++t)
      for (int a = 0; a < na; ++a) Fo[o2++] = H[(long)(na + t) * nz + a];  // H_ta (test t, trial a)
    for (int a = 0; a < na; ++a)
      for (int t = 0; t < 3 * m; ++t) Fo[o2++] = H[(long)a * nz + na + t];  // H_at
    for (int r = 0; r < nP; ++r) Fo[o2++] = mean[r];
  }
  // ---- right-hand sides
  int ncol = mode == EL_CONDENSE ? nK : mode == EL_GRADNU ? 2 : 1;
  for (long i = 0; i < (long)nkkt * ncol; ++i) Bx[i] = 0.0;
  if (mode == EL_CONDENSE) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < m; ++j) {
        int ln = (i * 2 + 0) * m + j, lt = (i * 2 + 1) * m + j;
        Bx[(long)(na + i * m + j) * ncol + ln] = 1.0;
        for (int a = 0; a < na; ++a) Bx[(long)a * ncol + lt] = -H[(long)a * nz + na + i * m + j];
      }
  } else {
    for (int cc = 0; cc < ncol; ++cc)
      for (int a = 0; a < na; ++a) Bx[(long)a * ncol + cc] = F[cc * na + a];
    if (mode == EL_RECOVER || mode == EL_GRADNU || mode == EL_POSTPROCESS) {
      for (int cc = 0; cc < ncol; ++cc) {
        const double* lm = cc == 0 ? lam : lam2;
        const bool tr = tcol && cc == 1;  // H^T: coupling H[t][a] in place of H[a][t]
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < m; ++j) {
            double cn = lm[(i * 2 + 0) * m + j], ct = lm[(i * 2 + 1) * m + j];
            Bx[(long)(na + i * m + j) * ncol + cc] += cn;
            const long tt = na + i * m + j;
            for (int a = 0; a < na; ++a)
              Bx[(long)a * ncol + cc] -= (tr ? H[tt * nz + a] : H[(long)a * nz + tt]) * ct;
          }
      }
    }
  }
  // The factors satisfy P KKT = L U (P: the row interchanges j <-> piv[j]
  // in order j = 0, 1, ...).  A transposed column solves
  // KKT^T x = U^T L^T P x = b: U^T z = b, L^T w = z, x = P^T w (the
  // interchanges undone in reverse order).
  const int ncol_fwd = tcol ? 1 : ncol;
  if (tcol) {
    const int c = 1;
    for (int i = 0; i < nkkt; ++i) {
      double s = Bx[(long)i * ncol + c];
      for (int p = 0; p < i; ++p) s -= Kk[(long)p * nkkt + i] * Bx[(long)p * ncol + c];
      Bx[(long)i * ncol + c] = s / Kk[(long)i * nkkt + i];
    }
    for (int i = nkkt - 1; i >= 0; --i) {
      double s = Bx[(long)i * ncol + c];
      for (int p = i + 1; p < nkkt; ++p) s -= Kk[(long)p * nkkt + i] * Bx[(long)p * ncol + c];
      Bx[(long)i * ncol + c] = s;
    }
    for (int j = nkkt - 1; j >= 0; --j) {
      int pr = (int)piv[j];
      if (pr != j) {
        double t = Bx[(long)j * ncol + c];
        Bx[(long)j * ncol + c] = Bx[(long)pr * ncol + c];
        Bx[(long)pr * ncol + c] = t;
      }
    }
  }
  // apply the row permutation, then forward / backward substitution
  for (int j = 0; j < nkkt; ++j) {
    int pr = (int)piv[j];
    if (pr != j)
      for (int c = 0; c < ncol_fwd; ++c) {
        double t = Bx[(long)j * ncol + c];
        Bx[(long)j * ncol + c] = Bx[(long)pr * ncol + c];
        Bx[(long)pr * ncol + c] = t;
      }
  }
  for (int c = 0; c < ncol_fwd; ++c) {
    for (int i = 0; i < nkkt; ++i) {
      double s = Bx[(long)i * ncol + c];
      for (int p = 0; p < i; ++p) s -= Kk[(long)i * nkkt + p] * Bx[(long)p * ncol + c];
      Bx[(long)i * ncol + c] = s;
    }
    for (int i = nkkt - 1; i >= 0; --i) {
      double s = Bx[(long)i * ncol + c];
      for (int p = i + 1; p < nkkt; ++p) s -= Kk[(long)i * nkkt + p] * Bx[(long)p * ncol + c];
      Bx[(long)i * ncol + c] = s / Kk[(long)i * nkkt + i];
    }
  }
  // ---- outputs
  if (mode == EL_CONDENSE || mode == EL_LOAD) {
    // rows of B^T X: normal (i,0,j) -> X[na + i m + j]; tangential (i,1,j) ->
    // -sum_a H[a][na + i m + j] X[a]
    for (int l1 = 0; l1 < nK; ++l1) {
      int i = l1 / (2 * m), c = (l1 / m) % 2, j = l1 % m;
      for (int cc = 0; cc < ncol; ++cc) {
        double btx;
        if (c == 0) {
          btx = Bx[(long)(na + i * m + j) * ncol + cc];
        } else {
          btx = 0.0;
          for (int a = 0; a < na; ++a) btx -= H[(long)(na + i * m + j) * nz + a] * Bx[(long)a * ncol + cc];
        }
        if (mode == EL_LOAD) {
          out[l1] = btx;
        } else {
          int l2 = cc;
          int i2 = l2 / (2 * m), c2 = (l2 / m) % 2, j2 = l2 % m;
          double htt = (c == 1 && c2 == 1) ? H[(long)(na + i * m + j) * nz + na + i2 * m + j2] : 0.0;
          out[l1 * nK + l2] = htt - btx;
        }
      }
    }
    if (mode == EL_CONDENSE && !conv) {
      for (int a = 0; a < nK; ++a)
        for (int b = 0; b < a; ++b) {
          double s = 0.5 * (out[a * nK + b] + out[b * nK + a]);
          out[a * nK + b] = s;
          out[b * nK + a] = s;
        }
    }
    if (mode == EL_CONDENSE) {
      for (int i1 = 0; i1 < 3; ++i1)
        for (int i2 = 0; i2 < 3; ++i2)
          out[(i1 * 2 * m) * nK + i2 * 2 * m] +=
              eps_inv / g.area * (g.sigma[i1] * g.len[i1]) * (g.sigma[i2] * g.len[i2]);
    }
  } else if (mode == EL_POSTPROCESS) {
    // lifting coefficients c_ij = M^-1 R_ij z (L_M, the Cholesky factor of
    // the P^k mass, held in M), kept in Y as [ij][nP]
    for (int ij = 0; ij < 4; ++ij) {
      for (int r = 0; r < nP; ++r) {
        const long row = ((long)ij * nP + r) * nz;
        double v = 0.0;
        for (int a = 0; a < na; ++a) v += R[row + a] * Bx[(long)a * ncol];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < m; ++j) v += R[row + na + i * m + j] * lam[(i * 2 + 1) * m + j];
        for (int p = 0; p < r; ++p) v -= M[r * nP + p] * Y[(long)ij * nP + p];
        Y[(long)ij * nP + r] = v / M[r * nP + r];
      }
      for (int r = nP - 1; r >= 0; --r) {
        double v = Y[(long)ij * nP + r];
        for (int p = r + 1; p < nP; ++p) v -= M[p * nP + r] * Y[(long)ij * nP + p];
        Y[(long)ij * nP + r] = v / M[r * nP + r];
      }
    }
    // P^{k+1} Neumann problem with the mean constraint, two right-hand
    // sides, in the (no longer needed) KKT storage: A [(nQ+1)^2], rhs
    // [2][nQ+1]
    const int nQ = (Q.k + 2) * (Q.k + 3) / 2, nA = nQ + 1;
    WS A{Kk.p, Kk.s};
    WS rhs{Kk.p + (long)nA * nA * Kk.s, Kk.s};
    for (int i = 0; i < nA * nA; ++i) A[i] = 0.0;
    for (int i = 0; i < 2 * nA; ++i) rhs[i] = 0.0;
    double qv[28], q1[28], q2[28];
    for (int q = 0; q < Q.nq; ++q) {
      const double x1 = Q.xi[q][0], x2 = Q.xi[q][1];
      const double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2,
                            g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
      const double wt = Q.wq[q] * g.area;
      rt_basis(D, g, x1, x2, xp, u, gr, mono);
      monomials(Q.k + 1, x1, x2, qv, q1, q2);
      double lift[4] = {0.0, 0.0, 0.0, 0.0}, uh[2] = {0.0, 0.0};
      for (int ij = 0; ij < 4; ++ij)
        for (int r = 0; r < nP; ++r) lift[ij] += Y[(long)ij * nP + r] * mono[r];
      for (int a = 0; a < na; ++a) {
        uh[0] += Bx[(long)a * ncol] * u[2 * a];
        uh[1] += Bx[(long)a * ncol] * u[2 * a + 1];
      }
      for (int r = 0; r < nQ; ++r) {
        // physical gradient of the reference monomial (xi = Ji (x - X0))
        const double gxr = q1[r] * g.Ji[0][0] + q2[r] * g.Ji[1][0];
        const double gyr = q1[r] * g.Ji[0][1] + q2[r] * g.Ji[1][1];
        for (int s2 = 0; s2 <= r; ++s2) {
          const double gxs = q1[s2] * g.Ji[0][0] + q2[s2] * g.Ji[1][0];
          const double gys = q1[s2] * g.Ji[0][1] + q2[s2] * g.Ji[1][1];
          A[(long)r * nA + s2] += wt * (gxr * gxs + gyr * gys);
        }
        A[(long)r * nA + nQ] += wt * qv[r];
        for (int i = 0; i < 2; ++i) rhs[(long)i * nA + r] += wt * (lift[2 * i] * gxr + lift[2 * i + 1] * gyr);
      }
      rhs[nQ] += wt * uh[0];
      rhs[(long)nA + nQ] += wt * uh[1];
    }
    for (int r = 0; r < nQ; ++r) {
      for (int s2 = 0; s2 < r; ++s2) A[(long)s2 * nA + r] = A[(long)r * nA + s2];
      A[(long)nQ * nA + r] = A[(long)r * nA + nQ];
    }
    A[(long)nQ * nA + nQ] = 0.0;
    // Gaussian elimination with partial pivoting on both right-hand sides
    for (int j = 0; j < nA; ++j) {
      int pr = j;
      double best = fabs(A[(long)j * nA + j]);
      for (int i = j + 1; i < nA; ++i)
        if (fabs(A[(long)i * nA + j]) > best) {
          best = fabs(A[(long)i * nA + j]);
          pr = i;
        }
      if (!(best > 0)) return 1;
      if (pr != j) {
        for (int c = 0; c < nA; ++c) {
          const double t = A[(long)j * nA + c];
          A[(long)j * nA + c] = A[(long)pr * nA + c];
          A[(long)pr * nA + c] = t;
        }
        for (int i = 0; i < 2; ++i) {
          const double t = rhs[(long)i * nA + j];
          rhs[(long)i * nA + j] = rhs[(long)i * nA + pr];
          rhs[(long)i * nA + pr] = t;
        }
      }
      const double dj = A[(long)j * nA + j];
      for (int r = j + 1; r < nA; ++r) {
        const double l = A[(long)r * nA + j] / dj;
        if (l == 0.0) continue;
        for (int c = j + 1; c < nA; ++c) A[(long)r * nA + c] -= l * A[(long)j * nA + c];
        for (int i = 0; i < 2; ++i) rhs[(long)i * nA + r] -= l * rhs[(long)i * nA + j];
      }
    }
    for (int i = 0; i < 2; ++i)
      for (int r = nA - 1; r >= 0; --r) {
        double v = rhs[(long)i * nA + r];
        for (int c = r + 1; c < nA; ++c) v -= A[(long)r * nA + c] * rhs[(long)i * nA + c];
        rhs[(long)i * nA + r] = v / A[(long)r * nA + r];
      }
    for (int q = 0; q < Q.nq; ++q) {
      monomials(Q.k + 1, Q.xi[q][0], Q.xi[q][1], qv, q1, q2);
      double us0 = 0.0, us1 = 0.0;
      for (int r = 0; r < nQ; ++r) {
        us0 += rhs[r] * qv[r];
        us1 += rhs[(long)nA + r] * qv[r];
      }
      out[2 * q] = us0;
      out[2 * q + 1] = us1;
    }
  } else if (mode == EL_GRADNU) {
    // -(Lift z, Lift z2)_K = -sum_ij (L_M^-1 R_ij z) . (L_M^-1 R_ij z2), with
    // z = (interior RT coefficients, tangential facet traces) and L_M the
    // Cholesky factor of the P^k mass matrix (held in M)
    double s = 0.0;
    for (int ij = 0; ij < 4; ++ij) {
      for (int cc = 0; cc < 2; ++cc) {
        const double* lm = cc == 0 ? lam : lam2;
        for (int r = 0; r < nP; ++r) {
          const long row = ((long)ij * nP + r) * nz;
          double v = 0.0;
          for (int a = 0; a < na; ++a) v += R[row + a] * Bx[(long)a * ncol + cc];
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < m; ++j) v += R[row + na + i * m + j] * lm[(i * 2 + 1) * m + j];
          for (int p = 0; p < r; ++p) v -= M[r * nP + p] * Y[(long)cc * nP + p];
          Y[(long)cc * nP + r] = v / M[r * nP + r];
        }
      }
      for (int r = 0; r < nP; ++r) s += Y[r] * Y[(long)nP + r];
    }
    out[0] = -s;
  } else {
    // recovery at the data points
    for (int q = 0; q < Q.nq; ++q) {
      double x1 = Q.xi[q][0], x2 = Q.xi[q][1];
      double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2,
                      g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
      rt_basis(D, g, x1, x2, xp, u, gr, mono);
      double ux = 0.0, uy = 0.0;
      for (int a = 0; a < na; ++a) {
        ux += Bx[a] * u[2 * a];
        uy += Bx[a] * u[2 * a + 1];
      }
      double p = p0;
      for (int r = 1; r < nP; ++r) p -= Bx[na + nN + r - 1] * (mono[r] - mean[r]);
      out[2 * q] = ux;
      out[2 * q + 1] = uy;
      out[2 * Q.nq + q] = p;
    }
  }
  return 0;
}

// Words per cell of the factors element_local keeps at condensation.
HDI long element_fac_size(int k) {
  const Dims D = dims_of(k);
  return (long)D.nkkt * D.nkkt + D.nkkt + 6L * D.m * D.na + D.nP;
}
// Workspace of element_cached (doubles per cell).
HDI long element_cached_ws_size(int k) {
  const Dims D = dims_of(k);
  return (long)D.na + D.nkkt;
}

// EL_LOAD / EL_RECOVER from the factors kept by element_local(EL_CONDENSE):
// the same local solve with the LU factors of the cell's KKT matrix, so only
// the source term and two triangular solves are computed.  Inputs and
// outputs as element_local.  nx: an additional local load (Newton), nz
// entries: RT test rows (added to the source moments) then tangential facet
// rows (added to the condensed load's tangential rows).
HDI void element_cached(const QuadTables& Q, const CellGeom& g, int mode, const double* f, const double* lam,
                        double p0, WS fac, WS w, double* out, const WS* nx = nullptr) {
  const Dims D = dims_of(Q.k);
  const int nP = D.nP, na = D.na, m = D.m, nK = D.nK, nN = D.nN, nkkt = D.nkkt;
  const long oK = 0, oP = (long)nkkt * nkkt, oHta = oP + nkkt, oHat = oHta + 3L * m * na, oMean = oHat + 3L * m * na;
  WS F{w.p, w.s};
  WS Bx{w.p + (long)na * w.s, w.s};
  double u[2 * 40], gr[4 * 40], mono[16];
  for (int a = 0; a < na; ++a) F[a] = 0.0;
  for (int q = 0; q < Q.nq; ++q) {
    double x1 = Q.xi[q][0], x2 = Q.xi[q][1];
    double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2, g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
    double wt = Q.wq[q] * g.area;
    rt_basis(D, g, x1, x2, xp, u, gr, mono);
    for (int a = 0; a < na; ++a) F[a] += wt * (f[2 * q] * u[2 * a] + f[2 * q + 1] * u[2 * a + 1]);
  }
  if (nx)
    for (int a = 0; a < na; ++a) F[a] += (*nx)[a];
  for (int i = 0; i < nkkt; ++i) Bx[i] = i < na ? F[i] : 0.0;
  if (mode == EL_RECOVER) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < m; ++j) {
        Bx[na + i * m + j] += lam[(i * 2 + 0) * m + j];
        const double ct = lam[(i * 2 + 1) * m + j];
        for (int a = 0; a < na; ++a) Bx[a] -= fac[oHat + (long)a * 3 * m + i * m + j] * ct;
      }
  }
  for (int j = 0; j < nkkt; ++j) {
    const int pr = (int)fac[oP + j];
    if (pr != j) {
      double t = Bx[j];
      Bx[j] = Bx[pr];
      Bx[pr] = t;
    }
  }
  for (int i = 0; i < nkkt; ++i) {
    double s = Bx[i];
    for (int p = 0; p < i; ++p) s -= fac[oK + (long)i * nkkt + p] * Bx[p];
    Bx[i] = s;
  }
  for (int i = nkkt - 1; i >= 0; --i) {
    double s = Bx[i];
    for (int p = i + 1; p < nkkt; ++p) s -= fac[oK + (long)i * nkkt + p] * Bx[p];
    Bx[i] = s / fac[oK + (long)i * nkkt + i];
  }
  if (mode == EL_LOAD) {
    for (int l1 = 0; l1 < nK; ++l1) {
      const int i = l1 / (2 * m), c = (l1 / m) % 2, j = l1 % m;
      double btx;
      if (c == 0) {
        btx = Bx[na + i * m + j];
      } else {
        btx = nx ? (*nx)[na + i * m + j] : 0.0;  // load on the facet unknown's test rows
        for (int a = 0; a < na; ++a) btx -= fac[oHta + (long)(i * m + j) * na + a] * Bx[a];
      }
      out[l1] = btx;
    }
    return;
  }
  for (int q = 0; q < Q.nq; ++q) {
    double x1 = Q.xi[q][0], x2 = Q.xi[q][1];
    double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2, g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
    rt_basis(D, g, x1, x2, xp, u, gr, mono);
    double ux = 0.0, uy = 0.0;
    for (int a = 0; a < na; ++a) {
      ux += Bx[a] * u[2 * a];
      uy += Bx[a] * u[2 * a + 1];
    }
    double p = p0;
    for (int r = 1; r < nP; ++r) p -= Bx[na + nN + r - 1] * (mono[r] - fac[oMean + r]);
    out[2 * q] = ux;
    out[2 * q + 1] = uy;
    out[2 * Q.nq + q] = p;
  }
}

// Coefficients in this cell's RT_k basis of a velocity field given at the
// data points: the L^2 projection with the data rule, which is exact for a
// field in RT_k (the products have degree <= 2k+2).  Workspace na*(na+1).
// Returns 1 if the Gram matrix is singular.
HDI int wind_fit(const QuadTables& Q, const CellGeom& g, const double* vals, WS w, double* coef) {
  const Dims D = dims_of(Q.k);
  const int na = D.na;
  WS G{w.p, w.s};
  WS r{w.p + (long)na * na * w.s, w.s};
  for (long i = 0; i < (long)na * na; ++i) G[i] = 0.0;
  for (int a = 0; a < na; ++a) r[a] = 0.0;
  double u[2 * 40], gr[4 * 40], mono[16];
  for (int q = 0; q < Q.nq; ++q) {
    double x1 = Q.xi[q][0], x2 = Q.xi[q][1];
    double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2,
                    g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
    double wt = Q.wq[q] * g.area;
    rt_basis(D, g, x1, x2, xp, u, gr, mono);
    for (int a = 0; a < na; ++a) {
      r[a] += wt * (vals[2 * q] * u[2 * a] + vals[2 * q + 1] * u[2 * a + 1]);
      for (int b = 0; b <= a; ++b) G[(long)a * na + b] += wt * (u[2 * a] * u[2 * b] + u[2 * a + 1] * u[2 * b + 1]);
    }
  }
  for (int j = 0; j < na; ++j) {
    double d = G[(long)j * na + j];
    for (int p = 0; p < j; ++p) d -= G[(long)j * na + p] * G[(long)j * na + p];
    if (!(d > 0)) return 1;
    d = sqrt(d);
    G[(long)j * na + j] = d;
    for (int i = j + 1; i < na; ++i) {
      double t = G[(long)i * na + j];
      for (int p = 0; p < j; ++p) t -= G[(long)i * na + p] * G[(long)j * na + p];
      G[(long)i * na + j] = t / d;
    }
  }
  for (int i = 0; i < na; ++i) {
    double t = r[i];
    for (int p = 0; p < i; ++p) t -= G[(long)i * na + p] * r[p];
    r[i] = t / G[(long)i * na + i];
  }
  for (int i = na - 1; i >= 0; --i) {
    double t = r[i];
    for (int p = i + 1; p < na; ++p) t -= G[(long)p * na + i] * r[p];
    r[i] = t / G[(long)i * na + i];
  }
  for (int a = 0; a < na; ++a) coef[a] = r[a];
  return 0;
}

// Closed-form lowest-order cell block of A^eps_{0,h} (k0-stOptForm) on the
// local DOFs (facet i, component c) -> 2i + c:
//   nu (grad Pi^CR u, grad Pi^CR v) + beta (u_RT0, v_RT0) + eps^-1 (div u, div v)
// CR basis gradient of facet i: |F_i| n_{K,i} / |K|; the RT0 basis with unit
// outward flux through facet i is (x - x_i) / (2|K|), whose products
// integrate exactly by int_K f g = |K|/12 [sum f_m . sum g_m + sum f_m . g_m]
// over vertex values of affine f, g.
HDI void cr_block(const CellGeom& g, double nu, double beta, double eps_inv, double* A) {
  double e[3][2][2];  // frame vectors (n, t) of each local facet
  double gradphi[3][2];
  double q[3];
  for (int i = 0; i < 3; ++i) {
    e[i][0][0] = g.n[i][0];
    e[i][0][1] = g.n[i][1];
    e[i][1][0] = g.t[i][0];
    e[i][1][1] = g.t[i][1];
    gradphi[i][0] = g.len[i] * g.sigma[i] * g.n[i][0] / g.area;
    gradphi[i][1] = g.len[i] * g.sigma[i] * g.n[i][1] / g.area;
    q[i] = g.sigma[i] * g.len[i];
  }
  double Mrt[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double si[2] = {0, 0}, sj[2] = {0, 0}, sd = 0.0;
      for (int mm = 0; mm < 3; ++mm) {
        double fi0 = g.X[mm][0] - g.X[i][0], fi1 = g.X[mm][1] - g.X[i][1];
        double fj0 = g.X[mm][0] - g.X[j][0], fj1 = g.X[mm][1] - g.X[j][1];
        si[0] += fi0;
        si[1] += fi1;
        sj[0] += fj0;
        sj[1] += fj1;
        sd += fi0 * fj0 + fi1 * fj1;
      }
      Mrt[i][j] = g.area / 12.0 * (si[0] * sj[0] + si[1] * sj[1] + sd) / (4.0 * g.area * g.area);
    }
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 2; ++a)
      for (int j = 0; j < 3; ++j)
        for (int b = 0; b < 2; ++b) {
          double ee = e[i][a][0] * e[j][b][0] + e[i][a][1] * e[j][b][1];
          double gg = gradphi[i][0] * gradphi[j][0] + gradphi[i][1] * gradphi[j][1];
          double v = nu * ee * gg * g.area;
          if (a == 0 && b == 0) v += beta * q[i] * q[j] * Mrt[i][j] + eps_inv * q[i] * q[j] / g.area;
          A[(2 * i + a) * 6 + 2 * j + b] = v;
        }
}

}  // namespace hdgmg
