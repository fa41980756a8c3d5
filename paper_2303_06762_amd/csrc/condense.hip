// Static condensation of the order-k cells (Sec. 3.2), a wavefront per cell.
//
// The same local problem as element_local(EL_CONDENSE) (element.hpp): the
// cell's matrices -- P^k mass M, lifting moments R_ij, the RT_k energy H,
// normal-trace moments N, divergence moments D, the KKT matrix and the
// condensed block -- live in LDS, and the 64 lanes of the wavefront share
// every step: each quadrature point's basis values are tabulated by the lanes
// (one RT_k function per lane), then every lane accumulates its own matrix
// entries; the KKT matrix is factorised by a right-looking LU with partial
// pivoting (pivot search by a wavefront reduction, one row or (row, column)
// entry per lane); the condensed columns are solved one per lane.  With a
// thread per cell the same work is a long serial chain of dependent memory
// accesses; here it is a few thousand LDS operations per lane.
#include <hip/hip_runtime.h>

#include "element.hpp"
#include "kernels.hpp"

namespace hdgmg {

namespace {

constexpr int WL = 64;  // lanes per cell

template <int K>
struct KD {
  static constexpr int m = K + 1, nP = (K + 1) * (K + 2) / 2, ntop = K + 1;
  static constexpr int na = 2 * nP + ntop, nz = na + 3 * m, nK = 6 * m, nN = 3 * m, nD = nP - 1;
  static constexpr int nkkt = na + nN + nD;
  // LDS: region A holds R and Y (the lifting step), then the KKT matrix and
  // the right-hand sides, then the condensed block
  static constexpr int nR = 4 * nP * nz, nY = 4 * nP * nz;
  static constexpr int nKk = nkkt * nkkt, nBx = nkkt * nK;
  static constexpr int nA = (nR + nY > nKk + nBx) ? nR + nY : nKk + nBx;
};

// One RT_k basis function (index a) at reference point (x1, x2), physical
// point xp: values (u0, u1) and gradient du_i/dx_j at v[2 + 2 i + j]; the
// same functions as rt_basis.
template <int K>
__device__ inline void rt_function(const CellGeom& g, int a, double x1, double x2, const double* xp, double* v) {
  using D = KD<K>;
  double mv[16], d1[16], d2[16];
  monomials(K, x1, x2, mv, d1, d2);
  if (a < 2 * D::nP) {
    const int r = a / 2, c = a % 2;
    const double gx = d1[r] * g.Ji[0][0] + d2[r] * g.Ji[1][0];
    const double gy = d1[r] * g.Ji[0][1] + d2[r] * g.Ji[1][1];
    v[0] = c == 0 ? mv[r] : 0.0;
    v[1] = c == 1 ? mv[r] : 0.0;
    v[2] = c == 0 ? gx : 0.0;
    v[3] = c == 0 ? gy : 0.0;
    v[4] = c == 1 ? gx : 0.0;
    v[5] = c == 1 ? gy : 0.0;
  } else {
    const int r = D::nP - D::ntop + (a - 2 * D::nP);
    const double gx = d1[r] * g.Ji[0][0] + d2[r] * g.Ji[1][0];
    const double gy = d1[r] * g.Ji[0][1] + d2[r] * g.Ji[1][1];
    const double y0 = (xp[0] - g.Xs0[0]) / g.h, y1 = (xp[1] - g.Xs0[1]) / g.h;
    v[0] = y0 * mv[r];
    v[1] = y1 * mv[r];
    v[2] = mv[r] / g.h + y0 * gx;
    v[3] = y0 * gy;
    v[4] = y1 * gx;
    v[5] = mv[r] / g.h + y1 * gy;
  }
}

// Tabulate the basis at one point into LDS: bu[a][6] (values, gradient),
// bm[r] (monomials), bphi[j] (facet functions at s, if s >= 0).
template <int K>
__device__ inline void tabulate(const CellGeom& g, double x1, double x2, const double* xp, double s, double* bu,
                                double* bm, double* bphi) {
  using D = KD<K>;
  const int lane = threadIdx.x;
  if (lane < D::na) rt_function<K>(g, lane, x1, x2, xp, bu + 6 * lane);
  if (lane == WL - 1) {
    double mv[16], d1[16], d2[16];
    monomials(K, x1, x2, mv, d1, d2);
    for (int r = 0; r < D::nP; ++r) bm[r] = mv[r];
    if (s >= 0.0) facet_legendre(K, s, bphi);
  }
  __syncthreads();
}

template <int K>
__global__ void __launch_bounds__(WL) k_condense_wave(ElemLevel E, double* __restrict__ S, int* status) {
  using D = KD<K>;
  constexpr int m = D::m, nP = D::nP, na = D::na, nz = D::nz, nK = D::nK, nN = D::nN, nkkt = D::nkkt;
  __shared__ double M[nP * nP], H[nz * nz], Nm[nN * na], Dr[nP * na], mean[nP];
  __shared__ double A[D::nA];
  __shared__ double bu[6 * na], bm[nP], bphi[m], wv[2];
  // Newton: the previous state's tangential traces per local facet and the
  // Newton load C_h(u_prev; u_prev, .) on the test functions
  __shared__ double tp[3 * m], nl[nz];
  __shared__ int piv[nkkt];
  __shared__ int sing;
  double* R = A;
  double* Y = A + D::nR;
  const int lane = threadIdx.x;
  const int c = blockIdx.x;
  CellGeom g;
  cell_geom(E.X, E.cells + 3 * c, g);
  const double nu = E.nu_per_cell ? E.nu[c] : E.nu[0];
  const ConvTables* CT = E.CT;
  const double* wc = E.wcoef ? E.wcoef + (long)c * E.na : nullptr;
  const bool conv = CT != nullptr && wc != nullptr;
  for (int e = lane; e < nP * nP; e += WL) M[e] = 0.0;
  for (int e = lane; e < nz * nz; e += WL) H[e] = 0.0;
  for (int e = lane; e < nN * na; e += WL) Nm[e] = 0.0;
  for (int e = lane; e < nP * na; e += WL) Dr[e] = 0.0;
  for (int e = lane; e < D::nR; e += WL) R[e] = 0.0;
  if (lane < nP) mean[lane] = 0.0;
  const bool newton = conv && E.nw_lam != nullptr;
  if (newton) {
    for (int e = lane; e < nz; e += WL) nl[e] = 0.0;
    for (int e = lane; e < 3 * m; e += WL) {
      const int i = e / m, j = e % m;
      const int d = E.cell_dofs[3 * c + i];
      tp[e] = d >= 0 ? E.nw_lam[((long)d * 2 + 1) * m + j] : (E.bdl ? E.bdl[(((long)c * 3 + i) * 2 + 1) * m + j] : 0.0);
    }
  }
  if (lane == 0) sing = 0;
  __syncthreads();

  // ---- volume terms (the convection rule when there is a wind)
  const int nvq = conv ? CT->nq : E.Q.nq;
  for (int q = 0; q < nvq; ++q) {
    const double x1 = conv ? CT->xi[q][0] : E.Q.xi[q][0], x2 = conv ? CT->xi[q][1] : E.Q.xi[q][1];
    const double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2, g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
    const double wt = (conv ? CT->wq[q] : E.Q.wq[q]) * g.area;
    tabulate<K>(g, x1, x2, xp, -1.0, bu, bm, bphi);
    if (conv && lane < 2) {
      double w = 0.0;
      for (int cc = 0; cc < na; ++cc) w += wc[cc] * bu[6 * cc + lane];
      wv[lane] = w;
    }
    if (lane < nP) mean[lane] += wt * bm[lane];
    for (int e = lane; e < nP * nP; e += WL) M[e] += wt * bm[e / nP] * bm[e % nP];
    for (int e = lane; e < nP * na; e += WL) {
      const int r = e / na, a = e % na;
      const double wm = wt * bm[r];
      const double* ga = bu + 6 * a + 2;
#pragma unroll
      for (int ij = 0; ij < 4; ++ij) R[((long)ij * nP + r) * nz + a] += wm * ga[ij];
      Dr[e] += wm * (ga[0] + ga[3]);
    }
    if (conv) __syncthreads();  // wv
    for (int e = lane; e < na * na; e += WL) {
      const int b = e / na, a = e % na;
      const double* ub = bu + 6 * b;
      const double* ua = bu + 6 * a;
      double h = E.beta * wt * (ua[0] * ub[0] + ua[1] * ub[1]);
      if (conv) {
        // - (u_a . (w . grad) v_b), test b, trial a
        const double g0 = wt * (wv[0] * ub[2] + wv[1] * ub[3]);
        const double g1 = wt * (wv[0] * ub[4] + wv[1] * ub[5]);
        h -= g0 * ua[0] + g1 * ua[1];
        if (newton) {
          // - sum_ij (u_prev,i du_j, d_j v_i) with du = u_a (u_prev = w)
          h -= wt * (ua[0] * (wv[0] * ub[2] + wv[1] * ub[4]) + ua[1] * (wv[0] * ub[3] + wv[1] * ub[5]));
        }
      }
      H[(long)b * nz + a] += h;
    }
    if (newton)
      for (int b = lane; b < na; b += WL) {
        // Newton load, volume part: - (u_prev . (u_prev . grad) v_b)
        const double* ub = bu + 6 * b;
        nl[b] -= wt * (wv[0] * (wv[0] * ub[2] + wv[1] * ub[3]) + wv[1] * (wv[0] * ub[4] + wv[1] * ub[5]));
      }
    __syncthreads();
  }
  if (lane < nP) mean[lane] /= g.area;

  // ---- facet terms
  for (int i = 0; i < 3; ++i) {
    const double* t = g.t[i];
    const double nk[2] = {g.sigma[i] * g.n[i][0], g.sigma[i] * g.n[i][1]};
    for (int l = 0; l < E.Q.nfq; ++l) {
      const double s = E.Q.s[l];
      const double xp[2] = {g.P0[i][0] + s * (g.P1[i][0] - g.P0[i][0]), g.P0[i][1] + s * (g.P1[i][1] - g.P0[i][1])};
      const double dx = xp[0] - g.Xs0[0], dy = xp[1] - g.Xs0[1];
      const double x1 = g.Ji[0][0] * dx + g.Ji[0][1] * dy, x2 = g.Ji[1][0] * dx + g.Ji[1][1] * dy;
      tabulate<K>(g, x1, x2, xp, s, bu, bm, bphi);
      const double wl = E.Q.ws[l] * g.len[i];
      // R_ij rows: -<u.t, t_i n_j mono_r> on the RT columns, + phi_j on this
      // facet's tangential trace columns
      for (int e = lane; e < 4 * nP * (na + m); e += WL) {
        const int row = e / (na + m), col = e % (na + m);
        const int ij = row / nP, r = row % nP, ii = ij / 2, jj = ij % 2;
        const double cf = wl * bm[r] * t[ii] * nk[jj];
        if (col < na) {
          const double* ua = bu + 6 * col;
          R[(long)row * nz + col] -= cf * (ua[0] * t[0] + ua[1] * t[1]);
        } else {
          const int j = col - na;
          R[(long)row * nz + na + i * m + j] += cf * bphi[j];
        }
      }
      for (int e = lane; e < m * na; e += WL) {
        const int j = e / na, a = e % na;
        const double* ua = bu + 6 * a;
        Nm[(long)(i * m + j) * na + a] += E.Q.ws[l] * bphi[j] * (ua[0] * g.n[i][0] + ua[1] * g.n[i][1]);
      }
      __syncthreads();
    }
  }
  // ---- convection facet terms: <(w.n_K) t(u_up), t(v) - vhat>
  if (conv) {
    for (int i = 0; i < 3; ++i) {
      const double* t = g.t[i];
      const double nk[2] = {g.sigma[i] * g.n[i][0], g.sigma[i] * g.n[i][1]};
      for (int l = 0; l < CT->n; ++l) {
        const double s = CT->s[l];
        const double xp[2] = {g.P0[i][0] + s * (g.P1[i][0] - g.P0[i][0]),
                              g.P0[i][1] + s * (g.P1[i][1] - g.P0[i][1])};
        const double dx = xp[0] - g.Xs0[0], dy = xp[1] - g.Xs0[1];
        const double x1 = g.Ji[0][0] * dx + g.Ji[0][1] * dy, x2 = g.Ji[1][0] * dx + g.Ji[1][1] * dy;
        tabulate<K>(g, x1, x2, xp, s, bu, bm, bphi);
        double wn = 0.0;
        for (int cc = 0; cc < na; ++cc) wn += wc[cc] * (bu[6 * cc] * nk[0] + bu[6 * cc + 1] * nk[1]);
        if (wn != 0.0) {
          const double cw = CT->ws[l] * g.len[i] * wn;
          // test rows: RT functions (v.t) and this facet's uhat modes (-phi)
          const int ntest = na + m, ntrial = wn > 0.0 ? na : m;
          for (int e = lane; e < ntest * ntrial; e += WL) {
            const int bt = e / ntrial, tr = e % ntrial;
            const int b = bt < na ? bt : na + i * m + (bt - na);
            const double tv = cw * (bt < na ? bu[6 * bt] * t[0] + bu[6 * bt + 1] * t[1] : -bphi[bt - na]);
            if (wn > 0.0)
              H[(long)b * nz + tr] += tv * (bu[6 * tr] * t[0] + bu[6 * tr + 1] * t[1]);
            else
              H[(long)b * nz + na + i * m + tr] += tv * bphi[tr];
          }
          const bool oflow = E.oflag && ((E.oflag[c] >> i) & 1);
          if (oflow) {
            __syncthreads();  // the upwind terms above touch the same entries
            // do-nothing facet: + <(w.n_K) u, vhat> (tangential on the facet
            // unknowns' rows, normal on the cell's normal trace), so that the
            // natural condition is (nu grad u - p I) n = 0
            for (int e = lane; e < (na + m) * na; e += WL) {
              const int bt = e / na, tr = e % na;
              const int b = bt < na ? bt : na + i * m + (bt - na);
              const double tv = bt < na ? bu[6 * bt] * nk[0] + bu[6 * bt + 1] * nk[1] : bphi[bt - na];
              const double uv = bt < na ? bu[6 * tr] * nk[0] + bu[6 * tr + 1] * nk[1]
                                        : bu[6 * tr] * t[0] + bu[6 * tr + 1] * t[1];
              H[(long)b * nz + tr] += cw * tv * uv;
            }
          }
          // (boundary facets: the increment's normal trace vanishes there and
          // u_prev.n_K is zero up to rounding, so the term is left out)
          if (newton && E.cell_dofs[3 * c + i] >= 0) {
            __syncthreads();  // the Picard terms above touch the same entries
            // upwind tangential value of the previous state: its own trace
            // where w.n_K > 0, its facet unknown where w.n_K < 0
            double up = 0.0;
            if (wn > 0.0)
              for (int cc = 0; cc < na; ++cc) up += wc[cc] * (bu[6 * cc] * t[0] + bu[6 * cc + 1] * t[1]);
            else
              for (int j = 0; j < m; ++j) up += tp[i * m + j] * bphi[j];
            const double cu = CT->ws[l] * g.len[i] * up;
            // <(du.n_K) up, t(v) - vhat>: trial du = u_a
            for (int e = lane; e < ntest * na; e += WL) {
              const int bt = e / na, tr = e % na;
              const int b = bt < na ? bt : na + i * m + (bt - na);
              const double tv = bt < na ? bu[6 * bt] * t[0] + bu[6 * bt + 1] * t[1] : -bphi[bt - na];
              H[(long)b * nz + tr] += cu * tv * (bu[6 * tr] * nk[0] + bu[6 * tr + 1] * nk[1]);
            }
            // Newton load, facet part: (w.n_K) up (t(v) - vhat)
            for (int bt = lane; bt < ntest; bt += WL) {
              const int b = bt < na ? bt : na + i * m + (bt - na);
              const double tv = bt < na ? bu[6 * bt] * t[0] + bu[6 * bt + 1] * t[1] : -bphi[bt - na];
              nl[b] += cw * up * tv;
            }
            if (oflow) {
              __syncthreads();
              // the do-nothing term's derivative in its first argument,
              // <(du.n_K) u_prev, vhat>, and its load (w.n_K) <u_prev, vhat>
              // (the wind is u_prev: its tangential and normal traces)
              double upt = 0.0;
              for (int cc = 0; cc < na; ++cc) upt += wc[cc] * (bu[6 * cc] * t[0] + bu[6 * cc + 1] * t[1]);
              const double cl = CT->ws[l] * g.len[i];
              for (int e = lane; e < (na + m) * na; e += WL) {
                const int bt = e / na, tr = e % na;
                const int b = bt < na ? bt : na + i * m + (bt - na);
                const double tv = bt < na ? wn * (bu[6 * bt] * nk[0] + bu[6 * bt + 1] * nk[1]) : upt * bphi[bt - na];
                H[(long)b * nz + tr] += cl * tv * (bu[6 * tr] * nk[0] + bu[6 * tr + 1] * nk[1]);
              }
              for (int bt = lane; bt < na + m; bt += WL) {
                const int b = bt < na ? bt : na + i * m + (bt - na);
                const double tv = bt < na ? wn * (bu[6 * bt] * nk[0] + bu[6 * bt + 1] * nk[1]) : upt * bphi[bt - na];
                nl[b] += cw * tv;
              }
            }
          }
        }
        __syncthreads();
      }
    }
  }

  // ---- transposed (adjoint) cell: H <- H^T (only the convection part is
  // nonsymmetric); one lane per pair
  if (conv && E.transpose) {
    for (int e = lane; e < nz * nz; e += WL) {
      const int a = e / nz, b = e % nz;
      if (b < a) {
        const double t = H[(long)a * nz + b];
        H[(long)a * nz + b] = H[(long)b * nz + a];
        H[(long)b * nz + a] = t;
      }
    }
    __syncthreads();
  }
  // ---- H += nu sum_ij R_ij^T M^-1 R_ij (Cholesky of M on one lane)
  if (lane == 0) {
    for (int j = 0; j < nP; ++j) {
      double d = M[j * nP + j];
      for (int p = 0; p < j; ++p) d -= M[j * nP + p] * M[j * nP + p];
      if (!(d > 0)) sing = 1;
      d = sqrt(d);
      M[j * nP + j] = d;
      for (int r = j + 1; r < nP; ++r) {
        double sm = M[r * nP + j];
        for (int p = 0; p < j; ++p) sm -= M[r * nP + p] * M[j * nP + p];
        M[r * nP + j] = sm / d;
      }
    }
  }
  __syncthreads();
  if (sing) {
    if (lane == 0) atomicOr(status, 1);
    return;
  }
  // Y_ij = L^-1 R_ij, a column (ij, col) per lane
  for (int e = lane; e < 4 * nz; e += WL) {
    const int ij = e / nz, col = e % nz;
    for (int r = 0; r < nP; ++r) {
      double sm = R[((long)ij * nP + r) * nz + col];
      for (int p = 0; p < r; ++p) sm -= M[r * nP + p] * Y[((long)ij * nP + p) * nz + col];
      Y[((long)ij * nP + r) * nz + col] = sm / M[r * nP + r];
    }
  }
  __syncthreads();
  for (int e = lane; e < nz * nz; e += WL) {
    const int a = e / nz, b = e % nz;
    double sm = 0.0;
    for (int ij = 0; ij < 4; ++ij)
      for (int r = 0; r < nP; ++r) sm += Y[((long)ij * nP + r) * nz + a] * Y[((long)ij * nP + r) * nz + b];
    H[e] += nu * sm;
  }
  __syncthreads();

  // ---- KKT matrix [H_aa N^T D^T; N 0 0; D 0 0] (R and Y are dead)
  double* Kk = A;
  double* Bx = A + D::nKk;
  for (int e = lane; e < nkkt * nkkt; e += WL) {
    const int r = e / nkkt, q = e % nkkt;
    double v = 0.0;
    if (r < na && q < na)
      v = H[(long)r * nz + q];
    else if (r < na && q < na + nN)
      v = Nm[(long)(q - na) * na + r];
    else if (q < na && r >= na && r < na + nN)
      v = Nm[(long)(r - na) * na + q];
    else if (r < na && q >= na + nN)
      v = Dr[(long)(q - na - nN + 1) * na + r] - mean[q - na - nN + 1] * Dr[r];
    else if (q < na && r >= na + nN)
      v = Dr[(long)(r - na - nN + 1) * na + q] - mean[r - na - nN + 1] * Dr[q];
    Kk[e] = v;
  }
  __syncthreads();
  // ---- LU with partial pivoting (largest magnitude, first index on ties)
  for (int j = 0; j < nkkt; ++j) {
    double bv = -1.0;
    int bi = nkkt;
    for (int r = j + lane; r < nkkt; r += WL) {
      const double v = fabs(Kk[(long)r * nkkt + j]);
      if (v > bv) {
        bv = v;
        bi = r;
      }
    }
    for (int off = WL / 2; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (!(bv > 0)) {
      if (lane == 0) atomicOr(status, 1);
      return;
    }
    const int pr = bi;
    if (lane == 0) piv[j] = pr;
    if (pr != j)
      for (int q = lane; q < nkkt; q += WL) {
        const double tq = Kk[(long)j * nkkt + q];
        Kk[(long)j * nkkt + q] = Kk[(long)pr * nkkt + q];
        Kk[(long)pr * nkkt + q] = tq;
      }
    __syncthreads();
    const double dj = Kk[(long)j * nkkt + j];
    for (int r = j + 1 + lane; r < nkkt; r += WL) Kk[(long)r * nkkt + j] /= dj;
    __syncthreads();
    const int w = nkkt - j - 1;
    for (int e = lane; e < w * w; e += WL) {
      const int r = j + 1 + e / w, q = j + 1 + e % w;
      Kk[(long)r * nkkt + q] -= Kk[(long)r * nkkt + j] * Kk[(long)j * nkkt + q];
    }
    __syncthreads();
  }
  // ---- factors kept for later loads and recoveries (element_cached)
  if (E.fac) {
    double* F = E.fac + c;
    const long nc = E.nc;
    long o = 0;
    for (int e = lane; e < nkkt * nkkt; e += WL) F[(o + e) * nc] = Kk[e];
    o += (long)nkkt * nkkt;
    for (int e = lane; e < nkkt; e += WL) F[(o + e) * nc] = (double)piv[e];
    o += nkkt;
    for (int e = lane; e < 3 * m * na; e += WL) F[(o + e) * nc] = H[(long)(na + e / na) * nz + e % na];
    o += 3L * m * na;
    for (int e = lane; e < na * 3 * m; e += WL) F[(o + e) * nc] = H[(long)(e / (3 * m)) * nz + na + e % (3 * m)];
    o += (long)na * 3 * m;
    for (int e = lane; e < nP; e += WL) F[(o + e) * nc] = mean[e];
  }
  if (newton && E.nw_load)
    for (int e = lane; e < nz; e += WL) E.nw_load[(long)e * E.nc + c] = nl[e];
  // ---- right-hand sides B = [[0, -H_at], [I, 0], [0, 0]] (columns c^n, c^t)
  for (int e = lane; e < nkkt * nK; e += WL) {
    const int r = e / nK, l = e % nK;
    const int i = l / (2 * m), cmp = (l / m) % 2, j = l % m;
    double v = 0.0;
    if (cmp == 0 && r == na + i * m + j) v = 1.0;
    if (cmp == 1 && r < na) v = -H[(long)r * nz + na + i * m + j];
    Bx[e] = v;
  }
  __syncthreads();
  // row permutation and the two triangular solves, a column per lane
  for (int l = lane; l < nK; l += WL) {
    for (int j = 0; j < nkkt; ++j) {
      const int pr = piv[j];
      if (pr != j) {
        const double tq = Bx[(long)j * nK + l];
        Bx[(long)j * nK + l] = Bx[(long)pr * nK + l];
        Bx[(long)pr * nK + l] = tq;
      }
    }
    for (int r = 0; r < nkkt; ++r) {
      double sm = Bx[(long)r * nK + l];
      for (int p = 0; p < r; ++p) sm -= Kk[(long)r * nkkt + p] * Bx[(long)p * nK + l];
      Bx[(long)r * nK + l] = sm;
    }
    for (int r = nkkt - 1; r >= 0; --r) {
      double sm = Bx[(long)r * nK + l];
      for (int p = r + 1; p < nkkt; ++p) sm -= Kk[(long)r * nkkt + p] * Bx[(long)p * nK + l];
      Bx[(long)r * nK + l] = sm / Kk[(long)r * nkkt + r];
    }
  }
  __syncthreads();
  // ---- S = blockdiag(0, H_tt) - B^T X, symmetrised without a wind, plus the
  // augmented-Lagrangian term; staged over the (dead) KKT factors
  double* Sl = Kk;
  for (int e = lane; e < nK * nK; e += WL) {
    const int l1 = e / nK, l2 = e % nK;
    const int i = l1 / (2 * m), cmp = (l1 / m) % 2, j = l1 % m;
    const int i2 = l2 / (2 * m), c2 = (l2 / m) % 2, j2 = l2 % m;
    double btx;
    if (cmp == 0) {
      btx = Bx[(long)(na + i * m + j) * nK + l2];
    } else {
      btx = 0.0;
      for (int a = 0; a < na; ++a) btx -= H[(long)(na + i * m + j) * nz + a] * Bx[(long)a * nK + l2];
    }
    const double htt = (cmp == 1 && c2 == 1) ? H[(long)(na + i * m + j) * nz + na + i2 * m + j2] : 0.0;
    Sl[e] = htt - btx;
  }
  __syncthreads();
  double* out = S + (long)c * nK * nK;
  for (int e = lane; e < nK * nK; e += WL) {
    const int a = e / nK, b = e % nK;
    double v = conv ? Sl[e] : 0.5 * (Sl[e] + Sl[b * nK + a]);
    if (a % (2 * m) == 0 && b % (2 * m) == 0) {
      const int i1 = a / (2 * m), i2 = b / (2 * m);
      v += E.eps_inv / g.area * (g.sigma[i1] * g.len[i1]) * (g.sigma[i2] * g.len[i2]);
    }
    out[e] = v;
  }
}

}  // namespace

bool condense_wave_supported(int k) { return k >= 1 && k <= 4; }

void launch_condense_wave(hipStream_t st, const ElemLevel& E, double* S, int* status) {
  if (E.nc <= 0) return;
  switch (E.Q.k) {
    case 1: hipLaunchKernelGGL(k_condense_wave<1>, dim3(E.nc), dim3(WL), 0, st, E, S, status); break;
    case 2: hipLaunchKernelGGL(k_condense_wave<2>, dim3(E.nc), dim3(WL), 0, st, E, S, status); break;
    case 3: hipLaunchKernelGGL(k_condense_wave<3>, dim3(E.nc), dim3(WL), 0, st, E, S, status); break;
    case 4: hipLaunchKernelGGL(k_condense_wave<4>, dim3(E.nc), dim3(WL), 0, st, E, S, status); break;
    default: break;
  }
}

}  // namespace hdgmg
