// Kernels of the tetrahedral path (see tet.hpp for the formulation).
#include "tet.hpp"

#include <algorithm>

namespace hdgmg {

namespace {

constexpr int NT = 256;  // threads of the element and patch workgroups

struct WsLayout {
  long psq, gsq, xtq, psf, xtf, uq, dvq, m, r, h, ka, total;
  int ldk, nrhs;
};

HDI WsLayout ws_layout(int k, int mode) {
  const Dims3 d = dims3(k);
  const int nq = (k + 2) * (k + 2) * (k + 2), nfq = (k + 2) * (k + 2);
  WsLayout w;
  w.nrhs = mode == TET_CONDENSE ? d.nK : 1;
  w.ldk = d.nkkt + w.nrhs;
  long o = 0;
  w.psq = o;
  o += (long)nq * d.nP;
  w.gsq = o;
  o += (long)nq * d.nP * 3;
  w.xtq = o;
  o += (long)nq * 3;
  w.psf = o;
  o += 4L * nfq * d.nP;
  w.xtf = o;
  o += 4L * nfq * 3;
  w.uq = o;
  o += (long)nq * d.na * 3;
  w.dvq = o;
  o += (long)nq * d.na;
  w.m = o;
  o += (long)d.nP * d.nP;
  w.r = o;
  long rsz = 9L * d.nP * d.nz;
  if ((long)d.nK * d.nK > rsz) rsz = (long)d.nK * d.nK;
  o += rsz;
  w.h = o;
  o += (long)d.nz * d.nz;
  w.ka = o;
  o += (long)d.nkkt * w.ldk;
  w.total = (o + 31) / 32 * 32;
  return w;
}

// monomials xi^(a,b,c) of degree <= k, ordered by degree d, then c = 0..d,
// then b = 0..d-c (a = d-b-c); values and reference gradients
__device__ inline void mono3(int k, const double* xi, double* v, double (*g)[3]) {
  double p[3][K3MAX + 2];
  for (int d = 0; d < 3; ++d) {
    p[d][0] = 1.0;
    for (int i = 1; i <= k; ++i) p[d][i] = p[d][i - 1] * xi[d];
  }
  int s = 0;
  for (int deg = 0; deg <= k; ++deg)
    for (int c = 0; c <= deg; ++c)
      for (int b = 0; b <= deg - c; ++b, ++s) {
        const int a = deg - b - c;
        v[s] = p[0][a] * p[1][b] * p[2][c];
        g[s][0] = a > 0 ? a * p[0][a - 1] * p[1][b] * p[2][c] : 0.0;
        g[s][1] = b > 0 ? b * p[0][a] * p[1][b - 1] * p[2][c] : 0.0;
        g[s][2] = c > 0 ? c * p[0][a] * p[1][b] * p[2][c - 1] : 0.0;
      }
}

struct Geo {
  double Xs[4][3];
  int pos[4];  // sorted position of stored vertex i
  double J[3][3], Ji[3][3];
  double vol, h;
  int rf[4][3];  // sorted positions of the vertices of local face i
  double n[4][3], t1[4][3], t2[4][3], area[4];
  int sigma[4];
  double nu;
};

__device__ void geometry(const TetCells& E, int cell, Geo& G) {
  int v[4];
  for (int i = 0; i < 4; ++i) v[i] = E.cells[4 * cell + i];
  int ord[4] = {0, 1, 2, 3};
  for (int i = 1; i < 4; ++i)
    for (int j = i; j > 0 && v[ord[j]] < v[ord[j - 1]]; --j) {
      int t = ord[j];
      ord[j] = ord[j - 1];
      ord[j - 1] = t;
    }
  for (int s = 0; s < 4; ++s) {
    G.pos[ord[s]] = s;
    for (int d = 0; d < 3; ++d) G.Xs[s][d] = E.X[3 * v[ord[s]] + d];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) G.J[r][c] = G.Xs[c + 1][r] - G.Xs[0][r];
  const double (*J)[3] = G.J;
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  G.Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  G.Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  G.Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  G.Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  G.Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  G.Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  G.Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  G.Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  G.Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  G.vol = fabs(det) / 6.0;
  double h2 = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) {
      double s = 0.0;
      for (int d = 0; d < 3; ++d) s += (G.Xs[a][d] - G.Xs[b][d]) * (G.Xs[a][d] - G.Xs[b][d]);
      h2 = fmax(h2, s);
    }
  G.h = sqrt(h2);
  for (int i = 0; i < 4; ++i) {
    int q = 0;
    for (int s = 0; s < 4; ++s)
      if (s != G.pos[i]) G.rf[i][q++] = s;
    const double* X0 = G.Xs[G.rf[i][0]];
    const double* X1 = G.Xs[G.rf[i][1]];
    const double* X2 = G.Xs[G.rf[i][2]];
    double a[3], b[3], n[3];
    for (int d = 0; d < 3; ++d) {
      a[d] = X1[d] - X0[d];
      b[d] = X2[d] - X0[d];
    }
    n[0] = a[1] * b[2] - a[2] * b[1];
    n[1] = a[2] * b[0] - a[0] * b[2];
    n[2] = a[0] * b[1] - a[1] * b[0];
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    G.area[i] = 0.5 * nn;
    for (int d = 0; d < 3; ++d) {
      G.n[i][d] = n[d] / nn;
      G.t1[i][d] = a[d] / la;
    }
    G.t2[i][0] = G.n[i][1] * G.t1[i][2] - G.n[i][2] * G.t1[i][1];
    G.t2[i][1] = G.n[i][2] * G.t1[i][0] - G.n[i][0] * G.t1[i][2];
    G.t2[i][2] = G.n[i][0] * G.t1[i][1] - G.n[i][1] * G.t1[i][0];
    double o = 0.0;
    const double* Xi = G.Xs[G.pos[i]];
    for (int d = 0; d < 3; ++d) o += ((X0[d] + X1[d] + X2[d]) / 3.0 - Xi[d]) * G.n[i][d];
    G.sigma[i] = o > 0 ? 1 : -1;
  }
  G.nu = E.nu_per_cell ? E.nu[cell] : E.nu[0];
}

// reference coordinates of point (s, t) of local face i
__device__ inline void face_xi(const Geo& G, int i, double s, double t, double* xi) {
  double e[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int d = 0; d < 3; ++d)
    xi[d] = e[G.rf[i][0]][d] + s * (e[G.rf[i][1]][d] - e[G.rf[i][0]][d]) +
            t * (e[G.rf[i][2]][d] - e[G.rf[i][0]][d]);
}

// Value of RT basis function a at a point with monomial values ps [nP] and
// scaled position xt = (x - X_s0)/h.
__device__ inline void rt_val(const Dims3& d, int a, const double* ps, const double* xt, double* u) {
  if (a < 3 * d.nP) {
    const int c = a / d.nP, s = a % d.nP;
    u[0] = u[1] = u[2] = 0.0;
    u[c] = ps[s];
  } else {
    const double m = ps[d.nP - d.ntop + (a - 3 * d.nP)];
    u[0] = xt[0] * m;
    u[1] = xt[1] * m;
    u[2] = xt[2] * m;
  }
}

// d u_i / d x_j of basis function a (gs: physical monomial gradients [nP][3])
__device__ inline double rt_grad(const Dims3& d, double h, int a, int i, int j, const double* ps, const double* gs,
                                 const double* xt) {
  if (a < 3 * d.nP) {
    const int c = a / d.nP, s = a % d.nP;
    return c == i ? gs[3 * s + j] : 0.0;
  }
  const int s = d.nP - d.ntop + (a - 3 * d.nP);
  return ((i == j ? ps[s] : 0.0) + xt[i] * gs[3 * s + j] * h) / h;
}

__device__ inline double rt_div(const Dims3& d, double h, int a, const double* ps, const double* gs,
                                const double* xt) {
  return rt_grad(d, h, a, 0, 0, ps, gs, xt) + rt_grad(d, h, a, 1, 1, ps, gs, xt) + rt_grad(d, h, a, 2, 2, ps, gs, xt);
}

__global__ void __launch_bounds__(NT) k_tet_local(TetCells E, int mode, int c0, double* ws, const double* f,
                                                  const double* lam, const double* p0, double* S, double* gK,
                                                  double* uo, double* po, int* status) {
  __shared__ Geo G;
  __shared__ double fct[160];
  __shared__ int piv;
  __shared__ double pinv_s;
  __shared__ double lamK[12 * MF3MAX];
  __shared__ double red_v[NT];
  __shared__ int red_i[NT];
  const int cell = c0 + blockIdx.x;
  const int tid = threadIdx.x;
  const TetTables& T = *E.T;
  const int k = E.k;
  const Dims3 d = dims3(k);
  const int nq = T.nq, nfq = T.nfq, nP = d.nP, nz = d.nz, na = d.na, mF = d.mF;
  const WsLayout L = ws_layout(k, mode);
  double* W = ws + (long)blockIdx.x * L.total;
  double* PSQ = W + L.psq;
  double* GSQ = W + L.gsq;
  double* XTQ = W + L.xtq;
  double* PSF = W + L.psf;
  double* XTF = W + L.xtf;
  double* UQ = W + L.uq;
  double* DVQ = W + L.dvq;
  double* M = W + L.m;
  double* R = W + L.r;
  double* H = W + L.h;
  double* KA = W + L.ka;
  const int ldk = L.ldk;
  if (tid == 0) geometry(E, cell, G);
  if (mode == TET_RECOVER)
    for (int i = tid; i < d.nK; i += NT) {
      const int fc = i / (3 * mF);
      const int dof = E.cell_dofs[4 * cell + fc];
      lamK[i] = dof < 0 ? 0.0 : lam[(long)dof * 3 * mF + i % (3 * mF)];
    }
  __syncthreads();
  // basis at the volume and face points
  for (int q = tid; q < nq + 4 * nfq; q += NT) {
    double xi[3], v[20], g[20][3];
    double* ps;
    double* xt;
    double* gs = nullptr;
    if (q < nq) {
      xi[0] = T.xq[q][0];
      xi[1] = T.xq[q][1];
      xi[2] = T.xq[q][2];
      ps = PSQ + (long)q * nP;
      gs = GSQ + (long)q * nP * 3;
      xt = XTQ + 3 * q;
    } else {
      const int fl = q - nq, fi = fl / nfq, l = fl % nfq;
      face_xi(G, fi, T.xf[l][0], T.xf[l][1], xi);
      ps = PSF + (long)fl * nP;
      xt = XTF + 3 * fl;
    }
    mono3(k, xi, v, g);
    for (int s = 0; s < nP; ++s) {
      ps[s] = v[s];
      if (gs)
        for (int j = 0; j < 3; ++j)
          gs[3 * s + j] = G.Ji[0][j] * g[s][0] + G.Ji[1][j] * g[s][1] + G.Ji[2][j] * g[s][2];
    }
    for (int r = 0; r < 3; ++r) xt[r] = (G.J[r][0] * xi[0] + G.J[r][1] * xi[1] + G.J[r][2] * xi[2]) / G.h;
  }
  __syncthreads();
  // RT basis values and divergences at the volume points
  for (long e = tid; e < (long)nq * na; e += NT) {
    const int q = (int)(e / na), a = (int)(e % na);
    rt_val(d, a, PSQ + (long)q * nP, XTQ + 3 * q, UQ + 3 * e);
    DVQ[e] = rt_div(d, G.h, a, PSQ + (long)q * nP, GSQ + (long)q * nP * 3, XTQ + 3 * q);
  }
  __syncthreads();
  // mass of P^k and the lifting blocks R_ij [9][nP][nz]
  for (int e = tid; e < nP * nP; e += NT) {
    const int r = e / nP, s = e % nP;
    double acc = 0.0;
    for (int q = 0; q < nq; ++q) acc += T.wq[q] * PSQ[(long)q * nP + r] * PSQ[(long)q * nP + s];
    M[e] = acc * G.vol;
  }
  // one (r, column) pair per item, all nine (i, j) blocks at once
  for (int e = tid; e < nP * nz; e += NT) {
    const int r = e / nz, col = e % nz;
    double acc[9];
    for (int ij = 0; ij < 9; ++ij) acc[ij] = 0.0;
    if (col < na) {
      for (int q = 0; q < nq; ++q) {
        const double wp = T.wq[q] * PSQ[(long)q * nP + r];
        const double* ps = PSQ + (long)q * nP;
        const double* gs = GSQ + (long)q * nP * 3;
        const double* xt = XTQ + 3 * q;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) acc[3 * i + j] += wp * rt_grad(d, G.h, col, i, j, ps, gs, xt);
      }
      for (int ij = 0; ij < 9; ++ij) acc[ij] *= G.vol;
      for (int fc = 0; fc < 4; ++fc) {
        double s1 = 0.0, s2 = 0.0;
        for (int l = 0; l < nfq; ++l) {
          const double* ps = PSF + ((long)fc * nfq + l) * nP;
          double u[3];
          rt_val(d, col, ps, XTF + 3 * (fc * nfq + l), u);
          const double wp = T.wf[l] * ps[r];
          s1 += wp * (u[0] * G.t1[fc][0] + u[1] * G.t1[fc][1] + u[2] * G.t1[fc][2]);
          s2 += wp * (u[0] * G.t2[fc][0] + u[1] * G.t2[fc][1] + u[2] * G.t2[fc][2]);
        }
        s1 *= G.area[fc];
        s2 *= G.area[fc];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            acc[3 * i + j] -= (G.t1[fc][i] * s1 + G.t2[fc][i] * s2) * G.sigma[fc] * G.n[fc][j];
      }
    } else {
      const int c2 = col - na, fc = c2 / (2 * mF), cc = (c2 / mF) % 2, m = c2 % mF;
      const double* t = cc == 0 ? G.t1[fc] : G.t2[fc];
      double sf = 0.0;
      for (int l = 0; l < nfq; ++l) sf += T.wf[l] * PSF[((long)fc * nfq + l) * nP + r] * T.phif[l][m];
      sf *= G.area[fc];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc[3 * i + j] = t[i] * G.sigma[fc] * G.n[fc][j] * sf;
    }
    for (int ij = 0; ij < 9; ++ij) R[((long)ij * nP + r) * nz + col] = acc[ij];
  }
  __syncthreads();
  // Cholesky of M (one thread; nP <= 20), then G_ij = L^-1 R_ij in place
  if (tid == 0) {
    for (int c = 0; c < nP; ++c) {
      double s = M[c * nP + c];
      for (int p = 0; p < c; ++p) s -= M[c * nP + p] * M[c * nP + p];
      if (!(s > 0.0)) {
        atomicOr(status, 1);
        s = 1.0;
      }
      M[c * nP + c] = sqrt(s);
      for (int r = c + 1; r < nP; ++r) {
        double t = M[r * nP + c];
        for (int p = 0; p < c; ++p) t -= M[r * nP + p] * M[c * nP + p];
        M[r * nP + c] = t / M[c * nP + c];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < 9 * nz; e += NT) {
    const int ij = e / nz, col = e % nz;
    double* Rc = R + (long)ij * nP * nz + col;
    for (int r = 0; r < nP; ++r) {
      double t = Rc[(long)r * nz];
      for (int p = 0; p < r; ++p) t -= M[r * nP + p] * Rc[(long)p * nz];
      Rc[(long)r * nz] = t / M[r * nP + r];
    }
  }
  __syncthreads();
  // H = nu sum_ij G_ij^T G_ij on FP64 matrix cores: G = [G_00; ..; G_22] is
  // a (9 nP) x nz matrix (row stride nz), H = G^T G its Gram matrix.  Each
  // wavefront owns 16 x 16 tiles (a-tile <= b-tile, mirrored) and
  // accumulates them over the 9 nP rows four at a time with
  // v_mfma_f64_16x16x4 (A operand: lane l holds G[k0 + l/16][a0 + l%16];
  // B operand: lane l holds G[k0 + l/16][b0 + l%16]; result register r of
  // lane l is H[a0 + l/16 + 4 r][b0 + l%16], the layout measured on gfx950).
  {
    const int wave = tid / 64, lane = tid % 64, nw = NT / 64;
    const int nt = (nz + 15) / 16, kdim = 9 * nP;
    const int li = lane % 16, lk = lane / 16;
    int tile = 0;
    for (int ta = 0; ta < nt; ++ta)
      for (int tb = ta; tb < nt; ++tb, ++tile) {
        if (tile % nw != wave) continue;
        const int a0 = 16 * ta, b0 = 16 * tb;
        const bool ina = a0 + li < nz, inb = b0 + li < nz;
        typedef double v4d __attribute__((ext_vector_type(4)));
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < kdim; k0 += 4) {
          const int kk = k0 + lk;
          const double av = (ina && kk < kdim) ? R[(long)kk * nz + a0 + li] : 0.0;
          const double bv = (inb && kk < kdim) ? R[(long)kk * nz + b0 + li] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        for (int r = 0; r < 4; ++r) {
          const int a = a0 + lk + 4 * r, b = b0 + li;
          if (a < nz && b < nz) {
            const double v = G.nu * acc[r];
            H[(long)a * nz + b] = v;
            H[(long)b * nz + a] = v;
          }
        }
      }
  }
  __syncthreads();
  // + beta (u_a, u_b) on the RT block
  if (E.beta != 0.0)
    for (long e = tid; e < (long)na * na; e += NT) {
      const int a = (int)(e / na), b = (int)(e % na);
      if (b < a) continue;
      double ms = 0.0;
      for (int q = 0; q < nq; ++q) {
        const double* ua = UQ + 3 * ((long)q * na + a);
        const double* ub = UQ + 3 * ((long)q * na + b);
        ms += T.wq[q] * (ua[0] * ub[0] + ua[1] * ub[1] + ua[2] * ub[2]);
      }
      const double v = H[(long)a * nz + b] + E.beta * G.vol * ms;
      H[(long)a * nz + b] = v;
      if (a != b) H[(long)b * nz + a] = v;
    }
  __syncthreads();
  // KKT with its right-hand side columns
  const int nkkt = d.nkkt;
  for (long e = tid; e < (long)nkkt * ldk; e += NT) KA[e] = 0.0;
  __syncthreads();
  for (long e = tid; e < (long)na * na; e += NT) {
    const int a = (int)(e / na), b = (int)(e % na);
    KA[(long)a * ldk + b] = H[(long)a * nz + b];
  }
  for (int e = tid; e < d.nN * na; e += NT) {
    const int row = e / na, a = e % na, fc = row / mF, m = row % mF;
    double s = 0.0;
    for (int l = 0; l < nfq; ++l) {
      double u[3];
      rt_val(d, a, PSF + ((long)fc * nfq + l) * nP, XTF + 3 * (fc * nfq + l), u);
      s += T.wf[l] * T.phif[l][m] * (u[0] * G.n[fc][0] + u[1] * G.n[fc][1] + u[2] * G.n[fc][2]);
    }
    KA[(long)(na + row) * ldk + a] = s;
    KA[(long)a * ldk + na + row] = s;
  }
  for (int e = tid; e < d.nD * na; e += NT) {
    const int r = e / na + 1, a = e % na;
    double mean = 0.0;
    for (int q = 0; q < nq; ++q) mean += T.wq[q] * PSQ[(long)q * nP + r];
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += T.wq[q] * (PSQ[(long)q * nP + r] - mean) * DVQ[(long)q * na + a];
    s *= G.vol;
    KA[(long)(na + d.nN + r - 1) * ldk + a] = s;
    KA[(long)a * ldk + na + d.nN + r - 1] = s;
  }
  if (mode == TET_CONDENSE) {
    for (int e = tid; e < d.nK * na; e += NT) {
      const int lam_i = e / na, a = e % na;
      const int fc = lam_i / (3 * mF), c = (lam_i / mF) % 3, m = lam_i % mF;
      if (c == 0) {
        if (a == 0) KA[(long)(na + fc * mF + m) * ldk + nkkt + lam_i] = 1.0;
      } else {
        KA[(long)a * ldk + nkkt + lam_i] = -H[(long)a * nz + na + (fc * 2 + c - 1) * mF + m];
      }
    }
  } else {
    // load F_a = (f, u_a); recovery subtracts H_at c^t and sets c^n
    for (int a = tid; a < na; a += NT) {
      double s = 0.0;
      const double* fq = f + (long)cell * nq * 3;
      for (int q = 0; q < nq; ++q) {
        const double* u = UQ + 3 * ((long)q * na + a);
        s += T.wq[q] * (u[0] * fq[3 * q] + u[1] * fq[3 * q + 1] + u[2] * fq[3 * q + 2]);
      }
      s *= G.vol;
      if (mode == TET_RECOVER)
        for (int fc = 0; fc < 4; ++fc)
          for (int cc = 0; cc < 2; ++cc)
            for (int m = 0; m < mF; ++m)
              s -= H[(long)a * nz + na + (fc * 2 + cc) * mF + m] * lamK[(fc * 3 + 1 + cc) * mF + m];
      KA[(long)a * ldk + nkkt] = s;
    }
    if (mode == TET_RECOVER)
      for (int e = tid; e < d.nN; e += NT) {
        const int fc = e / mF, m = e % mF;
        KA[(long)(na + e) * ldk + nkkt] = lamK[(fc * 3) * mF + m];
      }
  }
  __syncthreads();
  // Gauss-Jordan elimination with partial pivoting (pivot: block-wide
  // argmax of |column j| below the diagonal, first index on ties)
  for (int j = 0; j < nkkt; ++j) {
    {
      double v = -1.0;
      int idx = j;
      for (int i = j + tid; i < nkkt; i += NT) {
        const double a = fabs(KA[(long)i * ldk + j]);
        if (a > v) {
          v = a;
          idx = i;
        }
      }
      red_v[tid] = v;
      red_i[tid] = idx;
      __syncthreads();
      for (int w = NT / 2; w > 0; w >>= 1) {
        if (tid < w && (red_v[tid + w] > red_v[tid] || (red_v[tid + w] == red_v[tid] && red_i[tid + w] < red_i[tid]))) {
          red_v[tid] = red_v[tid + w];
          red_i[tid] = red_i[tid + w];
        }
        __syncthreads();
      }
      if (tid == 0) {
        piv = red_i[0];
        if (!(red_v[0] > 0.0)) atomicOr(status, 2);
      }
    }
    __syncthreads();
    const int p = piv;
    if (p != j)
      for (int c = tid; c < ldk; c += NT) {
        const double t = KA[(long)j * ldk + c];
        KA[(long)j * ldk + c] = KA[(long)p * ldk + c];
        KA[(long)p * ldk + c] = t;
      }
    __syncthreads();
    if (tid == 0) {
      const double v = KA[(long)j * ldk + j];
      pinv_s = v != 0.0 ? 1.0 / v : 0.0;
    }
    __syncthreads();
    for (int c = j + tid; c < ldk; c += NT) KA[(long)j * ldk + c] *= pinv_s;
    for (int i = tid; i < nkkt; i += NT) fct[i] = i == j ? 0.0 : KA[(long)i * ldk + j];
    __syncthreads();
    const int w = ldk - j;
    for (long e = tid; e < (long)nkkt * w; e += NT) {
      const int i = (int)(e / w), c = j + (int)(e % w);
      if (i == j) continue;
      KA[(long)i * ldk + c] -= fct[i] * KA[(long)j * ldk + c];
    }
    __syncthreads();
  }
  // outputs; X = KA[:, nkkt:]
  if (mode == TET_CONDENSE) {
    const int nK = d.nK;
    // P = H_at^T X_a (8 m_F x nK) on FP64 matrix cores: A[i][k] =
    // H[k][na + t0 + i], B[k][j] = X[k][l0 + j], k over the na RT unknowns
    double* P = UQ;  // the basis values are no longer needed
    {
      const int wave = tid / 64, lane = tid % 64, nw = NT / 64;
      const int nT = 8 * mF, ntr = (nT + 15) / 16, ntc = (nK + 15) / 16;
      const int li = lane % 16, lk = lane / 16;
      typedef double v4d __attribute__((ext_vector_type(4)));
      for (int tile = wave; tile < ntr * ntc; tile += nw) {
        const int t0 = 16 * (tile / ntc), l0 = 16 * (tile % ntc);
        const bool ini = t0 + li < nT, inj = l0 + li < nK;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < na; k0 += 4) {
          const int kk = k0 + lk;
          const double av = (ini && kk < na) ? H[(long)kk * nz + na + t0 + li] : 0.0;
          const double bv = (inj && kk < na) ? KA[(long)kk * ldk + nkkt + l0 + li] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        for (int r = 0; r < 4; ++r) {
          const int i = t0 + lk + 4 * r, j = l0 + li;
          if (i < nT && j < nK) P[(long)i * nK + j] = acc[r];
        }
      }
    }
    __syncthreads();
    double* St = R;  // R is no longer needed
    for (long e = tid; e < (long)nK * nK; e += NT) {
      const int rho = (int)(e / nK), lc = (int)(e % nK);
      const int fr = rho / (3 * mF), cr = (rho / mF) % 3, mr = rho % mF;
      const int fl = lc / (3 * mF), cl = (lc / mF) % 3, ml = lc % mF;
      double v = 0.0;
      if (cr == 0) {
        v = -KA[(long)(na + fr * mF + mr) * ldk + nkkt + lc];
      } else {
        const int t = (fr * 2 + cr - 1) * mF + mr, tr = na + t;
        v = P[(long)t * nK + lc];
        if (cl != 0) v += H[(long)tr * nz + na + (fl * 2 + cl - 1) * mF + ml];
      }
      if (cr == 0 && mr == 0 && cl == 0 && ml == 0)
        v += E.eps_inv / G.vol * (G.sigma[fr] * G.area[fr]) * (G.sigma[fl] * G.area[fl]);
      St[e] = v;
    }
    __syncthreads();
    double* out = S + (long)cell * nK * nK;
    for (long e = tid; e < (long)nK * nK; e += NT) {
      const int rho = (int)(e / nK), lc = (int)(e % nK);
      out[sblk(rho, lc, 3 * mF, nK)] = 0.5 * (St[e] + St[(long)lc * nK + rho]);
    }
  } else if (mode == TET_LOAD) {
    for (int rho = tid; rho < d.nK; rho += NT) {
      const int fr = rho / (3 * mF), cr = (rho / mF) % 3, mr = rho % mF;
      double v;
      if (cr == 0) {
        v = KA[(long)(na + fr * mF + mr) * ldk + nkkt];
      } else {
        const int tr = na + (fr * 2 + cr - 1) * mF + mr;
        double s = 0.0;
        for (int a = 0; a < na; ++a) s += H[(long)a * nz + tr] * KA[(long)a * ldk + nkkt];
        v = -s;
      }
      gK[(long)cell * d.nK + rho] = v;
    }
  } else {
    const double* fq = f;
    (void)fq;
    for (int q = tid; q < nq; q += NT) {
      double u[3] = {0, 0, 0};
      for (int a = 0; a < na; ++a) {
        const double* ua = UQ + 3 * ((long)q * na + a);
        const double c = KA[(long)a * ldk + nkkt];
        u[0] += c * ua[0];
        u[1] += c * ua[1];
        u[2] += c * ua[2];
      }
      for (int dd = 0; dd < 3; ++dd) uo[((long)cell * nq + q) * 3 + dd] = u[dd];
      double pv = p0[cell];
      for (int r = 1; r < nP; ++r) {
        double mean = 0.0;
        for (int qq = 0; qq < nq; ++qq) mean += T.wq[qq] * PSQ[(long)qq * nP + r];
        pv -= KA[(long)(na + d.nN + r - 1) * ldk + nkkt] * (PSQ[(long)q * nP + r] - mean);
      }
      po[(long)cell * nq + q] = pv;
    }
  }
}

// closed-form lowest-order block of one tetrahedron
__global__ void k_cr_blocks3(const double* __restrict__ X, const int* __restrict__ cells, int nc,
                             const double* __restrict__ nu, double beta, double eps_inv, double* A) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double V[4][3];
  int vid[4];
  for (int i = 0; i < 4; ++i) {
    vid[i] = cells[4 * c + i];
    for (int dd = 0; dd < 3; ++dd) V[i][dd] = X[3 * vid[i] + dd];
  }
  double a[3], b[3], e3[3];
  for (int dd = 0; dd < 3; ++dd) {
    a[dd] = V[1][dd] - V[0][dd];
    b[dd] = V[2][dd] - V[0][dd];
    e3[dd] = V[3][dd] - V[0][dd];
  }
  const double vol = fabs(e3[0] * (a[1] * b[2] - a[2] * b[1]) + e3[1] * (a[2] * b[0] - a[0] * b[2]) +
                          e3[2] * (a[0] * b[1] - a[1] * b[0])) / 6.0;
  double fr[4][3][3], q[4], g[4][3];
  for (int i = 0; i < 4; ++i) {
    int w[3], n = 0;
    for (int j = 0; j < 4; ++j)
      if (j != i) w[n++] = j;
    // the face's vertices sorted by global index
    for (int s = 1; s < 3; ++s)
      for (int t = s; t > 0 && vid[w[t]] < vid[w[t - 1]]; --t) {
        int tmp = w[t];
        w[t] = w[t - 1];
        w[t - 1] = tmp;
      }
    double u[3], v[3], nn[3];
    for (int dd = 0; dd < 3; ++dd) {
      u[dd] = V[w[1]][dd] - V[w[0]][dd];
      v[dd] = V[w[2]][dd] - V[w[0]][dd];
    }
    nn[0] = u[1] * v[2] - u[2] * v[1];
    nn[1] = u[2] * v[0] - u[0] * v[2];
    nn[2] = u[0] * v[1] - u[1] * v[0];
    const double ln = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    const double lu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double area = 0.5 * ln;
    for (int dd = 0; dd < 3; ++dd) {
      fr[i][0][dd] = nn[dd] / ln;
      fr[i][1][dd] = u[dd] / lu;
    }
    fr[i][2][0] = fr[i][0][1] * fr[i][1][2] - fr[i][0][2] * fr[i][1][1];
    fr[i][2][1] = fr[i][0][2] * fr[i][1][0] - fr[i][0][0] * fr[i][1][2];
    fr[i][2][2] = fr[i][0][0] * fr[i][1][1] - fr[i][0][1] * fr[i][1][0];
    double o = 0.0;
    for (int dd = 0; dd < 3; ++dd) o += ((V[w[0]][dd] + V[w[1]][dd] + V[w[2]][dd]) / 3.0 - V[i][dd]) * fr[i][0][dd];
    const double sg = o > 0 ? 1.0 : -1.0;
    q[i] = sg * area;
    for (int dd = 0; dd < 3; ++dd) g[i][dd] = q[i] * fr[i][0][dd] / vol;  // grad of 1 - 3 lambda_i
  }
  // RT0 mass: psi_i = (x - V_i) / (3|K|); int_K (x-a).(x-b) = |K|/20 (sum_v |v|^2
  // + |s|^2) - |K| (a+b).xbar + |K| a.b with s the vertex sum, xbar = s/4
  double s[3] = {0, 0, 0}, sv = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int dd = 0; dd < 3; ++dd) {
      s[dd] += V[i][dd];
      sv += V[i][dd] * V[i][dd];
    }
  const double ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
  double Mrt[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double ab = 0.0, axb = 0.0;
      for (int dd = 0; dd < 3; ++dd) {
        ab += V[i][dd] * V[j][dd];
        axb += (V[i][dd] + V[j][dd]) * s[dd] / 4.0;
      }
      Mrt[i][j] = vol * ((sv + ss) / 20.0 - axb + ab) / (9.0 * vol * vol);
    }
  const double nuc = nu[c];
  double* out = A + (long)c * 144;
  for (int i = 0; i < 4; ++i)
    for (int aa = 0; aa < 3; ++aa)
      for (int j = 0; j < 4; ++j)
        for (int bb = 0; bb < 3; ++bb) {
          const double ff = fr[i][aa][0] * fr[j][bb][0] + fr[i][aa][1] * fr[j][bb][1] + fr[i][aa][2] * fr[j][bb][2];
          const double gg = g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2];
          double v = nuc * ff * gg * vol;
          if (aa == 0 && bb == 0) v += beta * q[i] * q[j] * Mrt[i][j] + eps_inv * q[i] * q[j] / vol;
          out[sblk(3 * i + aa, 3 * j + bb, 3, 12)] = v;
        }
}

template <typename TS>
__global__ void __launch_bounds__(64) k_cell_apply3(Level3View<TS> L, const double* __restrict__ x,
                                                    double* __restrict__ yK) {
  __shared__ double xs[12 * MF3MAX];
  const int c = blockIdx.x, lane = threadIdx.x, nK = L.nK, m3 = 3 * L.mF;
  for (int i = lane; i < nK; i += 64) {
    const int dof = L.cell_dofs[4 * c + i / m3];
    xs[i] = dof < 0 ? 0.0 : x[(long)dof * m3 + i % m3];
  }
  __syncthreads();
  const TS* Sc = L.S + (long)c * nK * nK;
  double dx = 0.0;  // d . x_K for the AL term kept apart
  if (L.al > 0.0)
    for (int i = 0; i < 4; ++i) dx += L.cdiv[4 * c + i] * xs[i * m3];
  for (int row = lane; row < nK; row += 64) {
    double acc = 0.0;
    const TS* Sr = Sc + (long)(row / m3) * m3 * nK + row % m3;  // row's face block
    for (int col = 0; col < nK; ++col) acc += (double)Sr[(long)col * m3] * xs[col];
    if (L.al > 0.0 && row % m3 == 0) acc += L.al / L.vol[c] * L.cdiv[4 * c + row / m3] * dx;
    yK[(long)c * nK + row] = acc;
  }
}

// The twelve mode-0 rows of every cell block (local face i, component q:
// row i m3 + q mF), cell-minor so that a wavefront's consecutive cells read
// consecutive words: entry (row i * 3 + q, column col) of cell K at
// S0[(col * 12 + i * 3 + q) * nc + K].
template <typename TS>
__global__ void k_pack_mode0_rows3(int nc, int mF, const TS* __restrict__ S, TS* __restrict__ S0) {
  const int nK = 12 * mF, m3 = 3 * mF;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nc * nK) return;
  const int col = (int)(t / nc), K = (int)(t % nc);
#pragma unroll
  for (int r = 0; r < 12; ++r)
    S0[((long)col * 12 + r) * nc + K] = S[(long)K * nK * nK + sblk((r / 3) * m3 + (r % 3) * mF, col, m3, nK)];
}

// Mode-0 rows of S_K x_K for M0_CELLS cells per workgroup: x_K of the cells
// into LDS (rows padded by one word against bank conflicts), then thread
// (row r, cell j) forms row r of cell j's product from S0 with eight loads
// in flight (a wavefront reads two rows of 32 consecutive cells per word).
// With al > 0 (S0 without its augmented-Lagrangian term) the term is added
// apart on the normal rows, as in the full apply.
constexpr int M0_CELLS = 32;
template <typename TS>
__global__ void __launch_bounds__(12 * M0_CELLS) k_cell_mode0_3(Level3View<TS> L, const TS* __restrict__ S0,
                                                                const double* __restrict__ x,
                                                                double* __restrict__ y0K) {
  __shared__ double xs[M0_CELLS][12 * MF3MAX + 1];
  const int nK = L.nK, m3 = 3 * L.mF, nc = L.nc;
  const int K0 = blockIdx.x * M0_CELLS, tid = threadIdx.x;
  for (int e = tid; e < M0_CELLS * nK; e += 12 * M0_CELLS) {
    const int j = e / nK, i = e % nK, K = min(K0 + j, nc - 1);
    const int dof = L.cell_dofs[4 * K + i / m3];
    xs[j][i] = dof < 0 ? 0.0 : x[(long)dof * m3 + i % m3];
  }
  __syncthreads();
  const int j = tid % M0_CELLS, r = tid / M0_CELLS, K = K0 + j;
  if (K >= nc) return;
  const TS* a = S0 + (long)r * nc + K;
  const long step = 12L * nc;  // next column
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int col = 0;
  for (; col + 8 <= nK; col += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (double)a[(long)(col + u) * step];
    a0 += v[0] * xs[j][col] + v[4] * xs[j][col + 4];
    a1 += v[1] * xs[j][col + 1] + v[5] * xs[j][col + 5];
    a2 += v[2] * xs[j][col + 2] + v[6] * xs[j][col + 6];
    a3 += v[3] * xs[j][col + 3] + v[7] * xs[j][col + 7];
  }
  for (; col < nK; ++col) a0 += (double)a[(long)col * step] * xs[j][col];
  double acc = (a0 + a1) + (a2 + a3);
  if (L.al > 0.0 && r % 3 == 0) {
    double dx = 0.0;
    for (int q = 0; q < 4; ++q) dx += L.cdiv[4 * K + q] * xs[j][q * m3];
    acc += L.al / L.vol[K] * L.cdiv[4 * K + r / 3] * dx;
  }
  y0K[(long)K * 12 + r] = acc;
}

// g0 = mode 0 of (b - A x) from the cells' mode-0 rows (face fi, component
// q: the rows of its two cells); zero_out (if not null) zeroed alike.
__global__ void k_mode0_gather3(int nint, int mF, const int* __restrict__ fcell, const int* __restrict__ floc,
                                const double* __restrict__ y0K, const double* __restrict__ b,
                                double* __restrict__ g0, double* __restrict__ zero_out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3L * nint) return;
  const int fi = (int)(t / 3), q = (int)(t % 3);
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) acc += y0K[(long)fcell[2 * fi + s] * 12 + floc[2 * fi + s] * 3 + q];
  g0[t] = b[(long)fi * 3 * mF + q * mF] - acc;
  if (zero_out) zero_out[t] = 0.0;
}

__global__ void k_blocks_to_dense(int nc, int m3, const double* __restrict__ in, double* __restrict__ out) {
  const int nK = 4 * m3;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nc * nK * nK) return;
  const long c = t / ((long)nK * nK);
  const int e = (int)(t % ((long)nK * nK)), r = e / nK, q = e % nK;
  out[t] = in[c * nK * nK + sblk(r, q, m3, nK)];
}

__global__ void k_f32_blocks_noal(int nc, int mF, const double* __restrict__ S, const double* __restrict__ cdiv,
                                  const double* __restrict__ vol, double al, float* __restrict__ out) {
  const int nK = 12 * mF, m3 = 3 * mF;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nc * nK * nK) return;
  const int c = (int)(t / ((long)nK * nK)), e = (int)(t % ((long)nK * nK));
  // storage position e of the sblk layout -> entry (r, q)
  const int r = e / (m3 * nK) * m3 + e % m3, q = (e % (m3 * nK)) / m3;
  double v = S[t];
  if (r % m3 == 0 && q % m3 == 0) v -= al / vol[c] * cdiv[4 * c + r / m3] * cdiv[4 * c + q / m3];
  out[t] = (float)v;
}

__global__ void k_face_gather3(int nint, int m3, int nK, const int* __restrict__ fcell, const int* __restrict__ floc,
                               const double* __restrict__ yK, double alpha, const double* __restrict__ b,
                               double* __restrict__ y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nint * m3) return;
  const int fi = (int)(t / m3), rr = (int)(t % m3);
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) acc += yK[(long)fcell[2 * fi + s] * nK + floc[2 * fi + s] * m3 + rr];
  y[t] = (b ? b[t] : 0.0) + alpha * acc;
}

constexpr int PMAX_CELLS = 12;  // cells around an edge handled per patch
constexpr int PMAX_FACES = 12;
// limits of the patch-inverse kernel (vertex patches of tetrahedral meshes:
// 24 cells and 36 interior faces around an interior vertex of a Kuhn mesh)
constexpr int PINV_MAX_CELLS = 32;
constexpr int PINV_MAX_FACES = 48;

__global__ void __launch_bounds__(NT) k_patch_inverse3(Level3View<double> L, const int* __restrict__ pf_ptr,
                                                       const int* __restrict__ pf, const int* __restrict__ pc_ptr,
                                                       const int* __restrict__ pc, const long* __restrict__ poff,
                                                       int p0, int ns_max, double* ws, double* pinv,
                                                       int* status) {
  __shared__ int slot[PINV_MAX_CELLS][4];
  __shared__ double pv;
  __shared__ double fct[PINV_MAX_FACES * 3 * MF3MAX];
  const int p = p0 + blockIdx.x, tid = threadIdx.x;
  const int f0 = pf_ptr[p], nf = pf_ptr[p + 1] - f0, c0 = pc_ptr[p], ncl = pc_ptr[p + 1] - c0;
  const int m3 = 3 * L.mF, ns = nf * m3, nK = L.nK, w = 2 * ns;
  double* A = ws + (long)blockIdx.x * ns_max * 2 * ns_max;
  if (nf > PINV_MAX_FACES || ncl > PINV_MAX_CELLS) {
    if (tid == 0) atomicOr(status, 4);
    return;
  }
  for (int e = tid; e < ncl * 4; e += NT) {
    const int ci = e / 4, i = e % 4;
    const int dof = L.cell_dofs[4 * pc[c0 + ci] + i];
    int s = -1;
    for (int q = 0; q < nf; ++q)
      if (pf[f0 + q] == dof) s = q;
    slot[ci][i] = dof < 0 ? -1 : s;
  }
  for (long e = tid; e < (long)ns * w; e += NT) {
    const int r = (int)(e / w), c = (int)(e % w);
    A[e] = c - ns == r ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int ci = 0; ci < ncl; ++ci) {
    const double* Sc = L.S + (long)pc[c0 + ci] * nK * nK;
    for (long e = tid; e < (long)nK * nK; e += NT) {
      // storage position e of the sblk layout -> entry (r, c)
      const int r = (int)(e / ((long)m3 * nK)) * m3 + (int)(e % m3), c = (int)((e % ((long)m3 * nK)) / m3);
      const int sr = slot[ci][r / m3], sc = slot[ci][c / m3];
      if (sr < 0 || sc < 0) continue;
      A[(long)(sr * m3 + r % m3) * w + sc * m3 + c % m3] += Sc[e];
    }
    __syncthreads();
  }
  // A_ss is symmetric positive definite: Gauss-Jordan without pivoting
  for (int j = 0; j < ns; ++j) {
    if (tid == 0) {
      const double v = A[(long)j * w + j];
      if (!(v > 0.0)) atomicOr(status, 2);
      pv = v > 0.0 ? 1.0 / v : 0.0;
    }
    __syncthreads();
    // row j is zero left of column j and right of column ns + j
    const int cw = ns + 1;
    for (int c = j + tid; c <= ns + j; c += NT) A[(long)j * w + c] *= pv;
    for (int i = tid; i < ns; i += NT) fct[i] = i == j ? 0.0 : A[(long)i * w + j];
    __syncthreads();
    for (long e = tid; e < (long)ns * cw; e += NT) {
      const int i = (int)(e / cw), c = j + (int)(e % cw);
      if (i != j) A[(long)i * w + c] -= fct[i] * A[(long)j * w + c];
    }
    __syncthreads();
  }
  double* out = pinv + poff[p];
  for (long e = tid; e < (long)ns * ns; e += NT) {
    const int c = (int)(e / ns), r = (int)(e % ns);
    out[e] = A[(long)r * w + ns + c];  // column c, row r
  }
}

// One edge patch per workgroup of BS threads, the block Gauss-Seidel step
// in its direct form x_s = A_ss^-1 (b_s - A_{s,r} x_r), r the unknowns
// outside the patch (the same value as x_s += A_ss^-1 (b - A x)_s, whose
// A_ss x_s term cancels).  Each patch cell contributes, for the rows of its
// (at most two) patch faces, only the columns of its two far faces (the
// faces that do not contain the edge): half of those rows of S_K, read along
// columns (symmetric blocks), eight loads in flight per thread.  Each
// face's two cells write their contributions to separate LDS slots, so the
// right-hand side is b - side0 - side1.
template <typename TS, typename TP, int BS, int MFC>
__global__ void __launch_bounds__(BS) k_patch_gs3(Level3View<TS> L, const int* __restrict__ pf_ptr,
                                                  const int* __restrict__ pf, const int* __restrict__ pc_ptr,
                                                  const int* __restrict__ pc, const long* __restrict__ poff,
                                                  const TP* __restrict__ pinv, int p0, double* x,
                                                  const double* __restrict__ b, int from_zero) {
  // from_zero: x is zero on every face the patches see, so the patch
  // residual is b_s and the cell blocks are not read.
  // LDS sized for at most MFC face modes (the launch picks the smallest
  // instance that fits the level): at lowest order 2 KB instead of 20 KB, so
  // that a CU holds many more of these latency-bound wavefronts
  constexpr int MFL = MFC;
  __shared__ int slot[PMAX_CELLS][4];
  __shared__ int cellid[PMAX_CELLS];
  __shared__ double xs[PMAX_CELLS][12 * MFL];
  __shared__ double res[PMAX_FACES * 3 * MFL];
  __shared__ double side[2][PMAX_FACES * 3 * MFL];
  const int p = p0 + blockIdx.x, tid = threadIdx.x;
  const int f0 = pf_ptr[p], nf = pf_ptr[p + 1] - f0, c0 = pc_ptr[p], ncl = pc_ptr[p + 1] - c0;
  const int m3 = 3 * L.mF, ns = nf * m3, nK = L.nK;
  if (nf > PMAX_FACES || ncl > PMAX_CELLS) return;  // rejected on the host
  const int ncx = from_zero ? 0 : ncl;
  for (int e = tid; e < ncx * 4; e += BS) {
    const int ci = e / 4, i = e % 4;
    const int cell = pc[c0 + ci];
    if (i == 0) cellid[ci] = cell;
    const int dof = L.cell_dofs[4 * cell + i];
    int sl = -1;
    for (int q = 0; q < nf; ++q)
      if (pf[f0 + q] == dof) sl = q;
    slot[ci][i] = dof < 0 ? -2 : sl;  // -2: boundary face, -1: interior face outside the patch
  }
  for (int e = tid; e < ncx * nK; e += BS) {
    const int ci = e / nK, i = e % nK;
    const int dof = L.cell_dofs[4 * pc[c0 + ci] + i / m3];
    xs[ci][i] = dof < 0 ? 0.0 : x[(long)dof * m3 + i % m3];
  }
  for (int q = tid; q < ns; q += BS) {
    res[q] = b[(long)pf[f0 + q / m3] * m3 + q % m3];
    side[0][q] = 0.0;
    side[1][q] = 0.0;
  }
  __syncthreads();
  const int nitem = ncx * 2 * m3;
  for (int it = tid; it < nitem; it += BS) {
    const int ci = it / (2 * m3), which = (it / m3) % 2, rr = it % m3;
    // the patch face `which` of the cell, and its far faces (the interior
    // faces of the cell outside the patch: the two faces that do not
    // contain the edge, less boundary faces)
    int i = -1, cnt = 0, q0 = 0, q1 = 0, nfar = 0;
    for (int q = 0; q < 4; ++q) {
      const int sq = slot[ci][q];
      if (sq >= 0) {
        if (cnt == which) i = q;
        ++cnt;
      } else if (sq == -1) {
        if (nfar == 0) q0 = q;
        else q1 = q;
        ++nfar;
      }
    }
    if (i < 0) continue;
    const int cell = cellid[ci];
    // face i's row block: rows contiguous, columns m3 apart; only the columns
    // of the far faces (x on the patch faces enters through A_ss)
    const TS* Sc = L.S + (long)cell * nK * nK + (long)i * m3 * nK + rr;
    const double* xc = xs[ci];
    const int ncol = min(nfar, 2) * m3;  // at most two (a tetrahedron's faces off the edge)
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int t = 0;
    for (; t + 8 <= ncol; t += 8) {
      double v[8];
      int cl[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int tt = t + u;
        cl[u] = tt < m3 ? q0 * m3 + tt : q1 * m3 + tt - m3;
        v[u] = (double)Sc[(long)cl[u] * m3];
      }
      a0 += v[0] * xc[cl[0]] + v[4] * xc[cl[4]];
      a1 += v[1] * xc[cl[1]] + v[5] * xc[cl[5]];
      a2 += v[2] * xc[cl[2]] + v[6] * xc[cl[6]];
      a3 += v[3] * xc[cl[3]] + v[7] * xc[cl[7]];
    }
    for (; t < ncol; ++t) {
      const int c = t < m3 ? q0 * m3 + t : q1 * m3 + t - m3;
      a0 += (double)Sc[(long)c * m3] * xc[c];
    }
    double acc = (a0 + a1) + (a2 + a3);
    if (L.al > 0.0 && rr == 0) {
      double dx = 0.0;
      if (nfar > 0) dx += L.cdiv[4 * cell + q0] * xc[q0 * m3];
      if (nfar > 1) dx += L.cdiv[4 * cell + q1] * xc[q1 * m3];
      acc += L.al / L.vol[cell] * L.cdiv[4 * cell + i] * dx;
    }
    const int dof = L.cell_dofs[4 * cell + i];
    const int sd = L.fcell[2 * dof] == cell ? 0 : 1;
    side[sd][slot[ci][i] * m3 + rr] = acc;
  }
  __syncthreads();
  for (int q = tid; q < ns; q += BS) res[q] -= side[0][q] + side[1][q];
  __syncthreads();
  const TP* Ai = pinv + poff[p];
  for (int q = tid; q < ns; q += BS) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = 0;
    // eight columns' loads in flight per step (the same four accumulators in
    // the same order as the four-column steps below)
    for (; j + 8 <= ns; j += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (double)Ai[(long)(j + u) * ns + q];
      a0 += v[0] * res[j];
      a1 += v[1] * res[j + 1];
      a2 += v[2] * res[j + 2];
      a3 += v[3] * res[j + 3];
      a0 += v[4] * res[j + 4];
      a1 += v[5] * res[j + 5];
      a2 += v[6] * res[j + 6];
      a3 += v[7] * res[j + 7];
    }
    for (; j + 4 <= ns; j += 4) {
      const double v0 = (double)Ai[(long)j * ns + q], v1 = (double)Ai[(long)(j + 1) * ns + q];
      const double v2 = (double)Ai[(long)(j + 2) * ns + q], v3 = (double)Ai[(long)(j + 3) * ns + q];
      a0 += v0 * res[j];
      a1 += v1 * res[j + 1];
      a2 += v2 * res[j + 2];
      a3 += v3 * res[j + 3];
    }
    for (; j < ns; ++j) a0 += (double)Ai[(long)j * ns + q] * res[j];
    x[(long)pf[f0 + q / m3] * m3 + q % m3] = (a0 + a1) + (a2 + a3);
  }
}

// One item of the lowest-order phase below: row rr of the patch face
// `which` of a patch cell (record rc: cell, code, far-face unknowns) times x
// on the cell's far faces (+ the AL coupling when it is kept apart), into
// side[sd][slot].  Absent far faces read a valid column and weigh it by 0.
template <typename TS>
__device__ __forceinline__ void gs3_lo_item(const Level3View<TS>& L, bool live, int which, int rr, int4 rc,
                                            const double* x, double (*side)[PMAX_FACES * 3]) {
  const int cell = rc.x, code = rc.y;
  const int i = (code >> (2 * which)) & 3, s = (code >> (4 + 4 * which)) & 15, sd = (code >> (12 + which)) & 1;
  const int q0 = (code >> 14) & 3, q1 = (code >> 16) & 3, nfar = (code >> 18) & 3;
  // row rr of face i's row block; column c at c * 3
  const TS* Sc = L.S + (long)cell * 144 + i * 36 + rr;
  double v[6], xc[6];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    v[u] = (double)Sc[(q0 * 3 + u) * 3];
    v[3 + u] = (double)Sc[(q1 * 3 + u) * 3];
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const double t0 = x[(long)max(rc.z, 0) * 3 + u], t1 = x[(long)max(rc.w, 0) * 3 + u];
    xc[u] = nfar > 0 ? t0 : 0.0;
    xc[3 + u] = nfar > 1 ? t1 : 0.0;
  }
  double cd0 = 0.0, cd1 = 0.0, cdi = 0.0, vK = 1.0;
  if (L.al > 0.0) {
    double c4[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) c4[f] = L.cdiv[4 * cell + f];
    cd0 = q0 == 0 ? c4[0] : q0 == 1 ? c4[1] : q0 == 2 ? c4[2] : c4[3];
    cd1 = q1 == 0 ? c4[0] : q1 == 1 ? c4[1] : q1 == 2 ? c4[2] : c4[3];
    cdi = i == 0 ? c4[0] : i == 1 ? c4[1] : i == 2 ? c4[2] : c4[3];
    vK = L.vol[cell];
  }
  double acc = (v[0] * xc[0] + v[1] * xc[1] + v[2] * xc[2]) + (v[3] * xc[3] + v[4] * xc[4] + v[5] * xc[5]);
  if (L.al > 0.0 && rr == 0) acc += L.al / vK * cdi * (cd0 * xc[0] + cd1 * xc[3]);
  if (live && s < 15) side[sd][s * 3 + rr] = acc;
}

// The same colour phase at lowest order (one mode per face component: 3
// unknowns per face, 12 per cell), a wavefront per patch.  A record built
// at set-up per patch cell (the cell; its two patch faces with their slots
// in the patch and sides; its far faces and their unknown numbers) makes
// every load at most two round trips deep (the patch's ranges, then its
// records and face list), and each lane issues its six row entries, six
// far-face values and its row of the patch inverse together; the direct
// form as in k_patch_gs3 (from_zero as there: the items are skipped).
template <typename TS, typename TP>
__global__ void __launch_bounds__(64) k_patch_gs3_lo(Level3View<TS> L, const int* __restrict__ pf_ptr,
                                                     const int* __restrict__ pf, const int* __restrict__ pc_ptr,
                                                     const int4* __restrict__ prec, const long* __restrict__ poff,
                                                     const TP* __restrict__ pinv, int p0, double* x,
                                                     const double* __restrict__ b, int from_zero) {
  __shared__ double res[PMAX_FACES * 3];
  __shared__ double side[2][PMAX_FACES * 3];
  const int p = p0 + blockIdx.x, lane = threadIdx.x;
  // the patch's ranges and inverse offset, loaded together
  const int f0 = pf_ptr[p], f1 = pf_ptr[p + 1], c0 = pc_ptr[p], c1 = pc_ptr[p + 1];
  const long po = poff[p];
  const int nf = f1 - f0, ncl = c1 - c0;
  if (nf < 1 || nf > PMAX_FACES || ncl < 1 || ncl > PMAX_CELLS) return;  // rejected on the host
  const int ns = 3 * nf, nit = 6 * ncl;
  // first: the face of this lane's patch unknown (lanes past ns: a copy of
  // the last, unused) and the record of its first item
  const int q = min(lane, ns - 1);
  const int fq = pf[f0 + q / 3];
  const int4 rcA = prec[c0 + min(lane / 6, ncl - 1)];
  // then its row of the patch inverse, every column index clamped into the
  // row: the loads carry no branch, so that waiting for any later load does
  // not wait for these (columns past ns are read again and not used)
  const TP* Ai = pinv + po;
  double av[3 * PMAX_FACES];
#pragma unroll
  for (int j = 0; j < 3 * PMAX_FACES; ++j) av[j] = (double)Ai[(long)min(j, ns - 1) * ns + q];
  const long xq = (long)fq * 3 + q % 3;
  const double bq = b[xq];
  if (lane < ns) {
    side[0][lane] = 0.0;
    side[1][lane] = 0.0;
  }
  __syncthreads();
  if (!from_zero) gs3_lo_item(L, lane < nit, (lane / 3) & 1, lane % 3, rcA, x, side);
  if (!from_zero && nit > 64) {  // more than ten cells around the edge
    const int it = 64 + lane;
    gs3_lo_item(L, it < nit, (it / 3) & 1, it % 3, prec[c0 + min(it / 6, ncl - 1)], x, side);
  }
  __syncthreads();
  if (lane < ns) res[lane] = bq - (side[0][lane] + side[1][lane]);
  __syncthreads();
  if (lane < ns) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int n4 = ns / 4 * 4;
#pragma unroll
    for (int j = 0; j < 3 * PMAX_FACES; j += 4)
      if (j < n4) {
        a0 += av[j] * res[j];
        a1 += av[j + 1] * res[j + 1];
        a2 += av[j + 2] * res[j + 2];
        a3 += av[j + 3] * res[j + 3];
      }
#pragma unroll
    for (int j = 0; j < 3 * PMAX_FACES; ++j)
      if (j >= n4 && j < ns) a0 += av[j] * res[j];
    x[xq] = (a0 + a1) + (a2 + a3);
  }
}

__global__ void k_mode0_extract3(int n, int mF, const double* __restrict__ r, double* __restrict__ g0,
                                 double* __restrict__ zero_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  g0[t] = r[(long)t * mF];
  if (zero_out) zero_out[t] = 0.0;
}

__global__ void k_mode0_add3(int n, int mF, const double* __restrict__ u0, double* __restrict__ x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  x[(long)t * mF] += u0[t];
}

__global__ void k_uzawa_rhs3(int nint, int mF, const double* __restrict__ g, const double* __restrict__ fdiv,
                             const int* __restrict__ fcell, const double* __restrict__ p0, double* b) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m3 = 3 * mF;
  if (t >= (long)nint * m3) return;
  double v = g[t];
  if (t % m3 == 0) {
    const int fi = (int)(t / m3);
    v += fdiv[2 * fi] * p0[fcell[2 * fi]] + fdiv[2 * fi + 1] * p0[fcell[2 * fi + 1]];
  }
  b[t] = v;
}

__global__ void __launch_bounds__(256) k_uzawa_update3(int nc, int mF, const int* __restrict__ cell_dofs,
                                                       const double* __restrict__ cdiv,
                                                       const double* __restrict__ vol,
                                                       const double* __restrict__ lam, double eps_inv, double* p0,
                                                       double* part) {
  __shared__ double sh[2][256];
  double s1 = 0.0, s2 = 0.0;
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long)gridDim.x * blockDim.x) {
    double dv = 0.0;
    for (int i = 0; i < 4; ++i) {
      const int dof = cell_dofs[4 * c + i];
      if (dof >= 0) dv += cdiv[4 * c + i] * lam[(long)dof * 3 * mF];
    }
    const double dp = -eps_inv * dv / vol[c];
    const double pn = p0[c] + dp;
    p0[c] = pn;
    s1 += vol[c] * dp * dp;
    s2 += vol[c] * pn * pn;
  }
  sh[0][threadIdx.x] = s1;
  sh[1][threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sh[0][0];
    part[gridDim.x + blockIdx.x] = sh[1][0];
  }
}

__global__ void k_f32_copy(long n, const double* __restrict__ in, float* __restrict__ out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = (float)in[t];
}

inline int blocks(long n, int tpb) { return (int)((n + tpb - 1) / tpb); }

}  // namespace

long tet_ws_words(int k, int mode) { return ws_layout(k, mode).total; }

void launch_tet_local(hipStream_t st, const TetCells& E, int mode, int c0, int nb, double* ws, const double* f,
                      const double* lam, const double* p0, double* S, double* gK, double* u, double* p,
                      int* status) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_tet_local, dim3(nb), dim3(NT), 0, st, E, mode, c0, ws, f, lam, p0, S, gK, u, p, status);
}

void launch_cr_blocks3(hipStream_t st, const double* X, const int* cells, int nc, const double* nu_cells,
                       double beta, double eps_inv, double* A) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_cr_blocks3, dim3(blocks(nc, 128)), dim3(128), 0, st, X, cells, nc, nu_cells, beta, eps_inv,
                     A);
}

template <typename TS>
void launch_cell_apply3(hipStream_t st, Level3View<TS> L, const double* x, double* yK) {
  if (L.nc <= 0) return;
  hipLaunchKernelGGL(k_cell_apply3<TS>, dim3(L.nc), dim3(64), 0, st, L, x, yK);
}
template void launch_cell_apply3<double>(hipStream_t, Level3View<double>, const double*, double*);
template void launch_cell_apply3<float>(hipStream_t, Level3View<float>, const double*, double*);

template <typename TS>
void launch_pack_mode0_rows3(hipStream_t st, int nc, int mF, const TS* S, TS* S0) {
  const long n = (long)nc * 12 * mF;
  if (n > 0) hipLaunchKernelGGL(k_pack_mode0_rows3<TS>, dim3(blocks(n, 256)), dim3(256), 0, st, nc, mF, S, S0);
}
template void launch_pack_mode0_rows3<double>(hipStream_t, int, int, const double*, double*);
template void launch_pack_mode0_rows3<float>(hipStream_t, int, int, const float*, float*);

template <typename TS>
void launch_mode0_residual3(hipStream_t st, Level3View<TS> L, const TS* S0, const double* x, double* y0K,
                            const double* b, double* g0, double* zero_out) {
  if (L.nc > 0)
    hipLaunchKernelGGL(k_cell_mode0_3<TS>, dim3((L.nc + M0_CELLS - 1) / M0_CELLS), dim3(12 * M0_CELLS), 0, st, L, S0,
                       x, y0K);
  const long n = 3L * L.nint;
  if (n > 0)
    hipLaunchKernelGGL(k_mode0_gather3, dim3(blocks(n, 256)), dim3(256), 0, st, L.nint, L.mF, L.fcell, L.floc, y0K,
                       b, g0, zero_out);
}
template void launch_mode0_residual3<double>(hipStream_t, Level3View<double>, const double*, const double*, double*,
                                             const double*, double*, double*);
template void launch_mode0_residual3<float>(hipStream_t, Level3View<float>, const float*, const double*, double*,
                                            const double*, double*, double*);

void launch_blocks_to_dense(hipStream_t st, int nc, int m3, const double* in, double* out) {
  const long n = (long)nc * 16 * m3 * m3;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_blocks_to_dense, dim3(blocks(n, 256)), dim3(256), 0, st, nc, m3, in, out);
}

void launch_face_gather3(hipStream_t st, int nint, int mF, int nK, const int* fcell, const int* floc,
                         const double* yK, double alpha, const double* b, double* y) {
  const long n = (long)nint * 3 * mF;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_face_gather3, dim3(blocks(n, 256)), dim3(256), 0, st, nint, 3 * mF, nK, fcell, floc, yK,
                     alpha, b, y);
}

void launch_patch_inverse3(hipStream_t st, Level3View<double> L, const int* pf_ptr, const int* pf,
                           const int* pc_ptr, const int* pc, const long* poff, int p0, int np, int ns_max,
                           double* ws, double* pinv, int* status) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_patch_inverse3, dim3(np), dim3(NT), 0, st, L, pf_ptr, pf, pc_ptr, pc, poff, p0, ns_max, ws,
                     pinv, status);
}

template <typename TS, typename TP>
void launch_patch_gs3(hipStream_t st, Level3View<TS> L, const int* pf_ptr, const int* pf, const int* pc_ptr,
                      const int* pc, const long* poff, const TP* pinv, int p0, int p1, double* x,
                      const double* b, bool from_zero) {
  if (p1 <= p0) return;
  // lowest-order patches (at most 36 unknowns): a wavefront each; order k:
  // a workgroup of NT with LDS for the level's face modes
#define GS3(B, M)                                                                                          \
  hipLaunchKernelGGL((k_patch_gs3<TS, TP, B, M>), dim3(p1 - p0), dim3(B), 0, st, L, pf_ptr, pf, pc_ptr, pc, poff, \
                     pinv, p0, x, b, from_zero ? 1 : 0)
  if (L.mF == 1)
    GS3(64, 1);
  else if (L.mF <= 3)
    GS3(NT, 3);
  else if (L.mF <= 6)
    GS3(NT, 6);
  else
    GS3(NT, MF3MAX);
#undef GS3
}
template void launch_patch_gs3<double, double>(hipStream_t, Level3View<double>, const int*, const int*, const int*,
                                               const int*, const long*, const double*, int, int, double*,
                                               const double*, bool);
template void launch_patch_gs3<float, float>(hipStream_t, Level3View<float>, const int*, const int*, const int*,
                                             const int*, const long*, const float*, int, int, double*,
                                             const double*, bool);
template void launch_patch_gs3<float, double>(hipStream_t, Level3View<float>, const int*, const int*, const int*,
                                              const int*, const long*, const double*, int, int, double*,
                                              const double*, bool);

template <typename TS, typename TP>
void launch_patch_gs3_lo(hipStream_t st, Level3View<TS> L, const int* pf_ptr, const int* pf, const int* pc_ptr,
                         const int* prec, const long* poff, const TP* pinv, int p0, int p1, double* x,
                         const double* b, bool from_zero) {
  if (p1 <= p0) return;
  hipLaunchKernelGGL((k_patch_gs3_lo<TS, TP>), dim3(p1 - p0), dim3(64), 0, st, L, pf_ptr, pf, pc_ptr,
                     reinterpret_cast<const int4*>(prec), poff, pinv, p0, x, b, from_zero ? 1 : 0);
}
template void launch_patch_gs3_lo<double, double>(hipStream_t, Level3View<double>, const int*, const int*,
                                                  const int*, const int*, const long*, const double*, int, int,
                                                  double*, const double*, bool);
template void launch_patch_gs3_lo<float, float>(hipStream_t, Level3View<float>, const int*, const int*, const int*,
                                                const int*, const long*, const float*, int, int, double*,
                                                const double*, bool);
template void launch_patch_gs3_lo<float, double>(hipStream_t, Level3View<float>, const int*, const int*,
                                                 const int*, const int*, const long*, const double*, int, int,
                                                 double*, const double*, bool);

void launch_mode0_extract3(hipStream_t st, int nint, int mF, const double* r, double* g0, double* zero_out) {
  const int n = 3 * nint;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mode0_extract3, dim3(blocks(n, 256)), dim3(256), 0, st, n, mF, r, g0, zero_out);
}

void launch_mode0_add3(hipStream_t st, int nint, int mF, const double* u0, double* x) {
  const int n = 3 * nint;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mode0_add3, dim3(blocks(n, 256)), dim3(256), 0, st, n, mF, u0, x);
}

void launch_uzawa_rhs3(hipStream_t st, int nint, int mF, const double* g, const double* fdiv, const int* fcell,
                       const double* p0, double* b) {
  const long n = (long)nint * 3 * mF;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_uzawa_rhs3, dim3(blocks(n, 256)), dim3(256), 0, st, nint, mF, g, fdiv, fcell, p0, b);
}

void launch_uzawa_update3(hipStream_t st, int nc, int mF, const int* cell_dofs, const double* cdiv,
                          const double* vol, const double* lam, double eps_inv, double* p0, double* part, int nb) {
  hipLaunchKernelGGL(k_uzawa_update3, dim3(nb), dim3(256), 0, st, nc, mF, cell_dofs, cdiv, vol, lam, eps_inv, p0,
                     part);
}

void launch_f32_blocks_noal(hipStream_t st, int nc, int mF, const double* S, const double* cdiv, const double* vol,
                            double al, float* out) {
  const long n = (long)nc * 144 * mF * mF;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_f32_blocks_noal, dim3(blocks(n, 256)), dim3(256), 0, st, nc, mF, S, cdiv, vol, al, out);
}

void launch_f32_copy(hipStream_t st, long n, const double* in, float* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_f32_copy, dim3(blocks(n, 256)), dim3(256), 0, st, n, in, out);
}

}  // namespace hdgmg
