// Device kernels of the skeleton solve (FP64).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace hdgmg {

namespace {

constexpr int TPB = 256;

inline int nblk(long n, int tpb = TPB) { return (int)((n + tpb - 1) / tpb); }

__global__ void k_condense(ElemLevel E, int c0, int nbatch, double* ws, double* S, int* status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbatch) return;
  int c = c0 + t;
  CellGeom g;
  cell_geom(E.X, E.cells + 3 * c, g);
  const int nK = 6 * (E.Q.k + 1);
  double nuc = E.nu_per_cell ? E.nu[c] : E.nu[0];
  const WS fv{E.fac ? E.fac + c : nullptr, E.nc};
  int rc = element_local(E.Q, g, nuc, E.beta, E.eps_inv, EL_CONDENSE, nullptr, nullptr, 0.0, WS{ws + t, nbatch},
                         S + (long)c * nK * nK, nullptr, nullptr, E.CT, E.wcoef ? E.wcoef + (long)c * E.na : nullptr,
                         E.fac ? &fv : nullptr, E.transpose != 0, E.oflag ? E.oflag[c] : 0);
  if (rc) atomicOr(status, 1);
}

// local tangential boundary values of cell c in the block's local order
__device__ inline void boundary_local(const ElemLevel& E, int c, double* lb) {
  const int m = E.m;
  for (int i = 0; i < 6 * m; ++i) lb[i] = 0.0;
  if (!E.bdl) return;
  for (int i = 0; i < 3; ++i)
    for (int cc = 0; cc < 2; ++cc)
      for (int j = 0; j < m; ++j) lb[(i * 2 + cc) * m + j] = E.bdl[(((long)c * 3 + i) * 2 + cc) * m + j];
}

__global__ void k_load(ElemLevel E, int c0, int nbatch, const double* __restrict__ f, double* ws, double* gK,
                       int* status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbatch) return;
  int c = c0 + t;
  CellGeom g;
  cell_geom(E.X, E.cells + 3 * c, g);
  const int nK = 6 * (E.Q.k + 1);
  double nuc = E.nu_per_cell ? E.nu[c] : E.nu[0];
  double* out = gK + (long)c * nK;
  if (E.fac) {
    const WS nx{E.nw_load ? E.nw_load + c : nullptr, E.nc};
    element_cached(E.Q, g, EL_LOAD, f + (long)c * E.Q.nq * 2, nullptr, 0.0, WS{E.fac + c, E.nc},
                   WS{ws + t, nbatch}, out, E.nw_load ? &nx : nullptr);
  } else {
    int rc = element_local(E.Q, g, nuc, E.beta, 0.0, EL_LOAD, f + (long)c * E.Q.nq * 2, nullptr, 0.0,
                           WS{ws + t, nbatch}, out, nullptr, nullptr, E.CT,
                           E.wcoef ? E.wcoef + (long)c * E.na : nullptr, nullptr, E.transpose != 0, E.oflag ? E.oflag[c] : 0);
    if (rc) atomicOr(status, 1);
  }
  if (E.bdl) {
    double lb[6 * (KMAX + 1)];
    boundary_local(E, c, lb);
    const double* SK = E.S + (long)c * nK * nK;
    for (int r = 0; r < nK; ++r) {
      double s = 0.0;
      for (int q = 0; q < nK; ++q) s += SK[(long)r * nK + q] * lb[q];
      out[r] -= s;
    }
  }
}

__global__ void k_recover(ElemLevel E, int c0, int nbatch, const double* __restrict__ f,
                          const double* __restrict__ lam, const double* __restrict__ p0, double* ws, double* u,
                          double* p, int* status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbatch) return;
  int c = c0 + t;
  const int m = E.m;
  CellGeom g;
  cell_geom(E.X, E.cells + 3 * c, g);
  double lk[6 * (KMAX + 1)];
  boundary_local(E, c, lk);
  for (int i = 0; i < 3; ++i) {
    int d = E.cell_dofs[3 * c + i];
    if (d < 0) continue;
    for (int cc = 0; cc < 2; ++cc)
      for (int j = 0; j < m; ++j) lk[(i * 2 + cc) * m + j] = lam[((long)d * 2 + cc) * m + j];
  }
  double out[3 * NQ_MAX];
  double nuc = E.nu_per_cell ? E.nu[c] : E.nu[0];
  if (E.fac) {
    const WS nx{E.nw_load ? E.nw_load + c : nullptr, E.nc};
    element_cached(E.Q, g, EL_RECOVER, f + (long)c * E.Q.nq * 2, lk, p0[c], WS{E.fac + c, E.nc},
                   WS{ws + t, nbatch}, out, E.nw_load ? &nx : nullptr);
  } else {
    int rc = element_local(E.Q, g, nuc, E.beta, 0.0, EL_RECOVER, f + (long)c * E.Q.nq * 2, lk, p0[c],
                           WS{ws + t, nbatch}, out, nullptr, nullptr, E.CT,
                           E.wcoef ? E.wcoef + (long)c * E.na : nullptr, nullptr, E.transpose != 0, E.oflag ? E.oflag[c] : 0);
    if (rc) atomicOr(status, 1);
  }
  for (int q = 0; q < E.Q.nq; ++q) {
    u[((long)c * E.Q.nq + q) * 2] = out[2 * q];
    u[((long)c * E.Q.nq + q) * 2 + 1] = out[2 * q + 1];
    p[(long)c * E.Q.nq + q] = out[2 * E.Q.nq + q];
  }
}

// u* (stPost) at the data points of every cell of the batch: the local
// solve from the skeleton data (and the prescribed boundary values), then
// the P^{k+1} post-processing; out [nc][nq][2].
__global__ void k_postprocess(ElemLevel E, int c0, int nbatch, const double* __restrict__ f,
                              const double* __restrict__ lam, double* ws, double* ustar, int* status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbatch) return;
  int c = c0 + t;
  const int m = E.m;
  CellGeom g;
  cell_geom(E.X, E.cells + 3 * c, g);
  double lk[6 * (KMAX + 1)];
  boundary_local(E, c, lk);
  for (int i = 0; i < 3; ++i) {
    int d = E.cell_dofs[3 * c + i];
    if (d < 0) continue;
    for (int cc = 0; cc < 2; ++cc)
      for (int j = 0; j < m; ++j) lk[(i * 2 + cc) * m + j] = lam[((long)d * 2 + cc) * m + j];
  }
  double nuc = E.nu_per_cell ? E.nu[c] : E.nu[0];
  int rc = element_local(E.Q, g, nuc, E.beta, 0.0, EL_POSTPROCESS, f + (long)c * E.Q.nq * 2, lk, 0.0,
                         WS{ws + t, nbatch}, ustar + (long)c * E.Q.nq * 2, nullptr, nullptr, E.CT,
                         E.wcoef ? E.wcoef + (long)c * E.na : nullptr, nullptr, E.transpose != 0, E.oflag ? E.oflag[c] : 0);
  if (rc) atomicOr(status, 1);
}

__global__ void k_wind_fit(QuadTables Q, const double* __restrict__ X, const int* __restrict__ cells, int c0,
                           int nbatch, const double* __restrict__ vals, double* ws, double* coef, int* status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbatch) return;
  const int c = c0 + t;
  CellGeom g;
  cell_geom(X, cells + 3 * c, g);
  const int na = dims_of(Q.k).na;
  if (wind_fit(Q, g, vals + (long)c * Q.nq * 2, WS{ws + t, nbatch}, coef + (long)c * na)) atomicOr(status, 1);
}

__global__ void k_wind_rt0(QuadTables Q0, const double* __restrict__ X, const int* __restrict__ cells,
                           const int* __restrict__ cell_dofs, int c0, int nbatch, const double* __restrict__ flux,
                           double* ws, double* coef, int* status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbatch) return;
  const int c = c0 + t;
  CellGeom g;
  cell_geom(X, cells + 3 * c, g);
  // the RT0 field with outward flux phi_i through local facet i:
  // sum_i phi_i (x - x_i) / (2|K|), x_i the vertex opposite facet i
  double phi[3], xv[3][2];
  for (int i = 0; i < 3; ++i) {
    int d = cell_dofs[3 * c + i];
    phi[i] = d >= 0 ? g.sigma[i] * flux[d] : 0.0;
    xv[i][0] = X[2 * cells[3 * c + i]];
    xv[i][1] = X[2 * cells[3 * c + i] + 1];
  }
  double vals[2 * NQ_MAX];
  for (int q = 0; q < Q0.nq; ++q) {
    double x1 = Q0.xi[q][0], x2 = Q0.xi[q][1];
    double xp[2] = {g.Xs0[0] + g.J[0][0] * x1 + g.J[0][1] * x2, g.Xs0[1] + g.J[1][0] * x1 + g.J[1][1] * x2};
    double wx = 0.0, wy = 0.0;
    for (int i = 0; i < 3; ++i) {
      wx += phi[i] * (xp[0] - xv[i][0]);
      wy += phi[i] * (xp[1] - xv[i][1]);
    }
    vals[2 * q] = wx / (2.0 * g.area);
    vals[2 * q + 1] = wy / (2.0 * g.area);
  }
  if (wind_fit(Q0, g, vals, WS{ws + t, nbatch}, coef + (long)c * 3)) atomicOr(status, 1);
}

__global__ void k_facet_flux(QuadTables Q, const double* __restrict__ X, const int* __restrict__ cells,
                             const int* __restrict__ fcell, const int* __restrict__ floc, int nint,
                             const double* __restrict__ coef, int na, double* __restrict__ flux) {
  int fi = blockIdx.x * blockDim.x + threadIdx.x;
  if (fi >= nint) return;
  const int c = fcell[2 * fi], i = floc[2 * fi];
  CellGeom g;
  cell_geom(X, cells + 3 * c, g);
  const Dims D = dims_of(Q.k);
  const double* wc = coef + (long)c * na;
  double u[2 * 40], gr[4 * 40], mono[16];
  double s_ = 0.0;
  for (int l = 0; l < Q.nfq; ++l) {
    double s = Q.s[l];
    double xp[2] = {g.P0[i][0] + s * (g.P1[i][0] - g.P0[i][0]), g.P0[i][1] + s * (g.P1[i][1] - g.P0[i][1])};
    double dx = xp[0] - g.Xs0[0], dy = xp[1] - g.Xs0[1];
    double x1 = g.Ji[0][0] * dx + g.Ji[0][1] * dy;
    double x2 = g.Ji[1][0] * dx + g.Ji[1][1] * dy;
    rt_basis(D, g, x1, x2, xp, u, gr, mono);
    double wn = 0.0;
    for (int a = 0; a < na; ++a) wn += wc[a] * (u[2 * a] * g.n[i][0] + u[2 * a + 1] * g.n[i][1]);
    s_ += Q.ws[l] * wn;
  }
  flux[fi] = s_ * g.len[i];
}

__global__ void k_bd_local(int nc, int m, const int* __restrict__ cbf, const double* __restrict__ uhat_b, int full,
                           double* __restrict__ bdl) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nc * 3 * 2 * m) return;
  const long ci = t / (2 * m);
  const int cc = (int)(t / m % 2), j = (int)(t % m);
  const int b = cbf[ci];
  double v = 0.0;
  if (b >= 0) v = full ? uhat_b[((long)b * 2 + cc) * m + j] : (cc == 1 ? uhat_b[(long)b * m + j] : 0.0);
  bdl[t] = v;
}

// flux of the prescribed normal values out of each cell: sum_i sigma|F_i| c^n_i,0
__global__ void k_bd_flux(int nc, int m, const double* __restrict__ bdiv, const double* __restrict__ bdl,
                          double* __restrict__ cflux) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double s = 0.0;
  for (int i = 0; i < 3; ++i) s += bdiv[3 * c + i] * bdl[((c * 3 + i) * 2) * m];
  cflux[c] = s;
}

// gnu[c] += -(Lift z, Lift z_adj)_K for the forward state (f, lam) and the
// adjoint state (fa, lama) of every cell of the batch.  With a wind the
// forward state is recovered with the cell's own local system and the
// adjoint state with its transpose; prescribed boundary values (E.bdl)
// belong to the forward state only (the adjoint's are zero).
__global__ void k_gradnu(ElemLevel E, int c0, int nbatch, const double* __restrict__ f,
                         const double* __restrict__ lam, const double* __restrict__ fa,
                         const double* __restrict__ lama, double* ws, double* gnu, int* status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbatch) return;
  int c = c0 + t;
  const int m = E.m;
  CellGeom g;
  cell_geom(E.X, E.cells + 3 * c, g);
  double lk[6 * (KMAX + 1)], la[6 * (KMAX + 1)];
  boundary_local(E, c, lk);
  for (int i = 0; i < 6 * m; ++i) la[i] = 0.0;
  for (int i = 0; i < 3; ++i) {
    int d = E.cell_dofs[3 * c + i];
    if (d < 0) continue;
    for (int cc = 0; cc < 2; ++cc)
      for (int j = 0; j < m; ++j) {
        const long gi = ((long)d * 2 + cc) * m + j;
        lk[(i * 2 + cc) * m + j] = lam[gi];
        la[(i * 2 + cc) * m + j] = lama[gi];
      }
  }
  double out[1];
  double nuc = E.nu_per_cell ? E.nu[c] : E.nu[0];
  int rc = element_local(E.Q, g, nuc, E.beta, 0.0, EL_GRADNU, f + (long)c * E.Q.nq * 2, lk, 0.0,
                         WS{ws + t, nbatch}, out, fa + (long)c * E.Q.nq * 2, la, E.CT,
                         E.wcoef ? E.wcoef + (long)c * E.na : nullptr, nullptr, false, E.oflag ? E.oflag[c] : 0);
  if (rc) atomicOr(status, 1);
  gnu[c] += out[0];
}

// out = in * (w_q |K|) (inverse = 0) or in / (w_q |K|) (inverse = 1) for
// [n_cells][n_q][2] data-point arrays (w_q: the data rule's weights on the
// reference cell, normalised to sum 1).
__global__ void k_data_weight(QuadTables Q, const double* __restrict__ X, const int* __restrict__ cells, int nc,
                              const double* in, int inverse, double* out) {  // in may equal out
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nc * Q.nq) return;
  const long c = t / Q.nq;
  const int q = (int)(t % Q.nq);
  const int* v = cells + 3 * c;
  const double ax = X[2 * v[1]] - X[2 * v[0]], ay = X[2 * v[1] + 1] - X[2 * v[0] + 1];
  const double bx = X[2 * v[2]] - X[2 * v[0]], by = X[2 * v[2] + 1] - X[2 * v[0] + 1];
  const double w = Q.wq[q] * 0.5 * fabs(ax * by - ay * bx);
  const double s = inverse ? 1.0 / w : w;
  out[2 * t] = in[2 * t] * s;
  out[2 * t + 1] = in[2 * t + 1] * s;
}

__global__ void k_cr_blocks(const double* __restrict__ X, const int* __restrict__ cells, int nc,
                            const double* __restrict__ nu_cells, double beta, double eps_inv,
                            double* A) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  CellGeom g;
  cell_geom(X, cells + 3 * c, g);
  double B[36];
  cr_block(g, nu_cells[c], beta, eps_inv, B);
  for (int i = 0; i < 36; ++i) A[(long)c * 36 + i] = B[i];
}

// Assemble the principal block A_ss of every patch from the cell blocks and
// invert it (Cholesky); one thread per patch, strided workspace.
__global__ void k_patch_inverse(LevelView L, const int* __restrict__ pc_ptr, const int* __restrict__ pc,
                                int npatch, int max_ns, int general, double* ws, double* pinv, int* status) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npatch) return;
  const int m2 = 2 * L.m;
  const int f0 = L.pf_ptr[p], nfp = L.pf_ptr[p + 1] - f0;
  const int ns = nfp * m2;
  WS A{ws + p, npatch};
  for (long i = 0; i < (long)ns * ns; ++i) A[i] = 0.0;
  for (int q = pc_ptr[p]; q < pc_ptr[p + 1]; ++q) {
    int K = pc[q];
    int pos[3];
    for (int i = 0; i < 3; ++i) {
      pos[i] = -1;
      int d = L.cell_dofs[3 * K + i];
      for (int a = 0; a < nfp && d >= 0; ++a)
        if (L.pf[f0 + a] == d) pos[i] = a;
    }
    const double* SK = L.S + (long)K * L.nK * L.nK;
    for (int i1 = 0; i1 < 3; ++i1) {
      if (pos[i1] < 0) continue;
      for (int i2 = 0; i2 < 3; ++i2) {
        if (pos[i2] < 0) continue;
        for (int r1 = 0; r1 < m2; ++r1)
          for (int r2 = 0; r2 < m2; ++r2)
            A[(long)(pos[i1] * m2 + r1) * ns + pos[i2] * m2 + r2] +=
                SK[(long)(i1 * m2 + r1) * L.nK + i2 * m2 + r2];
      }
    }
  }
  double* out = pinv + L.pinv_off[p];
  if (general) {
    // LU with partial pivoting (nonsymmetric blocks); row swaps kept after A
    WS piv{ws + (long)max_ns * max_ns * npatch + p, npatch};
    for (int j = 0; j < ns; ++j) {
      int pr = j;
      double best = fabs(A[(long)j * ns + j]);
      for (int i = j + 1; i < ns; ++i) {
        double v = fabs(A[(long)i * ns + j]);
        if (v > best) {
          best = v;
          pr = i;
        }
      }
      if (!(best > 0)) {
        atomicOr(status, 2);
        return;
      }
      piv[j] = (double)pr;
      if (pr != j)
        for (int c = 0; c < ns; ++c) {
          double t = A[(long)j * ns + c];
          A[(long)j * ns + c] = A[(long)pr * ns + c];
          A[(long)pr * ns + c] = t;
        }
      const double dj = A[(long)j * ns + j];
      for (int i = j + 1; i < ns; ++i) {
        double l = A[(long)i * ns + j] / dj;
        A[(long)i * ns + j] = l;
        if (l != 0.0)
          for (int c = j + 1; c < ns; ++c) A[(long)i * ns + c] -= l * A[(long)j * ns + c];
      }
    }
    for (int c = 0; c < ns; ++c) {
      double* col = out + (long)c * ns;  // column c of the inverse
      for (int i = 0; i < ns; ++i) col[i] = i == c ? 1.0 : 0.0;
      for (int j = 0; j < ns; ++j) {
        int pr = (int)piv[j];
        if (pr != j) {
          double t = col[j];
          col[j] = col[pr];
          col[pr] = t;
        }
      }
      for (int i = 0; i < ns; ++i) {
        double s = col[i];
        for (int q = 0; q < i; ++q) s -= A[(long)i * ns + q] * col[q];
        col[i] = s;
      }
      for (int i = ns - 1; i >= 0; --i) {
        double s = col[i];
        for (int q = i + 1; q < ns; ++q) s -= A[(long)i * ns + q] * col[q];
        col[i] = s / A[(long)i * ns + i];
      }
    }
    return;
  }
  // Cholesky (lower, in place)
  for (int j = 0; j < ns; ++j) {
    double d = A[(long)j * ns + j];
    for (int q = 0; q < j; ++q) d -= A[(long)j * ns + q] * A[(long)j * ns + q];
    if (!(d > 0)) {
      atomicOr(status, 2);
      return;
    }
    d = sqrt(d);
    A[(long)j * ns + j] = d;
    for (int i = j + 1; i < ns; ++i) {
      double s = A[(long)i * ns + j];
      for (int q = 0; q < j; ++q) s -= A[(long)i * ns + q] * A[(long)j * ns + q];
      A[(long)i * ns + j] = s / d;
    }
  }
  for (int c = 0; c < ns; ++c) {
    double* col = out + (long)c * ns;  // column c of the inverse
    for (int i = 0; i < ns; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) s -= A[(long)i * ns + q] * col[q];
      col[i] = s / A[(long)i * ns + i];
    }
    for (int i = ns - 1; i >= 0; --i) {
      double s = col[i];
      for (int q = i + 1; q < ns; ++q) s -= A[(long)q * ns + i] * col[q];
      col[i] = s / A[(long)i * ns + i];
    }
  }
}

// The same inverses with one wavefront per patch: A_ss assembled in LDS
// next to the identity, Gauss-Jordan elimination with partial pivoting
// (lanes over columns, pivot search across lanes), inverse written
// column-major.  For patches of at most PI_WAVE_NS unknowns.
__device__ inline void wave_argmax(double& v, int& idx) {
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

__global__ void __launch_bounds__(64) k_patch_inverse_wave(LevelView L, const int* __restrict__ pc_ptr,
                                                           const int* __restrict__ pc, double* pinv, int* status) {
  extern __shared__ double sm[];
  const int p = blockIdx.x, lane = threadIdx.x;
  const int m2 = 2 * L.m;
  const int f0 = L.pf_ptr[p], nfp = L.pf_ptr[p + 1] - f0;
  const int ns = nfp * m2, w = 2 * ns;
  double* A = sm;              // [ns][2 ns]: A_ss | I
  double* fct = sm + ns * w;   // [ns] elimination factors
  for (int e = lane; e < ns * w; e += 64) {
    const int i = e / w, c = e % w;
    A[e] = (c - ns == i) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int q = pc_ptr[p]; q < pc_ptr[p + 1]; ++q) {
    const int K = pc[q];
    int pos[3];
    for (int i = 0; i < 3; ++i) {
      pos[i] = -1;
      const int d = L.cell_dofs[3 * K + i];
      for (int a = 0; a < nfp && d >= 0; ++a)
        if (L.pf[f0 + a] == d) pos[i] = a;
    }
    const double* SK = L.S + (long)K * L.nK * L.nK;
    for (int e = lane; e < L.nK * L.nK; e += 64) {
      const int r = e / L.nK, c = e % L.nK;
      const int i1 = r / m2, i2 = c / m2;
      if (pos[i1] < 0 || pos[i2] < 0) continue;
      A[(pos[i1] * m2 + r % m2) * w + pos[i2] * m2 + c % m2] += SK[e];
    }
    __syncthreads();
  }
  for (int j = 0; j < ns; ++j) {
    double v = -1.0;
    int idx = j;
    for (int i = j + lane; i < ns; i += 64) {
      const double a = fabs(A[i * w + j]);
      if (a > v) {
        v = a;
        idx = i;
      }
    }
    wave_argmax(v, idx);
    if (!(v > 0.0)) {
      if (lane == 0) atomicOr(status, 2);
      return;
    }
    if (idx != j)
      for (int c = lane; c < w; c += 64) {
        const double t = A[j * w + c];
        A[j * w + c] = A[idx * w + c];
        A[idx * w + c] = t;
      }
    __syncthreads();
    const double dinv = 1.0 / A[j * w + j];
    __syncthreads();
    for (int c = lane; c < w; c += 64) A[j * w + c] *= dinv;
    for (int i = lane; i < ns; i += 64) fct[i] = i == j ? 0.0 : A[i * w + j];
    __syncthreads();
    for (int c = lane; c < w; c += 64) {
      const double rj = A[j * w + c];
      for (int i = 0; i < ns; ++i) A[i * w + c] -= fct[i] * rj;
    }
    __syncthreads();
  }
  double* out = pinv + L.pinv_off[p];
  for (int e = lane; e < ns * ns; e += 64) {
    const int c = e / ns, i = e % ns;
    out[e] = A[i * w + ns + c];  // column c, row i
  }
}

// Row (facet fi, local row rr) of A x: sum over the two cells of fi.
template <typename TS>
__device__ inline double row_dot(const LevelViewT<TS>& L, int fi, int rr, const double* __restrict__ x) {
  const int m2 = 2 * L.m;
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    int K = L.fcell[2 * fi + s];
    if (K < 0) continue;  // do-nothing facet: one cell
    int i = L.floc[2 * fi + s];
    const TS* row = L.S + ((long)K * L.nK + i * m2 + rr) * L.nK;
    for (int i2 = 0; i2 < 3; ++i2) {
      int d = L.cell_dofs[3 * K + i2];
      if (d < 0) continue;
      const double* xd = x + (long)d * m2;
      const TS* rw = row + i2 * m2;
      for (int c = 0; c < m2; ++c) acc += (double)rw[c] * xd[c];
    }
  }
  return acc;
}

template <typename TS>
__global__ void k_apply(LevelViewT<TS> L, const double* __restrict__ x, double* __restrict__ y,
                        double alpha, const double* __restrict__ b) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m2 = 2 * L.m;
  if (t >= (long)L.nint * m2) return;
  int fi = (int)(t / m2), rr = (int)(t % m2);
  double v = alpha * row_dot(L, fi, rr, x);
  y[t] = b ? b[t] + v : v;
}

__global__ void k_gather_cells(LevelView L, const double* __restrict__ vK, double* __restrict__ y) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m2 = 2 * L.m;
  if (t >= (long)L.nint * m2) return;
  int fi = (int)(t / m2), rr = (int)(t % m2);
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    int K = L.fcell[2 * fi + s], i = L.floc[2 * fi + s];
    if (K >= 0) acc += vK[(long)K * L.nK + i * m2 + rr];
  }
  y[t] = acc;
}

// Block Gauss-Seidel step on the patches [p0, p1) of one colour: one
// wavefront per patch.  x_s += (A_ss)^-1 (b - A x)_s.  Patches of a colour
// share no cell, so their reads of x never see a same-phase write.
template <typename TS>
__global__ void __launch_bounds__(64) k_gs(LevelViewT<TS> L, int p0, double* x, const double* __restrict__ b) {
  __shared__ double res[GS_MAX_NS];
  const int p = p0 + blockIdx.x;
  const int m2 = 2 * L.m;
  const int f0 = L.pf_ptr[p], nfp = L.pf_ptr[p + 1] - f0;
  const int ns = nfp * m2;
  for (int t = threadIdx.x; t < ns; t += blockDim.x) {
    int fi = L.pf[f0 + t / m2], rr = t % m2;
    long d = (long)fi * m2 + rr;
    res[t] = b[d] - row_dot(L, fi, rr, x);
  }
  __syncthreads();
  const TS* Ai = L.pinv + L.pinv_off[p];
  double dlt[GS_MAX_NS / 64];
  int cnt = 0;
  for (int t = threadIdx.x; t < ns; t += blockDim.x, ++cnt) {
    double s = 0.0;
    for (int j = 0; j < ns; ++j) s += (double)Ai[(long)j * ns + t] * res[j];
    dlt[cnt] = s;
  }
  __syncthreads();
  cnt = 0;
  for (int t = threadIdx.x; t < ns; t += blockDim.x, ++cnt) {
    int fi = L.pf[f0 + t / m2], rr = t % m2;
    x[(long)fi * m2 + rr] += dlt[cnt];
  }
}

template <typename TP>
__global__ void __launch_bounds__(256) k_patch_correct(const int* __restrict__ pf_ptr, const int* __restrict__ pf,
                                                       const long* __restrict__ poff, const TP* __restrict__ pinv,
                                                       int nd, int p0, const double* __restrict__ r, double* x,
                                                       double damp) {
  extern __shared__ double res[];
  const int p = p0 + blockIdx.x;
  const int f0 = pf_ptr[p], ns = (pf_ptr[p + 1] - f0) * nd;
  for (int t = threadIdx.x; t < ns; t += blockDim.x) res[t] = r[(long)pf[f0 + t / nd] * nd + t % nd];
  __syncthreads();
  const TP* A = pinv + poff[p];
  for (int t = threadIdx.x; t < ns; t += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < ns; ++j) s += (double)A[(long)j * ns + t] * res[j];
    x[(long)pf[f0 + t / nd] * nd + t % nd] += damp * s;
  }
}

// The six mode-0 rows of every order-k cell block (local facet i, component
// c: row (i 2 + c) m), cell-minor: entry (row i 2 + c, column col) of cell K
// at S0[(col * 6 + i * 2 + c) * nc + K]; S full row-major [nc][nK][nK].
template <typename TS>
__global__ void k_pack_mode0_rows(int nc, int m, const double* __restrict__ S, TS* __restrict__ S0) {
  const int nK = 6 * m;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nc * nK) return;
  const int col = (int)(t / nc), K = (int)(t % nc);
#pragma unroll
  for (int r = 0; r < 6; ++r) S0[((long)col * 6 + r) * nc + K] = (TS)S[((long)K * nK + r * m) * nK + col];
}

// Mode-0 rows of S_K x_K, M0_CELLS2 cells per workgroup: x_K into LDS (rows
// padded by one word), then thread (row r, cell j) forms its row from S0 with
// eight loads in flight (a wavefront reads one row of 64 consecutive cells
// per word).
constexpr int M0_CELLS2 = 64;
template <typename TS>
__global__ void __launch_bounds__(6 * M0_CELLS2) k_cell_mode0(int nc, int m, const int* __restrict__ cell_dofs,
                                                              const TS* __restrict__ S0,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ y0K) {
  __shared__ double xs[M0_CELLS2][6 * 5 + 1];
  const int nK = 6 * m, m2 = 2 * m;
  const int K0 = blockIdx.x * M0_CELLS2, tid = threadIdx.x;
  for (int e = tid; e < M0_CELLS2 * nK; e += 6 * M0_CELLS2) {
    const int j = e / nK, i = e % nK, K = min(K0 + j, nc - 1);
    const int dof = cell_dofs[3 * K + i / m2];
    xs[j][i] = dof < 0 ? 0.0 : x[(long)dof * m2 + i % m2];
  }
  __syncthreads();
  const int j = tid % M0_CELLS2, r = tid / M0_CELLS2, K = K0 + j;
  if (K >= nc) return;
  const TS* a = S0 + (long)r * nc + K;
  const long step = 6L * nc;  // next column
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
  y0K[(long)K * 6 + r] = (a0 + a1) + (a2 + a3);
}

// g0 = mode 0 of (b - A x) from the cells' mode-0 rows (facet fi, component
// c: the rows of its cells; a do-nothing facet has one); zero_out (if not
// null) zeroed alike.
__global__ void k_mode0_gather(int nint, int m, const int* __restrict__ fcell, const int* __restrict__ floc,
                               const double* __restrict__ y0K, const double* __restrict__ b,
                               double* __restrict__ g0, double* __restrict__ zero_out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2L * nint) return;
  const int fi = (int)(t / 2), c = (int)(t % 2);
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int K = fcell[2 * fi + s];
    if (K >= 0) acc += y0K[(long)K * 6 + floc[2 * fi + s] * 2 + c];
  }
  g0[t] = b[t * m] - acc;
  if (zero_out) zero_out[t] = 0.0;
}

__global__ void k_mode0_extract(int nint, int m, const double* __restrict__ r, double* __restrict__ g0,
                                double* __restrict__ zero_out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nint) return;
  g0[t] = r[(long)t * m];
  if (zero_out) zero_out[t] = 0.0;
}

__global__ void k_mode0_add(int nint, int m, const double* __restrict__ u0, double* __restrict__ x) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nint) return;
  x[(long)t * m] += u0[t];
}

// ELL (padded, column-major) sparse matrix-vector product: entry k of row r
// at [k * n + r], padding has value 0 and column 0.  Slots go in chunks of
// eight, so that a thread has eight value and column loads, then eight
// gathers, in flight at once; slots past the width re-read the last one
// and count zero.
template <typename TS>
__global__ void k_ell_spmv(int n, int w, const int* __restrict__ ci, const TS* __restrict__ v,
                           const double* __restrict__ x, double* y, double beta_y, double* zero_out) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  if (zero_out) zero_out[r] = 0.0;
  if (w <= 0) return;
  double s = 0.0;
  for (int k0 = 0; k0 < w; k0 += 8) {
    TS vv[8];
    int cc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const long k = min(k0 + q, w - 1);
      vv[q] = v[k * n + r] * (TS)(k0 + q < w);
      cc[q] = ci[k * n + r];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s += (double)vv[q] * x[cc[q]];
  }
  y[r] = beta_y == 0.0 ? s : beta_y * y[r] + s;
}

// The same product with a group of L lanes per row (L a power of two, at
// most 8): lane j of the group takes the slots j, j + L, ..., eight of them
// in flight at once, and the group sums by shuffles -- wide rows (the
// restrictions carry the harmonic-extension correction) cost one or two
// memory round trips instead of one per eight slots.
template <typename TS, int L>
__global__ void k_ell_spmv_g(int n, int w, const int* __restrict__ ci, const TS* __restrict__ v,
                             const double* __restrict__ x, double* y, double beta_y, double* zero_out) {
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long r = tid / L;
  const int j = (int)(tid % L);
  const bool ok = r < n;  // every lane stays for the shuffles
  double s = 0.0;
  if (ok) {
    for (int k0 = j; k0 < w; k0 += 8 * L) {
      TS vv[8];
      int cc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + q * L;
        const long kk = min(k, w - 1);
        vv[q] = v[kk * n + r] * (TS)(k < w);
        cc[q] = ci[kk * n + r];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s += (double)vv[q] * x[cc[q]];
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (ok && j == 0) {
    if (zero_out) zero_out[r] = 0.0;
    y[r] = beta_y == 0.0 ? s : beta_y * y[r] + s;
  }
}


// The same grouped product on a sliced ELL matrix: the rows in slices of
// H = 64 / L (the rows one wavefront covers), each slice padded only to its
// own widest row (sw[s] slots; entry (slot k, row sH + rr) at
// soff[s] + k H + rr), so that rows of different lengths in different
// slices (the prolongations' rows inside a coarse cell against those on its
// facets) stop paying for the widest row of the matrix.
template <typename TS, int L>
__global__ void k_sell_spmv_g(int n, const long* __restrict__ soff, const int* __restrict__ sw,
                              const int* __restrict__ ci, const TS* __restrict__ v, const double* __restrict__ x,
                              double* y, double beta_y, double* zero_out) {
  constexpr int H = 64 / L;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long r = tid / L;
  const int j = (int)(tid % L);
  const bool ok = r < n;  // every lane stays for the shuffles
  double s = 0.0;
  if (ok) {
    const long sl = r / H;
    const long base = soff[sl] + (r - sl * H);
    const int w = sw[sl];
    for (int k0 = j; k0 < w; k0 += 8 * L) {
      TS vv[8];
      int cc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + q * L;
        const long e = base + (long)min(k, w - 1) * H;
        vv[q] = v[e] * (TS)(k < w);
        cc[q] = ci[e];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s += (double)vv[q] * x[cc[q]];
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (ok && j == 0) {
    if (zero_out) zero_out[r] = 0.0;
    y[r] = beta_y == 0.0 ? s : beta_y * y[r] + s;
  }
}

// y = A x for a dense row-major A (n x n, storage TS, row stride ld: a
// multiple of 4, zero-padded), a wavefront per row: each lane reads four
// consecutive entries per 16-byte load (two for FP64), eight such loads in
// flight before any is used, FP64 accumulation, then a wavefront reduction.
template <typename TS>
__global__ void __launch_bounds__(256) k_gemv_rows(int n, int ld, const TS* __restrict__ A,
                                                   const double* __restrict__ x, double* __restrict__ y) {
  constexpr int U = 8;
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const TS* a = A + row * ld;
  double s = 0.0;
  for (int j0 = 0; j0 < ld; j0 += 4 * 64 * U) {
    TS av[U][4];
    double xv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + 4 * (64 * u + lane);
      if (j < ld) {
        if constexpr (sizeof(TS) == 4) {
          const float4 v = *(const float4*)(a + j);
          av[u][0] = v.x, av[u][1] = v.y, av[u][2] = v.z, av[u][3] = v.w;
        } else {
          const double2 v0 = *(const double2*)(a + j), v1 = *(const double2*)(a + j + 2);
          av[u][0] = v0.x, av[u][1] = v0.y, av[u][2] = v1.x, av[u][3] = v1.y;
        }
      } else {
        av[u][0] = av[u][1] = av[u][2] = av[u][3] = (TS)0;
      }
      // x with the matrix entries (the padding columns past n read nothing)
      if (j + 3 < n) {
        const double2 x0 = *(const double2*)(x + j), x1 = *(const double2*)(x + j + 2);
        xv[u][0] = x0.x, xv[u][1] = x0.y, xv[u][2] = x1.x, xv[u][3] = x1.y;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) xv[u][e] = j + e < n ? x[j + e] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) s += (double)av[u][e] * xv[u][e];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) y[row] = s;
}

// out (row-major, storage TS, row stride ld >= n, padding zeroed) = the
// transpose of the column-major n x n matrix in
template <typename TS>
__global__ void k_transpose_to(int n, int ld, const double* __restrict__ in, TS* __restrict__ out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * ld) return;
  const long i = t / ld, j = t % ld;  // out[i][j] = in column j, row i
  out[t] = j < n ? (TS)in[j * n + i] : (TS)0;
}

// columns of the n x n identity (column-major)
__global__ void k_identity(int n, double* __restrict__ out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * n) return;
  out[t] = (t / n == t % n) ? 1.0 : 0.0;
}

__global__ void k_to_f32(long n, const double* __restrict__ in, float* __restrict__ out) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = (float)in[t];
}

__global__ void k_fill(long n, double v, double* x) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}

__global__ void k_copy(long n, const double* __restrict__ x, double* __restrict__ y) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = x[t];
}

// Sum over the workgroup (a multiple of 64 threads), returned to every
// thread: each wavefront sums by shuffles, then the wavefronts' sums meet in
// LDS (sh: one word per wavefront, reusable after the return).
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// block partials of sum_{K,q} w_q |K| |a - b|^2 over [nc][nq][2] fields (b may be null)
__global__ void k_wdiff2(QuadTables Q, const double* __restrict__ X, const int* __restrict__ cells, int nc,
                         const double* __restrict__ a, const double* __restrict__ b, double* part) {
  __shared__ double sh[TPB / 64];
  double s = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < (long)nc * Q.nq; t += (long)gridDim.x * blockDim.x) {
    const long c = t / Q.nq;
    const int q = (int)(t % Q.nq);
    const int* v = cells + 3 * c;
    const double ax = X[2 * v[1]] - X[2 * v[0]], ay = X[2 * v[1] + 1] - X[2 * v[0] + 1];
    const double bx = X[2 * v[2]] - X[2 * v[0]], by = X[2 * v[2] + 1] - X[2 * v[0] + 1];
    const double w = Q.wq[q] * 0.5 * fabs(ax * by - ay * bx);
    const double d0 = a[2 * t] - (b ? b[2 * t] : 0.0), d1 = a[2 * t + 1] - (b ? b[2 * t + 1] : 0.0);
    s += w * (d0 * d0 + d1 * d1);
  }
  const double r = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void k_axpy(long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] += a * x[t];
}

// tangential Dirichlet coefficients of constant boundary velocities:
// uhat_b[f][0] = g_b[f] . t_F, higher modes 0 (the facet L2 projection of a
// constant onto the orthonormal Legendre modes)
__global__ void k_dirichlet_const(int nb, int m, const double* __restrict__ tb, const double* __restrict__ gb,
                                  double* __restrict__ uhat) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nb * m) return;
  const int f = (int)(t / m), j = (int)(t % m);
  uhat[t] = j == 0 ? gb[2 * f] * tb[2 * f] + gb[2 * f + 1] * tb[2 * f + 1] : 0.0;
}

__global__ void k_dot(long n, const double* __restrict__ x, const double* __restrict__ y, double* part) {
  __shared__ double sh[TPB / 64];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  double r = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void k_dot2(long n, const double* __restrict__ z, const double* __restrict__ r,
                       const double* __restrict__ r2, double* part) {
  __shared__ double sh[TPB / 64];
  double s1 = 0.0, s2 = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    s1 += z[i] * r[i];
    s2 += z[i] * r2[i];
  }
  double a = block_sum(s1, sh);
  double b = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

// part[i * gridDim.x + block] = partial sums of V_i . w, i < nv (V_i = V + i * ld);
// eight basis vectors per pass, so that w is read once per eight
__global__ void k_mdot(long n, int nv, const double* __restrict__ V, long ld, const double* __restrict__ w,
                       double* part) {
  __shared__ double sh[TPB / 64];
  for (int i0 = 0; i0 < nv; i0 += 8) {
    const int g = min(8, nv - i0);
    double s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = 0.0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
      const double wt = w[t];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < g) s[i] += V[(long)(i0 + i) * ld + t] * wt;
    }
    for (int i = 0; i < g; ++i) {
      const double r = block_sum(s[i], sh);
      if (threadIdx.x == 0) part[(long)(i0 + i) * gridDim.x + blockIdx.x] = r;
    }
  }
}

// w += sign * sum_i h[i] V_i
__global__ void k_maxpy(long n, int nv, const double* __restrict__ V, long ld, const double* __restrict__ h,
                        double sign, double* __restrict__ w) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s += h[i] * V[(long)i * ld + t];
    w[t] += sign * s;
  }
}

__global__ void k_scale(long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = a * x[t];
}

__global__ void k_finalize(const double* __restrict__ part, int nblocks, int nvals, double* sc, int slot0) {
  __shared__ double sh[TPB / 64];
  for (int v = 0; v < nvals; ++v) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part[(long)v * nblocks + i];
    double r = block_sum(s, sh);
    if (threadIdx.x == 0) sc[slot0 + v] = r;
  }
}

__global__ void k_fcg_xr(long n, double* x, double* r, double* r_old, const double* __restrict__ p,
                         const double* __restrict__ q, const double* __restrict__ sc, double* part) {
  __shared__ double sh[TPB / 64];
  const double alpha = sc[SC_ZR] / sc[SC_PQ];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    double ri = r[i];
    r_old[i] = ri;
    ri -= alpha * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_fcg_p(long n, double* p, const double* __restrict__ z, const double* __restrict__ sc) {
  const double beta = (sc[SC_ZRN] - sc[SC_ZRO]) / sc[SC_ZR];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

__global__ void k_scalar_move(double* sc, int from, int to) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc[to] = sc[from];
}

__global__ void k_uzawa_rhs(int nint, int m, const double* __restrict__ g, const double* __restrict__ fdiv,
                            const int* __restrict__ fcell, const double* __restrict__ p0, double* b) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nint * 2 * m) return;
  double v = g[t];
  if (t % (2 * m) == 0) {
    int fi = (int)(t / (2 * m));
    v += fdiv[2 * fi] * p0[fcell[2 * fi]];
    if (fcell[2 * fi + 1] >= 0) v += fdiv[2 * fi + 1] * p0[fcell[2 * fi + 1]];
  }
  b[t] = v;
}

__global__ void k_uzawa_update(int nc, int m, const int* __restrict__ cell_dofs, const double* __restrict__ cdiv,
                               const double* __restrict__ area, const double* __restrict__ lam,
                               double eps_inv, const double* __restrict__ cflux, double* p0, double* part) {
  __shared__ double sh[TPB / 64];
  double s1 = 0.0, s2 = 0.0;
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long)gridDim.x * blockDim.x) {
    double dv = cflux ? cflux[c] : 0.0;  // prescribed boundary flux
    for (int i = 0; i < 3; ++i) {
      int d = cell_dofs[3 * c + i];
      if (d >= 0) dv += cdiv[3 * c + i] * lam[(long)d * 2 * m];
    }
    double dp = -eps_inv * dv / area[c];
    double pn = p0[c] + dp;
    p0[c] = pn;
    s1 += area[c] * dp * dp;
    s2 += area[c] * pn * pn;
  }
  double a = block_sum(s1, sh);
  double b = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

}  // namespace

void launch_condense(hipStream_t st, const ElemLevel& E, int c0, int nbatch, double* ws, double* S, int* status) {
  hipLaunchKernelGGL(k_condense, dim3(nblk(nbatch, 64)), dim3(64), 0, st, E, c0, nbatch, ws, S, status);
}
void launch_load(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, double* ws, double* gK,
                 int* status) {
  hipLaunchKernelGGL(k_load, dim3(nblk(nbatch, 64)), dim3(64), 0, st, E, c0, nbatch, f, ws, gK, status);
}
void launch_recover(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, const double* lam,
                    const double* p0, double* ws, double* u, double* p, int* status) {
  hipLaunchKernelGGL(k_recover, dim3(nblk(nbatch, 64)), dim3(64), 0, st, E, c0, nbatch, f, lam, p0, ws, u, p,
                     status);
}
void launch_wind_fit(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, int c0, int nbatch,
                     const double* vals, double* ws, double* coef, int* status) {
  if (nbatch > 0)
    hipLaunchKernelGGL(k_wind_fit, dim3(nblk(nbatch, 64)), dim3(64), 0, st, Q, X, cells, c0, nbatch, vals, ws, coef,
                       status);
}
void launch_wind_rt0(hipStream_t st, const QuadTables& Q0, const double* X, const int* cells,
                     const int* cell_dofs, int c0, int nbatch, const double* flux, double* ws, double* coef,
                     int* status) {
  if (nbatch > 0)
    hipLaunchKernelGGL(k_wind_rt0, dim3(nblk(nbatch, 64)), dim3(64), 0, st, Q0, X, cells, cell_dofs, c0, nbatch,
                       flux, ws, coef, status);
}
void launch_facet_flux(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, const int* fcell,
                       const int* floc, int nint, const double* coef, int na, double* flux) {
  if (nint > 0)
    hipLaunchKernelGGL(k_facet_flux, dim3(nblk(nint, 64)), dim3(64), 0, st, Q, X, cells, fcell, floc, nint, coef,
                       na, flux);
}
void launch_bd_flux(hipStream_t st, int nc, int m, const double* bdiv, const double* bdl, double* cflux) {
  if (nc > 0) hipLaunchKernelGGL(k_bd_flux, dim3(nblk(nc)), dim3(TPB), 0, st, nc, m, bdiv, bdl, cflux);
}
void launch_bd_local(hipStream_t st, int nc, int m, const int* cbf, const double* uhat_b, int full, double* bdl) {
  const long n = (long)nc * 3 * 2 * m;
  if (n > 0) hipLaunchKernelGGL(k_bd_local, dim3(nblk(n)), dim3(TPB), 0, st, nc, m, cbf, uhat_b, full, bdl);
}
void launch_postprocess(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, const double* lam,
                        double* ws, double* ustar, int* status) {
  hipLaunchKernelGGL(k_postprocess, dim3(nblk(nbatch, 64)), dim3(64), 0, st, E, c0, nbatch, f, lam, ws, ustar,
                     status);
}
void launch_gradnu(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, const double* lam,
                   const double* fa, const double* lama, double* ws, double* gnu, int* status) {
  hipLaunchKernelGGL(k_gradnu, dim3(nblk(nbatch, 64)), dim3(64), 0, st, E, c0, nbatch, f, lam, fa, lama, ws, gnu,
                     status);
}
void launch_data_weight(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, int nc,
                        const double* in, int inverse, double* out) {
  const long n = (long)nc * Q.nq;
  if (n > 0) hipLaunchKernelGGL(k_data_weight, dim3(nblk(n)), dim3(TPB), 0, st, Q, X, cells, nc, in, inverse, out);
}
void launch_cr_blocks(hipStream_t st, const double* X, const int* cells, int nc, const double* nu_cells,
                      double beta, double eps_inv, double* A) {
  hipLaunchKernelGGL(k_cr_blocks, dim3(nblk(nc)), dim3(TPB), 0, st, X, cells, nc, nu_cells, beta,
                     eps_inv, A);
}
void launch_patch_inverse(hipStream_t st, LevelView L, const int* pc_ptr, const int* pc, int npatch,
                          int max_ns, int general, double* ws, double* pinv, int* status) {
  if (npatch <= 0) return;
  if (max_ns <= PI_WAVE_NS) {
    const size_t shm = sizeof(double) * ((size_t)max_ns * 2 * max_ns + max_ns);
    hipLaunchKernelGGL(k_patch_inverse_wave, dim3(npatch), dim3(64), shm, st, L, pc_ptr, pc, pinv, status);
    return;
  }
  hipLaunchKernelGGL(k_patch_inverse, dim3(nblk(npatch, 64)), dim3(64), 0, st, L, pc_ptr, pc, npatch, max_ns,
                     general, ws, pinv, status);
}
template <typename TS>
void launch_apply(hipStream_t st, LevelViewT<TS> L, const double* x, double* y, double alpha, const double* b) {
  long n = (long)L.nint * 2 * L.m;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_apply<TS>, dim3(nblk(n)), dim3(TPB), 0, st, L, x, y, alpha, b);
}
template void launch_apply<double>(hipStream_t, LevelViewT<double>, const double*, double*, double,
                                   const double*);
template void launch_apply<float>(hipStream_t, LevelViewT<float>, const double*, double*, double,
                                  const double*);
void launch_to_f32(hipStream_t st, long n, const double* in, float* out) {
  if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(nblk(n)), dim3(TPB), 0, st, n, in, out);
}
void launch_gather_cells(hipStream_t st, LevelView L, const double* vK, double* y) {
  long n = (long)L.nint * 2 * L.m;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_cells, dim3(nblk(n)), dim3(TPB), 0, st, L, vK, y);
}
template <typename TS>
void launch_gs(hipStream_t st, LevelViewT<TS> L, int p0, int p1, double* x, const double* b) {
  if (p1 <= p0) return;
  hipLaunchKernelGGL(k_gs<TS>, dim3(p1 - p0), dim3(64), 0, st, L, p0, x, b);
}
template <typename TP>
void launch_patch_correct(hipStream_t st, const int* pf_ptr, const int* pf, const long* poff, const TP* pinv, int nd,
                          int ns_max, int p0, int p1, const double* r, double* x, double damp) {
  if (p1 <= p0) return;
  const int threads = ns_max <= 64 ? 64 : (ns_max <= 128 ? 128 : 256);
  hipLaunchKernelGGL(k_patch_correct<TP>, dim3(p1 - p0), dim3(threads), (size_t)ns_max * sizeof(double), st, pf_ptr,
                     pf, poff, pinv, nd, p0, r, x, damp);
}
template void launch_patch_correct<double>(hipStream_t, const int*, const int*, const long*, const double*, int, int,
                                           int, int, const double*, double*, double);
template void launch_patch_correct<float>(hipStream_t, const int*, const int*, const long*, const float*, int, int,
                                          int, int, const double*, double*, double);
template void launch_gs<double>(hipStream_t, LevelViewT<double>, int, int, double*, const double*);
template void launch_gs<float>(hipStream_t, LevelViewT<float>, int, int, double*, const double*);
template <typename TS>
void launch_pack_mode0_rows(hipStream_t st, int nc, int m, const double* S, TS* S0) {
  const long n = (long)nc * 6 * m;
  if (n > 0) hipLaunchKernelGGL(k_pack_mode0_rows<TS>, dim3(nblk(n)), dim3(TPB), 0, st, nc, m, S, S0);
}
template void launch_pack_mode0_rows<double>(hipStream_t, int, int, const double*, double*);
template void launch_pack_mode0_rows<float>(hipStream_t, int, int, const double*, float*);
template <typename TS>
void launch_mode0_residual(hipStream_t st, int nc, int nint, int m, const int* cell_dofs, const int* fcell,
                           const int* floc, const TS* S0, const double* x, double* y0K, const double* b, double* g0,
                           double* zero_out) {
  if (nc > 0)
    hipLaunchKernelGGL(k_cell_mode0<TS>, dim3((nc + M0_CELLS2 - 1) / M0_CELLS2), dim3(6 * M0_CELLS2), 0, st, nc, m,
                       cell_dofs, S0, x, y0K);
  if (nint > 0)
    hipLaunchKernelGGL(k_mode0_gather, dim3(nblk(2L * nint)), dim3(TPB), 0, st, nint, m, fcell, floc, y0K, b, g0,
                       zero_out);
}
template void launch_mode0_residual<double>(hipStream_t, int, int, int, const int*, const int*, const int*,
                                            const double*, const double*, double*, const double*, double*, double*);
template void launch_mode0_residual<float>(hipStream_t, int, int, int, const int*, const int*, const int*,
                                           const float*, const double*, double*, const double*, double*, double*);
void launch_mode0_extract(hipStream_t st, int nint, int m, const double* r, double* g0, double* zero_out) {
  if (nint <= 0) return;
  hipLaunchKernelGGL(k_mode0_extract, dim3(nblk(2L * nint)), dim3(TPB), 0, st, nint, m, r, g0, zero_out);
}
void launch_mode0_add(hipStream_t st, int nint, int m, const double* u0, double* x) {
  if (nint <= 0) return;
  hipLaunchKernelGGL(k_mode0_add, dim3(nblk(2L * nint)), dim3(TPB), 0, st, nint, m, u0, x);
}
template <typename TS>
void launch_ell_spmv(hipStream_t st, int n, int w, const int* ci, const TS* v, const double* x, double* y,
                     double beta_y, double* zero_out) {
  if (n <= 0) return;
  if (w <= 8) {
    hipLaunchKernelGGL(k_ell_spmv<TS>, dim3(nblk(n)), dim3(TPB), 0, st, n, w, ci, v, x, y, beta_y, zero_out);
    return;
  }
  const long nt2 = 2L * n, nt4 = 4L * n, nt8 = 8L * n;
  if (w <= 16)
    hipLaunchKernelGGL((k_ell_spmv_g<TS, 2>), dim3(nblk(nt2)), dim3(TPB), 0, st, n, w, ci, v, x, y, beta_y,
                       zero_out);
  else if (w <= 32)
    hipLaunchKernelGGL((k_ell_spmv_g<TS, 4>), dim3(nblk(nt4)), dim3(TPB), 0, st, n, w, ci, v, x, y, beta_y,
                       zero_out);
  else
    hipLaunchKernelGGL((k_ell_spmv_g<TS, 8>), dim3(nblk(nt8)), dim3(TPB), 0, st, n, w, ci, v, x, y, beta_y,
                       zero_out);
}
template void launch_ell_spmv<double>(hipStream_t, int, int, const int*, const double*, const double*, double*,
                                      double, double*);
template void launch_ell_spmv<float>(hipStream_t, int, int, const int*, const float*, const double*, double*,
                                     double, double*);
int sell_lanes(int w) { return w <= 8 ? 0 : w <= 16 ? 2 : w <= 32 ? 4 : 8; }
template <typename TS>
void launch_sell_spmv(hipStream_t st, int n, int L, const long* soff, const int* sw, const int* ci, const TS* v,
                      const double* x, double* y, double beta_y, double* zero_out) {
  if (n <= 0) return;
  const long nt = (long)L * n;
  if (L == 2)
    hipLaunchKernelGGL((k_sell_spmv_g<TS, 2>), dim3(nblk(nt)), dim3(TPB), 0, st, n, soff, sw, ci, v, x, y, beta_y,
                       zero_out);
  else if (L == 4)
    hipLaunchKernelGGL((k_sell_spmv_g<TS, 4>), dim3(nblk(nt)), dim3(TPB), 0, st, n, soff, sw, ci, v, x, y, beta_y,
                       zero_out);
  else
    hipLaunchKernelGGL((k_sell_spmv_g<TS, 8>), dim3(nblk(nt)), dim3(TPB), 0, st, n, soff, sw, ci, v, x, y, beta_y,
                       zero_out);
}
template void launch_sell_spmv<double>(hipStream_t, int, int, const long*, const int*, const int*, const double*,
                                       const double*, double*, double, double*);
template void launch_sell_spmv<float>(hipStream_t, int, int, const long*, const int*, const int*, const float*,
                                      const double*, double*, double, double*);
template <typename TS>
void launch_gemv_rows(hipStream_t st, int n, int ld, const TS* A, const double* x, double* y) {
  if (n > 0) hipLaunchKernelGGL(k_gemv_rows<TS>, dim3((n + 3) / 4), dim3(256), 0, st, n, ld, A, x, y);
}
template void launch_gemv_rows<double>(hipStream_t, int, int, const double*, const double*, double*);
template void launch_gemv_rows<float>(hipStream_t, int, int, const float*, const double*, double*);
template <typename TS>
void launch_transpose_to(hipStream_t st, int n, int ld, const double* in, TS* out) {
  const long nn = (long)n * ld;
  if (nn > 0) hipLaunchKernelGGL(k_transpose_to<TS>, dim3(nblk(nn)), dim3(TPB), 0, st, n, ld, in, out);
}
template void launch_transpose_to<double>(hipStream_t, int, int, const double*, double*);
template void launch_transpose_to<float>(hipStream_t, int, int, const double*, float*);
void launch_identity(hipStream_t st, int n, double* out) {
  const long nn = (long)n * n;
  if (nn > 0) hipLaunchKernelGGL(k_identity, dim3(nblk(nn)), dim3(TPB), 0, st, n, out);
}
void launch_fill(hipStream_t st, long n, double v, double* x) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(TPB), 0, st, n, v, x);
}
void launch_copy(hipStream_t st, long n, const double* x, double* y) {
  if (n > 0) hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(TPB), 0, st, n, x, y);
}
void launch_dot(hipStream_t st, long n, const double* x, const double* y, double* part, int nblocks) {
  hipLaunchKernelGGL(k_dot, dim3(nblocks), dim3(TPB), 0, st, n, x, y, part);
}
void launch_dot2(hipStream_t st, long n, const double* z, const double* r, const double* r2, double* part,
                 int nblocks) {
  hipLaunchKernelGGL(k_dot2, dim3(nblocks), dim3(TPB), 0, st, n, z, r, r2, part);
}
void launch_finalize(hipStream_t st, const double* part, int nblocks, int nvals, double* sc, int slot0) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TPB), 0, st, part, nblocks, nvals, sc, slot0);
}
void launch_mdot(hipStream_t st, long n, int nv, const double* V, long ld, const double* w, double* part, int nb) {
  if (nv > 0) hipLaunchKernelGGL(k_mdot, dim3(nb), dim3(TPB), 0, st, n, nv, V, ld, w, part);
}
void launch_maxpy(hipStream_t st, long n, int nv, const double* V, long ld, const double* h, double sign, double* w) {
  if (nv > 0 && n > 0)
    hipLaunchKernelGGL(k_maxpy, dim3(std::min<long>(nblk(n), 4096)), dim3(TPB), 0, st, n, nv, V, ld, h, sign, w);
}
void launch_wdiff2(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, int nc, const double* a,
                   const double* b, double* part, int nblocks) {
  hipLaunchKernelGGL(k_wdiff2, dim3(nblocks), dim3(TPB), 0, st, Q, X, cells, nc, a, b, part);
}
void launch_axpy(hipStream_t st, long n, double a, const double* x, double* y) {
  if (n > 0) hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(TPB), 0, st, n, a, x, y);
}
void launch_dirichlet_const(hipStream_t st, int nb, int m, const double* tb, const double* gb, double* uhat) {
  const long n = (long)nb * m;
  if (n > 0) hipLaunchKernelGGL(k_dirichlet_const, dim3(nblk(n)), dim3(TPB), 0, st, nb, m, tb, gb, uhat);
}
void launch_scale(hipStream_t st, long n, double a, const double* x, double* y) {
  if (n > 0) hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(TPB), 0, st, n, a, x, y);
}
void launch_fcg_xr(hipStream_t st, long n, double* x, double* r, double* r_old, const double* p,
                   const double* q, const double* sc, double* part, int nblocks) {
  hipLaunchKernelGGL(k_fcg_xr, dim3(nblocks), dim3(TPB), 0, st, n, x, r, r_old, p, q, sc, part);
}
void launch_fcg_p(hipStream_t st, long n, double* p, const double* z, const double* sc) {
  hipLaunchKernelGGL(k_fcg_p, dim3(RED_BLOCKS), dim3(TPB), 0, st, n, p, z, sc);
}
void launch_scalar_move(hipStream_t st, double* sc, int from, int to) {
  hipLaunchKernelGGL(k_scalar_move, dim3(1), dim3(64), 0, st, sc, from, to);
}
void launch_uzawa_rhs(hipStream_t st, int nint, int m, const double* g, const double* fdiv, const int* fcell,
                      const double* p0, double* b) {
  long n = (long)nint * 2 * m;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_uzawa_rhs, dim3(nblk(n)), dim3(TPB), 0, st, nint, m, g, fdiv, fcell, p0, b);
}
void launch_uzawa_update(hipStream_t st, int nc, int m, const int* cell_dofs, const double* cdiv,
                         const double* area, const double* lam, double eps_inv, const double* cflux, double* p0,
                         double* part, int nblocks) {
  hipLaunchKernelGGL(k_uzawa_update, dim3(nblocks), dim3(TPB), 0, st, nc, m, cell_dofs, cdiv, area, lam,
                     eps_inv, cflux, p0, part);
}

}  // namespace hdgmg
