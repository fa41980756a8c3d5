// Device kernels of the skeleton solve (declarations shared by the host
// orchestration).  All kernels are FP64; vectors are skeleton vectors of a
// level with m modes per facet component (m = k+1 on the order-k level,
// m = 1 on the lowest-order levels), indexed (F * 2 + c) * m + j.
#pragma once
#include <hip/hip_runtime.h>

#include "element.hpp"

namespace hdgmg {

// Level data on the device; TS is the storage type of the operators.
template <typename TS>
struct LevelViewT {
  int nc, nint, m, nK;
  const int* cell_dofs;   // [nc][3] interior facet id or -1
  const int* fcell;       // [nint][2] the two cells of each interior facet
  const int* floc;        // [nint][2] local facet index in those cells
  const TS* S;            // [nc][nK][nK] cell blocks of A^eps (symmetric)
  const int* pf_ptr;      // patch -> facets CSR
  const int* pf;
  const long* pinv_off;   // patch -> offset of its inverse (column-major)
  const TS* pinv;
};
using LevelView = LevelViewT<double>;

// Scalars of the flexible-CG recurrence kept on the device.
enum { SC_ZR = 0, SC_PQ, SC_RR, SC_ZRN, SC_ZRO, SC_BB, SC_DP, SC_PP, SC_N };

// What the per-cell local solver of one level needs.
struct ElemLevel {
  QuadTables Q;             // data rule of the level's order
  const ConvTables* CT;     // device convection rules, or null (no wind)
  const double* X;          // [nv][2]
  const int* cells;         // [nc][3]
  const double* nu;         // [nc] or [1]
  int nu_per_cell;
  double beta, eps_inv;
  const double* wcoef;      // [nc][na] wind coefficients in the RT_k basis, or null
  int na;
  const int* cell_dofs;     // [nc][3] interior facet ids, -1 on the boundary
  int m;
  const double* bdl;        // [nc][3][2][m] prescribed boundary values (normal, tangential), or null
  const double* S;          // [nc][nK][nK] condensed blocks (the loads' boundary lift)
  double* fac;              // kept local factors (element_fac_size per cell, element i
                            // of cell c at fac[i * nc + c]), or null
  int nc;
  int transpose;            // 1: cells of the transposed (adjoint) system (with a wind)
  const int* oflag;         // [nc] bit i: local facet i is a do-nothing facet (the
                            // convection form's outflow term), or null
  // Newton linearisation (order-k level, with a wind): the previous state's
  // skeleton vector [N_skel] and the per-cell Newton load written by the
  // condensation (element i of cell c at nw_load[i * nc + c], nz entries:
  // RT rows then tangential facet rows); both null for Picard / Stokes
  const double* nw_lam;
  double* nw_load;
};

void launch_condense(hipStream_t st, const ElemLevel& E, int c0, int nbatch, double* ws, double* S, int* status);
// The same condensation with a wavefront per cell and the cell's matrices in
// LDS (condense.hip), all E.nc cells in one launch, for 1 <= k <= 4.
bool condense_wave_supported(int k);
void launch_condense_wave(hipStream_t st, const ElemLevel& E, double* S, int* status);
// gK = g_K(f) - S_K lambda_K^b (boundary lift when E.bdl is set)
void launch_load(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, double* ws, double* gK,
                 int* status);
void launch_recover(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, const double* lam,
                    const double* p0, double* ws, double* u, double* p, int* status);
// Wind coefficients of a field given at the data points ([nc][nq][2]) for
// cells c0 .. c0+nbatch (workspace: nbatch * na * (na+1) doubles).
void launch_wind_fit(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, int c0, int nbatch,
                     const double* vals, double* ws, double* coef, int* status);
// Lowest-order wind: the RT0 field with the given flux per interior facet
// (boundary fluxes zero), as coefficients in the k = 0 basis ([nc][3]).
void launch_wind_rt0(hipStream_t st, const QuadTables& Q0, const double* X, const int* cells,
                     const int* cell_dofs, int c0, int nbatch, const double* flux, double* ws, double* coef,
                     int* status);
// flux[F] = int_F w . n_F for every interior facet (from its first cell).
void launch_facet_flux(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, const int* fcell,
                       const int* floc, int nint, const double* coef, int na, double* flux);
// bdl[c][i][comp][j] = the prescribed value of local facet i of cell c
// (0 where cbf < 0): from uhat_b[cbf][comp][j] (full) or, tangential only,
// from uhat_b[cbf][j] with comp 0 (normal) zero.
void launch_bd_local(hipStream_t st, int nc, int m, const int* cbf, const double* uhat_b, int full, double* bdl);
// cflux[c] = sum_i bdiv[c][i] bdl[c][i][0][0]: the cell's outflow of the
// prescribed normal values (|K| div of the boundary lift)
void launch_bd_flux(hipStream_t st, int nc, int m, const double* bdiv, const double* bdl, double* cflux);
// gnu[c] += -(Lift z, Lift z_adj)_K for cells c0 .. c0+nbatch (forward
// source f and skeleton vector lam, adjoint source fa and skeleton vector lama).
// u* (stPost) of every cell in [c0, c0 + nbatch) at the data points:
// ustar [nc][nq][2] (workspace: element_ws_size per cell of the batch)
void launch_postprocess(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, const double* lam,
                        double* ws, double* ustar, int* status);
void launch_gradnu(hipStream_t st, const ElemLevel& E, int c0, int nbatch, const double* f, const double* lam,
                   const double* fa, const double* lama, double* ws, double* gnu, int* status);
// out = in * (w_q |K|), or in / (w_q |K|) when inverse != 0, on [nc][nq][2].
void launch_data_weight(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, int nc,
                        const double* in, int inverse, double* out);
void launch_cr_blocks(hipStream_t st, const double* X, const int* cells, int nc,
                      const double* nu_cells, double beta, double eps_inv, double* A);
// Inverses of the patch blocks A_ss (column-major).  Patches of at most
// PI_WAVE_NS unknowns: a wavefront per patch, Gauss-Jordan with partial
// pivoting in LDS; larger ones: a thread per patch, Cholesky or (general != 0)
// LU with partial pivoting (workspace max_ns^2 + max_ns per patch).
constexpr int PI_WAVE_NS = 60;
void launch_patch_inverse(hipStream_t st, LevelView L, const int* pc_ptr, const int* pc,
                          int npatch, int max_ns, int general, double* ws, double* pinv, int* status);
// y = alpha * A x + (b ? b : 0)
template <typename TS>
void launch_apply(hipStream_t st, LevelViewT<TS> L, const double* x, double* y, double alpha,
                  const double* b);
// y[d] = sum over the two cells of F of per-cell vector entries (gather)
void launch_gather_cells(hipStream_t st, LevelView L, const double* vK, double* y);
template <typename TS>
void launch_gs(hipStream_t st, LevelViewT<TS> L, int p0, int p1, double* x, const double* b);
// Damped block Jacobi correction (eq. bjac) for the patches [p0, p1) of one
// colour: x_s += damp * A_ss^-1 r_s from a residual r computed before the
// sweep, a workgroup per patch.  Patch p holds the nd unknowns of each of
// its facets pf[pf_ptr[p] ..] (unknown = facet * nd + i), its inverse is
// column-major at pinv + poff[p]; ns_max bounds the patch sizes (dynamic
// LDS).  Patches of one colour share no unknown.
template <typename TP>
void launch_patch_correct(hipStream_t st, const int* pf_ptr, const int* pf, const long* poff, const TP* pinv, int nd,
                          int ns_max, int p0, int p1, const double* r, double* x, double damp);
// out[i] = (float) in[i]
void launch_to_f32(hipStream_t st, long n, const double* in, float* out);
// g0 = mode 0 of r (restriction to the lowest-order space); zero_out (if not
// null) is set to zero over the same 2 nint entries.
void launch_mode0_extract(hipStream_t st, int nint, int m, const double* r, double* g0, double* zero_out = nullptr);
void launch_mode0_add(hipStream_t st, int nint, int m, const double* u0, double* x);
// The six mode-0 rows (local facet i, component c) of every order-k cell
// block of S (full row-major, nK = 6 m <= 30) as S0 [nK][6][nc] (cell-minor).
template <typename TS>
void launch_pack_mode0_rows(hipStream_t st, int nc, int m, const double* S, TS* S0);
// g0 = mode 0 of (b - A x) [2 nint] from S0, y0K [nc][6] scratch (only the
// mode-0 rows of the cell products); zero_out (if not null) zeroed over the
// same entries.
template <typename TS>
void launch_mode0_residual(hipStream_t st, int nc, int nint, int m, const int* cell_dofs, const int* fcell,
                           const int* floc, const TS* S0, const double* x, double* y0K, const double* b, double* g0,
                           double* zero_out);
// y = A x + beta_y y for an ELL matrix (n rows, width w); zero_out (if not
// null) is set to zero over the same n rows.
template <typename TS>
void launch_ell_spmv(hipStream_t st, int n, int w, const int* ci, const TS* v, const double* x, double* y,
                     double beta_y, double* zero_out = nullptr);
// The same for a sliced ELL matrix with L lanes per row (sell_lanes of its
// widest row: 2, 4 or 8; 0 when every row has at most 8 entries, for which
// the plain ELL kernel is used): rows in slices of 64 / L, slice s padded to
// its own width sw[s], entry (slot k, row s H + rr) at soff[s] + k H + rr.
int sell_lanes(int w);
template <typename TS>
void launch_sell_spmv(hipStream_t st, int n, int L, const long* soff, const int* sw, const int* ci, const TS* v,
                      const double* x, double* y, double beta_y, double* zero_out = nullptr);
// y = A x, A dense row-major n x n in storage TS with row stride ld (a
// multiple of 4, rows zero-padded; a wavefront per row, 16-byte loads)
template <typename TS>
void launch_gemv_rows(hipStream_t st, int n, int ld, const TS* A, const double* x, double* y);
// out (row-major, TS, row stride ld, padding zeroed) = transpose of the
// column-major n x n matrix in
template <typename TS>
void launch_transpose_to(hipStream_t st, int n, int ld, const double* in, TS* out);
// the n x n identity, column-major
void launch_identity(hipStream_t st, int n, double* out);
void launch_fill(hipStream_t st, long n, double v, double* x);
void launch_copy(hipStream_t st, long n, const double* x, double* y);
// partial sums of x.y into part[nblocks]; finalize part into sc[slot]
void launch_dot(hipStream_t st, long n, const double* x, const double* y, double* part,
                int nblocks);
void launch_dot2(hipStream_t st, long n, const double* z, const double* r, const double* r2,
                 double* part, int nblocks);
void launch_finalize(hipStream_t st, const double* part, int nblocks, int nvals, double* sc,
                     int slot0);
// part[i * nb + block] = block partials of V_i . w for i < nv (V_i = V + i*ld);
// reduce with launch_finalize(part, nb, nv, out, 0).
void launch_mdot(hipStream_t st, long n, int nv, const double* V, long ld, const double* w, double* part, int nb);
// w += sign * sum_{i < nv} h[i] V_i (h on the device)
void launch_maxpy(hipStream_t st, long n, int nv, const double* V, long ld, const double* h, double sign, double* w);
// y = a x
void launch_scale(hipStream_t st, long n, double a, const double* x, double* y);
// y += a x
void launch_axpy(hipStream_t st, long n, double a, const double* x, double* y);
// block partials of sum_{K,q} w_q |K| |a - b|^2 on [nc][nq][2] (b may be null);
// reduce with launch_finalize(part, nblocks, 1, ...)
void launch_wdiff2(hipStream_t st, const QuadTables& Q, const double* X, const int* cells, int nc, const double* a,
                   const double* b, double* part, int nblocks);
// uhat_b [nb][m] from constant velocities g_b [nb][2] and facet tangents tb [nb][2]
void launch_dirichlet_const(hipStream_t st, int nb, int m, const double* tb, const double* gb, double* uhat);
void launch_fcg_xr(hipStream_t st, long n, double* x, double* r, double* r_old, const double* p,
                   const double* q, const double* sc, double* part, int nblocks);
void launch_fcg_p(hipStream_t st, long n, double* p, const double* z, const double* sc);
void launch_scalar_move(hipStream_t st, double* sc, int from, int to);
// Uzawa helpers
void launch_uzawa_rhs(hipStream_t st, int nint, int m, const double* g, const double* fdiv,
                      const int* fcell, const double* p0, double* b);
void launch_uzawa_update(hipStream_t st, int nc, int m, const int* cell_dofs, const double* cdiv,
                         const double* area, const double* lam, double eps_inv, const double* cflux, double* p0,
                         double* part, int nblocks);

constexpr int RED_BLOCKS = 512;
// Largest vertex-patch block the Gauss-Seidel kernel holds in LDS.
constexpr int GS_MAX_NS = 256;

}  // namespace hdgmg
