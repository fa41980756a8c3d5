// Tetrahedral cells of the H(div)-HDG scheme on the device: reference
// tables, sizes, and the kernels of the three-dimensional path (local
// solver and static condensation, lowest-order blocks, skeleton apply,
// edge-patch inverses and block Gauss-Seidel, p-transfer, AL-Uzawa helpers).
//
// Order-k cell (scheme stWeak of Sec. 3.2 on a tetrahedron).  Lift(u, uhat)
// in [P^k]^{3x3} is defined by (Lift, G) = (grad u, G) - <tng(u - uhat),
// G n_K> with tng(v) = v - (v.n) n; the cell energy is
// 1/2 [nu |Lift|^2 + beta |u|^2] - (f, u).  Given the skeleton data
// lambda = (c^n, c^t1, c^t2) the interior u in RT_k(K) satisfies
//   N a = c^n   (normal trace moments against the orthonormal face basis)
//   D a = 0     (div u orthogonal to mean-free P^k, i.e. div u in P^0)
// and minimises the energy: the saddle point
//   [H_aa N^T D^T] [a ]   [F - H_at c^t]
//   [N    0   0  ] [mu] = [c^n         ]
//   [D    0   0  ] [pi]   [0           ]
// solved by Gauss-Jordan elimination with partial pivoting.  The condensed
// block is S = blockdiag(0, H_tt) - B^T KKT^-1 B with
// B = [[0, -H_at], [I, 0], [0, 0]] (columns c^n, then c^t), the load
// g = B^T KKT^-1 [F; 0; 0], and the interior pressure p^o = -sum_r pi_r
// (q_r - mean q_r).  The AL term eps^-1 |K|^-1 d d^T of stALform is added to
// S, with d = sigma_{K,F} |F| on each mode-0 normal coefficient.
//
// Basis: monomials xi^alpha of the reference coordinates of the affine map
// x = X_s0 + J xi from the cell's vertices sorted by global index;
// RT_k = [P^k]^3 + (x - X_s0)/h * {degree-k monomials}, h the longest edge.
// Face basis: orthonormal (normalised measure) polynomials in the face's
// reference coordinates (Gram-Schmidt of xi^a eta^b by degree, then b),
// tabulated at the face rule on the host.  Quadrature: Stroud conical rules
// with k+2 points per direction (exact to degree 2k+3) on the cell and on
// each face.  Local skeleton order (i*3 + c)*m_F + j, face i opposite
// stored vertex i, c = 0 normal, 1 t1, 2 t2.
#pragma once
#include <hip/hip_runtime.h>

namespace hdgmg {

#ifndef HDI
#define HDI __host__ __device__ inline
#endif

constexpr int K3MAX = 3;
constexpr int NQ3 = (K3MAX + 2) * (K3MAX + 2) * (K3MAX + 2);
constexpr int NFQ3 = (K3MAX + 2) * (K3MAX + 2);
constexpr int MF3MAX = (K3MAX + 1) * (K3MAX + 2) / 2;

struct Dims3 {
  int k, mF, nP, ntop, na, nz, nK, nN, nD, nkkt;
};

HDI Dims3 dims3(int k) {
  Dims3 d;
  d.k = k;
  d.mF = (k + 1) * (k + 2) / 2;
  d.nP = (k + 1) * (k + 2) * (k + 3) / 6;
  d.ntop = d.mF;
  d.na = 3 * d.nP + d.ntop;
  d.nz = d.na + 8 * d.mF;
  d.nK = 12 * d.mF;
  d.nN = 4 * d.mF;
  d.nD = d.nP - 1;
  d.nkkt = d.na + d.nN + d.nD;
  return d;
}

// Storage of a symmetric cell block (nK = 4 m3 unknowns, m3 per face): by
// face row blocks -- the m3 rows of local face f form an m3 x nK
// column-major block at offset f m3 nK -- so that the rows of one face, the
// unit a patch sweep reads, are one contiguous run.  Entry (r, c):
HDI long sblk(int r, int c, int m3, int nK) { return (long)(r / m3) * m3 * nK + (long)c * m3 + r % m3; }

// Reference rules (device memory, read through a pointer).
struct TetTables {
  int k, nq, nfq;
  double xq[NQ3][3];          // Stroud points on the reference tetrahedron
  double wq[NQ3];             // weights, sum 1
  double xf[NFQ3][2];         // Stroud points on the reference triangle
  double wf[NFQ3];            // weights, sum 1
  double phif[NFQ3][MF3MAX];  // face basis at the face points
};

// Per-level data of the tetrahedral skeleton operators on the device.
template <typename TS>
struct Level3View {
  int nc, nint, mF, nK;
  const int* cell_dofs;  // [nc][4] interior face id or -1
  const int* fcell;      // [nint][2] cells of each interior face
  const int* floc;       // [nint][2] local face index in those cells
  const TS* S;           // [nc][nK * nK] symmetric cell blocks of A^eps, or of A,
                         // entry (r, c) of cell K at K nK^2 + sblk(r, c, m3, nK)
                         // (al > 0: the AL term is added apart, in FP64)
  // AL term eps^-1 |K|^-1 d d^T applied apart when al > 0: d_i = cdiv[4K+i]
  // on the mode-0 normal unknown of local face i
  double al;
  const double* cdiv;    // [nc][4]
  const double* vol;     // [nc]
};

enum { TET_CONDENSE = 0, TET_LOAD = 1, TET_RECOVER = 2 };

// Element kernels, a workgroup per cell of [c0, c0 + nb): TET_CONDENSE
// writes S (+ AL term) [nc][nK * nK] (sblk layout); TET_LOAD writes gK [nc][nK] from
// f [nc][nq][3]; TET_RECOVER reads lam (skeleton) and p0 [nc] and writes
// u [nc][nq][3], p [nc][nq].  ws: tet_ws_words(k, mode) doubles per cell of
// the batch.  status bit 1: a singular local system.
long tet_ws_words(int k, int mode);
struct TetCells {
  const TetTables* T;    // device
  const double* X;       // [nv][3]
  const int* cells;      // [nc][4]
  const int* cell_dofs;  // [nc][4]
  const double* nu;      // [nc] or [1]
  int nu_per_cell;
  double beta, eps_inv;
  int k, nc;
};
void launch_tet_local(hipStream_t st, const TetCells& E, int mode, int c0, int nb, double* ws, const double* f,
                      const double* lam, const double* p0, double* S, double* gK, double* u, double* p,
                      int* status);
// Closed-form lowest-order blocks [nc][144] (k0-stOptForm on tetrahedra;
// sblk layout with m3 = 3).
void launch_cr_blocks3(hipStream_t st, const double* X, const int* cells, int nc, const double* nu_cells,
                       double beta, double eps_inv, double* A);
// yK = S_K x_K for every cell (a wavefront per cell), then y = alpha * (sum
// of the two cells' rows) + b (b may be null).
template <typename TS>
void launch_cell_apply3(hipStream_t st, Level3View<TS> L, const double* x, double* yK);
void launch_face_gather3(hipStream_t st, int nint, int mF, int nK, const int* fcell, const int* floc,
                         const double* yK, double alpha, const double* b, double* y);
// The twelve mode-0 rows (local face i, component q) of every cell block of
// S (sblk layout), as S0 [nK][12][nc] (cell-minor).
template <typename TS>
void launch_pack_mode0_rows3(hipStream_t st, int nc, int mF, const TS* S, TS* S0);
// g0 = mode 0 of (b - A x) [nint][3] from S0 (only the mode-0 rows of the
// cell products: y0K [nc][12] scratch; L.al > 0: the AL term apart);
// zero_out (if not null) zeroed over the same 3 nint entries.
template <typename TS>
void launch_mode0_residual3(hipStream_t st, Level3View<TS> L, const TS* S0, const double* x, double* y0K,
                            const double* b, double* g0, double* zero_out);
// Edge-patch inverses (column-major, pinv + poff[p]) of the patches
// [p0, p0 + np): a workgroup per patch, Gauss-Jordan with partial pivoting
// in global workspace (ws: np * ns_max * 2 * ns_max doubles).
void launch_patch_inverse3(hipStream_t st, Level3View<double> L, const int* pf_ptr, const int* pf,
                           const int* pc_ptr, const int* pc, const long* poff, int p0, int np, int ns_max,
                           double* ws, double* pinv, int* status);
// Block Gauss-Seidel on the patches [p0, p1) of one colour:
// x_s = A_ss^-1 (b_s - A_{s,r} x_r) (r: the unknowns outside the patch; the
// same value as x_s += A_ss^-1 (b - A x)_s), a workgroup per patch.
// (TS: storage of the cell blocks, TP: of the patch inverses; from_zero:
// x is zero on the faces of every patch cell, so (b - A x)_s = b_s and the
// cell blocks are not read)
template <typename TS, typename TP>
void launch_patch_gs3(hipStream_t st, Level3View<TS> L, const int* pf_ptr, const int* pf, const int* pc_ptr,
                      const int* pc, const long* poff, const TP* pinv, int p0, int p1, double* x,
                      const double* b, bool from_zero = false);
// The same at lowest order (mF = 1), a wavefront per patch, from one record
// per patch cell in patch-cell order (prec [4] ints, 16-byte aligned): the
// cell; a code packing the local indices i0, i1 of its patch faces (bits
// 0-3), their slots in the patch face list (4 bits each, bits 4-11; 15 =
// none), their sides (the cell is fcell[2f + side]; bits 12, 13), the local
// indices of its far faces (the interior faces not containing the edge;
// bits 14-15, 16-17) and their count (bits 18-19); the far faces' interior
// numbers (0 where absent).
template <typename TS, typename TP>
void launch_patch_gs3_lo(hipStream_t st, Level3View<TS> L, const int* pf_ptr, const int* pf, const int* pc_ptr,
                         const int* prec, const long* poff, const TP* pinv, int p0, int p1, double* x,
                         const double* b, bool from_zero = false);
// Lowest-order part of an order-k skeleton vector (mode 0 of each face
// component) and its injection.
void launch_mode0_extract3(hipStream_t st, int nint, int mF, const double* r, double* g0, double* zero_out);
void launch_mode0_add3(hipStream_t st, int nint, int mF, const double* u0, double* x);
// AL-Uzawa: b = g + D^T p (mode-0 normal entries), and
// p_K -= eps^-1 (D lambda)_K / |K| with block partial sums of
// |K| dp^2 and |K| p^2 (two rows of nb).
void launch_uzawa_rhs3(hipStream_t st, int nint, int mF, const double* g, const double* fdiv, const int* fcell,
                       const double* p0, double* b);
void launch_uzawa_update3(hipStream_t st, int nc, int mF, const int* cell_dofs, const double* cdiv,
                          const double* vol, const double* lam, double eps_inv, double* p0, double* part, int nb);
// Cell blocks from the sblk layout to dense [nc][nK][nK] (row-major).
void launch_blocks_to_dense(hipStream_t st, int nc, int m3, const double* in, double* out);
// out[i] = (float) in[i]
void launch_f32_copy(hipStream_t st, long n, const double* in, float* out);
// FP32 copy of cell blocks without their AL term: out = S - al |K|^-1 d d^T
void launch_f32_blocks_noal(hipStream_t st, int nc, int mF, const double* S, const double* cdiv, const double* vol,
                            double al, float* out);

}  // namespace hdgmg
