// Single-workgroup MG_h on the coarse lowest-order levels.
#pragma once
#include <hip/hip_runtime.h>

namespace hdgmg {

constexpr int COARSE_THREADS = 1024;
constexpr int COARSE_MAX_LEVELS = 8;
// A lowest-order unknown couples with the 10 unknowns of the facets of its
// two cells (fewer next to the boundary): rows are padded to 10 entries,
// both components of 5 facets.
constexpr int COARSE_NNZ = 10;
// Patch-row record key: the unknown in bits 0-17, the row inside its patch
// in bits 18-31; padding items carry the row REC_PAD.
constexpr int REC_LOC_SHIFT = 18;
constexpr unsigned REC_DOF_MASK = (1u << REC_LOC_SHIFT) - 1;
constexpr unsigned REC_PAD = 0x3fffu;
// Level vectors u, g, r of the coarse levels live in LDS: at most this many
// doubles in total.
constexpr int COARSE_LDS_DOUBLES = 6144;
// Largest number of batches of one level's sweep (its schedule is staged in LDS).
constexpr int COARSE_MAX_BATCH = 64;
// LDS of one workgroup on gfx950.
constexpr int COARSE_LDS_BYTES = 160 * 1024;

// One lowest-order level as seen by the coarse kernel (device pointers;
// per-item arrays are structure-of-arrays: entry e of item t at [e*nitems+t]).
// Operator values (it_val, it_ainv, rw_val, R_v, P_v) are stored in the
// storage type the kernel is launched with (double or float).
struct CoarseLevel {
  int n;                      // unknowns (2 per interior facet)
  int ncol, nitems, ns_max;   // colours, patch rows, largest patch
  int nbatch;
  int off_u, off_g, off_r;    // LDS offsets of the level vectors (doubles)
  int lds_meta, lds_val, lds_ainv;  // byte offsets of record parts copied
                              // to LDS at kernel start, -1: read from memory
  const int* cb_ptr;          // [ncol+1] batch range of each colour
  const int* bitem;           // [nbatch+1] item range of each batch
                              // (<= COARSE_THREADS items, patch-aligned)
  const int* bseq_bwd;        // [nbatch] batches in reverse colour order
  const uint4* it_meta;       // [nitems]: (key, F0 | F1 << 16, F2 | F3 << 16,
                              // F4): the residual row's 5 facets (16-bit),
                              // columns 2F and 2F + 1 each
  const void* it_val;         // residual row values (facet q, component c) at
                              // 2q + c, in 16-byte groups over items
  const void* it_ainv;        // [ns_max/2][nitems][2] row of the patch inverse (pairs)
  const int* rw_col;          // [COARSE_NNZ][n] rows of A for the residual
  const void* rw_val;
  int R_w, P_w;               // ELL widths of the transfers
  const int* R_ci;            // restriction to level l-1, ELL over its
  const void* R_v;            // unknowns: slot k of row i at [k * n(l-1) + i]
  const int* P_ci;            // prolongation from level l-1, ELL over these
  const void* P_v;            // unknowns: slot k of row i at [k * n + i]
  double* u_glob;             // level vectors in HBM (used at the top level)
  double* g_glob;
};

// Threads (items) per batch of the record-based Gauss-Seidel.
constexpr int GS_REC_THREADS = 256;

// One colour phase of block Gauss-Seidel on a launched lowest-order level
// from its patch-row records (the same structure-of-arrays record layout as
// CoarseLevel: meta, val, ainv over nit items), batches [b0, b0 + nb) of
// exactly GS_REC_THREADS item slots each (patch-aligned, padded with items
// whose row marker is REC_PAD): u += A_ss^-1 (g - A u)_s for every patch of
// the colour.  f32: val and ainv are float, else double.  wide: two meta
// words per item, (unknown, row in patch, F0, F1), (F2, F3, F4, 0) with
// 32-bit fields, for levels beyond 16-bit facet indices.
void launch_gs_records(hipStream_t st, const unsigned* meta, const void* val, const void* ainv, int nit, int nsm,
                       int b0, int nb, double* u, const double* g, int f32, int wide);

// u_top <- MG_h(top, g_top, u_top, m_top, q) with m(l-1) = growth m(l) on
// levels 0..top (top <= the levels described by Ls); level 0 is solved with
// the dense column-major inverse inv0 (n0 x n0).  lds_doubles: the dynamic
// LDS the descriptors' offsets need.
// f32 != 0: operator values (and inv0) are float, else double.
// prepare_coarse_cycle: allow lds_bytes of dynamic LDS for the kernel (once
// at setup, before any launch or capture).
hipError_t prepare_coarse_cycle(int ns_max, size_t lds_bytes, int f32);
// Static LDS of the coarse kernel (bytes), to subtract from COARSE_LDS_BYTES.
size_t coarse_cycle_static_lds();
void launch_coarse_cycle(hipStream_t st, const CoarseLevel* Ls, int top, int m_top, int growth, int q,
                         const void* inv0, int n0, int ns_max, int lds_doubles, int f32);
// The same cycle for nb independent top-level right-hand sides, a workgroup
// each: workgroup b reads g_top + b*bstride and u_top + b*bstride (the
// initial iterate) and writes the result to u_top + b*bstride; the level
// descriptors' own top-level vectors are not touched.  With g_top the
// columns of the identity and u_top zero this tabulates MG_h on the top
// level as a dense matrix (column j = MG_h(e_j)).  r_top non-null: the top
// level's vectors stay in memory (u_top, g_top and the residual r_top, each
// column at b*bstride), for a top level too large for LDS (its descriptor's
// LDS offsets are ignored).
void launch_coarse_cycle_batch(hipStream_t st, const CoarseLevel* Ls, int top, int m_top, int growth, int q,
                               const void* inv0, int n0, int ns_max, int lds_doubles, int f32, int nb,
                               const double* g_top, double* u_top, double* r_top, long bstride);

}  // namespace hdgmg
