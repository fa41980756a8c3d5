// Streaming skeleton apply and vertex-patch Gauss-Seidel (see fast.hip for
// the storage layouts).
#pragma once
#include <hip/hip_runtime.h>

namespace hdgmg {

// Largest vertex patch (in facets) the streaming Gauss-Seidel handles; every
// interior vertex of the structured triangulations and their red
// refinements has six edges.
constexpr int FAST_NF = 6;

// Cell-block storage of the streaming layout: packed upper triangle for
// symmetric blocks up to 18 x 18 (k <= 2), full otherwise (full = true for
// the nonsymmetric blocks of the Oseen operator).
inline bool fast_cell_packed(int nK, bool full) { return nK <= 18 && !full; }
// Packed blocks are stored in 16-byte groups (pairs of doubles, quads of
// floats): room for the words rounded up to a multiple of 4.  The FP16 copy
// (groups of eight halves) holds fast_cell_words16 halves per cell.
inline long fast_cell_words(int nK, bool full = false) {
  return fast_cell_packed(nK, full) ? ((long)nK * (nK + 1) / 2 + 3) / 4 * 4 : (long)nK * nK;
}
inline long fast_cell_words16(int nK) { return ((long)nK * (nK + 1) / 2 + 7) / 8 * 8; }

// Words of one slot of the fused colour phase's cell storage: the coupling
// of the two patch facets to the far facet (the 2 m2 x m2 block of rows
// 0..2 m2 - 1 and columns 2 m2..3 m2 - 1 of the reordered block), row by
// row, rounded up to whole 16-byte groups (word: bytes per word).
__host__ __device__ constexpr int fast_cell_words_patch(int m2, int word) {
  return (2 * m2 * m2 * word + 15) / 16 * 16 / word;
}

// Patch-inverse storage of the zero-padded NS = FAST_NF*m2 square inverses:
// symmetric operators (full = false) the upper triangle, patch after patch,
// NS(NS+1)/2 words rounded up to a multiple of 8 (16-byte aligned in every
// precision); else the square.
__host__ __device__ constexpr int fast_patch_words_sym(int ns) { return (ns * (ns + 1) / 2 + 7) / 8 * 8; }
inline long fast_patch_words(int m2, bool full) {
  const long ns = (long)FAST_NF * m2;
  return full ? ns * ns : fast_patch_words_sym((int)ns);
}

// y_F[(2F+side)*m2 + c] = rows of S_K x_K for every cell K (m2 = 2 modes
// per facet component x 2 components).
// TS = _Float16 (packed blocks only): al[K] = (s, c0, c1, c2) as
// launch_cells_f16 writes it; else al is null.
// ev: when given, the launch records ev->start and ev->stop as part of its
// dispatch (hipExtLaunchKernelGGL), so that their interval is the kernel's
// own execution; eager launches only (timers are off under graph capture).
struct KernelEvents {
  hipEvent_t start, stop;
};
template <typename TS>
void launch_cell_apply(hipStream_t st, int m2, int nc, const TS* Sp, const int* cdof, const double* x,
                       double* yF, bool full = false, const float4* al = nullptr,
                       const KernelEvents* ev = nullptr);
// y = b + alpha * (y_F[side 0] + y_F[side 1]) (b may be null)
void launch_facet_sum(hipStream_t st, int nint, int m2, const double* yF, const double* b, double alpha,
                      double* y);
// x_s += A_ss^-1 (b - y)_s for the np patches of one colour (Pp in the
// layout fast_patch_words(m2, full) describes; sc: per-patch scales of FP16
// inverses, else null); yF null: y = 0
template <typename TS>
void launch_patch_relax(hipStream_t st, int m2, int np, const int* pf, const TS* Pp, const double* b,
                        const double* yF, double* x, bool full = true, const float* sc = nullptr,
                        const KernelEvents* ev = nullptr);
// One Gauss-Seidel colour phase of symmetric operators in one launch, in
// the direct form x_s = A_ss^-1 (b_s - A_{s,r} x_r) for the np patches of
// the colour (r: the far facets of the patch cells), from the patches'
// upper-triangle inverses Pp, the colour's patch-ordered coupling slots Sc
// and its metadata (see fast.hip); m2 in {2, 4, 6} and ncp in {6, 7} slots
// per patch (fast_fused_supported).
bool fast_fused_supported(int m2, int ncp);
template <typename TS>
void launch_patch_gs_fused(hipStream_t st, int m2, int ncp, int np, const int* pf, const int* meta, const TS* Pp,
                           const TS* Sc, const double* b, double* x, const KernelEvents* ev = nullptr);
// Full row-major FP64 blocks S [nc][3 m2][3 m2] -> one colour's slots (the
// coupling of each cell's two patch facets to its far facet):
// code[t] = cell * 4 + local index of the facet opposite the patch vertex,
// or -1 for a padding slot.
template <typename TS>
void launch_pack_cells_patch(hipStream_t st, int nslot, int m2, const int* code, const double* S, TS* Sc);
void launch_pack_cells(hipStream_t st, int nc, int nK, const double* S, double* Sp, bool full = false);
// FP32 copy of packed blocks (pair groups -> quad groups).
void launch_regroup_cells_f32(hipStream_t st, int nc, int nK, const double* Sp, float* Sp32);
void launch_pack_patches(hipStream_t st, int np, int gp0, int m2, const int* pf_ptr, const long* pinv_off,
                         const double* pinv, double* Pp, bool full = true);
// FP16 copies for the half-precision V-cycle storage.  Packed cell blocks
// (FP64 pair groups -> groups of eight): S0_K = S_K without its
// augmented-Lagrangian term eps^-1 |K|^-1 d d^T (d_i = cdiv[3K+i] on the
// mode-0 normal unknowns) and without boundary rows and columns, divided by
// its largest magnitude s; al[K] = (s, sqrt(eps^-1/|K|) d_0, .. d_1, .. d_2).
// Patch inverses (full or upper-triangle layout, as Pp): each divided by its
// largest magnitude (sc: np floats).
void launch_cells_f16(hipStream_t st, int nc, int m2, const double* Sp, const int* cdof, const double* cdiv,
                      const double* area, double eps_inv, _Float16* Sp16, float4* al);
void launch_patches_f16(hipStream_t st, int np, int m2, const double* Pp, _Float16* P16, float* sc, bool full);

}  // namespace hdgmg
