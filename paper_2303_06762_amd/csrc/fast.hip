// Streaming kernels for the skeleton apply and the vertex-patch block
// Gauss-Seidel on levels whose patches have at most FAST_NF facets.
//
// Storage (structure-of-arrays so that consecutive threads read consecutive
// addresses):
//   Sp   cell blocks of A^eps, packed upper triangle row by row, in
//        16-byte groups (G = 2 doubles or 4 floats): entry e of cell K at
//        Sp[((e / G) * nc + K) * G + e % G]
//   cdof per cell and local facet: 2 * interior facet + side (the side the
//        cell occupies in that facet's cell pair), or -1 on the boundary:
//        cdof[i * nc + K]
//   yF   per interior facet and side, the facet's rows of S_K x_K:
//        yF[(2 F + side) * M2 + c]
//   pf   per patch of one colour its facets, padded with -1: pf[a * np + p]
//   Sf   (k >= 3) cell blocks in full: entry (a, b) of cell K at
//        Sf[(b * nc + K) * NK + a]; a thread per (cell, row)
//   Pp   patch inverses, zero-padded to FAST_NF facets (NS = FAST_NF m2 rows).
//        Nonsymmetric operators: in full, entry (i, j) of patch p at
//        Pp[(j * np + p) * NS + i]; a thread per (patch, row) so that every
//        j-step reads one contiguous run of the workgroup.  Symmetric
//        operators: the upper triangle, entry (a <= b) at Pp[e(a, b) * np + p]
//        with e(a, b) = a NS - a (a - 1) / 2 + b - a; a thread per (row,
//        patch), 16 consecutive patches per row, so that a wavefront reads
//        four 16-patch runs per step
//   Sc   (fused colour phase) per colour, the blocks of each patch's cells
//        in patch order, NCP slots per patch (zero padding slots): with the
//        cell's local facets reordered so that the facet opposite the patch
//        vertex (the far facet) comes last, a slot holds the coupling of the
//        two patch facets to the far facet, rows 0..2 m2 - 1 and columns
//        2 m2..3 m2 - 1 of the reordered block, row by row,
//        fast_cell_words_patch words
//   meta (fused colour phase) per patch of one colour, field-major
//        ([field][np]): for each cell slot the interior ids of its three
//        reordered facets (-1 on the boundary and in padding slots), and for
//        each patch facet slot the two (cell slot, place among the cell's
//        two patch facets) pairs holding it, one byte each (slot * 4 + place)
// A Gauss-Seidel colour phase is a cell apply (y = S x for every cell) then
// k_patch_relax (x_s += A_ss^-1 (b - y)_s for the colour's patches), or one
// fused kernel (k_patch_gs_fused) in the direct form of the same step,
// x_s = A_ss^-1 (b_s - A_{s,r} x_r) (r: the unknowns outside the patch, here
// those of the far facets; the A_ss x_s term of the other form cancels).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fast.hpp"

namespace hdgmg {

namespace {

// Packed blocks are read in 16-byte groups per lane: pairs of doubles,
// quads of floats (entry e of cell K at [((e / G) * nc + K) * G + e % G]).
template <typename TS>
struct Grp;
template <>
struct Grp<double> {
  using T = double2;
  static constexpr int G = 2;
  __device__ static double get(const double2& v, int i) { return i == 0 ? v.x : v.y; }
};
template <>
struct Grp<float> {
  using T = float4;
  static constexpr int G = 4;
  __device__ static float get(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
};
template <>
struct Grp<_Float16> {
  using T = _Float16 __attribute__((ext_vector_type(8)));
  static constexpr int G = 8;
  __device__ static float get(const T& v, int i) { return (float)v[i]; }
};

// al: FP16 blocks only (else null), per cell (s, c0, c1, c2): the stored
// block is S0_K / s, where S0_K is S_K without the augmented-Lagrangian term
// c c^T on the mode-0 normal unknowns (c_i = sqrt(eps^-1 / |K|) sigma_i |F_i|)
// and without the rows and columns of boundary facets; the term is applied
// here from c.
template <int M2, typename TS>
__global__ void __launch_bounds__(256) k_cell_apply(int nc, const TS* __restrict__ Sp, const int* __restrict__ cdof,
                                                    const double* __restrict__ x, double* __restrict__ yF,
                                                    const float4* __restrict__ al) {
  constexpr int NK = 3 * M2;
  using GT = Grp<TS>;
  using V = typename GT::T;
  constexpr int G = GT::G;
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nc) return;
  int cd[3];
  double xl[NK], yl[NK];
#pragma unroll
  for (int i = 0; i < 3; ++i) cd[i] = cdof[i * nc + K];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < M2; ++c) xl[i * M2 + c] = cd[i] >= 0 ? x[(long)(cd[i] >> 1) * M2 + c] : 0.0;
#pragma unroll
  for (int a = 0; a < NK; ++a) yl[a] = 0.0;
  // walk the packed entries (a, b >= a) in order, one group load per G entries
  const V* q = (const V*)Sp + K;
  V cur{};
  int e = 0;
#pragma unroll
  for (int a = 0; a < NK; ++a) {
#pragma unroll
    for (int b = a; b < NK; ++b, ++e) {
      if (e % G == 0) {
        cur = *q;
        q += nc;
      }
      const double s = (double)GT::get(cur, e % G);
      yl[a] += s * xl[b];
      if (b != a) yl[b] += s * xl[a];
    }
  }
  if (al) {
    const float4 w = al[K];
    const double c[3] = {(double)w.y, (double)w.z, (double)w.w};
    const double dx = c[0] * xl[0] + c[1] * xl[M2] + c[2] * xl[2 * M2];
#pragma unroll
    for (int a = 0; a < NK; ++a) yl[a] *= (double)w.x;
#pragma unroll
    for (int i = 0; i < 3; ++i) yl[i * M2] += c[i] * dx;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (cd[i] >= 0)
#pragma unroll
      for (int c = 0; c < M2; ++c) yF[(long)cd[i] * M2 + c] = yl[i * M2 + c];
}

__global__ void k_facet_sum(long n, int m2, const double* __restrict__ yF, const double* __restrict__ b,
                            double alpha, double* __restrict__ y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const long F = t / m2, c = t % m2;
  const double v = alpha * (yF[(2 * F) * m2 + c] + yF[(2 * F + 1) * m2 + c]);
  y[t] = b ? b[t] + v : v;
}

// Rows of S_K x_K with a thread per (cell, row): x_K staged in LDS.
template <int M2, typename TS>
__global__ void __launch_bounds__(256) k_cell_apply_rows(int nc, const TS* __restrict__ Sf,
                                                         const int* __restrict__ cdof,
                                                         const double* __restrict__ x, double* __restrict__ yF) {
  constexpr int NK = 3 * M2, CPB = 256 / NK;
  __shared__ double xs[CPB][NK];
  const int lc = threadIdx.x / NK, a = threadIdx.x % NK;
  const int K = blockIdx.x * CPB + lc;
  const bool on = lc < CPB && K < nc;
  int cd = -1;
  if (on) {
    const int cda = cdof[(a / M2) * nc + K];
    xs[lc][a] = cda >= 0 ? x[(long)(cda >> 1) * M2 + a % M2] : 0.0;
    cd = cda;
  }
  __syncthreads();
  if (!on) return;
  double y = 0.0;
  const TS* q = Sf + (long)K * NK + a;
#pragma unroll
  for (int b = 0; b < NK; ++b) {
    y += (double)*q * xs[lc][b];
    q += (long)nc * NK;
  }
  if (cd >= 0) yF[(long)cd * M2 + a % M2] = y;
}

// x_s += A_ss^-1 (b - y)_s for the patches of one colour: a thread per
// (patch, row), the patch residual shared through LDS.
// sc: per-patch scale of FP16 inverses, else null.
template <int M2, typename TS>
__global__ void __launch_bounds__(256) k_patch_relax(int np, const int* __restrict__ pf, const TS* __restrict__ Pp,
                                                     const double* __restrict__ b, const double* __restrict__ yF,
                                                     double* __restrict__ x, const float* __restrict__ sc) {
  constexpr int NS = FAST_NF * M2, PPB = 256 / NS;
  __shared__ double rs[PPB][NS];
  const int lp = threadIdx.x / NS, i = threadIdx.x % NS;
  const int p = blockIdx.x * PPB + lp;
  const bool on = lp < PPB && p < np;
  int f = -1;
  if (on) {
    f = pf[(i / M2) * np + p];
    const int c = i % M2;
    double r = 0.0;
    if (f >= 0) {
      r = b[(long)f * M2 + c];
      if (yF) r -= yF[(long)(2 * f) * M2 + c] + yF[(long)(2 * f + 1) * M2 + c];
    }
    rs[lp][i] = r;
  }
  __syncthreads();
  if (!on) return;
  double d = 0.0;
  const TS* q = Pp + (long)p * NS + i;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    d += (double)*q * rs[lp][j];
    q += (long)np * NS;
  }
  if (sc) d *= (double)sc[p];
  if (f >= 0) x[(long)f * M2 + i % M2] += d;
}

// The same relaxation from the upper triangles of symmetric inverses, a
// wavefront per patch (per 64 / NS consecutive patches when NS <= 32): the
// triangles (contiguous, PW words each) are read once with 16-byte loads by
// all 64 lanes into LDS, the patch residuals go to LDS, and lane (patch,
// row i) forms row i of the inverse times the residual from the triangle:
// entry (i, j) at e(min(i, j), max(i, j)), e(a, b) = a NS - a (a - 1) / 2 +
// b - a.  Every entry crosses HBM once.  sc: per-patch scale of FP16
// triangles, else null.
template <int M2>
struct WaveShape {
  static constexpr int NS = FAST_NF * M2;
  static constexpr int PPW = NS <= 32 ? 64 / NS : 1;  // patches per wavefront
};
template <int M2, typename TS, bool HY>
__global__ void __launch_bounds__(64) k_patch_relax_wave(int np, const int* __restrict__ pf, const TS* __restrict__ Pp,
                                                         const double* __restrict__ b, const double* __restrict__ yF,
                                                         double* __restrict__ x, const float* __restrict__ sc) {
  constexpr int NS = FAST_NF * M2, PPW = WaveShape<M2>::PPW;
  constexpr int PW = fast_patch_words_sym(NS);
  constexpr int N16 = PPW * PW * (int)sizeof(TS) / 16;  // the wavefront's triangles
  constexpr int NL = (N16 + 63) / 64;
  __shared__ uint4 As[NL * 64];
  __shared__ double rs[PPW * NS];
  const int lane = threadIdx.x;
  const int lp = lane / NS, i = lane % NS;  // patch of the wavefront, row
  const int p0 = blockIdx.x * PPW;
  const int p = p0 + lp;
  const bool on = lp < PPW && p < np;
  const int f = on ? pf[(i / M2) * np + p] : -1;
  // every load of the triangles in flight before the first LDS store (the
  // last patches of the colour re-read the final triangle)
  const long last16 = (long)np * PW * (long)sizeof(TS) / 16 - 1;
  const uint4* src = (const uint4*)(Pp + (long)p0 * PW);
  const long rem = last16 - (long)p0 * PW * (long)sizeof(TS) / 16;
  uint4 w[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) w[q] = src[min((long)min(lane + 64 * q, N16 - 1), rem)];
  // the residual's gathers without branches (row 0 stands in for padding)
  const int fc = f >= 0 ? f : 0, c = i % M2;
  const double bv = b[(long)fc * M2 + c];
  double y0 = 0.0, y1 = 0.0;
  if constexpr (HY) {
    y0 = yF[(long)(2 * fc) * M2 + c];
    y1 = yF[(long)(2 * fc + 1) * M2 + c];
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) As[lane + 64 * q] = w[q];  // slots past N16 are never read
  if (lp < PPW) rs[lane] = f >= 0 ? bv - (y0 + y1) : 0.0;
  __syncthreads();
  if (!on) return;
  const TS* A = (const TS*)As + lp * PW;
  const double* r = rs + lp * NS;
  const int rowi = i * NS - i * (i - 1) / 2 - i;  // e(i, j) = rowi + j for j >= i
  double d = 0.0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int colj = j * NS - j * (j - 1) / 2 - j;  // e(j, i) = colj + i for j < i
    const int e = j < i ? colj + i : rowi + j;
    d += (double)A[e] * r[j];
  }
  if (sc) d *= (double)sc[p];
  if (f >= 0) x[(long)f * M2 + c] += d;
}

// One Gauss-Seidel colour phase in one kernel, symmetric operators: a
// wavefront per patch (per PPW consecutive patches).  Within a colour the
// cells around a patch vertex belong to no other patch of the colour, the
// patch facets to no other patch, and the cells' remaining facets to no
// patch of the colour at all, so the step needs only the patch's own cells
// and x values no other wavefront of the launch changes.  In its direct form
//   g_s = b_s - sum over the patch cells K of (S_K)_{patch facets, far facet} x_far,
//   x_s = A_ss^-1 g_s
// (equal to x_s += A_ss^-1 (b - A x)_s: the A_ss x_s term cancels), each
// cell contributes only the coupling of its two patch facets to its far
// facet.  The colour's coupling blocks are stored patch by patch (Sc, see
// the layout notes at the top), so a wavefront's blocks and triangles are
// two contiguous runs, loaded with the metadata in the first round; the x
// (far facets) and b gathers wait on the metadata.  Every load is issued
// before the first LDS store; the triangles go to LDS once the right-hand
// side no longer needs the blocks.
// 16-byte words as a native vector (plain loads and stores, kept in
// registers)
typedef unsigned int U4 __attribute__((ext_vector_type(4)));
template <int M2, int NCP, typename TS>
struct FusedShape {
  static constexpr int NS = FAST_NF * M2, NK = 3 * M2, PPW = WaveShape<M2>::PPW;
  static constexpr int PW = fast_patch_words_sym(NS);
  static constexpr int CR = fast_cell_words_patch(M2, (int)sizeof(TS));  // one slot
  static constexpr int T16 = PPW * PW * (int)sizeof(TS) / 16;  // the wavefront's triangles
  static constexpr int C16 = PPW * NCP * CR * (int)sizeof(TS) / 16;  // ... and cell blocks
  static constexpr int NCELL = PPW * NCP;
  static constexpr int NX = NCELL * M2;  // x on the cells' far facets
  static constexpr int NLT = (T16 + 63) / 64, NLC = (C16 + 63) / 64, NLX = (NX + 63) / 64;
};
// (LDS holds about 16 wavefronts per CU; four per SIMD leave 128 registers,
// so that the triangles stay in registers while the residual is formed)
template <int M2, int NCP, typename TS>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_patch_gs_fused(int np, const int* __restrict__ pf, const int* __restrict__ meta, const TS* __restrict__ Pp,
                 const TS* __restrict__ Sc, const double* __restrict__ b, double* __restrict__ x) {
  using F = FusedShape<M2, NCP, TS>;
  constexpr int NS = F::NS, PPW = F::PPW, PW = F::PW, CR = F::CR;
  constexpr int T16 = F::T16, C16 = F::C16, NX = F::NX;
  __shared__ U4 Bs[T16 > C16 ? T16 : C16];  // the coupling blocks, then the triangles
  __shared__ double xs[NX];
  __shared__ double rs[PPW * NS];
  const int lane = threadIdx.x;
  const int lp = lane / NS, i = lane % NS;  // patch of the wavefront, row
  // workgroups go round-robin to the eight XCDs (each with its own L2):
  // give each XCD a contiguous run of the colour's patches, whose cells,
  // facets and x and b rows are neighbours (the last partial round keeps
  // its order)
  const int nb = gridDim.x, full = nb / 8 * 8;
  const int g = (int)blockIdx.x < full ? ((int)blockIdx.x % 8) * (full / 8) + (int)blockIdx.x / 8 : (int)blockIdx.x;
  const int p0 = g * PPW;
  const int p = p0 + lp;
  const bool on = lp < PPW && p < np;
  // metadata first, every load unconditional (indices clamped into the
  // colour; what a lane of a padding patch reads is never used): the far
  // facets of the x items, the patch rows' facet and sides
  int xf[F::NLX];
#pragma unroll
  for (int q = 0; q < F::NLX; ++q) {
    const int t = min(lane + 64 * q, NX - 1), j = t / M2;
    xf[q] = meta[((j % NCP) * 3 + 2) * np + min(p0 + j / NCP, np - 1)];
  }
  const int pc = min(p, np - 1);
  const int fr = pf[(i / M2) * np + pc];
  const int ps = meta[(3 * NCP + i / M2) * np + pc];
  const int f = on ? fr : -1;
  const int c = i % M2;
  // then the triangles and the cell blocks (a lane past the end of the
  // colour re-reads its last word), then the x and b gathers
  const long lastT = (long)np * PW * (long)sizeof(TS) / 16 - 1;
  const long remT = lastT - (long)p0 * PW * (long)sizeof(TS) / 16;
  const U4* srcT = (const U4*)(Pp + (long)p0 * PW);
  U4 w[F::NLT];
#pragma unroll
  for (int q = 0; q < F::NLT; ++q) w[q] = srcT[min((long)min(lane + 64 * q, T16 - 1), remT)];
  const long lastC = (long)np * NCP * CR * (long)sizeof(TS) / 16 - 1;
  const long remC = lastC - (long)p0 * NCP * CR * (long)sizeof(TS) / 16;
  const U4* srcC = (const U4*)(Sc + (long)p0 * NCP * CR);
  U4 cw[F::NLC];
#pragma unroll
  for (int q = 0; q < F::NLC; ++q) cw[q] = srcC[min((long)min(lane + 64 * q, C16 - 1), remC)];
  const double bv = b[(long)max(f, 0) * M2 + c];
  double xv[F::NLX];
#pragma unroll
  for (int q = 0; q < F::NLX; ++q) {
    const int t = min(lane + 64 * q, NX - 1);
    const double v = x[(long)max(xf[q], 0) * M2 + t % M2];
    xv[q] = xf[q] >= 0 ? v : 0.0;  // boundary facets carry no unknowns
  }
  // stores without branches: a lane past the end loaded the last word and
  // writes it again
#pragma unroll
  for (int q = 0; q < F::NLC; ++q) Bs[min(lane + 64 * q, C16 - 1)] = cw[q];
#pragma unroll
  for (int q = 0; q < F::NLX; ++q) xs[min(lane + 64 * q, NX - 1)] = xv[q];
  // the row's sides and b are used only after the barrier; an empty
  // statement that takes both in registers keeps their loads with the others
  asm volatile("" ::"v"(bv), "v"(ps));
  __syncthreads();
  // right-hand side rows: lane (patch, row i = facet slot * M2 + c).  Every
  // lane computes one without branches (so that the loads above stay ahead
  // of the stores); lanes past the wavefront's patches and padding rows
  // keep their slots and rows in range and discard the result.  A side's
  // code is slot * 4 + its place (0 or 1) among the cell's two patch
  // facets; row a < 2 M2 of a slot couples to the far facet's M2 values
  // (entry (a, c') at a M2 + c').
  {
    const int lpc = min(lp, PPW - 1);
    double y = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int code = (ps >> (8 * s)) & 0xff;
      const int slot = lpc * NCP + min(code >> 2, NCP - 1), row = min(code & 3, 1) * M2 + c;
      const TS* S = (const TS*)Bs + slot * CR + row * M2;
      const double* xk = xs + slot * M2;
#pragma unroll
      for (int bb = 0; bb < M2; ++bb) y += (double)S[bb] * xk[bb];
    }
    const double r = f >= 0 ? bv - y : 0.0;
    if (lp < PPW) rs[lane] = r;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::NLT; ++q) Bs[min(lane + 64 * q, T16 - 1)] = w[q];
  __syncthreads();
  if (!on) return;
  const TS* A = (const TS*)Bs + lp * PW;
  const double* rr = rs + lp * NS;
  const int rowi = i * NS - i * (i - 1) / 2 - i;
  double d = 0.0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int colj = j * NS - j * (j - 1) / 2 - j;
    const int e = j < i ? colj + i : rowi + j;
    d += (double)A[e] * rr[j];
  }
  if (f >= 0) x[(long)f * M2 + c] = d;
}

// Full row-major FP64 cell blocks -> the patch-ordered slots of one colour:
// slot t holds cell K = code >> 2 with its local facets reordered as (the
// two others in increasing order, far = code & 3), the coupling of the
// first two reordered facets to the far facet (row a < 2 m2, column c < m2
// at a m2 + c); code < 0 (padding): zeros.
template <typename TS>
__global__ void k_pack_cells_patch(int nslot, int m2, int cr, const int* __restrict__ code,
                                   const double* __restrict__ S, TS* __restrict__ Sc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslot) return;
  const int nK = 3 * m2, cd = code[t];
  TS* out = Sc + (long)t * cr;
  int e = 0;
  if (cd >= 0) {
    const int K = cd >> 2, far = cd & 3;
    const int perm[2] = {far == 0 ? 1 : 0, far == 2 ? 1 : 2};
    const double* B = S + (long)K * nK * nK;
    for (int a = 0; a < 2 * m2; ++a)
      for (int c = 0; c < m2; ++c, ++e) out[e] = (TS)B[(perm[a / m2] * m2 + a % m2) * nK + far * m2 + c];
  }
  for (; e < cr; ++e) out[e] = (TS)0;
}

// Full row-major cell blocks -> packed SoA in groups of G (G = 2 for the
// FP64 copy; the FP32 copy is regrouped by k_regroup_f32).
template <typename TS>
__global__ void k_pack_cells(int nc, int nK, const double* __restrict__ S, TS* __restrict__ Sp) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nc) return;
  long e = 0;
  for (int a = 0; a < nK; ++a)
    for (int b = a; b < nK; ++b, ++e) Sp[((e / 2) * nc + K) * 2 + e % 2] = (TS)S[((long)K * nK + a) * nK + b];
}

// FP64 pair-grouped packed blocks -> FP32 quad-grouped copy.
__global__ void k_regroup_f32(int nc, long nw, const double* __restrict__ Sp, float* __restrict__ Sp32) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nw * nc) return;
  const long e = t / nc, K = t % nc;
  Sp32[((e / 4) * nc + K) * 4 + e % 4] = (float)Sp[((e / 2) * nc + K) * 2 + e % 2];
}

// FP64 pair-grouped packed blocks -> FP16 groups of eight (the layout
// k_cell_apply<M2, _Float16> reads): the augmented-Lagrangian term and the
// boundary rows and columns removed, the rest divided by its largest
// magnitude; al[K] = (that magnitude, c0, c1, c2).  cdiv: sigma |F| per
// (cell, local facet), 0 on the boundary; area: |K|.
__global__ void k_regroup_f16(int nc, int m2, const double* __restrict__ Sp, const int* __restrict__ cdof,
                              const double* __restrict__ cdiv, const double* __restrict__ area, double eps_inv,
                              _Float16* __restrict__ Sp16, float4* __restrict__ al) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nc) return;
  const int nK = 3 * m2;
  const double w = eps_inv / area[K];
  double dv[3];
  bool in[3];
  for (int i = 0; i < 3; ++i) {
    dv[i] = cdiv[3 * K + i];
    in[i] = cdof[i * nc + K] >= 0;
  }
  auto value = [&](int a, int b, long e) {
    const int fa = a / m2, fb = b / m2;
    if (!in[fa] || !in[fb]) return 0.0;
    double v = Sp[((e / 2) * nc + K) * 2 + e % 2];
    if (a % m2 == 0 && b % m2 == 0) v -= w * dv[fa] * dv[fb];
    return v;
  };
  double mx = 0.0;
  long e = 0;
  for (int a = 0; a < nK; ++a)
    for (int b = a; b < nK; ++b, ++e) mx = fmax(mx, fabs(value(a, b, e)));
  const double f = mx > 0.0 ? mx : 1.0;
  const double sw = sqrt(w);
  al[K] = make_float4((float)f, (float)(sw * dv[0]), (float)(sw * dv[1]), (float)(sw * dv[2]));
  e = 0;
  for (int a = 0; a < nK; ++a)
    for (int b = a; b < nK; ++b, ++e) Sp16[((e / 8) * nc + K) * 8 + e % 8] = (_Float16)(value(a, b, e) / f);
}

// FP64 full patch inverses ([j][p][i]) -> FP16, each divided by its largest
// magnitude (kept in sc[p]).
__global__ void k_patches_f16(int np, int ns, const double* __restrict__ Pp, _Float16* __restrict__ P16,
                              float* __restrict__ sc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double mx = 0.0;
  for (int j = 0; j < ns; ++j)
    for (int i = 0; i < ns; ++i) mx = fmax(mx, fabs(Pp[((long)j * np + p) * ns + i]));
  const double f = mx > 0.0 ? mx : 1.0;
  sc[p] = (float)f;
  for (int j = 0; j < ns; ++j)
    for (int i = 0; i < ns; ++i) P16[((long)j * np + p) * ns + i] = (_Float16)(Pp[((long)j * np + p) * ns + i] / f);
}

// Full row-major cell blocks -> [b][K][a] SoA.
template <typename TS>
__global__ void k_pack_cells_full(int nc, int nK, const double* __restrict__ S, TS* __restrict__ Sf) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nc) return;
  for (int a = 0; a < nK; ++a)
    for (int b = 0; b < nK; ++b) Sf[((long)b * nc + K) * nK + a] = (TS)S[((long)K * nK + a) * nK + b];
}

// Column-major per-patch inverses (patches gp0 .. gp0+np of one colour) ->
// [j][p][i] zero-padded to FAST_NF facets.
template <typename TS>
__global__ void k_pack_patches(int np, int gp0, int m2, const int* __restrict__ pf_ptr,
                               const long* __restrict__ pinv_off, const double* __restrict__ pinv,
                               TS* __restrict__ Pp) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int gp = gp0 + p;
  const int ns = (pf_ptr[gp + 1] - pf_ptr[gp]) * m2;
  const int NS = FAST_NF * m2;
  const double* A = pinv + pinv_off[gp];
  for (int j = 0; j < NS; ++j)
    for (int i = 0; i < NS; ++i)
      Pp[((long)j * np + p) * NS + i] = (i < ns && j < ns) ? (TS)A[(long)j * ns + i] : (TS)0;
}

// Column-major per-patch inverses -> upper triangles, patch p at
// Pp[p * PW ...] (the mean of the two computed entries; zero padding).
template <typename TS>
__global__ void k_pack_patches_sym(int np, int gp0, int m2, const int* __restrict__ pf_ptr,
                                   const long* __restrict__ pinv_off, const double* __restrict__ pinv,
                                   TS* __restrict__ Pp) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int gp = gp0 + p;
  const int ns = (pf_ptr[gp + 1] - pf_ptr[gp]) * m2;
  const int NS = FAST_NF * m2;
  const long PW = fast_patch_words_sym(NS);
  const double* A = pinv + pinv_off[gp];
  TS* out = Pp + (long)p * PW;
  long e = 0;
  for (int a = 0; a < NS; ++a)
    for (int c = a; c < NS; ++c, ++e)
      out[e] = (a < ns && c < ns) ? (TS)(0.5 * (A[(long)c * ns + a] + A[(long)a * ns + c])) : (TS)0;
  for (; e < PW; ++e) out[e] = (TS)0;
}

// FP64 upper triangles -> FP16, each divided by its largest magnitude
// (kept in sc[p]).
__global__ void k_patches_sym_f16(int np, int m2, const double* __restrict__ Pp, _Float16* __restrict__ P16,
                                  float* __restrict__ sc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const long PW = fast_patch_words_sym(FAST_NF * m2);
  const double* in = Pp + (long)p * PW;
  double mx = 0.0;
  for (long e = 0; e < PW; ++e) mx = fmax(mx, fabs(in[e]));
  const double f = mx > 0.0 ? mx : 1.0;
  sc[p] = (float)f;
  for (long e = 0; e < PW; ++e) P16[(long)p * PW + e] = (_Float16)(in[e] / f);
}

inline int nblk(long n, int t = 256) { return (int)((n + t - 1) / t); }

// A launch on st, through hipExtLaunchKernelGGL with ev's start / stop
// events when ev is given.
#define LAUNCH_EV(KERNEL, GRID, BLOCK, ...)                                                        \
  do {                                                                                             \
    if (ev)                                                                                        \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, st, ev->start, ev->stop, 0, __VA_ARGS__);      \
    else                                                                                           \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, st, __VA_ARGS__);                                 \
  } while (0)

template <typename TS>
void cell_apply_t(hipStream_t st, int m2, int nc, const TS* Sp, const int* cdof, const double* x, double* yF,
                  bool full, const float4* sc, const KernelEvents* ev) {
  if (!fast_cell_packed(3 * m2, full)) {
    switch (m2) {
#define CASE(M)                                                                                        \
  case M:                                                                                              \
    LAUNCH_EV((k_cell_apply_rows<M, TS>), dim3((nc + 256 / (3 * M) - 1) / (256 / (3 * M))), dim3(256), \
              nc, Sp, cdof, x, yF);                                                            \
    break;
      CASE(2) CASE(4) CASE(6) CASE(8) CASE(10)
#undef CASE
    }
    return;
  }
  switch (m2) {
#define CASE(M)                                                                                  \
  case M:                                                                                        \
    LAUNCH_EV((k_cell_apply<M, TS>), dim3(nblk(nc)), dim3(256), nc, Sp, cdof, x, yF, sc); \
    break;
    CASE(2) CASE(4) CASE(6)
#undef CASE
  }
}

template <typename TS>
void patch_relax_t(hipStream_t st, int m2, int np, const int* pf, const TS* Pp, const double* b, const double* yF,
                   double* x, bool full, const float* sc, const KernelEvents* ev) {
  if (!full) {
    switch (m2) {
#define CASE(M)                                                                                                \
  case M:                                                                                                      \
    if (yF)                                                                                                    \
      LAUNCH_EV((k_patch_relax_wave<M, TS, true>), dim3((np + WaveShape<M>::PPW - 1) / WaveShape<M>::PPW),     \
                dim3(64), np, pf, Pp, b, yF, x, sc);                                                          \
    else                                                                                                       \
      LAUNCH_EV((k_patch_relax_wave<M, TS, false>), dim3((np + WaveShape<M>::PPW - 1) / WaveShape<M>::PPW),    \
                dim3(64), np, pf, Pp, b, yF, x, sc);                                                          \
    break;
      CASE(2) CASE(4) CASE(6) CASE(8) CASE(10)
#undef CASE
    }
    return;
  }
  switch (m2) {
#define CASE(M)                                                                                            \
  case M:                                                                                                  \
    LAUNCH_EV((k_patch_relax<M, TS>), dim3((np + 256 / (6 * M) - 1) / (256 / (6 * M))), dim3(256), np, pf, Pp, \
              b, yF, x, sc);                                                                               \
    break;
    CASE(2) CASE(4) CASE(6) CASE(8) CASE(10)
#undef CASE
  }
}

template <typename TS>
void patch_gs_fused_t(hipStream_t st, int m2, int ncp, int np, const int* pf, const int* meta, const TS* Pp,
                      const TS* Sc, const double* b, double* x, const KernelEvents* ev) {
#define CASE(M, N)                                                                                            \
  if (m2 == M && ncp == N) {                                                                                 \
    LAUNCH_EV((k_patch_gs_fused<M, N, TS>), dim3((np + WaveShape<M>::PPW - 1) / WaveShape<M>::PPW), dim3(64), \
              np, pf, meta, Pp, Sc, b, x);                                                                   \
    return;                                                                                                  \
  }
  CASE(2, 6) CASE(2, 7) CASE(4, 6) CASE(4, 7) CASE(6, 6) CASE(6, 7)
#undef CASE
}

#undef LAUNCH_EV

}  // namespace

bool fast_fused_supported(int m2, int ncp) { return (m2 == 2 || m2 == 4 || m2 == 6) && (ncp == 6 || ncp == 7); }

template <typename TS>
void launch_patch_gs_fused(hipStream_t st, int m2, int ncp, int np, const int* pf, const int* meta, const TS* Pp,
                           const TS* Sc, const double* b, double* x, const KernelEvents* ev) {
  if (np > 0) patch_gs_fused_t<TS>(st, m2, ncp, np, pf, meta, Pp, Sc, b, x, ev);
}
template void launch_patch_gs_fused<double>(hipStream_t, int, int, int, const int*, const int*, const double*,
                                            const double*, const double*, double*, const KernelEvents*);
template void launch_patch_gs_fused<float>(hipStream_t, int, int, int, const int*, const int*, const float*,
                                           const float*, const double*, double*, const KernelEvents*);

template <typename TS>
void launch_pack_cells_patch(hipStream_t st, int nslot, int m2, const int* code, const double* S, TS* Sc) {
  if (nslot > 0)
    hipLaunchKernelGGL(k_pack_cells_patch<TS>, dim3(nblk(nslot)), dim3(256), 0, st, nslot, m2,
                       fast_cell_words_patch(m2, (int)sizeof(TS)), code, S, Sc);
}
template void launch_pack_cells_patch<double>(hipStream_t, int, int, const int*, const double*, double*);
template void launch_pack_cells_patch<float>(hipStream_t, int, int, const int*, const double*, float*);

template <typename TS>
void launch_cell_apply(hipStream_t st, int m2, int nc, const TS* Sp, const int* cdof, const double* x,
                       double* yF, bool full, const float4* al, const KernelEvents* ev) {
  if (nc > 0) cell_apply_t<TS>(st, m2, nc, Sp, cdof, x, yF, full, al, ev);
}
template void launch_cell_apply<double>(hipStream_t, int, int, const double*, const int*, const double*, double*,
                                        bool, const float4*, const KernelEvents*);
template void launch_cell_apply<float>(hipStream_t, int, int, const float*, const int*, const double*, double*,
                                       bool, const float4*, const KernelEvents*);
template void launch_cell_apply<_Float16>(hipStream_t, int, int, const _Float16*, const int*, const double*,
                                          double*, bool, const float4*, const KernelEvents*);

void launch_facet_sum(hipStream_t st, int nint, int m2, const double* yF, const double* b, double alpha,
                      double* y) {
  const long n = (long)nint * m2;
  if (n > 0) hipLaunchKernelGGL(k_facet_sum, dim3(nblk(n)), dim3(256), 0, st, n, m2, yF, b, alpha, y);
}

template <typename TS>
void launch_patch_relax(hipStream_t st, int m2, int np, const int* pf, const TS* Pp, const double* b,
                        const double* yF, double* x, bool full, const float* sc, const KernelEvents* ev) {
  if (np > 0) patch_relax_t<TS>(st, m2, np, pf, Pp, b, yF, x, full, sc, ev);
}
template void launch_patch_relax<double>(hipStream_t, int, int, const int*, const double*, const double*,
                                         const double*, double*, bool, const float*, const KernelEvents*);
template void launch_patch_relax<float>(hipStream_t, int, int, const int*, const float*, const double*,
                                        const double*, double*, bool, const float*, const KernelEvents*);
template void launch_patch_relax<_Float16>(hipStream_t, int, int, const int*, const _Float16*, const double*,
                                           const double*, double*, bool, const float*, const KernelEvents*);

void launch_cells_f16(hipStream_t st, int nc, int m2, const double* Sp, const int* cdof, const double* cdiv,
                      const double* area, double eps_inv, _Float16* Sp16, float4* al) {
  if (nc > 0)
    hipLaunchKernelGGL(k_regroup_f16, dim3(nblk(nc)), dim3(256), 0, st, nc, m2, Sp, cdof, cdiv, area, eps_inv, Sp16,
                       al);
}

void launch_patches_f16(hipStream_t st, int np, int m2, const double* Pp, _Float16* P16, float* sc, bool full) {
  if (np <= 0) return;
  if (full)
    hipLaunchKernelGGL(k_patches_f16, dim3(nblk(np)), dim3(256), 0, st, np, FAST_NF * m2, Pp, P16, sc);
  else
    hipLaunchKernelGGL(k_patches_sym_f16, dim3(nblk(np)), dim3(256), 0, st, np, m2, Pp, P16, sc);
}

void launch_regroup_cells_f32(hipStream_t st, int nc, int nK, const double* Sp, float* Sp32) {
  const long nw = (long)nK * (nK + 1) / 2;
  if (nc > 0) hipLaunchKernelGGL(k_regroup_f32, dim3(nblk(nw * nc)), dim3(256), 0, st, nc, nw, Sp, Sp32);
}

void launch_pack_cells(hipStream_t st, int nc, int nK, const double* S, double* Sp, bool full) {
  if (nc <= 0) return;
  if (fast_cell_packed(nK, full))
    hipLaunchKernelGGL(k_pack_cells<double>, dim3(nblk(nc)), dim3(256), 0, st, nc, nK, S, Sp);
  else
    hipLaunchKernelGGL(k_pack_cells_full<double>, dim3(nblk(nc)), dim3(256), 0, st, nc, nK, S, Sp);
}

void launch_pack_patches(hipStream_t st, int np, int gp0, int m2, const int* pf_ptr, const long* pinv_off,
                         const double* pinv, double* Pp, bool full) {
  if (np <= 0) return;
  if (full)
    hipLaunchKernelGGL(k_pack_patches<double>, dim3(nblk(np)), dim3(256), 0, st, np, gp0, m2, pf_ptr, pinv_off,
                       pinv, Pp);
  else
    hipLaunchKernelGGL(k_pack_patches_sym<double>, dim3(nblk(np)), dim3(256), 0, st, np, gp0, m2, pf_ptr,
                       pinv_off, pinv, Pp);
}

}  // namespace hdgmg
