// MG_h (Alg. 1) on the coarse lowest-order levels inside one workgroup.
//
// Below a few thousand unknowns a level's work is far smaller than the cost
// of a kernel launch, while the variable V-cycle doubles the number of
// smoothing sweeps on every coarser level.  This kernel runs the recursion
// MG_h(top, g, u, m(top), q) -- pre-smoothing, residual, restriction, the
// coarser visits, prolongation, post-smoothing, the exact coarsest solve --
// with workgroup barriers between dependent phases, in the same order as the
// level-by-level launches: block Gauss-Seidel colour by colour, forward
// before and backward after the coarse correction.
//
// Latency is what matters here, so the level vectors stay in LDS, the level
// descriptors are copied to LDS once, and every patch row carries its own
// padded residual row and inverse row (structure-of-arrays) so that a thread
// issues independent, coalesced loads and then works from LDS.
#include <hip/hip_runtime.h>

#include "coarse.hpp"

namespace hdgmg {

namespace {

constexpr int CT = COARSE_THREADS;

// The descriptors live in LDS, so the compiler cannot tell that the device
// pointers they hold address global memory and would read through them with
// flat loads, which are counted together with LDS accesses: every wait for
// an LDS read would then also wait for all outstanding record loads.  Reads
// through gmem() are global loads, counted apart.
template <typename T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// The record of one patch row: its unknown and row, the facets of its
// residual row (two 16-bit indices per word), residual row, inverse row.
template <int NS, typename TS>
struct Rec {
  unsigned key;
  unsigned fac[3];
  TS val[COARSE_NNZ];
  TS ai[NS];
};

// Groups of record values read with one 16-byte load per lane: pairs of
// doubles, quads of floats (native vector types, which load through
// global-address pointers).  get(v, i) returns component i of a group.
using u32x4 = unsigned __attribute__((ext_vector_type(4)));
template <typename TS>
struct Grp;
template <>
struct Grp<double> {
  using T = double __attribute__((ext_vector_type(2)));
  static constexpr int G = 2;
  __device__ static double get(const T& v, int i) { return v[i]; }
};
template <>
struct Grp<float> {
  using T = float __attribute__((ext_vector_type(4)));
  static constexpr int G = 4;
  __device__ static float get(const T& v, int i) { return v[i]; }
};

// Record parts come from LDS (copied at kernel start) or from memory; each
// part's source is uniform per level.  Part pointers are typed per address
// space so that LDS parts are read with LDS instructions.
template <int NS, typename TS>
__device__ inline void load_rec(const CoarseLevel& L, const char* lds, int t, Rec<NS, TS>& r) {
  using GT = Grp<TS>;
  using V = typename GT::T;
  constexpr int G = GT::G;
  const int nit = L.nitems;
  u32x4 m0;
  if (L.lds_meta >= 0)
    m0 = ((const u32x4*)(lds + L.lds_meta))[t];
  else
    m0 = gmem((const u32x4*)L.it_meta)[t];
  r.key = m0.x;
  r.fac[0] = m0.y;
  r.fac[1] = m0.z;
  r.fac[2] = m0.w;
  constexpr int NVG = (COARSE_NNZ + G - 1) / G;
  V vg[NVG];
  if (L.lds_val >= 0) {
    const V* val = (const V*)(lds + L.lds_val);
#pragma unroll
    for (int e = 0; e < NVG; ++e) vg[e] = val[e * nit + t];
  } else {
    const auto val = gmem((const V*)L.it_val);
#pragma unroll
    for (int e = 0; e < NVG; ++e) vg[e] = val[e * nit + t];
  }
#pragma unroll
  for (int e = 0; e < NVG; ++e)
#pragma unroll
    for (int i = 0; i < G; ++i)
      if (e * G + i < COARSE_NNZ) r.val[e * G + i] = GT::get(vg[e], i);
  V ag[NS / G];
  if (L.lds_ainv >= 0) {
    const V* ainv = (const V*)(lds + L.lds_ainv);
#pragma unroll
    for (int j = 0; j < NS / G; ++j) {
      ag[j] = (V)(TS)0;
      if (j * G < L.ns_max) ag[j] = ainv[j * nit + t];
    }
  } else {
    const auto ainv = gmem((const V*)L.it_ainv);
#pragma unroll
    for (int j = 0; j < NS / G; ++j) {
      ag[j] = (V)(TS)0;
      if (j * G < L.ns_max) ag[j] = ainv[j * nit + t];
    }
  }
#pragma unroll
  for (int j = 0; j < NS / G; ++j)
#pragma unroll
    for (int i = 0; i < G; ++i) r.ai[j * G + i] = GT::get(ag[j], i);
}

// Copy n 16-byte words from memory to LDS with the whole workgroup, eight
// loads in flight per thread before the stores.
__device__ inline void copy_to_lds(void* dst, const void* src, int n) {
  u32x4* d = (u32x4*)dst;
  const auto sp = gmem((const u32x4*)src);
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * CT) {
    u32x4 w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = min(i0 + q * CT, n - 1);
      w[q] = sp[i];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (i0 + q * CT < n) d[i0 + q * CT] = w[q];
  }
}

// `sweeps` block Gauss-Seidel sweeps over the colours (forward or reversed),
// as a flat list of batches.  bitem / bwd: the level's batch item ranges and
// backward batch order, staged in LDS.  A step loads its records when it
// starts: the inverse rows arrive while the residual rows are computed.
// (Holding the next step's records in registers instead, to hide their
// latency, costs more than it saves: with 1024 threads a lane has 128
// registers, and the LDS reads of the residual then run one at a time.)
template <int NS, typename TS>
__device__ void smooth(const CoarseLevel& Ld, const char* lds, const int* bitem, const int* bwd, int sweeps,
                       bool forward, double* __restrict__ res, double* __restrict__ u,
                       const double* __restrict__ g) {
  // the descriptor is read from LDS once: inside the loop its fields would
  // be re-read after every barrier
  const CoarseLevel L = Ld;
  const int tid = threadIdx.x;
  const int nb = L.nbatch;
  const int steps = sweeps * nb;
  for (int s = 0; s < steps; ++s) {
    const int b = forward ? s % nb : bwd[s % nb];
    const int t = bitem[b] + tid;
    const bool on = t < bitem[b + 1];
    Rec<NS, TS> cur;
    if (on) load_rec<NS, TS>(L, lds, t, cur);
    const int dof = cur.key & REC_DOF_MASK, loc = cur.key >> REC_LOC_SHIFT;
    if (on) {
      double r = g[dof];
#pragma unroll
      for (int q = 0; q < COARSE_NNZ / 2; ++q) {
        const int F = (cur.fac[q / 2] >> (16 * (q % 2))) & 0xffff;
        r -= (double)cur.val[2 * q] * u[2 * F] + (double)cur.val[2 * q + 1] * u[2 * F + 1];
      }
      res[tid] = r;
    }
    __syncthreads();
    if (on) {
      const int base = tid - loc;
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < NS; ++j) d += (double)cur.ai[j] * res[base + j];
      u[dof] += d;
    }
    __syncthreads();
  }
}

// GT: the top level's vectors u, g, r live in memory (column blockIdx.x of
// g_top / u_top / r_top, stride bstride) instead of LDS -- a level too large
// for LDS, used when MG_h on it is tabulated; the lower levels stay in LDS.
template <int NS, typename TS, bool GT>
__global__ void __launch_bounds__(CT) k_coarse_cycle(const CoarseLevel* __restrict__ Lg, int top, int m_top,
                                                     int growth, int q, const TS* __restrict__ inv0, int n0,
                                                     const double* __restrict__ g_top, double* u_top,
                                                     double* r_top, long bstride) {
  extern __shared__ double smem[];
  __shared__ CoarseLevel Ls[COARSE_MAX_LEVELS];
  __shared__ int sbitem[COARSE_MAX_LEVELS][COARSE_MAX_BATCH + 1];
  __shared__ int sbwd[COARSE_MAX_LEVELS][COARSE_MAX_BATCH];
  const int tid = threadIdx.x;
  double* res = smem;  // [CT + NS], the tail stays zero
  for (int i = tid; i < CT + NS; i += CT) res[i] = 0.0;
  if (tid <= top) Ls[tid] = Lg[tid];
  __syncthreads();
  const char* lds = (const char*)smem;
  constexpr int G = Grp<TS>::G;
  for (int l = 1; l <= top; ++l) {
    const CoarseLevel& L = Ls[l];
    if (tid <= L.nbatch) sbitem[l][tid] = gmem(L.bitem)[tid];
    if (tid < L.nbatch) sbwd[l][tid] = gmem(L.bseq_bwd)[tid];
    // record parts resident in LDS for the whole kernel (16-byte words)
    const int nit = L.nitems;
    if (L.lds_meta >= 0) copy_to_lds((char*)smem + L.lds_meta, L.it_meta, nit);
    if (L.lds_val >= 0) copy_to_lds((char*)smem + L.lds_val, L.it_val, (COARSE_NNZ + G - 1) / G * nit);
    if (L.lds_ainv >= 0) copy_to_lds((char*)smem + L.lds_ainv, L.it_ainv, (L.ns_max + G - 1) / G * nit);
  }
  if constexpr (!GT) {
    const CoarseLevel& T = Ls[top];
    double* u = smem + T.off_u;
    double* g = smem + T.off_g;
    // top-level vectors: the level's own, or column blockIdx.x of a batch
    const double* gsrc = g_top ? g_top + blockIdx.x * bstride : T.g_glob;
    const double* usrc = g_top ? u_top + blockIdx.x * bstride : T.u_glob;
    for (int i = tid; i < T.n; i += CT) {
      u[i] = gmem(usrc)[i];
      g[i] = gmem(gsrc)[i];
    }
  }
  __syncthreads();
  int state[COARSE_MAX_LEVELS], cnt[COARSE_MAX_LEVELS], mlev[COARSE_MAX_LEVELS];
  mlev[top] = m_top;
  for (int l = top - 1; l >= 0; --l) mlev[l] = mlev[l + 1] * growth;
  int l = top;
  state[l] = 0;
  while (true) {
    if (l == 0) {
      const CoarseLevel& C = Ls[0];
      double* u0 = smem + C.off_u;
      const double* g0 = smem + C.off_g;
      for (int i = tid; i < n0; i += CT) {
        double s = 0.0;
#pragma unroll 8
        for (int j = 0; j < n0; ++j) s += (double)inv0[(long)j * n0 + i] * g0[j];
        u0[i] = s;
      }
      __syncthreads();
      if (top == 0) break;
      l = 1;
      continue;
    }
    const CoarseLevel& L = Ls[l];
    const CoarseLevel& B = Ls[l - 1];
    double* u = smem + L.off_u;
    double* g = smem + L.off_g;
    double* r = smem + L.off_r;
    if (GT && l == top) {
      u = u_top + blockIdx.x * bstride;
      g = const_cast<double*>(g_top) + blockIdx.x * bstride;
      r = r_top + blockIdx.x * bstride;
    }
    double* ub = smem + B.off_u;
    double* gb = smem + B.off_g;
    if (state[l] == 0) {
      smooth<NS, TS>(L, lds, sbitem[l], sbwd[l], mlev[l], true, res, u, g);
      const auto rwv = gmem((const TS*)L.rw_val);
      const auto rwc = gmem(L.rw_col);
      const auto Rv = gmem((const TS*)L.R_v);
      const auto Rci = gmem(L.R_ci);
      for (int i = tid; i < L.n; i += CT) {
        double s = g[i];
#pragma unroll
        for (int k = 0; k < COARSE_NNZ; ++k) s -= (double)rwv[k * L.n + i] * u[rwc[k * L.n + i]];
        r[i] = s;
      }
      __syncthreads();
      for (int i = tid; i < B.n; i += CT) {
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < L.R_w; ++k) s += (double)Rv[k * B.n + i] * r[Rci[k * B.n + i]];
        gb[i] = s;
        ub[i] = 0.0;
      }
      __syncthreads();
      state[l] = 1;
      cnt[l] = 0;
      state[l - 1] = 0;
      --l;
      continue;
    }
    if (++cnt[l] < q) {
      state[l - 1] = 0;
      --l;
      continue;
    }
    const auto Pv = gmem((const TS*)L.P_v);
    const auto Pci = gmem(L.P_ci);
    for (int i = tid; i < L.n; i += CT) {
      double s = 0.0;
#pragma unroll 8
      for (int k = 0; k < L.P_w; ++k) s += (double)Pv[k * L.n + i] * ub[Pci[k * L.n + i]];
      u[i] += s;
    }
    __syncthreads();
    smooth<NS, TS>(L, lds, sbitem[l], sbwd[l], mlev[l], false, res, u, g);
    if (l == top) break;
    ++l;
  }
  if constexpr (!GT) {
    const CoarseLevel& T = Ls[top];
    const double* u = smem + T.off_u;
    double* udst = g_top ? u_top + blockIdx.x * bstride : T.u_glob;
    for (int i = tid; i < T.n; i += CT) udst[i] = u[i];
  }
}

// One colour phase of record-based block Gauss-Seidel: a workgroup per
// patch-aligned batch of exactly GS_REC_THREADS item slots (batches padded
// with items whose row marker is REC_PAD), a thread per patch row, so that a
// thread's item index needs no lookup.  Patches of one colour share no cell,
// so the rows a batch reads are never written by another batch of the same
// launch.  W (wide records, levels beyond 16-bit facet indices): two meta
// words per item, (unknown, row in patch, F0, F1) and (F2, F3, F4, 0).
template <int NS, typename TS, bool W>
__global__ void __launch_bounds__(GS_REC_THREADS)
    k_gs_records(const uint4* __restrict__ meta, const TS* __restrict__ val, const TS* __restrict__ ainv, int nit,
                 int nsm, int b0, double* __restrict__ u, const double* __restrict__ g) {
  __shared__ double res[GS_REC_THREADS + NS];
  const int tid = threadIdx.x;
  const int t = (b0 + blockIdx.x) * GS_REC_THREADS + tid;
  if (tid < NS) res[GS_REC_THREADS + tid] = 0.0;
  using GT = Grp<TS>;
  using V = typename GT::T;
  constexpr int G = GT::G;
  // every load of the item is independent of the others: issue them
  // together, the meta word first (the gathers wait only for it).  The two
  // orders below are the faster schedules measured for each precision.
  const uint4 m0 = meta[W ? 2 * (long)t : t];
  const uint4 m1 = W ? meta[2 * (long)t + 1] : m0;
  V vv[(COARSE_NNZ + G - 1) / G];
  V av[NS / G];
  if constexpr (G == 4) {
#pragma unroll
    for (int e = 0; e < (COARSE_NNZ + G - 1) / G; ++e) vv[e] = ((const V*)val)[e * nit + t];
#pragma unroll
    for (int j = 0; j < NS / G; ++j) av[j] = ((const V*)ainv)[min(j, (nsm + G - 1) / G - 1) * nit + t];
  } else {
#pragma unroll
    for (int j = 0; j < NS / G; ++j) av[j] = j * G < nsm ? ((const V*)ainv)[j * nit + t] : (V)(TS)0;
#pragma unroll
    for (int e = 0; e < (COARSE_NNZ + G - 1) / G; ++e) vv[e] = ((const V*)val)[e * nit + t];
  }
  TS vals[((COARSE_NNZ + G - 1) / G) * G];
#pragma unroll
  for (int e = 0; e < (COARSE_NNZ + G - 1) / G; ++e)
#pragma unroll
    for (int i = 0; i < G; ++i) vals[e * G + i] = GT::get(vv[e], i);
  const unsigned dof = W ? m0.x : (m0.x & REC_DOF_MASK);
  const unsigned loc = W ? m0.y : (m0.x >> REC_LOC_SHIFT);
  const bool on = loc != REC_PAD;
  const unsigned fw[3] = {m0.y, m0.z, m0.w};
  const unsigned fwide[5] = {m0.z, m0.w, m1.x, m1.y, m1.z};
  double r = g[dof];
#pragma unroll
  for (int q = 0; q < COARSE_NNZ / 2; ++q) {
    const unsigned F = W ? fwide[q] : (fw[q / 2] >> (16 * (q % 2))) & 0xffff;
    const double2 uf = *(const double2*)(u + 2 * (long)F);
    r -= (double)vals[2 * q] * uf.x + (double)vals[2 * q + 1] * uf.y;
  }
  res[tid] = on ? r : 0.0;
  // the inverse rows are needed only after the barrier, but their loads
  // must not move past it (one more memory round trip): mark them used here
  // (FP32 records; the FP64 schedule is faster without it)
  if constexpr (G == 4)
#pragma unroll
    for (int j = 0; j < NS / G; ++j) asm volatile("" ::"v"(av[j]));
  __syncthreads();
  if (on) {
    const int base = tid - (int)loc;
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < NS / G; ++j)
      if (G == 2 || j * G < nsm)  // FP64 rows past nsm are zero; FP32 ones are not loaded
#pragma unroll
        for (int i = 0; i < G; ++i) d += (double)GT::get(av[j], i) * res[base + j * G + i];
    u[dof] += d;
  }
}

template <typename TS, bool W>
void gs_records_tw(hipStream_t st, const uint4* meta, const TS* val, const TS* ainv, int nit, int nsm, int b0,
                   int nb, double* u, const double* g) {
  if (nsm <= 12)
    hipLaunchKernelGGL((k_gs_records<12, TS, W>), dim3(nb), dim3(GS_REC_THREADS), 0, st, meta, val, ainv, nit, nsm,
                       b0, u, g);
  else if (nsm <= 16)
    hipLaunchKernelGGL((k_gs_records<16, TS, W>), dim3(nb), dim3(GS_REC_THREADS), 0, st, meta, val, ainv, nit, nsm,
                       b0, u, g);
  else
    hipLaunchKernelGGL((k_gs_records<32, TS, W>), dim3(nb), dim3(GS_REC_THREADS), 0, st, meta, val, ainv, nit, nsm,
                       b0, u, g);
}
template <typename TS>
void gs_records_t(hipStream_t st, const uint4* meta, const TS* val, const TS* ainv, int nit, int nsm, int b0,
                  int nb, double* u, const double* g, bool wide) {
  if (wide)
    gs_records_tw<TS, true>(st, meta, val, ainv, nit, nsm, b0, nb, u, g);
  else
    gs_records_tw<TS, false>(st, meta, val, ainv, nit, nsm, b0, nb, u, g);
}

}  // namespace

void launch_gs_records(hipStream_t st, const unsigned* meta, const void* val, const void* ainv, int nit, int nsm,
                       int b0, int nb, double* u, const double* g, int f32, int wide) {
  if (nb <= 0) return;
  const uint4* m = (const uint4*)meta;
  if (f32)
    gs_records_t<float>(st, m, (const float*)val, (const float*)ainv, nit, nsm, b0, nb, u, g, wide != 0);
  else
    gs_records_t<double>(st, m, (const double*)val, (const double*)ainv, nit, nsm, b0, nb, u, g, wide != 0);
}

template <typename TS, bool GT>
void coarse_t(hipStream_t st, const CoarseLevel* Ls, int top, int m_top, int growth, int q, const TS* inv0,
              int n0, int ns_max, size_t shm, int nb, const double* g_top, double* u_top, double* r_top,
              long bstride) {
  if (ns_max <= 12)
    hipLaunchKernelGGL((k_coarse_cycle<12, TS, GT>), dim3(nb), dim3(CT), shm, st, Ls, top, m_top, growth, q, inv0,
                       n0, g_top, u_top, r_top, bstride);
  else if (ns_max <= 16)
    hipLaunchKernelGGL((k_coarse_cycle<16, TS, GT>), dim3(nb), dim3(CT), shm, st, Ls, top, m_top, growth, q, inv0,
                       n0, g_top, u_top, r_top, bstride);
  else
    hipLaunchKernelGGL((k_coarse_cycle<32, TS, GT>), dim3(nb), dim3(CT), shm, st, Ls, top, m_top, growth, q, inv0,
                       n0, g_top, u_top, r_top, bstride);
}

template <typename TS, bool GT>
hipError_t prepare_tg(int ns_max, int v) {
  if (ns_max <= 12)
    return hipFuncSetAttribute((const void*)k_coarse_cycle<12, TS, GT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               v);
  if (ns_max <= 16)
    return hipFuncSetAttribute((const void*)k_coarse_cycle<16, TS, GT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               v);
  return hipFuncSetAttribute((const void*)k_coarse_cycle<32, TS, GT>, hipFuncAttributeMaxDynamicSharedMemorySize, v);
}
template <typename TS>
hipError_t prepare_t(int ns_max, size_t lds_bytes) {
  const int v = (int)lds_bytes;
  hipError_t e = prepare_tg<TS, false>(ns_max, v);
  return e != hipSuccess ? e : prepare_tg<TS, true>(ns_max, v);
}

hipError_t prepare_coarse_cycle(int ns_max, size_t lds_bytes, int f32) {
  return f32 ? prepare_t<float>(ns_max, lds_bytes) : prepare_t<double>(ns_max, lds_bytes);
}

size_t coarse_cycle_static_lds() {
  return sizeof(CoarseLevel) * COARSE_MAX_LEVELS + sizeof(int) * COARSE_MAX_LEVELS * (2 * COARSE_MAX_BATCH + 1);
}

void launch_coarse_cycle(hipStream_t st, const CoarseLevel* Ls, int top, int m_top, int growth, int q,
                         const void* inv0, int n0, int ns_max, int lds_doubles, int f32) {
  launch_coarse_cycle_batch(st, Ls, top, m_top, growth, q, inv0, n0, ns_max, lds_doubles, f32, 1, nullptr,
                            nullptr, nullptr, 0);
}

void launch_coarse_cycle_batch(hipStream_t st, const CoarseLevel* Ls, int top, int m_top, int growth, int q,
                               const void* inv0, int n0, int ns_max, int lds_doubles, int f32, int nb,
                               const double* g_top, double* u_top, double* r_top, long bstride) {
  if (nb <= 0) return;
  size_t shm = sizeof(double) * (size_t)lds_doubles;
  if (r_top) {
    if (f32)
      coarse_t<float, true>(st, Ls, top, m_top, growth, q, (const float*)inv0, n0, ns_max, shm, nb, g_top, u_top,
                            r_top, bstride);
    else
      coarse_t<double, true>(st, Ls, top, m_top, growth, q, (const double*)inv0, n0, ns_max, shm, nb, g_top, u_top,
                             r_top, bstride);
  } else {
    if (f32)
      coarse_t<float, false>(st, Ls, top, m_top, growth, q, (const float*)inv0, n0, ns_max, shm, nb, g_top, u_top,
                             nullptr, bstride);
    else
      coarse_t<double, false>(st, Ls, top, m_top, growth, q, (const double*)inv0, n0, ns_max, shm, nb, g_top,
                              u_top, nullptr, bstride);
  }
}

}  // namespace hdgmg
