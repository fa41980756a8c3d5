// Host orchestration of the skeleton solve and the C ABI (include/hdgmg.h).
//
//   setup     mesh hierarchy, skeleton topology, patches, colouring,
//             averaging weights (host); device buffers
//   assemble  order-k condensation and lowest-order cell blocks (device),
//             patch inverses (device), harmonic-extension transfers and the
//             coarsest inverse (host, FP64), uploads
//   solve     condensed load -> AL-Uzawa { flexible CG + MG_hp } -> recovery,
//             every vector operation on the device
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hdgmg.h"
#include "coarse.hpp"
#include "fast.hpp"
#include "kernels.hpp"
#include "host_setup.hpp"
#include "topology.hpp"
#include "solve3d.hpp"

using namespace hdgmg;

// See g_scratch_dev: the no-allocation inner solve's Krylov scratch.
static __device__ __align__(256) double scratch[36000];


namespace {

std::string g_setup_error;

// Fixed device scratch of hdgmg_inner_solve_noalloc: the Krylov solvers'
// scalars and reduction partials (KrylovScratch below) in one file-scope
// array, so that the call needs no allocation.  Each GPU holds its own copy
// until the process ends; its address on a device is looked up once, with
// that device current (hipGetSymbolAddress), and only that address is used
// from host code.  Layout in words: sc [0, 32), part [32, 32 + 4 RED_BLOCKS),
// gm_part (65 RED_BLOCKS: restart <= 64), gm_h (512), gm_y (128).
constexpr long NA_SC = 0, NA_PART = 32, NA_GMPART = NA_PART + 4 * RED_BLOCKS,
               NA_GMH = NA_GMPART + 65 * RED_BLOCKS, NA_GMY = NA_GMH + 512, NA_WORDS = NA_GMY + 128;
constexpr int NA_MAX_DEVICES = 64;
static_assert(NA_WORDS == 36000, "scratch layout must fill the array");
double* g_scratch_dev[NA_MAX_DEVICES] = {};
std::mutex g_scratch_mu;

struct DevLevel {
  int nc = 0, nint = 0, m = 1, nK = 6;
  long ndof = 0;
  int* cells = nullptr;
  int* cell_dofs = nullptr;
  int* fcell = nullptr;
  int* floc = nullptr;
  double* X = nullptr;
  double* S = nullptr;
  int* pf_ptr = nullptr;
  int* pf = nullptr;
  int* pc_ptr = nullptr;
  int* pc = nullptr;
  long* pinv_off = nullptr;
  double* pinv = nullptr;
  int npatch = 0, max_ns = 0;
  long pinv_len = 0;
  std::vector<int> colour_ptr;
  double* nu = nullptr;  // per cell
  int* oflag = nullptr;  // [nc] bit i: local facet i is a do-nothing facet (null without any)
  double *u = nullptr, *g = nullptr, *r = nullptr;  // multigrid vectors
  // record-based Gauss-Seidel (launched lowest-order levels): patch-row
  // records in the V-cycle's storage, batches per colour
  bool rec = false, rwide = false;  // rwide: 32-bit record fields (8 meta words per item)
  unsigned* rk = nullptr;  // [nit][4] meta words ([nit][8] when rwide)
  const void *rv = nullptr, *ra = nullptr;
  std::vector<int> rcb;
  int rnit = 0, rnsm = 0;
  std::vector<double> rec_bytes;
  // lowest-order wind (Oseen): facet fluxes and RT0 coefficients per cell
  double* flux = nullptr;   // [nint]
  double* wcoef = nullptr;  // [nc][3]
  // streaming layout (fast.hip), used when every patch has <= FAST_NF facets
  bool fast = false;
  bool full = false;      // cell blocks stored in full (nonsymmetric operators)
  long sp_words = 0;      // words per cell of the streaming cell blocks
  double* Sp = nullptr;   // packed SoA cell blocks
  int* cdof = nullptr;    // [3][nc] 2*facet+side or -1
  // order-k level: the six mode-0 rows of every cell block ([nK][6][nc], in
  // the V-cycle's storage) and their products, for the residual that MG_hp
  // restricts to the lowest-order space
  double* S0 = nullptr;
  float* S0_32 = nullptr;
  double* y0K = nullptr;
  double* yF = nullptr;   // [nint][2][2m] per-side facet rows
  std::vector<int> npc;   // patches per colour
  std::vector<int*> pfc;  // per colour [FAST_NF][npc] facets
  std::vector<double*> Ppc;  // per colour packed SoA patch inverses
  // fused colour phase (order-k level, symmetric packed blocks)
  bool fused = false;
  int fused_ncp = 0;             // cell slots per patch (6 or 7)
  std::vector<int*> fmeta;       // per colour [3 ncp + FAST_NF][npc]
  std::vector<int*> fcode;       // per colour [npc][ncp] cell * 4 + far facet, or -1
  std::vector<double*> Scc;      // per colour patch-ordered cell slots, FP64
  std::vector<float*> Scc32;     // ... or FP32 (the V-cycle's storage)
  std::vector<double> bytes_fused_vc;
  bool pfull = true;         // patch inverses stored in full (else upper triangles)
  double bytes_cell = 0.0, bytes_sum = 0.0;
  std::vector<double> bytes_relax;
  // storage the preconditioner reads: FP64 arrays above, or FP32 copies
  bool f32 = false;
  float *S32 = nullptr, *pinv32 = nullptr, *Sp32 = nullptr;
  std::vector<float*> Pp32;
  // FP16 copies of the streaming operators of the order-k level
  // (vcycle_precision 2), each block divided by its largest magnitude
  bool f16 = false;
  _Float16* Sp16 = nullptr;
  float4* al16 = nullptr;
  std::vector<_Float16*> Pp16;
  std::vector<float*> psc16;
  double bytes_cell_vc = 0.0;
  std::vector<double> bytes_relax_vc;
  template <typename TS>
  LevelViewT<TS> view_t() const {
    LevelViewT<TS> v;
    v.nc = nc;
    v.nint = nint;
    v.m = m;
    v.nK = nK;
    v.cell_dofs = cell_dofs;
    v.fcell = fcell;
    v.floc = floc;
    v.S = (const TS*)(f32 ? (const void*)S32 : (const void*)S);
    v.pf_ptr = pf_ptr;
    v.pf = pf;
    v.pinv_off = pinv_off;
    v.pinv = (const TS*)(f32 ? (const void*)pinv32 : (const void*)pinv);
    return v;
  }
  LevelView view() const {
    LevelView v;
    v.nc = nc;
    v.nint = nint;
    v.m = m;
    v.nK = nK;
    v.cell_dofs = cell_dofs;
    v.fcell = fcell;
    v.floc = floc;
    v.S = S;
    v.pf_ptr = pf_ptr;
    v.pf = pf;
    v.pinv_off = pinv_off;
    v.pinv = pinv;
    return v;
  }
};

// Prolongation and restriction of a level in ELL form (column-major, zero
// padded); nnz: stored entries of the larger of the two.
struct DevTransfer {
  int nfine = 0, ncoarse = 0;
  long nnz = 0;
  int Pw = 0, Rw = 0;
  int *Pe_ci = nullptr, *Re_ci = nullptr;
  double *Pe_v = nullptr, *Re_v = nullptr;
  float *Pe_v32 = nullptr, *Re_v32 = nullptr;
  // the same in sliced ELL form for the launched product (L lanes per row,
  // slices of 64 / L rows each padded to its own width; L = 0: not built)
  int PL = 0, RL = 0;
  long *Ps_off = nullptr, *Rs_off = nullptr;
  int *Ps_w = nullptr, *Rs_w = nullptr, *Ps_ci = nullptr, *Rs_ci = nullptr;
  double *Ps_v = nullptr, *Rs_v = nullptr;
  float *Ps_v32 = nullptr, *Rs_v32 = nullptr;
};

// CSR -> ELL (column-major, zero padding).
void to_ell(const CSR& A, int& w, std::vector<int>& ci, std::vector<double>& v) {
  w = 0;
  for (int r = 0; r < A.n; ++r) w = std::max(w, A.rp[r + 1] - A.rp[r]);
  ci.assign((size_t)w * A.n, 0);
  v.assign((size_t)w * A.n, 0.0);
  for (int r = 0; r < A.n; ++r)
    for (int k = A.rp[r]; k < A.rp[r + 1]; ++k) {
      ci[(size_t)(k - A.rp[r]) * A.n + r] = A.ci[k];
      v[(size_t)(k - A.rp[r]) * A.n + r] = A.v[k];
    }
}

// CSR -> sliced ELL with L lanes per row: slices of H = 64 / L rows, slice
// s padded to its widest row, entry (slot k, row s H + rr) at
// off[s] + k H + rr (padding: column 0, value 0).
void to_sell(const CSR& A, int L, std::vector<long>& off, std::vector<int>& sw, std::vector<int>& ci,
             std::vector<double>& v) {
  const int H = 64 / L, ns = (A.n + H - 1) / H;
  off.assign(ns + 1, 0);
  sw.assign(std::max(ns, 1), 0);
  for (int sl = 0; sl < ns; ++sl) {
    int w = 0;
    for (int r = sl * H; r < std::min(A.n, (sl + 1) * H); ++r) w = std::max(w, A.rp[r + 1] - A.rp[r]);
    sw[sl] = w;
    off[sl + 1] = off[sl] + (long)w * H;
  }
  ci.assign(std::max<long>(off[ns], 1), 0);
  v.assign(std::max<long>(off[ns], 1), 0.0);
  for (int r = 0; r < A.n; ++r) {
    const int sl = r / H, rr = r - sl * H;
    for (int k = A.rp[r]; k < A.rp[r + 1]; ++k) {
      ci[off[sl] + (long)(k - A.rp[r]) * H + rr] = A.ci[k];
      v[off[sl] + (long)(k - A.rp[r]) * H + rr] = A.v[k];
    }
  }
}

}  // namespace

struct hdgmg_ctx {
  std::string err;
  hipStream_t st = nullptr;
  hipStream_t own = nullptr;  // created when the caller passes no stream
  // MG_hp replayed as a HIP graph for fixed (r, z) pointers
  hipGraphExec_t vc_exec = nullptr;
  const double* vc_r = nullptr;
  double* vc_z = nullptr;
  bool use_graph = true;
  int k = 0, J = 0;
  double beta = 0, gamma = 0;
  std::vector<double> nu_fine;
  hdgmg_opts opts;
  std::vector<Level> lv;
  std::vector<Averaging> avg;
  QuadTables Q;
  QuadTables Q0;              // data rule of the lowest-order levels
  ConvTables* CTk = nullptr;  // device convection rules of order k and 0
  ConvTables* CT0 = nullptr;
  bool has_wind = false;
  double* wcoef = nullptr;    // [n_cells][na] wind coefficients (order-k level)
  double* fac = nullptr;      // kept local factors of the order-k cells (loads, recovery)
  // lowest-order cell blocks of every level on the host (transfers, coarse levels)
  std::vector<std::vector<double>> hostB;
  // tangential Dirichlet data on the finest boundary facets
  std::vector<int> bfacets;   // boundary facets in facet order
  int* cbf = nullptr;         // [n_cells][3] boundary facet number or -1
  double* bdl = nullptr;      // [n_cells][3][2][k+1] local boundary values (normal, tangential)
  double* btan = nullptr;     // [n_boundary_facets][2] tangents t_F (first use of constant data)
  double* bvals = nullptr;    // [n_boundary_facets][k+1] coefficients built from constant data
  // Alg. 3 (hdgmg_picard_newton): previous velocity and state
  double* a3_u = nullptr;
  double* a3_state = nullptr;
  double* a3_f = nullptr;     // pseudo-time load f + dt_inv u_{n-1}
  bool has_bd = false;
  bool has_outflow = false;   // do-nothing facets: launch-per-colour kernels on every level
  double* bdiv = nullptr;     // [n_cells][3] sigma |F| on Dirichlet boundary facets, else 0
  double* cflux = nullptr;    // [n_cells] flux of the prescribed normal boundary values
  bool has_flux = false;
  // FGMRES basis: V [(restart+1)][N_skel], Z [restart][N_skel], scalars
  double *gm_V = nullptr, *gm_Z = nullptr, *gm_h = nullptr, *gm_y = nullptr, *gm_part = nullptr;
  // allocations of one hdgmg_assemble (released by the next one)
  std::vector<std::pair<void*, size_t>> asm_allocs;
  bool in_assemble = false;
  DevLevel K;
  std::vector<DevLevel> cr;
  std::vector<DevTransfer> tr;
  double* coarse_inv = nullptr;
  float* coarse_inv32 = nullptr;
  // the coarsest inverse row by row (rows padded to ld0 words) for the
  // wavefront-per-row GEMV, in the V-cycle's storage precision
  double* coarse_rows = nullptr;
  float* coarse_rows32 = nullptr;
  int ld0 = 0;
  int n0 = 0;
  // Krylov / Uzawa vectors
  double *x = nullptr, *r = nullptr, *r_old = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double *b = nullptr, *gvec = nullptr, *lam = nullptr, *p0 = nullptr;
  double *sc = nullptr, *part = nullptr;
  int dev = 0;  // device current at hdgmg_setup (the stream's device)
  Ctx3* d3 = nullptr;  // tetrahedral meshes: the three-dimensional context
  double *fdiv = nullptr, *cdiv = nullptr, *area = nullptr;
  double* gK = nullptr;
  double* statebuf = nullptr;  // [N_skel + n_cells] for hdgmg_solve without state
  // MG_h on the coarse kernel's top level tabulated as a dense row-major
  // matrix (storage of the V-cycle precision), applied by one GEMV when the
  // cycle enters that level from zero with dense_m sweeps
  bool dense_on = false;
  void* dense_M = nullptr;
  int dense_n = 0, dense_ld = 0, dense_m = 0, dense_level = -1;
  // level Lc + 1 described to the coarse kernel with its vectors in memory,
  // only for the tabulation (-1: none)
  int Lt = -1;
  // Newton linearisation: the previous state's skeleton vector and the
  // per-cell Newton loads (allocated at the first hdgmg_set_newton)
  bool has_newton = false;
  double* nw_lam = nullptr;
  double* nw_load = nullptr;
  // adjoint solve buffers (allocated at the first hdgmg_solve_adjoint)
  double* adj_f = nullptr;      // [n_cells][n_q][2] adjoint source values
  double* adj_p = nullptr;      // [n_cells][n_q] adjoint pressure
  double* adj_state = nullptr;  // [N_skel + n_cells]
  double* adj_gnu = nullptr;    // [n_cells] this context's share of a batch's dJ/dnu
  double* ws = nullptr;
  size_t ws_bytes = 0;
  int* status = nullptr;
  bool assembled = false;
  size_t bytes = 0;
  std::vector<void*> allocs;
  // caller's device allocator (null: hipMalloc / hipFree)
  hdgmg_alloc_fn alloc_fn = nullptr;
  hdgmg_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  // live kernel timers (hdgmg_kernel_timer)
  struct KTimer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    double bytes = 0.0;
  } timers[5];
  // single-workgroup coarse MG_h: levels 0..Lc (Lc < 0: disabled)
  int Lc = -1;
  CoarseLevel* coarse_desc = nullptr;
  int coarse_lds = 0, coarse_ns = 0;
  // algorithmic bytes of one Gauss-Seidel colour phase, per level / colour
  std::vector<double> relax_bytes;                // order-k level
  std::vector<std::vector<double>> smooth_bytes;  // lowest-order levels
  double apply_bytes = 0.0, vcycle_bytes = 0.0;
  // the V-cycle's compulsory bytes: every stored operator read once per use
  // in packed symmetric form (cell blocks n(n+1)/2 words, patch inverses
  // n_s(n_s+1)/2), in its storage precision, plus the vectors
  double vcycle_compulsory = 0.0;
};

// The preconditioner reads FP32 (vcycle_precision 1) or FP32 with FP16
// order-k blocks (2) copies of its operators.
inline bool vc_f32(const hdgmg_ctx* ctx) { return ctx->opts.vcycle_precision >= 1; }

namespace {

#define HIPC(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr; \
      return HDGMG_EHIP;                                                             \
    }                                                                                \
  } while (0)

// Device memory through the caller's allocator when one was given at setup
// (e.g. PyTorch's caching allocator), else hipMalloc / hipFree.
// Largest level (unknowns) whose MG_h is tabulated as a dense matrix.
constexpr int DENSE_MAX_N = 8192;
// Launched lowest-order levels with at most this many interior facets smooth
// with the patch-row record kernel (beyond 65535: the 32-bit record form).
constexpr int REC_MAX_FACETS = 1 << 22;

void* dmalloc(hdgmg_ctx* ctx, size_t bytes) {
  if (ctx->alloc_fn) return ctx->alloc_fn(bytes, ctx->alloc_ctx);
  void* v = nullptr;
  return hipMalloc(&v, bytes) == hipSuccess ? v : nullptr;
}
void dfree(hdgmg_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->free_fn)
    ctx->free_fn(p, ctx->alloc_ctx);
  else
    (void)hipFree(p);
}

template <class T>
hdgmg_status dalloc(hdgmg_ctx* ctx, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return HDGMG_OK;
  void* v = dmalloc(ctx, n * sizeof(T));
  if (!v) {
    ctx->err = "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed";
    return HDGMG_ENOMEM;
  }
  if (ctx->in_assemble)
    ctx->asm_allocs.push_back({v, n * sizeof(T)});
  else
    ctx->allocs.push_back(v);
  ctx->bytes += n * sizeof(T);
  *p = (T*)v;
  return HDGMG_OK;
}

template <class T>
hdgmg_status upload(hdgmg_ctx* ctx, T** p, const std::vector<T>& h) {
  hdgmg_status s = dalloc(ctx, p, h.size());
  if (s) return s;
  if (!h.empty()) {
    HIPC(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, ctx->st));
    HIPC(hipStreamSynchronize(ctx->st));  // h may be a temporary
  }
  return HDGMG_OK;
}

#define TRY(expr)                 \
  do {                            \
    hdgmg_status s_ = (expr);     \
    if (s_ != HDGMG_OK) return s_; \
  } while (0)

// ------------------------------------------------------------- kernel timers
int kt_begin(hdgmg_ctx* ctx, int cls) {
  auto& T = ctx->timers[cls];
  if (!T.on) return -1;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1;
  }
  (void)hipEventRecord(a, ctx->st);
  T.ev.push_back({a, b});
  return (int)T.ev.size() - 1;
}

void kt_end(hdgmg_ctx* ctx, int cls, int idx, double bytes) {
  if (idx < 0) return;
  auto& T = ctx->timers[cls];
  (void)hipEventRecord(T.ev[idx].second, ctx->st);
  T.bytes += bytes;
}

// A timed launch whose events the dispatch itself records (launchers taking
// a KernelEvents*): the interval excludes the event packets that kt_begin /
// kt_end put around a launch.  Returns the events to pass, or null when the
// class is not timed; kd_end adds the launch's bytes.
struct KtDispatch {
  int idx = -1;
  KernelEvents ev{};
  const KernelEvents* ptr() const { return idx < 0 ? nullptr : &ev; }
};
KtDispatch kd_begin(hdgmg_ctx* ctx, int cls) {
  KtDispatch d;
  auto& T = ctx->timers[cls];
  if (!T.on) return d;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return d;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return d;
  }
  T.ev.push_back({a, b});
  d.idx = (int)T.ev.size() - 1;
  d.ev = {a, b};
  return d;
}
void kd_end(hdgmg_ctx* ctx, int cls, const KtDispatch& d, double bytes) {
  if (d.idx >= 0) ctx->timers[cls].bytes += bytes;
}

void kt_clear(hdgmg_ctx::KTimer& T) {
  for (auto& e : T.ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  T.ev.clear();
  T.bytes = 0.0;
}

// Algorithmic bytes of one Gauss-Seidel colour phase of the current kernel:
// per patch its inverse (ns^2 words), for every patch facet the rows of both
// cells (2m x nK words each), the cell vectors it gathers, b_s and x_s.
double gs_phase_bytes(const Level& L, int m, int c) {
  const int m2 = 2 * m, nK = 6 * m;
  double w = 0.0;
  for (int p = L.colour_ptr[c]; p < L.colour_ptr[c + 1]; ++p) {
    int nfp = L.patch_facet_ptr[p + 1] - L.patch_facet_ptr[p];
    double ns = nfp * m2;
    int ncell = L.patch_cell_ptr[p + 1] - L.patch_cell_ptr[p];
    w += ns * ns + nfp * 2.0 * m2 * nK + ncell * (double)nK + 2.0 * ns;
  }
  return w * 8.0;
}

// ------------------------------------------------------------- device level
// Damped Jacobi, do-nothing facets and edge patches run the
// launch-per-colour kernels on every level (the streaming, record and
// single-workgroup forms assume Gauss-Seidel on vertex patches of interior
// facets).
bool generic_only(const hdgmg_ctx* ctx) {
  return ctx->opts.smoother != 0 || ctx->has_outflow || ctx->opts.patch_relax == 2 || ctx->opts.patch_smooth == 2;
}

hdgmg_status upload_level(hdgmg_ctx* ctx, const Level& L, int m, DevLevel& D) {
  D.nc = L.nc;
  D.nint = L.nint;
  D.m = m;
  D.nK = 6 * m;
  D.ndof = (long)L.nint * 2 * m;
  TRY(upload(ctx, &D.cells, L.cells));
  TRY(upload(ctx, &D.cell_dofs, L.cell_dofs));
  TRY(upload(ctx, &D.X, L.X));
  std::vector<int> fc(2 * (size_t)L.nint), fl(2 * (size_t)L.nint);
  for (int i = 0; i < L.nint; ++i) {
    int f = L.int_facet[i];
    for (int s = 0; s < 2; ++s) {
      fc[2 * i + s] = L.facet_cells[2 * f + s];
      fl[2 * i + s] = L.facet_loc[2 * f + s];
    }
  }
  TRY(upload(ctx, &D.fcell, fc));
  TRY(upload(ctx, &D.floc, fl));
  if (ctx->has_outflow) {
    std::vector<int> of(L.nc, 0);
    for (int c = 0; c < L.nc; ++c)
      for (int i = 0; i < 3; ++i) {
        const int f = L.cell_facets[3 * c + i];
        if (L.int_id[f] >= 0 && L.facet_cells[2 * f + 1] < 0) of[c] |= 1 << i;
      }
    TRY(upload(ctx, &D.oflag, of));
  }
  TRY(upload(ctx, &D.pf_ptr, L.patch_facet_ptr));
  TRY(upload(ctx, &D.pf, L.patch_facets));
  TRY(upload(ctx, &D.pc_ptr, L.patch_cell_ptr));
  TRY(upload(ctx, &D.pc, L.patch_cells));
  D.npatch = (int)L.patch_vertex.size();
  std::vector<long> off(D.npatch);
  long tot = 0;
  D.max_ns = 0;
  for (int p = 0; p < D.npatch; ++p) {
    int ns = (L.patch_facet_ptr[p + 1] - L.patch_facet_ptr[p]) * 2 * m;
    off[p] = tot;
    tot += (long)ns * ns;
    D.max_ns = std::max(D.max_ns, ns);
  }
  D.pinv_len = tot;
  TRY(upload(ctx, &D.pinv_off, off));
  TRY(dalloc(ctx, &D.pinv, (size_t)tot));
  TRY(dalloc(ctx, &D.S, (size_t)L.nc * D.nK * D.nK));
  D.colour_ptr = L.colour_ptr;
  // streaming kernels pay off on large levels; small ones keep the one-launch
  // Gauss-Seidel phase
  D.fast = L.max_patch_facets <= FAST_NF && (long)L.nint * 2 * m >= ctx->opts.stream_dofs && !generic_only(ctx);
  D.full = ctx->opts.oseen != 0;
  D.sp_words = fast_cell_words(D.nK, D.full);
  if (D.fast) {
    const int m2 = 2 * m;
    std::vector<int> cd(3 * (size_t)L.nc, -1);
    double ncd = 0;
    for (int c = 0; c < L.nc; ++c)
      for (int i = 0; i < 3; ++i) {
        int f = L.cell_facets[3 * c + i];
        int fi = L.int_id[f];
        if (fi < 0) continue;
        int side = L.facet_cells[2 * f] == c ? 0 : 1;
        cd[(size_t)i * L.nc + c] = 2 * fi + side;
        ncd += 1;
      }
    TRY(upload(ctx, &D.cdof, cd));
    TRY(dalloc(ctx, &D.Sp, (size_t)L.nc * D.sp_words));
    TRY(dalloc(ctx, &D.yF, (size_t)L.nint * 2 * m2));
    // compulsory bytes of one cell apply: the blocks, the facet map, x once
    // per interior facet, y_F once per (cell, interior facet)
    const double vec = ((double)L.nint + ncd) * m2 * 8.0 + L.nc * 12.0;
    D.bytes_cell = (double)L.nc * D.sp_words * 8.0 + vec;
    const double ws = vc_f32(ctx) ? 4.0 : 8.0;
    D.bytes_cell_vc = (double)L.nc * D.sp_words * ws + vec;
    D.bytes_sum = 3.0 * L.nint * m2 * 8.0;
    // symmetric patch inverses are stored as upper triangles
    D.pfull = D.full;
    const long pw = fast_patch_words(m2, D.pfull);
    for (int cc = 0; cc < L.ncol; ++cc) {
      int p0 = L.colour_ptr[cc], np = L.colour_ptr[cc + 1] - p0;
      std::vector<int> pf((size_t)FAST_NF * std::max(np, 1), -1);
      double nfac = 0;
      for (int p = 0; p < np; ++p) {
        int a0 = L.patch_facet_ptr[p0 + p], na = L.patch_facet_ptr[p0 + p + 1] - a0;
        for (int a = 0; a < na; ++a) pf[(size_t)a * np + p] = L.patch_facets[a0 + a];
        nfac += na;
      }
      int* dpf;
      double* dPp;
      TRY(upload(ctx, &dpf, pf));
      TRY(dalloc(ctx, &dPp, (size_t)std::max(np, 1) * pw));
      D.npc.push_back(np);
      D.pfc.push_back(dpf);
      D.Ppc.push_back(dPp);
      D.bytes_relax.push_back((double)np * pw * 8.0 + np * FAST_NF * 4.0 + 5.0 * nfac * m2 * 8.0);
      D.bytes_relax_vc.push_back((double)np * pw * ws + np * FAST_NF * 4.0 + 5.0 * nfac * m2 * 8.0);
    }
  }
  TRY(dalloc(ctx, &D.u, (size_t)D.ndof));
  TRY(dalloc(ctx, &D.g, (size_t)D.ndof));
  TRY(dalloc(ctx, &D.r, (size_t)D.ndof));
  return HDGMG_OK;
}

// Metadata, byte model and patch-ordered cell storage of the fused colour
// phase on a streamed level, when its streaming layout is symmetric and
// packed, the level is stored FP64 or FP32 (with vcycle_precision 2 the
// order-k level keeps FP16 blocks and the pair; the lowest-order levels are
// FP32), and every patch has at most 7 cells (else the level keeps the
// cell-apply / patch-relaxation pair).
hdgmg_status setup_fused(hdgmg_ctx* ctx, const Level& L, DevLevel& D) {
  if (!D.fast || D.full || D.pfull || !fast_cell_packed(D.nK, false) ||
      (ctx->opts.vcycle_precision > 1 && &D == &ctx->K))
    return HDGMG_OK;
  int maxc = 0;
  for (int p = 0; p < D.npatch; ++p) maxc = std::max(maxc, L.patch_cell_ptr[p + 1] - L.patch_cell_ptr[p]);
  const int m2 = 2 * D.m, ncp = maxc <= 6 ? 6 : 7;
  if (maxc > 7 || !fast_fused_supported(m2, ncp)) return HDGMG_OK;
  const bool f32 = vc_f32(ctx);
  const double ws = f32 ? 4.0 : 8.0;
  const int cr = fast_cell_words_patch(m2, (int)ws);
  const long pw = fast_patch_words(m2, false);
  const int nfield = 3 * ncp + FAST_NF;
  std::vector<std::vector<int>> metas, codes;
  std::vector<double> bytes;
  for (int cc = 0; cc < L.ncol; ++cc) {
    const int p0 = L.colour_ptr[cc], np = L.colour_ptr[cc + 1] - p0;
    std::vector<int> meta((size_t)nfield * std::max(np, 1), -1), code((size_t)ncp * std::max(np, 1), -1);
    double nfac = 0, nfar = 0;
    for (int p = 0; p < np; ++p) {
      const int gp = p0 + p, v = L.patch_vertex[gp];
      const int c0 = L.patch_cell_ptr[gp], nk = L.patch_cell_ptr[gp + 1] - c0;
      const int a0 = L.patch_facet_ptr[gp], na = L.patch_facet_ptr[gp + 1] - a0;
      auto in_patch = [&](int fi) {
        return fi >= 0 && std::binary_search(L.patch_facets.begin() + a0, L.patch_facets.begin() + a0 + na, fi);
      };
      std::vector<int> far_ids;
      int perm[7][3];
      for (int j = 0; j < nk; ++j) {
        const int K = L.patch_cells[c0 + j];
        int far = -1;
        for (int lv = 0; lv < 3; ++lv)
          if (L.cells[3 * K + lv] == v) far = lv;  // the facet opposite the patch vertex
        if (far < 0) return HDGMG_OK;
        perm[j][0] = far == 0 ? 1 : 0;
        perm[j][1] = far == 2 ? 1 : 2;
        perm[j][2] = far;
        code[(size_t)p * ncp + j] = K * 4 + far;
        for (int lf = 0; lf < 3; ++lf)
          meta[(size_t)(j * 3 + lf) * np + p] = L.int_id[L.cell_facets[3 * K + perm[j][lf]]];
        const int ff = L.int_id[L.cell_facets[3 * K + far]];
        if (ff >= 0) far_ids.push_back(ff);
        // the two patch facets of the cell are its other two facets
        for (int lf = 0; lf < 2; ++lf) {
          const int fi = L.int_id[L.cell_facets[3 * K + perm[j][lf]]];
          if (fi >= 0 && !in_patch(fi)) return HDGMG_OK;
        }
        if (in_patch(ff)) return HDGMG_OK;
      }
      for (int a = 0; a < na; ++a) {
        const int fi = L.patch_facets[a0 + a];
        int cd = 0, found = 0;
        for (int j = 0; j < nk; ++j)
          for (int lf = 0; lf < 2; ++lf)
            if (L.int_id[L.cell_facets[3 * L.patch_cells[c0 + j] + perm[j][lf]]] == fi && found < 2)
              cd |= (j * 4 + lf) << (8 * found++);
        if (found != 2) return HDGMG_OK;  // a patch facet outside the patch cells: keep the pair
        meta[(size_t)(3 * ncp + a) * np + p] = cd;
      }
      std::sort(far_ids.begin(), far_ids.end());
      nfar += (double)(std::unique(far_ids.begin(), far_ids.end()) - far_ids.begin());
      nfac += na;
    }
    metas.push_back(std::move(meta));
    codes.push_back(std::move(code));
    // the triangles, the coupling blocks as stored, the metadata read (far
    // facet per slot, patch facets, sides), b once per patch facet, x once
    // per far facet, the update of x
    bytes.push_back((double)np * pw * ws + (double)np * ncp * cr * ws + (double)np * (ncp + 2 * FAST_NF) * 4.0 +
                    (2.0 * nfac + nfar) * m2 * 8.0);
  }
  for (int cc = 0; cc < L.ncol; ++cc) {
    int *dm, *dc;
    TRY(upload(ctx, &dm, metas[cc]));
    TRY(upload(ctx, &dc, codes[cc]));
    D.fmeta.push_back(dm);
    D.fcode.push_back(dc);
    const size_t n = codes[cc].size() * cr;
    if (f32) {
      float* q;
      TRY(dalloc(ctx, &q, n));
      D.Scc32.push_back(q);
    } else {
      double* q;
      TRY(dalloc(ctx, &q, n));
      D.Scc.push_back(q);
    }
  }
  D.bytes_fused_vc = bytes;
  D.fused_ncp = ncp;
  D.fused = true;
  return HDGMG_OK;
}

// The patch-ordered cell slots of a fused level from its assembled blocks.
hdgmg_status pack_fused(hdgmg_ctx* ctx, const DevLevel& D) {
  if (!D.fused) return HDGMG_OK;
  for (size_t c = 0; c < D.fcode.size(); ++c) {
    const int nslot = std::max(D.npc[c], 1) * D.fused_ncp;
    if (!D.Scc32.empty())
      launch_pack_cells_patch<float>(ctx->st, nslot, 2 * D.m, D.fcode[c], D.S, D.Scc32[c]);
    else
      launch_pack_cells_patch<double>(ctx->st, nslot, 2 * D.m, D.fcode[c], D.S, D.Scc[c]);
  }
  HIPC(hipGetLastError());
  return HDGMG_OK;
}

hdgmg_status check_status(hdgmg_ctx* ctx, const char* what) {
  int h = 0;
  HIPC(hipMemcpyAsync(&h, ctx->status, sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  HIPC(hipStreamSynchronize(ctx->st));
  if (h) {
    ctx->err = std::string(what) + ": singular local problem (status " + std::to_string(h) + ")";
    return HDGMG_ENONFINITE;
  }
  return HDGMG_OK;
}

hdgmg_status patch_inverses(hdgmg_ctx* ctx, DevLevel& D) {
  size_t need = ((size_t)D.max_ns * D.max_ns + D.max_ns) * D.npatch * sizeof(double);
  if (need > ctx->ws_bytes) {
    ctx->err = "patch workspace too small";
    return HDGMG_ENOMEM;
  }
  HIPC(hipMemsetAsync(ctx->status, 0, sizeof(int), ctx->st));
  launch_patch_inverse(ctx->st, D.view(), D.pc_ptr, D.pc, D.npatch, D.max_ns, ctx->opts.oseen ? 1 : 0, ctx->ws,
                       D.pinv, ctx->status);
  HIPC(hipGetLastError());
  return check_status(ctx, "patch inverse");
}

// Pack the cell blocks and patch inverses of a level into the streaming layout.
hdgmg_status pack_fast(hdgmg_ctx* ctx, DevLevel& D) {
  if (!D.fast) return HDGMG_OK;
  launch_pack_cells(ctx->st, D.nc, D.nK, D.S, D.Sp, D.full);
  for (size_t c = 0; c < D.npc.size(); ++c)
    launch_pack_patches(ctx->st, D.npc[c], D.colour_ptr[c], 2 * D.m, D.pf_ptr, D.pinv_off, D.pinv, D.Ppc[c],
                        D.pfull);
  HIPC(hipGetLastError());
  return HDGMG_OK;
}

// FP32 copies of the operators a level's smoothing and residuals read;
// with vcycle_precision 2, FP16 copies of the order-k level's streaming
// operators (packed cell blocks and full patch inverses) as well.
hdgmg_status make_f32(hdgmg_ctx* ctx, DevLevel& D, bool order_k = false) {
  if (!vc_f32(ctx)) return HDGMG_OK;
  D.f32 = true;
  long nS = (long)D.nc * D.nK * D.nK;
  TRY(dalloc(ctx, &D.S32, (size_t)nS));
  launch_to_f32(ctx->st, nS, D.S, D.S32);
  TRY(dalloc(ctx, &D.pinv32, (size_t)std::max(D.pinv_len, 1L)));
  launch_to_f32(ctx->st, D.pinv_len, D.pinv, D.pinv32);
  if (D.fast) {
    long nSp = (long)D.nc * D.sp_words;
    TRY(dalloc(ctx, &D.Sp32, (size_t)nSp));
    if (fast_cell_packed(D.nK, D.full))
      launch_regroup_cells_f32(ctx->st, D.nc, D.nK, D.Sp, D.Sp32);
    else
      launch_to_f32(ctx->st, nSp, D.Sp, D.Sp32);
    const long pw = fast_patch_words(2 * D.m, D.pfull);
    D.Pp32.assign(D.Ppc.size(), nullptr);
    for (size_t c = 0; c < D.Ppc.size(); ++c) {
      long n = std::max(D.npc[c], 1) * pw;
      TRY(dalloc(ctx, &D.Pp32[c], (size_t)n));
      launch_to_f32(ctx->st, n, D.Ppc[c], D.Pp32[c]);
    }
    if (order_k && ctx->opts.vcycle_precision == 2 && fast_cell_packed(D.nK, D.full)) {
      D.f16 = true;
      TRY(dalloc(ctx, &D.Sp16, (size_t)D.nc * fast_cell_words16(D.nK)));
      TRY(dalloc(ctx, &D.al16, (size_t)D.nc));
      launch_cells_f16(ctx->st, D.nc, 2 * D.m, D.Sp, D.cdof, ctx->cdiv, ctx->area, ctx->gamma, D.Sp16, D.al16);
      D.Pp16.assign(D.Ppc.size(), nullptr);
      D.psc16.assign(D.Ppc.size(), nullptr);
      for (size_t c = 0; c < D.Ppc.size(); ++c) {
        const int np = std::max(D.npc[c], 1);
        TRY(dalloc(ctx, &D.Pp16[c], (size_t)np * pw));
        TRY(dalloc(ctx, &D.psc16[c], (size_t)np));
        launch_patches_f16(ctx->st, D.npc[c], 2 * D.m, D.Ppc[c], D.Pp16[c], D.psc16[c], D.pfull);
      }
      // the preconditioner's bytes: halves plus one scale per block
      const double vec = D.bytes_cell_vc - (double)D.nc * D.sp_words * 4.0;
      D.bytes_cell_vc = (double)D.nc * (fast_cell_words16(D.nK) * 2.0 + 16.0) + vec;
      for (size_t c = 0; c < D.bytes_relax_vc.size(); ++c)
        D.bytes_relax_vc[c] -= (double)D.npc[c] * pw * 2.0 - (double)D.npc[c] * 4.0;
    }
  }
  HIPC(hipGetLastError());
  return HDGMG_OK;
}

template <typename T>
hdgmg_status upload_f32(hdgmg_ctx* ctx, float** p, const std::vector<T>& h) {
  std::vector<float> f(h.begin(), h.end());
  return upload(ctx, p, f);
}

// ------------------------------------------------------------ multigrid
// Algorithmic bytes of Gauss-Seidel colour phase c of a level (level < 0:
// the order-k level) in the storage the V-cycle reads.
double phase_bytes(const hdgmg_ctx* ctx, const DevLevel& D, int level, int c) {
  if (D.fused) return D.bytes_fused_vc[c];
  if (D.rec) return D.rec_bytes[c];
  if (D.fast) return D.bytes_cell_vc + D.bytes_relax_vc[c];
  const double scale = D.f32 ? 0.5 : 1.0;  // operator words dominate the phase bytes
  const std::vector<double>& t = level < 0 ? ctx->relax_bytes : ctx->smooth_bytes[level];
  return c < (int)t.size() ? scale * t[c] : 0.0;
}

// One Gauss-Seidel sweep over the colours.  x_zero: x is zero on entry, so
// the first colour phase of the streaming layout needs no cell apply (its
// residual is b).
void level_apply(hdgmg_ctx* ctx, DevLevel& D, const double* x, double* y, double alpha, const double* b,
                 int cls, bool vc);

// Damped block Jacobi sweep (eq. bjac): r = b - A x once, then every
// colour's patches add damp A_ss^-1 r_s (launch-per-colour layout only).
void jacobi_sweep(hdgmg_ctx* ctx, DevLevel& D, double* x, const double* b, int level) {
  const int nc = (int)D.colour_ptr.size() - 1;
  const int cls = level < 0 ? 0 : 2;
  level_apply(ctx, D, x, D.r, -1.0, b, cls, true);
  for (int c = 0; c < nc; ++c) {
    int t = kt_begin(ctx, cls);
    if (D.f32)
      launch_patch_correct<float>(ctx->st, D.pf_ptr, D.pf, D.pinv_off, D.pinv32, 2 * D.m, D.max_ns,
                                  D.colour_ptr[c], D.colour_ptr[c + 1], D.r, x, 1.0 / nc);
    else
      launch_patch_correct<double>(ctx->st, D.pf_ptr, D.pf, D.pinv_off, D.pinv, 2 * D.m, D.max_ns,
                                   D.colour_ptr[c], D.colour_ptr[c + 1], D.r, x, 1.0 / nc);
    kt_end(ctx, cls, t, phase_bytes(ctx, D, level, c));
  }
}

void sweep(hdgmg_ctx* ctx, DevLevel& D, double* x, const double* b, bool forward, int level, bool x_zero = false) {
  if (ctx->opts.smoother == 1) {
    jacobi_sweep(ctx, D, x, b, level);
    return;
  }
  const int nc = (int)D.colour_ptr.size() - 1;
  for (int i = 0; i < nc; ++i) {
    int c = forward ? i : nc - 1 - i;
    if (D.fused && !(x_zero && i == 0)) {
      // the colour phase in one launch
      const int fcls = level < 0 ? 0 : 2;
      const KtDispatch kf = kd_begin(ctx, fcls);
      if (D.f32)
        launch_patch_gs_fused<float>(ctx->st, 2 * D.m, D.fused_ncp, D.npc[c], D.pfc[c], D.fmeta[c], D.Pp32[c],
                                     D.Scc32[c], b, x, kf.ptr());
      else
        launch_patch_gs_fused<double>(ctx->st, 2 * D.m, D.fused_ncp, D.npc[c], D.pfc[c], D.fmeta[c], D.Ppc[c],
                                      D.Scc[c], b, x, kf.ptr());
      kd_end(ctx, fcls, kf, D.bytes_fused_vc[c]);
    } else if (D.rec) {
      int t = kt_begin(ctx, 2);
      launch_gs_records(ctx->st, D.rk, D.rv, D.ra, D.rnit, D.rnsm, D.rcb[c], D.rcb[c + 1] - D.rcb[c], x, b,
                        D.f32 ? 1 : 0, D.rwide ? 1 : 0);
      kt_end(ctx, 2, t, phase_bytes(ctx, D, level, c));
    } else if (D.fast) {
      // colour phase = cell apply (all cells) + patch relaxation (colour c)
      // (the first phase from a zero iterate of a fused level: relaxation only)
      const bool skip = x_zero && i == 0;
      if (!skip) {
        const int ccls = level < 0 ? 1 : 2;
        const KtDispatch kd = kd_begin(ctx, ccls);
        if (D.f16)
          launch_cell_apply<_Float16>(ctx->st, 2 * D.m, D.nc, D.Sp16, D.cdof, x, D.yF, false, D.al16, kd.ptr());
        else if (D.f32)
          launch_cell_apply<float>(ctx->st, 2 * D.m, D.nc, D.Sp32, D.cdof, x, D.yF, D.full, nullptr, kd.ptr());
        else
          launch_cell_apply<double>(ctx->st, 2 * D.m, D.nc, D.Sp, D.cdof, x, D.yF, D.full, nullptr, kd.ptr());
        kd_end(ctx, ccls, kd, D.bytes_cell_vc);
      }
      const double* yF = skip ? nullptr : D.yF;
      const int rcls = level < 0 ? 0 : 2;
      const KtDispatch kr = kd_begin(ctx, rcls);
      if (D.f16)
        launch_patch_relax<_Float16>(ctx->st, 2 * D.m, D.npc[c], D.pfc[c], D.Pp16[c], b, yF, x, D.pfull,
                                     D.psc16[c], kr.ptr());
      else if (D.f32)
        launch_patch_relax<float>(ctx->st, 2 * D.m, D.npc[c], D.pfc[c], D.Pp32[c], b, yF, x, D.pfull, nullptr,
                                  kr.ptr());
      else
        launch_patch_relax<double>(ctx->st, 2 * D.m, D.npc[c], D.pfc[c], D.Ppc[c], b, yF, x, D.pfull, nullptr,
                                   kr.ptr());
      kd_end(ctx, rcls, kr, D.bytes_relax_vc[c]);
    } else {
      const int cls = level < 0 ? 0 : 2;
      int t = kt_begin(ctx, cls);
      if (D.f32)
        launch_gs<float>(ctx->st, D.view_t<float>(), D.colour_ptr[c], D.colour_ptr[c + 1], x, b);
      else
        launch_gs<double>(ctx->st, D.view_t<double>(), D.colour_ptr[c], D.colour_ptr[c + 1], x, b);
      kt_end(ctx, cls, t, phase_bytes(ctx, D, level, c));
    }
  }
}

// y = alpha A x + b on any level (streaming layout when available); vc:
// read the preconditioner's storage (FP32 when so configured).
void level_apply(hdgmg_ctx* ctx, DevLevel& D, const double* x, double* y, double alpha, const double* b,
                 int cls, bool vc) {
  const bool f32 = vc && D.f32;
  if (D.fast) {
    const KtDispatch kd = kd_begin(ctx, cls);
    if (vc && D.f16)
      launch_cell_apply<_Float16>(ctx->st, 2 * D.m, D.nc, D.Sp16, D.cdof, x, D.yF, false, D.al16, kd.ptr());
    else if (f32)
      launch_cell_apply<float>(ctx->st, 2 * D.m, D.nc, D.Sp32, D.cdof, x, D.yF, D.full, nullptr, kd.ptr());
    else
      launch_cell_apply<double>(ctx->st, 2 * D.m, D.nc, D.Sp, D.cdof, x, D.yF, D.full, nullptr, kd.ptr());
    kd_end(ctx, cls, kd, f32 ? D.bytes_cell_vc : D.bytes_cell);
    launch_facet_sum(ctx->st, D.nint, 2 * D.m, D.yF, b, alpha, y);
  } else {
    int t = kt_begin(ctx, cls);
    if (f32) {
      LevelViewT<float> v = D.view_t<float>();
      launch_apply<float>(ctx->st, v, x, y, alpha, b);
    } else {
      LevelViewT<double> v = D.view_t<double>();
      v.S = D.S;
      launch_apply<double>(ctx->st, v, x, y, alpha, b);
    }
    kt_end(ctx, cls, t, (f32 ? 0.5 : 1.0) * ctx->apply_bytes + (b ? D.ndof * 8.0 : 0.0));
  }
}

// Skeleton apply on the order-k level, timed as class 1.
void apply_k(hdgmg_ctx* ctx, const double* x, double* y, double alpha, const double* b, bool vc = false) {
  level_apply(ctx, ctx->K, x, y, alpha, b, 1, vc);
}

// Alg. 1 on lowest-order level l: u_l <- MG_h(l, g_l, u_l, m_l, q); u_zero:
// u_l is zero on entry.
void mg_h(hdgmg_ctx* ctx, int l, int m_l, bool u_zero) {
  DevLevel& D = ctx->cr[l];
  if (ctx->dense_on && l == ctx->dense_level && u_zero && m_l == ctx->dense_m) {
    // u = MG_h(l, g, 0): the tabulated operator
    int t = kt_begin(ctx, 4);
    const bool f32 = vc_f32(ctx);
    const int n = ctx->dense_n;
    if (f32)
      launch_gemv_rows<float>(ctx->st, n, ctx->dense_ld, (const float*)ctx->dense_M, D.g, D.u);
    else
      launch_gemv_rows<double>(ctx->st, n, ctx->dense_ld, (const double*)ctx->dense_M, D.g, D.u);
    kt_end(ctx, 4, t, (double)n * n * (f32 ? 4.0 : 8.0) + 2.0 * n * 8.0);
    return;
  }
  if (l <= ctx->Lc) {
    int t = kt_begin(ctx, 4);
    const bool f32 = vc_f32(ctx);
    launch_coarse_cycle(ctx->st, ctx->coarse_desc, l, m_l, ctx->opts.vcycle_growth, ctx->opts.cycle,
                        f32 ? (const void*)ctx->coarse_inv32 : (const void*)ctx->coarse_inv, ctx->n0,
                        ctx->coarse_ns, ctx->coarse_lds, f32 ? 1 : 0);
    kt_end(ctx, 4, t, 0.0);
    return;
  }
  if (l == 0) {
    if (vc_f32(ctx))
      launch_gemv_rows<float>(ctx->st, ctx->n0, ctx->ld0, ctx->coarse_rows32, D.g, D.u);
    else
      launch_gemv_rows<double>(ctx->st, ctx->n0, ctx->ld0, ctx->coarse_rows, D.g, D.u);
    return;
  }
  for (int s = 0; s < m_l; ++s) sweep(ctx, D, D.u, D.g, true, l, u_zero && s == 0);
  level_apply(ctx, D, D.u, D.r, -1.0, D.g, 2, true);
  DevTransfer& T = ctx->tr[l];
  DevLevel& C = ctx->cr[l - 1];
  if (T.RL && vc_f32(ctx))
    launch_sell_spmv<float>(ctx->st, T.ncoarse, T.RL, T.Rs_off, T.Rs_w, T.Rs_ci, T.Rs_v32, D.r, C.g, 0.0, C.u);
  else if (T.RL)
    launch_sell_spmv<double>(ctx->st, T.ncoarse, T.RL, T.Rs_off, T.Rs_w, T.Rs_ci, T.Rs_v, D.r, C.g, 0.0, C.u);
  else if (vc_f32(ctx))
    launch_ell_spmv<float>(ctx->st, T.ncoarse, T.Rw, T.Re_ci, T.Re_v32, D.r, C.g, 0.0, C.u);
  else
    launch_ell_spmv<double>(ctx->st, T.ncoarse, T.Rw, T.Re_ci, T.Re_v, D.r, C.g, 0.0, C.u);  // and C.u = 0
  for (int n = 0; n < ctx->opts.cycle; ++n) mg_h(ctx, l - 1, ctx->opts.vcycle_growth * m_l, n == 0);
  if (T.PL && vc_f32(ctx))
    launch_sell_spmv<float>(ctx->st, T.nfine, T.PL, T.Ps_off, T.Ps_w, T.Ps_ci, T.Ps_v32, C.u, D.u, 1.0);
  else if (T.PL)
    launch_sell_spmv<double>(ctx->st, T.nfine, T.PL, T.Ps_off, T.Ps_w, T.Ps_ci, T.Ps_v, C.u, D.u, 1.0);
  else if (vc_f32(ctx))
    launch_ell_spmv<float>(ctx->st, T.nfine, T.Pw, T.Pe_ci, T.Pe_v32, C.u, D.u, 1.0);
  else
    launch_ell_spmv<double>(ctx->st, T.nfine, T.Pw, T.Pe_ci, T.Pe_v, C.u, D.u, 1.0);
  for (int s = 0; s < m_l; ++s) sweep(ctx, D, D.u, D.g, false, l);
}

// Alg. 2 with zero initial guess: z = MG_hp(r)
void mg_hp_body(hdgmg_ctx* ctx, const double* r, double* z);
// Per-kernel timers (every class but the whole-cycle one, 3) bracket each
// launch with events, so the cycle then runs eagerly; the whole-cycle timer
// alone brackets the graph replay.
bool timers_on(const hdgmg_ctx* ctx) {
  for (int c = 0; c < (int)(sizeof(ctx->timers) / sizeof(ctx->timers[0])); ++c)
    if (c != 3 && ctx->timers[c].on) return true;
  return false;
}

void drop_graph(hdgmg_ctx* ctx) {
  if (ctx->vc_exec) (void)hipGraphExecDestroy(ctx->vc_exec);
  ctx->vc_exec = nullptr;
  ctx->vc_r = nullptr;
  ctx->vc_z = nullptr;
}

// The launch sequence of MG_hp depends only on the hierarchy and the
// options, so it is captured once per (r, z) pair and replayed.  While live
// kernel timers are on, the launches go eagerly (events bracket them).
void mg_hp(hdgmg_ctx* ctx, const double* r, double* z) {
  int t = kt_begin(ctx, 3);
  if (!ctx->use_graph || timers_on(ctx)) {
    mg_hp_body(ctx, r, z);
  } else {
    if (!ctx->vc_exec || ctx->vc_r != r || ctx->vc_z != z) {
      drop_graph(ctx);
      hipGraph_t g = nullptr;
      bool ok = hipStreamBeginCapture(ctx->st, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        mg_hp_body(ctx, r, z);
        ok = hipStreamEndCapture(ctx->st, &g) == hipSuccess && g;
      }
      if (ok) ok = hipGraphInstantiate(&ctx->vc_exec, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
      if (!ok) {
        // capture unavailable on this stream: run eagerly from now on
        (void)hipGetLastError();
        ctx->vc_exec = nullptr;
        ctx->use_graph = false;
        mg_hp_body(ctx, r, z);
        kt_end(ctx, 3, t, ctx->vcycle_bytes);
        return;
      }
      ctx->vc_r = r;
      ctx->vc_z = z;
    }
    (void)hipGraphLaunch(ctx->vc_exec, ctx->st);
  }
  kt_end(ctx, 3, t, ctx->vcycle_bytes);
}
void mg_hp_body(hdgmg_ctx* ctx, const double* r, double* z) {
  DevLevel& KL = ctx->K;
  DevLevel& DJ = ctx->cr[ctx->J - 1];
  if (ctx->k == 0) {
    launch_copy(ctx->st, DJ.ndof, r, DJ.g);
    launch_fill(ctx->st, DJ.ndof, 0.0, DJ.u);
    mg_h(ctx, ctx->J - 1, ctx->opts.m_smooth, true);
    launch_copy(ctx->st, DJ.ndof, DJ.u, z);
    return;
  }
  launch_fill(ctx->st, KL.ndof, 0.0, z);
  if (ctx->opts.additive) {
    // additive counterpart: relaxation and lowest-order correction of r
    for (int s = 0; s < ctx->opts.m_relax; ++s) sweep(ctx, KL, z, r, true, -1, s == 0);
    for (int s = 0; s < ctx->opts.m_relax; ++s) sweep(ctx, KL, z, r, false, -1);
    launch_mode0_extract(ctx->st, KL.nint, KL.m, r, DJ.g, DJ.u);
    mg_h(ctx, ctx->J - 1, ctx->opts.m_smooth, true);
    launch_mode0_add(ctx->st, KL.nint, KL.m, DJ.u, z);
    return;
  }
  for (int s = 0; s < ctx->opts.m_relax; ++s) sweep(ctx, KL, z, r, true, -1, s == 0);
  // Pi_k^0 (r - A z): only the mode-0 rows of A z (and DJ.u = 0)
  if (vc_f32(ctx))
    launch_mode0_residual<float>(ctx->st, KL.nc, KL.nint, KL.m, KL.cell_dofs, KL.fcell, KL.floc, KL.S0_32, z,
                                 KL.y0K, r, DJ.g, DJ.u);
  else
    launch_mode0_residual<double>(ctx->st, KL.nc, KL.nint, KL.m, KL.cell_dofs, KL.fcell, KL.floc, KL.S0, z,
                                  KL.y0K, r, DJ.g, DJ.u);
  mg_h(ctx, ctx->J - 1, ctx->opts.m_smooth, true);
  launch_mode0_add(ctx->st, KL.nint, KL.m, DJ.u, z);
  for (int s = 0; s < ctx->opts.m_relax; ++s) sweep(ctx, KL, z, r, false, -1);
}

// Device scratch of the Krylov solvers: the recurrence scalars (sc, SC_N
// words), block partials of the dot products (part, 4 RED_BLOCKS words) and,
// for FGMRES, the partials of the projections on the basis (gm_part,
// (restart+1) RED_BLOCKS words), the projection coefficients of both
// Gram-Schmidt passes plus the new norm (gm_h, 4*128 words) and the
// least-squares solution (gm_y, 128 words).  Every word is written before it
// is read within one solve.
struct KrylovScratch {
  double *sc, *part, *gm_part, *gm_h, *gm_y;
};
KrylovScratch ctx_scratch(const hdgmg_ctx* ctx) {
  return KrylovScratch{ctx->sc, ctx->part, ctx->gm_part, ctx->gm_h, ctx->gm_y};
}

// Flexible CG for A^eps x = b from x = 0.
hdgmg_status fcg(hdgmg_ctx* ctx, const KrylovScratch& W, const double* b, double* x, int* its_out,
                 double* rel_out) {
  const long n = ctx->K.ndof;
  const int NB = RED_BLOCKS;
  hipStream_t st = ctx->st;
  double hs[SC_N];
  launch_fill(st, n, 0.0, x);
  launch_copy(st, n, b, ctx->r);
  launch_dot(st, n, ctx->r, ctx->r, W.part, NB);
  launch_finalize(st, W.part, NB, 1, W.sc, SC_BB);
  HIPC(hipMemcpyAsync(hs, W.sc, sizeof(hs), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  const double r0 = std::sqrt(hs[SC_BB]);
  if (!std::isfinite(r0)) {
    ctx->err = "non-finite right-hand side";
    return HDGMG_ENONFINITE;
  }
  const double tol = std::max(ctx->opts.rtol * r0, ctx->opts.atol);
  if (its_out) *its_out = 0;
  if (rel_out) *rel_out = r0 > 0 ? 1.0 : 0.0;
  if (r0 <= tol) return HDGMG_OK;
  mg_hp(ctx, ctx->r, ctx->z);
  launch_dot(st, n, ctx->z, ctx->r, W.part, NB);
  launch_finalize(st, W.part, NB, 1, W.sc, SC_ZR);
  launch_copy(st, n, ctx->z, ctx->p);
  int it = 0;
  double rn = r0;
  while (it < ctx->opts.max_it) {
    apply_k(ctx, ctx->p, ctx->q, 1.0, nullptr);
    launch_dot(st, n, ctx->p, ctx->q, W.part, NB);
    launch_finalize(st, W.part, NB, 1, W.sc, SC_PQ);
    launch_fcg_xr(st, n, x, ctx->r, ctx->r_old, ctx->p, ctx->q, W.sc, W.part, NB);
    launch_finalize(st, W.part, NB, 1, W.sc, SC_RR);
    HIPC(hipMemcpyAsync(hs, W.sc, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    ++it;
    // breakdown first: with z.r = 0 or p.Ap = 0 the step itself is 0/0
    if (hs[SC_PQ] <= 0.0 || hs[SC_ZR] <= 0.0) {
      ctx->err = "flexible CG breakdown (p.Ap <= 0 or z.r <= 0)";
      return HDGMG_EBREAKDOWN;
    }
    if (!std::isfinite(hs[SC_RR]) || !std::isfinite(hs[SC_PQ]) || !std::isfinite(hs[SC_ZR])) {
      ctx->err = "non-finite value in flexible CG";
      return HDGMG_ENONFINITE;
    }
    rn = std::sqrt(hs[SC_RR]);
    if (its_out) *its_out = it;
    if (rel_out) *rel_out = rn / r0;
    if (rn <= tol) return HDGMG_OK;
    mg_hp(ctx, ctx->r, ctx->z);
    launch_dot2(st, n, ctx->z, ctx->r, ctx->r_old, W.part, NB);
    launch_finalize(st, W.part, NB, 2, W.sc, SC_ZRN);
    launch_fcg_p(st, n, ctx->p, ctx->z, W.sc);
    launch_scalar_move(st, W.sc, SC_ZRN, SC_ZR);
  }
  ctx->err = "inner solve reached max_it";
  return HDGMG_NOT_CONVERGED;
}

// Flexible GMRES(restart) with right preconditioning by MG_hp (Sec. 4.2),
// from the iterate in x.  Orthogonalisation: classical Gram-Schmidt applied
// twice (two fused passes over the basis; the same projections as modified
// Gram-Schmidt in exact arithmetic).  The Hessenberg least-squares problem
// (Givens rotations) is solved on the host, one transfer of the new column
// per iteration.  Stops at |residual estimate| <= max(rtol ||r_0||, atol).
hdgmg_status fgmres(hdgmg_ctx* ctx, const KrylovScratch& W, const double* b, double* x, int* its_out,
                    double* rel_out) {
  const long n = ctx->K.ndof;
  const int m = ctx->opts.restart, NB = RED_BLOCKS;
  hipStream_t st = ctx->st;
  double* V = ctx->gm_V;
  double* Z = ctx->gm_Z;
  auto Vj = [&](int j) { return V + (long)j * n; };
  auto Zj = [&](int j) { return Z + (long)j * n; };
  auto norm_of = [&](const double* v, double* out) -> hdgmg_status {
    launch_dot(st, n, v, v, W.part, NB);
    launch_finalize(st, W.part, NB, 1, W.sc, SC_BB);
    double hs[SC_N];
    HIPC(hipMemcpyAsync(hs, W.sc, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    *out = std::sqrt(hs[SC_BB]);
    return HDGMG_OK;
  };
  apply_k(ctx, x, Vj(0), -1.0, b);  // r = b - A x
  double beta;
  TRY(norm_of(Vj(0), &beta));
  if (!std::isfinite(beta)) {
    ctx->err = "non-finite residual";
    return HDGMG_ENONFINITE;
  }
  const double beta0 = beta, tol = std::max(ctx->opts.rtol * beta0, ctx->opts.atol);
  if (its_out) *its_out = 0;
  if (rel_out) *rel_out = beta0 > 0 ? 1.0 : 0.0;
  if (beta <= tol) return HDGMG_OK;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hb(4 * 128);
  int its = 0;
  double res = beta;
  while (true) {
    launch_scale(st, n, 1.0 / beta, Vj(0), Vj(0));
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      // z_j = MG_hp(v_j) through the preconditioner's fixed buffers
      launch_copy(st, n, Vj(j), ctx->r);
      mg_hp(ctx, ctx->r, ctx->z);
      launch_copy(st, n, ctx->z, Zj(j));
      double* w = Vj(j + 1);
      apply_k(ctx, Zj(j), w, 1.0, nullptr);
      for (int pass = 0; pass < 2; ++pass) {
        launch_mdot(st, n, j + 1, V, n, w, W.gm_part, NB);
        launch_finalize(st, W.gm_part, NB, j + 1, W.gm_h + 128 * pass, 0);
        launch_maxpy(st, n, j + 1, V, n, W.gm_h + 128 * pass, -1.0, w);
      }
      launch_dot(st, n, w, w, W.part, NB);
      launch_finalize(st, W.part, NB, 1, W.gm_h + 256, 0);
      HIPC(hipGetLastError());
      HIPC(hipMemcpyAsync(hb.data(), W.gm_h, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hb[i] + hb[128 + i];
      const double hn = std::sqrt(std::max(hb[256], 0.0));
      if (!std::isfinite(hn)) {
        ctx->err = "non-finite value in FGMRES";
        return HDGMG_ENONFINITE;
      }
      if (hn > 0.0) launch_scale(st, n, 1.0 / hn, w, w);
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * m + j], den = std::hypot(a, hn);
      if (!(den > 0.0)) {
        ctx->err = "FGMRES breakdown (zero Hessenberg column)";
        return HDGMG_EBREAKDOWN;
      }
      cs[j] = a / den;
      sn[j] = hn / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      jend = j + 1;
      res = std::fabs(g[j + 1]);
      if (res <= tol || its >= ctx->opts.max_it || hn == 0.0) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < jend; ++q) t -= H[(size_t)i * m + q] * y[q];
      y[i] = t / H[(size_t)i * m + i];
    }
    HIPC(hipMemcpyAsync(W.gm_y, y.data(), jend * sizeof(double), hipMemcpyHostToDevice, st));
    launch_maxpy(st, n, jend, Z, n, W.gm_y, 1.0, x);
    HIPC(hipStreamSynchronize(st));  // y is read before it goes out of scope
    if (its_out) *its_out = its;
    if (rel_out) *rel_out = res / beta0;
    if (res <= tol) return HDGMG_OK;
    if (its >= ctx->opts.max_it) break;
    apply_k(ctx, x, Vj(0), -1.0, b);
    TRY(norm_of(Vj(0), &beta));
    if (!std::isfinite(beta)) {
      ctx->err = "non-finite residual";
      return HDGMG_ENONFINITE;
    }
    if (beta <= tol) {
      if (rel_out) *rel_out = beta / beta0;
      return HDGMG_OK;
    }
  }
  ctx->err = "inner solve reached max_it";
  return HDGMG_NOT_CONVERGED;
}

hdgmg_status build_transfers(hdgmg_ctx* ctx) {
  ctx->tr.assign(ctx->J, DevTransfer());
  const bool general = ctx->opts.oseen != 0;
  // host construction of every level's transfers at once (a thread per level
  // and operator; the large levels split their coarse cells further)
  const int J = ctx->J;
  std::vector<CSR> Ps(J), Pts(J);
  std::vector<char> okP(J, 1), okT(J, 1);
  {
    std::vector<std::thread> th;
    for (int l = 1; l < J; ++l) {
      // prolongation harmonic for A; restriction the transpose of the same
      // construction for A^T (the transpose of P when A is symmetric)
      th.emplace_back([&, l] {
        okP[l] = stabilised_transfer(ctx->lv[l - 1], ctx->lv[l], ctx->avg[l], ctx->hostB[l], false, general, Ps[l]);
      });
      if (ctx->has_wind)
        th.emplace_back([&, l] {
          okT[l] = stabilised_transfer(ctx->lv[l - 1], ctx->lv[l], ctx->avg[l], ctx->hostB[l], true, general, Pts[l]);
        });
    }
    for (auto& t : th) t.join();
  }
  for (int l = 1; l < ctx->J; ++l) {
    CSR& P = Ps[l];
    CSR R;
    bool ok = okP[l] && okT[l];
    if (ok) csr_transpose(ctx->has_wind ? Pts[l] : P, 2 * ctx->lv[l - 1].nint, R);
    if (!ok) {
      ctx->err = "singular interior block in harmonic extension";
      return HDGMG_ENONFINITE;
    }
    DevTransfer& Tt = ctx->tr[l];
    Tt.nfine = P.n;
    Tt.ncoarse = R.n;
    Tt.nnz = (long)std::max(P.ci.size(), R.ci.size());
    std::vector<int> eci;
    std::vector<double> ev;
    to_ell(P, Tt.Pw, eci, ev);
    TRY(upload(ctx, &Tt.Pe_ci, eci));
    TRY(upload(ctx, &Tt.Pe_v, ev));
    if (vc_f32(ctx)) TRY(upload_f32(ctx, &Tt.Pe_v32, ev));
    to_ell(R, Tt.Rw, eci, ev);
    TRY(upload(ctx, &Tt.Re_ci, eci));
    TRY(upload(ctx, &Tt.Re_v, ev));
    if (vc_f32(ctx)) TRY(upload_f32(ctx, &Tt.Re_v32, ev));
    // sliced copies for the launched products with wide rows on large
    // levels (below 65536 rows the extra slice-offset load costs more than
    // the padding it saves)
    std::vector<long> soff;
    std::vector<int> sw;
    constexpr int kSellRows = 65536;
    Tt.PL = P.n >= kSellRows ? sell_lanes(Tt.Pw) : 0;
    if (Tt.PL) {
      to_sell(P, Tt.PL, soff, sw, eci, ev);
      TRY(upload(ctx, &Tt.Ps_off, soff));
      TRY(upload(ctx, &Tt.Ps_w, sw));
      TRY(upload(ctx, &Tt.Ps_ci, eci));
      TRY(upload(ctx, &Tt.Ps_v, ev));
      if (vc_f32(ctx)) TRY(upload_f32(ctx, &Tt.Ps_v32, ev));
    }
    Tt.RL = R.n >= kSellRows ? sell_lanes(Tt.Rw) : 0;
    if (Tt.RL) {
      to_sell(R, Tt.RL, soff, sw, eci, ev);
      TRY(upload(ctx, &Tt.Rs_off, soff));
      TRY(upload(ctx, &Tt.Rs_w, sw));
      TRY(upload(ctx, &Tt.Rs_ci, eci));
      TRY(upload(ctx, &Tt.Rs_v, ev));
      if (vc_f32(ctx)) TRY(upload_f32(ctx, &Tt.Rs_v32, ev));
    }
  }
  std::vector<double> inv;
  if (!coarse_inverse(ctx->lv[0], ctx->hostB[0], general, inv)) {
    ctx->err = general ? "coarsest operator singular" : "coarsest operator not positive definite";
    return HDGMG_ENONFINITE;
  }
  ctx->n0 = 2 * ctx->lv[0].nint;
  TRY(upload(ctx, &ctx->coarse_inv, inv));
  if (vc_f32(ctx)) TRY(upload_f32(ctx, &ctx->coarse_inv32, inv));
  ctx->ld0 = (ctx->n0 + 3) / 4 * 4;
  if (vc_f32(ctx)) {
    TRY(dalloc(ctx, &ctx->coarse_rows32, (size_t)std::max(ctx->n0, 1) * std::max(ctx->ld0, 4)));
    launch_transpose_to<float>(ctx->st, ctx->n0, ctx->ld0, ctx->coarse_inv, ctx->coarse_rows32);
  } else {
    TRY(dalloc(ctx, &ctx->coarse_rows, (size_t)std::max(ctx->n0, 1) * std::max(ctx->ld0, 4)));
    launch_transpose_to<double>(ctx->st, ctx->n0, ctx->ld0, ctx->coarse_inv, ctx->coarse_rows);
  }
  HIPC(hipGetLastError());
  return HDGMG_OK;
}

// Descriptors of the levels handled by the single-workgroup coarse kernel:
// per patch row its padded residual row (from the assembled operator) and its
// row of the patch inverse (host FP64 Cholesky), structure-of-arrays.
// Patch-row records of a lowest-order level (structure-of-arrays over
// items; per item two 16-byte meta words (key, columns 0-2), (columns 3-4)
// at [w][t]; values and inverse rows in groups of G = 2 (FP64) or 4 (FP32),
// entry e at [((e / G) * nit + t) * G + e % G], so that a lane reads a group
// with one 16-byte load): the unknown and its row inside
// the patch, the padded residual row (16-bit column pairs) and the row of the
// patch inverse; items colour by colour in patch-aligned batches of at most
// max_items.  Also the padded residual rows per unknown.
struct LevelRecords {
  int n = 0, nit = 0, nsm = 0;
  bool wide = false;  // 32-bit fields, 8 meta words per item
  std::vector<unsigned> meta;
  std::vector<double> val, ainv;
  std::vector<int> cb, bitem, bwd;
  std::vector<int> rw_col;
  std::vector<double> rw_val;
};

// pad: every batch fills exactly max_items item slots (padding items carry
// the row marker REC_PAD and zero values), so that batch b starts at item
// b * max_items.
hdgmg_status level_records(hdgmg_ctx* ctx, int l, int max_items, LevelRecords& R, bool pad = false,
                           bool wide = false) {
  const Level& L = ctx->lv[l];
  const int n = 2 * L.nint;
  R = LevelRecords();
  R.n = n;
  R.wide = wide;
  if (!wide && (L.nint > 65535 || n > (int)REC_DOF_MASK)) {
    ctx->err = "level too large for 16-bit record facet indices";
    return HDGMG_EMESH;
  }
  CSR A;
  assemble_csr(L, ctx->hostB[l], A);
  R.rw_col.assign((size_t)COARSE_NNZ * n, 0);
  R.rw_val.assign((size_t)COARSE_NNZ * n, 0.0);
  for (int i = 0; i < n; ++i)
    if (A.rp[i + 1] - A.rp[i] > COARSE_NNZ) {
      ctx->err = "lowest-order row with more than 10 entries";
      return HDGMG_EMESH;
    }
  for (int k = 0; k < COARSE_NNZ; ++k)  // entry-major: contiguous writes
    for (int i = 0; i < n; ++i)
      if (k < A.rp[i + 1] - A.rp[i]) {
        R.rw_col[(size_t)k * n + i] = A.ci[A.rp[i] + k];
        R.rw_val[(size_t)k * n + i] = A.v[A.rp[i] + k];
      }
  const int nsm = 2 * L.max_patch_facets;
  R.nsm = nsm;
  R.cb.assign(1, 0);
  R.bitem.assign(1, 0);
  // the patch inverses as the assembly computed them on the device
  // (patch_inverses: column-major per patch, in the level's patch order,
  // singular blocks already rejected there), copied back once
  const int npatch = L.colour_ptr[L.ncol];
  const DevLevel& DL = ctx->cr[l];
  std::vector<long> poff(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) {
    const long ns = 2L * (L.patch_facet_ptr[p + 1] - L.patch_facet_ptr[p]);
    poff[p + 1] = poff[p] + ns * ns;
  }
  if (poff[npatch] != DL.pinv_len) {
    ctx->err = "record construction: patch inverse layout mismatch";
    return HDGMG_EMESH;
  }
  std::vector<double> pinv_h((size_t)std::max<long>(DL.pinv_len, 1));
  if (DL.pinv_len > 0) {
    HIPC(hipMemcpyAsync(pinv_h.data(), DL.pinv, (size_t)DL.pinv_len * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->st));
    HIPC(hipStreamSynchronize(ctx->st));
  }
  std::vector<int> idof, iloc;
  std::vector<double> irow;  // [item][nsm]
  {
    const size_t items = (size_t)2 * L.patch_facet_ptr[npatch] * (pad ? 5 : 4) / 4;  // padding: about a quarter more
    idof.reserve(items);
    iloc.reserve(items);
    irow.reserve(items * nsm);
  }
  for (int c = 0; c < L.ncol; ++c) {
    for (int p = L.colour_ptr[c]; p < L.colour_ptr[c + 1]; ++p) {
      int f0 = L.patch_facet_ptr[p], nfp = L.patch_facet_ptr[p + 1] - f0;
      int ns = 2 * nfp;
      std::vector<int> dofs(ns);
      for (int a = 0; a < nfp; ++a)
        for (int comp = 0; comp < 2; ++comp) dofs[2 * a + comp] = 2 * L.patch_facets[f0 + a] + comp;
      const double* inv = pinv_h.data() + poff[p];
      if ((int)idof.size() - R.bitem.back() + ns > max_items) {
        while (pad && (int)idof.size() - R.bitem.back() < max_items) {
          idof.push_back(-1);
          iloc.push_back((int)REC_PAD);
          for (int j = 0; j < nsm; ++j) irow.push_back(0.0);
        }
        R.bitem.push_back((int)idof.size());
      }
      for (int i = 0; i < ns; ++i) {
        idof.push_back(dofs[i]);
        iloc.push_back(i);
        for (int j = 0; j < nsm; ++j) irow.push_back(j < ns ? inv[(size_t)j * ns + i] : 0.0);  // row i
      }
    }
    if ((int)idof.size() > R.bitem.back()) {
      while (pad && (int)idof.size() - R.bitem.back() < max_items) {
        idof.push_back(-1);
        iloc.push_back((int)REC_PAD);
        for (int j = 0; j < nsm; ++j) irow.push_back(0.0);
      }
      R.bitem.push_back((int)idof.size());
    }
    R.cb.push_back((int)R.bitem.size() - 1);
  }
  const int nit = (int)idof.size();
  R.nit = nit;
  const int MW = wide ? 8 : 4;  // meta words per item
  R.meta.assign((size_t)MW * nit, 0u);
  // value groups: pairs for FP64 storage, quads for FP32 (16-byte loads)
  const int G = vc_f32(ctx) ? 4 : 2;
  const int nvg = (COARSE_NNZ + G - 1) / G, nag = (std::max(nsm, 1) + G - 1) / G;
  R.val.assign((size_t)nvg * G * nit, 0.0);
  R.ainv.assign((size_t)nag * G * nit, 0.0);
  // items are independent: contiguous ranges of them on host threads
  std::atomic<bool> bad_pairs{false};
  auto fill = [&](int t_begin, int t_end) {
  for (int t = t_begin; t < t_end; ++t) {
    if (idof[t] < 0) {  // padding: row marker REC_PAD, unknown 0, zero values
      if (wide)
        R.meta[(size_t)t * 8 + 1] = REC_PAD;
      else
        R.meta[(size_t)t * 4] = REC_PAD << REC_LOC_SHIFT;
      continue;
    }
    // meta (key, F0 | F1 << 16, F2 | F3 << 16, F4): the row's columns come in
    // facet pairs (2F, 2F + 1), sorted, padded with zero entries; wide:
    // (unknown, row, F0, F1), (F2, F3, F4, 0)
    if (wide) {
      R.meta[(size_t)t * 8] = (unsigned)idof[t];
      R.meta[(size_t)t * 8 + 1] = (unsigned)iloc[t];
    } else {
      R.meta[(size_t)t * 4] = (unsigned)idof[t] | ((unsigned)iloc[t] << REC_LOC_SHIFT);
    }
    // values in groups of G: entry e of item t at [((e / G) * nit + t) * G + e % G]
    // the row's entries straight from the CSR (contiguous), zero beyond its length
    const int r0 = A.rp[idof[t]], nz = A.rp[idof[t] + 1] - r0;
    auto col = [&](int k) { return k < nz ? A.ci[r0 + k] : 0; };
    auto val = [&](int k) { return k < nz ? A.v[r0 + k] : 0.0; };
    for (int k = 0; k < COARSE_NNZ; ++k) R.val[((size_t)(k / G) * nit + t) * G + k % G] = val(k);
    for (int q = 0; q < COARSE_NNZ / 2; ++q) {
      const int c0 = col(2 * q), c1 = col(2 * q + 1);
      const double v0 = val(2 * q), v1 = val(2 * q + 1);
      const bool padded = c0 == 0 && c1 == 0 && v0 == 0.0 && v1 == 0.0;
      if (!padded && (c0 % 2 != 0 || c1 != c0 + 1)) {
        bad_pairs = true;
        return;
      }
      if (wide)
        R.meta[(size_t)t * 8 + 2 + q] = (unsigned)(padded ? 0 : c0 / 2);
      else
        R.meta[(size_t)t * 4 + 1 + q / 2] |= (unsigned)(padded ? 0 : c0 / 2) << (16 * (q % 2));
    }
    for (int j = 0; j < nsm; ++j) R.ainv[((size_t)(j / G) * nit + t) * G + j % G] = irow[(size_t)t * nsm + j];
  }
  };
  {
    const int nth = nit >= 16384 ? (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency())) : 1;
    const int chunk = (nit + nth - 1) / nth;
    std::vector<std::thread> th;
    for (int w = 0; w < nth; ++w) th.emplace_back(fill, std::min(nit, w * chunk), std::min(nit, (w + 1) * chunk));
    for (auto& t : th) t.join();
  }
  if (bad_pairs) {
    ctx->err = "lowest-order row whose columns are not facet pairs";
    return HDGMG_EMESH;
  }
  for (int c = L.ncol - 1; c >= 0; --c)
    for (int bb = R.cb[c]; bb < R.cb[c + 1]; ++bb) R.bwd.push_back(bb);
  return HDGMG_OK;
}

// Upload a float or double copy of host values (the V-cycle's storage).
hdgmg_status upload_vals(hdgmg_ctx* ctx, const std::vector<double>& h, const void** out) {
  if (vc_f32(ctx)) {
    float* tf;
    TRY(upload_f32(ctx, &tf, h));
    *out = tf;
  } else {
    double* td;
    TRY(upload(ctx, &td, h));
    *out = td;
  }
  return HDGMG_OK;
}

// Descriptors of the levels handled by the single-workgroup coarse kernel:
// per patch row its padded residual row (from the assembled operator) and its
// row of the patch inverse (host FP64 factorisation), structure-of-arrays.
hdgmg_status build_coarse(hdgmg_ctx* ctx) {
  ctx->Lc = -1;
  if (ctx->opts.coarse_dofs <= 0 || generic_only(ctx)) return HDGMG_OK;
  int Lc = -1, vec = 0, nsmax = 0;
  for (int l = 0; l < ctx->J && l < COARSE_MAX_LEVELS; ++l) {
    const Level& L = ctx->lv[l];
    vec += 3 * 2 * L.nint;
    if (2 * L.nint > ctx->opts.coarse_dofs || vec > COARSE_LDS_DOUBLES) break;
    if (2 * L.max_patch_facets > 32) break;
    nsmax = std::max(nsmax, 2 * L.max_patch_facets);
    Lc = l;
  }
  if (Lc < 0) return HDGMG_OK;
  std::vector<CoarseLevel> desc(Lc + 1);
  int off = COARSE_THREADS + 32;
  for (int l = 0; l <= Lc; ++l) {
    const Level& L = ctx->lv[l];
    DevLevel& D = ctx->cr[l];
    CoarseLevel& C = desc[l];
    std::memset(&C, 0, sizeof(C));
    const int n = 2 * L.nint;
    C.n = n;
    C.off_u = off;
    C.off_g = off + n;
    C.off_r = off + 2 * n;
    off += 3 * n;
    C.u_glob = D.u;
    C.g_glob = D.g;
    C.lds_meta = C.lds_val = C.lds_ainv = -1;
    if (l == 0) continue;
    LevelRecords R;
    TRY(level_records(ctx, l, COARSE_THREADS, R));
    C.ncol = L.ncol;
    C.nitems = R.nit;
    C.ns_max = R.nsm;
    C.nbatch = (int)R.bitem.size() - 1;
    if (C.nbatch > COARSE_MAX_BATCH) {
      ctx->err = "coarse level has too many batches";
      return HDGMG_EMESH;
    }
    int* ti;
    unsigned* tu;
    TRY(upload(ctx, &ti, R.bwd));
    C.bseq_bwd = ti;
    TRY(upload(ctx, &tu, R.meta));
    C.it_meta = (const uint4*)tu;
    TRY(upload(ctx, &ti, R.cb));
    C.cb_ptr = ti;
    TRY(upload(ctx, &ti, R.bitem));
    C.bitem = ti;
    TRY(upload_vals(ctx, R.val, &C.it_val));
    TRY(upload_vals(ctx, R.ainv, &C.it_ainv));
    TRY(upload_vals(ctx, R.rw_val, &C.rw_val));
    TRY(upload(ctx, &ti, R.rw_col));
    C.rw_col = ti;
    const bool f32 = vc_f32(ctx);
    const DevTransfer& T = ctx->tr[l];
    C.R_w = T.Rw;
    C.R_ci = T.Re_ci;
    C.R_v = f32 ? (const void*)T.Re_v32 : (const void*)T.Re_v;
    C.P_w = T.Pw;
    C.P_ci = T.Pe_ci;
    C.P_v = f32 ? (const void*)T.Pe_v32 : (const void*)T.Pe_v;
  }
  // The next level, vectors in memory, for the tabulation of MG_h on it
  // (V-cycle with coarse_dense only; its operator must stay a modest dense
  // matrix)
  ctx->Lt = -1;
  if (ctx->opts.coarse_dense && ctx->opts.cycle == 1 && Lc + 1 < ctx->J && Lc + 1 < COARSE_MAX_LEVELS &&
      2 * ctx->lv[Lc + 1].nint <= DENSE_MAX_N && 2 * ctx->lv[Lc + 1].max_patch_facets <= 32 && Lc >= 1) {
    const int l = Lc + 1;
    const Level& L = ctx->lv[l];
    DevLevel& D = ctx->cr[l];
    CoarseLevel C;
    std::memset(&C, 0, sizeof(C));
    C.n = 2 * L.nint;
    C.off_u = C.off_g = C.off_r = 0;
    C.u_glob = D.u;
    C.g_glob = D.g;
    C.lds_meta = C.lds_val = C.lds_ainv = -1;
    LevelRecords R;
    TRY(level_records(ctx, l, COARSE_THREADS, R));
    C.ncol = L.ncol;
    C.nitems = R.nit;
    C.ns_max = R.nsm;
    C.nbatch = (int)R.bitem.size() - 1;
    if (C.nbatch <= COARSE_MAX_BATCH) {
      int* ti;
      unsigned* tu;
      TRY(upload(ctx, &ti, R.bwd));
      C.bseq_bwd = ti;
      TRY(upload(ctx, &tu, R.meta));
      C.it_meta = (const uint4*)tu;
      TRY(upload(ctx, &ti, R.cb));
      C.cb_ptr = ti;
      TRY(upload(ctx, &ti, R.bitem));
      C.bitem = ti;
      TRY(upload_vals(ctx, R.val, &C.it_val));
      TRY(upload_vals(ctx, R.ainv, &C.it_ainv));
      TRY(upload_vals(ctx, R.rw_val, &C.rw_val));
      TRY(upload(ctx, &ti, R.rw_col));
      C.rw_col = ti;
      const bool f32 = vc_f32(ctx);
      const DevTransfer& T = ctx->tr[l];
      C.R_w = T.Rw;
      C.R_ci = T.Re_ci;
      C.R_v = f32 ? (const void*)T.Re_v32 : (const void*)T.Re_v;
      C.P_w = T.Pw;
      C.P_ci = T.Pe_ci;
      C.P_v = f32 ? (const void*)T.Pe_v32 : (const void*)T.Pe_v;
      desc.push_back(C);
      nsmax = std::max(nsmax, 2 * L.max_patch_facets);
      ctx->Lt = l;
    }
  }
  // Record parts that stay in LDS for the whole kernel, coarsest levels
  // first (they have the most sweeps): residual rows before inverse rows.
  {
    const bool f32 = vc_f32(ctx);
    const size_t G = f32 ? 4 : 2;
    const size_t cap = COARSE_LDS_BYTES - coarse_cycle_static_lds() - 256;
    size_t bytes = ((size_t)off * sizeof(double) + 15) / 16 * 16;
    for (int l = 1; l <= Lc; ++l) {
      CoarseLevel& C = desc[l];
      const size_t nit = C.nitems;
      const size_t mb = 16 * nit, vb = (COARSE_NNZ + G - 1) / G * 16 * nit;
      const size_t ab = (std::max(C.ns_max, 1) + G - 1) / G * 16 * nit;
      if (bytes + mb + vb <= cap) {
        C.lds_meta = (int)bytes;
        C.lds_val = (int)(bytes + mb);
        bytes += mb + vb;
        if (bytes + ab <= cap) {
          C.lds_ainv = (int)bytes;
          bytes += ab;
        }
      }
    }
    off = (int)((bytes + sizeof(double) - 1) / sizeof(double));
    HIPC(prepare_coarse_cycle(nsmax, (size_t)off * sizeof(double), f32 ? 1 : 0));
  }
  std::vector<char> raw(sizeof(CoarseLevel) * desc.size());
  std::memcpy(raw.data(), desc.data(), raw.size());
  char* d;
  TRY(upload(ctx, &d, raw));
  ctx->coarse_desc = (CoarseLevel*)d;
  ctx->coarse_lds = off;
  ctx->coarse_ns = nsmax;
  ctx->Lc = Lc;
  return HDGMG_OK;
}

// Record-based Gauss-Seidel for the launched lowest-order levels that are
// not streamed (see k_gs_records): patch-aligned batches of 256 items.
hdgmg_status build_record_levels(hdgmg_ctx* ctx) {
  for (int l = std::max(ctx->Lc + 1, 1); l < ctx->J; ++l) {
    DevLevel& D = ctx->cr[l];
    D.rec = false;
    const Level& L = ctx->lv[l];
    // records replace the streaming pair (cell apply + patch relaxation) on
    // the launched lowest-order levels (32-bit fields beyond 16-bit facet
    // indices); stream_dofs = 0 keeps the streaming kernels on every level
    if (L.nint > REC_MAX_FACETS || 2 * L.max_patch_facets > 32 || (D.fast && ctx->opts.stream_dofs == 0) || D.fused ||
        generic_only(ctx))
      continue;
    const bool wide = ctx->opts.rec_wide || L.nint > 65535 || 2 * L.nint > (int)REC_DOF_MASK;
    LevelRecords R;
    TRY(level_records(ctx, l, GS_REC_THREADS, R, true, wide));
    D.rwide = wide;
    TRY(upload(ctx, &D.rk, R.meta));
    TRY(upload_vals(ctx, R.val, &D.rv));
    TRY(upload_vals(ctx, R.ainv, &D.ra));
    D.rcb = R.cb;
    D.rnit = R.nit;
    D.rnsm = R.nsm;
    const double ws = vc_f32(ctx) ? 4.0 : 8.0;
    D.rec_bytes.assign(L.ncol, 0.0);
    for (int c = 0; c < L.ncol; ++c) {
      double items = 0.0;  // patch rows, padding excluded
      for (int t = R.bitem[R.cb[c]]; t < R.bitem[R.cb[c + 1]]; ++t)
        items += wide ? R.meta[(size_t)t * 8 + 1] != REC_PAD : (R.meta[(size_t)t * 4] >> REC_LOC_SHIFT) != REC_PAD;
      D.rec_bytes[c] = items * ((wide ? 32.0 : 16.0) + ws * (COARSE_NNZ + R.nsm) + 8.0 * (COARSE_NNZ + 2));
    }
    D.rec = true;
  }
  return HDGMG_OK;
}

// Element data of a level for the local solver kernels.  wind: with the
// level's wind coefficients (order-k: ctx->wcoef; lowest order: D.wcoef).
// Tabulate u = MG_h(Lc, g, 0) (Alg. 1 on levels 0..Lc, the V-cycle's sweep
// count there) as a dense matrix: the single-workgroup kernel applied to the
// columns of the identity, a workgroup per column, then stored row-major in
// the V-cycle's storage precision.  The V-cycle (q = 1) enters level Lc
// from a zero iterate once per application, so one GEMV replaces the
// kernel's sequence of dependent colour phases by a bandwidth-bound read.
hdgmg_status build_dense_coarse(hdgmg_ctx* ctx) {
  ctx->dense_on = false;
  ctx->dense_M = nullptr;
  if (!ctx->opts.coarse_dense || ctx->opts.cycle != 1 || ctx->Lc < 1) return HDGMG_OK;
  // the level whose MG_h is tabulated: Lc + 1 (vectors in memory) when the
  // coarse kernel describes it, else Lc
  const int Ld = ctx->Lt >= 0 ? ctx->Lt : ctx->Lc;
  const bool gtop = ctx->Lt >= 0;
  const int n = 2 * ctx->lv[Ld].nint;
  int m = ctx->opts.m_smooth;
  for (int l = ctx->J - 1; l > Ld; --l) m *= ctx->opts.vcycle_growth;
  const bool f32 = vc_f32(ctx);
  const size_t nn = (size_t)n * n;
  double* G = (double*)dmalloc(ctx, nn * sizeof(double));
  double* U = (double*)dmalloc(ctx, nn * sizeof(double));
  double* Rw = gtop ? (double*)dmalloc(ctx, nn * sizeof(double)) : nullptr;
  if (!G || !U || (gtop && !Rw)) {
    dfree(ctx, G);
    dfree(ctx, U);
    dfree(ctx, Rw);
    ctx->err = "device allocation for the dense coarse operator failed";
    return HDGMG_ENOMEM;
  }
  hipStream_t st = ctx->st;
  launch_identity(st, n, G);
  launch_fill(st, (long)nn, 0.0, U);
  launch_coarse_cycle_batch(st, ctx->coarse_desc, Ld, m, ctx->opts.vcycle_growth, 1,
                            f32 ? (const void*)ctx->coarse_inv32 : (const void*)ctx->coarse_inv, ctx->n0,
                            ctx->coarse_ns, ctx->coarse_lds, f32 ? 1 : 0, n, G, U, Rw, n);
  hdgmg_status s = HDGMG_OK;
  const int ld = (n + 3) / 4 * 4;  // rows start on 16-byte boundaries
  if (f32) {
    float* M = nullptr;
    s = dalloc(ctx, &M, (size_t)n * ld);
    if (!s) launch_transpose_to<float>(st, n, ld, U, M);
    ctx->dense_M = M;
  } else {
    double* M = nullptr;
    s = dalloc(ctx, &M, (size_t)n * ld);
    if (!s) launch_transpose_to<double>(st, n, ld, U, M);
    ctx->dense_M = M;
  }
  ctx->dense_ld = ld;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(ctx, G);
  dfree(ctx, U);
  dfree(ctx, Rw);
  if (s) return s;
  if (e != hipSuccess) {
    ctx->err = std::string("HIP error: ") + hipGetErrorString(e) + " in the coarse tabulation";
    return HDGMG_EHIP;
  }
  ctx->dense_n = n;
  ctx->dense_m = m;
  ctx->dense_level = Ld;
  ctx->dense_on = true;
  return HDGMG_OK;
}

ElemLevel elem_level(const hdgmg_ctx* ctx, const DevLevel& D, bool order_k, bool wind) {
  ElemLevel E;
  E.Q = order_k ? ctx->Q : ctx->Q0;
  E.CT = nullptr;
  E.wcoef = nullptr;
  E.na = dims_of(E.Q.k).na;
  if (wind && ctx->has_wind) {
    E.CT = order_k ? ctx->CTk : ctx->CT0;
    E.wcoef = order_k ? ctx->wcoef : D.wcoef;
  }
  E.X = D.X;
  E.cells = D.cells;
  E.nu = D.nu;
  E.nu_per_cell = 1;
  E.beta = ctx->beta;
  E.eps_inv = ctx->gamma;
  E.cell_dofs = D.cell_dofs;
  E.m = D.m;
  E.bdl = order_k && ctx->has_bd ? ctx->bdl : nullptr;
  E.S = D.S;
  E.fac = order_k ? ctx->fac : nullptr;
  E.nc = D.nc;
  E.transpose = E.CT && ctx->opts.transpose ? 1 : 0;
  E.oflag = D.oflag;
  const bool nw = order_k && E.CT && ctx->has_newton;
  E.nw_lam = nw ? ctx->nw_lam : nullptr;
  E.nw_load = nw ? ctx->nw_load : nullptr;
  return E;
}

// Local solver kernels over all cells of a level in workspace-sized batches.
hdgmg_status batched(hdgmg_ctx* ctx, DevLevel& D, const ElemLevel& E, int mode, const double* f,
                     const double* lam, const double* p0, double* out1, double* out2, const double* f2 = nullptr,
                     const double* lam2 = nullptr) {
  const int nc = D.nc;
  long per = element_ws_size(E.Q.k);
  long batch = std::max<long>(1, std::min<long>(nc, (long)(ctx->ws_bytes / (per * sizeof(double)))));
  HIPC(hipMemsetAsync(ctx->status, 0, sizeof(int), ctx->st));
  if (mode == EL_CONDENSE && condense_wave_supported(E.Q.k)) {
    launch_condense_wave(ctx->st, E, out1, ctx->status);
    HIPC(hipGetLastError());
    return check_status(ctx, "condensation");
  }
  for (long c0 = 0; c0 < nc; c0 += batch) {
    int nb = (int)std::min<long>(batch, nc - c0);
    if (mode == EL_CONDENSE)
      launch_condense(ctx->st, E, (int)c0, nb, ctx->ws, out1, ctx->status);
    else if (mode == EL_LOAD)
      launch_load(ctx->st, E, (int)c0, nb, f, ctx->ws, out1, ctx->status);
    else if (mode == EL_GRADNU)
      launch_gradnu(ctx->st, E, (int)c0, nb, f, lam, f2, lam2, ctx->ws, out1, ctx->status);
    else if (mode == EL_POSTPROCESS)
      launch_postprocess(ctx->st, E, (int)c0, nb, f, lam, ctx->ws, out1, ctx->status);
    else
      launch_recover(ctx->st, E, (int)c0, nb, f, lam, p0, ctx->ws, out1, out2, ctx->status);
    HIPC(hipGetLastError());
  }
  return check_status(ctx, mode == EL_CONDENSE ? "condensation"
                           : mode == EL_LOAD   ? "load"
                           : mode == EL_GRADNU ? "viscosity gradient"
                           : mode == EL_POSTPROCESS ? "post-processing"
                                               : "recovery");
}

// Order-k blocks and patch factors, lowest-order blocks (closed form, or
// the generic k = 0 condensation with the level's RT0 wind), transfers and
// coarse-level data.
hdgmg_status assemble_levels(hdgmg_ctx* ctx) {
  TRY(batched(ctx, ctx->K, elem_level(ctx, ctx->K, true, true), EL_CONDENSE, nullptr, nullptr, nullptr, ctx->K.S,
              nullptr));
  TRY(patch_inverses(ctx, ctx->K));
  TRY(pack_fast(ctx, ctx->K));
  TRY(make_f32(ctx, ctx->K, true));
  TRY(pack_fused(ctx, ctx->K));
  if (ctx->k > 0) {
    DevLevel& K = ctx->K;
    const size_t n0r = (size_t)std::max(K.nc, 1) * 6 * K.nK;
    TRY(dalloc(ctx, &K.y0K, (size_t)std::max(K.nc, 1) * 6));
    if (vc_f32(ctx)) {
      TRY(dalloc(ctx, &K.S0_32, n0r));
      launch_pack_mode0_rows<float>(ctx->st, K.nc, K.m, K.S, K.S0_32);
    } else {
      TRY(dalloc(ctx, &K.S0, n0r));
      launch_pack_mode0_rows<double>(ctx->st, K.nc, K.m, K.S, K.S0);
    }
    HIPC(hipGetLastError());
  }
  ctx->hostB.assign(ctx->J, {});
  std::vector<std::vector<double>> nu;
  level_viscosities(ctx->lv, ctx->nu_fine, nu);
  for (int l = 0; l < ctx->J; ++l) {
    DevLevel& D = ctx->cr[l];
    if (ctx->has_wind) {
      TRY(batched(ctx, D, elem_level(ctx, D, false, true), EL_CONDENSE, nullptr, nullptr, nullptr, D.S, nullptr));
      ctx->hostB[l].resize((size_t)D.nc * 36);
      HIPC(hipMemcpyAsync(ctx->hostB[l].data(), D.S, ctx->hostB[l].size() * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->st));
      HIPC(hipStreamSynchronize(ctx->st));
    } else {
      launch_cr_blocks(ctx->st, D.X, D.cells, D.nc, D.nu, ctx->beta, ctx->gamma, D.S);
      HIPC(hipGetLastError());
      host_cr_blocks(ctx->lv[l], nu[l], ctx->beta, ctx->gamma, ctx->hostB[l]);
    }
  }
  TRY(build_transfers(ctx));
  for (int l = 1; l < ctx->J; ++l) {
    DevLevel& D = ctx->cr[l];
    TRY(patch_inverses(ctx, D));
    TRY(pack_fast(ctx, D));
    TRY(make_f32(ctx, D));
    TRY(pack_fused(ctx, D));
  }
  TRY(build_coarse(ctx));
  TRY(build_dense_coarse(ctx));
  TRY(build_record_levels(ctx));
  HIPC(hipStreamSynchronize(ctx->st));
  return HDGMG_OK;
}

}  // namespace

// Batches over several identical contexts: right-hand side i goes to
// context i % nctx; each context works through its share on its own stream
// in a host thread of its own, so that the contexts' latency-bound V-cycles
// overlap on the device.
namespace {
hdgmg_status batch_check(hdgmg_ctx* const* ctxs, int nctx, int nrhs) {
  if (!ctxs || nctx < 1 || nrhs < 0) return HDGMG_EINVAL;
  for (int c = 0; c < nctx; ++c) {
    if (!ctxs[c]) return HDGMG_EINVAL;
    if (!ctxs[c]->assembled) {
      ctxs[c]->err = "batch solve before hdgmg_assemble";
      return HDGMG_ESTATE;
    }
    if (ctxs[c]->K.nc != ctxs[0]->K.nc || ctxs[c]->K.ndof != ctxs[0]->K.ndof || ctxs[c]->Q.nq != ctxs[0]->Q.nq) {
      ctxs[c]->err = "batch contexts of different sizes";
      return HDGMG_EINVAL;
    }
    for (int d = 0; d < c; ++d)
      if (ctxs[d] == ctxs[c]) {
        ctxs[c]->err = "a context appears twice in a batch";
        return HDGMG_EINVAL;
      }
  }
  return HDGMG_OK;
}

template <class F>
hdgmg_status batch_run(hdgmg_ctx* const* ctxs, int nctx, int nrhs, F&& one) {
  std::vector<hdgmg_status> st(nctx, HDGMG_OK);
  auto work = [&](int c) {
    for (int i = c; i < nrhs; i += nctx) {
      hdgmg_status s = one(ctxs[c], i);
      if (s < 0) {
        st[c] = s;
        return;
      }
      if (s > st[c]) st[c] = s;
    }
  };
  if (nctx == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int c = 0; c < nctx; ++c) th.emplace_back(work, c);
    for (auto& t : th) t.join();
  }
  hdgmg_status r = HDGMG_OK;
  for (hdgmg_status s : st)
    if (s < 0) return s;
    else if (s > r) r = s;
  return r;
}
}  // namespace

extern "C" {

void hdgmg_default_opts(hdgmg_opts* o) {
  if (!o) return;
  o->m_relax = 1;
  o->m_smooth = 1;
  o->cycle = 1;
  o->vcycle_growth = 2;
  o->rtol = 1e-8;
  o->atol = 1e-10;
  o->max_it = 500;
  o->uzawa_max = 50;
  o->uzawa_tol = 1e-10;
  o->coarse_dofs = 2048;
  o->stream_dofs = 65536;
  o->vcycle_precision = 0;
  o->oseen = 0;
  o->restart = 50;
  o->transpose = 0;
  o->coarse_dense = 1;
  o->rec_wide = 0;
  o->smoother = 0;
  o->additive = 0;
  o->patch_relax = 0;
  o->patch_smooth = 0;
  o->fused_phase = 1;
}

const char* hdgmg_last_error(const hdgmg_ctx* ctx) {
  if (ctx && ctx->d3) return d3_error(ctx->d3);
  return ctx ? ctx->err.c_str() : g_setup_error.c_str();
}

void hdgmg_destroy(hdgmg_ctx* ctx) {
  if (!ctx) return;
  if (ctx->d3) {
    d3_destroy(ctx->d3);
    delete ctx;
    return;
  }
  if (ctx->st) (void)hipStreamSynchronize(ctx->st);
  drop_graph(ctx);
  for (auto& T : ctx->timers) kt_clear(T);
  for (auto& a : ctx->asm_allocs) dfree(ctx, a.first);
  for (void* p : ctx->allocs) dfree(ctx, p);
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  delete ctx;
}

hdgmg_status hdgmg_setup(const hdgmg_mesh* mesh, int k, double beta, const double* nu, int nu_len,
                         double gamma, const hdgmg_opts* opts, void* stream, hdgmg_alloc_fn alloc_fn,
                         hdgmg_free_fn free_fn, void* alloc_ctx, hdgmg_ctx** out) {
  if (out) *out = nullptr;
  g_setup_error.clear();
  if (!mesh || !out || !nu) {
    g_setup_error = "null argument";
    return HDGMG_EINVAL;
  }
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) {
    g_setup_error = "give both allocator callbacks or neither";
    return HDGMG_EINVAL;
  }
  if (mesh->dim == 3 && mesh->coords && mesh->cells) {
    if (mesh->n_outflow != 0) {
      g_setup_error = "do-nothing facets are provided on triangular meshes only";
      return HDGMG_EINVAL;
    }
    if (!(beta >= 0) || !(gamma > 0)) {
      g_setup_error = "need beta >= 0, gamma > 0";
      return HDGMG_EINVAL;
    }
    for (int i = 0; i < nu_len; ++i)
      if (!(nu[i] > 0) || !std::isfinite(nu[i])) {
        g_setup_error = "nu must be positive and finite";
        return HDGMG_EINVAL;
      }
    Ctx3* c3 = nullptr;
    hdgmg_status s3 = d3_setup(mesh, k, beta, nu, nu_len, gamma, opts, stream, alloc_fn, free_fn, alloc_ctx, &c3,
                               g_setup_error);
    if (s3 != HDGMG_OK) return s3;
    hdgmg_ctx* ctx = new hdgmg_ctx();
    ctx->d3 = c3;
    ctx->k = k;
    *out = ctx;
    return HDGMG_OK;
  }
  if (mesh->dim != 2 || mesh->n_vertices < 3 || mesh->n_cells < 1 || !mesh->coords || !mesh->cells ||
      mesh->n_refine < 0 || mesh->n_refine > 12) {
    g_setup_error = "mesh must be 2D (or 3D) with >= 1 cell and 0 <= n_refine <= 12";
    return HDGMG_EMESH;
  }
  if (k < 0 || k > KMAX || !(beta >= 0) || !(gamma > 0)) {
    g_setup_error = "need 0 <= k <= 4, beta >= 0, gamma > 0";
    return HDGMG_EINVAL;
  }
  long nfine = (long)mesh->n_cells << (2 * mesh->n_refine);
  if (nu_len != 1 && nu_len != nfine) {
    g_setup_error = "nu must have 1 or n_fine_cells entries";
    return HDGMG_EINVAL;
  }
  for (int i = 0; i < nu_len; ++i)
    if (!(nu[i] > 0) || !std::isfinite(nu[i])) {
      g_setup_error = "nu must be positive and finite";
      return HDGMG_EINVAL;
    }
  hdgmg_ctx* ctx = new hdgmg_ctx();
  ctx->alloc_fn = alloc_fn;
  ctx->free_fn = free_fn;
  ctx->alloc_ctx = alloc_ctx;
  ctx->k = k;
  ctx->beta = beta;
  ctx->gamma = gamma;
  hdgmg_default_opts(&ctx->opts);
  if (opts) ctx->opts = *opts;
  if (ctx->opts.m_relax < 0 || ctx->opts.m_smooth < 1 || ctx->opts.cycle < 1 || ctx->opts.cycle > 2 ||
      ctx->opts.vcycle_growth < 1 || ctx->opts.max_it < 1 || ctx->opts.uzawa_max < 1 ||
      ctx->opts.uzawa_max > HDGMG_MAX_UZAWA || !(ctx->opts.rtol >= 0) || !(ctx->opts.atol >= 0) ||
      ctx->opts.vcycle_precision < 0 || ctx->opts.vcycle_precision > 2 || ctx->opts.oseen < 0 ||
      ctx->opts.oseen > 1 || ctx->opts.restart < 1 || ctx->opts.restart > 64 || ctx->opts.transpose < 0 ||
      ctx->opts.transpose > 1 || (ctx->opts.transpose && !ctx->opts.oseen) || ctx->opts.coarse_dense < 0 ||
      ctx->opts.coarse_dense > 1 || ctx->opts.rec_wide < 0 || ctx->opts.rec_wide > 1 || ctx->opts.smoother < 0 ||
      ctx->opts.smoother > 1 || ctx->opts.additive < 0 || ctx->opts.additive > 1 || ctx->opts.patch_relax < 0 ||
      ctx->opts.patch_relax > 2 || ctx->opts.patch_smooth < 0 || ctx->opts.patch_smooth > 2 ||
      ctx->opts.fused_phase < 0 || ctx->opts.fused_phase > 1) {
    g_setup_error = "invalid options";
    delete ctx;
    return HDGMG_EINVAL;
  }
  ctx->st = (hipStream_t)stream;
  if (!ctx->st) {
    // a stream of our own (default priority); the legacy null stream cannot
    // be captured into a graph
    if (hipStreamCreate(&ctx->own) != hipSuccess) {
      g_setup_error = "hipStreamCreate failed";
      delete ctx;
      return HDGMG_EHIP;
    }
    ctx->st = ctx->own;
  }
  // address of the no-allocation scratch on this device (once per device)
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAX_DEVICES) {
      g_setup_error = "hipGetDevice failed or device index out of range";
      if (ctx->own) (void)hipStreamDestroy(ctx->own);
      delete ctx;
      return HDGMG_EHIP;
    }
    ctx->dev = dev;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
      void* ptr = nullptr;
      hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        g_setup_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        if (ctx->own) (void)hipStreamDestroy(ctx->own);
        delete ctx;
        return HDGMG_EHIP;
      }
      g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
  }
  ctx->J = mesh->n_refine + 1;
  ctx->lv.resize(ctx->J);
  Level& L0 = ctx->lv[0];
  L0.nv = mesh->n_vertices;
  L0.nc = mesh->n_cells;
  L0.X.assign(mesh->coords, mesh->coords + 2 * (size_t)L0.nv);
  L0.cells.assign(mesh->cells, mesh->cells + 3 * (size_t)L0.nc);
  if (mesh->n_outflow < 0 || (mesh->n_outflow > 0 && !mesh->outflow)) {
    g_setup_error = "n_outflow < 0, or outflow pairs missing";
    delete ctx;
    return HDGMG_EINVAL;
  }
  for (int i = 0; i < mesh->n_outflow; ++i) L0.outflow_in.push_back({mesh->outflow[2 * i], mesh->outflow[2 * i + 1]});
  ctx->has_outflow = mesh->n_outflow > 0;
  std::string e = build_level(L0);
  for (int l = 1; l < ctx->J && e.empty(); ++l) {
    refine(ctx->lv[l - 1], ctx->lv[l]);
    e = build_level(ctx->lv[l]);
  }
  if (!e.empty()) {
    g_setup_error = "mesh: " + e;
    delete ctx;
    return HDGMG_EMESH;
  }
  // patches: vertex (default) or edge (facet) patches, opts.patch_smooth on
  // the lowest-order levels, opts.patch_relax on the order-k level
  const bool erelax = ctx->opts.patch_relax == 2, esmooth = ctx->opts.patch_smooth == 2;
  for (int l = 0; l < ctx->J; ++l) {
    if (l == ctx->J - 1 ? erelax : esmooth)
      build_facet_patches(ctx->lv[l]);
    else
      build_patches(ctx->lv[l]);
  }
  if (ctx->lv.back().max_patch_facets * 2 * (k + 1) > GS_MAX_NS) {
    g_setup_error = "mesh: a vertex patch exceeds " + std::to_string(GS_MAX_NS) + " unknowns";
    delete ctx;
    return HDGMG_EMESH;
  }
  ctx->avg.resize(ctx->J);
  for (int l = 1; l < ctx->J; ++l) build_averaging(ctx->lv[l - 1], ctx->lv[l], ctx->avg[l]);
  const Level& LF = ctx->lv.back();
  ctx->nu_fine.assign(LF.nc, nu[0]);
  if (nu_len > 1) ctx->nu_fine.assign(nu, nu + nu_len);
  ctx->Q = make_tables(k);
  hdgmg_status s = HDGMG_OK;
  auto fail = [&](hdgmg_status st) {
    g_setup_error = ctx->err;
    hdgmg_destroy(ctx);
    return st;
  };
  if ((s = upload_level(ctx, LF, k + 1, ctx->K))) return fail(s);
  if (ctx->opts.fused_phase && (s = setup_fused(ctx, LF, ctx->K))) return fail(s);
  // per-colour byte model of the order-k relaxation, from its own patches
  ctx->relax_bytes.resize(LF.ncol);
  for (int c = 0; c < LF.ncol; ++c) ctx->relax_bytes[c] = gs_phase_bytes(LF, k + 1, c);
  if (erelax != esmooth) {
    // the finest lowest-order level smooths on the other patch type
    if (esmooth)
      build_facet_patches(ctx->lv.back());
    else
      build_patches(ctx->lv.back());
  }
  if ((s = upload(ctx, &ctx->K.nu, ctx->nu_fine))) return fail(s);
  ctx->cr.resize(ctx->J);
  for (int l = 0; l < ctx->J; ++l) {
    if ((s = upload_level(ctx, ctx->lv[l], 1, ctx->cr[l]))) return fail(s);
    if (ctx->opts.fused_phase && (s = setup_fused(ctx, ctx->lv[l], ctx->cr[l]))) return fail(s);
  }
  {
    std::vector<std::vector<double>> nul;
    level_viscosities(ctx->lv, ctx->nu_fine, nul);
    for (int l = 0; l < ctx->J; ++l)
      if ((s = upload(ctx, &ctx->cr[l].nu, nul[l]))) return fail(s);
  }
  ctx->Q0 = make_tables(0);
  if (ctx->opts.oseen) {
    // convection rules, wind storage, FGMRES basis
    std::vector<ConvTables> ct = {make_conv_tables(k)}, ct0 = {make_conv_tables(0)};
    if ((s = upload(ctx, &ctx->CTk, ct))) return fail(s);
    if ((s = upload(ctx, &ctx->CT0, ct0))) return fail(s);
    if ((s = dalloc(ctx, &ctx->wcoef, (size_t)LF.nc * dims_of(k).na))) return fail(s);
    for (auto& D : ctx->cr) {
      if ((s = dalloc(ctx, &D.flux, (size_t)std::max(D.nint, 1)))) return fail(s);
      if ((s = dalloc(ctx, &D.wcoef, (size_t)D.nc * 3))) return fail(s);
    }
    const size_t nv = (size_t)std::max<long>(ctx->K.ndof, 1);
    if ((s = dalloc(ctx, &ctx->gm_V, nv * (ctx->opts.restart + 1)))) return fail(s);
    if ((s = dalloc(ctx, &ctx->gm_Z, nv * ctx->opts.restart))) return fail(s);
    if ((s = dalloc(ctx, &ctx->gm_h, 4 * 128))) return fail(s);
    if ((s = dalloc(ctx, &ctx->gm_y, 128))) return fail(s);
    if ((s = dalloc(ctx, &ctx->gm_part, (size_t)(ctx->opts.restart + 1) * RED_BLOCKS))) return fail(s);
  }
  {
    // boundary facets of the finest level in facet order, and per cell side
    std::vector<int> num(LF.nf, -1);
    for (int f = 0; f < LF.nf; ++f)
      if (LF.int_id[f] < 0) {
        num[f] = (int)ctx->bfacets.size();
        ctx->bfacets.push_back(f);
      }
    std::vector<int> cbf(3 * (size_t)LF.nc);
    for (int c = 0; c < LF.nc; ++c)
      for (int i = 0; i < 3; ++i) cbf[3 * c + i] = num[LF.cell_facets[3 * c + i]];
    if ((s = upload(ctx, &ctx->cbf, cbf))) return fail(s);
    if ((s = dalloc(ctx, &ctx->bdl, (size_t)LF.nc * 3 * 2 * (k + 1)))) return fail(s);
  }
  const long n = ctx->K.ndof;
  double** vecs[] = {&ctx->x, &ctx->r, &ctx->r_old, &ctx->z, &ctx->p, &ctx->q, &ctx->b, &ctx->gvec, &ctx->lam};
  for (double** v : vecs)
    if ((s = dalloc(ctx, v, (size_t)std::max<long>(n, 1)))) return fail(s);
  if ((s = dalloc(ctx, &ctx->p0, (size_t)LF.nc))) return fail(s);
  if ((s = dalloc(ctx, &ctx->sc, SC_N))) return fail(s);
  if ((s = dalloc(ctx, &ctx->part, 4 * RED_BLOCKS))) return fail(s);
  if ((s = dalloc(ctx, &ctx->gK, (size_t)LF.nc * 6 * (k + 1)))) return fail(s);
  if ((s = dalloc(ctx, &ctx->status, 1))) return fail(s);
  if ((s = dalloc(ctx, &ctx->statebuf, (size_t)(n + LF.nc)))) return fail(s);
  if ((s = dalloc(ctx, &ctx->fac, (size_t)LF.nc * element_fac_size(k)))) return fail(s);
  // Uzawa geometry: per interior facet and side sigma|F|, per cell sigma|F| and |K|
  std::vector<double> fdiv(2 * (size_t)LF.nint), cdiv(3 * (size_t)LF.nc), area(LF.area);
  for (int i = 0; i < LF.nint; ++i) {
    int f = LF.int_facet[i];
    for (int sd = 0; sd < 2; ++sd) {
      int c = LF.facet_cells[2 * f + sd], li = LF.facet_loc[2 * f + sd];
      fdiv[2 * i + sd] = c < 0 ? 0.0 : LF.sigma[3 * c + li] * LF.len[f];  // one side on a do-nothing facet
    }
  }
  std::vector<double> bdiv(3 * (size_t)LF.nc);
  for (int c = 0; c < LF.nc; ++c)
    for (int i = 0; i < 3; ++i) {
      int f = LF.cell_facets[3 * c + i];
      cdiv[3 * c + i] = LF.int_id[f] >= 0 ? LF.sigma[3 * c + i] * LF.len[f] : 0.0;
      bdiv[3 * c + i] = LF.int_id[f] < 0 ? LF.sigma[3 * c + i] * LF.len[f] : 0.0;
    }
  if ((s = upload(ctx, &ctx->fdiv, fdiv))) return fail(s);
  if ((s = upload(ctx, &ctx->cdiv, cdiv))) return fail(s);
  if ((s = upload(ctx, &ctx->bdiv, bdiv))) return fail(s);
  if ((s = dalloc(ctx, &ctx->cflux, (size_t)LF.nc))) return fail(s);
  if ((s = upload(ctx, &ctx->area, area))) return fail(s);
  // workspace: element batches and patch factorisations share it
  size_t need = 0;
  for (auto* D : {&ctx->K})
    need = std::max(need, ((size_t)D->max_ns * D->max_ns + D->max_ns) * D->npatch * sizeof(double));
  for (auto& D : ctx->cr)
    need = std::max(need, ((size_t)D.max_ns * D.max_ns + D.max_ns) * D.npatch * sizeof(double));
  // the local solves run a thread per cell, so a launch should cover as many
  // cells as the workspace allows (all of them up to 6 GiB)
  const size_t per_cell = (size_t)element_ws_size(k) * sizeof(double);
  size_t el = per_cell * std::min<size_t>(LF.nc, std::max<size_t>(1, (6ull << 30) / per_cell));
  need = std::max(need, el);
  ctx->ws_bytes = need;
  double* ws = nullptr;
  if ((s = dalloc(ctx, &ws, need / sizeof(double) + 1))) return fail(s);
  ctx->ws = ws;
  hipError_t he = hipStreamSynchronize(ctx->st);
  if (he != hipSuccess) {
    ctx->err = std::string("HIP error: ") + hipGetErrorString(he);
    return fail(HDGMG_EHIP);
  }
  // algorithmic byte models of the timed kernel classes
  {
    const int m = k + 1, nK = 6 * m;
    ctx->smooth_bytes.resize(ctx->J);
    for (int l = 0; l < ctx->J; ++l) {
      ctx->smooth_bytes[l].resize(ctx->lv[l].ncol);
      for (int c = 0; c < ctx->lv[l].ncol; ++c) ctx->smooth_bytes[l][c] = gs_phase_bytes(ctx->lv[l], 1, c);
    }
    // apply: every cell block once, the cell vectors it gathers, y written
    ctx->apply_bytes = ((double)LF.nc * nK * nK + (double)LF.nc * nK + (double)ctx->K.ndof) * 8.0;
  }
  *out = ctx;
  return HDGMG_OK;
}

hdgmg_status hdgmg_assemble(hdgmg_ctx* ctx) {
  if (ctx && ctx->d3) return d3_assemble(ctx->d3);
  if (!ctx) return HDGMG_EINVAL;
  ctx->assembled = false;
  drop_graph(ctx);
  HIPC(hipStreamSynchronize(ctx->st));
  for (auto& a : ctx->asm_allocs) {
    dfree(ctx, a.first);
    ctx->bytes -= a.second;
  }
  ctx->asm_allocs.clear();
  ctx->in_assemble = true;
  hdgmg_status s = assemble_levels(ctx);
  ctx->in_assemble = false;
  if (s != HDGMG_OK) return s;
  // algorithmic bytes of one MG_hp application (sum over its launches,
  // operators in the storage precision the V-cycle reads)
  {
    const auto& o = ctx->opts;
    double v = 0.0;
    // (the first colour phase from a zero iterate has no cell apply)
    if (ctx->k > 0) {
      const DevLevel& K = ctx->K;
      double sw = 0.0;
      for (int c = 0; c < (int)K.colour_ptr.size() - 1; ++c) sw += phase_bytes(ctx, K, -1, c);
      // the residual: its mode-0 rows (the six rows' words, x once per cell
      // facet, the rows' products written and read, b's and g0's entries)
      const double res = o.additive ? 0.0
                                    : (vc_f32(ctx) ? 4.0 : 8.0) * K.nc * 6.0 * K.nK +
                                          8.0 * (K.nc * (double)K.nK + 3.0 * K.nc * 6.0 + 2.0 * 2.0 * K.nint);
      const double first = K.fused ? K.bytes_fused_vc[0] - K.bytes_relax_vc[0] : K.fast ? K.bytes_cell_vc : 0.0;
      v += 2.0 * o.m_relax * sw - first + res;  // sweeps, residual
      v += 2.0 * K.ndof * 8.0;                                                 // the mode-0 transfers
    }
    double visits = 1.0, m_l = o.m_smooth;
    bool dense_done = false;
    for (int l = ctx->J - 1; l >= 1; --l) {
      if (ctx->dense_on && l == ctx->dense_level) {
        // levels 0..Lc: one read of the tabulated operator
        v += (double)ctx->dense_n * ctx->dense_n * (o.vcycle_precision >= 1 ? 4.0 : 8.0) + 2.0 * ctx->dense_n * 8.0;
        dense_done = true;
        break;
      }
      const DevLevel& D = ctx->cr[l];
      double sw = 0.0;
      for (int c = 0; c < (int)D.colour_ptr.size() - 1; ++c) sw += phase_bytes(ctx, D, l, c);
      const double ws = D.f32 ? 4.0 : 8.0;
      double res = D.fast ? D.bytes_cell_vc + D.bytes_sum
                          : (double)D.nc * 36 * ws + (D.nc * 6.0 + 2.0 * D.ndof) * 8.0;
      double trn = 2.0 * (ctx->tr[l].nnz * (4.0 + ws) + (ctx->tr[l].nfine + ctx->tr[l].ncoarse) * 8.0);
      const double zero_starts = l == ctx->J - 1 ? 1.0 : visits / o.cycle;
      const double first = D.fused ? D.bytes_fused_vc[0] - D.bytes_relax_vc[0] : D.fast && !D.rec ? D.bytes_cell_vc : 0.0;
      v += visits * (2.0 * m_l * sw + res + trn) - zero_starts * first;
      visits *= o.cycle;
      m_l *= o.vcycle_growth;
    }
    if (!dense_done) v += visits * (double)ctx->n0 * ctx->n0 * (o.vcycle_precision >= 1 ? 4.0 : 8.0);
    ctx->vcycle_bytes = v;
    // compulsory bytes of the same V-cycle
    auto tri = [](double n) { return n * (n + 1.0) / 2.0; };
    auto sweep_c = [&](const Level& L, int m, double wb) {
      double pb = 0.0;
      for (size_t q = 0; q + 1 < L.patch_facet_ptr.size(); ++q)
        pb += tri(2.0 * m * (L.patch_facet_ptr[q + 1] - L.patch_facet_ptr[q]));
      return (L.nc * tri(6.0 * m) + pb) * wb + 3.0 * 8.0 * 2.0 * m * L.nint;
    };
    auto res_c = [&](const Level& L, int m, double wb) {
      return L.nc * tri(6.0 * m) * wb + 3.0 * 8.0 * 2.0 * m * L.nint;
    };
    const double wk = o.vcycle_precision == 0 ? 8.0 : (o.vcycle_precision == 2 && ctx->K.f16 ? 2.0 : 4.0);
    const double wl = o.vcycle_precision == 0 ? 8.0 : 4.0;
    double vc = 0.0;
    if (ctx->k > 0) {
      // the order-k residual enters MG_hp only through its mode-0 rows
      const Level& LK = ctx->lv[ctx->J - 1];
      const double w0 = vc_f32(ctx) ? 4.0 : 8.0;
      vc += 2.0 * o.m_relax * sweep_c(LK, ctx->k + 1, wk) +
            (o.additive ? 0.0 : LK.nc * 6.0 * 6.0 * (ctx->k + 1) * w0 + 3.0 * 8.0 * 2.0 * LK.nint);
    }
    double vis = 1.0, ml = o.m_smooth;
    for (int l = ctx->J - 1; l >= 1; --l) {
      const Level& L = ctx->lv[l];
      vc += vis * (2.0 * ml * sweep_c(L, 1, wl) + res_c(L, 1, wl) +
                   2.0 * (ctx->tr[l].nnz * (4.0 + wl) + (ctx->tr[l].nfine + ctx->tr[l].ncoarse) * 8.0));
      vis *= o.cycle;
      ml *= o.vcycle_growth;
    }
    vc += vis * tri((double)ctx->n0) * wl;
    ctx->vcycle_compulsory = vc;
  }
  ctx->assembled = true;
  return HDGMG_OK;
}

hdgmg_status hdgmg_rhs(hdgmg_ctx* ctx, const double* f_qp, double* g) {
  if (ctx && ctx->d3) return f_qp && g ? d3_rhs(ctx->d3, f_qp, g) : HDGMG_EINVAL;
  if (!ctx || !f_qp || !g) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_rhs before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  TRY(batched(ctx, ctx->K, elem_level(ctx, ctx->K, true, true), EL_LOAD, f_qp, nullptr, nullptr, ctx->gK, nullptr));
  launch_gather_cells(ctx->st, ctx->K.view(), ctx->gK, g);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(ctx->st));
  return HDGMG_OK;
}

hdgmg_status hdgmg_apply(hdgmg_ctx* ctx, const double* x, double* y) {
  if (ctx && ctx->d3) return x && y ? d3_apply(ctx->d3, x, y) : HDGMG_EINVAL;
  if (!ctx || !x || !y) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_apply before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  apply_k(ctx, x, y, 1.0, nullptr);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(ctx->st));
  return HDGMG_OK;
}

hdgmg_status hdgmg_precondition(hdgmg_ctx* ctx, const double* r, double* z) {
  if (ctx && ctx->d3) return r && z ? d3_precondition(ctx->d3, r, z) : HDGMG_EINVAL;
  if (!ctx || !r || !z) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_precondition before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  mg_hp(ctx, r, z);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(ctx->st));
  return HDGMG_OK;
}

hdgmg_status hdgmg_inner_solve(hdgmg_ctx* ctx, const double* b, double* x, int* its, double* rel_res) {
  if (ctx && ctx->d3) return b && x ? d3_inner_solve(ctx->d3, b, x, its, rel_res, nullptr, nullptr) : HDGMG_EINVAL;
  if (!ctx || !b || !x) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_inner_solve before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  hdgmg_status s;
  if (ctx->opts.oseen) {
    launch_fill(ctx->st, ctx->K.ndof, 0.0, x);
    s = fgmres(ctx, ctx_scratch(ctx), b, x, its, rel_res);
  } else {
    s = fcg(ctx, ctx_scratch(ctx), b, x, its, rel_res);
  }
  HIPC(hipStreamSynchronize(ctx->st));
  return s;
}

hdgmg_status hdgmg_inner_solve_noalloc(hdgmg_ctx* ctx, const double* b, double* x, int* its,
                                       double* rel_res) {
  if (!ctx || !b || !x) return HDGMG_EINVAL;
  if (ctx->d3) return HDGMG_ESTATE;  // triangular meshes only
  if (!ctx->assembled) {
    ctx->err = "hdgmg_inner_solve_noalloc before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  if ((long)(ctx->opts.restart + 1) * RED_BLOCKS > NA_GMH - NA_GMPART) {
    ctx->err = "hdgmg_inner_solve_noalloc: restart exceeds the fixed scratch (at most 64)";
    return HDGMG_EINVAL;
  }
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_dev[ctx->dev];
  }
  if (!base) {
    ctx->err = "hdgmg_inner_solve_noalloc: no scratch address for the context's device";
    return HDGMG_ESTATE;
  }
  const KrylovScratch W{base + NA_SC, base + NA_PART, base + NA_GMPART, base + NA_GMH, base + NA_GMY};
  // the array keeps the previous call's contents: start from zeros
  launch_fill(ctx->st, NA_WORDS, 0.0, base);
  hdgmg_status s;
  if (ctx->opts.oseen) {
    launch_fill(ctx->st, ctx->K.ndof, 0.0, x);
    s = fgmres(ctx, W, b, x, its, rel_res);
  } else {
    s = fcg(ctx, W, b, x, its, rel_res);
  }
  HIPC(hipStreamSynchronize(ctx->st));
  return s;
}

hdgmg_status hdgmg_set_wind(hdgmg_ctx* ctx, const double* w_qp) {
  if (ctx && ctx->d3) {
    return HDGMG_ESTATE;
  }
  if (!ctx) return HDGMG_EINVAL;
  if (!ctx->opts.oseen) {
    ctx->err = "hdgmg_set_wind needs a context set up with opts.oseen = 1";
    return HDGMG_ESTATE;
  }
  drop_graph(ctx);
  ctx->assembled = false;
  ctx->has_wind = false;
  ctx->has_newton = false;  // a Newton state belongs to the wind it came with
  if (!w_qp) return HDGMG_OK;
  hipStream_t st = ctx->st;
  DevLevel& KL = ctx->K;
  const int na = dims_of(ctx->k).na;
  // RT_k coefficients of the wind on the order-k level
  long per = (long)na * (na + 1);
  long batch = std::max<long>(1, std::min<long>(KL.nc, (long)(ctx->ws_bytes / (per * sizeof(double)))));
  HIPC(hipMemsetAsync(ctx->status, 0, sizeof(int), st));
  for (long c0 = 0; c0 < KL.nc; c0 += batch)
    launch_wind_fit(st, ctx->Q, KL.X, KL.cells, (int)c0, (int)std::min<long>(batch, KL.nc - c0), w_qp, ctx->ws,
                    ctx->wcoef, ctx->status);
  HIPC(hipGetLastError());
  TRY(check_status(ctx, "wind fit"));
  // facet fluxes on the finest level, summed over facet halves downwards
  const int J = ctx->J;
  std::vector<std::vector<double>> fl(J);
  fl[J - 1].resize(KL.nint);
  launch_facet_flux(st, ctx->Q, KL.X, KL.cells, KL.fcell, KL.floc, KL.nint, ctx->wcoef, na, ctx->cr[J - 1].flux);
  HIPC(hipGetLastError());
  if (KL.nint > 0)
    HIPC(hipMemcpyAsync(fl[J - 1].data(), ctx->cr[J - 1].flux, KL.nint * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  for (int l = J - 1; l > 0; --l) {
    const Level& F = ctx->lv[l];
    const Level& C = ctx->lv[l - 1];
    fl[l - 1].assign(C.nint, 0.0);
    for (int f = 0; f < F.nf; ++f) {
      const int a = F.edges[2 * f], b = F.edges[2 * f + 1];
      if (a >= C.nv || b < C.nv || F.int_id[f] < 0) continue;
      const int E = b - C.nv;  // the coarse facet this half lies on
      if (C.int_id[E] < 0) continue;
      const double sgn = F.norm[2 * f] * C.norm[2 * E] + F.norm[2 * f + 1] * C.norm[2 * E + 1];
      fl[l - 1][C.int_id[E]] += fl[l][F.int_id[f]] * sgn;
    }
    if (C.nint > 0)
      HIPC(hipMemcpyAsync(ctx->cr[l - 1].flux, fl[l - 1].data(), C.nint * sizeof(double), hipMemcpyHostToDevice,
                          st));
    HIPC(hipStreamSynchronize(st));
  }
  // RT0 winds of the lowest-order levels
  HIPC(hipMemsetAsync(ctx->status, 0, sizeof(int), st));
  for (int l = 0; l < J; ++l) {
    DevLevel& D = ctx->cr[l];
    long b0 = std::max<long>(1, std::min<long>(D.nc, (long)(ctx->ws_bytes / (12 * sizeof(double)))));
    for (long c0 = 0; c0 < D.nc; c0 += b0)
      launch_wind_rt0(st, ctx->Q0, D.X, D.cells, D.cell_dofs, (int)c0, (int)std::min<long>(b0, D.nc - c0), D.flux,
                      ctx->ws, D.wcoef, ctx->status);
  }
  HIPC(hipGetLastError());
  TRY(check_status(ctx, "lowest-order wind"));
  HIPC(hipStreamSynchronize(st));
  ctx->has_wind = true;
  return HDGMG_OK;
}

hdgmg_status hdgmg_set_newton(hdgmg_ctx* ctx, const double* state_prev) {
  if (ctx && ctx->d3) {
    return HDGMG_ESTATE;
  }
  if (!ctx) return HDGMG_EINVAL;
  if (!state_prev) {
    if (ctx->has_newton) {
      drop_graph(ctx);
      ctx->assembled = false;
    }
    ctx->has_newton = false;
    return HDGMG_OK;
  }
  if (!ctx->opts.oseen || ctx->opts.transpose || ctx->k < 1 || !ctx->has_wind) {
    ctx->err = "hdgmg_set_newton needs an opts.oseen context (not transposed), k >= 1 and a wind";
    return HDGMG_ESTATE;
  }
  const DevLevel& KL = ctx->K;
  if (!ctx->nw_lam) {
    TRY(dalloc(ctx, &ctx->nw_lam, (size_t)std::max<long>(KL.ndof, 1)));
    TRY(dalloc(ctx, &ctx->nw_load, (size_t)KL.nc * dims_of(ctx->k).nz));
  }
  drop_graph(ctx);
  ctx->assembled = false;
  if (KL.ndof > 0) launch_copy(ctx->st, KL.ndof, state_prev, ctx->nw_lam);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(ctx->st));
  ctx->has_newton = true;
  return HDGMG_OK;
}

static hdgmg_status set_dirichlet(hdgmg_ctx* ctx, const double* uhat_b, bool full) {
  if (ctx && ctx->d3) {
    return HDGMG_ESTATE;
  }
  if (!ctx) return HDGMG_EINVAL;
  ctx->has_bd = false;
  ctx->has_flux = false;
  if (!uhat_b) return HDGMG_OK;
  launch_bd_local(ctx->st, ctx->K.nc, ctx->k + 1, ctx->cbf, uhat_b, full ? 1 : 0, ctx->bdl);
  if (full) launch_bd_flux(ctx->st, ctx->K.nc, ctx->k + 1, ctx->bdiv, ctx->bdl, ctx->cflux);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(ctx->st));
  ctx->has_bd = true;
  ctx->has_flux = full;
  return HDGMG_OK;
}

hdgmg_status hdgmg_set_dirichlet(hdgmg_ctx* ctx, const double* uhat_b) { return set_dirichlet(ctx, uhat_b, false); }

hdgmg_status hdgmg_set_dirichlet_full(hdgmg_ctx* ctx, const double* uhat_b) { return set_dirichlet(ctx, uhat_b, true); }

hdgmg_status hdgmg_set_dirichlet_velocity(hdgmg_ctx* ctx, const double* g_b) {
  if (ctx && ctx->d3) return HDGMG_ESTATE;
  if (!ctx) return HDGMG_EINVAL;
  if (!g_b) return hdgmg_set_dirichlet(ctx, nullptr);
  const int nb = (int)ctx->bfacets.size();
  if (!ctx->btan) {
    const Level& LF = ctx->lv[ctx->J - 1];
    std::vector<double> t(2 * (size_t)std::max(nb, 1), 0.0);
    for (int i = 0; i < nb; ++i) {
      t[2 * i] = LF.tang[2 * ctx->bfacets[i]];
      t[2 * i + 1] = LF.tang[2 * ctx->bfacets[i] + 1];
    }
    TRY(upload(ctx, &ctx->btan, t));
    TRY(dalloc(ctx, &ctx->bvals, (size_t)std::max(nb, 1) * (ctx->k + 1)));
  }
  launch_dirichlet_const(ctx->st, nb, ctx->k + 1, ctx->btan, g_b, ctx->bvals);
  HIPC(hipGetLastError());
  return hdgmg_set_dirichlet(ctx, ctx->bvals);
}

// ||a - b||_0 over the data points (b may be null)
static hdgmg_status wnorm(hdgmg_ctx* ctx, const double* a, const double* b, double* out) {
  const DevLevel& KL = ctx->K;
  launch_wdiff2(ctx->st, ctx->Q, KL.X, KL.cells, KL.nc, a, b, ctx->part, RED_BLOCKS);
  launch_finalize(ctx->st, ctx->part, RED_BLOCKS, 1, ctx->sc, SC_BB);
  double hs[SC_N];
  HIPC(hipMemcpyAsync(hs, ctx->sc, sizeof(hs), hipMemcpyDeviceToHost, ctx->st));
  HIPC(hipStreamSynchronize(ctx->st));
  *out = std::sqrt(std::max(hs[SC_BB], 0.0));
  return HDGMG_OK;
}

hdgmg_status hdgmg_picard_newton(hdgmg_ctx* ctx, const double* f_qp, const hdgmg_alg3_opts* a, double* u_qp,
                                 double* p_qp, double* state, hdgmg_alg3_info* info, hdgmg_alg3_step_fn step_fn,
                                 void* step_ctx) {
  if (ctx && ctx->d3) return HDGMG_ESTATE;
  if (!ctx || !f_qp || !a || !u_qp || !p_qp || !state) return HDGMG_EINVAL;
  if (!ctx->opts.oseen || ctx->opts.transpose) {
    ctx->err = "hdgmg_picard_newton needs a context with opts.oseen = 1, opts.transpose = 0";
    return HDGMG_ESTATE;
  }
  if (a->max_picard < 0 || a->max_newton < 0 || a->max_picard + a->max_newton + 1 > HDGMG_MAX_ALG3 ||
      (a->max_newton > 0 && ctx->k < 1)) {
    ctx->err = "hdgmg_picard_newton: step caps out of range (Newton needs k >= 1)";
    return HDGMG_EINVAL;
  }
  const auto t0 = std::chrono::steady_clock::now();
  const DevLevel& KL = ctx->K;
  const long nqd = (long)KL.nc * ctx->Q.nq, ns = KL.ndof + KL.nc;
  if (!(a->dt_inv >= 0.0) || !std::isfinite(a->dt_inv)) {
    ctx->err = "hdgmg_picard_newton: dt_inv must be finite and >= 0";
    return HDGMG_EINVAL;
  }
  if (!ctx->a3_u) {
    TRY(dalloc(ctx, &ctx->a3_u, (size_t)nqd * 2));
    TRY(dalloc(ctx, &ctx->a3_state, (size_t)ns));
  }
  const bool ptime = a->dt_inv > 0.0;
  if (ptime && !ctx->a3_f) TRY(dalloc(ctx, &ctx->a3_f, (size_t)nqd * 2));
  const double beta0 = ctx->beta;
  // pseudo-time steps (Stokes and Picard phases): mass term dt_inv u in the
  // operator (beta + dt_inv at assembly) and dt_inv u_{n-1} in the load
  struct BetaGuard {
    hdgmg_ctx* c;
    double b;
    ~BetaGuard() { c->beta = b; }
  } guard{ctx, beta0};
  if (ptime) {
    ctx->beta = beta0 + a->dt_inv;
    launch_copy(ctx->st, nqd * 2, f_qp, ctx->a3_f);
  }
  if (info) std::memset(info, 0, sizeof(*info));
  TRY(hdgmg_set_wind(ctx, nullptr));
  TRY(hdgmg_assemble(ctx));
  int kind = 0, n_p = 0, n_n = 0, step = 0;
  hdgmg_status result = HDGMG_OK;
  while (true) {
    hdgmg_info inf;
    const bool warm = step > 0;
    const double* f_step = ptime && kind < 2 ? ctx->a3_f : f_qp;
    hdgmg_status s = hdgmg_solve_x0(ctx, f_step, warm ? ctx->a3_state : nullptr,
                                    kind == 2 ? ctx->a3_state + KL.ndof : nullptr, u_qp, p_qp, state, &inf);
    if (s < 0) return s;
    result = std::max(result, s);
    double du = -1.0, un = 0.0;
    if (warm) TRY(wnorm(ctx, u_qp, ctx->a3_u, &du));
    if (kind == 2) TRY(wnorm(ctx, u_qp, nullptr, &un));
    if (info) {
      info->n_steps = step + 1;
      info->kind[step] = kind;
      info->du[step] = du;
      info->status[step] = s;
      info->uzawa_steps[step] = inf.uzawa_steps;
      for (int i = 0; i < inf.uzawa_steps; ++i) info->its[step] += inf.its[i];
    }
    if (step_fn) {
      HIPC(hipStreamSynchronize(ctx->st));
      step_fn(step_ctx, step, kind, s, du, &inf);
    }
    ++step;
    bool done = false;
    if (kind == 2) {
      ++n_n;
      done = du <= std::max(a->newton_rtol * un, a->newton_atol) || n_n >= a->max_newton;
    } else if (kind == 1) {
      ++n_p;
      if (du < a->eps_picard || n_p >= a->max_picard) {
        kind = 2;
        done = a->max_newton == 0;
      }
    } else {
      kind = a->max_picard > 0 ? 1 : 2;
      done = a->max_picard == 0 && a->max_newton == 0;
    }
    if (done) break;
    // the next step linearises at this one
    launch_copy(ctx->st, nqd * 2, u_qp, ctx->a3_u);
    launch_copy(ctx->st, ns, state, ctx->a3_state);
    if (ptime) {
      if (kind < 2) {
        launch_copy(ctx->st, nqd * 2, f_qp, ctx->a3_f);
        launch_axpy(ctx->st, nqd * 2, a->dt_inv, ctx->a3_u, ctx->a3_f);
      }
      ctx->beta = kind < 2 ? beta0 + a->dt_inv : beta0;
    }
    TRY(hdgmg_set_wind(ctx, ctx->a3_u));
    if (kind == 2) TRY(hdgmg_set_newton(ctx, ctx->a3_state));
    TRY(hdgmg_assemble(ctx));
  }
  if (info) info->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return result;
}

hdgmg_status hdgmg_recover(hdgmg_ctx* ctx, const double* f_qp, const double* state, double* u_qp,
                           double* p_qp) {
  if (ctx && ctx->d3) return f_qp && state && u_qp && p_qp ? d3_recover(ctx->d3, f_qp, state, u_qp, p_qp) : HDGMG_EINVAL;
  if (!ctx || !f_qp || !state || !u_qp || !p_qp) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_recover before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  TRY(batched(ctx, ctx->K, elem_level(ctx, ctx->K, true, true), EL_RECOVER, f_qp, state, state + ctx->K.ndof, u_qp,
              p_qp));
  HIPC(hipStreamSynchronize(ctx->st));
  return HDGMG_OK;
}

hdgmg_status hdgmg_postprocess(hdgmg_ctx* ctx, const double* f_qp, const double* state, double* ustar_qp) {
  if (ctx && ctx->d3) {
    return HDGMG_ESTATE;
  }
  if (!ctx || !f_qp || !state || !ustar_qp) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_postprocess before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  if (ctx->has_newton) {
    ctx->err = "hdgmg_postprocess of a Newton step is not provided (its local load is kept apart)";
    return HDGMG_ESTATE;
  }
  TRY(batched(ctx, ctx->K, elem_level(ctx, ctx->K, true, true), EL_POSTPROCESS, f_qp, state, nullptr, ustar_qp,
              nullptr));
  HIPC(hipStreamSynchronize(ctx->st));
  return HDGMG_OK;
}

hdgmg_status hdgmg_solve(hdgmg_ctx* ctx, int nrhs, const double* f_qp, double* u_qp, double* p_qp, double* state,
                         hdgmg_info* info) {
  if (!ctx || nrhs < 1 || !f_qp || !u_qp || !p_qp) return HDGMG_EINVAL;
  int64_t nc = 0, nq = 0, ns = 0, dim = 2;
  TRY(hdgmg_query(ctx, 0, 0, &nc));
  TRY(hdgmg_query(ctx, 1, 0, &nq));
  TRY(hdgmg_query(ctx, 2, 0, &ns));
  TRY(hdgmg_query(ctx, 11, 0, &dim));
  hdgmg_status result = HDGMG_OK;
  for (int i = 0; i < nrhs; ++i) {
    const long o = (long)i * nc * nq;
    hdgmg_status s = hdgmg_solve_x0(ctx, f_qp + o * dim, nullptr, nullptr, u_qp + o * dim, p_qp + o,
                                    state ? state + (long)i * (ns + nc) : nullptr, info ? info + i : nullptr);
    if (s < 0) return s;
    result = std::max(result, s);
  }
  return result;
}

hdgmg_status hdgmg_solve_x0(hdgmg_ctx* ctx, const double* f_qp, const double* x0, const double* p_init,
                            double* u_qp, double* p_qp, double* state, hdgmg_info* info) {
  if (ctx && ctx->d3) {
    if (!f_qp || !u_qp || !p_qp) return HDGMG_EINVAL;
    if (x0 || p_init) return HDGMG_EINVAL;
    return d3_solve(ctx->d3, f_qp, nullptr, u_qp, p_qp, state, info);
  }
  if (!ctx || !f_qp || !u_qp || !p_qp) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_solve before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = ctx->st;
  const DevLevel& KL = ctx->K;
  if (x0)
    launch_copy(st, KL.ndof, x0, ctx->lam);
  else
    launch_fill(st, KL.ndof, 0.0, ctx->lam);
  // p^(0) before the load: p_init may alias the caller's state
  if (p_init)
    launch_copy(st, KL.nc, p_init, ctx->p0);
  else
    launch_fill(st, KL.nc, 0.0, ctx->p0);
  TRY(hdgmg_rhs(ctx, f_qp, ctx->gvec));
  hdgmg_status result = HDGMG_OK;
  for (int n = 0; n < ctx->opts.uzawa_max; ++n) {
    launch_uzawa_rhs(st, KL.nint, KL.m, ctx->gvec, ctx->fdiv, KL.fcell, ctx->p0, ctx->b);
    int its = 0;
    double rel = 0.0;
    // Oseen: FGMRES from the latest iterate; Stokes: flexible CG from zero
    hdgmg_status s = ctx->opts.oseen ? fgmres(ctx, ctx_scratch(ctx), ctx->b, ctx->lam, &its, &rel)
                                     : fcg(ctx, ctx_scratch(ctx), ctx->b, ctx->lam, &its, &rel);
    if (s < 0) return s;
    if (s == HDGMG_NOT_CONVERGED) result = s;
    launch_uzawa_update(st, KL.nc, KL.m, KL.cell_dofs, ctx->cdiv, ctx->area, ctx->lam, ctx->gamma,
                        ctx->has_flux ? ctx->cflux : nullptr, ctx->p0, ctx->part, RED_BLOCKS);
    launch_finalize(st, ctx->part, RED_BLOCKS, 2, ctx->sc, SC_DP);
    double hs[SC_N];
    HIPC(hipMemcpyAsync(hs, ctx->sc, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    double dn = std::sqrt(hs[SC_DP]), pn = std::sqrt(hs[SC_PP]);
    if (info) {
      info->uzawa_steps = n + 1;
      info->its[n] = its;
      info->rel_res[n] = rel;
      info->dp_l2[n] = dn;
      info->div_l2 = dn / ctx->gamma;
    }
    if (dn <= ctx->opts.uzawa_tol * std::max(1.0, pn)) break;
    if (n == ctx->opts.uzawa_max - 1 && ctx->opts.uzawa_tol >= 0) {
      result = HDGMG_NOT_CONVERGED;
      ctx->err = "AL-Uzawa reached uzawa_max";
    }
  }
  if (state) {
    launch_copy(st, KL.ndof, ctx->lam, state);
    launch_copy(st, KL.nc, ctx->p0, state + KL.ndof);
  }
  // recovery reads the skeleton vector and pressure from one buffer
  double* stt = state ? state : ctx->statebuf;
  if (!state) {
    launch_copy(st, KL.ndof, ctx->lam, stt);
    launch_copy(st, KL.nc, ctx->p0, stt + KL.ndof);
  }
  TRY(hdgmg_recover(ctx, f_qp, stt, u_qp, p_qp));
  HIPC(hipStreamSynchronize(st));
  if (info) info->t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return result;
}

// Buffers of the adjoint solve, allocated at its first call on the calling
// thread (the batch entry point calls this before it starts its workers, so
// that the caller's allocator only runs on the caller's thread).
static hdgmg_status adjoint_buffers(hdgmg_ctx* ctx) {
  if (ctx->adj_f) return HDGMG_OK;
  const long nqd = (long)ctx->K.nc * ctx->Q.nq;
  TRY(dalloc(ctx, &ctx->adj_f, (size_t)nqd * 2));
  TRY(dalloc(ctx, &ctx->adj_p, (size_t)nqd));
  TRY(dalloc(ctx, &ctx->adj_state, (size_t)(ctx->K.ndof + ctx->K.nc)));
  TRY(dalloc(ctx, &ctx->adj_gnu, (size_t)ctx->K.nc));
  return HDGMG_OK;
}

static hdgmg_status adjoint_one(hdgmg_ctx* ctx, const double* f_qp, const double* state, const double* gu_qp,
                                double* gf_qp, double* gnu, double* adj_state, hdgmg_info* info) {
  if (!ctx || !f_qp || !state || !gu_qp || !gf_qp) return HDGMG_EINVAL;
  if (!ctx->assembled) {
    ctx->err = "hdgmg_solve_adjoint before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  if (ctx->has_wind && !ctx->opts.transpose) {
    ctx->err = "the adjoint of an Oseen system needs a context set up with opts.transpose = 1";
    return HDGMG_ESTATE;
  }
  const DevLevel& KL = ctx->K;
  TRY(adjoint_buffers(ctx));
  double* ast = adj_state ? adj_state : ctx->adj_state;
  // the adjoint load v -> sum gu . v(x_q) is the forward load of gu / (w_q |K|)
  launch_data_weight(ctx->st, ctx->Q, KL.X, KL.cells, KL.nc, gu_qp, 1, ctx->adj_f);
  HIPC(hipGetLastError());
  // the adjoint state has homogeneous boundary data; the prescribed values
  // enter only the forward state's local fields in the viscosity gradient
  const bool bd = ctx->has_bd;
  ctx->has_bd = false;
  hdgmg_status result = hdgmg_solve_x0(ctx, ctx->adj_f, nullptr, nullptr, gf_qp, ctx->adj_p, ast, info);
  ctx->has_bd = bd;
  if (result < 0) return result;
  // dJ/df = w_q |K| u_adj(x_q)
  launch_data_weight(ctx->st, ctx->Q, KL.X, KL.cells, KL.nc, gf_qp, 0, gf_qp);
  HIPC(hipGetLastError());
  if (gnu)
    TRY(batched(ctx, ctx->K, elem_level(ctx, ctx->K, true, true), EL_GRADNU, f_qp, state, nullptr, gnu, nullptr,
                ctx->adj_f, ast));
  HIPC(hipStreamSynchronize(ctx->st));
  return result;
}

hdgmg_status hdgmg_solve_adjoint(hdgmg_ctx* ctx, int nrhs, const double* f_qp, const double* state,
                                 const double* gu_qp, double* gf_qp, double* gnu, double* adj_state,
                                 hdgmg_info* info) {
  if (ctx && ctx->d3) return HDGMG_ESTATE;
  if (!ctx || nrhs < 1) return HDGMG_EINVAL;
  const long nqd = (long)ctx->K.nc * ctx->Q.nq, ns = ctx->K.ndof + ctx->K.nc;
  hdgmg_status result = HDGMG_OK;
  for (int i = 0; i < nrhs; ++i) {
    hdgmg_status s = adjoint_one(ctx, f_qp + i * nqd * 2, state + i * ns, gu_qp + i * nqd * 2, gf_qp + i * nqd * 2,
                                 gnu, adj_state ? adj_state + i * ns : nullptr, info ? info + i : nullptr);
    if (s < 0) return s;
    result = std::max(result, s);
  }
  return result;
}

hdgmg_status hdgmg_solve_batch(hdgmg_ctx* const* ctxs, int nctx, int nrhs, const double* f_qp, double* u_qp,
                               double* p_qp, double* states, hdgmg_info* infos) {
  TRY(batch_check(ctxs, nctx, nrhs));
  if (nrhs > 0 && (!f_qp || !u_qp || !p_qp)) return HDGMG_EINVAL;
  const long nqd = (long)ctxs[0]->K.nc * ctxs[0]->Q.nq, ns = ctxs[0]->K.ndof + ctxs[0]->K.nc;
  return batch_run(ctxs, nctx, nrhs, [&](hdgmg_ctx* ctx, int i) {
    return hdgmg_solve_x0(ctx, f_qp + i * nqd * 2, nullptr, nullptr, u_qp + i * nqd * 2, p_qp + i * nqd,
                          states ? states + i * ns : nullptr, infos ? infos + i : nullptr);
  });
}

hdgmg_status hdgmg_solve_adjoint_batch(hdgmg_ctx* const* ctxs, int nctx, int nrhs, const double* f_qp,
                                       const double* states, const double* gu_qp, double* gf_qp, double* gnu,
                                       hdgmg_info* infos) {
  TRY(batch_check(ctxs, nctx, nrhs));
  if (nrhs > 0 && (!f_qp || !states || !gu_qp || !gf_qp)) return HDGMG_EINVAL;
  const long nqd = (long)ctxs[0]->K.nc * ctxs[0]->Q.nq, ns = ctxs[0]->K.ndof + ctxs[0]->K.nc;
  const long nc = ctxs[0]->K.nc;
  for (int c = 0; c < nctx && nrhs > 0; ++c) {
    hdgmg_status s = adjoint_buffers(ctxs[c]);
    if (s != HDGMG_OK) return s;
  }
  // each context accumulates into a buffer of its own (no two streams add
  // into the same array); the shares are summed into gnu at the end
  if (gnu)
    for (int c = 0; c < nctx; ++c) launch_fill(ctxs[c]->st, nc, 0.0, ctxs[c]->adj_gnu);
  hdgmg_status result = batch_run(ctxs, nctx, nrhs, [&](hdgmg_ctx* ctx, int i) {
    return adjoint_one(ctx, f_qp + i * nqd * 2, states + i * ns, gu_qp + i * nqd * 2, gf_qp + i * nqd * 2,
                       gnu ? ctx->adj_gnu : nullptr, nullptr, infos ? infos + i : nullptr);
  });
  if (result < 0 || !gnu || nrhs <= 0) return result;
  hdgmg_ctx* ctx = ctxs[0];
  for (int c = 0; c < nctx; ++c) launch_axpy(ctx->st, nc, 1.0, ctxs[c]->adj_gnu, gnu);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(ctx->st));
  return result;
}

hdgmg_status hdgmg_kernel_timer(hdgmg_ctx* ctx, int cls, int enable) {
  if (ctx && ctx->d3) return d3_kernel_timer(ctx->d3, cls, enable);
  if (!ctx || cls < 0 || cls > 4) return HDGMG_EINVAL;
  HIPC(hipStreamSynchronize(ctx->st));
  kt_clear(ctx->timers[cls]);
  ctx->timers[cls].on = enable != 0;
  return HDGMG_OK;
}

hdgmg_status hdgmg_kernel_timer_read(hdgmg_ctx* ctx, int cls, double* total_ms, int64_t* launches,
                                     double* bytes) {
  if (ctx && ctx->d3) return d3_kernel_timer_read(ctx->d3, cls, total_ms, launches, bytes);
  if (!ctx || cls < 0 || cls > 4) return HDGMG_EINVAL;
  HIPC(hipStreamSynchronize(ctx->st));
  auto& T = ctx->timers[cls];
  double tot = 0.0;
  for (auto& e : T.ev) {
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, e.first, e.second));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)T.ev.size();
  if (bytes) *bytes = T.bytes;
  return HDGMG_OK;
}

hdgmg_status hdgmg_query(const hdgmg_ctx* ctx, int what, int level, int64_t* value) {
  if (ctx && ctx->d3) return value ? d3_query(ctx->d3, what, level, value) : HDGMG_EINVAL;
  if (!ctx || !value) return HDGMG_EINVAL;
  const Level& LF = ctx->lv.back();
  switch (what) {
    case 0: *value = LF.nc; return HDGMG_OK;
    case 1: *value = ctx->Q.nq; return HDGMG_OK;
    case 2: *value = ctx->K.ndof; return HDGMG_OK;
    case 3: *value = ctx->J; return HDGMG_OK;
    case 4: *value = (int64_t)ctx->bytes; return HDGMG_OK;
    case 5: *value = LF.nint; return HDGMG_OK;
    case 6: *value = ctx->k; return HDGMG_OK;
    case 7: *value = LF.ncol; return HDGMG_OK;
    case 8:
    case 9:
      if (level < 0 || level >= ctx->J) return HDGMG_EINVAL;
      *value = what == 8 ? ctx->lv[level].nc : 2L * ctx->lv[level].nint;
      return HDGMG_OK;
    case 10: *value = (int64_t)ctx->bfacets.size(); return HDGMG_OK;
    case 11: *value = 2; return HDGMG_OK;
    case 12: *value = (int64_t)ctx->vcycle_bytes; return HDGMG_OK;
    case 13: *value = (int64_t)ctx->vcycle_compulsory; return HDGMG_OK;
    case 14:
      if (level < 1 || level >= ctx->J || !ctx->assembled) return HDGMG_EINVAL;
      *value = ctx->tr[level].nnz;
      return HDGMG_OK;
    default: return HDGMG_EINVAL;
  }
}

hdgmg_status hdgmg_export(const hdgmg_ctx* cctx, int what, int level, void* dst, size_t bytes) {
  if (cctx && cctx->d3) return dst ? d3_export(cctx->d3, what, level, dst, bytes) : HDGMG_EINVAL;
  hdgmg_ctx* ctx = const_cast<hdgmg_ctx*>(cctx);
  if (!ctx || !dst) return HDGMG_EINVAL;
  if (!ctx->assembled && (what == 0 || what == 1)) {
    ctx->err = "hdgmg_export of an operator before hdgmg_assemble";
    return HDGMG_ESTATE;
  }
  const double* src = nullptr;
  size_t n = 0;
  if (what == 4) {
    const Level& LF = ctx->lv.back();
    n = (size_t)LF.nc * ctx->Q.nq;
    if (bytes < n * sizeof(double)) {
      ctx->err = "hdgmg_export: destination too small";
      return HDGMG_EINVAL;
    }
    std::vector<double> w(n);
    for (int c = 0; c < LF.nc; ++c)
      for (int q = 0; q < ctx->Q.nq; ++q) w[(size_t)c * ctx->Q.nq + q] = ctx->Q.wq[q] * LF.area[c];
    HIPC(hipMemcpyAsync(dst, w.data(), n * sizeof(double), hipMemcpyHostToDevice, ctx->st));
    HIPC(hipStreamSynchronize(ctx->st));
    return HDGMG_OK;
  }
  if (what == 5) {
    if (!ctx->bvals) {
      ctx->err = "hdgmg_export 5: no hdgmg_set_dirichlet_velocity data on this context";
      return HDGMG_ESTATE;
    }
    n = ctx->bfacets.size() * (ctx->k + 1);
    if (bytes < n * sizeof(double)) {
      ctx->err = "hdgmg_export: destination too small";
      return HDGMG_EINVAL;
    }
    if (n > 0) HIPC(hipMemcpyAsync(dst, ctx->bvals, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->st));
    HIPC(hipStreamSynchronize(ctx->st));
    return HDGMG_OK;
  }
  if (what == 3) {
    const Level& LF = ctx->lv.back();
    n = ctx->bfacets.size() * 4;
    if (bytes < n * sizeof(double)) {
      ctx->err = "hdgmg_export: destination too small";
      return HDGMG_EINVAL;
    }
    std::vector<double> e(std::max<size_t>(n, 1));
    for (size_t i = 0; i < ctx->bfacets.size(); ++i) {
      const int f = ctx->bfacets[i];
      for (int v = 0; v < 2; ++v)
        for (int d = 0; d < 2; ++d) e[4 * i + 2 * v + d] = LF.X[2 * (size_t)LF.edges[2 * f + v] + d];
    }
    if (n > 0) HIPC(hipMemcpyAsync(dst, e.data(), n * sizeof(double), hipMemcpyHostToDevice, ctx->st));
    HIPC(hipStreamSynchronize(ctx->st));
    return HDGMG_OK;
  }
  if (what == 0) {
    src = ctx->K.S;
    n = (size_t)ctx->K.nc * ctx->K.nK * ctx->K.nK;
  } else if (what == 1 && level >= 0 && level < ctx->J) {
    src = ctx->cr[level].S;
    n = (size_t)ctx->cr[level].nc * 36;
  } else if (what == 2) {
    const Level& LF = ctx->lv.back();
    const QuadTables& Q = ctx->Q;
    n = (size_t)LF.nc * Q.nq * 2;
    if (bytes < n * sizeof(double)) {
      ctx->err = "hdgmg_export: destination too small";
      return HDGMG_EINVAL;
    }
    std::vector<double> pts(n);
    for (int c = 0; c < LF.nc; ++c) {
      CellGeom g;
      cell_geom(LF.X.data(), LF.cells.data() + 3 * c, g);
      for (int q = 0; q < Q.nq; ++q) {
        pts[((size_t)c * Q.nq + q) * 2] = g.Xs0[0] + g.J[0][0] * Q.xi[q][0] + g.J[0][1] * Q.xi[q][1];
        pts[((size_t)c * Q.nq + q) * 2 + 1] = g.Xs0[1] + g.J[1][0] * Q.xi[q][0] + g.J[1][1] * Q.xi[q][1];
      }
    }
    HIPC(hipMemcpyAsync(dst, pts.data(), n * sizeof(double), hipMemcpyHostToDevice, ctx->st));
    HIPC(hipStreamSynchronize(ctx->st));
    return HDGMG_OK;
  } else {
    ctx->err = "hdgmg_export: bad what/level";
    return HDGMG_EINVAL;
  }
  if (bytes < n * sizeof(double)) {
    ctx->err = "hdgmg_export: destination too small";
    return HDGMG_EINVAL;
  }
  HIPC(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->st));
  HIPC(hipStreamSynchronize(ctx->st));
  return HDGMG_OK;
}

}  // extern "C"
