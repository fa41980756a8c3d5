/*
 * hdgmg.h -- C ABI of the MI355X (gfx950) library for the hp-multigrid
 * preconditioned solve of the statically condensed, augmented-Lagrangian
 * H(div)-HDG skeleton system of the generalized Stokes problem
 *     -div(nu grad u) + beta u + grad p = f,  div u = 0,  u = 0 on the boundary
 * (Fu & Kuang, arXiv 2303.06762: Sec. 3.1 model, Sec. 3.2 scheme, Sec. 3.3
 * augmented-Lagrangian Uzawa iteration, Sec. 3.4-3.5 Alg. 1 / Alg. 2).
 *
 * Life cycle: hdgmg_setup -> hdgmg_assemble -> hdgmg_solve (any number of
 * times) -> hdgmg_destroy.  The operator-level calls (hdgmg_rhs,
 * hdgmg_apply, hdgmg_precondition, hdgmg_inner_solve, hdgmg_recover) expose
 * the individual steps of hdgmg_solve on caller-owned device vectors.
 *
 * Conventions shared by every call
 *  - Every function returns hdgmg_status (or a pointer / void where noted);
 *    none throws, aborts or exits.  A negative status leaves outputs
 *    undefined; hdgmg_last_error(ctx) describes the failure.
 *  - "host" pointers are read during the call only.  "device" pointers are
 *    device (HBM) addresses owned by the caller; they must stay valid until
 *    the call returns.  All device work is enqueued on the stream given at
 *    setup; calls return after that stream has been synchronised unless
 *    stated otherwise.  The library owns the context and its workspace.
 *  - A context must not be used from two threads at once.
 *  - Meshes are 2D conforming triangulations.  The coarse mesh is refined
 *    n_refine times by red refinement (each triangle into four through its
 *    edge midpoints), giving the nested hierarchy T_1 .. T_J of Sec. 3.4.2,
 *    J = n_refine + 1.  Numbering of the refined meshes: the midpoint of
 *    coarse facet e becomes vertex n_vertices + e; coarse cell c = (a,b,c)
 *    has children 4c+0 = (a,m_ab,m_ca), 4c+1 = (m_ab,b,m_bc),
 *    4c+2 = (m_ca,m_bc,c), 4c+3 = (m_bc,m_ca,m_ab).  Facets are sorted vertex
 *    pairs (v0 < v1) numbered lexicographically; interior facets are
 *    numbered in facet order.
 *  - Skeleton vectors (length N_skel = 2 (k+1) n_interior_facets, FP64)
 *    hold, per interior facet F, component c (0: normal trace u.n_F,
 *    1: tangential trace uhat.t_F, with t_F = (x_v1 - x_v0)/|.|,
 *    n_F = (t_y, -t_x)) and mode j the coefficient of the orthonormal
 *    facet Legendre function sqrt(2j+1) P_j(2s-1), s in [0,1] from v0 to v1;
 *    index (F * 2 + c) * (k+1) + j.
 *  - Cell data (f, u, p) live at the data quadrature points of each cell:
 *    the Stroud conical rule with k+2 points per direction (Gauss-Legendre
 *    in u, Gauss-Jacobi with weight (1-v) in v, point (u(1-v), v), u fastest)
 *    mapped from the cell's vertices sorted by global index; n_q = (k+2)^2.
 *    Layouts (C order, FP64): f and u [n_cells][n_q][2]; p [n_cells][n_q].
 *  - The augmented-Lagrangian weight is eps^-1 = gamma (the paper's
 *    (nu eps)^-1 with unit reference viscosity).
 */
#ifndef HDGMG_H
#define HDGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HDGMG_OK = 0,
  HDGMG_NOT_CONVERGED = 1,  /* outputs hold the last iterate; see info     */
  HDGMG_EINVAL = -1,        /* bad argument                                 */
  HDGMG_EMESH = -2,         /* non-conforming / degenerate mesh             */
  HDGMG_ENOMEM = -3,        /* device or host allocation failed             */
  HDGMG_EHIP = -4,          /* HIP runtime error                            */
  HDGMG_ESTATE = -5,        /* call out of order (e.g. solve before assemble) */
  HDGMG_EBREAKDOWN = -6,    /* Krylov breakdown: p.Ap <= 0 or z.r <= 0      */
  HDGMG_ENONFINITE = -7     /* NaN/Inf met in the iteration                 */
} hdgmg_status;

typedef struct hdgmg_ctx hdgmg_ctx;

/* Coarsest mesh T_1 (host arrays, copied during hdgmg_setup). */
typedef struct {
  int dim;                 /* must be 2                                    */
  int n_vertices;
  const double* coords;    /* host, [n_vertices][2]                        */
  int n_cells;
  const int32_t* cells;    /* host, [n_cells][3] vertex indices            */
  int n_refine;            /* J = n_refine + 1 levels                      */
  int n_outflow;           /* do-nothing (outflow) facets of T_1 (Sec. 5.3:
                              (nu grad u - p I) n = 0 holds weakly there);
                              0 for none.  Both halves of such a facet are
                              do-nothing facets on the next level.  They
                              carry skeleton unknowns (both components)
                              like interior facets; with any of them the
                              pressure is determined (no mean-free
                              normalisation) and the preconditioner runs
                              its launch-per-colour kernels on every level.
                              Triangular meshes only.                    */
  const int32_t* outflow;  /* host, [n_outflow][2] vertex pairs of boundary
                              facets of T_1 (EMESH if a pair is not one)   */
} hdgmg_mesh;

/* Solver options (Alg. 1 / Alg. 2 parameters and stopping rules, Sec. 5). */
typedef struct {
  int m_relax;             /* m_p: order-k block Gauss-Seidel sweeps       */
  int m_smooth;            /* m_h: sweeps on the finest lowest-order level */
  int cycle;               /* q: 1 = V-cycle, 2 = W-cycle (Alg. 1)          */
  int vcycle_growth;       /* m(l-1) = growth * m(l); 2 = variable V-cycle  */
  double rtol, atol;       /* inner stop: ||r||_2 <= max(rtol ||r0||_2, atol) */
  int max_it;              /* inner iteration cap                          */
  int uzawa_max;           /* AL-Uzawa step cap                            */
  double uzawa_tol;        /* stop when ||p_n - p_{n-1}||_L2 <= tol*max(1,||p_n||);
                              < 0: exactly uzawa_max steps (the paper's fixed
                              count at large eps^-1), not reported as
                              NOT_CONVERGED                                */
  int coarse_dofs;         /* lowest-order levels with at most this many
                              unknowns run MG_h inside one single-workgroup
                              kernel (0: every level launch by launch)     */
  int stream_dofs;         /* levels with at least this many unknowns (and
                              vertex patches of at most 6 facets) use the
                              streaming kernels (see fused_phase); other
                              launched lowest-order levels smooth with the
                              patch-row record kernel, and so do streamed
                              ones without the fused phase unless
                              stream_dofs is 0 (streaming on every
                              level)                                      */
  int vcycle_precision;    /* storage of every operator the preconditioner
                              reads: 0 FP64, 1 FP32, 2 FP32 with the
                              order-k level's streaming cell blocks (k <= 2,
                              symmetric) and patch inverses in FP16, each
                              block scaled by its largest magnitude
                              (vectors, accumulation and the outer Krylov
                              solver stay FP64).  Tetrahedral meshes: 0,
                              1 (cell blocks without their AL term, which
                              is applied apart in FP64, and every other
                              operator FP32) or 3 (as 1 with the order-k
                              edge-patch inverses kept FP64)              */
  int oseen;               /* 1: the context solves Picard-linearised
                              (Oseen) systems (Sec. 4): hdgmg_set_wind is
                              allowed, every block and patch factor is
                              stored and inverted as nonsymmetric, and the
                              inner solver is FGMRES(restart) with right
                              preconditioning; 0: generalized Stokes with
                              flexible CG                                   */
  int restart;             /* FGMRES restart length, 1..64                  */
  int transpose;           /* 1 (with oseen = 1): the context assembles and
                              solves the transposed system A^T of the
                              Picard-linearised scheme at the wind it is
                              given (every cell's convection form
                              transposed; blocks, patch factors, transfers
                              and the coarsest inverse are then those of
                              A^T): the adjoint of the Oseen system, used
                              by hdgmg_solve_adjoint; 0: the system itself */
  int coarse_dense;        /* 1 (V-cycle only): at assembly MG_h on the top
                              level of the single-workgroup kernel (levels
                              0..Lc, from a zero iterate, with the sweep
                              count the V-cycle uses there) is tabulated as
                              a dense matrix -- the kernel applied to the
                              columns of the identity, a workgroup per
                              column -- and each V-cycle applies it by one
                              GEMV instead of running the kernel (the same
                              linear operator up to rounding); 0: the
                              kernel runs in every V-cycle              */
  int rec_wide;            /* 1: every record-smoothed level uses the 32-bit
                              record form (otherwise only levels beyond
                              65535 interior facets); same results      */
  int smoother;            /* patch smoother of the order-k relaxation and
                              the lowest-order smoothing (Sec. 3.4.2):
                              0 block Gauss-Seidel, colour by colour, the
                              transposed sweep in reverse colour order;
                              1 damped block Jacobi (eq. bjac): every patch
                              corrected from the residual at the start of
                              the sweep, damping 1 / (number of patch
                              colours of the level) -- within one colour
                              the patch projections sum to a projection --
                              its own transpose.  Jacobi runs the
                              launch-per-colour kernels on every level of a
                              triangular mesh (the streaming, record and
                              single-workgroup forms are Gauss-Seidel only) */
  int additive;            /* 0: MG_hp of Alg. 2 (relaxation, lowest-order
                              correction of the new residual, relaxation);
                              1: its additive counterpart (Remark 3.4):
                              m_relax forward then m_relax transposed sweeps
                              from zero on r, plus Pi_0^k MG_h(Pi_k^0 r) of
                              the same r                                   */
  int patch_relax;         /* patches of the order-k relaxation: 0 the
                              dimension's default (vertex patches on
                              triangles, edge patches on tetrahedra),
                              1 vertex patches, 2 edge patches (tetrahedra
                              only: EINVAL on triangles)                   */
  int patch_smooth;        /* patches of the lowest-order smoothing, the
                              same codes                                   */
  int fused_phase;         /* 1 (default): on every streamed level of a
                              triangle mesh with symmetric blocks (the
                              order-k level for k <= 2 with
                              vcycle_precision 0 or 1, and the
                              lowest-order levels; vertex patches of at
                              most 7 cells) a Gauss-Seidel colour phase is
                              one launch that takes the step in its direct
                              form x_s = A_ss^-1 (b_s - A_{s,r} x_r) from
                              the patch's own cells, read from a
                              per-colour, patch-ordered copy of their
                              coupling blocks; such lowest-order levels
                              use it in place of the record kernel.  0:
                              the cell-apply / patch-relaxation pair
                              (records on the lowest-order levels).  Same
                              iterates up to rounding (FP64; with FP32
                              storage the two forms agree to FP32
                              rounding amplified by the patch condition
                              numbers); ignored on tetrahedra             */
} hdgmg_opts;

/* Defaults: m_p = m_h = 1, V-cycle, growth 2, rtol 1e-8, atol 1e-10,
 * max_it 500, uzawa_max 50, uzawa_tol 1e-10, coarse_dofs 2048,
 * stream_dofs 65536, vcycle_precision 0, oseen 0, restart 50, transpose 0,
 * coarse_dense 1, rec_wide 0, smoother 0, additive 0, patch_relax 0,
 * patch_smooth 0. */
void hdgmg_default_opts(hdgmg_opts* opts);

#define HDGMG_MAX_UZAWA 64
typedef struct {
  int uzawa_steps;                 /* Uzawa steps taken                     */
  int its[HDGMG_MAX_UZAWA];        /* inner iterations per Uzawa step       */
  double rel_res[HDGMG_MAX_UZAWA]; /* final ||r||/||r0|| per Uzawa step     */
  double dp_l2[HDGMG_MAX_UZAWA];   /* ||p_n - p_{n-1}||_L2 per step         */
  double div_l2;                   /* ||div u_h||_L2 of the returned velocity:
                                      div u_h is constant per cell (its
                                      normal traces), equal to
                                      (p_n - p_{n-1}) / (-eps^-1) of the
                                      last step                             */
  double t_solve;                  /* host wall time of the call, seconds   */
} hdgmg_info;

/* Device allocator of the caller (e.g. PyTorch's caching allocator):
 * alloc returns `bytes` bytes of device memory aligned to at least 256 bytes,
 * or NULL on failure; free releases a pointer alloc returned.  Both are
 * called on the thread that called the library, only from hdgmg_setup,
 * hdgmg_assemble, hdgmg_set_newton (its first call), hdgmg_solve_adjoint and
 * hdgmg_solve_adjoint_batch (the first adjoint solve of a context; the batch
 * allocates for every context before its worker threads start) and
 * hdgmg_destroy, after the context's stream has been synchronised for
 * frees. */
typedef void* (*hdgmg_alloc_fn)(size_t bytes, void* alloc_ctx);
typedef void (*hdgmg_free_fn)(void* ptr, void* alloc_ctx);

/* Build the mesh hierarchy, skeleton topology, vertex patches with their
 * colouring, and the intergrid transfers; allocate device workspace.
 *   k      polynomial order, 0 <= k <= 4
 *   beta   >= 0, the zeroth-order coefficient
 *   nu     host, nu_len values: 1 (constant viscosity) or the number of
 *          finest cells (per-cell viscosity); all > 0
 *   gamma  > 0, eps^-1
 *   opts   host, may be NULL for the defaults
 *   stream hipStream_t used for every device operation (NULL: a stream of
 *          the library's own)
 *   alloc_fn, free_fn, alloc_ctx  the caller's device allocator, through which
 *          every device buffer of the context is allocated and released
 *          (workspace, operators, factors, transfers); both NULL: hipMalloc
 *          and hipFree.  Giving only one is EINVAL.
 * On success *out receives a new context (release with hdgmg_destroy).
 * Errors: EINVAL (bad k, beta, nu, gamma, opts), EMESH (dim != 2, bad
 * indices, zero-area cell, facet shared by > 2 cells), ENOMEM, EHIP. */
hdgmg_status hdgmg_setup(const hdgmg_mesh* mesh, int k, double beta,
                         const double* nu, int nu_len, double gamma,
                         const hdgmg_opts* opts, void* stream,
                         hdgmg_alloc_fn alloc_fn, hdgmg_free_fn free_fn,
                         void* alloc_ctx, hdgmg_ctx** out);

/* Element local solvers and static condensation of the order-k scheme
 * (stWeak -> stOptForm, with the AL term of stALform), the lowest-order
 * CR-equivalent operators of every level (k0-stOptForm), the patch block
 * inverses of every level, the harmonic-extension transfers (div-transfer,
 * harmonic-ex) and the coarsest-level inverse.  Errors: ESTATE (setup
 * failed), EHIP, ENONFINITE (a singular local problem). */
hdgmg_status hdgmg_assemble(hdgmg_ctx* ctx);

/* Full solve (stOpEq-ALU): condensed load from f, AL-Uzawa outer loop with
 * a flexible-CG inner solve preconditioned by MG_hp (Alg. 2), then local
 * recovery, for nrhs >= 1 right-hand sides one after the other on this
 * context (arrays stacked over the right-hand sides; hdgmg_solve_batch
 * spreads a batch over several contexts and streams instead).
 *   f_qp   device, [nrhs][n_cells][n_q][d] source at the data points
 *          (d = 2 on triangles, 3 on tetrahedra)
 *   u_qp   device, [nrhs][n_cells][n_q][d] velocity at the data points (output)
 *   p_qp   device, [nrhs][n_cells][n_q] pressure, mean zero (output)
 *   state  device or NULL, [nrhs][N_skel + n_cells]: skeleton coefficients
 *          then the piecewise-constant pressure (output)
 *   info   host or NULL, [nrhs] (output)
 * Returns OK, NOT_CONVERGED (an inner solve hit max_it or Uzawa hit
 * uzawa_max; outputs hold the last iterate), ESTATE, EBREAKDOWN, ENONFINITE,
 * EHIP. */
hdgmg_status hdgmg_solve(hdgmg_ctx* ctx, int nrhs, const double* f_qp, double* u_qp,
                         double* p_qp, double* state, hdgmg_info* info);

/* Adjoint solve for a functional J(u_qp) of the velocity at the data points
 * (not in the paper; derived from the scheme of Sec. 3.2, whose system is a
 * symmetric saddle point in which the viscosity enters only through the
 * nu-weighted lifting energy of each cell, and from its Picard-linearised
 * form of Sec. 4.2 at a fixed wind, whose convection form is nonsymmetric
 * and independent of the viscosity).
 * For nrhs >= 1 right-hand sides one after the other (f_qp, state, gu_qp,
 * gf_qp, adj_state and info stacked over them; gnu accumulates all).
 *   f_qp   device [n_cells][n_q][2], input: the forward source
 *   state  device [N_skel + n_cells], input: the forward state written by
 *          hdgmg_solve for f_qp (the forward solution is checkpointed as
 *          this state; no Krylov data is kept)
 *   gu_qp  device [n_cells][n_q][2], input: dJ/du_qp
 *   gf_qp  device [n_cells][n_q][2], output: dJ/df_qp = w_q |K| u_adj(x_q),
 *          w_q the data-rule weights (sum 1) and |K| the cell area
 *   gnu    device [n_cells] (finest cells), ACCUMULATED, may be NULL:
 *          gnu[K] += dJ/dnu_K = -(Lift(u, uhat), Lift(u_adj, uhat_adj))_K
 *   adj_state device [N_skel + n_cells], output, may be NULL: the adjoint state
 *   info   host, may be NULL: the adjoint solve's Uzawa / inner iterations
 * The adjoint state solves the transposed system with the load
 * v -> sum_{K,q} gu_qp . v(x_q): for generalized Stokes (symmetric) the
 * forward system itself (same AL-Uzawa, flexible CG and MG_hp); for the
 * Oseen system at a wind, the context must have been set up with
 * opts.oseen = 1 and opts.transpose = 1 and given the forward wind
 * (hdgmg_set_wind, hdgmg_assemble): it then holds A^T, the adjoint state
 * is its AL-Uzawa + FGMRES solve preconditioned by MG_hp of A^T, and in
 * gnu the forward state's local fields are recovered with the forward
 * cell systems and the adjoint's with the transposed ones.  state must
 * come from a context with the same mesh, order, coefficients and wind.
 * Tangential Dirichlet data set on the context (hdgmg_set_dirichlet; on an
 * adjoint context, the forward context's values) are the forward state's:
 * the adjoint state has homogeneous data, and the values enter only the
 * forward local fields of gnu.  gf_qp must not alias the inputs.  Returns
 * as hdgmg_solve; outputs are undefined on a negative status.  ESTATE with a
 * wind on a context without opts.transpose. */
hdgmg_status hdgmg_solve_adjoint(hdgmg_ctx* ctx, int nrhs, const double* f_qp, const double* state,
                                 const double* gu_qp, double* gf_qp, double* gnu,
                                 double* adj_state, hdgmg_info* info);

/* A batch of nrhs right-hand sides over nctx contexts set up and assembled
 * for the same problem (identical mesh, order, coefficients and options;
 * sizes are checked): right-hand side i is solved by context i % nctx, each
 * context working through its share on its own stream in a host thread of
 * its own, so that independent solves overlap on the device.  Arrays are
 * the single-solve layouts stacked over the batch: f_qp, u_qp
 * [nrhs][n_cells][n_q][2], p_qp [nrhs][n_cells][n_q], states (may be NULL)
 * [nrhs][N_skel + n_cells], infos (host, may be NULL) [nrhs].  The inputs
 * must be complete before the call (synchronise the stream that produced
 * them); the call returns after every context's stream has finished.
 * Returns the first negative status, else the largest (NOT_CONVERGED if
 * any solve did not converge); EINVAL for a context given twice. */
hdgmg_status hdgmg_solve_batch(hdgmg_ctx* const* ctxs, int nctx, int nrhs,
                               const double* f_qp, double* u_qp, double* p_qp,
                               double* states, hdgmg_info* infos);

/* The adjoint of a batch (hdgmg_solve_adjoint per right-hand side, spread
 * over the contexts as hdgmg_solve_batch): f_qp, states, gu_qp and gf_qp
 * stacked over the batch; gnu device [n_cells] or NULL, ACCUMULATED with
 * dJ/dnu summed over the whole batch (each context collects its share in a
 * buffer of its own, added into gnu on the first context's stream at the
 * end). */
hdgmg_status hdgmg_solve_adjoint_batch(hdgmg_ctx* const* ctxs, int nctx, int nrhs,
                                       const double* f_qp, const double* states,
                                       const double* gu_qp, double* gf_qp,
                                       double* gnu, hdgmg_info* infos);

/* hdgmg_solve from an initial iterate: x0 (device, N_skel, may be NULL for
 * zero) starts the first inner solve of the AL-Uzawa iteration; for Picard
 * and Newton steps (Sec. 4.2) it is the previous step's skeleton vector
 * (state[0 .. N_skel)).  p_init (device, n_cells, may be NULL for zero) is
 * the initial piecewise-constant pressure p^(0) of the AL-Uzawa loop: zero
 * for the Picard form (nsOpEq-ALU); the previous pressure for a Newton
 * step, which makes the loop on (u_n, p_n) the paper's loop on the
 * increments (du, dp) from (0, 0).  With opts.oseen every later inner solve
 * starts from the latest iterate; the Stokes path starts every inner solve
 * from zero.  x0 and p_init may alias state. */
hdgmg_status hdgmg_solve_x0(hdgmg_ctx* ctx, const double* f_qp, const double* x0,
                            const double* p_init, double* u_qp, double* p_qp,
                            double* state, hdgmg_info* info);

/* Local post-processing (stPost): per cell the velocity u* in [P^{k+1}(K)]^2
 * with (grad u*_i, grad v)_K = (Lift_i., grad v)_K for every v in
 * P^{k+1}(K), Lift = -L_h / nu the scheme's gradient approximation (the
 * displayed right-hand side (L_h, grad v) drops the factor -1/nu of the
 * mixed form nu^-1 L + grad u = 0), and the cell mean of u_h; for k >= 1 it
 * converges at order k+2.
 *   f_qp     device [n_cells][n_q][2]: the source of the solve
 *   state    device [N_skel + n_cells]: the state written by hdgmg_solve
 *   ustar_qp device [n_cells][n_q][2] (output): u* at the data points
 * Tangential Dirichlet data and a wind set on the context are those of the
 * state.  ESTATE before hdgmg_assemble or with a Newton state set. */
hdgmg_status hdgmg_postprocess(hdgmg_ctx* ctx, const double* f_qp, const double* state, double* ustar_qp);

/* Wind of the Picard-linearised convection (Sec. 4.2: the previous
 * velocity), given by its values at the data points, w_qp device
 * [n_cells][n_q][2] (for instance u_qp of a previous solve), or NULL for no
 * convection.  The field must be a discrete velocity of the scheme (RT_k in
 * every cell, normal-continuous, zero normal component on the boundary):
 * its RT_k coefficients are recovered exactly by the data-rule L^2
 * projection.  Its facet fluxes define the lowest-order winds of MG_h (the
 * RT0 field with the same fluxes on the finest level, and on each coarser
 * level the sums over the two halves of every facet).  Requires
 * opts.oseen; takes effect at the next hdgmg_assemble (the context is
 * unassembled until then).  Returns ESTATE without opts.oseen, ENONFINITE
 * for a degenerate fit. */
hdgmg_status hdgmg_set_wind(hdgmg_ctx* ctx, const double* w_qp);

/* Newton linearisation (Sec. 4.2): the next hdgmg_assemble builds the
 * Jacobian of the scheme (nsWeak) at the previous state u_prev, i.e. the
 * Picard form plus C_h(du; u_prev, v) with the upwind switch frozen on
 * u_prev . n_K, and every load gains C_h(u_prev; u_prev, v), so that
 * hdgmg_solve returns the Newton iterate u_n = u_prev + du itself.
 *   state_prev  device [N_skel (+ n_cells, ignored)]: the skeleton vector of
 *          u_prev (as written by hdgmg_solve); copied during the call.  Its
 *          velocity at the data points must be the wind last given to
 *          hdgmg_set_wind; on boundary facets the tangential values are the
 *          Dirichlet data of hdgmg_set_dirichlet.  NULL: back to Picard.
 * The lowest-order levels of MG_h keep the Picard operators of the
 * RT0-projected wind.  hdgmg_set_wind clears the Newton state.  Requires
 * opts.oseen = 1, opts.transpose = 0, k >= 1 and a wind (else ESTATE). */
hdgmg_status hdgmg_set_newton(hdgmg_ctx* ctx, const double* state_prev);

/* Alg. 3 (Sec. 4.2) in the library: a Stokes solve, Picard steps until
 * ||u_n - u_{n-1}||_0 < eps_picard (or max_picard of them), then Newton
 * steps until ||u_n - u_{n-1}||_0 <= max(newton_rtol ||u_n||_0, newton_atol)
 * (or max_newton of them).  Each step after the first takes the previous
 * velocity as the wind (hdgmg_set_wind), a Newton step also its state
 * (hdgmg_set_newton), re-assembles, and starts from the previous skeleton
 * vector (a Newton step's AL-Uzawa loop from the previous pressure); norms
 * are L^2 norms by the data rule, computed on the device.  The context's
 * Dirichlet data (hdgmg_set_dirichlet) apply to every step.
 *   f_qp   device [n_cells][n_q][2] body force
 *   a      host, the parameters below
 *   u_qp, p_qp, state  device (outputs, as hdgmg_solve): the last step's
 *          solution; during step_fn they hold the current step's
 *   info   host or NULL: per step kind (0 Stokes, 1 Picard, 2 Newton),
 *          ||u_n - u_{n-1}||_0 (-1 for the first), status, Uzawa steps and
 *          summed inner iterations
 *   step_fn, step_ctx  NULL, or called on the calling thread after every
 *          step with the step's index, kind, status, norm and hdgmg_info
 *          (the outputs then hold that step's solution; the stream is
 *          synchronised)
 * Requires opts.oseen = 1, opts.transpose = 0 (ESTATE), Newton k >= 1.
 * Allocates two buffers (previous velocity and state) at the first call,
 * a third (the pseudo-time load) at the first call with dt_inv > 0.
 * Returns the largest status of the steps (NOT_CONVERGED if any inner
 * solve did not converge), or the first negative one. */
#define HDGMG_MAX_ALG3 128
typedef struct {
  double eps_picard;       /* Picard -> Newton switch (1e-4 in Sec. 5)      */
  double newton_rtol;      /* relative Newton stop (1e-8)                   */
  double newton_atol;      /* absolute Newton stop (1e-10)                  */
  int max_picard;          /* Picard step cap                                */
  int max_newton;          /* Newton step cap (0: Picard only)               */
  double dt_inv;           /* 0: none; > 0: the Stokes and Picard steps are
                              backward-Euler pseudo-time steps of size
                              1/dt_inv (Sec. 5.2.2): dt_inv u added to the
                              operator (beta + dt_inv) and dt_inv u_{n-1} to
                              the load (u_{-1} = 0); at their fixed point the
                              two cancel; the Newton steps solve the steady
                              system                                       */
} hdgmg_alg3_opts;
typedef struct {
  int n_steps;
  int kind[HDGMG_MAX_ALG3];
  double du[HDGMG_MAX_ALG3];
  int status[HDGMG_MAX_ALG3];
  int uzawa_steps[HDGMG_MAX_ALG3];
  int its[HDGMG_MAX_ALG3];
  double t_total;          /* host wall time of the call, seconds            */
} hdgmg_alg3_info;
typedef void (*hdgmg_alg3_step_fn)(void* step_ctx, int step, int kind, int status, double du,
                                   const hdgmg_info* info);
hdgmg_status hdgmg_picard_newton(hdgmg_ctx* ctx, const double* f_qp, const hdgmg_alg3_opts* a, double* u_qp,
                                 double* p_qp, double* state, hdgmg_alg3_info* info,
                                 hdgmg_alg3_step_fn step_fn, void* step_ctx);

/* Normal and tangential Dirichlet data on the Dirichlet boundary facets (an
 * inflow, Sec. 5.3): uhat_b device [n_boundary_facets][2][k+1] (facet
 * order of hdgmg_export what 3; component 0 the normal coefficients c^n
 * along n_F = (t_y, -t_x), 1 the tangential ones, modes as the skeleton's),
 * NULL: homogeneous.  The prescribed normal values enter the cells'
 * divergence: hdgmg_solve imposes div u_h = 0 with their flux included
 * (the AL-Uzawa update and the load's AL term carry it).  Without
 * do-nothing facets the data must have zero net flux.  With opts.oseen the
 * lowest-order levels' RT0 winds carry no flux through Dirichlet facets (as
 * without normal data).  Triangular meshes only. */
hdgmg_status hdgmg_set_dirichlet_full(hdgmg_ctx* ctx, const double* uhat_b);

/* Tangential Dirichlet data given as one constant velocity per boundary
 * facet, g_b device [n_boundary_facets][2] (facet order, hdgmg_export what
 * 3): the library sets uhat . t_F = g_b . t_F (mode 0; the exact facet L^2
 * projection of a constant) and the higher modes to zero, then applies them
 * as hdgmg_set_dirichlet does (the lid of a cavity: (1, 0) on the top
 * facets, zero elsewhere).  NULL restores homogeneous data.  Allocates two
 * small buffers at the first call. */
hdgmg_status hdgmg_set_dirichlet_velocity(hdgmg_ctx* ctx, const double* g_b);

/* Tangential Dirichlet data on the boundary facets (the lid of a cavity):
 * uhat_b device [n_boundary_facets][k+1], per boundary facet (in facet
 * order, see hdgmg_export what 3) the coefficients of uhat . t_F in the
 * facet Legendre basis; NULL restores homogeneous data.  The normal
 * component stays zero.  The data enter the condensed load (hdgmg_rhs, as
 * -S_K lambda_b) and the recovery; the array is read during the call. */
hdgmg_status hdgmg_set_dirichlet(hdgmg_ctx* ctx, const double* uhat_b);

/* Condensed load g (length N_skel, device, output) of f_qp (device), the
 * right-hand side F_{k,h} of stOptForm. */
hdgmg_status hdgmg_rhs(hdgmg_ctx* ctx, const double* f_qp, double* g);

/* y = A^eps_{k,h} x for device skeleton vectors x, y (N_skel). */
hdgmg_status hdgmg_apply(hdgmg_ctx* ctx, const double* x, double* y);

/* z = MG_hp(r, 0, m_p, m_h, q) (Alg. 2 with zero initial guess) for device
 * skeleton vectors r, z (N_skel); the preconditioner of the inner solve. */
hdgmg_status hdgmg_precondition(hdgmg_ctx* ctx, const double* r, double* z);

/* Inner solve A^eps x = b (stOpEq-ALU1) by flexible CG from x = 0,
 * preconditioned by MG_hp.  b, x device (N_skel).  *its (host) receives the
 * iteration count and *rel_res (host) the final ||r||/||r0||; either may be
 * NULL.  Returns OK, NOT_CONVERGED, EBREAKDOWN, ENONFINITE, EHIP. */
hdgmg_status hdgmg_inner_solve(hdgmg_ctx* ctx, const double* b, double* x,
                               int* its, double* rel_res);

/* hdgmg_inner_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same solve, kernels and arguments, but the Krylov
 * solvers' scalars and reduction partials live in a fixed file-scope device
 * array of the library (36,000 FP64 words = 288,000 bytes per GPU, held until
 * the process ends) instead of the context's workspace.  The call allocates
 * nothing (no hipMalloc / hipFree, no allocator callback); the context's
 * vectors, operators and preconditioner are those hdgmg_setup and
 * hdgmg_assemble allocated.  Every call on one GPU shares that array and
 * clears it first: calls that overlap on one GPU (contexts on different
 * streams or threads) race and must be serialised by the caller.  Limit:
 * FGMRES restart <= 64 (EINVAL beyond).  Results equal hdgmg_inner_solve's.
 * Triangular meshes only (ESTATE on a tetrahedral context). */
hdgmg_status hdgmg_inner_solve_noalloc(hdgmg_ctx* ctx, const double* b, double* x,
                                       int* its, double* rel_res);

/* Local recovery (Sec. 3.2): from state [N_skel + n_cells] (device) and
 * f_qp (device) compute u_qp and p_qp (device) at the data points.  The
 * pressure is returned as stored (the Uzawa iteration keeps it mean-free). */
hdgmg_status hdgmg_recover(hdgmg_ctx* ctx, const double* f_qp,
                           const double* state, double* u_qp, double* p_qp);

/* Sizes.  what: 0 n_cells (finest), 1 n_q, 2 N_skel, 3 levels J,
 * 4 device bytes held, 5 n_interior_facets (finest), 6 k,
 * 7 n_colours (finest level), 8 n_cells of level `level`,
 * 9 N of the lowest-order space of level `level` (d n_interior_facets),
 * 10 n_boundary_facets (finest), 11 the dimension d,
 * 12 bytes one MG_hp application moves in this implementation (every
 *    operator entry its launches use, in the stored layout and precision,
 *    plus vectors), 13 its compulsory bytes (every stored operator read
 *    once per use in packed symmetric form -- cell blocks n(n+1)/2 words,
 *    patch inverses n_s(n_s+1)/2, the coarsest inverse n_0(n_0+1)/2 -- in
 *    the storage precision, plus the vectors); both after hdgmg_assemble,
 * 14 nonzeros of the lowest-order transfer from level `level` - 1 into
 *    `level` (its transpose, the restriction, has the same count;
 *    1 <= level < J, after hdgmg_assemble; triangles only).
 * level counts from 0 (coarsest) and is ignored by 0..7 and 10..13. */
hdgmg_status hdgmg_query(const hdgmg_ctx* ctx, int what, int level, int64_t* value);

/* Copy an assembled operator to caller memory (device pointer dst, FP64):
 *   what 0: order-k cell blocks of A^eps [n_cells][6(k+1)][6(k+1)]
 *   what 1: lowest-order cell blocks of A^eps_{0,l} on level `level`
 *           [n_cells(level)][6][6]
 *   what 2: coordinates of the data points of the finest cells
 *           [n_cells][n_q][2]
 *   what 3: end points of the finest (Dirichlet) boundary facets -- every
 *           boundary facet but the do-nothing ones -- in facet order,
 *           [n_boundary_facets][2][2] (vertex v0 < v1 first: t_F points
 *           from the first to the second)
 *   what 4: data-rule weights times cell areas, w_q |K|, [n_cells][n_q]
 *   what 5: the tangential boundary coefficients the last
 *           hdgmg_set_dirichlet_velocity built, [n_boundary_facets][k+1]
 *           (ESTATE before the first such call)
 * Local DOF order inside a block: (local facet i, component c, mode j) ->
 * (i*2 + c)*m + j, local facet i opposite the cell's i-th stored vertex.
 * `bytes` is the size of dst; EINVAL if too small. */
hdgmg_status hdgmg_export(const hdgmg_ctx* ctx, int what, int level, void* dst,
                          size_t bytes);

/* Live kernel timing for roofline measurements.  While enabled for a
 * kernel class, every launch of that class on the context's stream is
 * timed by a pair of HIP events (the order-k cell apply and patch
 * relaxation launch through hipExtLaunchKernelGGL, whose dispatch records
 * the pair around the kernel itself; other launches are bracketed by event
 * records), and the preconditioner runs eagerly instead of as a graph
 * replay unless only class 3 is enabled; hdgmg_kernel_timer_read synchronises
 * the stream and returns the summed elapsed time (ms), the number of
 * launches and the summed algorithmic bytes of those launches (the bytes
 * the launch must move given the stored operators: every matrix entry it
 * uses read once, its vectors read/written once).  Enabling resets the
 * accumulators.  Classes:
 *   0 order-k vertex-patch Gauss-Seidel, one colour phase (Alg. 2 relaxation)
 *   1 order-k skeleton apply y = A^eps x
 *   2 lowest-order patch Gauss-Seidel phases launched per level (Alg. 1)
 *   3 whole preconditioner applications z = MG_hp(r)
 *   4 single-workgroup MG_h on the coarse levels (opts.coarse_dofs) */
hdgmg_status hdgmg_kernel_timer(hdgmg_ctx* ctx, int kernel_class, int enable);
hdgmg_status hdgmg_kernel_timer_read(hdgmg_ctx* ctx, int kernel_class, double* total_ms,
                                     int64_t* launches, double* bytes);

/* Message of the last failure on ctx (or of the last failed hdgmg_setup when
 * ctx is NULL).  The pointer stays valid until the next call on ctx. */
const char* hdgmg_last_error(const hdgmg_ctx* ctx);

/* Release the context and its device memory.  NULL is ignored. */
void hdgmg_destroy(hdgmg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
