"""Python binding of libhdgmg (include/hdgmg.h): argument marshalling only.

Every step of the solve runs in the HIP library; PyTorch provides device
memory and the stream.  Importing works without a GPU; creating a Solver
needs the built library (python -m paper_2303_06762_amd.build) and a GPU,
and raises otherwise -- there is no fallback.
"""
import ctypes
import os
import sys

_IS_FINALIZING = sys.is_finalizing

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdgmg.so")
_LIB = None

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "EMESH", -3: "ENOMEM",
          -4: "EHIP", -5: "ESTATE", -6: "EBREAKDOWN", -7: "ENONFINITE"}
MAX_UZAWA = 64


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_vertices", ctypes.c_int),
                ("coords", ctypes.POINTER(ctypes.c_double)), ("n_cells", ctypes.c_int),
                ("cells", ctypes.POINTER(ctypes.c_int32)), ("n_refine", ctypes.c_int),
                ("n_outflow", ctypes.c_int), ("outflow", ctypes.POINTER(ctypes.c_int32))]


class Opts(ctypes.Structure):
    _fields_ = [("m_relax", ctypes.c_int), ("m_smooth", ctypes.c_int), ("cycle", ctypes.c_int),
                ("vcycle_growth", ctypes.c_int), ("rtol", ctypes.c_double),
                ("atol", ctypes.c_double), ("max_it", ctypes.c_int), ("uzawa_max", ctypes.c_int),
                ("uzawa_tol", ctypes.c_double), ("coarse_dofs", ctypes.c_int),
                ("stream_dofs", ctypes.c_int), ("vcycle_precision", ctypes.c_int),
                ("oseen", ctypes.c_int), ("restart", ctypes.c_int), ("transpose", ctypes.c_int),
                ("coarse_dense", ctypes.c_int), ("rec_wide", ctypes.c_int), ("smoother", ctypes.c_int),
                ("additive", ctypes.c_int), ("patch_relax", ctypes.c_int), ("patch_smooth", ctypes.c_int),
                ("fused_phase", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("uzawa_steps", ctypes.c_int), ("its", ctypes.c_int * MAX_UZAWA),
                ("rel_res", ctypes.c_double * MAX_UZAWA), ("dp_l2", ctypes.c_double * MAX_UZAWA),
                ("div_l2", ctypes.c_double), ("t_solve", ctypes.c_double)]


def _info_dict(info):
    n = info.uzawa_steps
    return dict(uzawa_steps=n, its=list(info.its[:n]), rel_res=list(info.rel_res[:n]),
                dp_l2=list(info.dp_l2[:n]), div_l2=info.div_l2, t_solve=info.t_solve)


MAX_ALG3 = 128


class Alg3Opts(ctypes.Structure):
    _fields_ = [("eps_picard", ctypes.c_double), ("newton_rtol", ctypes.c_double),
                ("newton_atol", ctypes.c_double), ("max_picard", ctypes.c_int), ("max_newton", ctypes.c_int),
                ("dt_inv", ctypes.c_double)]


class Alg3Info(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int), ("kind", ctypes.c_int * MAX_ALG3),
                ("du", ctypes.c_double * MAX_ALG3), ("status", ctypes.c_int * MAX_ALG3),
                ("uzawa_steps", ctypes.c_int * MAX_ALG3), ("its", ctypes.c_int * MAX_ALG3),
                ("t_total", ctypes.c_double)]


ALG3_STEP_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.POINTER(Info))
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """Device memory of a context from PyTorch's caching allocator: each
    buffer the library asks for is a uint8 CUDA tensor kept alive here
    until the library frees it (hdgmg_alloc_fn / hdgmg_free_fn)."""

    def __init__(self, torch):
        self.torch = torch
        self.live = {}
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, _ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ptr, _ctx):
        self.live.pop(ptr, None)

    def bytes(self):
        return sum(t.numel() for t in self.live.values())


class HdgmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


SYMBOLS = ["hdgmg_default_opts", "hdgmg_setup", "hdgmg_assemble", "hdgmg_solve",
           "hdgmg_solve_adjoint", "hdgmg_solve_x0", "hdgmg_set_wind", "hdgmg_set_newton", "hdgmg_set_dirichlet",
           "hdgmg_set_dirichlet_velocity", "hdgmg_set_dirichlet_full", "hdgmg_picard_newton", "hdgmg_postprocess",
           "hdgmg_solve_batch", "hdgmg_solve_adjoint_batch",
           "hdgmg_rhs",
           "hdgmg_apply", "hdgmg_precondition", "hdgmg_inner_solve", "hdgmg_inner_solve_noalloc", "hdgmg_recover",
           "hdgmg_query", "hdgmg_export", "hdgmg_kernel_timer", "hdgmg_kernel_timer_read",
           "hdgmg_last_error", "hdgmg_destroy"]


def lib():
    """Load libhdgmg.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} missing: build it with `python -m paper_2303_06762_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    L.hdgmg_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.hdgmg_default_opts.restype = None
    L.hdgmg_setup.argtypes = [ctypes.POINTER(Mesh), i32, dbl, ctypes.POINTER(dbl), i32, dbl,
                              ctypes.POINTER(Opts), vp, ALLOC_FN, FREE_FN, vp, ctypes.POINTER(vp)]
    L.hdgmg_setup.restype = i32
    L.hdgmg_assemble.argtypes = [vp]
    L.hdgmg_assemble.restype = i32
    L.hdgmg_solve.argtypes = [vp, i32, vp, vp, vp, vp, ctypes.POINTER(Info)]
    L.hdgmg_solve.restype = i32
    L.hdgmg_solve_adjoint.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Info)]
    L.hdgmg_solve_adjoint.restype = i32
    L.hdgmg_picard_newton.argtypes = [vp, vp, ctypes.POINTER(Alg3Opts), vp, vp, vp, ctypes.POINTER(Alg3Info),
                                      ALG3_STEP_FN, vp]
    L.hdgmg_picard_newton.restype = i32
    L.hdgmg_solve_x0.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Info)]
    L.hdgmg_solve_x0.restype = i32
    for name in ("hdgmg_set_wind", "hdgmg_set_newton", "hdgmg_set_dirichlet", "hdgmg_set_dirichlet_velocity",
                 "hdgmg_set_dirichlet_full"):
        getattr(L, name).argtypes = [vp, vp]
        getattr(L, name).restype = i32
    for name in ("hdgmg_rhs", "hdgmg_apply", "hdgmg_precondition"):
        getattr(L, name).argtypes = [vp, vp, vp]
        getattr(L, name).restype = i32
    for name in ("hdgmg_inner_solve", "hdgmg_inner_solve_noalloc"):
        getattr(L, name).argtypes = [vp, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
        getattr(L, name).restype = i32
    L.hdgmg_solve_batch.argtypes = [ctypes.POINTER(vp), i32, i32, vp, vp, vp, vp, ctypes.POINTER(Info)]
    L.hdgmg_solve_batch.restype = i32
    L.hdgmg_solve_adjoint_batch.argtypes = [ctypes.POINTER(vp), i32, i32, vp, vp, vp, vp, vp,
                                            ctypes.POINTER(Info)]
    L.hdgmg_solve_adjoint_batch.restype = i32
    L.hdgmg_postprocess.argtypes = [vp, vp, vp, vp]
    L.hdgmg_postprocess.restype = i32
    L.hdgmg_recover.argtypes = [vp, vp, vp, vp, vp]
    L.hdgmg_recover.restype = i32
    L.hdgmg_query.argtypes = [vp, i32, i32, ctypes.POINTER(i64)]
    L.hdgmg_query.restype = i32
    L.hdgmg_export.argtypes = [vp, i32, i32, vp, ctypes.c_size_t]
    L.hdgmg_export.restype = i32
    L.hdgmg_kernel_timer.argtypes = [vp, i32, i32]
    L.hdgmg_kernel_timer.restype = i32
    L.hdgmg_kernel_timer_read.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                          ctypes.POINTER(dbl)]
    L.hdgmg_kernel_timer_read.restype = i32
    L.hdgmg_last_error.argtypes = [vp]
    L.hdgmg_last_error.restype = ctypes.c_char_p
    L.hdgmg_destroy.argtypes = [vp]
    L.hdgmg_destroy.restype = None
    _LIB = L
    return L


def default_opts(**kw):
    o = Opts()
    lib().hdgmg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """hdgmg context: setup(mesh hierarchy, k, beta, nu, gamma) -> assemble ->
    solve(f) -> (u, p).  Tensors are torch float64 CUDA tensors."""

    def __init__(self, coords, cells, n_refine, k, beta, nu, gamma, opts=None, stream=None, allocator="torch",
                 outflow=None, **kw):
        import torch
        self.torch = torch
        L = lib()
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        nu = np.ascontiguousarray(np.atleast_1d(np.asarray(nu, dtype=np.float64)))
        out = np.ascontiguousarray(np.asarray(outflow if outflow is not None else np.zeros((0, 2)), dtype=np.int32))
        self._keep = (coords, cells, nu, out)
        self.dim = int(coords.shape[1])
        m = Mesh(self.dim, len(coords), coords.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 len(cells), cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(n_refine),
                 len(out), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if len(out) else None)
        if opts is None:
            opts = default_opts(**kw)
        self.opts = opts
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        # device memory: PyTorch's caching allocator ("torch") or the
        # library's own hipMalloc ("hip")
        if allocator == "torch":
            self.allocator = TorchAllocator(torch)
            afn, ffn = self.allocator.alloc, self.allocator.free
        elif allocator == "hip":
            self.allocator = None
            afn, ffn = ALLOC_FN(), FREE_FN()
        else:
            raise ValueError("allocator must be 'torch' or 'hip'")
        h = ctypes.c_void_p()
        st = L.hdgmg_setup(ctypes.byref(m), int(k), float(beta),
                           nu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(nu),
                           float(gamma), ctypes.byref(opts), ctypes.c_void_p(stream.cuda_stream),
                           afn, ffn, None, ctypes.byref(h))
        if st != 0:
            raise HdgmgError(st, L.hdgmg_last_error(None).decode())
        self._h = h
        self.k = int(k)
        self.n_cells = self.query(0)
        self.n_q = self.query(1)
        self.n_skel = self.query(2)
        self.levels = self.query(3)

    def close(self):
        """Release the context (also done on garbage collection)."""
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.hdgmg_destroy(h)
        self._h = None

    def __del__(self):
        # at interpreter exit the process releases the device memory; the
        # allocator callbacks must not run into a half torn-down torch
        try:
            if _IS_FINALIZING():
                return
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=(0,)):
        if st not in allow:
            raise HdgmgError(st, lib().hdgmg_last_error(self._h).decode())
        return st

    def _vec(self, n):
        return self.torch.empty(n, dtype=self.torch.float64, device="cuda")

    def query(self, what, level=0):
        v = ctypes.c_int64()
        self._check(lib().hdgmg_query(self._h, what, level, ctypes.byref(v)))
        return v.value

    def assemble(self):
        self._check(lib().hdgmg_assemble(self._h))

    def rhs(self, f_qp):
        g = self._vec(self.n_skel)
        self._check(lib().hdgmg_rhs(self._h, _ptr(f_qp), _ptr(g)))
        return g

    def apply(self, x):
        y = self._vec(self.n_skel)
        self._check(lib().hdgmg_apply(self._h, _ptr(x), _ptr(y)))
        return y

    def precondition(self, r, out=None):
        z = self._vec(self.n_skel) if out is None else out
        self._check(lib().hdgmg_precondition(self._h, _ptr(r), _ptr(z)))
        return z

    def inner_solve(self, b, x=None):
        x = self._vec(self.n_skel) if x is None else x
        its, rel = ctypes.c_int(), ctypes.c_double()
        st = self._check(lib().hdgmg_inner_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(its),
                                                 ctypes.byref(rel)), allow=(0, 1))
        return x, its.value, rel.value, st

    def inner_solve_noalloc(self, b, x):
        """inner_solve into the caller's x with the library's fixed device
        scratch (no allocation during the call)."""
        its, rel = ctypes.c_int(), ctypes.c_double()
        st = self._check(lib().hdgmg_inner_solve_noalloc(self._h, _ptr(b), _ptr(x), ctypes.byref(its),
                                                         ctypes.byref(rel)), allow=(0, 1))
        return x, its.value, rel.value, st

    def recover(self, f_qp, state):
        u = self.torch.empty((self.n_cells, self.n_q, self.dim), dtype=self.torch.float64, device="cuda")
        p = self.torch.empty((self.n_cells, self.n_q), dtype=self.torch.float64, device="cuda")
        self._check(lib().hdgmg_recover(self._h, _ptr(f_qp), _ptr(state), _ptr(u), _ptr(p)))
        return u, p

    def solve(self, f_qp, x0=None, p_init=None):
        """Returns (u_qp, p_qp, state, info dict, status).  x0: initial
        skeleton iterate (N_skel), e.g. state[:n_skel] of a previous solve;
        p_init: initial P0 pressure of the AL-Uzawa loop (n_cells), e.g.
        state[n_skel:] of the previous state for a Newton step."""
        u = self.torch.empty((self.n_cells, self.n_q, self.dim), dtype=self.torch.float64, device="cuda")
        p = self.torch.empty((self.n_cells, self.n_q), dtype=self.torch.float64, device="cuda")
        state = self._vec(self.n_skel + self.n_cells)
        info = Info()
        x0p = ctypes.c_void_p(None) if x0 is None else _ptr(x0)
        pip = ctypes.c_void_p(None) if p_init is None else _ptr(p_init)
        st = self._check(lib().hdgmg_solve_x0(self._h, _ptr(f_qp), x0p, pip, _ptr(u), _ptr(p), _ptr(state),
                                              ctypes.byref(info)), allow=(0, 1))
        return u, p, state, _info_dict(info), st

    def solve_adjoint(self, f_qp, state, gu_qp, gnu=None, adj_state=None):
        """Adjoint of solve() for dJ/du_qp = gu_qp: returns (gf_qp, gnu,
        adj_state, info dict, status); gnu (n_cells) is accumulated into
        when given, else a new zeroed tensor."""
        t = self.torch
        gf = t.empty((self.n_cells, self.n_q, self.dim), dtype=t.float64, device="cuda")
        if gnu is None:
            gnu = t.zeros(self.n_cells, dtype=t.float64, device="cuda")
        if adj_state is None:
            adj_state = self._vec(self.n_skel + self.n_cells)
        info = Info()
        st = self._check(lib().hdgmg_solve_adjoint(self._h, 1, _ptr(f_qp), _ptr(state), _ptr(gu_qp), _ptr(gf),
                                                   _ptr(gnu), _ptr(adj_state), ctypes.byref(info)),
                         allow=(0, 1))
        return gf, gnu, adj_state, _info_dict(info), st

    def solve_many(self, f_qp):
        """hdgmg_solve over nrhs = f_qp.shape[0] sources stacked
        [nrhs][n_cells][n_q][d]: returns (u, p, states, infos, status)."""
        t = self.torch
        n = f_qp.shape[0]
        u = t.empty((n, self.n_cells, self.n_q, self.dim), dtype=t.float64, device="cuda")
        p = t.empty((n, self.n_cells, self.n_q), dtype=t.float64, device="cuda")
        states = t.zeros((n, self.n_skel + self.n_cells), dtype=t.float64, device="cuda")
        infos = (Info * n)()
        st = self._check(lib().hdgmg_solve(self._h, n, _ptr(f_qp.contiguous()), _ptr(u), _ptr(p), _ptr(states),
                                           infos), allow=(0, 1))
        return u, p, states, [_info_dict(i) for i in infos], st

    def solve_adjoint_many(self, f_qp, states, gu_qp):
        """hdgmg_solve_adjoint over nrhs = f_qp.shape[0] stacked forward
        sources, states and dJ/du: returns (gf [nrhs][n_cells][n_q][d], gnu
        [n_cells] summed over the right-hand sides, adj_states, infos,
        status)."""
        t = self.torch
        n = f_qp.shape[0]
        gf = t.empty((n, self.n_cells, self.n_q, self.dim), dtype=t.float64, device="cuda")
        gnu = t.zeros(self.n_cells, dtype=t.float64, device="cuda")
        adj = t.zeros((n, self.n_skel + self.n_cells), dtype=t.float64, device="cuda")
        infos = (Info * n)()
        st = self._check(lib().hdgmg_solve_adjoint(self._h, n, _ptr(f_qp.contiguous()), _ptr(states.contiguous()),
                                                   _ptr(gu_qp.contiguous()), _ptr(gf), _ptr(gnu), _ptr(adj),
                                                   infos), allow=(0, 1))
        return gf, gnu, adj, [_info_dict(i) for i in infos], st

    def set_wind(self, w_qp):
        """Picard wind at the data points [n_cells][n_q][2] (None: no
        convection); re-assemble afterwards."""
        self._check(lib().hdgmg_set_wind(self._h, ctypes.c_void_p(None) if w_qp is None else _ptr(w_qp)))

    def postprocess(self, f_qp, state):
        """u* (stPost) at the data points [n_cells][n_q][2] of a solved state."""
        out = self.torch.empty((self.n_cells, self.n_q, self.dim), dtype=self.torch.float64, device="cuda")
        self._check(lib().hdgmg_postprocess(self._h, _ptr(f_qp), _ptr(state), _ptr(out)))
        return out

    def set_newton(self, state_prev):
        """Newton linearisation at the previous state (its skeleton vector,
        whose velocity is the current wind); None: Picard.  Re-assemble
        afterwards."""
        self._check(lib().hdgmg_set_newton(self._h, ctypes.c_void_p(None) if state_prev is None
                                           else _ptr(state_prev)))

    def set_dirichlet(self, uhat_b):
        """Tangential boundary coefficients [n_boundary_facets][k+1] (None:
        homogeneous)."""
        self._check(lib().hdgmg_set_dirichlet(self._h, ctypes.c_void_p(None) if uhat_b is None else _ptr(uhat_b)))

    def data_weights(self):
        """w_q |K| at the data points [n_cells][n_q] (integrals of data-point fields)."""
        out = self.torch.empty((self.n_cells, self.n_q), dtype=self.torch.float64, device="cuda")
        self._check(lib().hdgmg_export(self._h, 4, 0, _ptr(out), out.numel() * 8))
        return out

    def boundary_facets(self):
        """End points [n_boundary_facets][2][2] of the boundary facets (facet order)."""
        nb = self.query(10)
        out = self.torch.empty((max(nb, 1), 2, 2), dtype=self.torch.float64, device="cuda")
        self._check(lib().hdgmg_export(self._h, 3, 0, _ptr(out), out.numel() * 8))
        return out[:nb]

    def set_dirichlet_full(self, uhat_b):
        """hdgmg_set_dirichlet_full: normal and tangential coefficients
        [n_boundary_facets][2][k+1] (None: homogeneous)."""
        self._check(lib().hdgmg_set_dirichlet_full(self._h, ctypes.c_void_p(None) if uhat_b is None
                                                   else _ptr(uhat_b.contiguous())))

    def set_dirichlet_velocity(self, g_b):
        """hdgmg_set_dirichlet_velocity: tangential data from one constant
        velocity per boundary facet (None: homogeneous)."""
        self._check(lib().hdgmg_set_dirichlet_velocity(self._h, ctypes.c_void_p(None) if g_b is None
                                                       else _ptr(g_b.contiguous())))

    def dirichlet_data(self):
        """The tangential boundary coefficients [n_boundary_facets][k+1] the
        last set_dirichlet_velocity built (hdgmg_export 5)."""
        nb = self.query(10)
        out = self.torch.empty((max(nb, 1), self.k + 1), dtype=self.torch.float64, device="cuda")
        self._check(lib().hdgmg_export(self._h, 5, 0, _ptr(out), out.numel() * 8))
        return out[:nb]

    def timer(self, kernel_class, enable=True):
        """Enable/disable the live event timer of a kernel class (see hdgmg.h)."""
        self._check(lib().hdgmg_kernel_timer(self._h, kernel_class, int(enable)))

    def timer_read(self, kernel_class):
        """(total ms, launches, algorithmic bytes) since the timer was enabled."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self._check(lib().hdgmg_kernel_timer_read(self._h, kernel_class, ctypes.byref(ms),
                                                  ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def data_points(self):
        out = self.torch.empty((self.n_cells, self.n_q, self.dim), dtype=self.torch.float64, device="cuda")
        self._check(lib().hdgmg_export(self._h, 2, 0, _ptr(out), out.numel() * 8))
        return out

    def export(self, what, level=0):
        if self.dim == 3:
            nK = 6 * (self.k + 1) * (self.k + 2) if what == 0 else 12
        else:
            nK = 6 * (self.k + 1) if what == 0 else 6
        n = self.n_cells if what == 0 else self.query(8, level)
        out = self.torch.empty((n, nK, nK), dtype=self.torch.float64, device="cuda")
        self._check(lib().hdgmg_export(self._h, what, level, _ptr(out), out.numel() * 8))
        return out


def _make_function():
    import torch

    class StokesSolve(torch.autograd.Function):
        """u_qp = solve(f_qp; nu) for a batch of sources [nrhs][n_cells][n_q][2]
        on an assembled Solver.  `nu` [n_cells] must hold the per-cell
        viscosities the Solver was set up with; it is an input only so that
        autograd can return dJ/dnu (summed over the batch).  The forward
        states are kept for the adjoint (no Krylov data)."""

        @staticmethod
        def forward(ctx, solver, f_qp, nu):
            pool = list(solver) if isinstance(solver, (list, tuple)) else [solver]
            us, _, states, _ = solve_batch(pool, f_qp)
            ctx.pool = pool
            ctx.save_for_backward(f_qp, states)
            return us

        @staticmethod
        def backward(ctx, gu):
            f_qp, states = ctx.saved_tensors
            gf, gnu = solve_adjoint_batch(ctx.pool, f_qp, states, gu)
            return None, gf, gnu

    return StokesSolve


def _batch_handles(pool):
    for p_ in pool:
        if getattr(p_, "_h", None) is None or not p_._h.value:
            raise ValueError("closed Solver in a batch")
    return (ctypes.c_void_p * len(pool))(*[p_._h.value for p_ in pool])


def _batch_error(pool, st):
    for p_ in pool:
        msg = lib().hdgmg_last_error(p_._h).decode()
        if msg:
            return HdgmgError(st, msg)
    return HdgmgError(st, "batch solve failed")


def solve_batch(pool, f_qp):
    """hdgmg_solve_batch: the sources f_qp [nrhs][n_cells][n_q][2] spread over
    the identical, assembled Solvers of `pool` (one HIP stream each) and
    solved concurrently.  Returns (u [nrhs][n_cells][n_q][2], p, states
    [nrhs][N_skel + n_cells], info dicts)."""
    torch = pool[0].torch
    s0 = pool[0]
    f_qp = f_qp.detach().contiguous()
    n = f_qp.shape[0]
    u = torch.empty((n, s0.n_cells, s0.n_q, 2), dtype=torch.float64, device="cuda")
    p = torch.empty((n, s0.n_cells, s0.n_q), dtype=torch.float64, device="cuda")
    states = torch.empty((n, s0.n_skel + s0.n_cells), dtype=torch.float64, device="cuda")
    infos = (Info * max(n, 1))()
    torch.cuda.synchronize()  # the inputs come from the caller's stream
    st = lib().hdgmg_solve_batch(_batch_handles(pool), len(pool), n, _ptr(f_qp), _ptr(u), _ptr(p), _ptr(states),
                                 infos)
    if st < 0:
        raise _batch_error(pool, st)
    ds = [dict(uzawa_steps=i.uzawa_steps, its=list(i.its[:i.uzawa_steps]), div_l2=i.div_l2, t_solve=i.t_solve)
          for i in infos[:n]]
    return u, p, states, ds


def solve_adjoint_batch(pool, f_qp, states, gu_qp):
    """hdgmg_solve_adjoint_batch for dJ/du = gu_qp of a batch solved by
    solve_batch: returns (dJ/df [nrhs][n_cells][n_q][2], dJ/dnu [n_cells]
    summed over the batch)."""
    torch = pool[0].torch
    s0 = pool[0]
    f_qp, states, gu_qp = (t_.detach().contiguous() for t_ in (f_qp, states, gu_qp))
    n = f_qp.shape[0]
    gf = torch.empty_like(f_qp)
    gnu = torch.zeros(s0.n_cells, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = lib().hdgmg_solve_adjoint_batch(_batch_handles(pool), len(pool), n, _ptr(f_qp), _ptr(states),
                                         _ptr(gu_qp), _ptr(gf), _ptr(gnu), None)
    if st < 0:
        raise _batch_error(pool, st)
    return gf, gnu


def solver_pool(n, coords, cells, n_refine, k, beta, nu, gamma, **kw):
    """n identical, assembled Solvers, each on a HIP stream of its own
    (default priority), for solve_batch / stokes_solve over a batch of
    sources."""
    import torch
    pool = [Solver(coords, cells, n_refine, k, beta, nu, gamma, stream=torch.cuda.Stream(), **kw)
            for _ in range(n)]
    for s in pool:
        s.assemble()
    return pool


_STOKES_SOLVE = None


def stokes_solve(solver, f_qp, nu):
    """Differentiable batched solve: u_qp = stokes_solve(solver, f_qp, nu).
    solver: an assembled Solver, or a list of identical ones (solver_pool)
    over which the batch is spread so that the solves run concurrently."""
    global _STOKES_SOLVE
    if _STOKES_SOLVE is None:
        _STOKES_SOLVE = _make_function()
    return _STOKES_SOLVE.apply(solver, f_qp, nu)


def picard(solver, f_qp, steps, dirichlet=None):
    """Stokes solve then `steps` Picard steps (Sec. 4.2) on an opts.oseen
    Solver: each step takes the previous velocity as the wind and the
    previous skeleton vector as the initial iterate.  Returns the list of
    (u_qp, p_qp, state, info, status) per solve."""
    if dirichlet is not None:
        solver.set_dirichlet(dirichlet)
    solver.set_wind(None)
    solver.assemble()
    out = []
    x0 = None
    for n in range(steps + 1):
        if n > 0:
            solver.set_wind(out[-1][0])
            solver.assemble()
        u, p, state, info, st = solver.solve(f_qp, x0=x0)
        out.append((u, p, state, info, st))
        x0 = state[:solver.n_skel]
    return out


def picard_newton(solver, f_qp, dirichlet=None, eps_picard=1e-4, newton_rtol=1e-8, newton_atol=1e-10,
                  max_picard=50, max_newton=20, dt_inv=0.0):
    """Alg. 3 on an opts.oseen Solver through hdgmg_picard_newton (the loop,
    its norms and the Picard -> Newton switch run in the library): a Stokes
    solve, Picard steps until ||u_n - u_{n-1}||_0 < eps_picard, then Newton
    steps until ||u_n - u_{n-1}||_0 <= max(newton_rtol ||u_n||_0,
    newton_atol).  dt_inv > 0: the Stokes and Picard steps are backward-Euler
    pseudo-time steps of size 1/dt_inv.  Returns a list of dicts (kind, u, p,
    state, info, status, du) per solve, the fields copied in the library's
    per-step callback."""
    torch = solver.torch
    if dirichlet is not None:
        solver.set_dirichlet(dirichlet)
    u = torch.empty((solver.n_cells, solver.n_q, 2), dtype=torch.float64, device="cuda")
    p = torch.empty((solver.n_cells, solver.n_q), dtype=torch.float64, device="cuda")
    state = solver._vec(solver.n_skel + solver.n_cells)
    kinds = ("stokes", "picard", "newton")
    out = []

    def step(_ctx, n, kind, st, du, info_p):
        i = info_p.contents
        out.append(dict(kind=kinds[kind], u=u.clone(), p=p.clone(), state=state.clone(), status=st,
                        du=None if du < 0 else du, info=_info_dict(i)))

    cb = ALG3_STEP_FN(step)
    a = Alg3Opts(eps_picard, newton_rtol, newton_atol, max_picard, max_newton, dt_inv)
    info = Alg3Info()
    solver._check(lib().hdgmg_picard_newton(solver._h, _ptr(f_qp), ctypes.byref(a), _ptr(u), _ptr(p), _ptr(state),
                                            ctypes.byref(info), cb, None), allow=(0, 1))
    return out
