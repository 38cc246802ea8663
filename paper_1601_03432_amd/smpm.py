"""Python binding of libsmpm (argument marshalling only).

Every numerical step runs in the HIP library; this module converts torch
tensors (device memory and streams) and numpy arrays (host-side setup data)
into the C ABI declared in include/smpm.h.  Importing it never computes
anything; constructing a Context loads libsmpm.so and fails loudly if the
library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmpm.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ESINGULAR, ENODEVICE = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
PROJ_L, PROJ_S, PROJ_P, PROJ_Q, PROJ_MEAN = 0, 1, 2, 3, 4
ROBIN = {"min": 0, "literal": 1, "reference": 2}  # smpm_robin
EXPORT_SCHUR, EXPORT_FLUX_SOLVE, EXPORT_PRECOND_INV, EXPORT_COARSE, EXPORT_COARSE_PINV = 0, 1, 2, 3, 4

# every symbol include/smpm.h declares
# recommended penalty alpha: tau = 2 alpha / (omega_0 h_perp^2)
DEFAULT_PENALTY = 8.0

ABI_SYMBOLS = (
    "smpm_default_opts", "smpm_plan", "smpm_setup", "smpm_plan_robin", "smpm_setup_robin", "smpm_destroy", "smpm_sizes", "smpm_stats", "smpm_slot_map",
    "smpm_node_coords", "smpm_quadrature_weights", "smpm_export", "smpm_null_vectors",
    "smpm_schur_apply", "smpm_schur_apply_prec", "smpm_precond_apply", "smpm_project", "smpm_solve",
    "smpm_boundary_transpose", "smpm_autotune", "smpm_solve_group",
    "smpm_project_noalloc", "smpm_last_error",
)


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("precision", C.c_int), ("transpose", C.c_int),
                ("variant", C.c_int), ("inner_tol", C.c_double), ("max_refine", C.c_int), ("graph", C.c_int),
                ("stop_rule", C.c_int), ("profile", C.c_int), ("block", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("refinements", C.c_int), ("rel_residual", C.c_double),
                ("removed_component", C.c_double), ("schur_precision", C.c_int),
                ("cycle_residual", C.c_double * 16), ("cycle_iterations", C.c_int * 16),
                ("history_len", C.c_int), ("history", C.c_double * 1001),
                ("phase_ms", C.c_double * 4)]


class TuneResult(C.Structure):
    _fields_ = [("nrhs", C.c_int), ("schur_columns_per_workgroup", C.c_int), ("schur_persistent", C.c_int),
                ("prereduce", C.c_int), ("schur_us", C.c_double), ("step_us", C.c_double)]


class PlanStats(C.Structure):
    _fields_ = [("element_classes", C.c_int64), ("block_classes", C.c_int64),
                ("schur_operator_bytes", C.c_int64), ("precond_operator_bytes", C.c_int64),
                ("flux_operator_bytes", C.c_int64), ("coarse_bytes", C.c_int64),
                ("coarse_singular", C.c_int32), ("has_coarse", C.c_int32),
                ("null_residual", C.c_double), ("null_iterations", C.c_int32), ("pad_", C.c_int32),
                ("schur_norm_bound", C.c_double)]


class SmpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsmpm error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libsmpm.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1601_03432_amd.build`")
    lib = C.CDLL(path)
    vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
    lib.smpm_last_error.restype = C.c_char_p
    lib.smpm_last_error.argtypes = [C.c_void_p]
    lib.smpm_default_opts.argtypes = [C.POINTER(SolveOpts)]
    lib.smpm_default_opts.restype = None
    lib.smpm_plan.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.POINTER(vp)]
    lib.smpm_setup.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, vp, C.POINTER(vp)]
    lib.smpm_plan_robin.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.c_int, C.POINTER(vp)]
    lib.smpm_setup_robin.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.c_int, vp, C.POINTER(vp)]
    lib.smpm_destroy.argtypes = [vp]
    lib.smpm_destroy.restype = None
    lib.smpm_sizes.argtypes = [vp, i64p, i64p, i64p]
    lib.smpm_stats.argtypes = [vp, C.POINTER(PlanStats)]
    lib.smpm_slot_map.argtypes = [vp, i64p]
    lib.smpm_node_coords.argtypes = [vp, dp, dp]
    lib.smpm_quadrature_weights.argtypes = [vp, dp]
    lib.smpm_export.argtypes = [vp, C.c_int, i64p, i64p, i64p, dp]
    lib.smpm_null_vectors.argtypes = [vp, dp, dp]
    lib.smpm_schur_apply.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp]
    lib.smpm_schur_apply_prec.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp]
    lib.smpm_precond_apply.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp]
    lib.smpm_project.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.c_int, vp]
    lib.smpm_project_noalloc.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.c_int, vp]
    lib.smpm_solve.argtypes = [vp, vp, vp, vp, C.c_int, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    lib.smpm_boundary_transpose.argtypes = [vp, vp, vp, C.c_int, vp]
    lib.smpm_autotune.argtypes = [vp, C.c_int, vp, C.POINTER(TuneResult)]
    lib.smpm_solve_group.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                     C.POINTER(C.c_int), C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    for name in ABI_SYMBOLS:
        if name not in ("smpm_destroy", "smpm_default_opts", "smpm_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise SmpmError(rc, _lib.smpm_last_error(None).decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i64ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _stream(torch, stream):
    if stream is None:
        # the current stream's handle without building a Stream object (when this
        # torch build exposes it)
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return C.c_void_p(raw(torch.cuda.current_device()))
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


@dataclass
class Info:
    iterations: int
    refinements: int
    rel_residual: float
    removed_component: float
    status: int
    schur_precision: int = FP64  # Schur operator precision of the last inner solve
    cycle_residuals: tuple = ()  # FP64 true residual at the start of each refinement cycle
    history: tuple = ()          # column 0, last GMRES cycle: residual estimates / stopping reference
    phase_ms: tuple = ()         # with profile=True: steps 1-3, 4-8, 9, total (ms)
    cycle_iterations: tuple = ()  # GMRES iterations of each solve / refinement cycle


def _info(si, rc):
    hist = list(si.cycle_residual)
    while len(hist) > 1 and hist[-1] == 0.0:
        hist.pop()
    ncyc = min(16, max(1, si.refinements))
    return Info(si.iterations, si.refinements, si.rel_residual, si.removed_component, rc, si.schur_precision,
                tuple(hist), tuple(si.history[:si.history_len]), tuple(si.phase_ms),
                tuple(si.cycle_iterations[:ncyc]))


class Context:
    """One grid: m_y x m_x elements with breakpoints, n GLL points, penalty alpha and
    the reading of the Robin operator ("min", "literal" or "reference", smpm_robin).

    device=False builds the host plan only (smpm_plan_robin); device=True also
    uploads it to the current GPU (smpm_setup_robin).
    """

    def __init__(self, m_y, m_x, n, x_breaks, y_breaks, penalty=DEFAULT_PENALTY, device=True, stream=None,
                 robin="min"):
        lib = load_library()
        xb = np.ascontiguousarray(x_breaks, np.float64)
        yb = np.ascontiguousarray(y_breaks, np.float64)
        if xb.size != m_x + 1 or yb.size != m_y + 1:
            raise ValueError("breakpoint arrays must have m_x+1 and m_y+1 entries")
        mode = ROBIN[robin] if isinstance(robin, str) else int(robin)
        h = C.c_void_p()
        if device:
            import torch
            rc = lib.smpm_setup_robin(m_y, m_x, n, _dptr(xb), _dptr(yb), float(penalty), mode,
                                      _stream(torch, stream), C.byref(h))
        else:
            rc = lib.smpm_plan_robin(m_y, m_x, n, _dptr(xb), _dptr(yb), float(penalty), mode, C.byref(h))
        _check(rc)
        self._h = h
        self._lib = lib
        self._opts_cache = {}  # SolveOpts by argument tuple (the library copies them)
        self.device = device
        self.robin = robin
        self.m_x, self.m_y, self.n = m_x, m_y, n
        r, k, d = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.smpm_sizes(h, C.byref(r), C.byref(k), C.byref(d)))
        self.r, self.k, self.d = r.value, k.value, d.value
        self.nbdry = 2 * n * (m_x + m_y)

    @classmethod
    def from_workload(cls, w, penalty=DEFAULT_PENALTY, device=True, robin="min"):
        return cls(w.m_y, w.m_x, w.n, w.x_breaks, w.y_breaks, penalty, device, robin=robin)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.smpm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- host queries
    def stats(self) -> dict:
        st = PlanStats()
        _check(self._lib.smpm_stats(self._h, C.byref(st)))
        return {name: getattr(st, name) for name, _ in PlanStats._fields_}

    def slot_map(self) -> np.ndarray:
        out = np.zeros(self.k, np.int64)
        _check(self._lib.smpm_slot_map(self._h, _i64ptr(out)))
        return out

    def node_coords(self):
        x = np.zeros(self.r)
        y = np.zeros(self.r)
        _check(self._lib.smpm_node_coords(self._h, _dptr(x), _dptr(y)))
        return x, y

    def quadrature_weights(self) -> np.ndarray:
        w = np.zeros(self.r)
        _check(self._lib.smpm_quadrature_weights(self._h, _dptr(w)))
        return w

    def boundary_arc(self):
        """Coordinates along the four edges in the boundary-data layout (S, N, W, E)."""
        x, y = self.node_coords()
        n, mx, my = self.n, self.m_x, self.m_y
        xs = np.concatenate([x[ix * n * n:ix * n * n + n] for ix in range(mx)])
        ys = np.concatenate([y[iy * mx * n * n:iy * mx * n * n + n * n:n] for iy in range(my)])
        return xs, xs.copy(), ys, ys.copy()

    def export(self, what):
        """Host copy of a setup operator: scipy COO for sparse kinds, dense array for C/G."""
        cnt = C.c_int64(0)
        _check(self._lib.smpm_export(self._h, what, C.byref(cnt), None, None, None))
        if what in (EXPORT_COARSE, EXPORT_COARSE_PINV):
            v = np.zeros(cnt.value)
            _check(self._lib.smpm_export(self._h, what, C.byref(cnt), None, None, _dptr(v)))
            return v.reshape(self.d, self.d)
        rows = np.zeros(cnt.value, np.int64)
        cols = np.zeros(cnt.value, np.int64)
        vals = np.zeros(cnt.value)
        _check(self._lib.smpm_export(self._h, what, C.byref(cnt), _i64ptr(rows), _i64ptr(cols), _dptr(vals)))
        import scipy.sparse as sp
        shape = (self.k, self.r) if what == EXPORT_FLUX_SOLVE else (self.k, self.k)
        return sp.coo_matrix((vals, (rows, cols)), shape=shape).tocsr()

    def null_vectors(self):
        uL = np.zeros(self.r)
        uS = np.zeros(self.k)
        _check(self._lib.smpm_null_vectors(self._h, _dptr(uL), _dptr(uS)))
        return uL, uS

    # ---------------------------------------------------------------- device calls
    @staticmethod
    def _as_cols(t, length):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
            raise TypeError("expected a CUDA float64 tensor")
        if t.dim() == 1:
            t = t.reshape(1, -1)
        if t.shape[-1] != length:
            raise ValueError(f"last dimension must be {length}")
        return t.contiguous()

    def schur_apply(self, v, transpose=False, stream=None):
        import torch
        v = self._as_cols(v, self.k)
        out = torch.empty_like(v)
        _check(self._lib.smpm_schur_apply(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr()),
                                          v.shape[0], int(transpose), _stream(torch, stream)))
        return out

    def schur_apply_into(self, v, out, transpose=False, stream=None):
        """S v written into a preallocated tensor `out` (same shape as v, both
        contiguous (columns, k) CUDA float64)."""
        import torch
        for t in (v, out):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                    and t.dim() == 2 and t.shape[1] == self.k and t.is_contiguous()):
                raise ValueError(f"expected contiguous CUDA float64 tensors of shape (columns, {self.k})")
        if out.shape != v.shape or out.data_ptr() == v.data_ptr():
            raise ValueError("out must match v in shape and must not alias it")
        _check(self._lib.smpm_schur_apply(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr()),
                                          v.shape[0], int(transpose), _stream(torch, stream)))
        return out

    def schur_apply_prec(self, v, out, precision, transpose=False, stream=None):
        """S v into `out` with the element operators in `precision` (FP64, MIXED_FP32 or
        MIXED_BF16; FP32 accumulation for the mixed ones); FP64 vectors."""
        import torch
        for t in (v, out):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                    and t.dim() == 2 and t.shape[1] == self.k and t.is_contiguous()):
                raise ValueError(f"expected contiguous CUDA float64 tensors of shape (columns, {self.k})")
        if out.shape != v.shape or out.data_ptr() == v.data_ptr():
            raise ValueError("out must match v in shape and must not alias it")
        _check(self._lib.smpm_schur_apply_prec(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr()),
                                               v.shape[0], int(transpose), int(precision), _stream(torch, stream)))
        return out

    def precond_apply(self, x, transpose=False, stream=None):
        import torch
        x = self._as_cols(x, self.k)
        out = torch.empty_like(x)
        _check(self._lib.smpm_precond_apply(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                            x.shape[0], int(transpose), _stream(torch, stream)))
        return out

    def project(self, which, x, transpose=False, stream=None):
        import torch
        length = self.r if which in (PROJ_L, PROJ_MEAN) else self.k
        x = self._as_cols(x, length)
        out = torch.empty_like(x)
        _check(self._lib.smpm_project(self._h, which, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                      x.shape[0], int(transpose), _stream(torch, stream)))
        return out

    def project_noalloc(self, which, x, out, transpose=False, stream=None):
        """smpm_project_noalloc: the projection into a preallocated `out` (same shape as
        x, contiguous (columns, length) CUDA float64; may be x itself) with the library's
        static scratch instead of its workspace (no device allocation)."""
        import torch
        length = self.r if which in (PROJ_L, PROJ_MEAN) else self.k
        for t in (x, out):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                    and t.dim() == 2 and t.shape[1] == length and t.is_contiguous()):
                raise ValueError(f"expected contiguous CUDA float64 tensors of shape (columns, {length})")
        if out.shape != x.shape:
            raise ValueError("out must match x in shape")
        _check(self._lib.smpm_project_noalloc(self._h, which, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                              x.shape[0], int(transpose), _stream(torch, stream)))
        return out

    def solve(self, f, g=None, tol=1e-10, maxit=400, variant=3, precision=FP64, transpose=False,
              inner_tol=1e-5, max_refine=20, stream=None, raise_on_noconv=True, graph=True, stop_rule=0,
              profile=False, block=False):
        import torch
        f = self._as_cols(f, self.r)
        nrhs = f.shape[0]
        gp = None
        if g is not None:
            if transpose:
                raise ValueError("the adjoint solve takes no boundary data")
            g = self._as_cols(g, self.nbdry)
            if g.shape[0] != nrhs:
                raise ValueError("g must have as many columns as f")
            gp = C.c_void_p(g.data_ptr())
        u = torch.empty_like(f)
        key = (tol, maxit, precision, transpose, variant, inner_tol, max_refine, graph, stop_rule, profile, block)
        opts = self._opts_cache.get(key)
        if opts is None:
            opts = SolveOpts(tol, maxit, precision, int(transpose), variant, inner_tol, max_refine, int(graph),
                             int(stop_rule), int(profile), int(block))
            if len(self._opts_cache) < 64:
                self._opts_cache[key] = opts
        info = SolveInfo()
        rc = self._lib.smpm_solve(self._h, C.c_void_p(f.data_ptr()), gp, C.c_void_p(u.data_ptr()), nrhs,
                                  C.byref(opts), C.byref(info), _stream(torch, stream))
        if rc != OK and not (rc == ENOCONV and not raise_on_noconv):
            _check(rc)
        return u, _info(info, rc)

    def autotune(self, nrhs, stream=None):
        """Time the launch-shape candidates for `nrhs` columns and keep the fastest
        (see smpm_autotune); returns the choice as a dict."""
        import torch
        r = TuneResult()
        _check(self._lib.smpm_autotune(self._h, int(nrhs), _stream(torch, stream), C.byref(r)))
        return {name: getattr(r, name) for name, _ in TuneResult._fields_}

    def boundary_transpose(self, mu, stream=None):
        """T^T mu: the gradient with respect to the Neumann data (columns of length
        2n(m_x+m_y), edges south, north, west, east) given mu = dLoss/d(f + T g)."""
        import torch
        mu = self._as_cols(mu, self.r)
        out = torch.empty(mu.shape[0], self.nbdry, dtype=torch.float64, device=mu.device)
        _check(self._lib.smpm_boundary_transpose(self._h, C.c_void_p(mu.data_ptr()), C.c_void_p(out.data_ptr()),
                                                 mu.shape[0], _stream(torch, stream)))
        return out


def solve_group(contexts, fs, gs=None, tol=1e-10, maxit=400, variant=3, precision=FP64, inner_tol=1e-5,
                max_refine=20, stream=None, raise_on_noconv=True, graph=True, block=False):
    """Solve independent problems concurrently (smpm_solve_group): problem i is
    contexts[i].solve(fs[i], gs[i] if gs else None, ...) with shared options.
    Returns [(u_i, Info_i)]."""
    import torch
    n = len(contexts)
    if len(fs) != n or (gs is not None and len(gs) != n):
        raise ValueError("one f (and g) per context")
    lib = contexts[0]._lib
    fs = [c._as_cols(f, c.r) for c, f in zip(contexts, fs)]
    gl = None
    if gs is not None:
        gl = []
        for c, f, g in zip(contexts, fs, gs):
            if g is not None:
                g = c._as_cols(g, c.nbdry)
                if g.shape[0] != f.shape[0]:
                    raise ValueError("g must have as many columns as f")
            gl.append(g)
    us = [torch.empty_like(f) for f in fs]
    vp = C.c_void_p
    arr = lambda xs: (vp * n)(*[vp(x) if isinstance(x, int) else x for x in xs])
    hs = arr([c._h for c in contexts])
    fp = arr([f.data_ptr() for f in fs])
    up = arr([u.data_ptr() for u in us])
    gp = None if gl is None else arr([None if g is None else g.data_ptr() for g in gl])
    nr = (C.c_int * n)(*[f.shape[0] for f in fs])
    opts = SolveOpts(tol, maxit, precision, 0, variant, inner_tol, max_refine, int(graph), 0, 0, int(block))
    infos = (SolveInfo * n)()
    rc = lib.smpm_solve_group(hs, n, fp, gp, up, nr, C.byref(opts), infos, _stream(torch, stream))
    if rc != OK and not (rc == ENOCONV and not raise_on_noconv):
        _check(rc)
    return [(u, _info(i, rc)) for u, i in zip(us, infos)]


_SchurSolve = None


def _schur_solve_function():
    """torch.autograd.Function: forward u = solve(f, g); backward by the adjoint solve
    (transpose = 1) giving dLoss/df = mu and dLoss/dg = T^T mu."""
    global _SchurSolve
    if _SchurSolve is not None:
        return _SchurSolve
    import torch

    class SchurSolve(torch.autograd.Function):
        @staticmethod
        def forward(actx, solver, opts, f, g):
            u, _ = solver.solve(f.detach(), None if g is None else g.detach(), **opts)
            actx.solver, actx.opts = solver, opts
            actx.f_shape = f.shape
            actx.g_shape = None if g is None else g.shape
            return u.reshape(f.shape)

        @staticmethod
        def backward(actx, gu):
            mu, _ = actx.solver.solve(gu.detach().contiguous(), transpose=True, **actx.opts)
            dg = None
            if actx.g_shape is not None and actx.needs_input_grad[3]:
                dg = actx.solver.boundary_transpose(mu).reshape(actx.g_shape)
            df = mu.reshape(actx.f_shape) if actx.needs_input_grad[2] else None
            return None, None, df, dg

    _SchurSolve = SchurSolve
    return SchurSolve


def solve_differentiable(solver: "Context", f, g=None, tol=1e-10, maxit=400, variant=3, precision=FP64,
                         inner_tol=1e-5, max_refine=20):
    """u = solver.solve(f, g) as a differentiable torch operation: its backward pass is
    the adjoint solve of the library (transposed Algorithm 3), so autograd gives
    dLoss/df and dLoss/dg.  f: (r,) or (nrhs, r); g: None or matching (.., nbdry)."""
    opts = dict(tol=tol, maxit=maxit, variant=variant, precision=precision, inner_tol=inner_tol,
                max_refine=max_refine)
    return _schur_solve_function().apply(solver, opts, f, g)
