"""MI355X-native ILU(0)-preconditioned BiCGSTAB for the 2-D advection-diffusion
problem of Datta & Carrasco Heres (arXiv:1308.5215).

Thin Python layer over the C ABI of ``libadr.so`` (include/adr.h): PyTorch
supplies device memory and the stream; every step of the solver runs in the
library's HIP kernels.

    import paper_1308_5215_amd as adr
    prob = adr.assemble(eps=0.1, X=1, Y=1, nx=64, ny=64, scheme="upwind", bc="dirichlet")
    prob.ilu0()
    res = prob.solve(tol=1e-10, maxit=1000)      # res.x is a CUDA tensor
"""
import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import (OK, MAXIT, BREAKDOWN_RHO, OMEGA_ZERO, ZERO_PIVOT, NONFINITE, INACCURATE, UPWIND, CENTERED,
                   DIRICHLET, NEUMANN_XY, FP64, FP32_FACTORS, FP32_SWEEPS, AdrError)

__all__ = ["assemble", "assemble_batch", "solve", "classify", "stream_copy", "amplification", "WarmStartNet",
           "cnn_param_count", "Problem", "Batch", "SolveResult", "BatchResult", "InstanceClass", "dot", "AdrError",
           "OK", "MAXIT", "BREAKDOWN_RHO", "OMEGA_ZERO", "ZERO_PIVOT", "NONFINITE", "INACCURATE", "UPWIND",
           "CENTERED", "DIRICHLET", "NEUMANN_XY", "FP64", "FP32_FACTORS", "FP32_SWEEPS"]

_SCHEMES = {"upwind": UPWIND, "hybrid": UPWIND, "centered": CENTERED, UPWIND: UPWIND, CENTERED: CENTERED}
_BCS = {"dirichlet": DIRICHLET, "neumann": NEUMANN_XY, DIRICHLET: DIRICHLET, NEUMANN_XY: NEUMANN_XY}
_PREC = {"fp64": FP64, "fp32_factors": FP32_FACTORS, "fp32_sweeps": FP32_SWEEPS,
         FP64: FP64, FP32_FACTORS: FP32_FACTORS, FP32_SWEEPS: FP32_SWEEPS}
_D = ctypes.POINTER(ctypes.c_double)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f64(t, n, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError("%s must be a CUDA float64 tensor" % name)
    if t.numel() != n or not t.is_contiguous():
        raise ValueError("%s must be contiguous with %d elements" % (name, n))
    return ctypes.c_void_p(t.data_ptr())


def _host_ptr(a):
    return a.ctypes.data_as(_D)


@dataclass
class SolveResult:
    x: object            # CUDA float64 tensor (nx*ny)
    status: int
    iters: int
    half_step: bool
    hist_l2: np.ndarray
    hist_max: np.ndarray
    bnorm: float
    true_relres: float
    solve_ms: float
    restarts: int = 0

    @property
    def amplification(self):
        """||r^{k+1}|| / ||r^k|| (the paper's amplification factor, Section 6.5)."""
        h = self.hist_l2
        return h[1:] / h[:-1]


class _Workspace:
    """Caller-owned device memory for the buffers a problem creates after
    assembly (adr_workspace_bytes / adr_bind_workspace)."""

    def workspace_bytes(self, precision="fp64"):
        return int(_lib.load().adr_workspace_bytes(self._h, _PREC[precision]))

    def bind_workspace(self, buf):
        """buf: a contiguous CUDA tensor of at least workspace_bytes() bytes
        (torch's allocator aligns it); call before ilu0.  The problem keeps a
        reference to it until it is destroyed."""
        if not (buf.is_cuda and buf.is_contiguous()):
            raise ValueError("the workspace must be a contiguous CUDA tensor")
        nbytes = buf.numel() * buf.element_size()
        _lib.check(_lib.load().adr_bind_workspace(self._h, ctypes.c_void_p(buf.data_ptr()), nbytes))
        self._ws = buf


class Problem(_Workspace):
    """One assembled five-point system on the current device."""

    def __init__(self, handle, eps, X, Y, nx, ny, scheme, bc, stream):
        self._h = handle
        self.eps, self.X, self.Y, self.nx, self.ny = eps, X, Y, nx, ny
        self.scheme, self.bc = scheme, bc
        self.n = nx * ny
        self._stream = stream
        self.precision = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.load().adr_destroy(h)
            except (AttributeError, TypeError):   # interpreter shutdown
                pass
            self._h = None

    def close(self):
        self.__del__()

    # -- the three calls of the method --
    def ilu0(self, precision="fp64"):
        prec = _PREC[precision]
        bad = ctypes.c_int64(-1)
        st = _lib.check(_lib.load().adr_ilu0(self._h, prec, ctypes.byref(bad)))
        if st == ZERO_PIVOT:
            raise AdrError(st, "zero or non-finite pivot at unknown %d" % bad.value)
        self.precision = prec
        return self

    def solve(self, tol=1e-10, maxit=1000, x0=None, out=None):
        torch = _torch()
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        xp = _dev_f64(x, self.n, "out")
        x0p = None if x0 is None else _dev_f64(x0, self.n, "x0")
        h2 = np.zeros(maxit + 1)
        hm = np.zeros(maxit + 1)
        info = _lib.SolveInfo()
        st = _lib.check(_lib.load().adr_bicgstab_solve(self._h, float(tol), int(maxit), x0p, xp,
                                                        _host_ptr(h2), _host_ptr(hm), ctypes.byref(info)))
        hl = info.hist_len
        return SolveResult(x, st, info.iters, bool(info.half_step), h2[:hl].copy(), hm[:hl].copy(),
                           info.bnorm, info.true_relres, info.solve_ms, info.restarts)

    def set_max_restarts(self, n):
        """Restarts allowed by the true-residual confirmation (default 8;
        -1: the recursive residual's test alone)."""
        _lib.check(_lib.load().adr_set_max_restarts(self._h, int(n)))

    def max_error(self, x):
        """max |U - u_exact| over all grid nodes (adr_max_error)."""
        out = np.zeros(1)
        _lib.check(_lib.load().adr_max_error(self._h, _dev_f64(x, self.n, "x"), _host_ptr(out)))
        return float(out[0])

    # -- inspection and single steps --
    def get_dia(self):
        arrs = [np.zeros(self.n) for _ in range(6)]
        _lib.check(_lib.load().adr_get_dia(self._h, *[_host_ptr(a) for a in arrs]))
        return dict(zip(("S", "W", "C", "E", "N", "rhs"), arrs))

    def set_dia(self, S, W, C, E, N, rhs):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (S, W, C, E, N, rhs)]
        for a in arrs:
            if a.size != self.n:
                raise ValueError("each array needs %d entries" % self.n)
        _lib.check(_lib.load().adr_set_dia(self._h, *[_host_ptr(a) for a in arrs]))
        self.precision = None

    def get_factors(self):
        arrs = [np.zeros(self.n) for _ in range(3)]
        _lib.check(_lib.load().adr_get_factors(self._h, *[_host_ptr(a) for a in arrs]))
        return dict(zip(("lw", "ls", "invd"), arrs))

    def spmv(self, x, out=None):
        torch = _torch()
        v = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        _lib.check(_lib.load().adr_spmv(self._h, _dev_f64(x, self.n, "x"), _dev_f64(v, self.n, "out")))
        return v

    def precond(self, q, out=None):
        torch = _torch()
        z = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        _lib.check(_lib.load().adr_precond(self._h, _dev_f64(q, self.n, "q"), _dev_f64(z, self.n, "out")))
        return z

    def lsolve(self, q, out=None):
        torch = _torch()
        y = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        _lib.check(_lib.load().adr_lsolve(self._h, _dev_f64(q, self.n, "q"), _dev_f64(y, self.n, "out")))
        return y

    def usolve(self, y, out=None):
        torch = _torch()
        z = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        _lib.check(_lib.load().adr_usolve(self._h, _dev_f64(y, self.n, "y"), _dev_f64(z, self.n, "out")))
        return z

    def set_sweep_rows(self, rows):
        """Strip height of the wavefront kernels: 16 or 32 rows (0: the default, 32)."""
        _lib.check(_lib.load().adr_set_sweep_rows(self._h, int(rows)))

    def set_sweep_ring(self, mode):
        """32-row sweep ring: -1 automatic, 0 deep (one workgroup per CU), 1 compact (two)."""
        _lib.check(_lib.load().adr_set_sweep_ring(self._h, int(mode)))

    @property
    def sweep_ring(self):
        return int(_lib.load().adr_sweep_ring(self._h))

    def use_stencil_tables(self, enable=True):
        """Allow (default) or forbid reading S, W, E, N from the separable
        stencil tables instead of the full diagonals (no result changes)."""
        _lib.check(_lib.load().adr_use_stencil_tables(self._h, 1 if enable else 0))

    @property
    def stencil_tables(self):
        """True if the next solve reads the stencil tables."""
        return bool(_lib.load().adr_stencil_tables(self._h))

    @property
    def last_call_ms(self):
        """Device time (ms) of the kernels of the last spmv / precond /
        lsolve / usolve call (HIP events on the problem's stream)."""
        return float(_lib.load().adr_last_call_ms(self._h))

    @property
    def device_bytes(self):
        return int(_lib.load().adr_device_bytes(self._h))


def _problem_data(f, u_x0, u_xX, u_y0, u_yY, keep):
    """adr_problem_data from Python values: None (manufactured), a scalar
    (broadcast), a host array, or (f only) a CUDA float64 tensor.  Arrays
    are kept alive in `keep` for the duration of the call."""
    torch = _torch()
    d = _lib.ProblemData()

    def host(v):
        a = np.ascontiguousarray(np.atleast_1d(np.asarray(v, dtype=np.float64)).ravel())
        keep.append(a)
        return ctypes.c_void_p(a.ctypes.data), a.size

    if f is not None:
        if isinstance(f, torch.Tensor) and f.is_cuda:
            if f.dtype != torch.float64 or not f.is_contiguous():
                raise TypeError("f must be a contiguous CUDA float64 tensor")
            keep.append(f)
            d.f, d.f_len, d.f_on_device = ctypes.c_void_p(f.data_ptr()), f.numel(), 1
        else:
            d.f, d.f_len = host(f)
    for name, v in (("u_x0", u_x0), ("u_xX", u_xX), ("u_y0", u_y0), ("u_yY", u_yY)):
        if v is not None:
            ptr, ln = host(v)
            setattr(d, name, ptr)
            setattr(d, name + "_len", ln)
    return d


def assemble(eps, X, Y, nx, ny, scheme="upwind", bc="dirichlet", field=None, amp=0.0, stream=None,
             f=None, u_x0=None, u_xX=None, u_y0=None, u_yY=None):
    """Section 4 assembly on the device; see adr_assemble in include/adr.h.
    field: optional CUDA float64 tensor (nx*ny) added to the manufactured
    forcing with amplitude amp * max|f_man|.
    f, u_x0, u_xX, u_y0, u_yY: the caller's forcing and boundary data
    (adr_assemble_data; for Neumann sides u_xX / u_yY are the normal
    derivatives): each None (manufactured), a scalar, or an array (f may be a
    CUDA tensor)."""
    L = _lib.load()
    sch, b = _SCHEMES[scheme], _BCS[bc]
    sh = _stream_handle(stream)
    h = ctypes.c_void_p()
    if any(v is not None for v in (f, u_x0, u_xX, u_y0, u_yY)):
        if field is not None:
            raise ValueError("give either field/amp or the problem data f, u_x0, ...")
        keep = []
        d = _problem_data(f, u_x0, u_xX, u_y0, u_yY, keep)
        _lib.check(L.adr_assemble_data(float(eps), float(X), float(Y), int(nx), int(ny), sch, b, ctypes.byref(d),
                                       sh, ctypes.byref(h)))
    else:
        fp = None if field is None else _dev_f64(field, int(nx) * int(ny), "field")
        _lib.check(L.adr_assemble(float(eps), float(X), float(Y), int(nx), int(ny), sch, b, fp, float(amp),
                                  sh, ctypes.byref(h)))
    return Problem(h, float(eps), float(X), float(Y), int(nx), int(ny), sch, b, stream)


@dataclass
class InstanceClass:
    """adr_classify: cell Peclet numbers, the Neumann growth exponent g_y,
    counts of negative couplings and of non-negative diagonal entries, and
    whether the solve is expected to fail."""
    pe_x: float
    pe_y: float
    g_y: float
    neg_offdiag: int
    nonneg_diag: int
    expect_fail: bool


def classify(eps, X, Y, nx, ny, scheme="upwind", bc="dirichlet", tol=1e-10):
    """What an instance's discretisation looks like before it is solved, and
    whether a solve to tol is expected to fail (adr_classify; Section 6.3
    mesh Reynolds number)."""
    c = _lib.InstanceClass()
    _lib.check(_lib.load().adr_classify(float(eps), float(X), float(Y), int(nx), int(ny), _SCHEMES[scheme],
                                        _BCS[bc], float(tol), ctypes.byref(c)))
    return InstanceClass(c.pe_x, c.pe_y, c.g_y, c.neg_offdiag, c.nonneg_diag, bool(c.expect_fail))


def stream_copy(src, dst, stream=None):
    """dst = src with the library's streaming copy kernel (adr_stream_copy)."""
    n = src.numel()
    _lib.check(_lib.load().adr_stream_copy(_dev_f64(src, n, "src"), _dev_f64(dst, n, "dst"), n,
                                           _stream_handle(stream)))
    return dst


def solve(eps, X, Y, nx, ny, scheme="upwind", bc="dirichlet", tol=1e-10, maxit=1000, precision="fp64",
          x0=None, field=None, amp=0.0, stream=None):
    """The method in one call: assemble (Section 4), ILU(0) (Section 5.1) and
    BiCGSTAB (Section 5.2) to ||r|| < tol ||b||.  Returns
    (x, hist_l2, hist_max, iters, status): x a CUDA float64 tensor, the
    residual histories as numpy arrays, the pass count and the adr_status."""
    prob = assemble(eps, X, Y, nx, ny, scheme, bc, field=field, amp=amp, stream=stream)
    prob.ilu0(precision)
    r = prob.solve(tol=tol, maxit=maxit, x0=x0)
    return r.x, r.hist_l2, r.hist_max, r.iters, r.status


def amplification(hist):
    """||r^{k+1}|| / ||r^k|| of a residual history (the paper's amplification
    factor, Section 6.5)."""
    h = np.asarray(hist, dtype=np.float64)
    return h[1:] / h[:-1]


@dataclass
class BatchResult:
    x: object              # batched CUDA float64 tensor
    status: np.ndarray     # per instance
    iters: np.ndarray
    half_step: np.ndarray
    hist_l2: list          # per instance arrays
    hist_max: list
    bnorm: np.ndarray
    true_relres: np.ndarray
    solve_ms: float
    overall: int           # adr_batch_solve's return value
    restarts: np.ndarray = None


class Batch(_Workspace):
    """Many independent instances advanced together (adr_batch_* calls)."""

    def __init__(self, handle, params, stream):
        self._h = handle
        self.params = params
        self._stream = stream
        L = _lib.load()
        cnt = ctypes.c_int32(0)
        _lib.check(L.adr_batch_layout(self._h, ctypes.byref(cnt), None))
        self.count = cnt.value
        offs = (ctypes.c_int64 * (self.count + 1))()
        _lib.check(L.adr_batch_layout(self._h, None, offs))
        self.offsets = np.array(offs[:], dtype=np.int64)
        self.n = int(self.offsets[-1])
        self.precision = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.load().adr_destroy(h)
            except (AttributeError, TypeError):   # interpreter shutdown
                pass
            self._h = None

    def close(self):
        self.__del__()

    def ilu0(self, precision="fp64"):
        prec = _PREC[precision]
        bad = (ctypes.c_int64 * self.count)()
        st = _lib.check(_lib.load().adr_batch_ilu0(self._h, prec, bad))
        if st == ZERO_PIVOT:
            raise AdrError(st, "zero pivot in instances %s" % [k for k in range(self.count) if bad[k] >= 0])
        self.precision = prec
        return self

    def autotune(self):
        rows = ctypes.c_int32(0)
        ms = ctypes.c_double(0.0)
        _lib.check(_lib.load().adr_autotune(self._h, ctypes.byref(rows), ctypes.byref(ms)))
        return rows.value, ms.value

    def set_sweep_rows(self, rows):
        """Strip height of the wavefront kernels: 16 or 32 rows (0: the default, 32)."""
        _lib.check(_lib.load().adr_set_sweep_rows(self._h, int(rows)))

    def set_sweep_ring(self, mode):
        """32-row sweep ring: -1 automatic, 0 deep (one workgroup per CU), 1 compact (two)."""
        _lib.check(_lib.load().adr_set_sweep_ring(self._h, int(mode)))

    @property
    def sweep_ring(self):
        return int(_lib.load().adr_sweep_ring(self._h))

    def use_stencil_tables(self, enable=True):
        _lib.check(_lib.load().adr_use_stencil_tables(self._h, 1 if enable else 0))

    @property
    def stencil_tables(self):
        return bool(_lib.load().adr_stencil_tables(self._h))

    def split(self, x):
        """Per-instance views of a batched vector."""
        return [x[self.offsets[k]:self.offsets[k + 1]] for k in range(self.count)]

    def solve(self, tol=1e-10, maxit=1000, x0=None, out=None):
        torch = _torch()
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        xp = _dev_f64(x, self.n, "out")
        x0p = None if x0 is None else _dev_f64(x0, self.n, "x0")
        h2 = np.zeros(self.count * (maxit + 1))
        hm = np.zeros(self.count * (maxit + 1))
        info = (_lib.SolveInfo * self.count)()
        st = _lib.check(_lib.load().adr_batch_solve(self._h, float(tol), int(maxit), x0p, xp,
                                                     _host_ptr(h2), _host_ptr(hm), info))
        h2 = h2.reshape(self.count, maxit + 1)
        hm = hm.reshape(self.count, maxit + 1)
        return BatchResult(
            x, np.array([i.status for i in info]), np.array([i.iters for i in info]),
            np.array([bool(i.half_step) for i in info]),
            [h2[k, :info[k].hist_len].copy() for k in range(self.count)],
            [hm[k, :info[k].hist_len].copy() for k in range(self.count)],
            np.array([i.bnorm for i in info]), np.array([i.true_relres for i in info]),
            info[0].solve_ms if self.count else 0.0, st, np.array([i.restarts for i in info]))

    def set_max_restarts(self, n):
        _lib.check(_lib.load().adr_set_max_restarts(self._h, int(n)))

    def max_error(self, x):
        """Per instance max |U - u_exact| over all grid nodes (adr_max_error)."""
        out = np.zeros(self.count)
        _lib.check(_lib.load().adr_max_error(self._h, _dev_f64(x, self.n, "x"), _host_ptr(out)))
        return out

    # -- learned initial guess (include/adr_cnn.h) --
    def features(self, first=0, count=None, out=None):
        """Input fields of instances [first, first + count) as a bfloat16
        tensor [count, ny+2, nx+2, 32] (adr_cnn_features)."""
        torch = _torch()
        count = self.count - first if count is None else int(count)
        p = self.params[first]
        shape = (count, p["ny"] + 2, p["nx"] + 2, 32)
        t = out if out is not None else torch.empty(shape, dtype=torch.bfloat16, device="cuda")
        if t.dtype != torch.bfloat16 or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError("out must be a contiguous bfloat16 tensor of shape %s" % (shape,))
        _lib.check(_lib.load().adr_cnn_features(self._h, int(first), count, ctypes.c_void_p(t.data_ptr())))
        return t

    def warm_start(self, net, out=None):
        """The network's initial guess for every instance with the zero-guess
        fallback (adr_batch_warm_start).  Returns (x0 tensor, used flags)."""
        torch = _torch()
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        used = (ctypes.c_int32 * self.count)()
        _lib.check(_lib.load().adr_batch_warm_start(self._h, net._h, _dev_f64(x, self.n, "out"), used))
        return x, np.array(used[:], dtype=bool)


def assemble_batch(eps, X, Y, nx, ny, scheme, bc, field=None, amp=0.0, stream=None):
    """Batched Section 4 assembly (adr_batch_assemble).  Every argument but
    field/amp/stream is a sequence with one entry per instance; field is an
    optional batched CUDA float64 tensor."""
    count = len(eps)
    f64a = lambda v: (ctypes.c_double * count)(*[float(a) for a in v])
    i32a = lambda v: (ctypes.c_int32 * count)(*[int(a) for a in v])
    sch = [_SCHEMES[s_] for s_ in scheme]
    bcs = [_BCS[b_] for b_ in bc]
    total = int(sum(int(a) * int(b) for a, b in zip(nx, ny)))
    fp = None if field is None else _dev_f64(field, total, "field")
    h = ctypes.c_void_p()
    _lib.check(_lib.load().adr_batch_assemble(count, f64a(eps), f64a(X), f64a(Y), i32a(nx), i32a(ny), i32a(sch),
                                              i32a(bcs), fp, float(amp), _stream_handle(stream), ctypes.byref(h)))
    params = [dict(eps=float(eps[k]), X=float(X[k]), Y=float(Y[k]), nx=int(nx[k]), ny=int(ny[k]), scheme=sch[k],
                   bc=bcs[k]) for k in range(count)]
    return Batch(h, params, stream)


from .cnn import WarmStartNet, param_count as cnn_param_count  # noqa: E402


def dot(x, y, stream=None):
    """Double-double inner product of two CUDA float64 vectors (adr_dot)."""
    n = x.numel()
    out = ctypes.c_double(0.0)
    _lib.check(_lib.load().adr_dot(_dev_f64(x, n, "x"), _dev_f64(y, n, "y"), n, _stream_handle(stream),
                                   ctypes.byref(out)))
    return out.value
