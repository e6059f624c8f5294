"""ctypes binding of the oracle's C implementation (``adr_oracle.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Every function here is
argument marshalling around the C code; the arithmetic lives in the C file,
which cites the paper passage each routine follows.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None

OK, ERR_ARG, MAXIT, BREAKDOWN_RHO, OMEGA_ZERO, ZERO_PIVOT, NONFINITE, INACCURATE = 0, -1, 1, 2, 3, 4, 5, 6
MAX_RESTARTS = 8   # default restarts from the current iterate (see or_bicgstab)
UPWIND, CENTERED = 0, 1
DIRICHLET, NEUMANN = 0, 1

_D = ctypes.POINTER(ctypes.c_double)


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("hist_len", ctypes.c_int32), ("half_step", ctypes.c_int32),
                ("bnorm", ctypes.c_double), ("true_relres", ctypes.c_double),
                ("restarts", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Class(ctypes.Structure):
    _fields_ = [("pe_x", ctypes.c_double), ("pe_y", ctypes.c_double), ("g_y", ctypes.c_double),
                ("neg_offdiag", ctypes.c_int64), ("nonneg_diag", ctypes.c_int64),
                ("expect_fail", ctypes.c_int32), ("pad", ctypes.c_int32)]


def lib():
    """Load ``liboracle.so``, building it first if it is missing or stale."""
    global _lib
    if _lib is None:
        if (not os.path.exists(_build.LIB)
                or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        i32, f64, i64 = ctypes.c_int32, ctypes.c_double, ctypes.c_int64
        L.or_u_exact.restype = f64
        L.or_u_exact.argtypes = [f64, f64, f64, f64]
        L.or_tables.argtypes = [f64, f64, i32, i32] + [_D] * 7
        L.or_f_point.restype = f64
        L.or_f_point.argtypes = [f64] * 9
        L.or_boundary.argtypes = [f64, f64, i32, i32] + [_D] * 6
        L.or_forcing.argtypes = [f64, f64, f64, i32, i32, _D]
        L.or_assemble.restype = ctypes.c_int
        L.or_assemble.argtypes = [f64, f64, f64, i32, i32, i32, i32, _D, f64] + [_D] * 6
        L.or_assemble_data.restype = ctypes.c_int
        L.or_assemble_data.argtypes = [f64, f64, f64, i32, i32, i32, i32, _D, _D, f64] + [_D] * 10
        L.or_classify.restype = ctypes.c_int
        L.or_classify.argtypes = [f64, f64, f64, i32, i32, i32, i32, f64, ctypes.POINTER(_Class)]
        L.or_spmv.argtypes = [i32, i32] + [_D] * 7
        L.or_ilu0.restype = ctypes.c_int
        L.or_ilu0.argtypes = [i32, i32] + [_D] * 8 + [ctypes.POINTER(i64)]
        L.or_lsolve.argtypes = [i32, i32] + [_D] * 4
        L.or_usolve.argtypes = [i32, i32] + [_D] * 5
        L.or_dot.restype = f64
        L.or_dot.argtypes = [i64, _D, _D]
        L.or_maxabs.restype = f64
        L.or_maxabs.argtypes = [i64, _D]
        L.or_bicgstab.restype = ctypes.c_int
        L.or_bicgstab.argtypes = ([i32, i32] + [_D] * 10 + [_D, _D, f64, i32, i32, i32, i32, _D, _D, _D,
                                                             ctypes.POINTER(_Info)])
        L.or_lsolve_f32.argtypes = [i32, i32] + [_D] * 4
        L.or_usolve_f32.argtypes = [i32, i32] + [_D] * 5
        L.or_max_error.restype = f64
        L.or_max_error.argtypes = [f64, f64, i32, i32, i32, _D, _D]
        _lib = L
    return _lib


def _p(a):
    """Pointer to a C-contiguous float64 array (or NULL for None)."""
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Problem:
    """Assembled five-diagonal system (arrays of length nx*ny, x fastest)."""
    eps: float
    X: float
    Y: float
    nx: int
    ny: int
    scheme: int
    bc: int
    S: np.ndarray
    W: np.ndarray
    C: np.ndarray
    E: np.ndarray
    N: np.ndarray
    rhs: np.ndarray

    @property
    def n(self):
        return self.nx * self.ny


def u_exact(x, y, X, Y):
    return lib().or_u_exact(float(x), float(y), float(X), float(Y))


def tables(X, Y, nx, ny):
    """x, y, a, b, ex, ey, eb tables (see ``or_tables``)."""
    x, a, ex = (np.zeros(nx) for _ in range(3))
    y, b, ey, eb = (np.zeros(ny) for _ in range(4))
    lib().or_tables(X, Y, nx, ny, _p(x), _p(y), _p(a), _p(b), _p(ex), _p(ey), _p(eb))
    return dict(x=x, y=y, a=a, b=b, ex=ex, ey=ey, eb=eb)


def f_point(eps, X, Y, x, y):
    """Manufactured forcing at one point, through the same C routine."""
    import math
    a = 1.0 + x * x
    return lib().or_f_point(eps, X, Y, x, y, a, math.exp(-x / X), math.exp(-y / Y), math.exp(-y))


def forcing(eps, X, Y, nx, ny):
    f = np.zeros(nx * ny)
    lib().or_forcing(eps, X, Y, nx, ny, _p(f))
    return f


def boundary(X, Y, nx, ny):
    out = dict(u_x0=np.zeros(ny), u_xX=np.zeros(ny), g_xX=np.zeros(ny),
               u_y0=np.zeros(nx), u_yY=np.zeros(nx), g_yY=np.zeros(nx))
    lib().or_boundary(X, Y, nx, ny, _p(out["u_x0"]), _p(out["u_xX"]), _p(out["u_y0"]),
                      _p(out["u_yY"]), _p(out["g_xX"]), _p(out["g_yY"]))
    return out


def assemble(eps, X, Y, nx, ny, scheme=UPWIND, bc=DIRICHLET, field=None, amp=0.0):
    n = nx * ny
    arrs = [np.zeros(n) for _ in range(6)]
    g = None if field is None else _f64(field).ravel()
    if g is not None:
        assert g.size == n
    rc = lib().or_assemble(float(eps), float(X), float(Y), int(nx), int(ny), int(scheme),
                           int(bc), _p(g), float(amp), *[_p(a) for a in arrs])
    if rc != OK:
        raise ValueError("or_assemble rejected its arguments (status %d)" % rc)
    return Problem(eps, X, Y, nx, ny, scheme, bc, *arrs)


def assemble_data(eps, X, Y, nx, ny, scheme=UPWIND, bc=DIRICHLET, f=None, u_x0=None, u_xX=None,
                  u_y0=None, u_yY=None):
    """Assembly from user problem data (see ``or_assemble_data``): f (nx*ny),
    u_x0, u_xX (ny each), u_y0, u_yY (nx each); for bc = NEUMANN u_xX and u_yY
    are the normal derivatives.  None = the manufactured value."""
    n = nx * ny
    arrs = [np.zeros(n) for _ in range(6)]
    conv = lambda a, m: None if a is None else _f64(a).ravel()
    data = [conv(f, n), conv(u_x0, ny), conv(u_xX, ny), conv(u_y0, nx), conv(u_yY, nx)]
    for a, m in zip(data, (n, ny, ny, nx, nx)):
        assert a is None or a.size == m
    rc = lib().or_assemble_data(float(eps), float(X), float(Y), int(nx), int(ny), int(scheme), int(bc),
                                _p(data[0]), None, 0.0, *[_p(a) for a in data[1:]], *[_p(a) for a in arrs])
    if rc != OK:
        raise ValueError("or_assemble_data rejected its arguments (status %d)" % rc)
    return Problem(eps, X, Y, nx, ny, scheme, bc, *arrs)


@dataclass
class Classification:
    pe_x: float
    pe_y: float
    g_y: float
    neg_offdiag: int
    nonneg_diag: int
    expect_fail: bool


def classify(eps, X, Y, nx, ny, scheme=UPWIND, bc=DIRICHLET, tol=1e-10):
    c = _Class()
    rc = lib().or_classify(float(eps), float(X), float(Y), int(nx), int(ny), int(scheme), int(bc), float(tol),
                           ctypes.byref(c))
    if rc != OK:
        raise ValueError("or_classify rejected its arguments (status %d)" % rc)
    return Classification(c.pe_x, c.pe_y, c.g_y, c.neg_offdiag, c.nonneg_diag, bool(c.expect_fail))


def spmv(P, x):
    x = _f64(x)
    v = np.zeros(P.n)
    lib().or_spmv(P.nx, P.ny, _p(P.S), _p(P.W), _p(P.C), _p(P.E), _p(P.N), _p(x), _p(v))
    return v


@dataclass
class Factors:
    """Five-point triangular factors: L = I + (lw at k-1, ls at k-nx),
    U = diag(1/invd) + (ue at k+1, un at k+nx)."""
    lw: np.ndarray
    ls: np.ndarray
    invd: np.ndarray
    ue: np.ndarray
    un: np.ndarray
    status: int = OK
    bad: int = -1


def ilu0(P):
    lw, ls, invd = (np.zeros(P.n) for _ in range(3))
    bad = ctypes.c_int64(-1)
    st = lib().or_ilu0(P.nx, P.ny, _p(P.S), _p(P.W), _p(P.C), _p(P.E), _p(P.N),
                       _p(lw), _p(ls), _p(invd), ctypes.byref(bad))
    return Factors(lw, ls, invd, P.E.copy(), P.N.copy(), st, bad.value)


def lsolve(nx, ny, F, q):
    q = _f64(q)
    y = np.zeros(nx * ny)
    lib().or_lsolve(nx, ny, _p(F.lw), _p(F.ls), _p(q), _p(y))
    return y


def usolve(nx, ny, F, y):
    y = _f64(y)
    z = np.zeros(nx * ny)
    lib().or_usolve(nx, ny, _p(F.ue), _p(F.un), _p(F.invd), _p(y), _p(z))
    return z


def lsolve_f32(nx, ny, F, q):
    q = _f64(q)
    y = np.zeros(nx * ny)
    lib().or_lsolve_f32(nx, ny, _p(F.lw), _p(F.ls), _p(q), _p(y))
    return y


def usolve_f32(nx, ny, F, y):
    y = _f64(y)
    z = np.zeros(nx * ny)
    lib().or_usolve_f32(nx, ny, _p(F.ue), _p(F.un), _p(F.invd), _p(y), _p(z))
    return z


def round_factors_f32(F):
    """The factors as the mixed-precision preconditioner stores them: every
    entry rounded to the nearest float (kept in float64 arrays)."""
    r = lambda a: a.astype(np.float32).astype(np.float64)
    return Factors(r(F.lw), r(F.ls), r(F.invd), r(F.ue), r(F.un), F.status, F.bad)


def dot(x, y):
    x, y = _f64(x).ravel(), _f64(y).ravel()
    return lib().or_dot(x.size, _p(x), _p(y))


def maxabs(x):
    x = _f64(x).ravel()
    return lib().or_maxabs(x.size, _p(x))


@dataclass
class Solve:
    x: np.ndarray
    hist_l2: np.ndarray
    hist_max: np.ndarray
    status: int
    iters: int
    half_step: bool
    bnorm: float
    true_relres: float
    restarts: int = 0


def bicgstab(P, F, tol=1e-10, maxit=1000, x0=None, abs_tol=False, b=None, sweep_f32=False,
             max_restarts=MAX_RESTARTS):
    """BiCGSTAB of Section 5.2 (``or_bicgstab``).  max_restarts < 0 keeps the
    recursive stopping test alone (the appendix's solver); otherwise a
    convergence of the recursion is confirmed on the true residual, with up to
    max_restarts restarts from the current iterate."""
    rhs = P.rhs if b is None else _f64(b)
    x = np.zeros(P.n)
    h2 = np.zeros(maxit + 1)
    hm = np.zeros(maxit + 1)
    info = _Info()
    x0p = None if x0 is None else _f64(x0)
    lib().or_bicgstab(P.nx, P.ny, _p(P.S), _p(P.W), _p(P.C), _p(P.E), _p(P.N),
                      _p(F.lw), _p(F.ls), _p(F.invd), _p(F.ue), _p(F.un),
                      _p(rhs), _p(x0p), float(tol), int(bool(abs_tol)), int(maxit), int(bool(sweep_f32)),
                      int(max_restarts), _p(x), _p(h2), _p(hm), ctypes.byref(info))
    hl = info.hist_len
    return Solve(x, h2[:hl].copy(), hm[:hl].copy(), info.status, info.iters,
                 bool(info.half_step), info.bnorm, info.true_relres, info.restarts)


def max_error(P, sol):
    sol = _f64(sol)
    return lib().or_max_error(P.X, P.Y, P.nx, P.ny, P.bc, _p(sol), None)


def grid(P, sol):
    sol = _f64(sol)
    g = np.zeros((P.ny + 2) * (P.nx + 2))
    lib().or_max_error(P.X, P.Y, P.nx, P.ny, P.bc, _p(sol), _p(g))
    return g.reshape(P.ny + 2, P.nx + 2)
