"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is either
printed in the paper (``tests/golden/paper_tables.json``, each with its table),
a closed form, an independent library routine (LAPACK, SciPy sparse), exact
rational arithmetic, or a structural invariant of the method.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import core, dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


@pytest.fixture(scope="module")
def tables():
    with open(GOLDEN) as fh:
        return json.load(fh)


SCHEME = {"upwind": core.UPWIND, "centered": core.CENTERED}
BC = {"dirichlet": core.DIRICHLET, "neumann": core.NEUMANN}


def agrees_to_printed(value, printed):
    """True if `value` matches `printed` to its printed significant digits,
    allowing 1.5 units in the last printed digit (the centered-Neumann entry of
    Table 6.1, printed 0.1256, comes out 0.12571: its maximum sits on the
    reconstructed corner node, whose treatment the paper varied; every other
    printed error agrees within one unit)."""
    s = repr(printed)
    mant = s.split("e")[0].replace("-", "").replace(".", "").lstrip("0")
    digits = max(len(mant), 1)
    exp10 = math.floor(math.log10(abs(printed)))
    unit = 10.0 ** (exp10 - digits + 1)
    return abs(value - printed) <= 1.5 * unit + 1e-15


# --------------------------------------------------------------------------
# Section 3: the manufactured forcing
# --------------------------------------------------------------------------

def _u(x, y, X, Y):
    return np.exp(-x / X) * (1 - np.exp(-y / Y)) * y


def _f_from_derivatives(eps, X, Y, x, y):
    """f = eps (u_xx + u_yy) + a u_x + b u_y with the derivatives of Section 3."""
    ux = -(1 / X) * np.exp(-x / X) * (1 - np.exp(-y / Y)) * y
    uxx = (1 / X ** 2) * np.exp(-x / X) * (1 - np.exp(-y / Y)) * y
    uy = np.exp(-x / X) * (1 - np.exp(-y / Y)) + (y / Y) * np.exp(-(x / X + y / Y))
    uyy = (2 / Y - y / Y ** 2) * np.exp(-(x / X + y / Y))
    a = 1 + x ** 2
    b = X * np.exp(-y)
    return eps * (uxx + uyy) + a * ux + b * uy


@pytest.mark.parametrize("eps,X,Y", [(4.0, 4.0, 4.0), (0.01, 1.0, 1.0), (1e-3, 2.0, 1.0), (0.3, 0.5, 2.0)])
def test_forcing_matches_section3_derivatives(orc, eps, X, Y):
    rng = np.random.default_rng(11)
    for _ in range(200):
        x, y = rng.uniform(0, X), rng.uniform(0, Y)
        f = orc.f_point(eps, X, Y, x, y)
        ref = _f_from_derivatives(eps, X, Y, x, y)
        assert abs(f - ref) <= 1e-13 * (1 + abs(ref))


@pytest.mark.parametrize("eps,X,Y", [(1.0, 1.0, 1.0), (0.01, 1.0, 1.0), (0.1, 2.0, 0.5)])
def test_forcing_by_fourth_order_finite_differences(orc, eps, X, Y):
    """Equation (1) applied to the closed-form u by 4th-order central
    differences (h = 1e-3) reproduces f to a relative residual <= 1e-9."""
    h = 1e-3
    rng = np.random.default_rng(5)
    for _ in range(100):
        x = rng.uniform(0.1 * X, 0.9 * X)
        y = rng.uniform(0.1 * Y, 0.9 * Y)
        c = [1 / 12, -2 / 3, 0, 2 / 3, -1 / 12]
        c2 = [-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12]
        off = [-2, -1, 0, 1, 2]
        ux = sum(ci * _u(x + o * h, y, X, Y) for ci, o in zip(c, off)) / h
        uy = sum(ci * _u(x, y + o * h, X, Y) for ci, o in zip(c, off)) / h
        uxx = sum(ci * _u(x + o * h, y, X, Y) for ci, o in zip(c2, off)) / h ** 2
        uyy = sum(ci * _u(x, y + o * h, X, Y) for ci, o in zip(c2, off)) / h ** 2
        lhs = eps * (uxx + uyy) + (1 + x * x) * ux + X * math.exp(-y) * uy
        f = orc.f_point(eps, X, Y, x, y)
        scale = abs(eps * (abs(uxx) + abs(uyy))) + abs((1 + x * x) * ux) + abs(X * math.exp(-y) * uy)
        assert abs(lhs - f) <= 1e-9 * scale


def test_boundary_data_is_the_exact_solution_and_its_normal_derivative(orc):
    X, Y, nx, ny = 2.0, 1.5, 7, 9
    bd = orc.boundary(X, Y, nx, ny)
    dx, dy = X / (nx + 1), Y / (ny + 1)
    y = dy * np.arange(1, ny + 1)
    x = dx * np.arange(1, nx + 1)
    np.testing.assert_allclose(bd["u_x0"], _u(0.0, y, X, Y), rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(bd["u_xX"], _u(X, y, X, Y), rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(bd["u_yY"], _u(x, Y, X, Y), rtol=1e-15, atol=1e-16)
    np.testing.assert_array_equal(bd["u_y0"], 0.0)
    h = 1e-4  # du/dx at x = X and du/dy at y = Y by central differences
    gx = (_u(X + h, y, X, Y) - _u(X - h, y, X, Y)) / (2 * h)
    gy = (_u(x, Y + h, X, Y) - _u(x, Y - h, X, Y)) / (2 * h)
    np.testing.assert_allclose(bd["g_xX"], gx, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(bd["g_yY"], gy, rtol=1e-7, atol=1e-12)


# --------------------------------------------------------------------------
# Section 4 + Section 6: the discretisation against the printed error tables
# --------------------------------------------------------------------------

def test_table_6_1_max_errors(orc, tables):
    t = tables["table_6_1"]
    nx = t["m"] - 1
    for case in t["cases"]:
        P = orc.assemble(t["eps"], t["X"], t["Y"], nx, nx, SCHEME[case["scheme"]], BC[case["bc"]])
        err = orc.max_error(P, dense.exact_discrete(P))
        assert agrees_to_printed(err, case["max_error"]), (case, err)


def test_table_6_2_max_errors(orc, tables):
    t = tables["table_6_2"]
    nx = t["m"] - 1
    checked = 0
    for name, sch in SCHEME.items():
        for eps, printed in zip(t["eps"], t[name + "_max_error"]):
            if printed is None:
                continue
            P = orc.assemble(eps, t["X"], t["Y"], nx, nx, sch, core.DIRICHLET)
            err = orc.max_error(P, dense.exact_discrete(P))
            assert agrees_to_printed(err, printed), (name, eps, err, printed)
            checked += 1
    assert checked == 14


def test_table_6_8_max_errors(orc, tables):
    t = tables["table_6_8"]
    for name, sch in SCHEME.items():
        for m, printed in zip(t["m"], t[name + "_max_error"]):
            P = orc.assemble(t["eps"], t["X"], t["Y"], m - 1, m - 1, sch, core.DIRICHLET)
            err = orc.max_error(P, dense.exact_discrete(P))
            assert agrees_to_printed(err, printed), (name, m, err, printed)


def test_assembly_against_the_stencil_written_per_node(orc):
    """The five diagonals equal the Section 4 stencil coefficients, node by
    node, with boundary couplings moved to the right-hand side."""
    eps, X, Y, nx, ny = 0.37, 1.3, 0.8, 6, 5
    dx, dy = X / (nx + 1), Y / (ny + 1)
    for sch in (core.UPWIND, core.CENTERED):
        for bc in (core.DIRICHLET, core.NEUMANN):
            P = orc.assemble(eps, X, Y, nx, ny, sch, bc)
            A = dense.dense_matrix(P)
            for j in range(ny):
                for i in range(nx):
                    x, y = (i + 1) * dx, (j + 1) * dy
                    a, b = 1 + x * x, X * math.exp(-y)
                    k = j * nx + i
                    if sch == core.UPWIND:
                        cs = eps * dx * dx - b * dx * dx * dy
                        cw = eps * dy * dy - a * dx * dy * dy
                        cc = -2 * eps * dy * dy - 2 * eps * dx * dx + a * dx * dy * dy + b * dx * dx * dy
                        ce, cn = eps * dy * dy, eps * dx * dx
                    else:
                        cs = eps * dx * dx - 0.5 * b * dx * dx * dy
                        cw = eps * dy * dy - 0.5 * a * dx * dy * dy
                        cc = -2 * eps * dy * dy - 2 * eps * dx * dx
                        ce = eps * dy * dy + 0.5 * a * dx * dy * dy
                        cn = eps * dx * dx + 0.5 * b * dx * dx * dy
                    rhs = _f_from_derivatives(eps, X, Y, x, y) * dx * dx * dy * dy
                    diag = cc
                    # neighbours: interior -> matrix entry; boundary -> rhs
                    nbrs = [(i, j - 1, cs, "S"), (i - 1, j, cw, "W"), (i + 1, j, ce, "E"), (i, j + 1, cn, "N")]
                    for (ii, jj, coef, tag) in nbrs:
                        if 0 <= ii < nx and 0 <= jj < ny:
                            assert A[k, jj * nx + ii] == pytest.approx(coef, rel=1e-13, abs=1e-18)
                        elif bc == core.NEUMANN and tag == "E":
                            diag += coef
                            rhs -= coef * dx * (-(1 / X) * math.exp(-1) * (1 - math.exp(-y / Y)) * y)
                        elif bc == core.NEUMANN and tag == "N":
                            diag += coef
                            rhs -= coef * dy * math.exp(-x / X)
                        else:
                            rhs -= coef * _u((ii + 1) * dx, (jj + 1) * dy, X, Y)
                    assert A[k, k] == pytest.approx(diag, rel=1e-13, abs=1e-18)
                    assert P.rhs[k] == pytest.approx(rhs, rel=1e-11, abs=1e-17)


@pytest.mark.parametrize("scheme,bc,eps,expect,lo,hi", [
    (core.UPWIND, core.DIRICHLET, 0.1, "first order", 0.85, 1.25),
    (core.CENTERED, core.DIRICHLET, 0.1, "second order", 1.85, 2.15),
    (core.UPWIND, core.NEUMANN, 1.0, "first order", 0.85, 1.25),
    (core.CENTERED, core.NEUMANN, 1.0, "first order (one-sided Neumann closure)", 0.85, 1.25),
])
def test_order_of_the_scheme(orc, scheme, bc, eps, expect, lo, hi):
    """Section 6.7: upwind is first order, centered second order under
    Dirichlet data, and the one-sided Neumann closure makes both first order.
    Observed order from the slope of log(error) against log(h), solved by the
    oracle's ILU(0)-BiCGSTAB to 1e-12."""
    errs, hs = [], []
    for n in (31, 63, 127):
        P = orc.assemble(eps, 1.0, 1.0, n, n, scheme, bc)
        F = orc.ilu0(P)
        s = orc.bicgstab(P, F, tol=1e-12, maxit=2000)
        assert s.status == core.OK
        errs.append(orc.max_error(P, s.x))
        hs.append(1.0 / (n + 1))
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert lo <= slope <= hi, (expect, slope, errs)


# --------------------------------------------------------------------------
# Section 5.1: ILU(0)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,scheme,bc,eps", [
    (7, 6, core.UPWIND, core.DIRICHLET, 0.5), (9, 9, core.CENTERED, core.DIRICHLET, 0.05),
    (8, 5, core.UPWIND, core.NEUMANN, 4.0), (6, 10, core.CENTERED, core.NEUMANN, 2.0),
    (19, 19, core.UPWIND, core.DIRICHLET, 4.0)])
def test_ilu0_product_equals_a_on_its_pattern(orc, nx, ny, scheme, bc, eps):
    """ILU(0): (L U)_ij = a_ij wherever a_ij != 0; the discarded fill sits
    only at offsets +-(nx-1)."""
    P = orc.assemble(eps, 1.0, 1.2, nx, ny, scheme, bc)
    F = orc.ilu0(P)
    assert F.status == core.OK
    R = dense.lu_product_minus_a(P, F)
    A = dense.dense_matrix(P)
    mask = A != 0
    scale = np.abs(A).max()
    assert np.abs(R[mask]).max() <= 8 * np.finfo(float).eps * scale
    off = np.subtract.outer(np.arange(P.n), np.arange(P.n))
    fill = (~mask) & (np.abs(R) > 8 * np.finfo(float).eps * scale)
    assert np.all(np.isin(np.abs(off[fill]), [nx - 1]))
    if nx > 1 and ny > 1:
        assert fill.any()


@pytest.mark.parametrize("nx,ny", [(1, 12), (12, 1), (1, 1)])
def test_ilu0_is_exact_lu_in_one_dimension(orc, nx, ny):
    """With one row or one column there is no fill, so ILU(0) is the exact LU
    and BiCGSTAB ends at the half-step of pass 1."""
    P = orc.assemble(0.2, 1.0, 1.0, nx, ny, core.CENTERED, core.DIRICHLET)
    F = orc.ilu0(P)
    np.testing.assert_allclose(dense.lu_product_minus_a(P, F), 0.0, atol=1e-15 * np.abs(P.C).max())
    s = orc.bicgstab(P, F, tol=1e-10, maxit=50)
    assert s.status == core.OK and s.iters == 1 and s.half_step
    np.testing.assert_allclose(s.x, dense.exact_discrete(P), rtol=1e-12, atol=1e-14)


def test_ilu0_matches_elimination_restricted_to_the_pattern(orc):
    """Gaussian elimination (Algorithm 5.1 with p = 0): every update outside
    the pattern of A is dropped as it happens.  Written as a dense loop."""
    P = orc.assemble(0.3, 1.0, 1.0, 5, 4, core.CENTERED, core.NEUMANN)
    A = dense.dense_matrix(P)
    pat = A != 0
    B = A.copy()
    n = P.n
    for i in range(1, n):
        for k in range(i):
            if not pat[i, k]:
                continue
            B[i, k] = B[i, k] / B[k, k]
            for j in range(k + 1, n):
                if pat[i, j]:
                    B[i, j] -= B[i, k] * B[k, j]
    F = orc.ilu0(P)
    np.testing.assert_allclose(1.0 / F.invd, np.diag(B), rtol=1e-14)
    k = np.arange(n)
    np.testing.assert_allclose(F.lw[1:], B[k[1:], k[1:] - 1], rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(F.ls[P.nx:], B[k[P.nx:], k[P.nx:] - P.nx], rtol=1e-14, atol=1e-300)


# --------------------------------------------------------------------------
# Building blocks against library routines and exact arithmetic
# --------------------------------------------------------------------------

def test_spmv_matches_scipy(orc):
    import scipy.sparse as sp
    P = orc.assemble(0.05, 1.0, 2.0, 13, 11, core.UPWIND, core.NEUMANN)
    A = sp.csr_matrix(dense.dense_matrix(P))
    x = np.random.default_rng(3).standard_normal(P.n)
    np.testing.assert_allclose(orc.spmv(P, x), A @ x, rtol=1e-13, atol=1e-13 * np.abs(A @ x).max())


def test_triangular_sweeps_match_scipy(orc):
    import scipy.sparse as sp
    from scipy.sparse.linalg import spsolve_triangular
    P = orc.assemble(0.05, 1.0, 1.0, 12, 9, core.CENTERED, core.DIRICHLET)
    F = orc.ilu0(P)
    n, nx = P.n, P.nx
    k = np.arange(n)
    L = np.eye(n)
    L[k[1:], k[1:] - 1] = F.lw[1:]
    L[k[nx:], k[nx:] - nx] = F.ls[nx:]
    U = np.diag(1.0 / F.invd)
    U[k[:-1], k[:-1] + 1] = F.ue[:-1]
    U[k[:-nx], k[:-nx] + nx] = F.un[:-nx]
    q = np.random.default_rng(4).standard_normal(n)
    y = orc.lsolve(P.nx, P.ny, F, q)
    np.testing.assert_allclose(y, spsolve_triangular(sp.csr_matrix(L), q, lower=True), rtol=1e-12, atol=1e-12)
    z = orc.usolve(P.nx, P.ny, F, y)
    np.testing.assert_allclose(z, spsolve_triangular(sp.csr_matrix(U), y, lower=False), rtol=1e-12, atol=1e-12)


def test_double_double_dot_is_the_rounded_exact_dot(orc):
    """Without heavy cancellation the double-double dot product is the exact
    dot product correctly rounded; with cancellation it stays within half an
    ulp plus the double-word bound 2 n u^2 sum|x_k y_k|."""
    rng = np.random.default_rng(7)
    u = np.finfo(float).eps / 2
    for trial in range(60):
        n = int(rng.integers(1, 400))
        x = rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5, n)
        y = rng.standard_normal(n)
        cancel = trial % 3 == 0
        if cancel:  # second half cancels the first half exactly up to rounding
            h = n // 2
            y = np.concatenate([y[:h], -y[:h] * x[:h] / x[h:2 * h], y[2 * h:]])
        exact = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
        d = orc.dot(x, y)
        if not cancel:
            assert d == float(exact)
        else:
            bound = 0.5 * np.spacing(abs(float(exact))) + 2 * n * u * u * float(np.sum(np.abs(x * y)))
            assert abs(Fraction(d) - exact) <= Fraction(bound)


def test_maxabs(orc):
    x = np.array([1.0, -7.5, 3.0, -0.0])
    assert orc.maxabs(x) == 7.5
    assert math.isnan(orc.maxabs(np.array([1.0, np.nan, 2.0])))


# --------------------------------------------------------------------------
# Section 5.2: BiCGSTAB
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,scheme,bc,eps", [
    (16, 16, core.UPWIND, core.DIRICHLET, 0.1), (16, 16, core.CENTERED, core.DIRICHLET, 0.1),
    (12, 16, core.UPWIND, core.NEUMANN, 2.0), (16, 9, core.CENTERED, core.NEUMANN, 4.0),
    (5, 16, core.CENTERED, core.DIRICHLET, 0.02)])
def test_bicgstab_reaches_the_dense_lu_solution(orc, nx, ny, scheme, bc, eps):
    P = orc.assemble(eps, 1.0, 1.0, nx, ny, scheme, bc)
    s = orc.bicgstab(P, orc.ilu0(P), tol=1e-14, maxit=500)
    assert s.status == core.OK
    ref = dense.exact_discrete(P)
    assert np.abs(s.x - ref).max() <= 1e-12 * np.abs(ref).max()
    # the recorded history is the 2-norm of the recursively updated residual
    assert s.hist_l2[0] == pytest.approx(np.linalg.norm(P.rhs), rel=1e-15)
    assert np.all(s.hist_max <= s.hist_l2 * (1 + 1e-15))
    assert s.hist_l2[-1] < 1e-14 * s.bnorm


def test_complete_lu_reproduces_a_and_scipy():
    """The complete factors behind the truncated preconditioner: L U = A, and
    the same factors as SciPy's LU of a matrix that needs no row exchange
    (diagonally dominant, so partial pivoting keeps the natural order)."""
    import scipy.linalg
    P = core.assemble(2.0, 1.0, 1.0, 7, 5, core.CENTERED, core.DIRICHLET)
    A = dense.dense_matrix(P)
    L, U = dense.lu_no_pivoting(A)
    assert np.abs(L @ U - A).max() <= 1e-14 * np.abs(A).max()
    perm, L2, U2 = scipy.linalg.lu(A)
    assert np.array_equal(perm, np.eye(P.n))
    np.testing.assert_allclose(L, L2, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(U, U2, rtol=1e-12, atol=1e-15 * np.abs(A).max())


def test_table_6_2_iterations_with_the_appendix_settings(orc, tables):
    """The appendix's solver settings (truncated full LU, x0 = 10, absolute
    1e-20 test) reproduce the Section 6.2 iteration counts: the upwind row
    exactly, the centered row within +-3 (the absolute 1e-20 test sits far
    below the rounding floor, so the last passes are rounding-sensitive)."""
    t = tables["table_6_2"]
    st = tables["solver_settings"]
    nx = t["m"] - 1
    for name, sch in SCHEME.items():
        for eps, printed in zip(t["eps"], t[name + "_iterations"]):
            P = orc.assemble(eps, t["X"], t["Y"], nx, nx, sch, core.DIRICHLET)
            s = orc.bicgstab(P, dense.truncated_lu(P), tol=st["abs_tol"], abs_tol=True, maxit=1000, max_restarts=-1,
                             x0=np.full(P.n, st["x0_preconditioned"]))
            if printed is None:  # "NC": not converged within 1000 passes
                assert s.status == core.MAXIT
            elif name == "upwind":
                assert s.status == core.OK and s.iters == printed, (eps, s.iters)
            else:
                assert s.status == core.OK and abs(s.iters - printed) <= 3, (eps, s.iters)


def test_table_6_1_iterations_with_the_appendix_settings(orc, tables):
    t = tables["table_6_1"]
    st = tables["solver_settings"]
    nx = t["m"] - 1
    for case in t["cases"]:
        P = orc.assemble(t["eps"], t["X"], t["Y"], nx, nx, SCHEME[case["scheme"]], BC[case["bc"]])
        s = orc.bicgstab(P, dense.truncated_lu(P), tol=st["abs_tol"], abs_tol=True, maxit=1000, max_restarts=-1,
                         x0=np.full(P.n, st["x0_preconditioned"]))
        assert s.status == core.OK and abs(s.iters - case["iterations"]) <= 3, (case, s.iters)
        assert agrees_to_printed(orc.max_error(P, s.x), case["max_error"])


def test_table_6_5_and_6_8_iterations_other_preconditioners(orc, tables):
    """Section 6.5 (splitting preconditioner; no preconditioner) and the
    iteration row of Section 6.8, which matches the unpreconditioned solver
    of the appendix (x0 = 1e5).  Rounding-sensitive: within +-5."""
    t5 = tables["table_6_5"]
    st = tables["solver_settings"]
    for bcname, bc in BC.items():
        P = orc.assemble(t5["eps"], t5["X"], t5["Y"], t5["m"] - 1, t5["m"] - 1, core.UPWIND, bc)
        s = orc.bicgstab(P, dense.split_lu(P), tol=st["abs_tol"], abs_tol=True, maxit=5000, max_restarts=-1,
                         x0=np.full(P.n, st["x0_preconditioned"]))
        assert s.status == core.OK
        assert abs(s.iters - t5["split_lu_bicgstab_iterations"][bcname]) <= 5, (bcname, s.iters)
        s = orc.bicgstab(P, dense.identity(P), tol=st["abs_tol"], abs_tol=True, maxit=5000, max_restarts=-1,
                         x0=np.full(P.n, st["x0_unpreconditioned"]))
        assert s.status == core.OK
        assert abs(s.iters - t5["unpreconditioned_iterations"][bcname]) <= 5, (bcname, s.iters)
        assert agrees_to_printed(orc.max_error(P, s.x), t5["max_error"][bcname])
    t8 = tables["table_6_8"]
    for name, sch in SCHEME.items():
        for m, printed in zip(t8["m"], t8[name + "_iterations"]):
            P = orc.assemble(t8["eps"], t8["X"], t8["Y"], m - 1, m - 1, sch, core.DIRICHLET)
            s = orc.bicgstab(P, dense.identity(P), tol=st["abs_tol"], abs_tol=True, maxit=1000, max_restarts=-1,
                             x0=np.full(P.n, st["x0_unpreconditioned"]))
            assert s.status == core.OK and abs(s.iters - printed) <= 5, (name, m, s.iters)


def test_status_codes(orc):
    P = orc.assemble(0.1, 1.0, 1.0, 10, 10, core.UPWIND, core.DIRICHLET)
    F = orc.ilu0(P)
    s = orc.bicgstab(P, F, tol=1e-10, maxit=1)
    assert s.status == core.MAXIT and s.iters == 1 and len(s.hist_l2) == 2
    # immediate convergence from the exact discrete solution
    ref = dense.exact_discrete(P)
    s = orc.bicgstab(P, F, tol=1e-10, maxit=10, x0=ref)
    assert s.status == core.OK and s.iters == 0
    # b = 0 returns x = 0
    s = orc.bicgstab(P, F, tol=1e-10, maxit=10, b=np.zeros(P.n), x0=np.ones(P.n))
    assert s.status == core.OK and s.iters == 0 and not s.x.any()
    # a NaN in the forcing
    g = np.zeros(P.n)
    g[17] = np.nan
    Pn = orc.assemble(0.1, 1.0, 1.0, 10, 10, core.UPWIND, core.DIRICHLET, field=g, amp=0.1)
    s = orc.bicgstab(Pn, orc.ilu0(Pn), tol=1e-10, maxit=10)
    assert s.status == core.NONFINITE
    # zero pivot: C_0 = 0 with no lower couplings in row 0
    P.C[0] = 0.0
    F = orc.ilu0(P)
    assert F.status == core.ZERO_PIVOT and F.bad == 0
    # argument errors
    with pytest.raises(ValueError):
        orc.assemble(0.0, 1.0, 1.0, 4, 4)
    with pytest.raises(ValueError):
        orc.assemble(1.0, 1.0, 1.0, 0, 4)


def test_forcing_field_is_added_with_relative_amplitude(orc):
    nx, ny = 9, 7
    g = np.random.default_rng(1).standard_normal(nx * ny)
    P0 = orc.assemble(0.2, 1.0, 1.0, nx, ny, core.CENTERED, core.DIRICHLET)
    P1 = orc.assemble(0.2, 1.0, 1.0, nx, ny, core.CENTERED, core.DIRICHLET, field=g, amp=0.1)
    fman = orc.forcing(0.2, 1.0, 1.0, nx, ny)
    dx, dy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    np.testing.assert_allclose(P1.rhs - P0.rhs, 0.1 * np.abs(fman).max() * g * dx * dx * dy * dy,
                               rtol=1e-9, atol=1e-20)


# --------------------------------------------------------------------------
# Mixed precision: factors stored in FP32, sweeps in FP64 or FP32
# --------------------------------------------------------------------------

def test_single_precision_sweeps_are_single_precision_solves(orc):
    """The FP32 substitutions agree with the FP64 substitutions of the same
    (float-rounded) factors to single-precision accuracy, and exactly invert
    their own triangular factors up to float rounding."""
    P = orc.assemble(0.05, 1.0, 1.0, 24, 20, core.CENTERED, core.DIRICHLET)
    F = orc.round_factors_f32(orc.ilu0(P))
    q = np.random.default_rng(2).standard_normal(P.n)
    y64 = orc.lsolve(P.nx, P.ny, F, q)
    y32 = orc.lsolve_f32(P.nx, P.ny, F, q)
    assert np.abs(y32 - y64).max() <= 1e-5 * np.abs(y64).max()
    assert np.all(y32 == y32.astype(np.float32))       # values are floats
    z64 = orc.usolve(P.nx, P.ny, F, y32)
    z32 = orc.usolve_f32(P.nx, P.ny, F, y32)
    assert np.abs(z32 - z64).max() <= 1e-4 * np.abs(z64).max()


@pytest.mark.parametrize("sweep_f32", [False, True])
def test_mixed_precision_preconditioner_still_reaches_the_fp64_solution(orc, sweep_f32):
    """A lower-precision M only changes the convergence rate: the FP64 outer
    iteration still reaches ||r|| < 1e-13 ||b|| and the dense LU solution."""
    P = orc.assemble(0.1, 1.0, 1.0, 16, 16, core.UPWIND, core.DIRICHLET)
    F = orc.round_factors_f32(orc.ilu0(P))
    s = orc.bicgstab(P, F, tol=1e-13, maxit=500, sweep_f32=sweep_f32)
    assert s.status == core.OK
    ref = dense.exact_discrete(P)
    assert np.abs(s.x - ref).max() <= 1e-11 * np.abs(ref).max()
