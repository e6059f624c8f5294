"""Pins of the oracle's stopping logic, its true-residual confirmation, the
instance classifier and the assembly from user data -- each checked against
something other than the oracle itself: exact rational arithmetic, closed
forms, quadrature, numpy residuals, or a problem the scheme solves exactly.
CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import core
from oracle import dense

import rational_ref as rr

HERE = os.path.dirname(os.path.abspath(__file__))


def crafted():
    with open(os.path.join(HERE, "golden", "crafted_stops.json")) as fh:
        return json.load(fh)


def crafted_problem(d):
    arr = {k: np.array(d[k], dtype=np.float64) for k in ("S", "W", "C", "E", "N", "rhs")}
    return core.Problem(1.0, 1.0, 1.0, d["nx"], d["ny"], 0, 0, arr["S"], arr["W"], arr["C"], arr["E"], arr["N"],
                        arr["rhs"])


def true_relres(P, x):
    A = dense.dense_matrix(P)
    return np.linalg.norm(P.rhs - A @ x) / np.linalg.norm(P.rhs)


# --------------------------------------------------------------------------
# Section 5.2: the exact-zero stops rho = 0 and omega = 0
# --------------------------------------------------------------------------

def test_crafted_systems_cover_both_exact_zero_stops():
    sts = set()
    for d in crafted()["systems"]:
        A = rr.dense_from_dia(d["nx"], d["ny"], d["S"], d["W"], d["C"], d["E"], d["N"])
        st, it, _ = rr.bicgstab(A, *rr.ilu0(A, rr.pattern_of(d["nx"], d["ny"])), d["rhs"], 1e-10, 20)
        sts.add(st)
    assert {rr.BREAKDOWN_RHO, rr.OMEGA_ZERO} <= sts


@pytest.mark.parametrize("k", range(3))
def test_exact_zero_stops_match_exact_arithmetic(orc, k):
    """The oracle stops on rho = 0 / omega = 0 at the pass where BiCGSTAB in
    exact rational arithmetic (with ILU(0) by elimination restricted to A's
    pattern) stops, and its residual history follows the exact one."""
    g = crafted()
    d = g["systems"][k]
    P = crafted_problem(d)
    A = rr.dense_from_dia(d["nx"], d["ny"], d["S"], d["W"], d["C"], d["E"], d["N"])
    st, it, hist2 = rr.bicgstab(A, *rr.ilu0(A, rr.pattern_of(d["nx"], d["ny"])), d["rhs"], g["tol"], g["maxit"])
    s = orc.bicgstab(P, orc.ilu0(P), tol=g["tol"], maxit=g["maxit"])
    assert (s.status, s.iters) == (st, it)
    exact = np.sqrt([float(h) for h in hist2])
    np.testing.assert_allclose(s.hist_l2, exact, rtol=1e-12, atol=1e-14 * exact[0])


def test_rational_ilu0_agrees_with_the_oracle_factors(orc):
    """The five-point pivot recurrence of the oracle equals elimination on the
    pattern of A written for a general sparse matrix (exact arithmetic)."""
    P = orc.assemble(0.3, 1.0, 1.5, 4, 3, core.CENTERED, core.NEUMANN)
    F = orc.ilu0(P)
    A = rr.dense_from_dia(P.nx, P.ny, P.S, P.W, P.C, P.E, P.N)
    L, U = rr.ilu0(A, rr.pattern_of(P.nx, P.ny))
    for k in range(P.n):
        assert float(U[k][k]) == pytest.approx(1.0 / F.invd[k], rel=1e-13)
        if k % P.nx:
            assert float(L[k][k - 1]) == pytest.approx(F.lw[k], rel=1e-13, abs=1e-300)
        if k >= P.nx:
            assert float(L[k][k - P.nx]) == pytest.approx(F.ls[k], rel=1e-13, abs=1e-300)


# --------------------------------------------------------------------------
# True-residual confirmation and restarts
# --------------------------------------------------------------------------

@pytest.mark.parametrize("eps,n,scheme,bc,tol", [(0.1, 64, 1, 0, 1e-14), (0.01, 96, 0, 0, 1e-10),
                                                  (2.0, 40, 1, 1, 1e-12), (0.05, 50, 0, 1, 1e-10)])
def test_ok_means_the_true_residual_passes(orc, eps, n, scheme, bc, tol):
    P = orc.assemble(eps, 1.0, 1.0, n, n, scheme, bc)
    s = orc.bicgstab(P, orc.ilu0(P), tol=tol, maxit=2000)
    assert s.status == core.OK
    assert true_relres(P, s.x) < tol
    assert s.true_relres == pytest.approx(true_relres(P, s.x), rel=1e-6)


def test_a_restart_is_a_solve_from_the_current_iterate(orc):
    """Centered, eps = 0.1, 64 x 64, tol 1e-14: the recursion converges at a
    pass k1 whose true residual is still above the tolerance; the solve then
    continues exactly as a new solve started from that iterate."""
    P = orc.assemble(0.1, 1.0, 1.0, 64, 64, core.CENTERED, core.DIRICHLET)
    F = orc.ilu0(P)
    first = orc.bicgstab(P, F, tol=1e-14, maxit=500, max_restarts=-1)
    assert first.status == core.OK and true_relres(P, first.x) >= 1e-14
    full = orc.bicgstab(P, F, tol=1e-14, maxit=500)
    assert full.status == core.OK and full.restarts >= 1
    k1 = first.iters
    np.testing.assert_array_equal(full.hist_l2[:k1 + 1], first.hist_l2)
    again = orc.bicgstab(P, F, tol=1e-14, maxit=500, x0=first.x, max_restarts=full.restarts - 1)
    assert again.status == full.status
    assert k1 + again.iters == full.iters
    np.testing.assert_array_equal(full.hist_l2[k1 + 1:], again.hist_l2[1:])
    np.testing.assert_array_equal(full.x, again.x)
    assert true_relres(P, full.x) < 1e-14


def test_inaccurate_after_the_allowed_restarts(orc):
    """Upwind, eps = 0.1, 64 x 64, tol 1e-15, below what the true residual can
    reach in FP64: the recursion keeps converging, the true residual does not,
    and the solve ends ADR_INACCURATE after exactly max_restarts restarts."""
    P = orc.assemble(0.1, 1.0, 1.0, 64, 64, core.UPWIND, core.DIRICHLET)
    F = orc.ilu0(P)
    for mr in (0, 2, core.MAX_RESTARTS):
        s = orc.bicgstab(P, F, tol=1e-15, maxit=2000, max_restarts=mr)
        assert s.status == core.INACCURATE and s.restarts == mr
        assert s.hist_l2[-1] < 1e-15 * s.bnorm            # the recursion passed
        assert true_relres(P, s.x) >= 1e-15               # the true residual did not
    s = orc.bicgstab(P, F, tol=1e-15, maxit=2000, max_restarts=-1)
    assert s.status == core.OK and s.restarts == 0        # the recursive test alone


def test_converging_on_the_last_allowed_pass_is_maxit(orc):
    P = orc.assemble(0.1, 1.0, 1.0, 64, 64, core.CENTERED, core.DIRICHLET)
    F = orc.ilu0(P)
    first = orc.bicgstab(P, F, tol=1e-14, maxit=500, max_restarts=-1)
    s = orc.bicgstab(P, F, tol=1e-14, maxit=first.iters)
    assert s.status == core.MAXIT and s.iters == first.iters and s.restarts == 0
    np.testing.assert_array_equal(s.x, first.x)


# --------------------------------------------------------------------------
# Instance classifier (Section 6.3 mesh Reynolds number; Section 6.1 Neumann)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("eps,X,Y", [(0.01, 1.0, 1.0), (1e-3, 2.0, 1.0), (0.3, 0.5, 1.7)])
def test_growth_exponent_is_the_integral_of_b_over_eps(orc, eps, X, Y):
    c = orc.classify(eps, X, Y, 33, 21, core.UPWIND, core.NEUMANN)
    q, _ = integrate.quad(lambda y: X * math.exp(-y) / eps, 0.0, Y, epsabs=0, epsrel=1e-13)
    assert c.g_y == pytest.approx(q, rel=1e-12)


def test_cell_peclet_numbers_in_closed_form(orc):
    eps, X, Y, nx, ny = 0.02, 1.5, 0.8, 57, 41
    c = orc.classify(eps, X, Y, nx, ny, core.CENTERED, core.DIRICHLET)
    dx, dy = X / (nx + 1), Y / (ny + 1)
    assert c.pe_x == pytest.approx((1 + (nx * dx) ** 2) * dx / eps, rel=1e-14)   # a grows with x
    assert c.pe_y == pytest.approx(X * math.exp(-dy) * dy / eps, rel=1e-14)      # b falls with y


def test_negative_couplings_counted_in_closed_form(orc):
    """Upwind W = eps dy^2 (1 - a dx / eps) < 0 exactly where the cell Peclet
    number a dx / eps exceeds 1, on every row; S likewise per row."""
    eps, X, Y, nx, ny = 0.01, 1.0, 1.0, 60, 70
    dx, dy = X / (nx + 1), Y / (ny + 1)
    cols = [i for i in range(1, nx) if (1 + ((i + 1) * dx) ** 2) * dx > eps]
    rows = [j for j in range(1, ny) if X * math.exp(-(j + 1) * dy) * dy > eps]
    c = orc.classify(eps, X, Y, nx, ny, core.UPWIND, core.DIRICHLET)
    assert c.neg_offdiag == len(cols) * ny + len(rows) * nx
    assert orc.classify(eps, X, Y, nx, ny, core.UPWIND, core.DIRICHLET).neg_offdiag > 0
    assert orc.classify(1.0, X, Y, nx, ny, core.UPWIND, core.DIRICHLET).neg_offdiag == 0


def test_diagonal_sign_counted_in_closed_form(orc):
    """Upwind with dx = dy = h: C = h^3 (a + b) - 4 eps h^2 >= 0 exactly where
    (a + b) h >= 4 eps."""
    eps, X, n = 0.0133, 1.0, 40
    h = X / (n + 1)
    cnt = sum(1 for j in range(n) for i in range(n)
              if (1 + ((i + 1) * h) ** 2 + X * math.exp(-(j + 1) * h)) * h >= 4 * eps)
    c = orc.classify(eps, X, X, n, n, core.UPWIND, core.DIRICHLET)
    assert 0 < cnt < n * n
    assert c.nonneg_diag == cnt
    assert orc.classify(eps, X, X, n, n, core.CENTERED, core.DIRICHLET).nonneg_diag == 0


def test_expectation_rule(orc):
    """The three failure mechanisms: the Neumann residual floor u exp(g_y)
    against tol (threshold ln(tol/u) = 13.71 at tol 1e-10, 9.11 at 1e-12),
    a diagonal that changes sign inside the grid, and downwind differencing
    beyond cell Peclet 2."""
    u = 2.0 ** -53
    assert math.log(1e-10 / u) == pytest.approx(13.7109, abs=1e-4)
    # g_y = (1 - e^-1) / eps: 13.0 at eps = 0.048626, 14.0 at 0.045153
    for eps, gy in ((0.048626, 13.0), (0.045153, 14.0)):
        c = orc.classify(eps, 1.0, 1.0, 64, 64, core.CENTERED, core.NEUMANN, tol=1e-10)
        assert c.g_y == pytest.approx(gy, rel=1e-4)
        assert c.expect_fail == (gy > 13.7109)
        assert orc.classify(eps, 1.0, 1.0, 64, 64, core.CENTERED, core.NEUMANN, tol=1e-12).expect_fail
        assert not orc.classify(eps, 1.0, 1.0, 64, 64, core.CENTERED, core.DIRICHLET, tol=1e-12).expect_fail
    # diagonal sign change inside the grid (see the closed-form count above)
    assert orc.classify(0.0133, 1.0, 1.0, 40, 40, core.UPWIND, core.DIRICHLET).expect_fail
    # downwind: upwind scheme, negative diagonal, Peclet 1.5 (fine) and 2.5 (not)
    for pe, fails in ((1.5, False), (2.5, True)):
        n = 99
        h = 1.0 / (n + 1)
        eps = 2.0 * h / pe      # max a = 1 + (n h)^2 ~ 2
        c = orc.classify(eps, 1.0, 1.0, n, n, core.UPWIND, core.DIRICHLET)
        assert c.nonneg_diag == 0 and c.pe_x == pytest.approx(pe, rel=0.02)
        assert c.expect_fail == fails
        assert not orc.classify(eps, 1.0, 1.0, n, n, core.CENTERED, core.DIRICHLET).expect_fail


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(HERE), "paper_1308_5215_amd", "libadr.so")),
                    reason="libadr.so not built")
def test_library_classifier_equals_the_oracle(orc):
    """adr_classify (host code of the library, no device work) against the
    oracle's classification from the assembled diagonals."""
    import paper_1308_5215_amd as adr
    rng = np.random.default_rng(5)
    for _ in range(40):
        eps = 10 ** rng.uniform(-3.5, 0.5)
        X, Y = rng.uniform(0.5, 2.0, 2)
        nx, ny = (int(v) for v in rng.integers(1, 120, 2))
        sc, bc = (int(v) for v in rng.integers(0, 2, 2))
        tol = 10 ** rng.uniform(-13, -6)
        a = adr.classify(eps, X, Y, nx, ny, sc, bc, tol)
        b = orc.classify(eps, X, Y, nx, ny, sc, bc, tol)
        assert (a.neg_offdiag, a.nonneg_diag, a.expect_fail) == (b.neg_offdiag, b.nonneg_diag, b.expect_fail)
        assert a.pe_x == pytest.approx(b.pe_x, rel=1e-14) and a.pe_y == pytest.approx(b.pe_y, rel=1e-14)
        assert a.g_y == pytest.approx(b.g_y, rel=1e-14)


# --------------------------------------------------------------------------
# Assembly from user data (the appendix's assembly routines take f and the
# boundary data as arguments)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", [core.UPWIND, core.CENTERED])
@pytest.mark.parametrize("bc", [core.DIRICHLET, core.NEUMANN])
def test_linear_solution_is_reproduced_exactly(orc, scheme, bc):
    """u = 1 + 2x + 3y: both schemes' differences are exact for a linear u,
    and so is the one-sided Neumann closure, so the discrete solution of the
    data f = a u_x + b u_y, u on the Dirichlet sides, (u_x, u_y) = (2, 3) on
    the Neumann sides is u at the nodes."""
    eps, X, Y, nx, ny = 0.2, 1.3, 0.9, 11, 9
    t = orc.tables(X, Y, nx, ny)
    u = lambda x, y: 1.0 + 2.0 * x + 3.0 * y
    f = (2.0 * t["a"][None, :] + 3.0 * t["b"][:, None]).ravel()
    data = dict(f=f, u_x0=u(0.0, t["y"]), u_y0=u(t["x"], 0.0))
    if bc == core.DIRICHLET:
        data.update(u_xX=u(X, t["y"]), u_yY=u(t["x"], Y))
    else:
        data.update(u_xX=np.full(ny, 2.0), u_yY=np.full(nx, 3.0))
    P = orc.assemble_data(eps, X, Y, nx, ny, scheme, bc, **data)
    sol = dense.exact_discrete(P)
    expect = u(t["x"][None, :], t["y"][:, None]).ravel()
    assert np.abs(sol - expect).max() <= 1e-12 * np.abs(expect).max()


def test_manufactured_data_given_explicitly_is_the_manufactured_assembly(orc):
    eps, X, Y, nx, ny = 0.07, 1.1, 0.6, 13, 17
    f = orc.forcing(eps, X, Y, nx, ny)
    bd = orc.boundary(X, Y, nx, ny)
    for bc in (core.DIRICHLET, core.NEUMANN):
        ref = orc.assemble(eps, X, Y, nx, ny, core.CENTERED, bc)
        xX = bd["u_xX"] if bc == core.DIRICHLET else bd["g_xX"]
        yY = bd["u_yY"] if bc == core.DIRICHLET else bd["g_yY"]
        P = orc.assemble_data(eps, X, Y, nx, ny, core.CENTERED, bc, f=f, u_x0=bd["u_x0"], u_xX=xX,
                              u_y0=bd["u_y0"], u_yY=yY)
        for name in ("S", "W", "C", "E", "N", "rhs"):
            np.testing.assert_array_equal(getattr(P, name), getattr(ref, name))
