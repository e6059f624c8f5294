"""GPU (HIP, through the C ABI) against the CPU oracle on the outcomes other
than plain convergence: the exact-zero stops of Section 5.2 (rho = 0,
omega = 0) on crafted systems, the true-residual confirmation with its
restarts and the INACCURATE / MAXIT outcomes, the Neumann-closed 4096^2 grid,
the convection-dominated case at the sizes where it stops converging, every
instance of the seeded 256-instance batch that does not converge, assembly
from user data, the discretisation error and the streaming copy.

Bars: status, pass count, restarts, both residual histories and x bit for
bit (the same fixed fma orders and double-double reductions on both sides);
the discretisation error to a few ulps of the grid function (device and
host exp may differ in the last bit)."""
import json
import os

import numpy as np
import pytest

from oracle import core as orc
from synthetic import fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def adr():
    import paper_1308_5215_amd as adr
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return adr


def say(*a):
    print(*a, flush=True)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def equal(a, b):
    return np.array_equal(a, b) or (np.array_equal(np.isnan(a), np.isnan(b)) and
                                    np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)]))


def same_solve(res, x, ref):
    assert res.status == ref.status, (res.status, ref.status)
    assert res.iters == ref.iters, (res.iters, ref.iters)
    assert res.restarts == ref.restarts, (res.restarts, ref.restarts)
    assert res.half_step == ref.half_step
    assert equal(res.hist_l2, ref.hist_l2)
    assert equal(res.hist_max, ref.hist_max)
    assert equal(x, ref.x)


# --------------------------------------------------------------------------
# Exact-zero stops (Section 5.2) on crafted integer systems
# --------------------------------------------------------------------------

def crafted():
    with open(os.path.join(HERE, "golden", "crafted_stops.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("k", range(3))
def test_exact_zero_stops_on_crafted_systems(adr, k):
    g = crafted()
    d = g["systems"][k]
    nx, ny = d["nx"], d["ny"]
    say("crafted stop", k, nx, ny)
    arr = {n: np.array(d[n], dtype=np.float64) for n in ("S", "W", "C", "E", "N", "rhs")}
    prob = adr.assemble(1.0, 1.0, 1.0, nx, ny, "upwind", "dirichlet")
    prob.set_dia(**arr)
    prob.ilu0()
    res = prob.solve(g["tol"], g["maxit"])
    P = orc.Problem(1.0, 1.0, 1.0, nx, ny, 0, 0, arr["S"], arr["W"], arr["C"], arr["E"], arr["N"], arr["rhs"])
    ref = orc.bicgstab(P, orc.ilu0(P), tol=g["tol"], maxit=g["maxit"])
    assert ref.status in (orc.BREAKDOWN_RHO, orc.OMEGA_ZERO)
    same_solve(res, host(res.x), ref)


# --------------------------------------------------------------------------
# True-residual confirmation and restarts
# --------------------------------------------------------------------------

@pytest.mark.parametrize("eps,n,scheme,bc,tol,mr,maxit", [
    (0.1, 64, 1, 0, 1e-14, 8, 500),       # one restart, then OK
    (0.1, 64, 0, 0, 1e-15, 8, 2000),      # INACCURATE after 8 restarts
    (0.1, 64, 0, 0, 1e-15, 2, 2000),      # ... after 2
    (0.1, 64, 0, 0, 1e-15, 0, 2000),      # no restart allowed
    (0.1, 64, 0, 0, 1e-15, -1, 2000),     # the recursive test alone: OK
    (0.1, 16, 0, 0, 1e-15, 8, 14),        # recursion converges on the last pass: MAXIT
    (0.2, 8, 0, 1, 1e-15, 8, 16),         # the same with Neumann data, maxit a whole graph chunk
    (0.2, 8, 0, 1, 1e-15, 8, 200),        # Neumann: INACCURATE
    (0.3, 16, 1, 1, 1e-15, 8, 200),       # several restarts, then OK
])
def test_restart_parity(adr, eps, n, scheme, bc, tol, mr, maxit):
    ny = 24 if n == 8 else n
    say("restart", eps, n, ny, scheme, bc, tol, mr, maxit)
    prob = adr.assemble(eps, 1.0, 1.0, n, ny, scheme, bc)
    prob.set_max_restarts(mr)
    prob.ilu0()
    res = prob.solve(tol, maxit)
    P = orc.assemble(eps, 1.0, 1.0, n, ny, scheme, bc)
    ref = orc.bicgstab(P, orc.ilu0(P), tol=tol, maxit=maxit, max_restarts=mr)
    same_solve(res, host(res.x), ref)
    assert res.true_relres == pytest.approx(ref.true_relres, rel=1e-12)
    if res.status == adr.OK and mr >= 0:
        assert res.true_relres < tol


def test_restarts_in_a_batch_stop_each_instance_on_its_own(adr):
    """Instances with different restart histories in one batch: each equals
    its own oracle solve."""
    cases = [(0.1, 64, 64, 1, 0), (0.1, 64, 64, 0, 0), (0.3, 16, 16, 1, 1), (0.2, 8, 24, 0, 1), (0.05, 40, 30, 1, 0)]
    say("batch restarts")
    b = adr.assemble_batch(*zip(*[(e, 1.0, 1.0, nx, ny, sc, bc) for e, nx, ny, sc, bc in cases]))
    b.ilu0()
    res = b.solve(1e-15, 600)
    xs = [host(v) for v in b.split(res.x)]
    for k, (e, nx, ny, sc, bc) in enumerate(cases):
        P = orc.assemble(e, 1.0, 1.0, nx, ny, sc, bc)
        ref = orc.bicgstab(P, orc.ilu0(P), tol=1e-15, maxit=600)
        assert (res.status[k], res.iters[k], res.restarts[k]) == (ref.status, ref.iters, ref.restarts), k
        assert equal(res.hist_l2[k], ref.hist_l2) and equal(xs[k], ref.x), k


# --------------------------------------------------------------------------
# Convection-dominated case (X = 2, Y = 1, eps = 1e-3, upwind) at the sizes
# where ILU(0)-BiCGSTAB stops converging
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,bc,precision,maxit", [(192, 0, "fp32_factors", 3000), (256, 1, "fp64", 3000),
                                                   (384, 0, "fp32_factors", 30), (384, 1, "fp32_factors", 30)])
def test_convection_dominated_upwind_parity(adr, n, bc, precision, maxit):
    """192^2 and 256^2 converge (with a restart) and agree to the last bit;
    from 384^2 the iterate blows up (||r|| ~ 1e40 ||b|| within 35 passes) and
    the solve ends INACCURATE in the oracle.  Once the iterate has blown up
    the inner products cancel far beyond the double-double accumulation's
    order-independence (O(u^2 sum|x_k y_k|)), so at 384^2 the first 30
    passes are compared."""
    say("convection-dominated upwind", n, bc, precision, maxit)
    prob = adr.assemble(1e-3, 2.0, 1.0, n, n, "upwind", bc)
    prob.ilu0(precision)
    res = prob.solve(1e-10, maxit)
    P = orc.assemble(1e-3, 2.0, 1.0, n, n, 0, bc)
    F = orc.ilu0(P)
    if precision == "fp32_factors":
        F = orc.round_factors_f32(F)
    ref = orc.bicgstab(P, F, tol=1e-10, maxit=maxit)
    say("  status %d passes %d restarts %d true relres %.2e" % (res.status, res.iters, res.restarts,
                                                                res.true_relres))
    same_solve(res, host(res.x), ref)


# --------------------------------------------------------------------------
# Full size: 4096^2 with Neumann data on x = X, y = Y (the boundary mix of the
# large single-instance workload), the first passes bit for bit
# --------------------------------------------------------------------------

@pytest.mark.slow
@pytest.mark.parametrize("scheme", [0, 1])
def test_full_size_neumann_prefix_parity(adr, scheme):
    n = 4096
    say("full size neumann prefix", scheme)
    prob = adr.assemble(0.01, 1.0, 1.0, n, n, scheme, 1)
    prob.ilu0()
    res = prob.solve(1e-10, 3)
    x = host(res.x)
    del prob
    P = orc.assemble(0.01, 1.0, 1.0, n, n, scheme, 1)
    ref = orc.bicgstab(P, orc.ilu0(P), tol=1e-10, maxit=3)
    same_solve(res, x, ref)


# --------------------------------------------------------------------------
# The 256-instance batch: every instance that does not converge
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_batch_instances_that_do_not_converge_match_the_oracle(adr):
    """The seeded batch in the benchmark's configuration (FP32 factors,
    autotuned strips): for every instance whose status is not OK, the oracle
    with the same float factors gives the same first K passes (history and,
    when the instance stopped within them, status and solution) bit for bit."""
    K = 3
    inst = fields.batch_instances(256, seed=1308)
    flds = [fields.gaussian_random_field(d["n"], d["n"], d["X"] / (d["n"] + 1), d["Y"] / (d["n"] + 1),
                                        length=0.1, seed=1308, instance=k).ravel() for k, d in enumerate(inst)]
    cols = ([d["eps"] for d in inst], [d["X"] for d in inst], [d["Y"] for d in inst], [d["n"] for d in inst],
            [d["n"] for d in inst], [d["scheme"] for d in inst], [d["bc"] for d in inst])
    say("batch ill-posed instances")
    b = adr.assemble_batch(*cols, field=cuda(np.concatenate(flds)), amp=0.1)
    b.ilu0("fp32_factors")
    b.autotune()
    res = b.solve(1e-10, 2000)
    xs = b.split(res.x)
    bad = [k for k in range(len(inst)) if res.status[k] != adr.OK]
    say("  %d of %d instances not OK: %s" % (len(bad), len(inst), {int(s): int((res.status == s).sum())
                                                                     for s in np.unique(res.status)}))
    assert len(bad) > 0
    for k in bad:
        d = inst[k]
        P = orc.assemble(d["eps"], d["X"], d["Y"], d["n"], d["n"], d["scheme"], d["bc"], field=flds[k], amp=0.1)
        m = min(K, int(res.iters[k]))
        ref = orc.bicgstab(P, orc.round_factors_f32(orc.ilu0(P)), tol=1e-10, maxit=m)
        c = adr.classify(d["eps"], d["X"], d["Y"], d["n"], d["n"], d["scheme"], d["bc"])
        say("  instance %d n %d status %d passes %d (expected to fail: %s)" % (k, d["n"], res.status[k],
                                                                            res.iters[k], c.expect_fail))
        np.testing.assert_array_equal(res.hist_l2[k][:m + 1], ref.hist_l2[:m + 1])
        np.testing.assert_array_equal(res.hist_max[k][:m + 1], ref.hist_max[:m + 1])
        if res.iters[k] <= K:
            assert res.status[k] == ref.status
            assert equal(host(xs[k]), ref.x)


# --------------------------------------------------------------------------
# Assembly from user data, discretisation error, streaming copy
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny", [(37, 53), (64, 64), (1, 9), (130, 3)])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("mode", ["host", "device", "scalar"])
def test_assembly_from_user_data_bitwise(adr, nx, ny, bc, mode):
    say("assembly from data", nx, ny, bc, mode)
    rng = np.random.default_rng(nx * 100 + ny + bc)
    f = rng.standard_normal(nx * ny)
    edges = dict(u_x0=rng.standard_normal(ny), u_xX=rng.standard_normal(ny), u_y0=rng.standard_normal(nx),
                 u_yY=rng.standard_normal(nx))
    if mode == "scalar":
        fa, ea = 0.75, dict(u_x0=0.5, u_xX=-1.25, u_y0=2.0, u_yY=0.125)
        f_ref = np.full(nx * ny, 0.75)
        e_ref = dict(u_x0=np.full(ny, 0.5), u_xX=np.full(ny, -1.25), u_y0=np.full(nx, 2.0), u_yY=np.full(nx, 0.125))
    else:
        fa, ea, f_ref, e_ref = (cuda(f) if mode == "device" else f), edges, f, edges
    for scheme in (0, 1):
        prob = adr.assemble(0.07, 1.3, 0.9, nx, ny, scheme, bc, f=fa, **ea)
        g = prob.get_dia()
        P = orc.assemble_data(0.07, 1.3, 0.9, nx, ny, scheme, bc, f=f_ref, **e_ref)
        for name in ("S", "W", "C", "E", "N", "rhs"):
            assert equal(g[name], getattr(P, name)), name


def test_assembly_from_user_data_argument_errors(adr):
    with pytest.raises(adr.AdrError):
        adr.assemble(0.1, 1.0, 1.0, 8, 8, f=np.zeros(7))             # neither 1 nor 64 values
    with pytest.raises(adr.AdrError):
        adr.assemble(0.1, 1.0, 1.0, 8, 6, u_x0=np.zeros(8))          # x-sides take ny values
    with pytest.raises(adr.AdrError):
        adr.assemble(0.1, 1.0, 1.0, 8, 8, f=torch.zeros(1, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("nx,ny,scheme,bc,eps", [(64, 64, 0, 0, 0.1), (64, 64, 1, 0, 0.1), (37, 53, 1, 1, 2.0),
                                                 (19, 19, 0, 1, 4.0), (120, 31, 0, 1, 0.5), (1, 17, 1, 1, 1.0)])
def test_max_error_matches_the_oracle(adr, nx, ny, scheme, bc, eps):
    say("max error", nx, ny, scheme, bc, eps)
    prob = adr.assemble(eps, 1.3, 0.8, nx, ny, scheme, bc)
    prob.ilu0()
    res = prob.solve(1e-12, 2000)
    x = host(res.x)
    P = orc.assemble(eps, 1.3, 0.8, nx, ny, scheme, bc)
    e_gpu, e_ref = prob.max_error(res.x), orc.max_error(P, x)
    assert e_gpu == pytest.approx(e_ref, rel=1e-9, abs=1e-15)


def test_max_error_of_a_batch(adr):
    cases = [(0.1, 1.0, 1.0, 64, 64, 0, 0), (2.0, 1.0, 1.5, 37, 53, 1, 1), (0.5, 0.7, 1.2, 20, 9, 0, 1)]
    b = adr.assemble_batch(*zip(*cases))
    b.ilu0()
    res = b.solve(1e-12, 2000)
    errs = b.max_error(res.x)
    for k, (e, X, Y, nx, ny, sc, bc) in enumerate(cases):
        P = orc.assemble(e, X, Y, nx, ny, sc, bc)
        assert errs[k] == pytest.approx(orc.max_error(P, host(b.split(res.x)[k])), rel=1e-9, abs=1e-15)


@pytest.mark.parametrize("n", [1, 2, 1001, 1 << 20, (1 << 22) + 3])
def test_stream_copy(adr, n):
    a = torch.randn(n, dtype=torch.float64, device="cuda")
    b = torch.full_like(a, float("nan"))
    adr.stream_copy(a, b)
    assert torch.equal(a, b)
