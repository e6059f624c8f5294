"""GPU (HIP, through the C ABI) against the CPU oracle, element by element, on
the same seeded inputs.

Bars: the assembly, SpMV, ILU(0) factors, L/U sweeps and inner products use
the same fixed per-point fma orders and double-double reductions on both
sides, so they must agree bit for bit.  Full solves must satisfy the stated
parity target: max |x_gpu - x_cpu| / max |x_cpu| <= 1e-9 at tolerance 1e-10
and iteration counts within +-2 (in practice they agree exactly).
"""
import numpy as np
import pytest

from oracle import core as orc
from synthetic import fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


SHAPES = [(64, 64), (37, 53), (1, 20), (20, 1), (1, 1), (130, 67), (33, 96)]


def oracle_problem(eps, X, Y, nx, ny, scheme, bc, field=None, amp=0.0):
    return orc.assemble(eps, X, Y, nx, ny, scheme, bc, field=field, amp=amp)


def equal(a, b):
    return np.array_equal(a, b) or (np.array_equal(np.isnan(a), np.isnan(b)) and
                                    np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)]))


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("bc", [0, 1])
def test_assembly_bitwise(adr, nx, ny, scheme, bc):
    say("assembly", nx, ny, scheme, bc)
    eps, X, Y = 0.07, 1.3, 0.9
    prob = adr.assemble(eps, X, Y, nx, ny, scheme, bc)
    g = prob.get_dia()
    P = oracle_problem(eps, X, Y, nx, ny, scheme, bc)
    for name in ("S", "W", "C", "E", "N", "rhs"):
        assert equal(g[name], getattr(P, name)), name


@pytest.mark.parametrize("nx,ny", [(64, 64), (70, 41)])
def test_assembly_with_random_forcing_bitwise(adr, nx, ny):
    say("assembly+field", nx, ny)
    g = fields.gaussian_random_field(nx, ny, 1.0 / (nx + 1), 1.0 / (ny + 1), length=0.1, seed=3, instance=1)
    prob = adr.assemble(0.05, 1.0, 1.0, nx, ny, 1, 0, field=cuda(g.ravel()), amp=0.1)
    d = prob.get_dia()
    P = oracle_problem(0.05, 1.0, 1.0, nx, ny, 1, 0, field=g.ravel(), amp=0.1)
    assert equal(d["rhs"], P.rhs)
    assert equal(d["C"], P.C)


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_spmv_bitwise(adr, nx, ny):
    say("spmv", nx, ny)
    prob = adr.assemble(0.3, 1.0, 2.0, nx, ny, 0, 1)
    P = oracle_problem(0.3, 1.0, 2.0, nx, ny, 0, 1)
    x = np.random.default_rng(nx * 1000 + ny).standard_normal(nx * ny)
    v = host(prob.spmv(cuda(x)))
    assert equal(v, orc.spmv(P, x))


@pytest.mark.parametrize("n", [1, 255, 256, 257, 4096, 100003, 1 << 20])
def test_dot_bitwise(adr, n):
    say("dot", n)
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) * 10.0 ** rng.integers(-6, 6, n)
    y = rng.standard_normal(n)
    assert adr.dot(cuda(x), cuda(y)) == orc.dot(x, y)


@pytest.mark.parametrize("rows", [16, 32])
@pytest.mark.parametrize("nx,ny,scheme,bc,eps", [
    (64, 64, 0, 0, 0.1), (37, 53, 1, 1, 2.0), (1, 40, 1, 0, 0.5), (45, 1, 0, 0, 0.5),
    (130, 67, 1, 0, 0.01), (33, 140, 0, 1, 1.0), (200, 200, 1, 0, 0.05), (50, 33, 0, 0, 0.2)])
def test_ilu0_and_sweeps_bitwise(adr, rows, nx, ny, scheme, bc, eps):
    say("ilu0+sweeps", rows, nx, ny, scheme, bc, eps)
    prob = adr.assemble(eps, 1.0, 1.0, nx, ny, scheme, bc)
    prob.set_sweep_rows(rows)
    prob.ilu0()
    f = prob.get_factors()
    P = oracle_problem(eps, 1.0, 1.0, nx, ny, scheme, bc)
    F = orc.ilu0(P)
    assert F.status == orc.OK
    for name in ("lw", "ls", "invd"):
        assert equal(f[name], getattr(F, name)), name
    q = np.random.default_rng(rows + nx).standard_normal(nx * ny)
    z = host(prob.precond(cuda(q)))
    zo = orc.usolve(nx, ny, F, orc.lsolve(nx, ny, F, q))
    assert equal(z, zo)
    # repeated application: the hand-off memory resets itself
    z2 = host(prob.precond(cuda(q)))
    assert equal(z2, zo)


def solve_both(adr, eps, X, Y, nx, ny, scheme, bc, tol=1e-10, maxit=2000, rows=0, x0=None, precision="fp64"):
    prob = adr.assemble(eps, X, Y, nx, ny, scheme, bc)
    if rows:
        prob.set_sweep_rows(rows)
    prob.ilu0(precision)
    res = prob.solve(tol=tol, maxit=maxit, x0=None if x0 is None else cuda(x0))
    P = oracle_problem(eps, X, Y, nx, ny, scheme, bc)
    ref = orc.bicgstab(P, orc.ilu0(P), tol=tol, maxit=maxit, x0=x0)
    return prob, res, P, ref


def maxrel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("scheme", [0, 1])
def test_solve_small_config_parity(adr, scheme):
    """X = Y = 1, eps = 0.1, 64 x 64, Dirichlet, zero guess, tol 1e-10."""
    say("solve 64x64", scheme)
    prob, res, P, ref = solve_both(adr, 0.1, 1.0, 1.0, 64, 64, scheme, 0)
    assert res.status == adr.OK and ref.status == orc.OK
    assert abs(res.iters - ref.iters) <= 2
    x = host(res.x)
    assert maxrel(x, ref.x) <= 1e-9
    n = min(len(res.hist_l2), len(ref.hist_l2))
    np.testing.assert_allclose(res.hist_l2[:n], ref.hist_l2[:n], rtol=1e-9)
    np.testing.assert_allclose(res.hist_max[:n], ref.hist_max[:n], rtol=1e-9)
    assert res.true_relres == pytest.approx(ref.true_relres, rel=1e-6)
    # the discretisation error matches the oracle's
    assert orc.max_error(P, x) == pytest.approx(orc.max_error(P, ref.x), rel=1e-6)


@pytest.mark.parametrize("rows", [16, 32])
@pytest.mark.parametrize("nx,ny,scheme,bc,eps,X,Y", [
    (127, 129, 0, 0, 0.01, 1.0, 1.0), (100, 80, 1, 1, 2.0, 1.0, 1.0), (257, 130, 1, 0, 0.05, 2.0, 1.0),
    (19, 19, 0, 1, 4.0, 4.0, 4.0), (5, 300, 1, 0, 0.2, 1.0, 1.0)])
def test_solve_parity(adr, rows, nx, ny, scheme, bc, eps, X, Y):
    say("solve", rows, nx, ny, scheme, bc, eps)
    prob, res, P, ref = solve_both(adr, eps, X, Y, nx, ny, scheme, bc, rows=rows)
    assert res.status == ref.status
    assert abs(res.iters - ref.iters) <= 2
    assert res.half_step == ref.half_step or abs(res.iters - ref.iters) > 0
    assert maxrel(host(res.x), ref.x) <= 1e-9


@pytest.mark.parametrize("nx,ny,scheme,bc", [(1, 1, 0, 0), (1, 1, 1, 1), (1, 300, 0, 1), (300, 1, 1, 0),
                                              (1, 70, 1, 0), (70, 1, 0, 1)])
def test_one_dimensional_grids_solve_in_one_pass(adr, nx, ny, scheme, bc):
    """With one row or one column the 5-point matrix is tridiagonal (or 1x1),
    ILU(0) is its exact LU factorisation, and BiCGSTAB stops in the first pass
    (on the s test) on the GPU as in the oracle."""
    say("1-D solve", nx, ny, scheme, bc)
    prob, res, P, ref = solve_both(adr, 0.2, 1.0, 1.0, nx, ny, scheme, bc)
    assert ref.status == orc.OK and ref.iters == 1
    assert res.status == adr.OK and res.iters == ref.iters and res.half_step == ref.half_step
    assert maxrel(host(res.x), ref.x) <= 1e-9
    assert res.true_relres < 1e-11


def test_solve_status_parity(adr):
    say("status")
    # maxit = 1
    prob, res, P, ref = solve_both(adr, 0.1, 1.0, 1.0, 30, 30, 0, 0, maxit=1)
    assert res.status == adr.MAXIT == ref.status and res.iters == 1 == ref.iters
    assert np.array_equal(host(res.x), ref.x)
    # immediate convergence from the exact discrete solution of the oracle
    import oracle.dense as dense
    P = oracle_problem(0.1, 1.0, 1.0, 12, 12, 1, 0)
    xe = dense.exact_discrete(P)
    prob, res, P, ref = solve_both(adr, 0.1, 1.0, 1.0, 12, 12, 1, 0, x0=xe)
    assert res.status == ref.status and res.iters == ref.iters
    # 1-D grids: ILU(0) is exact, the half-step exit of pass 1
    prob, res, P, ref = solve_both(adr, 0.2, 1.0, 1.0, 1, 50, 1, 0)
    assert res.status == adr.OK and res.iters == 1 and res.half_step and ref.half_step
    assert maxrel(host(res.x), ref.x) <= 1e-12


def test_zero_pivot_and_nonfinite(adr):
    say("zero pivot / nonfinite")
    prob = adr.assemble(0.1, 1.0, 1.0, 20, 20, 0, 0)
    d = prob.get_dia()
    d["C"][47] = 0.0
    d["W"][47] = 0.0
    d["S"][47] = 0.0
    prob.set_dia(**d)
    with pytest.raises(adr.AdrError) as ei:
        prob.ilu0()
    P = orc.Problem(0.1, 1.0, 1.0, 20, 20, 0, 0, d["S"], d["W"], d["C"], d["E"], d["N"], d["rhs"])
    F = orc.ilu0(P)
    assert F.status == orc.ZERO_PIVOT
    assert str(F.bad) in str(ei.value)
    # NaN in the forcing -> NONFINITE on both sides
    g = np.zeros(400)
    g[123] = np.nan
    prob = adr.assemble(0.1, 1.0, 1.0, 20, 20, 0, 0, field=cuda(g), amp=0.1)
    prob.ilu0()
    res = prob.solve(1e-10, 50)
    P = oracle_problem(0.1, 1.0, 1.0, 20, 20, 0, 0, field=g, amp=0.1)
    ref = orc.bicgstab(P, orc.ilu0(P), 1e-10, 50)
    assert res.status == adr.NONFINITE == ref.status
    # b = 0 gives x = 0 and no pass
    prob = adr.assemble(0.1, 1.0, 1.0, 10, 10, 0, 0)
    d = prob.get_dia()
    d["rhs"][:] = 0.0
    prob.set_dia(**d)
    prob.ilu0()
    res = prob.solve(1e-10, 10, x0=cuda(np.ones(100)))
    assert res.status == adr.OK and res.iters == 0 and not host(res.x).any()


@pytest.mark.parametrize("scheme,bc,precision", [(0, 0, "fp64"), (1, 1, "fp64"), (1, 0, "fp32_factors"),
                                               (0, 1, "fp32_sweeps")])
def test_stencil_tables_change_no_bit(adr, scheme, bc, precision):
    """An assembled operator is solved with S, W, E, N read from its column and
    row tables; forbidding the tables (full diagonals) gives the same bits in
    the preconditioner and in the whole solve."""
    say("stencil tables", scheme, bc, precision)
    prob = adr.assemble(0.05, 1.3, 0.8, 97, 75, scheme, bc)
    assert prob.stencil_tables
    prob.ilu0(precision)
    q = np.random.default_rng(5).standard_normal(97 * 75)
    z_tab = host(prob.precond(cuda(q)))
    r_tab = prob.solve(1e-10, 3000)
    x_tab = host(r_tab.x)
    prob.use_stencil_tables(False)
    assert not prob.stencil_tables
    z_dia = host(prob.precond(cuda(q)))
    r_dia = prob.solve(1e-10, 3000)
    assert equal(z_tab, z_dia)
    assert r_tab.status == r_dia.status and r_tab.iters == r_dia.iters
    assert equal(x_tab, host(r_dia.x))
    assert equal(r_tab.hist_l2, r_dia.hist_l2) and equal(r_tab.hist_max, r_dia.hist_max)
    prob.use_stencil_tables(True)
    assert prob.stencil_tables
    # single-step calls report the device time of their kernels
    prob.usolve(cuda(q))
    assert 0.0 < prob.last_call_ms < 1000.0


def test_operator_that_is_not_separable_uses_the_diagonals(adr):
    """A matrix given through set_dia whose W varies along a column is
    detected, solved from the full diagonals and matches the oracle; the
    original (separable) matrix turns the tables back on."""
    say("non-separable operator")
    nx, ny = 64, 48
    prob = adr.assemble(0.05, 1.0, 1.0, nx, ny, 1, 0)
    orig = prob.get_dia()
    d = {k: v.copy() for k, v in orig.items()}
    d["W"][20 * nx + 30] *= 1.25
    d["N"][7 * nx + 3] *= 0.75
    prob.set_dia(**d)
    assert not prob.stencil_tables
    prob.ilu0()
    f = prob.get_factors()
    P = orc.Problem(0.05, 1.0, 1.0, nx, ny, 1, 0, d["S"], d["W"], d["C"], d["E"], d["N"], d["rhs"])
    F = orc.ilu0(P)
    assert equal(f["lw"], F.lw) and equal(f["invd"], F.invd)
    q = np.random.default_rng(9).standard_normal(nx * ny)
    assert equal(host(prob.precond(cuda(q))), orc.usolve(nx, ny, F, orc.lsolve(nx, ny, F, q)))
    res = prob.solve(1e-10, 2000)
    ref = orc.bicgstab(P, F, tol=1e-10, maxit=2000)
    assert res.status == ref.status == orc.OK and abs(res.iters - ref.iters) <= 2
    assert maxrel(host(res.x), ref.x) <= 1e-9
    prob.set_dia(**orig)
    assert prob.stencil_tables


def test_caller_workspace_gives_the_same_solve(adr):
    """Factors, iteration vectors and hand-off memory carved out of a torch
    tensor: the same bits as with the library's own allocations, less
    library-allocated memory, and the binding rules enforced."""
    say("workspace")
    ref = adr.assemble(0.05, 1.0, 1.0, 90, 70, 1, 0)
    ref.ilu0()
    r0 = ref.solve(1e-10, 2000)
    prob = adr.assemble(0.05, 1.0, 1.0, 90, 70, 1, 0)
    need = prob.workspace_bytes()
    assert need >= 12 * 90 * 70 * 8 and prob.workspace_bytes("fp32_factors") > need
    with pytest.raises(adr.AdrError):     # too small
        prob.bind_workspace(torch.empty(need - 256, dtype=torch.uint8, device="cuda"))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    prob.bind_workspace(ws)
    with pytest.raises(adr.AdrError):     # only once
        prob.bind_workspace(ws)
    before = prob.device_bytes
    prob.ilu0()
    r1 = prob.solve(1e-10, 2000)
    assert r1.status == r0.status and r1.iters == r0.iters
    assert equal(host(r1.x), host(r0.x)) and equal(r1.hist_l2, r0.hist_l2)
    # the library allocated only the histories beyond the assembly
    assert prob.device_bytes - before < ref.device_bytes - before
    with pytest.raises(adr.AdrError):     # FP32 factors need more than this workspace holds
        prob.ilu0("fp32_factors")
    # bound after ilu0: refused
    late = adr.assemble(0.05, 1.0, 1.0, 20, 20, 0, 0)
    late.ilu0()
    with pytest.raises(adr.AdrError):
        late.bind_workspace(torch.empty(late.workspace_bytes(), dtype=torch.uint8, device="cuda"))
    # a batch
    b = adr.assemble_batch([0.1, 0.3], [1.0, 1.5], [1.0, 0.7], [40, 33], [25, 50], ["upwind", "centered"],
                           ["dirichlet", "neumann"])
    wsb = torch.empty(b.workspace_bytes("fp32_factors"), dtype=torch.uint8, device="cuda")
    b.bind_workspace(wsb)
    b.ilu0("fp32_factors")
    rb = b.solve(tol=1e-10, maxit=500)
    b2 = adr.assemble_batch([0.1, 0.3], [1.0, 1.5], [1.0, 0.7], [40, 33], [25, 50], ["upwind", "centered"],
                            ["dirichlet", "neumann"])
    b2.ilu0("fp32_factors")
    rb2 = b2.solve(tol=1e-10, maxit=500)
    assert np.array_equal(rb.iters, rb2.iters) and equal(host(rb.x), host(rb2.x))


def test_one_call_solve(adr):
    """adr.solve: assemble, ilu0 and solve in one call, returning
    (x, hist_l2, hist_max, iters, status) -- the oracle's result."""
    say("one-call solve")
    x, h2, hm, iters, status = adr.solve(0.1, 1.0, 1.0, 64, 64, "centered", "dirichlet", tol=1e-10, maxit=500)
    P = oracle_problem(0.1, 1.0, 1.0, 64, 64, 1, 0)
    ref = orc.bicgstab(P, orc.ilu0(P), tol=1e-10, maxit=500)
    assert status == adr.OK == ref.status and abs(iters - ref.iters) <= 2
    assert maxrel(host(x), ref.x) <= 1e-9
    assert len(h2) == len(hm) == iters + 1
    amp = adr.amplification(h2)
    assert amp.shape == (iters,) and np.all(amp > 0)


def test_argument_errors(adr):
    with pytest.raises(adr.AdrError):
        adr.assemble(0.0, 1.0, 1.0, 8, 8)
    with pytest.raises(adr.AdrError):
        adr.assemble(1.0, 1.0, 1.0, 0, 8)
    prob = adr.assemble(1.0, 1.0, 1.0, 8, 8)
    with pytest.raises(adr.AdrError):   # solve before ilu0
        prob.solve(1e-10, 10)
    prob.ilu0()
    with pytest.raises(adr.AdrError):
        prob.solve(-1.0, 10)


def test_repeated_solves_are_identical(adr):
    say("repeat")
    prob = adr.assemble(0.01, 1.0, 1.0, 150, 150, 1, 0)
    prob.ilu0()
    a = prob.solve(1e-10, 1000)
    xa = host(a.x)
    b = prob.solve(1e-10, 1000)
    assert a.iters == b.iters and np.array_equal(xa, host(b.x))
    assert np.array_equal(a.hist_l2, b.hist_l2)


@pytest.mark.slow
@pytest.mark.parametrize("scheme", [0, 1])
def test_full_size_prefix_parity(adr, scheme):
    """4096 x 4096 (the large single-instance grid), eps = 0.01, Dirichlet,
    in the launch configuration the benchmark uses: the first 3 passes of the
    GPU solve equal the oracle's bit for bit (x and both histories)."""
    n = 4096
    say("full size prefix", scheme)
    prob = adr.assemble(0.01, 1.0, 1.0, n, n, scheme, 0)
    prob.ilu0()
    res = prob.solve(1e-10, 3)
    x = host(res.x)
    P = oracle_problem(0.01, 1.0, 1.0, n, n, scheme, 0)
    ref = orc.bicgstab(P, orc.ilu0(P), tol=1e-10, maxit=3)
    assert res.status == ref.status == orc.MAXIT
    assert np.array_equal(res.hist_l2, ref.hist_l2)
    assert np.array_equal(res.hist_max, ref.hist_max)
    assert equal(x, ref.x)


@pytest.mark.slow
def test_large_grid_prefix_parity(adr):
    """8192 x 8192, X = 2, Y = 1, eps = 1e-3, centered, FP32-stored factors
    with FP64 BiCGSTAB (the convection-dominated large grid, in the launch
    configuration the benchmark uses): the first 2 passes equal the oracle's
    passes with the same float factors bit for bit."""
    n = 8192
    say("large grid prefix")
    prob = adr.assemble(1e-3, 2.0, 1.0, n, n, 1, 0)
    prob.ilu0("fp32_factors")
    res = prob.solve(1e-10, 2)
    x = host(res.x)
    del prob
    P = oracle_problem(1e-3, 2.0, 1.0, n, n, 1, 0)
    ref = orc.bicgstab(P, orc.round_factors_f32(orc.ilu0(P)), tol=1e-10, maxit=2)
    assert res.status == ref.status == orc.MAXIT
    assert np.array_equal(res.hist_l2, ref.hist_l2)
    assert np.array_equal(res.hist_max, ref.hist_max)
    assert equal(x, ref.x)


@pytest.mark.slow
def test_batch_workload_sampled_instances_match_oracle(adr):
    """The 256-instance batched workload in the benchmark's configuration
    (FP32 factors, autotuned strips, one batch): three of its instances,
    solved again by the oracle with the same float factors, agree in status,
    pass count, history and solution bit for bit."""
    say("batch workload sample")
    inst = fields.batch_instances(256, seed=1308)
    flds = [fields.gaussian_random_field(d["n"], d["n"], d["X"] / (d["n"] + 1), d["Y"] / (d["n"] + 1),
                                        length=0.1, seed=1308, instance=k).ravel() for k, d in enumerate(inst)]
    cols = ([d["eps"] for d in inst], [d["X"] for d in inst], [d["Y"] for d in inst], [d["n"] for d in inst],
            [d["n"] for d in inst], [d["scheme"] for d in inst], [d["bc"] for d in inst])
    b = adr.assemble_batch(*cols, field=cuda(np.concatenate(flds)), amp=0.1)
    b.ilu0("fp32_factors")
    b.autotune()
    res = b.solve(1e-10, 2000)
    xs = b.split(res.x)
    order = sorted(range(len(inst)), key=lambda k: inst[k]["n"])
    sample = [order[0], order[1], order[len(order) // 8]]
    for k in sample:
        d = inst[k]
        P = oracle_problem(d["eps"], d["X"], d["Y"], d["n"], d["n"], d["scheme"], d["bc"], field=flds[k], amp=0.1)
        ref = orc.bicgstab(P, orc.round_factors_f32(orc.ilu0(P)), tol=1e-10, maxit=2000)
        say("  instance %d n %d: status %d/%d passes %d/%d" % (k, d["n"], res.status[k], ref.status,
                                                              res.iters[k], ref.iters))
        assert res.status[k] == ref.status
        assert res.iters[k] == ref.iters
        np.testing.assert_array_equal(res.hist_l2[k], ref.hist_l2)
        assert equal(host(xs[k]), ref.x)


@pytest.mark.parametrize("rows", [16, 32])
@pytest.mark.parametrize("precision", ["fp32_factors", "fp32_sweeps"])
def test_mixed_precision_precond_bitwise(adr, rows, precision):
    """FP32-stored factors (rounded from the FP64 ILU(0)) applied with FP64
    or FP32 sweep arithmetic equal the oracle's substitutions of the same
    float factors."""
    say("mixed precond", rows, precision)
    nx, ny = 150, 97
    prob = adr.assemble(0.02, 1.0, 1.0, nx, ny, 1, 0)
    prob.set_sweep_rows(rows)
    prob.ilu0(precision)
    P = oracle_problem(0.02, 1.0, 1.0, nx, ny, 1, 0)
    F = orc.round_factors_f32(orc.ilu0(P))
    q = np.random.default_rng(9).standard_normal(nx * ny)
    z = host(prob.precond(cuda(q)))
    if precision == "fp32_factors":
        zo = orc.usolve(nx, ny, F, orc.lsolve(nx, ny, F, q))
    else:
        zo = orc.usolve_f32(nx, ny, F, orc.lsolve_f32(nx, ny, F, q))
    assert equal(z, zo)


@pytest.mark.parametrize("precision", ["fp32_factors", "fp32_sweeps"])
@pytest.mark.parametrize("scheme", [0, 1])
def test_mixed_precision_solve(adr, precision, scheme):
    """Mixed-precision solves match the oracle run in the same mode, and their
    error against the FP64 oracle solution is stated (and bounded)."""
    say("mixed solve", precision, scheme)
    n, eps = 200, 0.01
    prob = adr.assemble(eps, 1.0, 1.0, n, n, scheme, 0)
    prob.ilu0(precision)
    res = prob.solve(1e-10, 3000)
    x = host(res.x)
    P = oracle_problem(eps, 1.0, 1.0, n, n, scheme, 0)
    F = orc.ilu0(P)
    ref = orc.bicgstab(P, orc.round_factors_f32(F), tol=1e-10, maxit=3000, sweep_f32=(precision == "fp32_sweeps"))
    ref64 = orc.bicgstab(P, F, tol=1e-10, maxit=3000)
    assert res.status == ref.status == orc.OK
    assert abs(res.iters - ref.iters) <= 2
    assert maxrel(x, ref.x) <= 1e-9
    err64 = maxrel(x, ref64.x)
    say("  iters %d (fp64 oracle %d), max-rel-diff vs fp64 oracle %.2e" % (res.iters, ref64.iters, err64))
    assert err64 <= 1e-6
    # the discretisation error is within 1% of the FP64 oracle's
    e_mixed, e64 = orc.max_error(P, x), orc.max_error(P, ref64.x)
    assert abs(e_mixed - e64) <= 0.01 * e64


# --------------------------------------------------------------------------
# Batches: many instances advanced by the same launches
# --------------------------------------------------------------------------

BATCH = [  # eps, X, Y, nx, ny, scheme, bc
    (0.1, 1.0, 1.0, 64, 64, 0, 0), (2.0, 1.0, 1.0, 37, 53, 1, 1), (0.01, 1.0, 1.0, 130, 67, 1, 0),
    (0.5, 1.0, 1.0, 1, 40, 1, 0), (0.5, 1.0, 1.0, 45, 1, 0, 0), (0.01, 1.0, 1.0, 96, 96, 0, 1),
    (0.003, 0.7, 1.6, 160, 128, 0, 0), (0.2, 1.9, 0.6, 33, 200, 1, 1), (0.3, 1.2, 0.8, 1, 1, 0, 1),
    (0.05, 1.0, 1.0, 2, 3, 1, 0)]


@pytest.mark.parametrize("with_field", [False, True])
def test_batch_matches_oracle_instance_by_instance(adr, with_field):
    say("batch", with_field)
    cols = list(zip(*BATCH))
    fields, flat = [], None
    if with_field:
        for k, (eps, X, Y, nx, ny, sc, bc) in enumerate(BATCH):
            fields.append(fields_grf(nx, ny, X, Y, k))
        flat = np.concatenate(fields)
    b = adr.assemble_batch(*cols, field=None if flat is None else cuda(flat), amp=0.1)
    b.ilu0()
    res = b.solve(1e-10, 1500)
    xs = [host(v) for v in b.split(res.x)]
    for k, (eps, X, Y, nx, ny, sc, bc) in enumerate(BATCH):
        P = oracle_problem(eps, X, Y, nx, ny, sc, bc, field=fields[k] if with_field else None,
                           amp=0.1 if with_field else 0.0)
        ref = orc.bicgstab(P, orc.ilu0(P), tol=1e-10, maxit=1500)
        assert res.status[k] == ref.status, (k, res.status[k], ref.status)
        assert res.iters[k] == ref.iters, (k, res.iters[k], ref.iters)
        np.testing.assert_array_equal(res.hist_l2[k], ref.hist_l2)
        assert equal(xs[k], ref.x), k


def fields_grf(nx, ny, X, Y, k):
    return fields.gaussian_random_field(nx, ny, X / (nx + 1), Y / (ny + 1), length=0.1, seed=1308, instance=k).ravel()


@pytest.mark.parametrize("precision", ["fp64", "fp32_factors", "fp32_sweeps"])
def test_sweep_ring_changes_no_bit(adr, precision):
    """32-row strips with one workgroup per CU (deep LDS ring) or two (compact
    ring) give the same preconditioner and the same solve, bit for bit, with
    the stencil tables and with the full diagonals."""
    say("sweep ring", precision)
    prob = adr.assemble(0.05, 1.3, 0.8, 97, 75, 1, 0)
    prob.ilu0(precision)
    q = np.random.default_rng(9).standard_normal(97 * 75)
    for tables in (True, False):
        prob.use_stencil_tables(tables)
        got = []
        for mode in (0, 1):
            prob.set_sweep_ring(mode)
            assert prob.sweep_ring == mode
            z = host(prob.precond(cuda(q)))
            r = prob.solve(1e-10, 3000)
            got.append((z, r, host(r.x)))
        (z0, r0, x0), (z1, r1, x1) = got
        assert equal(z0, z1)
        assert r0.status == r1.status and r0.iters == r1.iters
        assert equal(x0, x1) and equal(r0.hist_l2, r1.hist_l2) and equal(r0.hist_max, r1.hist_max)
    prob.use_stencil_tables(True)
    prob.set_sweep_ring(-1)
    assert prob.sweep_ring == 1   # three strips, one per CU: the automatic choice is the compact ring
    with pytest.raises(adr.AdrError):
        prob.set_sweep_ring(2)


def test_batch_autotune_keeps_results(adr):
    say("autotune")
    cols = list(zip(*BATCH[:4]))
    b = adr.assemble_batch(*cols)
    b.ilu0()
    r0 = b.solve(1e-10, 500)
    x0 = host(r0.x).copy()
    rows, ms = b.autotune()
    assert rows in (16, 32) and ms > 0
    r1 = b.solve(1e-10, 500)
    assert np.array_equal(host(r1.x), x0)
    assert list(r1.iters) == list(r0.iters)
    # both rings of the 32-row strips, forced
    for mode in (0, 1):
        b.set_sweep_rows(32)
        b.set_sweep_ring(mode)
        assert b.sweep_ring == mode
        r2 = b.solve(1e-10, 500)
        assert np.array_equal(host(r2.x), x0)
        assert list(r2.iters) == list(r0.iters)
    # strip heights are multiples of the 16-column chunk
    for bad in (15, 31, 48):
        with pytest.raises(adr.AdrError):
            b.set_sweep_rows(bad)
