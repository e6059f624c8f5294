"""GPU parity of the warm-start network (include/adr_cnn.h) against the CPU
FP64 reference (oracle/cnn.py), which rounds to bfloat16 at the same points:
the remaining differences come from FP32 accumulation and the rare bfloat16
rounding decision it flips, hence normwise tolerances."""
import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import core
from synthetic import warmstart as ws

pytestmark = pytest.mark.gpu

# (1, 52, 50): four 16 x 16 tiles whose halo lies inside the grid and nine
# whose outputs all do, so the bounds-test-free load and store paths run
SHAPES = [(2, 20, 20), (1, 19, 35), (3, 3, 3), (1, 34, 17), (1, 52, 50)]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(B, H, W, seed):
    """bfloat16-exact input fields [B, H, W, NFIELD] (float64) and the
    32-channel bfloat16 device tensor holding them."""
    torch = _torch()
    nf = ocnn.NFIELD
    x = ocnn.bf16(ws.random_fields(B, H, W, nf, seed=seed))
    pad = np.zeros((B, H, W, 32), dtype=np.float32)
    pad[..., :nf] = x
    return x, torch.from_numpy(pad).cuda().to(torch.bfloat16).contiguous()


def _params(seed):
    p = ws.initial_params(seed)
    r = np.random.default_rng(seed + 100)
    # non-zero biases so that the bias paths are exercised
    off = 0
    for ci, co in zip(ocnn.CIN, ocnn.COUT):
        off += 9 * ci * co
        p[off:off + co] = (0.1 * r.standard_normal(co)).astype(np.float32)
        off += co
    return p


def _net(H, W, B):
    import paper_1308_5215_amd as adr
    return adr.WarmStartNet(H, W, B)


# The reference rounds every stored activation to bfloat16 at the same points
# as the kernels but sums in FP64 where they sum in FP32, so now and then a
# pre-activation lands on the other side of a bfloat16 rounding boundary and
# one activation moves by one bfloat16 ulp (2^-8 relative); over the output
# such flips stay below half an ulp in the relative L2 norm.
U_TOL = 2.0 ** -9


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("B,H,W", SHAPES)
def test_forward_matches_reference(B, H, W):
    torch = _torch()
    p = _params(B * 7 + H)
    x, xd = _inputs(B, H, W, seed=H * 100 + W)
    net = _net(H, W, B)
    net.set_params(p)
    u = net.forward(xd).cpu().numpy()
    ref, _ = ocnn.forward(p.astype(np.float64), x, emulate=True)
    assert u.shape == ref.shape
    assert _rel(u, ref) <= U_TOL, _rel(u, ref)
    assert np.max(np.abs(u - ref)) <= 2e-2 * np.max(np.abs(ref))
    # the reference without bfloat16 rounding is measurably further away
    raw, _ = ocnn.forward(p.astype(np.float64), x, emulate=False)
    if H * W > 100:
        assert _rel(u, raw) > _rel(u, ref)


@pytest.mark.parametrize("B,H,W", SHAPES)
def test_gradient_matches_reference(B, H, W):
    torch = _torch()
    p = _params(B + H + W)
    x, xd = _inputs(B, H, W, seed=H * 31 + W)
    t = np.random.default_rng(H + W).standard_normal((B, H - 2, W - 2)).astype(np.float32)
    net = _net(H, W, B)
    net.set_params(p)
    loss, g, u = net.gradient(xd, torch.from_numpy(t).cuda(), want_u=True)
    rl, rg, ru = ocnn.loss_and_grad(p.astype(np.float64), x, t.astype(np.float64), emulate=True)
    # the loss moves by 2 (u - t).du / N: with |du| <= U_TOL |u| and random
    # targets (|u - t| >= |u|) its relative change is below about 2 U_TOL
    assert abs(loss - rl) <= U_TOL * rl
    assert _rel(u.cpu().numpy(), ru) <= U_TOL
    off = 0
    for l, (ci, co) in enumerate(zip(ocnn.CIN, ocnn.COUT)):
        nw = 9 * ci * co
        gw, rw = g[off:off + nw], rg[off:off + nw]
        gb, rb = g[off + nw:off + nw + co], rg[off + nw:off + nw + co]
        assert _rel(gw, rw) <= 5e-3, (l, _rel(gw, rw))
        assert _rel(gb, rb) <= 5e-3, (l, _rel(gb, rb))
        off += nw + co


def test_gradient_is_deterministic_and_batch_slices_are_independent():
    torch = _torch()
    B, H, W = 3, 20, 18
    p = _params(3)
    x, xd = _inputs(B, H, W, seed=9)
    t = torch.from_numpy(np.random.default_rng(1).standard_normal((B, H - 2, W - 2)).astype(np.float32)).cuda()
    net = _net(H, W, B)
    net.set_params(p)
    l1, g1 = net.gradient(xd, t)
    l2, g2 = net.gradient(xd, t)
    assert l1 == l2 and np.array_equal(g1, g2)
    u_all = net.forward(xd).cpu().numpy()
    u_one = net.forward(xd[1:2].contiguous()).cpu().numpy()
    assert np.array_equal(u_all[1:2], u_one)


def test_adam_steps_follow_the_reference():
    torch = _torch()
    B, H, W = 2, 18, 18
    p = _params(11)
    x, xd = _inputs(B, H, W, seed=4)
    t = np.random.default_rng(2).standard_normal((B, H - 2, W - 2))
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    net = _net(H, W, B)
    net.set_params(p)
    opt = ocnn.Adam(p.astype(np.float64), lr=1e-3)
    for step in range(3):
        lg = net.train_step(xd, td, lr=1e-3)
        lr_, gr, _ = ocnn.loss_and_grad(opt.p, x, t, emulate=True)
        opt.step(gr)
        assert abs(lg - lr_) <= 1e-3 * lr_, (step, lg, lr_)
    pg = net.get_params().astype(np.float64)
    dref = opt.p - p
    assert np.linalg.norm((pg - p) - dref) <= 0.05 * np.linalg.norm(dref)


def test_training_lowers_the_loss():
    torch = _torch()
    B, H, W = 4, 18, 18
    x, xd = _inputs(B, H, W, seed=21)
    t = torch.from_numpy((0.5 * x[:, 1:-1, 1:-1, 0] - 0.25 * x[:, 1:-1, 1:-1, 2]).astype(np.float32)).cuda()
    net = _net(H, W, B)
    net.set_params(ws.initial_params(5))
    first = net.train_step(xd, t, lr=3e-3)
    for _ in range(150):
        last = net.train_step(xd, t, lr=3e-3)
    assert last < 0.2 * first, (first, last)


def test_bad_arguments_are_rejected():
    torch = _torch()
    import paper_1308_5215_amd as adr
    with pytest.raises(adr.AdrError):
        adr.WarmStartNet(2, 10, 1)
    net = _net(10, 10, 2)
    _, xd = _inputs(3, 10, 10, seed=0)
    with pytest.raises(adr.AdrError):
        net.forward(xd)              # batch 3 > max_batch 2
    with pytest.raises(adr.AdrError):
        net.adam()                   # no gradient yet
    with pytest.raises(ValueError):
        net.set_params(np.zeros(10, np.float32))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_features_match_reference(bc):
    torch = _torch()
    import paper_1308_5215_amd as adr
    from synthetic.fields import gaussian_random_field
    n, count = 21, 3
    inst = [ws.warmstart_instance(s, n=n) for s in range(count)]
    fields = [gaussian_random_field(n, n, d["X"] / (n + 1), d["Y"] / (n + 1), seed=d["field_seed"]).ravel()
              for d in inst]
    fd = torch.from_numpy(np.concatenate(fields)).cuda()
    bcs = [bc] * count
    schemes = ["upwind", "centered", "upwind"][:count]
    batch = adr.assemble_batch([d["eps"] for d in inst], [d["X"] for d in inst], [d["Y"] for d in inst],
                               [n] * count, [n] * count, schemes, bcs, field=fd, amp=0.1)
    got = batch.features().float().cpu().numpy().astype(np.float64)
    assert got.shape == (count, n + 2, n + 2, 32)
    nf = ocnn.NFIELD
    assert np.all(got[..., nf:] == 0)
    b = core.DIRICHLET if bc == "dirichlet" else core.NEUMANN
    for k, d in enumerate(inst):
        sc = core.CENTERED if schemes[k] == "centered" else core.UPWIND
        ref = ocnn.bf16(ocnn.features(d["eps"], d["X"], d["Y"], n, n, b, field=fields[k], amp=0.1, scheme=sc))
        # device and host exponentials may differ in the last bit: one bfloat16 step at most
        assert np.all(np.abs(got[k, ..., :nf] - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-30)
        assert np.mean(got[k, ..., :nf] == ref) > 0.99


def test_warm_start_falls_back_to_zero_for_a_useless_guess():
    torch = _torch()
    import paper_1308_5215_amd as adr
    n, count = 24, 4
    inst = [ws.warmstart_instance(s, n=n) for s in range(10, 10 + count)]
    args = ([d["eps"] for d in inst], [d["X"] for d in inst], [d["Y"] for d in inst], [n] * count, [n] * count,
            ["upwind"] * count, ["dirichlet"] * count)
    batch = adr.assemble_batch(*args)
    batch.ilu0()
    net = _net(n + 2, n + 2, 3)
    p = np.full(adr.cnn_param_count(), np.nan, dtype=np.float32)
    net.set_params(p)
    x0, used = batch.warm_start(net)
    assert not used.any()
    assert torch.all(x0 == 0)
    zero = batch.solve(tol=1e-10, maxit=500)
    warm = batch.solve(tol=1e-10, maxit=500, x0=x0)
    assert np.array_equal(zero.iters, warm.iters)
    assert torch.equal(zero.x, warm.x)
    # an all-zero network predicts u = 0: the fallback keeps nothing either
    net.set_params(np.zeros(adr.cnn_param_count(), dtype=np.float32))
    _, used = batch.warm_start(net)
    assert not used.any()
