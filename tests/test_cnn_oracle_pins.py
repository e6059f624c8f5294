"""Pins of the CPU reference of the warm-start network (oracle/cnn.py) against
what does not depend on it: library convolutions and roundings, adjoint
identities, finite differences, closed forms of GELU, a library Adam, and the
solver oracle's own exact solution and forcing."""
import math

import numpy as np
import pytest

from oracle import cnn, core
from synthetic import warmstart as ws


def test_param_count_and_layout():
    assert cnn.param_count() == 40193
    p = np.arange(cnn.param_count(), dtype=np.float64)
    layers = cnn.unpack(p)
    assert [w.shape for w, _ in layers] == [(3, 3, ci, co) for ci, co in zip(cnn.CIN, cnn.COUT)]
    assert np.array_equal(cnn.pack(layers), p)
    assert ws.initial_params(0).size == cnn.param_count()
    assert ws.CIN == cnn.CIN and ws.COUT == cnn.COUT


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(3)
    v = np.concatenate([
        r.standard_normal(20000).astype(np.float32),
        (r.standard_normal(2000) * 1e-38).astype(np.float32),       # subnormal range
        (r.standard_normal(2000) * 1e30).astype(np.float32),
        # exact ties: 8 significant bits plus a half
        (np.arange(256, 512, dtype=np.float32) + np.float32(0.5)) * np.float32(2.0 ** -8),
        np.array([0.0, -0.0, 1.0, -1.0], dtype=np.float32),
    ])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = cnn.bf16(v.astype(np.float64))
    assert np.array_equal(got, ref)


def test_conv_matches_scipy_correlate2d():
    from scipy.signal import correlate2d
    r = np.random.default_rng(1)
    x = r.standard_normal((2, 7, 9, 3))
    w = r.standard_normal((3, 3, 3, 4))
    b = r.standard_normal(4)
    z = cnn.conv(x, w, b)
    for bi in range(2):
        for co in range(4):
            ref = sum(correlate2d(x[bi, :, :, ci], w[:, :, ci, co], mode="same") for ci in range(3)) + b[co]
            assert np.allclose(z[bi, :, :, co], ref, rtol=0, atol=1e-12)


def test_conv_matches_torch_conv2d_layout():
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(2)
    x = r.standard_normal((2, 6, 5, 4))
    w = r.standard_normal((3, 3, 4, 3))
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2),
                                     torch.from_numpy(w).permute(3, 2, 0, 1), padding=1)
    assert np.allclose(cnn.conv(x, w), ref.permute(0, 2, 3, 1).numpy(), rtol=0, atol=1e-12)


def test_conv_gradients_are_adjoints():
    r = np.random.default_rng(4)
    x = r.standard_normal((2, 5, 6, 3))
    w = r.standard_normal((3, 3, 3, 4))
    g = r.standard_normal((2, 5, 6, 4))
    lhs = np.sum(cnn.conv(x, w) * g)
    assert math.isclose(lhs, np.sum(x * cnn.conv_input_grad(g, w)), rel_tol=1e-12)
    assert math.isclose(lhs, np.sum(w * cnn.conv_weight_grad(x, g)), rel_tol=1e-12)


def test_gelu_closed_forms():
    assert cnn.gelu(np.array(0.0)) == 0.0
    # Phi(1) and Phi(2) of the standard normal distribution
    assert math.isclose(float(cnn.gelu(np.array(1.0))), 0.8413447460685429, rel_tol=1e-14)
    assert math.isclose(float(cnn.gelu(np.array(2.0))), 2 * 0.9772498680518208, rel_tol=1e-14)
    z = np.linspace(-6, 6, 101)
    assert np.allclose(cnn.gelu(z) - cnn.gelu(-z), z, rtol=0, atol=1e-14)   # Phi(z) + Phi(-z) = 1
    h = 1e-6
    fd = (cnn.gelu(z + h) - cnn.gelu(z - h)) / (2 * h)
    assert np.allclose(cnn.gelu_d(z), fd, rtol=0, atol=1e-8)


def _loss(params, x, t):
    return cnn.loss_and_grad(params, x, t, emulate=False)[0]


def test_backward_matches_finite_differences():
    """Directional derivatives of the FP64 loss (no rounding) along random
    directions confined to each layer's weights, each layer's biases, and all
    parameters at once."""
    r = np.random.default_rng(5)
    p = ws.initial_params(7).astype(np.float64)
    p += 0.05 * r.standard_normal(p.size)       # non-zero biases too
    x = r.standard_normal((2, 6, 5, cnn.NFIELD))
    t = r.standard_normal((2, 4, 3))
    L0, g, _ = cnn.loss_and_grad(p, x, t, emulate=False)
    assert L0 > 0
    off = 0
    dirs = []
    for ci, co in zip(cnn.CIN, cnn.COUT):
        nw = 9 * ci * co
        for lo, hi in ((off, off + nw), (off + nw, off + nw + co)):
            v = np.zeros_like(p)
            v[lo:hi] = r.standard_normal(hi - lo)
            dirs.append(v)
        off += nw + co
    dirs.append(r.standard_normal(p.size))
    for v in dirs:
        v = v / np.linalg.norm(v)
        h = 1e-4
        fd = (_loss(p + h * v, x, t) - _loss(p - h * v, x, t)) / (2 * h)
        an = float(g @ v)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-7, (fd, an)


def test_emulated_rounding_stays_close_to_fp64():
    r = np.random.default_rng(6)
    p = ws.initial_params(1)
    x = cnn.bf16(r.standard_normal((1, 8, 8, cnn.NFIELD)))
    t = r.standard_normal((1, 6, 6))
    L64, g64, u64 = cnn.loss_and_grad(p, x, t, emulate=False)
    Lq, gq, uq = cnn.loss_and_grad(p, x, t, emulate=True)
    assert np.linalg.norm(uq - u64) <= 0.05 * np.linalg.norm(u64)
    assert np.linalg.norm(gq - g64) <= 0.05 * np.linalg.norm(g64)
    # the emulated values are bfloat16 numbers
    _, c = cnn.forward(p, x, emulate=True)
    for h in c["h"]:
        assert np.array_equal(cnn.bf16(h), h)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(8)
    p0 = r.standard_normal(50)
    grads = [r.standard_normal(50) for _ in range(5)]
    ref = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([ref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    mine = cnn.Adam(p0, lr=1e-2)
    for g in grads:
        ref.grad = torch.from_numpy(g.copy())
        opt.step()
        mine.step(g)
    assert np.allclose(mine.p, ref.detach().numpy(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("bc", [core.DIRICHLET, core.NEUMANN])
def test_features_pinned_to_exact_solution_and_forcing(bc):
    eps, X, Y, nx, ny = 0.05, 1.3, 0.7, 9, 6
    f = cnn.features(eps, X, Y, nx, ny, bc)
    assert f.shape == (ny + 2, nx + 2, cnn.NFIELD)
    dx, dy = X / (nx + 1), Y / (ny + 1)
    fman = core.forcing(eps, X, Y, nx, ny).reshape(ny, nx)
    assert np.allclose(f[1:-1, 1:-1, 2], fman / 10.0, rtol=1e-15, atol=0)
    assert np.all(f[:, :, 3] == math.log10(eps) / 3.0)
    for J in range(ny + 2):
        for I in range(nx + 2):
            x, y = I * dx, J * dy
            assert math.isclose(f[J, I, 0], (1 + x * x) / 5, rel_tol=1e-15)
            assert math.isclose(f[J, I, 1], X * math.exp(-y) / 2, rel_tol=1e-15)
            assert math.isclose(f[J, I, 5], x / X, rel_tol=1e-15) and math.isclose(f[J, I, 6], y / Y, rel_tol=1e-15)
            assert f[J, I, 7] == X / 2 and f[J, I, 8] == Y / 2 and f[J, I, 9] == 0.0
            ring = not (1 <= I <= nx and 1 <= J <= ny)
            if not ring:
                assert f[J, I, 4] == 0.0
                continue
            neumann = bc == core.NEUMANN and (I == nx + 1 and J >= 1 or J == ny + 1 and I >= 1)
            if not neumann:
                assert f[J, I, 4] == 1.0
                assert math.isclose(f[J, I, 2], core.u_exact(x, y, X, Y), rel_tol=1e-14, abs_tol=1e-300)
                continue
            assert f[J, I, 4] == -1.0
            h = 1e-6
            if I == nx + 1 and J == ny + 1:
                assert f[J, I, 2] == 0.0
            elif I == nx + 1:      # normal derivative on x = X
                d = (core.u_exact(X + h, y, X, Y) - core.u_exact(X - h, y, X, Y)) / (2 * h)
                assert math.isclose(f[J, I, 2], d, rel_tol=1e-7, abs_tol=1e-9)
            else:                  # normal derivative on y = Y
                d = (core.u_exact(x, Y + h, X, Y) - core.u_exact(x, Y - h, X, Y)) / (2 * h)
                assert math.isclose(f[J, I, 2], d, rel_tol=1e-7, abs_tol=1e-9)


def test_scheme_field_marks_the_centered_scheme_only():
    eps, X, Y, nx, ny = 0.05, 1.3, 0.7, 9, 6
    f0 = cnn.features(eps, X, Y, nx, ny, core.DIRICHLET)
    f1 = cnn.features(eps, X, Y, nx, ny, core.DIRICHLET, scheme=core.CENTERED)
    assert core.CENTERED == 1 and core.UPWIND == 0
    assert np.all(f0[..., 9] == 0.0) and np.all(f1[..., 9] == 1.0)
    assert np.array_equal(f0[..., :9], f1[..., :9])


def test_features_with_field_use_the_assembled_forcing():
    eps, X, Y, nx, ny = 0.3, 1.0, 1.5, 7, 5
    g = np.linspace(-1, 1, nx * ny)
    f = cnn.features(eps, X, Y, nx, ny, core.DIRICHLET, field=g, amp=0.1)
    P0 = core.assemble(eps, X, Y, nx, ny)
    P1 = core.assemble(eps, X, Y, nx, ny, field=g, amp=0.1)
    # the right-hand sides differ by (f1 - f0) dx^2 dy^2
    dx, dy = X / (nx + 1), Y / (ny + 1)
    df = (P1.rhs - P0.rhs) / (dx * dx * dy * dy)
    f0 = cnn.features(eps, X, Y, nx, ny, core.DIRICHLET)
    assert np.allclose((f[1:-1, 1:-1, 2] - f0[1:-1, 1:-1, 2]).ravel() * 10.0, df, rtol=1e-9, atol=1e-9)
