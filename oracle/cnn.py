"""CPU FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Plain numpy, written from the network's definition rather than from the GPU
kernels: six 3x3 cross-correlations with zero padding, channels
10 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, exact GELU x*Phi(x) after the first
five, mean squared error over the interior nodes, Adam.  Every sum is in
FP64.  With ``emulate=True`` the values the network stores in bfloat16
(input fields, weights, hidden activations, and the gradients entering each
convolution in the backward pass) are rounded to bfloat16 at the same points,
so that the GPU result differs from this one only by its FP32 accumulation.

Tensors are [B, H, W, C] (channels last); weights W[ky, kx, ci, co] (output
node (y, x) reads input (y + ky - 1, x + kx - 1)); parameters are packed per
layer as the weights in that index order followed by the biases.

The input fields of an instance are also defined here (``features``), from
the oracle's own forcing and exact solution.
"""
import math

import numpy as np
from scipy.special import erf

from . import core

NFIELD = 10
CIN = (NFIELD, 32, 32, 32, 32, 32)
COUT = (32, 32, 32, 32, 32, 1)
NLAYER = 6


def param_count():
    return sum(9 * ci * co + co for ci, co in zip(CIN, COUT))


def unpack(params):
    """Packed vector -> list of (W [3, 3, ci, co], b [co]) in float64."""
    p = np.asarray(params, dtype=np.float64).ravel()
    assert p.size == param_count()
    out, off = [], 0
    for ci, co in zip(CIN, COUT):
        nw = 9 * ci * co
        out.append((p[off:off + nw].reshape(3, 3, ci, co), p[off + nw:off + nw + co]))
        off += nw + co
    return out


def pack(layers):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


def bf16(a):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even,
    FP32's exponent range including its subnormals); returned as float64."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                      # a = m 2^e, 0.5 <= |m| < 1
    q = np.ldexp(1.0, np.maximum(e - 8, -133))
    with np.errstate(invalid="ignore"):
        r = np.rint(a / q) * q              # np.rint rounds ties to even
    return np.where(np.isfinite(a), r, a)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def conv(x, w, b=None):
    """Zero-padded 3x3 cross-correlation: [B, H, W, ci] -> [B, H, W, co]."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    z = np.zeros((B, H, W, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            z += np.tensordot(xp[:, ky:ky + H, kx:kx + W, :], w[ky, kx], axes=([3], [0]))
    if b is not None:
        z += b
    return z


def conv_input_grad(g, w):
    """Gradient of sum(conv(x, w) * g) with respect to x."""
    B, H, W, _ = g.shape
    gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
    d = np.zeros((B, H, W, w.shape[2]))
    for ky in range(3):
        for kx in range(3):
            d += np.tensordot(gp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W, :], w[ky, kx], axes=([3], [1]))
    return d


def conv_weight_grad(x, g):
    """Gradient of sum(conv(x, w) * g) with respect to w [3, 3, ci, co]."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((3, 3, x.shape[3], g.shape[3]))
    for ky in range(3):
        for kx in range(3):
            dw[ky, kx] = np.tensordot(xp[:, ky:ky + H, kx:kx + W, :], g, axes=([0, 1, 2], [0, 1, 2]))
    return dw


def forward(params, x, emulate=True):
    """Network output u [B, H, W] and the cache of the backward pass."""
    layers = unpack(params)
    rnd = bf16 if emulate else (lambda a: a)
    h = rnd(np.asarray(x, dtype=np.float64))
    hs, zs, ws = [h], [], []
    for l, (w, b) in enumerate(layers):
        wq = rnd(w)
        ws.append(wq)
        z = conv(h, wq, b)
        zs.append(z)
        if l < NLAYER - 1:
            h = rnd(gelu(z))
            hs.append(h)
    return zs[-1][..., 0], dict(h=hs, z=zs, w=ws, emulate=emulate)


def interior_mask(H, W):
    m = np.zeros((H, W))
    m[1:H - 1, 1:W - 1] = 1.0
    return m


def loss_and_grad(params, x, target, emulate=True):
    """L = sum over batch and interior nodes of (u - t)^2 / (B (H-2) (W-2));
    target is [B, H-2, W-2].  Returns (L, packed dL/dparams, u)."""
    u, c = forward(params, x, emulate)
    B, H, W = u.shape
    count = B * (H - 2) * (W - 2)
    t = np.zeros_like(u)
    t[:, 1:H - 1, 1:W - 1] = target
    d = (u - t) * interior_mask(H, W)
    loss = float(np.sum(d * d) / count)
    rnd = bf16 if c["emulate"] else (lambda a: a)
    g = rnd((2.0 * d / count)[..., None])
    grads = [None] * NLAYER
    for l in range(NLAYER - 1, -1, -1):
        grads[l] = (conv_weight_grad(c["h"][l], g), g.sum(axis=(0, 1, 2)))
        if l > 0:
            g = rnd(conv_input_grad(g, c["w"][l]) * gelu_d(c["z"][l - 1]))
    return loss, pack(grads), u


class Adam:
    """Adam (Kingma & Ba, ICLR 2015) with bias correction, in FP64."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.p = np.asarray(params, dtype=np.float64).copy()
        self.m = np.zeros_like(self.p)
        self.v = np.zeros_like(self.p)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        self.p = self.p - self.lr * mh / (np.sqrt(vh) + self.eps)
        return self.p


def features(eps, X, Y, nx, ny, bc, field=None, amp=0.0, scheme=0):
    """The input fields on the (ny+2) x (nx+2) node grid, [ny+2, nx+2, 10]:
    a/5, b/2, (interior) f/10 or (ring) the boundary datum, log10(eps)/3, the
    ring mask (+1 Dirichlet, -1 Neumann, 0 interior), x/X, y/Y, X/2, Y/2 and
    the scheme (0 upwind, 1 centered).
    f is the forcing the solver is assembled with:
    f_man + amp max|f_man| field."""
    H, W = ny + 2, nx + 2
    dx, dy = X / (nx + 1), Y / (ny + 1)
    out = np.zeros((H, W, NFIELD))
    f = core.forcing(eps, X, Y, nx, ny)
    if field is not None:
        f = f + amp * np.max(np.abs(f)) * np.asarray(field, dtype=np.float64).ravel()
    f = f.reshape(ny, nx)
    for J in range(H):
        y = J * dy
        for I in range(W):
            x = I * dx
            out[J, I, 0] = (1.0 + x * x) / 5.0
            out[J, I, 1] = X * math.exp(-y) / 2.0
            out[J, I, 3] = math.log10(eps) / 3.0
            out[J, I, 5] = x / X
            out[J, I, 6] = y / Y
            out[J, I, 7] = X / 2.0
            out[J, I, 8] = Y / 2.0
            out[J, I, 9] = float(scheme)
            if 1 <= I <= nx and 1 <= J <= ny:
                out[J, I, 2] = f[J - 1, I - 1] / 10.0
                continue
            neu_x = bc == core.NEUMANN and I == nx + 1 and J >= 1
            neu_y = bc == core.NEUMANN and J == ny + 1 and I >= 1
            if neu_x and neu_y:
                val, mask = 0.0, -1.0
            elif neu_x:   # du/dx on x = X
                val, mask = -(1.0 / X) * math.exp(-1.0) * (1.0 - math.exp(-y / Y)) * y, -1.0
            elif neu_y:   # du/dy on y = Y
                val, mask = math.exp(-x / X), -1.0
            else:
                val, mask = core.u_exact(x, y, X, Y), 1.0
            out[J, I, 2] = val
            out[J, I, 4] = mask
    return out
