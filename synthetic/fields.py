"""Gaussian random fields and batched workload draws.

Random numbers come from numpy's Philox4x32-10 counter-based generator
(Salmon et al., SC'11), keyed by (seed, instance), so every draw is
reproducible and independent of the order in which instances are made.
"""
import numpy as np


def _rng(seed, instance):
    return np.random.Generator(np.random.Philox(key=[int(seed) & 0xFFFFFFFFFFFFFFFF,
                                                     int(instance) & 0xFFFFFFFFFFFFFFFF]))


def gaussian_random_field(nx, ny, dx, dy, length=0.1, seed=0, instance=0):
    """Zero-mean stationary Gaussian field with squared-exponential covariance
    exp(-r^2 / (2 length^2)) (length in physical units) on the nx x ny grid of
    spacing (dx, dy), sampled by spectral filtering of white noise on a
    zero-padded periodic grid (padding >= 4 length per side, so the
    wrap-around correlation is below exp(-8)).  Returned as an (ny, nx)
    float64 array scaled to max |g| = 1."""
    padx = int(np.ceil(4.0 * length / dx))
    pady = int(np.ceil(4.0 * length / dy))
    mx = int(2 ** np.ceil(np.log2(nx + padx))) if nx + padx > 1 else 1
    my = int(2 ** np.ceil(np.log2(ny + pady))) if ny + pady > 1 else 1
    w = _rng(seed, instance).standard_normal((my, mx))
    fx = np.fft.fftfreq(mx, d=dx)
    fy = np.fft.fftfreq(my, d=dy)
    spec = np.exp(-2.0 * np.pi ** 2 * length ** 2 * (fx[None, :] ** 2 + fy[:, None] ** 2))
    g = np.fft.ifft2(np.fft.fft2(w) * np.sqrt(spec)).real[:ny, :nx]
    m = np.abs(g).max()
    return np.ascontiguousarray(g / m if m > 0 else g)


def batch_instances(count=256, seed=1308, n_min=128, n_max=1024, n_step=32):
    """Instance parameters of the batched workload: grid n x n with n uniform
    in {n_min, n_min + n_step, ..., n_max}, eps log-uniform in [1e-3, 1],
    X and Y uniform in [0.5, 2], scheme and boundary type each with p = 1/2,
    and a per-instance random-field seed."""
    out = []
    sizes = np.arange(n_min, n_max + 1, n_step)
    for k in range(count):
        r = _rng(seed, k)
        out.append(dict(
            n=int(sizes[r.integers(0, len(sizes))]),
            eps=float(10.0 ** r.uniform(-3.0, 0.0)),
            X=float(r.uniform(0.5, 2.0)),
            Y=float(r.uniform(0.5, 2.0)),
            scheme=int(r.integers(0, 2)),
            bc=int(r.integers(0, 2)),
            field_seed=int(r.integers(0, 2 ** 31 - 1)),
        ))
    return out


def random_vector(n, seed=0, instance=0):
    return _rng(seed, instance).standard_normal(n)
