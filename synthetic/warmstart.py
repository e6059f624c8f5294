"""Seeded draws of the learned-warm-start workload: instance parameters per
seed and the network's initial parameters.  Random numbers only."""
import numpy as np

from .fields import _rng

# layer channels of the warm-start network (input fields -> u)
CIN = (10, 32, 32, 32, 32, 32)
COUT = (32, 32, 32, 32, 32, 1)


def warmstart_instance(seed, n=256, scheme=None):
    """One instance for seed `seed`: n x n interior grid, eps log-uniform in
    [1e-3, 1], X and Y uniform in [0.5, 2], boundary type (0 Dirichlet,
    1 Neumann on x = X and y = Y) with p = 1/2, the scheme (0 upwind,
    1 centered; drawn with p = 1/2 from a stream of its own unless given),
    and the seed of its random forcing field."""
    r = _rng(0x57A27, seed)
    d = dict(
        n=int(n),
        eps=float(10.0 ** r.uniform(-3.0, 0.0)),
        X=float(r.uniform(0.5, 2.0)),
        Y=float(r.uniform(0.5, 2.0)),
        bc=int(r.integers(0, 2)),
        field_seed=int(r.integers(0, 2 ** 31 - 1)),
    )
    d["scheme"] = int(_rng(0x5C4E3E, seed).integers(0, 2)) if scheme is None else int(scheme)
    return d


def initial_params(seed=0):
    """He-normal initial weights (std sqrt(2 / (9 ci))) and zero biases in the
    packed layout W[ky][kx][ci][co] then b[co], per layer; float32."""
    r = _rng(0xC0DE, seed)
    parts = []
    for ci, co in zip(CIN, COUT):
        parts.append(r.standard_normal(9 * ci * co) * np.sqrt(2.0 / (9 * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def random_fields(count, H, W, channels=5, seed=0):
    """Input-like fields for gradient checks: [count, H, W, channels] float64,
    standard normal, rounded by the caller as needed."""
    return _rng(0xF1E1D, seed).standard_normal((count, H, W, channels))
