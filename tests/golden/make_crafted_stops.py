"""Writes crafted_stops.json: tiny five-point systems (integer coefficients)
on which BiCGSTAB stops on one of the exact-zero tests of Section 5.2
(rho = r^.r = 0, or omega = 0).

Seeded search: random integer systems are run through the CPU oracle; a
system is kept when the oracle stops on rho = 0 or omega = 0 and the exact
rational-arithmetic reference (tests/rational_ref.py) stops the same way at
the same pass.  Only the inputs are stored; the tests recompute the expected
stop in exact arithmetic.

    python tests/golden/make_crafted_stops.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import core as orc  # noqa: E402
import rational_ref as rr  # noqa: E402


def main(seed=7, trials=300000):
    rng = np.random.default_rng(seed)
    keep = {}
    for trial in range(trials):
        nx, ny = [(2, 2), (3, 2), (2, 3), (3, 3)][trial % 4]
        n = nx * ny
        i = np.arange(n) % nx
        j = np.arange(n) // nx
        S = rng.integers(-2, 3, n).astype(float); S[j == 0] = 0
        W = rng.integers(-2, 3, n).astype(float); W[i == 0] = 0
        E = rng.integers(-2, 3, n).astype(float); E[i == nx - 1] = 0
        N = rng.integers(-2, 3, n).astype(float); N[j == ny - 1] = 0
        C = rng.choice([-4., -2., -1., 1., 2., 4.], n)
        b = rng.integers(-2, 3, n).astype(float)
        if not b.any():
            continue
        P = orc.Problem(1.0, 1.0, 1.0, nx, ny, 0, 0, S, W, C, E, N, b)
        F = orc.ilu0(P)
        if F.status != orc.OK:
            continue
        s = orc.bicgstab(P, F, tol=1e-10, maxit=20)
        if s.status not in (orc.BREAKDOWN_RHO, orc.OMEGA_ZERO) or (s.status, s.iters) in keep:
            continue
        A = rr.dense_from_dia(nx, ny, S, W, C, E, N)
        LU = rr.ilu0(A, rr.pattern_of(nx, ny))
        if LU is None:
            continue
        st, it, _ = rr.bicgstab(A, *LU, b, 1e-10, 20)
        if (st, it) == (s.status, s.iters):
            keep[(st, it)] = dict(nx=nx, ny=ny, S=S.tolist(), W=W.tolist(), C=C.tolist(), E=E.tolist(),
                                  N=N.tolist(), rhs=b.tolist())
    out = dict(source="seeded search (seed %d) over integer five-point systems; see make_crafted_stops.py" % seed,
               tol=1e-10, maxit=20, systems=[keep[k] for k in sorted(keep)])
    with open(os.path.join(HERE, "crafted_stops.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(sorted(keep))


if __name__ == "__main__":
    main()
