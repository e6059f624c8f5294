"""Small dense helpers that pin the oracle (grids of a few hundred unknowns).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``dense_matrix``: the five diagonals as a dense array (the appendix builds A
  dense, ``zeros(dime,dime)``, with the same lexicographic ordering).
* ``exact_discrete``: the exact solution of the discrete system by LU with
  partial pivoting (numpy/LAPACK), for the error tables of Section 6.
* ``truncated_lu``: the appendix's "ILUdecomposition2" routine -- full Gaussian
  elimination with fill, then every entry outside A's pattern set to zero --
  which the printed iteration counts of Section 6 were produced with.
* ``split_lu``: the instructor's splitting ("ILUdecomposition"): L = unit
  lower part of A, U = upper part of A (Section 6.4-6.5 comparisons).
* ``identity``: M = I, the unpreconditioned BiCGSTAB of Section 6.5 / 6.8.
"""
import numpy as np

from . import core


def dense_matrix(P):
    n, nx = P.n, P.nx
    A = np.zeros((n, n))
    k = np.arange(n)
    A[k, k] = P.C
    A[k[1:], k[1:] - 1] = P.W[1:]
    A[k[:-1], k[:-1] + 1] = P.E[:-1]
    A[k[nx:], k[nx:] - nx] = P.S[nx:]
    A[k[:-nx], k[:-nx] + nx] = P.N[:-nx]
    return A


def exact_discrete(P, rhs=None):
    return np.linalg.solve(dense_matrix(P), P.rhs if rhs is None else rhs)


def _five_point_factors(P, Lo, Up):
    n, nx = P.n, P.nx
    k = np.arange(n)
    lw = np.zeros(n); ls = np.zeros(n); ue = np.zeros(n); un = np.zeros(n)
    lw[1:] = Lo[k[1:], k[1:] - 1]
    ls[nx:] = Lo[k[nx:], k[nx:] - nx]
    ue[:-1] = Up[k[:-1], k[:-1] + 1]
    un[:-nx] = Up[k[:-nx], k[:-nx] + nx]
    invd = 1.0 / np.diag(Up)
    return core.Factors(lw, ls, invd, ue, un)


def truncated_lu(P):
    """Full LU without pivoting (with fill), then truncation to A's pattern."""
    A0 = dense_matrix(P)
    A = A0.copy()
    n = A.shape[0]
    for kk in range(n - 1):
        rows = np.nonzero(A[kk + 1:, kk])[0] + kk + 1
        for i in rows:
            lam = A[i, kk] / A[kk, kk]
            A[i, kk + 1:] -= lam * A[kk, kk + 1:]
            A[i, kk] = lam
    A[A0 == 0] = 0.0
    Lo = np.tril(A, -1) + np.eye(n)
    Up = np.triu(A)
    return _five_point_factors(P, Lo, Up)


def split_lu(P):
    A = dense_matrix(P)
    n = A.shape[0]
    return _five_point_factors(P, np.tril(A, -1) + np.eye(n), np.triu(A))


def identity(P):
    n = P.n
    z = np.zeros(n)
    return core.Factors(z.copy(), z.copy(), np.ones(n), z.copy(), z.copy())


def lu_product_minus_a(P, F):
    """Dense L*U - A for five-point factors F (ILU(0) invariant checks)."""
    n, nx = P.n, P.nx
    k = np.arange(n)
    L = np.eye(n)
    L[k[1:], k[1:] - 1] = F.lw[1:]
    L[k[nx:], k[nx:] - nx] = F.ls[nx:]
    U = np.zeros((n, n))
    U[k, k] = 1.0 / F.invd
    U[k[:-1], k[:-1] + 1] = F.ue[:-1]
    U[k[:-nx], k[:-nx] + nx] = F.un[:-nx]
    return L @ U - dense_matrix(P)
