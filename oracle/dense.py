"""Small dense helpers that pin the oracle (grids of a few hundred unknowns).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``dense_matrix``: the five diagonals as a dense array, in the paper's
  lexicographic ordering.
* ``exact_discrete``: the exact solution of the discrete system by LU with
  partial pivoting (numpy/LAPACK), for the error tables of Section 6.
* ``truncated_lu``: the preconditioner under which the printed iteration
  counts of Section 6 come out -- the complete LU factors of A (no pivoting,
  fill kept during the elimination) with every entry outside A's pattern
  dropped afterwards, i.e. not the ILU(0) of Section 5.1, whose elimination
  drops the fill as it goes.
* ``split_lu``: the splitting preconditioner of the Section 6.4-6.5
  comparisons: L = unit lower part of A, U = upper part of A.
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


def lu_no_pivoting(A):
    """Complete LU factors of A without pivoting, A = L U with L unit lower,
    in the right-looking (outer-product) form of Golub & Van Loan, Matrix
    Computations, Algorithm 3.2.1: column k of L is column k of the current
    Schur complement over its pivot, which is then updated by a rank-one
    product."""
    S = np.array(A, dtype=np.float64)
    n = S.shape[0]
    L = np.eye(n)
    for k in range(n - 1):
        L[k + 1:, k] = S[k + 1:, k] / S[k, k]
        S[k + 1:, k + 1:] -= np.outer(L[k + 1:, k], S[k, k + 1:])
        S[k + 1:, k] = 0.0
    return L, np.triu(S)


def truncated_lu(P):
    """The complete factors (``lu_no_pivoting``) restricted to A's pattern."""
    A = dense_matrix(P)
    L, U = lu_no_pivoting(A)
    keep = A != 0
    np.fill_diagonal(keep, True)
    return _five_point_factors(P, np.where(keep, L, 0.0), np.where(keep, U, 0.0))


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
