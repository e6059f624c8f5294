"""Exact rational arithmetic references for tiny systems (test helper).

* ``ilu0``: incomplete LU of Section 5.1 with the drop pattern of A, written
  from its definition as Gaussian elimination on a dense matrix in which every
  update that would create an entry outside A's pattern is dropped (row by
  row, the IKJ order of Saad, Iterative Methods for Sparse Linear Systems,
  2nd ed., Algorithm 10.4).  Works on any matrix, not only five-point ones.
* ``bicgstab``: the right-preconditioned BiCGSTAB of Section 5.2 with the
  same stopping tests as the oracle (relative ||r||_2 < tol ||b||_2, compared
  as squared norms, so nothing is rounded), the exact-zero stops rho = 0 and
  omega = 0, a division by zero reported as a non-finite scalar, and no
  restarts.

Every value is a ``fractions.Fraction``: the results are those of exact
arithmetic, independent of any floating-point evaluation order.
"""
from fractions import Fraction


def dense_from_dia(nx, ny, S, W, C, E, N):
    n = nx * ny
    A = [[Fraction(0)] * n for _ in range(n)]
    for k in range(n):
        i, j = k % nx, k // nx
        A[k][k] = Fraction(C[k])
        if i > 0:
            A[k][k - 1] = Fraction(W[k])
        if i < nx - 1:
            A[k][k + 1] = Fraction(E[k])
        if j > 0:
            A[k][k - nx] = Fraction(S[k])
        if j < ny - 1:
            A[k][k + nx] = Fraction(N[k])
    return A


def pattern_of(nx, ny):
    n = nx * ny
    P = set()
    for k in range(n):
        i, j = k % nx, k // nx
        P.add((k, k))
        if i > 0:
            P.add((k, k - 1))
        if i < nx - 1:
            P.add((k, k + 1))
        if j > 0:
            P.add((k, k - nx))
        if j < ny - 1:
            P.add((k, k + nx))
    return P


def ilu0(A, pattern):
    """L (unit lower) and U with L*U = A on the pattern; None on a zero pivot."""
    n = len(A)
    a = [row[:] for row in A]
    for i in range(1, n):
        for k in range(i):
            if (i, k) not in pattern:
                continue
            if a[k][k] == 0:
                return None
            a[i][k] = a[i][k] / a[k][k]
            for j in range(k + 1, n):
                if (i, j) in pattern:
                    a[i][j] -= a[i][k] * a[k][j]
    if any(a[k][k] == 0 for k in range(n)):
        return None
    L = [[(a[i][j] if j < i else Fraction(int(i == j))) for j in range(n)] for i in range(n)]
    U = [[(a[i][j] if j >= i else Fraction(0)) for j in range(n)] for i in range(n)]
    return L, U


def matvec(A, x):
    return [sum((a * b for a, b in zip(row, x)), Fraction(0)) for row in A]


def dot(x, y):
    return sum((a * b for a, b in zip(x, y)), Fraction(0))


def lsolve(L, q):
    y = []
    for i in range(len(q)):
        y.append(q[i] - sum((L[i][j] * y[j] for j in range(i)), Fraction(0)))
    return y


def usolve(U, y):
    n = len(y)
    z = [Fraction(0)] * n
    for i in reversed(range(n)):
        z[i] = (y[i] - sum((U[i][j] * z[j] for j in range(i + 1, n)), Fraction(0))) / U[i][i]
    return z


OK, MAXIT, BREAKDOWN_RHO, OMEGA_ZERO, NONFINITE = 0, 1, 2, 3, 5


def bicgstab(A, L, U, b, tol, maxit, x0=None):
    """Returns (status, passes started, history of squared residual norms)."""
    n = len(b)
    b = [Fraction(v) for v in b]
    x = [Fraction(0)] * n if x0 is None else [Fraction(v) for v in x0]
    t2 = Fraction(tol) ** 2
    bb = dot(b, b)
    thr2 = t2 * bb
    Ax = matvec(A, x)
    r = [bi - ai for bi, ai in zip(b, Ax)]
    rh = r[:]
    hist = [dot(r, r)]
    if hist[0] < thr2:
        return OK, 0, hist
    rho = dot(rh, r)
    rho_prev = alpha = omega = None
    p = v = None
    for i in range(1, maxit + 1):
        if rho == 0:
            return BREAKDOWN_RHO, i, hist
        if i == 1:
            p = r[:]
        else:
            beta = (rho / rho_prev) * (alpha / omega)
            p = [ri + beta * (pi - omega * vi) for ri, pi, vi in zip(r, p, v)]
        ph = usolve(U, lsolve(L, p))
        v = matvec(A, ph)
        rv = dot(rh, v)
        if rv == 0:              # alpha would be infinite
            return NONFINITE, i, hist
        alpha = rho / rv
        s = [ri - alpha * vi for ri, vi in zip(r, v)]
        ss = dot(s, s)
        if ss < thr2:
            hist.append(ss)
            return OK, i, hist
        z = usolve(U, lsolve(L, s))
        t = matvec(A, z)
        tt = dot(t, t)
        if tt == 0:              # omega would be 0/0
            return NONFINITE, i, hist
        omega = dot(t, s) / tt
        x = [xi + alpha * pi + omega * zi for xi, pi, zi in zip(x, ph, z)]
        r = [si - omega * ti for si, ti in zip(s, t)]
        hist.append(dot(r, r))
        rho_prev, rho = rho, dot(rh, r)
        if hist[-1] < thr2:
            return OK, i, hist
        if omega == 0:
            return OMEGA_ZERO, i, hist
    return MAXIT, maxit, hist
