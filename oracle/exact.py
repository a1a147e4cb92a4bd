"""Exact rational Schur formation and PCG with fractions.Fraction (test infrastructure).

Used on tiny problems only (nx, nu, N of a few units).  In exact arithmetic PCG on the
symmetric positive definite system (Algorithm 1 of MPCGPU) reaches r = 0 after at most
as many iterations as Phi^-1 S has distinct eigenvalues, and never more than dim S.  For
the symmetric stair preconditioner Phi^-1 S = I - (D^-1 E)^2 where D^-1 E is similar to
a 2-cyclic block-tridiagonal matrix, so the eigenvalues come in equal pairs and the bound
tightens to floor(N/2)*nx + 1 distinct values.

The steps follow Section III-B (theta/phi/zeta blocks), Section IV-A (preconditioner
blocks -D_b^-1 S_{b,b+-1} D_{b+-1}^-1) and Algorithm 1, on Fractions.
"""
from __future__ import annotations

from fractions import Fraction as F


def mat(rows):
    return [[F(x) for x in row] for row in rows]


def zeros(n, m):
    return [[F(0)] * m for _ in range(n)]


def eye(n):
    return [[F(int(i == j)) for j in range(n)] for i in range(n)]


def mm(a, b):
    n, k, m = len(a), len(b), len(b[0])
    return [[sum((a[i][t] * b[t][j] for t in range(k)), F(0)) for j in range(m)] for i in range(n)]


def tr(a):
    return [list(r) for r in zip(*a)]


def add(a, b, s=1):
    return [[x + s * y for x, y in zip(ra, rb)] for ra, rb in zip(a, b)]


def neg(a):
    return [[-x for x in r] for r in a]


def mv(a, x):
    return [sum((a[i][j] * x[j] for j in range(len(x))), F(0)) for i in range(len(a))]


def inv(a):
    """Gauss-Jordan inverse with row pivoting on exact rationals."""
    n = len(a)
    M = [list(a[i]) + [F(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def form(Q, R, A, B, q, r, x0, e=None):
    """Exact S, Phi^-1 (lists of [sub, diag, super] blocks per row) and gamma."""
    N = len(Q)
    nx = len(Q[0])
    Qi = [inv(Qk) for Qk in Q]
    Ri = [inv(Rk) for Rk in R]
    Z = zeros(nx, nx)
    S = [[Z, Z, Z] for _ in range(N)]
    gam = [None] * N
    S[0][1] = Qi[0]
    gam[0] = [a + b for a, b in zip(mv(Qi[0], q[0]), x0)]
    for k in range(N - 1):
        AQ = mm(A[k], Qi[k])
        theta = add(add(mm(AQ, tr(A[k])), mm(mm(B[k], Ri[k]), tr(B[k]))), Qi[k + 1])
        phi = neg(AQ)
        S[k + 1][1] = theta
        S[k + 1][0] = phi
        S[k][2] = tr(phi)
        zeta = [-a - b + c for a, b, c in zip(mv(AQ, q[k]), mv(mm(B[k], Ri[k]), r[k]),
                                               mv(Qi[k + 1], q[k + 1]))]
        ek = e[k] if e is not None else [F(0)] * nx
        gam[k + 1] = [z - d for z, d in zip(zeta, ek)]
    Di = [inv(S[b][1]) for b in range(N)]
    P = [[Z, Di[b], Z] for b in range(N)]
    for b in range(N):
        if b > 0:
            P[b][0] = neg(mm(mm(Di[b], S[b][0]), Di[b - 1]))
        if b < N - 1:
            P[b][2] = neg(mm(mm(Di[b], S[b][2]), Di[b + 1]))
    return S, P, gam


def bt_mv(M, x):
    N = len(M)
    out = []
    for b in range(N):
        acc = mv(M[b][1], x[b])
        if b > 0:
            acc = [u + v for u, v in zip(acc, mv(M[b][0], x[b - 1]))]
        if b < N - 1:
            acc = [u + v for u, v in zip(acc, mv(M[b][2], x[b + 1]))]
        out.append(acc)
    return out


def dotv(a, b):
    return sum((u * v for ra, rb in zip(a, b) for u, v in zip(ra, rb)), F(0))


def pcg(S, P, gam, max_iter=None):
    """Algorithm 1 from lambda = 0 in exact arithmetic, run until r = 0.
    Returns (lambda, iterations, [eta_0, eta_1, ...])."""
    N = len(S)
    nx = len(S[0][1])
    max_iter = max_iter or N * nx + 5
    lam = [[F(0)] * nx for _ in range(N)]
    r = [list(g) for g in gam]
    rt = bt_mv(P, r)
    p = [list(v) for v in rt]
    eta = dotv(r, rt)
    etas = [eta]
    if eta == 0:
        return lam, 0, etas
    for it in range(1, max_iter + 1):
        Sp = bt_mv(S, p)
        alpha = eta / dotv(p, Sp)
        r = [[a - alpha * b for a, b in zip(ra, rb)] for ra, rb in zip(r, Sp)]
        lam = [[a + alpha * b for a, b in zip(la, pa)] for la, pa in zip(lam, p)]
        rt = bt_mv(P, r)
        eta_new = dotv(r, rt)
        etas.append(eta_new)
        if eta_new == 0:
            return lam, it, etas
        beta = eta_new / eta
        p = [[a + beta * b for a, b in zip(ra, pa)] for ra, pa in zip(rt, p)]
        eta = eta_new
    return lam, max_iter, etas
