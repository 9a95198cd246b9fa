"""Algebraic multigrid for the scalar-potential system (CPU FP64 oracle).

Test infrastructure only: the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product path never
does. Plain numpy, written for reading, not speed.

The paper solves the scalar-potential system K u = b with conjugate
gradients preconditioned by algebraic multigrid (Sec. 3.1; Sec. 3.5 names
the magnetostatic solve as the main cost of an evaluation). It does not fix
the variant. The reading taken here is the textbook smoothed
aggregation method:

  strength    j is a strong neighbour of i (j != i) when
              |a_ij| >= theta_l sqrt(a_ii a_jj), theta_l = 0.08 / 2^l;
  aggregates  pass 1, rows in order: a row that is not yet in an aggregate
              and whose strong neighbours are all free starts an aggregate
              with them; pass 2: every row still free joins the pass-1
              aggregate of its strongest strong neighbour, looked up in the
              pass-1 assignment (weights within a relative TIE of each other
              count as equal and the lowest column wins, so that round-off
              in how a matrix was summed does not decide);
  prolongator P0 = aggregate indicator (one 1 per row), smoothed once:
              P = (I - omega D^-1 A) P0, omega = (4/3) / rho,
              rho = max_i sum_j |a_ij| / a_ii (a Gershgorin bound on the
              spectral radius of D^-1 A);
  coarse      A_c = P^T A P (Galerkin);
  levels      until a level has at most COARSE_MAX rows (solved with its
              dense inverse; a parameter of the hierarchy, 2048 by default),
              or coarsening stalls (n_c > 0.9 n), or MAX_LEVELS;
  cycle       V(1,1) with damped Jacobi, the same omega: from zero,
              y = omega D^-1 b, t = b - A y, y += P V_{l+1}(P^T t),
              y += omega D^-1 (b - A y).

With a symmetric pre/post smoother pair and restriction P^T the cycle is a
symmetric positive definite operator M whose product with A has its spectrum
in (0, 1]: the preconditioner of a plain PCG.
"""
from __future__ import annotations

import numpy as np

THETA0 = 0.08
COARSE_MAX = 2048
MAX_LEVELS = 12
STALL = 0.9
TIE = 1e-12


class Csr:
    """Compressed sparse rows: row pointers p (n+1), columns j, values v."""

    def __init__(self, p, j, v, ncols):
        self.p = np.asarray(p, dtype=np.int64)
        self.j = np.asarray(j, dtype=np.int64)
        self.v = np.asarray(v, dtype=np.float64)
        self.n = self.p.size - 1
        self.ncols = int(ncols)

    def rows(self):
        """Row index of every stored entry."""
        return np.repeat(np.arange(self.n), np.diff(self.p))

    def diag(self):
        d = np.zeros(self.n)
        r = self.rows()
        on = self.j == r
        np.add.at(d, r[on], self.v[on])
        return d

    def matvec(self, x):
        y = np.zeros(self.n)
        np.add.at(y, self.rows(), self.v * x[self.j])
        return y

    def transpose(self):
        return from_coo(self.j, self.rows(), self.v, self.ncols, self.n)

    def dense(self):
        d = np.zeros((self.n, self.ncols))
        np.add.at(d, (self.rows(), self.j), self.v)
        return d


def from_coo(i, j, v, n, ncols):
    """CSR with duplicates summed, columns ascending within each row and
    entries that sum to exactly zero dropped."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    v = np.asarray(v, dtype=np.float64)
    key = i * ncols + j
    order = np.argsort(key, kind="stable")
    key, v = key[order], v[order]
    if key.size:
        first = np.concatenate([[True], key[1:] != key[:-1]])
        starts = np.nonzero(first)[0]
        vs = np.add.reduceat(v, starts)
        ks = key[starts]
    else:
        vs, ks = v, key
    keep = vs != 0.0
    vs, ks = vs[keep], ks[keep]
    ri, cj = ks // ncols, ks % ncols
    p = np.zeros(n + 1, dtype=np.int64)
    np.add.at(p, ri + 1, 1)
    return Csr(np.cumsum(p), cj, vs, ncols)


def spmm(A, B):
    """Sparse product A B: every stored a_ik times every stored b_kj."""
    ra = A.rows()
    cnt = np.diff(B.p)[A.j]
    ai = np.repeat(ra, cnt)
    av = np.repeat(A.v, cnt)
    # positions in B of the entries of row A.j[e]
    starts = np.repeat(B.p[A.j], cnt)
    offs = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    pos = starts + offs
    return from_coo(ai, B.j[pos], av * B.v[pos], A.n, B.ncols)


def strong_neighbours(A, theta):
    """Per row, the strong off-diagonal neighbours (a list of arrays)."""
    d = A.diag()
    out = []
    for i in range(A.n):
        js = A.j[A.p[i]:A.p[i + 1]]
        vs = A.v[A.p[i]:A.p[i + 1]]
        keep = (js != i) & (np.abs(vs) >= theta * np.sqrt(np.abs(d[i] * d[js])))
        out.append((js[keep], np.abs(vs[keep])))
    return out


def aggregate(A, theta):
    """Aggregate of every row (two greedy passes, see the module text)."""
    S = strong_neighbours(A, theta)
    agg = np.full(A.n, -1, dtype=np.int64)
    na = 0
    for i in range(A.n):
        if agg[i] >= 0:
            continue
        js = S[i][0]
        if np.all(agg[js] < 0):
            agg[i] = na
            agg[js] = na
            na += 1
    first = agg.copy()
    for i in range(A.n):
        if first[i] >= 0:
            continue
        js, ws = S[i]
        best, bw = -1, -1.0
        for j, w in zip(js, ws):
            if first[j] >= 0 and w > bw * (1.0 + TIE):
                best, bw = j, w
        if best < 0:
            raise RuntimeError("row without an aggregated strong neighbour")
        agg[i] = first[best]
    return agg, na


def gershgorin_rho(A):
    """max_i sum_j |a_ij| / a_ii, an upper bound on rho(D^-1 A)."""
    s = np.zeros(A.n)
    np.add.at(s, A.rows(), np.abs(A.v))
    return float(np.max(s / A.diag()))


def smoothed_prolongator(A, agg, na, omega):
    P0 = Csr(np.arange(A.n + 1), agg, np.ones(A.n), na)
    d = A.diag()
    # (I - omega D^-1 A) P0 = P0 - omega D^-1 (A P0)
    AP = spmm(A, P0)
    r = AP.rows()
    return from_coo(np.concatenate([np.arange(A.n), r]), np.concatenate([agg, AP.j]),
                    np.concatenate([np.ones(A.n), -omega * AP.v / d[r]]), A.n, na)


class Level:
    def __init__(self, A, theta):
        self.A = A
        self.d = A.diag()
        self.rho = gershgorin_rho(A)
        self.omega = (4.0 / 3.0) / self.rho
        self.theta = theta
        self.agg = None
        self.P = None
        self.R = None
        self.Ainv = None


def hierarchy(A, coarse_max=COARSE_MAX):
    """The levels, fine to coarse; the last holds a dense inverse. Stored
    zeros of A are dropped first (they are neither strong nor part of any
    product)."""
    A = from_coo(A.rows(), A.j, A.v, A.n, A.ncols)
    levels = []
    theta = THETA0
    while True:
        L = Level(A, theta)
        levels.append(L)
        if A.n <= coarse_max or len(levels) == MAX_LEVELS:
            break
        agg, na = aggregate(A, theta)
        if na > STALL * A.n or na == 0:
            break
        L.agg = agg
        L.P = smoothed_prolongator(A, agg, na, L.omega)
        L.R = L.P.transpose()
        A = spmm(L.R, spmm(A, L.P))
        theta *= 0.5
    last = levels[-1]
    last.Ainv = np.linalg.inv(last.A.dense())
    return levels


def vcycle(levels, b, l=0):
    """One V(1,1) cycle from zero at level l for right-hand side b."""
    L = levels[l]
    if L.Ainv is not None:
        return L.Ainv @ b
    y = L.omega * b / L.d
    t = b - L.A.matvec(y)
    y = y + L.P.matvec(vcycle(levels, L.R.matvec(t), l + 1))
    return y + L.omega * (b - L.A.matvec(y)) / L.d


def pcg(A, b, x0, precond, rtol, maxit=10000):
    """Preconditioned CG (Hestenes-Stiefel form). Stops when r.r <= rtol^2
    b.b, tested before every update; returns (x, updates)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    bb = float(b @ b)
    if bb == 0.0:
        return np.zeros_like(x), 0
    r = b - A.matvec(x)
    z = precond(r)
    p = z.copy()
    gam = float(r @ z)
    it = 0
    while float(r @ r) > rtol * rtol * bb:
        if it >= maxit:
            raise RuntimeError("PCG did not converge")
        q = A.matvec(p)
        alpha = gam / float(p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        z = precond(r)
        gnew = float(r @ z)
        p = z + (gnew / gam) * p
        gam = gnew
    return x, it


def solve(A, b, x0=None, rtol=1e-10, levels=None, coarse_max=COARSE_MAX):
    """AMG-preconditioned CG for A x = b."""
    levels = hierarchy(A, coarse_max) if levels is None else levels
    x0 = np.zeros(A.n) if x0 is None else x0
    return pcg(A, b, x0, lambda r: vcycle(levels, r), rtol)
