"""Pins of the algebraic-multigrid oracle (CPU only).

The oracle's smoothed aggregation, prolongator, Galerkin product, V-cycle
and PCG are checked against what can be fixed independently of its code:
aggregates and prolongator entries worked out by hand for a chain and a 3x3
grid, a dense Galerkin product, the symmetry and spectrum bounds the V-cycle
must have as a symmetric positive definite preconditioner, the exact inverse
when a single level remains, and a dense direct solve.
"""
import numpy as np
import pytest

import oracle
import oracle.amg as M
from paper_1801_03690_amd import inputs


def laplacian_chain(n):
    rows, cols, vals = [], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
                vals.append(v)
    return M.from_coo(rows, cols, vals, n, n)


def laplacian_grid(nx, ny):
    rows, cols, vals = [], [], []
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            rows.append(i)
            cols.append(i)
            vals.append(4.0)
            for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                if 0 <= x + dx < nx and 0 <= y + dy < ny:
                    rows.append(i)
                    cols.append(x + dx + nx * (y + dy))
                    vals.append(-1.0)
    return M.from_coo(rows, cols, vals, nx * ny, nx * ny)


def kuhn_K(ncell):
    o = oracle.Oracle(inputs.small_box(ncell, 4.0))
    p, j, v = o.K_csr()
    return o, M.Csr(p, j, v, o.np)


def test_chain_aggregates_and_prolongator_by_hand():
    # pass 1 in row order: {0,1} (row 0), {2,3,4} (row 3), {5,6,7}, {8,9,10};
    # rows 2, 5, 8 are skipped by pass 1 (a neighbour is taken) and picked up
    # by a later root
    A = laplacian_chain(11)
    agg, na = M.aggregate(A, M.THETA0)
    assert na == 4
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3]
    # rho (Gershgorin) = 2, omega = 2/3; P = (I - A/3) P0
    assert M.gershgorin_rho(A) == 2.0
    P = M.smoothed_prolongator(A, agg, na, 2.0 / 3.0).dense()
    want = np.zeros((11, 4))
    want[0] = [2 / 3, 0, 0, 0]        # end of the chain: (2 - 1) / 3 leaks to no aggregate
    want[1] = [2 / 3, 1 / 3, 0, 0]    # neighbour 2 lies in aggregate 1
    want[2] = [1 / 3, 2 / 3, 0, 0]
    want[3] = [0, 1, 0, 0]            # inside its aggregate
    want[4] = [0, 2 / 3, 1 / 3, 0]
    want[5] = [0, 1 / 3, 2 / 3, 0]
    want[6] = [0, 0, 1, 0]
    want[7] = [0, 0, 2 / 3, 1 / 3]
    want[8] = [0, 0, 1 / 3, 2 / 3]
    want[9] = [0, 0, 0, 1]
    want[10] = [0, 0, 0, 2 / 3]
    assert np.abs(P - want).max() < 1e-15


def test_grid_aggregates_by_hand():
    # 3x3 grid, 5-point stencil, rows x-fastest:
    #   row 0 starts {0, 1, 3}; rows 2 and 4 have a taken neighbour; row 5
    #   starts {2, 4, 5, 8}; pass 2: row 6 joins aggregate 0 (via 3), row 7
    #   ties between 4 and 8 (same weight) and takes the lower column, 4
    A = laplacian_grid(3, 3)
    agg, na = M.aggregate(A, M.THETA0)
    assert na == 2
    assert agg.tolist() == [0, 0, 1, 0, 1, 1, 0, 1, 1]


def test_aggregates_partition_into_connected_sets():
    _, A = kuhn_K((4, 4, 4))
    A = M.from_coo(A.rows(), A.j, A.v, A.n, A.ncols)
    agg, na = M.aggregate(A, M.THETA0)
    assert agg.min() == 0 and agg.max() == na - 1
    assert np.bincount(agg, minlength=na).min() >= 1
    S = M.strong_neighbours(A, M.THETA0)
    for a in range(na):
        mem = set(np.nonzero(agg == a)[0].tolist())
        seen, stack = set(), [min(mem)]
        while stack:
            i = stack.pop()
            if i in seen:
                continue
            seen.add(i)
            stack.extend(j for j in S[i][0].tolist() if j in mem)
        assert seen == mem, a


def test_galerkin_product_matches_dense():
    _, A = kuhn_K((4, 4, 4))
    lv = M.hierarchy(A, coarse_max=64)
    assert len(lv) >= 2
    for l in range(len(lv) - 1):
        Ad, Pd = lv[l].A.dense(), lv[l].P.dense()
        Ac = lv[l + 1].A.dense()
        ref = Pd.T @ Ad @ Pd
        assert np.abs(Ac - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(Ac - Ac.T).max() <= 1e-13 * np.abs(Ac).max()
        assert np.all(np.linalg.eigvalsh(Ac) > 0)
        assert lv[l].R.dense().tolist() == Pd.T.tolist()


def test_vcycle_is_spd_with_spectrum_in_unit_interval():
    """The error propagator of a symmetric V(1,1) cycle with a convergent
    smoother is A-self-adjoint and positive semidefinite with norm < 1, so
    the cycle M is symmetric and eig(M A) lies in (0, 1]."""
    _, A = kuhn_K((4, 4, 4))
    lv = M.hierarchy(A, coarse_max=64)
    assert len(lv) >= 3
    n = A.n
    Md = np.stack([M.vcycle(lv, e) for e in np.eye(n)], axis=1)
    assert np.abs(Md - Md.T).max() <= 1e-12 * np.abs(Md).max()
    Ad = lv[0].A.dense()
    # M A is similar to the symmetric A^1/2 M A^1/2
    w, V = np.linalg.eigh(Ad)
    Ah = (V * np.sqrt(w)) @ V.T
    ev = np.linalg.eigvalsh(Ah @ Md @ Ah)
    assert ev.min() > 1e-3, ev.min()
    assert ev.max() <= 1.0 + 1e-10, ev.max()


def test_single_level_is_the_exact_inverse():
    _, A = kuhn_K((2, 2, 2))
    assert A.n <= M.COARSE_MAX
    lv = M.hierarchy(A)
    assert len(lv) == 1
    b = np.random.default_rng(3).standard_normal(A.n)
    x = np.linalg.solve(A.dense(), b)
    assert np.abs(M.vcycle(lv, b) - x).max() <= 1e-12 * np.abs(x).max()
    y, it = M.solve(A, b, rtol=1e-12, levels=lv)
    assert it == 1


def test_amg_pcg_matches_direct_and_beats_jacobi():
    o, A = kuhn_K((6, 6, 6))
    b = np.random.default_rng(4).standard_normal(A.n)
    x, it = M.solve(A, b, rtol=1e-10, coarse_max=128)
    xd = np.linalg.solve(A.dense(), b)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()
    _, itj = o.poisson(b, rtol=1e-10)
    assert it <= 20 and itj >= 3 * it, (it, itj)
    # a warm start at the solution needs no update
    _, it0 = M.solve(A, b, x0=xd, rtol=1e-8)
    assert it0 == 0


def test_pcg_zero_rhs():
    _, A = kuhn_K((2, 2, 2))
    x, it = M.solve(A, np.zeros(A.n), x0=np.ones(A.n))
    assert it == 0 and not x.any()
