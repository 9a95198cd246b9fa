"""GPU: the multigrid-preconditioned scalar-potential CG against its oracle.

The library builds its smoothed-aggregation hierarchy from its own assembled
matrix, the oracle from its own: the aggregates must agree exactly on every
level, the level operators and prolongators to round-off, one cycle in FP64
to 1e-11 of its size (FP32 to 1e-5), and the multigrid-preconditioned solve
to the solve tolerance, with iteration counts within one of the oracle's
(the two CG forms differ only in rounding). Meshes span several SELL slices
with a ragged last one, and two or three levels; the 2x2x2 magnet has a
single level.
"""
import numpy as np
import pytest

import oracle
import oracle.amg as M
from paper_1801_03690_amd import inputs

pytestmark = pytest.mark.gpu


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="module")
def B():
    if not _gpu_available():
        pytest.skip("no GPU")
    from paper_1801_03690_amd import binding
    return binding


def setup(B, ncell, **mat):
    mesh = inputs.small_box(ncell, 4.0, **mat)
    ctx = B.Context(0).upload(mesh)
    o = oracle.Oracle(mesh)
    p, j, v = o.K_csr()
    lv = M.hierarchy(M.Csr(p, j, v, o.np))
    return mesh, ctx, o, lv


def sparse_diff(ptr, col, val, ref):
    """Largest |entry difference| between a CSR (ptr, col, val) and an
    oracle Csr with the same shape (entries missing on one side count as 0)."""
    n, nc = ptr.size - 1, ref.ncols
    ka = np.repeat(np.arange(n), np.diff(ptr)).astype(np.int64) * nc + col
    kb = ref.rows().astype(np.int64) * nc + ref.j
    keys = np.union1d(ka, kb)
    va = np.zeros(keys.size)
    vb = np.zeros(keys.size)
    va[np.searchsorted(keys, ka)] = val
    vb[np.searchsorted(keys, kb)] = ref.v
    return np.abs(va - vb).max(), np.abs(vb).max()


@pytest.mark.parametrize("ncell", [(6, 6, 6), (9, 8, 7), (14, 14, 14)])
def test_hierarchy_matches_oracle(B, ncell):
    mesh, ctx, o, lv = setup(B, ncell)
    info = ctx.amg_info()
    print(ncell, info)
    assert info["levels"] == len(lv) >= 2
    assert info["rows"] == [L.A.n for L in lv]
    if ncell == (14, 14, 14):
        assert len(lv) >= 3
    for l in range(len(lv)):
        pa, ja, va = ctx.amg_level_matrix(l, 0)
        d, sc = sparse_diff(pa, ja, va, lv[l].A)
        assert d <= 1e-12 * sc, l
        if l + 1 < len(lv):
            agg = ctx.amg_aggregates(l)
            assert np.array_equal(agg, lv[l].agg), l
            pp, jp, vp = ctx.amg_level_matrix(l, 1)
            d, sc = sparse_diff(pp, jp, vp, lv[l].P)
            assert d <= 1e-12 * sc, l
    ctx.close()


@pytest.mark.parametrize("ncell", [(9, 8, 7), (14, 14, 14)])
def test_cycle_matches_oracle(B, ncell):
    mesh, ctx, o, lv = setup(B, ncell)
    rng = np.random.default_rng(5)
    for k in range(2):
        r = rng.standard_normal(o.np)
        z = M.vcycle(lv, r)
        z64 = ctx.amg_apply(r, B.MM_FP64)
        z32 = ctx.amg_apply(r, B.MM_FP32_BULK)
        sc = np.abs(z).max()
        assert np.abs(z64 - z).max() <= 1e-11 * sc
        assert np.abs(z32 - z).max() <= 1e-5 * sc
        # linear: the cycle of 2r is twice the cycle of r (FP64)
        assert np.abs(ctx.amg_apply(2.0 * r, B.MM_FP64) - 2.0 * z64).max() <= 1e-14 * sc
    ctx.close()


def test_single_level_is_the_dense_inverse(B):
    mesh, ctx, o, lv = setup(B, (2, 2, 2))
    assert len(lv) == 1 and ctx.amg_info()["levels"] == 1
    b = np.random.default_rng(6).standard_normal(o.np)
    x = np.linalg.solve(lv[0].A.dense(), b)
    assert np.abs(ctx.amg_apply(b) - x).max() <= 1e-11 * np.abs(x).max()
    ctx.set_opts(poisson_prec=B.MM_PREC_AMG, poisson_rtol=1e-12)
    u, it = ctx.poisson(b, rtol=1e-12)
    assert it == 1
    assert np.abs(u - x).max() <= 1e-10 * np.abs(x).max()
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_amg_solve_matches_oracle(B, precision):
    mesh, ctx, o, lv = setup(B, (9, 8, 7))
    prec = B.MM_FP64 if precision == "fp64" else B.MM_FP32_BULK
    ctx.set_opts(poisson_prec=B.MM_PREC_AMG, precision=prec)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(o.np)
    xo, ito = M.solve(lv[0].A, b, rtol=1e-10, levels=lv)
    u, it = ctx.poisson(b, rtol=1e-10)
    xj, itj = o.poisson(b, rtol=1e-12)
    print(precision, "amg iterations", it, "oracle", ito, "jacobi oracle", itj)
    assert np.abs(u - xj).max() <= 1e-8 * np.abs(xj).max()
    if precision == "fp64":
        assert abs(it - ito) <= 1
    # warm start at the answer: nothing to do
    u2, it2 = ctx.poisson(b, u0=u, rtol=1e-8)
    assert it2 == 0
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_amg_curve_matches_jacobi_curve(B, precision):
    """The preconditioner of the scalar-potential CG changes none of the
    method's results beyond the solve tolerance."""
    w = inputs.hard_cube(n=6, step_T=0.5, stop_T=-4.0)
    ctx = B.Context(0).upload(w.mesh)
    prec = B.MM_FP64 if precision == "fp64" else B.MM_FP32_BULK
    rj = ctx.curve(w.m0, w.fields, opts=B.default_opts(jmax=10, precision=prec))
    ctx.reset_warm_start()
    ra = ctx.curve(w.m0, w.fields, opts=B.default_opts(jmax=10, precision=prec, poisson_prec=B.MM_PREC_AMG))
    assert rj["rc"] == 0 and ra["rc"] == 0
    dE = np.abs(ra["E"] - rj["E"]) / np.abs(rj["E"])
    tol = 1e-8 if precision == "fp64" else 1e-5
    print(precision, "max rel dE", dE.max(), "CG iterations jacobi", sum(s["mi"] for s in rj["stats"]),
          "amg", sum(s["mi"] for s in ra["stats"]))
    assert dE.max() <= tol
    assert np.abs(ra["m_avg"] - rj["m_avg"]).max() <= 1e-5
    assert sum(s["mi"] for s in ra["stats"]) < sum(s["mi"] for s in rj["stats"])
    ctx.close()


def test_amg_batch_limits(B):
    """The hierarchy queries are single-instance calls; a batch with an
    instance small enough for a single dense level is refused."""
    ws = [inputs.small_box((3, 3, 3), 4.0), inputs.small_box((4, 3, 3), 4.0)]
    ctx = B.Context(0)
    ctx.upload_batch(ws)
    with pytest.raises(B.MMError):
        ctx.amg_info()
    m0 = np.concatenate([inputs.random_unit(ctx.inst_info[i]["n_mag"], i) for i in range(2)])
    with pytest.raises(B.MMError):
        ctx.batch_curve(m0, np.zeros((2, 1, 3)), jmax=4, poisson_prec=B.MM_PREC_AMG)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_amg_matches_single_instances(B, precision):
    """A batch whose instances have two- and three-level hierarchies (dense
    solves on different levels in one launch) gives every instance the curve
    of its own single-instance multigrid run, and of the Jacobi batch, to the
    solve tolerance."""
    ws = [inputs.hard_cube(n=6, step_T=0.5, stop_T=-2.0),
          inputs.hard_cube(n=14, step_T=0.5, stop_T=-2.0, seed=3),
          inputs.hard_cube(n=9, step_T=0.5, stop_T=-2.0, seed=4)]
    prec = B.MM_FP64 if precision == "fp64" else B.MM_FP32_BULK
    F = np.stack([w.fields for w in ws])
    m0 = np.concatenate([w.m0 for w in ws])
    levels = []
    singles = []
    for w in ws:
        ctx = B.Context(0).upload(w.mesh)
        levels.append(ctx.amg_info()["levels"])
        singles.append(ctx.curve(w.m0, w.fields, opts=B.default_opts(jmax=10, precision=prec,
                                                                         poisson_prec=B.MM_PREC_AMG)))
        ctx.close()
    assert len(set(levels)) >= 2, levels
    ctx = B.Context(0).upload_batch([w.mesh for w in ws])
    ra = ctx.batch_curve(m0, F, opts=B.default_opts(jmax=10, precision=prec, poisson_prec=B.MM_PREC_AMG))
    ctx.reset_warm_start()
    rj = ctx.batch_curve(m0, F, opts=B.default_opts(jmax=10, precision=prec))
    ctx.close()
    assert ra["rc"] == 0 and rj["rc"] == 0
    for i, r1 in enumerate(singles):
        dE = np.abs(ra["E"][i] - r1["E"]) / np.abs(r1["E"])
        dJ = np.abs(ra["E"][i] - rj["E"][i]) / np.abs(rj["E"][i])
        print(precision, i, levels[i], "max rel dE vs single", dE.max(), "vs jacobi batch", dJ.max(),
              "CG iterations batch", sum(s["mi"] for s in ra["stats"][i]), "single",
              sum(s["mi"] for s in r1["stats"]), "jacobi", sum(s["mi"] for s in rj["stats"][i]))
        assert dE.max() <= 1e-9 and dJ.max() <= 1e-8
        assert np.abs(ra["m_avg"][i] - r1["m_avg"]).max() <= 1e-6
        assert sum(s["mi"] for s in ra["stats"][i]) < sum(s["mi"] for s in rj["stats"][i])


def test_hard_cube_curve_is_run_to_run_identical(B):
    """The headline configuration (20^3 hard cube, FP32 bulk, multigrid CG,
    the workload's j_max) on its first 12 fields, twice in fresh contexts:
    every reduction has a fixed order, so states, energies and iteration
    counts agree bit for bit."""
    w = inputs.hard_cube()
    out = []
    for _ in range(2):
        ctx = B.Context(0).upload(w.mesh)
        r = ctx.curve(np.array(w.m0), w.fields[:12], jmax=w.jmax, precision=B.MM_FP32_BULK,
                      poisson_prec=B.MM_PREC_AMG)
        assert r["rc"] == 0
        out.append(r)
        ctx.close()
    np.testing.assert_array_equal(out[0]["m"], out[1]["m"])
    np.testing.assert_array_equal(out[0]["E"], out[1]["E"])
    np.testing.assert_array_equal(out[0]["m_avg"], out[1]["m_avg"])
    for a, b in zip(out[0]["stats"], out[1]["stats"]):
        for k in ("evals", "nli", "li", "mi", "restarts", "fallbacks", "status"):
            assert a[k] == b[k], k
