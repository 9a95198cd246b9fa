"""The adapted rotation cap (mm_opts.theta_adapt) on the GPU against the
oracle's, through the C ABI: the soft cube's whole curve and a full reversal
of a soft magnet, each to the bar of the FP64 curve tests (energy within 1e-8
of its scale, every nodal m within 1e-5), and fewer nonlinear iterations than
the fixed cap on the reversal."""
import numpy as np
import pytest

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


def test_soft_cube_curve_with_the_adapted_cap_matches_oracle(B, oracle_mod):
    w = inputs.soft_cube()
    o = oracle_mod.Oracle(w.mesh)
    ro = o.curve(w.m0, w.fields, jmax=w.jmax, keep_hist=True, theta_adapt=1)
    assert ro["rc"] == 0
    scale = np.array([max(abs(ro["E"][k]), float(np.abs(o.eval_T(ro["hist"][k], w.fields[k])["E"][:4]).sum()))
                      for k in range(len(w.fields))])
    ctx = B.Context(0)
    ctx.upload(w.mesh)
    rg = ctx.curve(w.m0, w.fields, jmax=w.jmax, theta_adapt=1, keep_hist=True)
    ctx.close()
    assert rg["rc"] == 0
    dE = np.abs(rg["E"] - ro["E"]) / scale
    dm = np.abs(rg["hist"] - ro["hist"]).max(axis=(1, 2))
    print(f"soft cube (adapted cap): max rel dE {dE.max():.2e}, max |dm| {dm.max():.2e}")
    assert dE.max() <= 1e-8, dE
    assert dm.max() <= 1e-5, dm


def test_reversal_with_the_adapted_cap_matches_oracle_in_fewer_iterations(B, oracle_mod):
    mesh = inputs.small_box((4, 4, 3), 4.0, **inputs.SOFT)
    o = oracle_mod.Oracle(mesh)
    m0 = inputs.tilted_state(o.nm, (0.0, 0.05, 1.0), 0.2, np.random.Generator(np.random.PCG64(7)))
    h = [0.0, 0.0, -1.0]
    mo, Eo, so, rco = o.minimize(m0, h, jmax=4, theta_adapt=1)
    ctx = B.Context(0)
    ctx.upload(mesh)
    mf, Ef, sf, rcf = ctx.minimize(m0, h, jmax=4)
    ctx.reset_warm_start()
    ma, Ea, sa, rca = ctx.minimize(m0, h, jmax=4, theta_adapt=1)
    ctx.close()
    assert rco == 0 and rcf == 0 and rca == 0
    assert abs(Ea[4] - Eo[4]) <= 1e-8 * max(abs(Eo[4]), 1.0)
    assert np.abs(ma - mo).max() <= 1e-5
    assert sa["nli"] < sf["nli"], (sa["nli"], sf["nli"])
