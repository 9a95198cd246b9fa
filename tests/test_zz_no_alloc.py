"""The allocation-free entry point mm_precondition_noalloc against
mm_precondition, through the C ABI: the same kernels on the same inputs, so
the results must be identical bit for bit (and match the oracle like
mm_precondition does). Two calls in a row on one GPU, the second on a smaller
problem, so that the second call reads the static scratch the first left.
"""
import math

import numpy as np
import pytest

from paper_1801_03690_amd import inputs

pytestmark = pytest.mark.gpu

MU0 = 4e-7 * math.pi


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


def _case(B, oracle_mod, mesh, seed, jmax, dscale):
    o = oracle_mod.Oracle(mesh)
    o.set_poisson(1e-13)
    ctx = B.Context(0)
    ctx.upload(mesh)
    ctx.set_opts(poisson_rtol=1e-13)
    m = inputs.tilted_state(o.nm, (0, 0, 1), 0.3, np.random.Generator(np.random.PCG64(seed)))
    ro = o.eval_T(m, [0.0, 0.0, 0.5])
    s = None if not dscale else np.linspace(0.5, 2.0, o.nm)
    y_na, it_na = ctx.precondition(m, ro["G"], ro["g"], jmax, dscale=s, noalloc=True)
    y, it = ctx.precondition(m, ro["G"], ro["g"], jmax, dscale=s)
    yo, ito = o.precond(m, ro["lam"], ro["g"], jmax, dscale=s)
    ctx.close()
    return (y_na, it_na), (y, it), (yo, ito)


@pytest.mark.parametrize("jmax", [3, 40])
def test_noalloc_matches_precondition_twice_second_smaller(B, oracle_mod, jmax):
    big = inputs.small_box((14, 12, 10), 2.0, Ms=1.61 / MU0, A=7.7e-12, K1=4.3e6, axis=(0.1, 0.0, 0.99))
    small = inputs.small_box((5, 4, 3), 3.0, Ms=1.61 / MU0, A=7.7e-12, K1=4.3e6, axis=(0.2, 0.1, 0.97))
    for mesh, seed, ds in ((big, 11, True), (small, 12, False)):
        (y_na, it_na), (y, it), (yo, ito) = _case(B, oracle_mod, mesh, seed, jmax, ds)
        assert it_na == it == ito
        np.testing.assert_array_equal(y_na, y)
        assert np.abs(y_na - yo).max() <= 1e-10 * np.abs(yo).max()


def test_noalloc_refuses_what_the_scratch_cannot_hold(B):
    """A magnet of 81^3 nodes (531,441, no air box) needs more than the 32 MiB
    static array holds: refused with MM_EINVAL, nothing written."""
    mesh = inputs.small_box((80, 80, 80), 2.0, air=False)
    ctx = B.Context(0)
    ctx.upload(mesh)
    m = np.tile([0.0, 0.0, 1.0], (ctx.n_mag, 1))
    g = np.zeros_like(m)
    with pytest.raises(B.MMError) as e:
        ctx.precondition(m, g, g, 3, noalloc=True)
    assert e.value.code == B.MM_EINVAL
    ctx.close()
