"""Single-domain limit of a soft cube (Sec. 3.3) on a coarse mesh (GPU).

12 cells per edge (0.58-0.83 exchange lengths) keep the test short; the
module's default is the paper's 0.35 l_ex. Checked:
* the stray-field energy density of the uniform cube is exactly 1/3 Kd; a
  zero potential on the air box's boundary can only understate it, less so
  for a larger box;
* well below the limit (7 l_ex) relaxing from two domains gains nothing over
  relaxing from saturation (the flower state has the lower or an equal
  energy); well above it (10 l_ex) the vortex state has the lower energy and
  the smaller net moment.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_uniform_cube_demag_bound_and_box_convergence():
    from paper_1801_03690_amd import binding as B, inputs, sp3
    ed = []
    for pad in (12, 24):
        w = inputs.sp3_cube(8.5, 12, "flower", pad=pad)
        ctx = B.Context(0).upload(w.mesh)
        ed.append(sp3.uniform_demag(ctx, w))
        ctx.close()
    assert 0.25 < ed[0] < ed[1] < 1.0 / 3.0, ed


def test_flower_below_and_vortex_above_the_limit():
    from paper_1801_03690_amd import sp3
    rep = sp3.main(["--sizes", "7,10", "--n", "12"])
    small, large = rep["sizes"]
    for r in (small, large):
        for k in ("flower", "vortex"):
            assert r[k]["rc"] == 0 and r[k]["status"] == 0, (r["size_lex"], k, r[k])
    assert small["flower"]["e"] <= small["vortex"]["e"] + 1e-9
    assert large["vortex"]["e"] < large["flower"]["e"]
    assert np.linalg.norm(large["vortex"]["m_avg"]) < np.linalg.norm(large["flower"]["m_avg"])
    assert len(rep["crossing_lex"]) <= 1 and all(7.0 < c < 10.0 for c in rep["crossing_lex"])
