"""Single-domain limit of a soft cube (Sec. 3.3) on a coarse mesh (GPU).

12 cells per edge (0.58-0.83 exchange lengths) keep the test short; the
module's default is the paper's 0.35 l_ex. Checked:
* the stray-field energy density of the uniform cube is exactly 1/3 Kd; a
  zero potential on the air box's boundary can only understate it, less so
  for a larger box;
* well below the limit (7 l_ex) relaxing from two domains gains nothing over
  relaxing from saturation (the flower state has the lower or an equal
  energy); well above it (10 l_ex) the vortex state has the lower energy and
  the smaller net moment;
* at the paper's mesh size the crossing lies at the paper's 8.52 l_ex
  (Sec. 3.3; tests/golden/sp3_single_domain_limit.txt).
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
    # at 7 l_ex both starts may end in the same flower, so their difference is
    # rounding and an interpolated crossing can sit on 7 itself
    assert len(rep["crossing_lex"]) <= 1 and all(7.0 <= c < 10.0 for c in rep["crossing_lex"])


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    kv = dict(line.split(None, 1) for line in open(path) if line.strip() and not line.startswith("#"))
    return {k: float(v) for k, v in kv.items()}


def test_single_domain_limit_matches_the_paper():
    """At the paper's mesh size (24 cells per edge, 0.35 l_ex near 8.5 l_ex)
    the flower-vortex crossing lies within 0.1 l_ex of the 8.52 l_ex of
    Sec. 3.3. The margin covers what separates independent solvers (the
    cited 8.56) and what the finite air box still moves: going from a 5x to
    the 7x box moved the crossing by 0.055 l_ex."""
    from paper_1801_03690_amd import sp3
    want = _golden("sp3_single_domain_limit.txt")["critical_size_lex"]
    rep = sp3.main(["--sizes", "8.3,8.7"])
    for r in rep["sizes"]:
        for k in ("flower", "vortex"):
            assert r[k]["rc"] == 0 and r[k]["status"] == 0, (r["size_lex"], k)
    assert len(rep["crossing_lex"]) == 1, rep["crossing_lex"]
    assert abs(rep["crossing_lex"][0] - want) < 0.1, rep["crossing_lex"]
