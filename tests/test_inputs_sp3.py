"""Inputs of the single-domain-limit workload (Sec. 3.3) and the crossing
interpolation (CPU)."""
import math

import numpy as np

from paper_1801_03690_amd import inputs, sp3


def test_exchange_length_and_mesh_size():
    kd = 0.5 * 4e-7 * math.pi * 8.0e5 ** 2
    assert abs(inputs.lex_soft() - 1e9 * math.sqrt(1.3e-11 / kd)) < 1e-12
    w = inputs.sp3_cube(8.5, 6, "flower", pad=2)
    assert abs(w.meta["h_nm"] * 6 - 8.5 * inputs.lex_soft()) < 1e-9
    mag = w.mesh.region > 0
    assert np.allclose(w.mesh.K1[mag], 0.1 * kd) and np.all(w.mesh.K1[~mag] == 0)


def test_two_domain_start_has_a_sharp_wall_at_x0():
    wf = inputs.sp3_cube(8.5, 6, "flower", pad=2)
    wv = inputs.sp3_cube(8.5, 6, "vortex", pad=2)
    x = wv.mesh.xyz[wv.mesh.magnet_nodes(), 0]
    assert np.allclose(np.linalg.norm(wv.m0, axis=1), 1.0)
    assert np.all(wf.m0[:, 2] > 0.99)
    assert np.all(wv.m0[x <= 0, 2] > 0.99) and np.all(wv.m0[x > 0, 2] < -0.99)
    # the same tilts, mirrored in z on the far side
    np.testing.assert_array_equal(wv.m0[:, :2], wf.m0[:, :2])


def test_crossing_interpolation():
    s = [8.0, 8.5, 9.0]
    assert sp3.crossing(s, [-2.0, -1.0, 1.0]) == [8.75]
    assert sp3.crossing(s, [-1.0, -0.5, -0.1]) == []
    assert sp3.crossing(s, [0.0, 1.0, 2.0]) == [8.0]
