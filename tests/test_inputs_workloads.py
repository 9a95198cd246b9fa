"""The synthetic workloads' recipes (CPU): shapes, materials, easy axes and
field schedules as stated for each workload, and the polycrystal's grain and
grain-boundary assignment by brute force on a small instance."""
import math

import numpy as np

from paper_1801_03690_amd import inputs

MU0 = 4e-7 * math.pi


def _angle_deg(a, b):
    c = np.clip((a * b).sum(axis=-1) / (np.linalg.norm(a, axis=-1) * np.linalg.norm(b, axis=-1)), -1.0, 1.0)
    return np.degrees(np.arccos(c))


def test_polycrystal_grains_and_boundary_phase_by_brute_force():
    n, edge, ng, width = 10, 25.0, 5, 2.0
    w = inputs.polycrystal(n=n, edge=edge, n_grains=ng, gb_width=width)
    mesh = w.mesh
    seeds = mesh.meta["seeds"]
    axes = mesh.meta["axes"]
    mag = np.nonzero(mesh.region > 0)[0]
    assert mag.size == 6 * n ** 3
    cen = mesh.xyz[mesh.tets[mag]].mean(axis=1)
    for t, c in zip(mag, cen):
        d = [float(np.sum((c - s) ** 2)) for s in seeds]
        p = int(np.argmin(d))
        # distance to the bisector plane of seeds p and q
        dist = min(abs(np.dot(c - 0.5 * (seeds[p] + seeds[q]), seeds[q] - seeds[p])) / np.linalg.norm(seeds[q] - seeds[p])
                   for q in range(ng) if q != p)
        if dist < width:
            assert mesh.region[t] == ng + 1
            assert mesh.K1[t] == 0.0 and mesh.A[t] == 1.0e-12
        else:
            assert mesh.region[t] == p + 1
            assert mesh.K1[t] == 4.3e6 and mesh.A[t] == 7.7e-12
        np.testing.assert_array_equal(mesh.axis[t], axes[p])
    assert np.all(mesh.Ms[mag] == 1.61 / MU0)
    assert np.all(_angle_deg(axes, np.array([0.0, 0.0, 1.0])) <= 20.0 + 1e-9)
    assert len(w.fields) == 121 and np.allclose(w.fields[-1], [0.0, 0.0, -6.0])


def test_batch_cubes_recipe():
    ws = inputs.batch_cubes()
    assert len(ws) == 64
    z = np.array([0.0, 0.0, 1.0])
    sizes = []
    for w in ws:
        mesh = w.mesh
        mag = mesh.region > 0
        nc = round((np.sum(mag) / 6) ** (1 / 3))
        sizes.append(nc)
        assert 8 <= nc <= 24 and np.sum(mag) == 6 * nc ** 3
        assert abs(mesh.h - 4.0) < 1e-12
        k1 = np.unique(mesh.K1[mag])
        assert k1.size == 1 and 3.0e6 <= k1[0] <= 4.9e6
        ax = np.unique(mesh.axis[mag], axis=0)
        assert ax.shape[0] == 1 and _angle_deg(ax[0], z) <= 15.0 + 1e-9
        assert len(w.fields) == 81 and np.allclose(w.fields[-1], [0.0, 0.0, -8.0])
    assert len(set(sizes)) > 8


def test_film_and_hard_cube_recipes():
    f = inputs.film()
    mag = f.mesh.region > 0
    assert np.sum(mag) == 6 * 200 * 200 * 2 and abs(f.mesh.h - 5.0) < 1e-12
    assert len(f.fields) == 101
    np.testing.assert_allclose(f.fields[0], [0.05, 0.0, 0.0])
    np.testing.assert_allclose(f.fields[-1], [-0.05, 0.0, 0.0], atol=1e-15)
    h = inputs.hard_cube()
    mag = h.mesh.region > 0
    assert np.sum(mag) == 6 * 20 ** 3 and abs(h.mesh.h - 4.0) < 1e-12
    ax = np.unique(h.mesh.axis[mag], axis=0)
    assert ax.shape[0] == 1
    assert abs(_angle_deg(ax[0], np.array([0.0, 0.0, 1.0])) - 1.0) < 1e-9 and ax[0][0] > 0
    assert len(h.fields) == 161 and np.allclose(h.fields[-1], [0.0, 0.0, -8.0])
    # the 3x air box: the magnet is centred with its own cell count of air per side
    assert h.mesh.shape == (60, 60, 60) and h.mesh.mag_cells == ((20, 40),) * 3
