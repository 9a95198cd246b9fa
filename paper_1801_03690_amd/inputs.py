"""Seeded synthetic inputs: meshes, materials, initial states and field schedules.

This module builds the *inputs* of the micromagnetic minimizer and nothing else:
node coordinates, tetrahedra, region labels, per-tetrahedron SI material
constants, the starting magnetization and the list of applied fields. It holds
none of the method's arithmetic (no finite-element quantities, no units
conversion, no energy): both the HIP library and the CPU oracle receive these
arrays and derive everything else on their own.

Meshes are structured boxes of cubic cells, each cell split into six
tetrahedra along its main diagonal (Kuhn/Freudenthal split). The magnet sits in
the middle of an air box whose edge is three times the magnet's edge per axis,
as the paper encloses the magnet in an air box for the scalar potential
(Sec. 3.1, implementation details). Sizes, materials and schedules follow the
synthetic stand-ins for the paper's workloads (standard problems 1 and 3 and
the granular permanent magnets of Sec. 3); the paper's own meshes are not
available, so these seeded meshes replace them.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

MU0 = 4e-7 * math.pi

# The six permutations of the axes; tet sigma = {x_s0 >= x_s1 >= x_s2} inside
# the unit cell, vertices 000 -> e_s0 -> e_s0+e_s1 -> 111.
_PERMS = list(itertools.permutations(range(3)))


def _perm_parity(p):
    inv = 0
    for i in range(3):
        for j in range(i + 1, 3):
            inv += p[i] > p[j]
    return inv % 2


def kuhn_cell_tets():
    """Local corner indices (bit0=x, bit1=y, bit2=z) of the 6 tets of a cell,
    ordered so that every tet has positive orientation."""
    out = []
    for p in _PERMS:
        v0 = 0
        v1 = 1 << p[0]
        v2 = v1 | (1 << p[1])
        v3 = 7
        t = [v0, v1, v2, v3]
        if _perm_parity(p):
            t[1], t[2] = t[2], t[1]
        out.append(t)
    return np.array(out, dtype=np.int64)


@dataclass
class Mesh:
    xyz: np.ndarray        # (nn, 3) float64, nm
    tets: np.ndarray       # (nt, 4) int32, 0-based
    region: np.ndarray     # (nt,) int32, 0 = air, k > 0 = material k
    Ms: np.ndarray         # (nt,) A/m
    A: np.ndarray          # (nt,) J/m
    K1: np.ndarray         # (nt,) J/m^3
    axis: np.ndarray       # (nt, 3) unit easy axis
    shape: tuple = ()      # (cells per axis of the box)
    mag_cells: tuple = ()  # (lo, hi) cell ranges of the magnet per axis
    h: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return self.xyz.shape[0]

    @property
    def n_tets(self):
        return self.tets.shape[0]

    def magnet_nodes(self):
        """Nodes touched by a tet with region > 0, ascending."""
        mask = np.zeros(self.n_nodes, dtype=bool)
        mask[self.tets[self.region > 0].ravel()] = True
        return np.nonzero(mask)[0].astype(np.int32)


def box_mesh(ncell, h, pad=None, air=True):
    """Structured Kuhn mesh of a box of `ncell` magnet cells (nx, ny, nz) with
    spacing h (nm). With air=True the magnet is centred in a box padded by
    `pad` cells per side (default: the magnet's own cell count, i.e. a 3x box).
    Returns (xyz, tets, cell_index (nt,3), magnet mask (nt,))."""
    ncell = tuple(int(c) for c in ncell)
    if air:
        if pad is None:
            pad = ncell
        pad = tuple(int(p) for p in pad)
    else:
        pad = (0, 0, 0)
    nb = tuple(ncell[i] + 2 * pad[i] for i in range(3))
    nx, ny, nz = nb
    gx = (np.arange(nx + 1) - pad[0] - ncell[0] / 2.0) * h
    gy = (np.arange(ny + 1) - pad[1] - ncell[1] / 2.0) * h
    gz = (np.arange(nz + 1) - pad[2] - ncell[2] / 2.0) * h
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    # node id = i + (nx+1)*(j + (ny+1)*k): x fastest
    xyz = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                    Z.transpose(2, 1, 0).ravel()], axis=1).astype(np.float64)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    ncells = ci.size
    local = kuhn_cell_tets()  # (6, 4) corner bits
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    base = ci + sx * cj + sy * ck
    corner_off = np.array([(b & 1) + sx * ((b >> 1) & 1) + sy * ((b >> 2) & 1) for b in range(8)],
                          dtype=np.int64)
    tets = (base[:, None, None] + corner_off[local][None, :, :]).reshape(ncells * 6, 4)
    cell = np.repeat(np.stack([ci, cj, ck], axis=1), 6, axis=0)
    mag = np.ones(ncells * 6, dtype=bool)
    for a in range(3):
        mag &= (cell[:, a] >= pad[a]) & (cell[:, a] < pad[a] + ncell[a])
    return xyz, tets.astype(np.int32), cell, mag, nb, pad


def uniform_material(nt, mag, Ms, A, K1, axis):
    Ms_t = np.where(mag, Ms, 0.0)
    A_t = np.where(mag, A, 0.0)
    K_t = np.where(mag, K1, 0.0)
    ax = np.zeros((nt, 3))
    ax[:] = np.asarray(axis, dtype=np.float64)
    return Ms_t, A_t, K_t, ax


def make_box_magnet(ncell, h, Ms, A, K1, axis, air=True, pad=None):
    xyz, tets, cell, mag, nb, padv = box_mesh(ncell, h, pad=pad, air=air)
    Ms_t, A_t, K_t, ax = uniform_material(tets.shape[0], mag, Ms, A, K1, axis)
    region = mag.astype(np.int32)
    return Mesh(xyz, tets, region, Ms_t, A_t, K_t, ax, shape=nb,
                mag_cells=tuple((padv[i], padv[i] + int(ncell[i])) for i in range(3)), h=h)


# ---------------------------------------------------------------------------
# random helpers (numpy PCG64)
# ---------------------------------------------------------------------------

def _orthonormal_frame(n):
    n = np.asarray(n, dtype=np.float64)
    n = n / np.linalg.norm(n)
    t = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = t - np.dot(t, n) * n
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    return e1, e2, n


def tilted_state(n_nodes, nominal, max_tilt, rng):
    """Unit vectors tilted from `nominal` by theta = max_tilt*U[0,1) at
    azimuth phi = 2*pi*U[0,1)."""
    e1, e2, n = _orthonormal_frame(nominal)
    th = max_tilt * rng.random(n_nodes)
    ph = 2.0 * math.pi * rng.random(n_nodes)
    m = (np.sin(th) * np.cos(ph))[:, None] * e1 + (np.sin(th) * np.sin(ph))[:, None] * e2 \
        + np.cos(th)[:, None] * n
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def cap_directions(k, centre, half_angle_rad, rng):
    """k directions uniform on the spherical cap of given half angle."""
    e1, e2, n = _orthonormal_frame(centre)
    c = rng.uniform(math.cos(half_angle_rad), 1.0, size=k)
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=k)
    d = (s * np.cos(ph))[:, None] * e1 + (s * np.sin(ph))[:, None] * e2 + c[:, None] * n
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def field_schedule(start_T, stop_T, step_T, direction):
    """Fields in Tesla (mu0*H): value * direction for values from start_T to
    stop_T (both included). A field "along -z from 0 to -8 T" is direction +z
    with values 0 .. -8."""
    n = int(round(abs(stop_T - start_T) / step_T)) + 1
    vals = np.linspace(start_T, stop_T, n)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    return vals[:, None] * d[None, :]


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

SOFT = dict(Ms=8.0e5, A=1.3e-11, K1=0.0)
HARD = dict(Ms=1.61 / MU0, A=7.7e-12, K1=4.3e6)


@dataclass
class Workload:
    name: str
    mesh: Mesh
    m0: np.ndarray          # (n_mag, 3)
    fields: np.ndarray      # (n_fields, 3) Tesla
    jmax: int
    meta: dict = field(default_factory=dict)
    theta_max: float = 0.2  # the line search's rotation cap (rad)


def soft_cube(n=10, h=4.0, seed=0, n_fields=21):
    """Soft cube (edge n*h nm), field along (0.01, 0.01, 1) from +1 T to -1 T.
    j_max = 4: the fastest of the sweep 0..1000 on this curve (as in Table 1)."""
    tilt = math.radians(1.0)
    mesh = make_box_magnet((n, n, n), h, axis=(0.0, 0.0, 1.0), **SOFT)
    rng = np.random.Generator(np.random.PCG64(seed))
    m0 = tilted_state(mesh.magnet_nodes().size, (0.0, 0.0, 1.0), 0.01, rng)
    step = 2.0 / (n_fields - 1)
    fields = field_schedule(1.0, -1.0, step, (0.01, 0.01, 1.0))
    return Workload(f"soft_cube_{n}", mesh, m0, fields, jmax=4,
                    meta=dict(seed=seed, edge_nm=n * h, tilt=tilt))


def hard_cube(n=20, h=4.0, seed=1, step_T=0.05, stop_T=-8.0):
    """Hard cube (edge n*h nm), easy axis z tilted 1 degree toward x, field
    along -z from 0 to stop_T. j_max = 1: the fastest of the sweep 0..100 on
    this curve (4 nm cells are coarser than the exchange length, so the
    exchange stiffness the preconditioner targets is weak here)."""
    u = (math.sin(math.radians(1.0)), 0.0, math.cos(math.radians(1.0)))
    mesh = make_box_magnet((n, n, n), h, axis=u, **HARD)
    rng = np.random.Generator(np.random.PCG64(seed))
    m0 = tilted_state(mesh.magnet_nodes().size, (0.0, 0.0, 1.0), 0.01, rng)
    # field along -z: h = (0, 0, B) with B from 0 down to stop_T
    fields = field_schedule(0.0, stop_T, step_T, (0.0, 0.0, 1.0))
    return Workload(f"hard_cube_{n}", mesh, m0, fields, jmax=1,
                    meta=dict(seed=seed, edge_nm=n * h))


def lex_soft():
    """Exchange length sqrt(A / Kd), Kd = mu0 Ms^2 / 2, of the soft material (nm)."""
    kd = 0.5 * MU0 * SOFT["Ms"] ** 2
    return math.sqrt(SOFT["A"] / kd) * 1e9


def sp3_cube(size_lex=8.5, n=24, start="flower", seed=5, max_tilt=0.01, pad=None):
    """Soft cube of edge size_lex exchange lengths for the single-domain limit
    in the spirit of standard problem 3 (Sec. 3.3): the soft material's Ms and
    A, uniaxial K1 = 0.1 Kd along z, n cells per edge (n = 24 gives the
    paper's mesh size of 0.35 l_ex at 8.5 l_ex), an air box padded by `pad`
    cells per side (default 3n: a 7x box, since the zero potential on a
    closer boundary understates the flower's stray-field energy), zero field.
    start='flower': saturated along +z; start='vortex': two domains, +z for
    x <= 0 and -z for x > 0, with a sharp wall. Both carry per-node tilts of
    at most max_tilt rad, which break the cube's symmetry."""
    lex = lex_soft()
    h = size_lex * lex / n
    kd = 0.5 * MU0 * SOFT["Ms"] ** 2
    p = 3 * n if pad is None else int(pad)
    mesh = make_box_magnet((n, n, n), h, SOFT["Ms"], SOFT["A"], 0.1 * kd, (0.0, 0.0, 1.0), pad=(p, p, p))
    nodes = mesh.magnet_nodes()
    rng = np.random.Generator(np.random.PCG64(seed))
    m0 = tilted_state(nodes.size, (0.0, 0.0, 1.0), max_tilt, rng)
    if start == "vortex":
        x = mesh.xyz[nodes, 0]
        m0[x > 1e-9 * h] *= np.array([1.0, 1.0, -1.0])
    elif start != "flower":
        raise ValueError(start)
    return Workload(f"sp3_{size_lex:g}lex_{start}", mesh, m0, np.zeros((1, 3)), jmax=12,
                    meta=dict(size_lex=size_lex, lex_nm=lex, h_nm=h, volume_nm3=(n * h) ** 3, kd=kd,
                              start=start, pad=p))


def batch_cubes(n_inst=64, seed=2, nmin=8, nmax=24, h=4.0, step_T=0.1, stop_T=-8.0):
    """Independent hard cubes of uneven size for a parameter study."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(nmin, nmax + 1, size=n_inst)
    K1s = rng.uniform(3.0e6, 4.9e6, size=n_inst)
    axes = cap_directions(n_inst, (0.0, 0.0, 1.0), math.radians(15.0), rng)
    out = []
    fields = field_schedule(0.0, stop_T, step_T, (0.0, 0.0, 1.0))
    for i in range(n_inst):
        mat = dict(HARD)
        mat["K1"] = float(K1s[i])
        mesh = make_box_magnet((int(sizes[i]),) * 3, h, axis=tuple(axes[i]), **mat)
        r = np.random.Generator(np.random.PCG64(2000 + i))
        m0 = tilted_state(mesh.magnet_nodes().size, (0.0, 0.0, 1.0), 0.01, r)
        out.append(Workload(f"batch_{i}_n{int(sizes[i])}", mesh, m0, fields, jmax=1,
                            meta=dict(seed=2000 + i, n=int(sizes[i]))))
    return out


FILM_THETA_MAX = 0.5  # the film's rotation cap: the fastest of 0.2, 0.35, 0.5, 0.7 and 1.0 on the whole curve


def film(nx=200, ny=200, nz=2, h=5.0, seed=3, step_T=0.001, start_T=0.05):
    """Soft thin film, field along x from +start_T to -start_T. j_max = 10: the
    fastest of 1, 10, 20 on the whole curve (and of 0, 1, 4, 10 on its first
    10 fields). Rotation cap FILM_THETA_MAX."""
    mesh = make_box_magnet((nx, ny, nz), h, axis=(1.0, 0.0, 0.0), **SOFT)
    rng = np.random.Generator(np.random.PCG64(seed))
    m0 = tilted_state(mesh.magnet_nodes().size, (1.0, 0.0, 0.0), 0.01, rng)
    fields = field_schedule(start_T, -start_T, step_T, (1.0, 0.0, 0.0))
    return Workload(f"film_{nx}x{ny}x{nz}", mesh, m0, fields, jmax=10,
                    meta=dict(seed=seed), theta_max=FILM_THETA_MAX)


def training_film(seed, h=5.0, lo=600.0, hi=1400.0, nz=2):
    """Film with side lengths drawn uniformly in [lo, hi] nm (rounded to h)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lx, Ly = rng.uniform(lo, hi, size=2)
    nx = max(1, int(round(Lx / h)))
    ny = max(1, int(round(Ly / h)))
    return film(nx=nx, ny=ny, nz=nz, h=h, seed=seed)


def polycrystal(n=96, edge=200.0, n_grains=27, seed=4, gb_width=2.0, step_T=0.05, stop_T=-6.0):
    """Voronoi polycrystal cube: each tet goes to the nearest of n_grains
    seeds (by centroid); tets whose centroid lies within gb_width nm of a
    Voronoi bisector form a grain-boundary phase (K1 = 0, A = 1e-12 J/m)."""
    h = edge / n
    xyz, tets, cell, mag, nb, padv = box_mesh((n, n, n), h)
    rng = np.random.Generator(np.random.PCG64(seed))
    seeds = rng.uniform(-edge / 2, edge / 2, size=(n_grains, 3))
    axes = cap_directions(n_grains, (0.0, 0.0, 1.0), math.radians(20.0), rng)
    nt = tets.shape[0]
    region = np.zeros(nt, dtype=np.int32)
    Ms_t = np.zeros(nt)
    A_t = np.zeros(nt)
    K_t = np.zeros(nt)
    ax = np.zeros((nt, 3))
    ax[:, 2] = 1.0
    idx = np.nonzero(mag)[0]
    cen = xyz[tets[idx]].mean(axis=1)
    # nearest seed (lowest index on ties) and distance to the nearest bisector
    d2 = ((cen[:, None, :] - seeds[None, :, :]) ** 2).sum(axis=2)
    g = np.argmin(d2, axis=1)
    di = d2[np.arange(idx.size), g]
    pg = seeds[g]
    sep = np.linalg.norm(seeds[None, :, :] - pg[:, None, :], axis=2)
    with np.errstate(divide="ignore", invalid="ignore"):
        bis = (d2 - di[:, None]) / (2.0 * sep)
    bis[np.arange(idx.size), g] = np.inf
    gb = bis.min(axis=1) < gb_width
    region[idx] = np.where(gb, n_grains + 1, g + 1)
    Ms_t[idx] = HARD["Ms"]
    A_t[idx] = np.where(gb, 1.0e-12, HARD["A"])
    K_t[idx] = np.where(gb, 0.0, HARD["K1"])
    ax[idx] = axes[g]
    mesh = Mesh(xyz, tets, region, Ms_t, A_t, K_t, ax, shape=nb,
                mag_cells=tuple((padv[i], padv[i] + n) for i in range(3)), h=h,
                meta=dict(seeds=seeds, axes=axes))
    m0 = tilted_state(mesh.magnet_nodes().size, (0.0, 0.0, 1.0), 0.01,
                      np.random.Generator(np.random.PCG64(seed + 1000)))
    fields = field_schedule(0.0, stop_T, step_T, (0.0, 0.0, 1.0))
    # j_max = 4: the fastest of 0, 1, 4, 10 on the first two fields
    return Workload(f"polycrystal_{n}", mesh, m0, fields, jmax=4, meta=dict(seed=seed))


def small_box(ncell=(3, 2, 2), h=4.0, Ms=8.0e5, A=1.3e-11, K1=0.0, axis=(0, 0, 1),
              air=True, pad=None):
    """Tiny meshes for unit tests."""
    return make_box_magnet(ncell, h, Ms, A, K1, axis, air=air, pad=pad)


def random_unit(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_vec(n, seed, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal((n, 3))


CONFIGS = {
    0: soft_cube,
    1: hard_cube,
    3: film,
    4: polycrystal,
}


# ---------------------------------------------------------------------------
# learned component: seeded parameters, probes and training films
# ---------------------------------------------------------------------------

GNN_F_IN, GNN_WIDTH, GNN_LAYERS, GNN_E_DIM = 32, 64, 3, 4


def gnn_param_shapes():
    """Flat parameter layout of the graph network (row-major [in][out])."""
    shp = [("W_in", (GNN_F_IN, GNN_WIDTH)), ("b_in", (GNN_WIDTH,))]
    for l in range(GNN_LAYERS):
        shp += [(f"We1_{l}", (GNN_WIDTH, GNN_WIDTH)), (f"We2_{l}", (GNN_E_DIM, GNN_WIDTH)),
                (f"W1_{l}", (2 * GNN_WIDTH, GNN_WIDTH)), (f"b1_{l}", (GNN_WIDTH,)),
                (f"W2_{l}", (GNN_WIDTH, GNN_WIDTH)), (f"b2_{l}", (GNN_WIDTH,))]
    shp += [("Wm", (GNN_WIDTH, 3)), ("bm", (3,)), ("Ws", (GNN_WIDTH, 1)), ("bs", (1,))]
    return shp


def gnn_init(seed, head_scale=0.01):
    """Uniform(-r, r) weights with r = sqrt(6 / (fan_in + fan_out)), zero
    biases; the residual branches' last matrices and the heads scaled down so
    that the untrained network starts near dm = 0, s = softplus(0) + 1/4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for name, s in gnn_param_shapes():
        if len(s) == 1:
            out.append(np.zeros(s))
            continue
        r = math.sqrt(6.0 / (s[0] + s[1]))
        w = rng.uniform(-r, r, size=s)
        if name.startswith("W2_"):
            w *= 0.1
        if name in ("Wm", "Ws"):
            w *= head_scale
        out.append(w)
    return np.concatenate([w.ravel() for w in out])


def rademacher(n_probe, n_rows, seed):
    """Probe vectors with independent +-1 entries, shape (n_probe, n_rows, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 2, size=(n_probe, n_rows, 3)).astype(np.float64) * 2.0 - 1.0


def small_film(seed, lo=120.0, hi=280.0, h=5.0, nz=2, step_T=0.001, start_T=0.05):
    """Training-size soft film: side lengths uniform in [lo, hi] nm (cells of
    h nm, nz cells thick), field along x from +start_T to -start_T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lx, Ly = rng.uniform(lo, hi, size=2)
    nx = max(2, int(round(Lx / h)))
    ny = max(2, int(round(Ly / h)))
    return film(nx=nx, ny=ny, nz=nz, h=h, seed=seed, step_T=step_T, start_T=start_T)
