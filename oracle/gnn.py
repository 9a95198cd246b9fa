"""FP64 oracle of the learned component (test infrastructure only).

Not part of the paper's method: a per-node graph network on the magnet nodes
of the mesh proposes, for the step from the minimizer m_k at field h_k to the
next field h_{k+1}, a tangent update dm (the start of the next minimization is
N(m_k + dm)) and a positive factor s per node that scales the Jacobi diagonal
of the preconditioner's inner CG. This module writes out its definitions
plainly in numpy FP64: graph, node features, forward pass, loss, backward pass
(checked against finite differences in the tests), Adam, and the Hutchinson
estimate of the diagonal of the magnetostatic Hessian block that provides the
scaling targets. Only tests/, smoke() and bench.py's CPU leg use it.

Network (widths fixed):
  h0 = SiLU(X W_in + b_in)                                  X: n x 32 features
  for l = 0, 1, 2:
      a = A h_l                     A: mean over the mesh neighbours
      q = a We1_l + ebar We2_l      ebar: mean edge features (n x 4)
      t = SiLU([h_l | q] W1_l + b1_l)
      h_{l+1} = h_l + t W2_l + b2_l
  dm = P_m (h3 Wm + bm),  P_m v = v - (v.m) m
  s  = clip(softplus(h3 Ws + bs) + 1/4, 1/4, 4)
Loss: inv_dm2 * sum_a L_a |dm_a - dm*_a|^2 / sum_a L_a
      + w_s * mean_a (log s_a - log s*_a)^2.
The GPU computes the products with W_in, We1, W1, W2 (forward and backward)
on BF16 operands with FP32 accumulation; `emulate_bf16=True` rounds the same
operands here (round to nearest even) so the two can be compared closely.
"""
from __future__ import annotations

import numpy as np

F_IN = 32
WIDTH = 64
N_LAYERS = 3
E_DIM = 4


def param_shapes():
    """Flat parameter layout (row-major [in][out] matrices), in order."""
    shp = [("W_in", (F_IN, WIDTH)), ("b_in", (WIDTH,))]
    for l in range(N_LAYERS):
        shp += [(f"We1_{l}", (WIDTH, WIDTH)), (f"We2_{l}", (E_DIM, WIDTH)),
                (f"W1_{l}", (2 * WIDTH, WIDTH)), (f"b1_{l}", (WIDTH,)),
                (f"W2_{l}", (WIDTH, WIDTH)), (f"b2_{l}", (WIDTH,))]
    shp += [("Wm", (WIDTH, 3)), ("bm", (3,)), ("Ws", (WIDTH, 1)), ("bs", (1,))]
    return shp


def n_params():
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, s in param_shapes():
        k = int(np.prod(s))
        out[name] = theta[o:o + k].reshape(s)
        o += k
    assert o == theta.size
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in param_shapes()])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even); FP64 result."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(a, w, emulate):
    if emulate:
        return bf16(a) @ bf16(w)
    return a @ w


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def silu(x):
    return x * sigmoid(x)


def dsilu(x):
    s = sigmoid(x)
    return s * (1.0 + x * (1.0 - s))


def softplus(x):
    return np.logaddexp(0.0, x)


# ---------------------------------------------------------------------------
# graph and features
# ---------------------------------------------------------------------------

class Graph:
    """Magnet nodes of a mesh; i ~ j when i != j share a tet with region > 0."""

    def __init__(self, mesh):
        nodes = mesh.magnet_nodes()
        n = nodes.size
        local = -np.ones(mesh.n_nodes, dtype=np.int64)
        local[nodes] = np.arange(n)
        T = local[mesh.tets[mesh.region > 0]]
        pairs = set()
        for t in T:
            for a in range(4):
                for b in range(4):
                    if a != b:
                        pairs.add((int(t[a]), int(t[b])))
        P = np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)
        self.n = n
        self.ptr = np.zeros(n + 1, dtype=np.int64)
        np.add.at(self.ptr, P[:, 0] + 1, 1)
        self.ptr = np.cumsum(self.ptr)
        self.idx = P[:, 1].copy()          # sorted by (row, col)
        self.deg = np.diff(self.ptr).astype(np.float64)
        x = mesh.xyz[nodes]
        d = x[P[:, 1]] - x[P[:, 0]]
        ln = np.linalg.norm(d, axis=1)
        self.ell = float(ln.mean())
        e = np.concatenate([d / self.ell, (ln / self.ell)[:, None]], axis=1)
        self.ebar = np.zeros((n, E_DIM))
        np.add.at(self.ebar, P[:, 0], e)
        self.ebar /= self.deg[:, None]
        self.max_deg = float(self.deg.max())

    def mean(self, h):
        """(A h)_i = mean of h_j over the neighbours j of i."""
        out = np.zeros_like(h)
        for i in range(self.n):
            out[i] = h[self.idx[self.ptr[i]:self.ptr[i + 1]]].mean(axis=0)
        return out

    def mean_T(self, g):
        """A^T g: (A^T g)_j = sum over i with j ~ i of g_i / deg_i."""
        out = np.zeros_like(g)
        for i in range(self.n):
            nb = self.idx[self.ptr[i]:self.ptr[i + 1]]
            out[nb] += g[i] / self.deg[i]
        return out


def features(o, graph, m, h_prev_T, h_next_T):
    """Node inputs for the step (m_k, h_k -> h_{k+1}); o is an oracle.Oracle
    of the same mesh. Columns: 0-2 m; 3-5 h_next; 6-8 h_next - h_prev
    (reduced units); 9-11 -(C m)_a / L_a; 12-14 -(B^T u)_a / L_a (stray
    field part of the gradient); 15-17 -g_a / L_a (projected gradient); 18
    D_a / mean D (exchange diagonal); 19 L_a / mean L; 20 deg_a / max deg;
    21-31 zero. Fields and gradients at (m_k, h_next), all energy terms."""
    m = np.asarray(m, dtype=np.float64).reshape(-1, 3)
    hn = o.reduce_field(np.asarray(h_next_T, dtype=np.float64))
    hp = o.reduce_field(np.asarray(h_prev_T, dtype=np.float64))
    r = o.eval(m, hn)
    L = o.lumped()
    D = o.jacobi_diag()
    Cm = o.apply_C(m)
    Gd = r["G"] - Cm + L[:, None] * hn[None, :]
    X = np.zeros((m.shape[0], F_IN))
    X[:, 0:3] = m
    X[:, 3:6] = hn
    X[:, 6:9] = hn - hp
    X[:, 9:12] = -Cm / L[:, None]
    X[:, 12:15] = -Gd / L[:, None]
    X[:, 15:18] = -r["g"] / L[:, None]
    X[:, 18] = D / D.mean()
    X[:, 19] = L / L.mean()
    X[:, 20] = graph.deg / graph.max_deg
    return X


def dm_target(m_k, m_next):
    """Tangent part of the step to the next minimizer: P_{m_k}(m_{k+1} - m_k)."""
    d = np.asarray(m_next, dtype=np.float64) - np.asarray(m_k, dtype=np.float64)
    return d - (d * m_k).sum(axis=1, keepdims=True) * m_k


def demag_diag(o, probes):
    """Hutchinson estimate of the diagonal of the magnetostatic Hessian block
    M = B^T K^-1 B (3n x 3n): mean over probes z of z * (M z)."""
    acc = np.zeros_like(np.asarray(probes[0], dtype=np.float64))
    for z in probes:
        u = o.poisson(o.bmul(z), rtol=1e-12)[0]
        acc += z * o.btmul(u)
    return acc / len(probes)


def s_target(diag3, m, D):
    """1 + t_a / D_a with t_a the mean of the diagonal of M over the two
    directions normal to m_a: (sum_c d_ac - sum_c m_ac^2 d_ac) / 2."""
    t = 0.5 * (diag3.sum(axis=1) - (m * m * diag3).sum(axis=1))
    return 1.0 + t / D


# ---------------------------------------------------------------------------
# forward / loss / backward
# ---------------------------------------------------------------------------

def forward(theta, X, graph, m, emulate_bf16=False):
    p = unpack(theta)
    em = emulate_bf16
    c = {"X": X, "m": m}
    y0 = _mm(X, p["W_in"], em) + p["b_in"]
    h = silu(y0)
    c["y0"] = y0
    c["h"] = [h]
    c["a"], c["q"], c["y1"], c["t"] = [], [], [], []
    for l in range(N_LAYERS):
        a = graph.mean(h)
        q = _mm(a, p[f"We1_{l}"], em) + graph.ebar @ p[f"We2_{l}"]
        z = np.concatenate([h, q], axis=1)
        y1 = _mm(z, p[f"W1_{l}"], em) + p[f"b1_{l}"]
        t = silu(y1)
        h = h + _mm(t, p[f"W2_{l}"], em) + p[f"b2_{l}"]
        for k, v in (("a", a), ("q", q), ("y1", y1), ("t", t)):
            c[k].append(v)
        c["h"].append(h)
    zm = h @ p["Wm"] + p["bm"]
    dm = zm - (zm * m).sum(axis=1, keepdims=True) * m
    zs = (h @ p["Ws"] + p["bs"])[:, 0]
    sp = softplus(zs) + 0.25
    s = np.clip(sp, 0.25, 4.0)
    c.update(zm=zm, zs=zs, sp=sp)
    return dm, s, c


def loss(dm, s, dm_t, s_t, L, inv_dm2, w_s):
    e = dm - dm_t
    lw = inv_dm2 * float((L * (e * e).sum(axis=1)).sum() / L.sum())
    ls = w_s * float(((np.log(s) - np.log(s_t)) ** 2).mean())
    return lw + ls


def backward(theta, c, graph, dm_t, s_t, L, inv_dm2, w_s, emulate_bf16=False):
    """Loss and its gradient with respect to the flat parameters."""
    p = unpack(theta)
    em = emulate_bf16
    g = {k: np.zeros_like(v) for k, v in p.items()}
    m = c["m"]
    zm = c["zm"]
    dm = zm - (zm * m).sum(axis=1, keepdims=True) * m
    sp = c["sp"]
    s = np.clip(sp, 0.25, 4.0)
    n = m.shape[0]
    val = loss(dm, s, dm_t, s_t, L, inv_dm2, w_s)
    # heads
    d_dm = inv_dm2 * 2.0 * L[:, None] * (dm - dm_t) / L.sum()
    d_zm = d_dm - (d_dm * m).sum(axis=1, keepdims=True) * m
    d_s = w_s * 2.0 * (np.log(s) - np.log(s_t)) / (n * s)
    inside = (sp > 0.25) & (sp < 4.0)
    d_zs = d_s * sigmoid(c["zs"]) * inside
    h3 = c["h"][-1]
    g["Wm"] = h3.T @ d_zm
    g["bm"] = d_zm.sum(axis=0)
    g["Ws"] = h3.T @ d_zs[:, None]
    g["bs"] = np.array([d_zs.sum()])
    dh = d_zm @ p["Wm"].T + d_zs[:, None] @ p["Ws"].T
    for l in reversed(range(N_LAYERS)):
        h, a, q, y1, t = c["h"][l], c["a"][l], c["q"][l], c["y1"][l], c["t"][l]
        z = np.concatenate([h, q], axis=1)
        g[f"W2_{l}"] = _mm(t.T, dh, em)
        g[f"b2_{l}"] = dh.sum(axis=0)
        dt = _mm(dh, p[f"W2_{l}"].T, em)
        dy1 = dt * dsilu(y1)
        g[f"W1_{l}"] = _mm(z.T, dy1, em)
        g[f"b1_{l}"] = dy1.sum(axis=0)
        dz = _mm(dy1, p[f"W1_{l}"].T, em)
        dq = dz[:, WIDTH:]
        g[f"We1_{l}"] = _mm(a.T, dq, em)
        g[f"We2_{l}"] = graph.ebar.T @ dq
        da = _mm(dq, p[f"We1_{l}"].T, em)
        dh = dh + dz[:, :WIDTH] + graph.mean_T(da)
    dy0 = dh * dsilu(c["y0"])
    g["W_in"] = _mm(c["X"].T, dy0, em)
    g["b_in"] = dy0.sum(axis=0)
    return val, pack(g)


class Adam:
    """Adam with bias correction (Kingma and Ba)."""

    def __init__(self, n, b1=0.9, b2=0.999, eps=1e-8):
        self.m1 = np.zeros(n)
        self.m2 = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, theta, grad, lr):
        self.t += 1
        self.m1 = self.b1 * self.m1 + (1 - self.b1) * grad
        self.m2 = self.b2 * self.m2 + (1 - self.b2) * grad * grad
        mh = self.m1 / (1 - self.b1 ** self.t)
        vh = self.m2 / (1 - self.b2 ** self.t)
        return theta - lr * mh / (np.sqrt(vh) + self.eps)
