"""CPU FP64 oracle for the micromagnetic PNCG path (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path (the HIP library and its binding) never
does. The oracle is a plain C file (`oracle.c`) built with gcc into
`liboracle.so` next to it; this module wraps it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

T_EXCH, T_ANIS, T_ZEE, T_DEMAG = 1, 2, 4, 8
T_ALL = 15


def build(force=False):
    """Compile oracle.c with gcc (FP contraction off, no fast-math)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


class Opts(C.Structure):
    _fields_ = [("jmax", C.c_int), ("tol_torque", C.c_double), ("stop_mode", C.c_int),
                ("tau_F", C.c_double), ("theta_max", C.c_double), ("theta_init", C.c_double),
                ("c1", C.c_double), ("c2", C.c_double), ("max_nli", C.c_long), ("terms", C.c_int),
                ("ls_max_halvings", C.c_int), ("beta", C.c_int), ("pform", C.c_int),
                ("theta_adapt", C.c_int), ("theta_hi", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("evals", C.c_long), ("nli", C.c_long), ("li", C.c_long), ("mi", C.c_long),
                ("restarts", C.c_long), ("fallbacks", C.c_long), ("ls_fail", C.c_long),
                ("F", C.c_double), ("tmax", C.c_double), ("status", C.c_long),
                ("max_trap_err", C.c_double), ("n_rise", C.c_long), ("max_rise", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def default_opts(jmax=4, **kw):
    o = Opts(jmax=jmax, tol_torque=1e-6, stop_mode=0, tau_F=1e-10, theta_max=0.2, theta_init=0.01,
             c1=1e-4, c2=0.1, max_nli=20000, terms=T_ALL, ls_max_halvings=20, beta=0, pform=0,
             theta_adapt=0, theta_hi=math.pi / 2)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)


def direction(kind, g1, g0, y, d, gy_prev):
    """The direction update of Alg. 4 alone (beta* of `kind` with the descent
    safeguard) on plain vectors: returns (d_new, <g, y> for the next step,
    whether the safeguard acted)."""
    L = _load()
    if not hasattr(L, "_dir_set"):
        L.or_direction_pub.restype = C.c_double
        L.or_direction_pub.argtypes = [C.c_int, C.c_long, _dp, _dp, _dp, _dp, C.c_double, _dp, _ip]
        L._dir_set = True
    g1, g0, y, d = (np.ascontiguousarray(v, dtype=np.float64).ravel() for v in (g1, g0, y, d))
    dn = np.zeros_like(g1)
    fb = C.c_int(0)
    gy = L.or_direction_pub(int(kind), g1.size, _d(g1), _d(g0), _d(y), _d(d), float(gy_prev), _d(dn),
                            C.byref(fb))
    return dn, float(gy), bool(fb.value)


def cubic_min(at, dFt, dp0, dpt):
    """The line search's interpolation step alone: the minimizer of the cubic
    through phi(0) = 0, phi'(0) = dp0, phi(at) = dFt, phi'(at) = dpt, or None
    when that cubic has no local minimizer."""
    L = _load()
    ac = np.zeros(1)
    ok = L.or_cubic_min_pub(float(at), float(dFt), float(dp0), float(dpt), _d(ac))
    return float(ac[0]) if ok else None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = C.CDLL(LIB)
    vp = C.c_void_p
    L.or_create.restype = vp
    L.or_create.argtypes = [_dp, C.c_long, _ip, C.c_long, _ip, _dp, _dp, _dp, _dp]
    L.or_destroy.argtypes = [vp]
    for name in ("or_n_mag", "or_n_pot", "or_K_nnz"):
        getattr(L, name).restype = C.c_long
        getattr(L, name).argtypes = [vp]
    L.or_ms_ref.restype = C.c_double
    L.or_ms_ref.argtypes = [vp]
    L.or_mag_nodes.argtypes = [vp, _ip]
    L.or_free_nodes.argtypes = [vp, _ip]
    L.or_lumped.argtypes = [vp, _dp]
    L.or_jacobi_diag.argtypes = [vp, _dp]
    L.or_set_poisson.argtypes = [vp, C.c_double, C.c_long]
    L.or_reset_warm.argtypes = [vp]
    L.or_get_potential.argtypes = [vp, _dp]
    L.or_set_potential.argtypes = [vp, _dp]
    L.or_counters.argtypes = [vp, _lp]
    L.or_K_csr.argtypes = [vp, _lp, _ip, _dp]
    L.or_reduce_field.argtypes = [vp, _dp, _dp]
    L.or_apply_C.argtypes = [vp, _dp, _dp, C.c_int]
    L.or_bmul.argtypes = [vp, _dp, _dp]
    L.or_btmul.argtypes = [vp, _dp, _dp]
    L.or_kmul.argtypes = [vp, _dp, _dp]
    L.or_poisson.restype = C.c_long
    L.or_poisson.argtypes = [vp, _dp, _dp, C.c_double, C.c_long]
    L.or_eval.restype = C.c_long
    L.or_eval.argtypes = [vp, _dp, _dp, C.c_int, _dp, _dp, _dp, _dp, _dp]
    L.or_apply_P.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, C.c_int, C.c_int]
    L.or_precond_pub.restype = C.c_long
    L.or_precond_pub.argtypes = [vp, _dp, _dp, _dp, C.c_int, _dp, _dp, C.c_int, C.c_int]
    L.or_minimize.restype = C.c_int
    L.or_minimize.argtypes = [vp, _dp, _dp, C.POINTER(Opts), C.POINTER(Stats), _dp]
    L.or_curve.restype = C.c_int
    L.or_curve.argtypes = [vp, _dp, _dp, C.c_long, C.POINTER(Opts), _dp, _dp, C.POINTER(Stats), _dp]
    L.or_cubic_min_pub.restype = C.c_int
    L.or_cubic_min_pub.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
    L.or_sizeof_opts.restype = C.c_long
    L.or_sizeof_stats.restype = C.c_long
    assert L.or_sizeof_opts() == C.sizeof(Opts), "oracle opts layout mismatch"
    assert L.or_sizeof_stats() == C.sizeof(Stats), "oracle stats layout mismatch"
    _lib = L
    return L


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """One discretized problem (mesh + materials) in the FP64 oracle."""

    def __init__(self, mesh, poisson_rtol=1e-10):
        L = _load()
        self._L = L
        self._keep = dict(
            xyz=_f64(mesh.xyz), tets=np.ascontiguousarray(mesh.tets, dtype=np.int32),
            region=np.ascontiguousarray(mesh.region, dtype=np.int32), Ms=_f64(mesh.Ms),
            A=_f64(mesh.A), K1=_f64(mesh.K1), axis=_f64(mesh.axis))
        k = self._keep
        self.h = L.or_create(_d(k["xyz"]), k["xyz"].shape[0], _i(k["tets"]), k["tets"].shape[0],
                             _i(k["region"]), _d(k["Ms"]), _d(k["A"]), _d(k["K1"]), _d(k["axis"]))
        if not self.h:
            raise ValueError("oracle: bad mesh or material")
        self.nm = L.or_n_mag(self.h)
        self.np = L.or_n_pot(self.h)
        self.ms_ref = L.or_ms_ref(self.h)
        self.set_poisson(poisson_rtol)

    def __del__(self):
        try:
            if self.h:
                self._L.or_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # --- bookkeeping --------------------------------------------------
    def set_poisson(self, rtol, maxit=100000):
        self._L.or_set_poisson(self.h, rtol, maxit)

    def reset_warm(self):
        self._L.or_reset_warm(self.h)

    def potential(self):
        u = np.zeros(self.np)
        self._L.or_get_potential(self.h, _d(u))
        return u

    def set_potential(self, u):
        u = _f64(u)
        self._L.or_set_potential(self.h, _d(u))

    def magnet_nodes(self):
        ids = np.zeros(self.nm, dtype=np.int32)
        self._L.or_mag_nodes(self.h, _i(ids))
        return ids

    def free_of_node(self):
        out = np.zeros(self._keep["xyz"].shape[0], dtype=np.int32)
        self._L.or_free_nodes(self.h, _i(out))
        return out

    def lumped(self):
        L = np.zeros(self.nm)
        self._L.or_lumped(self.h, _d(L))
        return L

    def jacobi_diag(self):
        D = np.zeros(self.nm)
        self._L.or_jacobi_diag(self.h, _d(D))
        return D

    def K_csr(self):
        nnz = self._L.or_K_nnz(self.h)
        p = np.zeros(self.np + 1, dtype=np.int64)
        j = np.zeros(nnz, dtype=np.int32)
        v = np.zeros(nnz)
        self._L.or_K_csr(self.h, p.ctypes.data_as(_lp), _i(j), _d(v))
        return p, j, v

    def reduce_field(self, BT):
        BT = _f64(BT, (3,))
        h = np.zeros(3)
        self._L.or_reduce_field(self.h, _d(BT), _d(h))
        return h

    # --- operators ----------------------------------------------------
    def apply_C(self, v, terms=T_EXCH | T_ANIS):
        v = _f64(v, (self.nm, 3))
        out = np.zeros_like(v)
        self._L.or_apply_C(self.h, _d(v), _d(out), terms)
        return out

    def bmul(self, m):
        m = _f64(m, (self.nm, 3))
        b = np.zeros(self.np)
        self._L.or_bmul(self.h, _d(m), _d(b))
        return b

    def btmul(self, u):
        u = _f64(u, (self.np,))
        out = np.zeros((self.nm, 3))
        self._L.or_btmul(self.h, _d(u), _d(out))
        return out

    def kmul(self, x):
        x = _f64(x, (self.np,))
        y = np.zeros(self.np)
        self._L.or_kmul(self.h, _d(x), _d(y))
        return y

    def poisson(self, b, u0=None, rtol=1e-10, maxit=100000):
        b = _f64(b, (self.np,))
        u = np.zeros(self.np) if u0 is None else _f64(u0, (self.np,)).copy()
        it = self._L.or_poisson(self.h, _d(b), _d(u), rtol, maxit)
        return u, it

    def eval(self, m, h_red, terms=T_ALL):
        """Energy parts (ex, an, zee, demag, total), gradient G, projected g,
        lambda, max torque, Poisson iterations. h_red is the reduced field."""
        m = _f64(m, (self.nm, 3))
        h = _f64(h_red, (3,))
        E = np.zeros(5)
        G = np.zeros((self.nm, 3))
        g = np.zeros((self.nm, 3))
        lam = np.zeros(self.nm)
        tm = np.zeros(1)
        it = self._L.or_eval(self.h, _d(m), _d(h), terms, _d(E), _d(G), _d(g), _d(lam), _d(tm))
        return dict(E=E, G=G, g=g, lam=lam, tmax=float(tm[0]), poisson_iters=int(it))

    def eval_T(self, m, BT, terms=T_ALL):
        return self.eval(m, self.reduce_field(BT), terms)

    def apply_P(self, m, lam, v, terms=T_EXCH | T_ANIS, g=None, form=0):
        """Preconditioner action of eq. (precond): form 0 without its last
        term (the paper's choice), 1 with all terms (needs the projected
        gradient g), 2 only the projected local part."""
        m = _f64(m, (self.nm, 3))
        lam = _f64(lam, (self.nm,))
        v = _f64(v, (self.nm, 3))
        gv = np.zeros_like(v) if g is None else _f64(g, (self.nm, 3))
        if form == 1 and g is None:
            raise ValueError("form 1 needs the projected gradient g")
        out = np.zeros_like(v)
        self._L.or_apply_P(self.h, _d(m), _d(lam), _d(gv), _d(v), _d(out), terms, int(form))
        return out

    def precond(self, m, lam, g, jmax, dscale=None, terms=T_EXCH | T_ANIS, form=0):
        m = _f64(m, (self.nm, 3))
        lam = _f64(lam, (self.nm,))
        g = _f64(g, (self.nm, 3))
        y = np.zeros_like(g)
        ds = None if dscale is None else _f64(dscale, (self.nm,))
        it = self._L.or_precond_pub(self.h, _d(m), _d(lam), _d(g), int(jmax),
                                    None if ds is None else _d(ds), _d(y), terms, int(form))
        return y, int(it)

    def minimize(self, m, BT, opts=None, **kw):
        opts = opts or default_opts(**kw)
        m = _f64(m, (self.nm, 3)).copy()
        h = self.reduce_field(BT)
        st = Stats()
        E = np.zeros(5)
        rc = self._L.or_minimize(self.h, _d(m), _d(h), C.byref(opts), C.byref(st), _d(E))
        return m, E, st.as_dict(), rc

    def curve(self, m, fields_T, opts=None, keep_hist=False, **kw):
        opts = opts or default_opts(**kw)
        m = _f64(m, (self.nm, 3)).copy()
        F = _f64(fields_T, (-1, 3))
        nf = F.shape[0]
        mavg = np.zeros((nf, 3))
        Et = np.zeros(nf)
        st = (Stats * nf)()
        hist = np.zeros((nf, self.nm, 3)) if keep_hist else None
        rc = self._L.or_curve(self.h, _d(m), _d(F), nf, C.byref(opts), _d(mavg), _d(Et), st,
                              None if hist is None else _d(hist))
        return dict(m=m, m_avg=mavg, E=Et, stats=[s.as_dict() for s in st], rc=rc, hist=hist)
