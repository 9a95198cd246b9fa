"""ctypes binding of libmmncg.so (the C ABI declared in include/mmncg.h).

Argument marshalling only: every step of the method runs in the HIP library.
Vectors may be numpy arrays (host) or torch tensors on the context's GPU
(device pointers are passed straight through). PyTorch supplies device memory
(its caching allocator, through the ABI's allocator callbacks) and the stream.
The library is loaded on first use, after torch (whose HIP runtime must be in
the process first). If it is missing, that first use raises ImportError: there
is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import re
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmncg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mmncg.h")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_EMESH, MM_ESTATE = 0, -1, -2, -3, -4, -5
MM_NOT_CONVERGED, MM_STALLED, MM_NONFINITE = 1, 2, 3
MM_FP64, MM_FP32_BULK = 0, 1
MM_PREC_JACOBI, MM_PREC_AMG = 0, 1
MM_BETA_ZA, MM_BETA_FR, MM_BETA_PRP, MM_BETA_HS = 0, 1, 2, 3
MM_PFORM_PAPER, MM_PFORM_FULL, MM_PFORM_LOCAL = 0, 1, 2
MM_STOP_TORQUE, MM_STOP_PAPER = 0, 1
MM_T_EXCH, MM_T_ANIS, MM_T_ZEE, MM_T_DEMAG, MM_T_ALL = 1, 2, 4, 8, 15
MM_OP_C, MM_OP_B, MM_OP_BT, MM_OP_K = 0, 1, 2, 3
MM_TUNE_DEFAULT, MM_TUNE_MEASURE, MM_TUNE_CACHE = 0, 1, 2
MM_LEARN_START, MM_LEARN_SCALE = 1, 2
MM_GNN_BF16, MM_GNN_FP32 = 0, 1


class MMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mmncg error {code}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("jmax", C.c_int), ("tol_torque", C.c_double), ("stop_mode", C.c_int), ("tau_F", C.c_double),
                ("theta_max", C.c_double), ("theta_init", C.c_double), ("c1", C.c_double), ("c2", C.c_double),
                ("poisson_rtol", C.c_double), ("max_nli", C.c_long), ("precision", C.c_int), ("terms", C.c_int),
                ("ls_max_halvings", C.c_int), ("poisson_maxit", C.c_long), ("poisson_prec", C.c_int),
                ("beta", C.c_int), ("prec_form", C.c_int), ("theta_adapt", C.c_int), ("theta_hi", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("evals", C.c_long), ("nli", C.c_long), ("li", C.c_long), ("mi", C.c_long),
                ("restarts", C.c_long), ("fallbacks", C.c_long), ("t_nl", C.c_double), ("t_lin", C.c_double),
                ("t_mag", C.c_double), ("F", C.c_double), ("torque_max", C.c_double), ("status", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("n_nodes", C.c_long), ("n_tets", C.c_long), ("n_mag", C.c_long), ("n_pot", C.c_long),
                ("nnz_C_blocks", C.c_long), ("nnz_K", C.c_long), ("nnz_B", C.c_long), ("Ms_ref", C.c_double),
                ("device_bytes", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_vp = C.c_void_p


def header_symbols():
    """Names of the functions the public header declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|long|const char \*)\s*(mm_\w+)\s*\(", txt, re.M)))


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libmmncg.so not built ({path}); run __graft_entry__.build()")
    # torch ships a HIP runtime of its own; it has to be in the process before
    # the library pulls in the system one, so that both sit on the HSA runtime
    # torch brought (the other order leaves hipGetDeviceCount failing)
    import torch  # noqa: F401
    L = C.CDLL(path)
    L.mm_opts_default.argtypes = [C.POINTER(Opts)]
    L.mm_amg_info.argtypes = [_vp, C.POINTER(C.c_int), _vp, _vp, _vp, C.POINTER(C.c_double)]
    L.mm_amg_aggregates.argtypes = [_vp, C.c_int, _vp]
    L.mm_amg_level_matrix.argtypes = [_vp, C.c_int, C.c_int, _vp, _vp, _vp]
    L.mm_amg_apply.argtypes = [_vp, _vp, _vp, C.c_int]
    L.mm_create.argtypes = [C.POINTER(_vp), C.c_int, _vp, ALLOC_FN, FREE_FN, _vp]
    L.mm_destroy.argtypes = [_vp]
    L.mm_last_error.restype = C.c_char_p
    L.mm_last_error.argtypes = [_vp]
    L.mm_get_info.argtypes = [_vp, C.POINTER(Info)]
    L.mm_mesh_upload.argtypes = [_vp, _dp, C.c_long, _ip, C.c_long, _ip]
    L.mm_material_set.argtypes = [_vp, _dp, _dp, _dp, _dp]
    L.mm_magnet_nodes.argtypes = [_vp, C.POINTER(C.c_long), _ip]
    L.mm_set_opts.argtypes = [_vp, C.POINTER(Opts)]
    L.mm_reset_warm_start.argtypes = [_vp]
    L.mm_energy_grad.argtypes = [_vp, _vp, _dp, _dp, _vp, _vp, _dp]
    L.mm_precondition.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _vp, _vp, _ip]
    L.mm_precondition_noalloc.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _vp, _vp, _ip]
    L.mm_ncg_minimize.argtypes = [_vp, _vp, _dp, C.POINTER(Opts), C.POINTER(Stats), _dp]
    L.mm_demag_curve.argtypes = [_vp, _vp, _dp, C.c_long, C.POINTER(Opts), _dp, _dp, C.POINTER(Stats), _vp]
    L.mm_operator_apply.argtypes = [_vp, C.c_int, _vp, _vp]
    L.mm_poisson_solve.argtypes = [_vp, _vp, _vp, C.c_double, C.POINTER(C.c_long)]
    L.mm_profile.argtypes = [_vp, C.c_int, _dp]
    L.mm_profile_kernels.argtypes = [_vp, C.c_int, _dp]
    _lp = C.POINTER(C.c_long)
    L.mm_batch_upload.argtypes = [_vp, C.c_int, _lp, _lp, _dp, _ip, _ip, _dp, _dp, _dp, _dp]
    L.mm_batch_size.argtypes = [_vp, _ip]
    L.mm_batch_info.argtypes = [_vp, C.c_int, C.POINTER(Info)]
    L.mm_batch_magnet_nodes.argtypes = [_vp, C.c_int, _lp, _ip]
    L.mm_batch_energy_grad.argtypes = [_vp, _vp, _dp, _dp, _vp, _vp, _dp]
    L.mm_tune.argtypes = [_vp, C.c_int, C.c_char_p, _ip, _ip, _ip]
    _fp = C.POINTER(C.c_float)
    L.mm_gnn_param_count.restype = C.c_long
    L.mm_gnn_param_count.argtypes = []
    L.mm_gnn_create.argtypes = [_vp, C.POINTER(_vp)]
    L.mm_gnn_destroy.argtypes = [_vp]
    L.mm_gnn_last_error.restype = C.c_char_p
    L.mm_gnn_last_error.argtypes = [_vp]
    L.mm_gnn_set_params.argtypes = [_vp, _vp]
    L.mm_gnn_get_params.argtypes = [_vp, _vp]
    L.mm_gnn_set_input_norm.argtypes = [_vp, _dp, _dp]
    L.mm_graph_create.argtypes = [_vp, C.POINTER(_vp)]
    L.mm_graph_destroy.argtypes = [_vp]
    L.mm_graph_size.argtypes = [_vp, _lp, _lp]
    L.mm_gnn_features.argtypes = [_vp, _vp, _dp, _dp, _vp]
    L.mm_gnn_forward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.mm_gnn_loss_grad.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_double, C.c_double, _dp, _vp]
    L.mm_gnn_train.argtypes = [_vp, C.c_long, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp),
                               C.POINTER(_vp), _dp, C.c_double, C.c_int, C.c_double, C.c_ulonglong, _dp]
    L.mm_gnn_save.argtypes = [_vp, C.c_char_p]
    L.mm_gnn_load.argtypes = [_vp, C.c_char_p]
    L.mm_gnn_targets.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.mm_gnn_moments.argtypes = [_vp, _vp, _dp, _dp]
    L.mm_gnn_adam.argtypes = [_vp, C.c_double, C.c_double, C.c_double, C.c_double]
    L.mm_gnn_set_precision.argtypes = [_vp, C.c_int]
    L.mm_demag_diag.argtypes = [_vp, _vp, C.c_int, C.c_double, _vp]
    L.mm_jacobi_diag.argtypes = [_vp, _vp]
    L.mm_demag_curve_learned.argtypes = [_vp, _vp, _vp, C.c_int, _vp, _dp, _dp, C.c_long, C.POINTER(Opts), _dp,
                                         _dp, C.POINTER(Stats), _ip]
    L.mm_batch_demag_curve.argtypes = [_vp, _vp, _dp, C.c_long, C.POINTER(Opts), _dp, _dp, C.POINTER(Stats)]
    for name in header_symbols():
        if name not in ("mm_last_error", "mm_gnn_last_error", "mm_gnn_param_count"):
            getattr(L, name).restype = C.c_int
    return L


_LIB = None
_LIVE = weakref.WeakSet()


_LIVE_NETS = weakref.WeakSet()


@atexit.register
def _close_all():
    # release device memory through the allocator callbacks while torch is
    # alive: networks and graphs first, then the contexts
    for net in list(_LIVE_NETS):
        try:
            net.close()
        except Exception:
            pass
    for ctx in list(_LIVE):
        try:
            ctx.close()
        except Exception:
            pass


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def default_opts(**kw):
    o = Opts()
    lib().mm_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _host_f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _vec_ptr(x, dtype=np.float64):
    """Pointer for a vector argument: torch CUDA tensor -> its device pointer,
    anything else -> contiguous numpy array of `dtype` on the host. Work
    queued by torch on its current stream is waited for first (the library
    may run on a stream of its own)."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            want = torch.float64 if dtype == np.float64 else torch.float32
            if x.dtype != want or not x.is_contiguous():
                raise TypeError(f"device vectors must be contiguous {want} tensors")
            if x.is_cuda:
                torch.cuda.current_stream(x.device).synchronize()
            return C.c_void_p(x.data_ptr()), x
    except ImportError:
        pass
    a = np.ascontiguousarray(x, dtype=dtype)
    return C.c_void_p(a.ctypes.data), a


class Context:
    """One mmncg context (device memory, stream, discretized problem)."""

    def __init__(self, device=0, stream=None, torch_allocator=True):
        self._L = lib()
        self.device = device
        self._alloc_cb = ALLOC_FN()
        self._free_cb = FREE_FN()
        sp = None
        if torch_allocator or stream is not None:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            sp = C.c_void_p(stream.cuda_stream)
            self._torch_stream = stream
            if torch_allocator:
                dev = device

                def _alloc(nbytes, user):
                    try:
                        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
                    except Exception:
                        return None

                def _free(ptr, user):
                    try:
                        torch.cuda.caching_allocator_delete(ptr)
                    except Exception:
                        pass

                self._alloc_cb = ALLOC_FN(_alloc)
                self._free_cb = FREE_FN(_free)
        h = C.c_void_p()
        rc = self._L.mm_create(C.byref(h), device, sp, self._alloc_cb, self._free_cb, None)
        if rc != MM_OK:
            raise MMError(rc, "mm_create failed")
        self.h = h
        self.last_rc = 0
        self.n_mag = 0
        self.n_pot = 0
        _LIVE.add(self)

    def close(self):
        if getattr(self, "h", None):
            self._L.mm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_warn=True):
        if rc < 0 or (rc > 0 and not allow_warn):
            raise MMError(rc, self._L.mm_last_error(self.h).decode())
        return rc

    # ----------------------------------------------------------------
    def upload(self, mesh):
        xyz = _host_f64(mesh.xyz)
        tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
        reg = np.ascontiguousarray(mesh.region, dtype=np.int32)
        self._check(self._L.mm_mesh_upload(self.h, xyz.ctypes.data_as(_dp), xyz.shape[0],
                                           tets.ctypes.data_as(_ip), tets.shape[0], reg.ctypes.data_as(_ip)))
        Ms, A, K1 = _host_f64(mesh.Ms), _host_f64(mesh.A), _host_f64(mesh.K1)
        ax = _host_f64(mesh.axis)
        self._check(self._L.mm_material_set(self.h, Ms.ctypes.data_as(_dp), A.ctypes.data_as(_dp),
                                            K1.ctypes.data_as(_dp), ax.ctypes.data_as(_dp)))
        inf = self.info()
        self.n_mag, self.n_pot = inf["n_mag"], inf["n_pot"]
        self.n_inst = 1
        self.n_mag_list = [self.n_mag]
        return self

    def info(self):
        i = Info()
        self._check(self._L.mm_get_info(self.h, C.byref(i)))
        return i.as_dict()

    def magnet_nodes(self):
        n = C.c_long()
        ids = np.zeros(self.n_mag, dtype=np.int32)
        self._check(self._L.mm_magnet_nodes(self.h, C.byref(n), ids.ctypes.data_as(_ip)))
        return ids

    def set_opts(self, opts=None, **kw):
        o = opts or default_opts(**kw)
        self._check(self._L.mm_set_opts(self.h, C.byref(o)))

    def reset_warm_start(self):
        self._check(self._L.mm_reset_warm_start(self.h))

    def energy_grad(self, m, h_T):
        mp, keep = _vec_ptr(m)
        h = _host_f64(h_T, (3,))
        E = np.zeros(5)
        G = np.zeros((self.n_mag, 3))
        g = np.zeros((self.n_mag, 3))
        t = C.c_double()
        self._check(self._L.mm_energy_grad(self.h, mp, h.ctypes.data_as(_dp), E.ctypes.data_as(_dp),
                                           C.c_void_p(G.ctypes.data), C.c_void_p(g.ctypes.data), C.byref(t)))
        return dict(E=E, G=G, g=g, tmax=t.value)

    def precondition(self, m, G, g, jmax, dscale=None, noalloc=False):
        """mm_precondition, or with noalloc=True mm_precondition_noalloc
        (the inner solve's scratch in the library's static device array)."""
        mp, k1 = _vec_ptr(m)
        Gp, k2 = _vec_ptr(G)
        gp, k3 = _vec_ptr(g)
        dsp = None
        if dscale is not None:
            dsp, k4 = _vec_ptr(dscale)
        y = np.zeros((self.n_mag, 3))
        it = C.c_int()
        fn = self._L.mm_precondition_noalloc if noalloc else self._L.mm_precondition
        self._check(fn(self.h, mp, Gp, gp, int(jmax), dsp, C.c_void_p(y.ctypes.data), C.byref(it)))
        return y, it.value

    def minimize(self, m, h_T, opts=None, **kw):
        o = opts or default_opts(**kw)
        mp, keep = _vec_ptr(m)
        if keep is m and isinstance(m, np.ndarray):
            keep = m.copy()
            mp = C.c_void_p(keep.ctypes.data)
        h = _host_f64(h_T, (3,))
        st = Stats()
        E = np.zeros(5)
        rc = self._check(self._L.mm_ncg_minimize(self.h, mp, h.ctypes.data_as(_dp), C.byref(o), C.byref(st),
                                                 E.ctypes.data_as(_dp)))
        return keep, E, st.as_dict(), rc

    def curve(self, m, fields_T, opts=None, keep_hist=False, **kw):
        o = opts or default_opts(**kw)
        mp, keep = _vec_ptr(m)
        if isinstance(keep, np.ndarray):
            keep = keep.copy()
            mp = C.c_void_p(keep.ctypes.data)
        F = _host_f64(fields_T, (-1, 3))
        nf = F.shape[0]
        mavg = np.zeros((nf, 3))
        Et = np.zeros(nf)
        st = (Stats * nf)()
        hist = np.zeros((nf, self.n_mag, 3)) if keep_hist else None
        rc = self._check(self._L.mm_demag_curve(self.h, mp, F.ctypes.data_as(_dp), nf, C.byref(o),
                                                mavg.ctypes.data_as(_dp), Et.ctypes.data_as(_dp), st,
                                                None if hist is None else C.c_void_p(hist.ctypes.data)))
        return dict(m=keep, m_avg=mavg, E=Et, stats=[s.as_dict() for s in st], rc=rc, hist=hist)

    def apply(self, op, x):
        xp, keep = _vec_ptr(x)
        n_out = {MM_OP_C: 3 * self.n_mag, MM_OP_B: self.n_pot, MM_OP_BT: 3 * self.n_mag, MM_OP_K: self.n_pot}[op]
        out = np.zeros(n_out)
        self._check(self._L.mm_operator_apply(self.h, op, xp, C.c_void_p(out.ctypes.data)))
        return out.reshape(-1, 3) if op in (MM_OP_C, MM_OP_BT) else out

    def profile(self, enable):
        out = np.zeros(4)
        self._check(self._L.mm_profile(self.h, int(enable), out.ctypes.data_as(_dp)))
        it = int(out[0])
        return dict(iterations=it, seconds=float(out[1]), bytes=float(out[2]),
                    bytes_per_iteration=float(out[2]) / it if it else 0.0, rows=int(out[3]))

    def profile_kernels(self, enable):
        """Per-launch timers of the field kernels (mm_profile_kernels):
        {name: dict(launches, seconds, bytes)} for the evaluation epilogue,
        B m and the preconditioner product."""
        out = np.zeros(9)
        self._check(self._L.mm_profile_kernels(self.h, int(enable), out.ctypes.data_as(_dp)))
        names = ("k_eval_epilogue", "k_bmul", "k_prec_apply")
        return {n: dict(launches=int(out[3 * k]), seconds=float(out[3 * k + 1]), bytes=float(out[3 * k + 2]))
                for k, n in enumerate(names)}

    def tune(self, mode=MM_TUNE_MEASURE, cache_path=None):
        """Pick the block shape of the scalar-potential kernels (mm_tune)."""
        ni = max(1, getattr(self, "n_inst", 1))
        nw = C.c_int()
        spw = np.zeros(ni, dtype=np.int32)
        path = None if cache_path is None else os.fsencode(cache_path)
        bm = C.c_int()
        self._check(self._L.mm_tune(self.h, int(mode), path, C.byref(nw), spw.ctypes.data_as(_ip), C.byref(bm)))
        self.block_mult = bm.value
        return nw.value, spw

    def poisson(self, b, u0=None, rtol=1e-10):
        bp, k1 = _vec_ptr(b)
        u = np.zeros(self.n_pot) if u0 is None else _host_f64(u0).copy()
        it = C.c_long()
        self.last_rc = self._check(self._L.mm_poisson_solve(self.h, bp, C.c_void_p(u.ctypes.data), rtol,
                                                            C.byref(it)))
        return u, it.value

    # ----------------------------------------------------------------
    # batches of independent instances
    def upload_batch(self, meshes):
        """Upload several meshes (with materials) as one batch."""
        meshes = list(meshes)
        nn = np.array([m.xyz.shape[0] for m in meshes], dtype=np.int64)
        nt = np.array([m.tets.shape[0] for m in meshes], dtype=np.int64)
        xyz = _host_f64(np.concatenate([m.xyz for m in meshes]))
        tets = np.ascontiguousarray(np.concatenate([m.tets for m in meshes]), dtype=np.int32)
        reg = np.ascontiguousarray(np.concatenate([m.region for m in meshes]), dtype=np.int32)
        Ms = _host_f64(np.concatenate([m.Ms for m in meshes]))
        A = _host_f64(np.concatenate([m.A for m in meshes]))
        K1 = _host_f64(np.concatenate([m.K1 for m in meshes]))
        ax = _host_f64(np.concatenate([m.axis for m in meshes]))
        self._check(self._L.mm_batch_upload(self.h, len(meshes), nn.ctypes.data_as(C.POINTER(C.c_long)),
                                            nt.ctypes.data_as(C.POINTER(C.c_long)), xyz.ctypes.data_as(_dp),
                                            tets.ctypes.data_as(_ip), reg.ctypes.data_as(_ip),
                                            Ms.ctypes.data_as(_dp), A.ctypes.data_as(_dp),
                                            K1.ctypes.data_as(_dp), ax.ctypes.data_as(_dp)))
        self.n_inst = len(meshes)
        self.inst_info = [self.batch_info(i) for i in range(self.n_inst)]
        self.n_mag_list = [d["n_mag"] for d in self.inst_info]
        self.n_mag = int(sum(self.n_mag_list))
        self.n_pot = int(sum(d["n_pot"] for d in self.inst_info))
        return self

    def batch_size(self):
        n = C.c_int()
        self._check(self._L.mm_batch_size(self.h, C.byref(n)))
        return n.value

    def batch_info(self, i):
        inf = Info()
        self._check(self._L.mm_batch_info(self.h, int(i), C.byref(inf)))
        return inf.as_dict()

    def batch_magnet_nodes(self, i):
        n = C.c_long()
        self._check(self._L.mm_batch_magnet_nodes(self.h, int(i), C.byref(n), None))
        ids = np.zeros(n.value, dtype=np.int32)
        self._check(self._L.mm_batch_magnet_nodes(self.h, int(i), C.byref(n), ids.ctypes.data_as(_ip)))
        return ids

    def split(self, v):
        """Split a concatenated (sum n_mag, ...) array into per-instance arrays."""
        out, o = [], 0
        for n in self.n_mag_list:
            out.append(v[o:o + n])
            o += n
        return out

    def batch_energy_grad(self, m, h_T):
        mp, keep = _vec_ptr(m)
        h = _host_f64(h_T, (-1, 3))
        ni = self.n_inst
        E = np.zeros(ni)
        t = np.zeros(ni)
        G = np.zeros((self.n_mag, 3))
        g = np.zeros((self.n_mag, 3))
        self._check(self._L.mm_batch_energy_grad(self.h, mp, h.ctypes.data_as(_dp), E.ctypes.data_as(_dp),
                                                 C.c_void_p(G.ctypes.data), C.c_void_p(g.ctypes.data),
                                                 t.ctypes.data_as(_dp)))
        return dict(E=E, G=G, g=g, tmax=t)

    def batch_curve(self, m, fields_T, opts=None, **kw):
        """fields_T: (n_inst, n, 3) Tesla. Returns per-instance curves."""
        o = opts or default_opts(**kw)
        mp, keep = _vec_ptr(m)
        if isinstance(keep, np.ndarray):
            keep = keep.copy()
            mp = C.c_void_p(keep.ctypes.data)
        F = _host_f64(fields_T)
        ni = self.n_inst
        F = F.reshape(ni, -1, 3)
        nf = F.shape[1]
        mavg = np.zeros((ni, nf, 3))
        Et = np.zeros((ni, nf))
        st = (Stats * (ni * nf))()
        rc = self._check(self._L.mm_batch_demag_curve(self.h, mp, F.ctypes.data_as(_dp), nf, C.byref(o),
                                                      mavg.ctypes.data_as(_dp), Et.ctypes.data_as(_dp), st))
        stats = [[st[i * nf + k].as_dict() for k in range(nf)] for i in range(ni)]
        return dict(m=keep, m_avg=mavg, E=Et, stats=stats, rc=rc)

    # ----------------------------------------------------------------
    # learned warm start / scaling (single instance)
    def demag_diag(self, probes, rtol=1e-10):
        """Hutchinson estimate of diag(B^T K^-1 B) from probes (P, n_mag, 3)."""
        pp, keep = _vec_ptr(probes)
        P = int(np.asarray(probes.shape)[0]) if hasattr(probes, "shape") else len(probes)
        out = np.zeros((self.n_mag, 3))
        self._check(self._L.mm_demag_diag(self.h, pp, P, float(rtol), C.c_void_p(out.ctypes.data)))
        return out

    # --- multigrid preconditioner of the scalar-potential CG ---
    def amg_info(self):
        """Levels of the multigrid hierarchy (built on first use): rows and
        stored entries of each level's operator and prolongator, and the
        host seconds of the build."""
        nl = C.c_int(0)
        rows, nA, nP = (np.zeros(12, dtype=np.int64) for _ in range(3))
        sec = C.c_double(0)
        self._check(self._L.mm_amg_info(self.h, C.byref(nl), C.c_void_p(rows.ctypes.data),
                                        C.c_void_p(nA.ctypes.data), C.c_void_p(nP.ctypes.data), C.byref(sec)))
        k = nl.value
        return dict(levels=k, rows=rows[:k].tolist(), nnz_A=nA[:k].tolist(), nnz_P=nP[:k].tolist(),
                    setup_seconds=sec.value)

    def amg_aggregates(self, level):
        info = self.amg_info()
        out = np.zeros(info["rows"][level], dtype=np.int32)
        self._check(self._L.mm_amg_aggregates(self.h, int(level), C.c_void_p(out.ctypes.data)))
        return out

    def amg_level_matrix(self, level, which):
        """(ptr, col, val) of level `level`'s operator (which 0) or prolongator (1)."""
        info = self.amg_info()
        n = info["rows"][level]
        nnz = (info["nnz_A"] if which == 0 else info["nnz_P"])[level]
        ptr = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(nnz)
        self._check(self._L.mm_amg_level_matrix(self.h, int(level), int(which), C.c_void_p(ptr.ctypes.data),
                                                C.c_void_p(col.ctypes.data), C.c_void_p(val.ctypes.data)))
        return ptr, col, val

    def amg_apply(self, r, precision=MM_FP64):
        rp, keep = _vec_ptr(r)
        out = np.zeros(self.n_pot)
        self._check(self._L.mm_amg_apply(self.h, rp, C.c_void_p(out.ctypes.data), int(precision)))
        return out

    def jacobi_diag(self):
        out = np.zeros(self.n_mag)
        self._check(self._L.mm_jacobi_diag(self.h, C.c_void_p(out.ctypes.data)))
        return out

    def curve_learned(self, net, graph, mode, m, fields_T, opts=None, h_prev_T=None, **kw):
        """h_prev_T: the field (Tesla) at which m is a minimizer, when the
        call continues a curve; the first field then gets the learned
        proposal too."""
        o = opts or default_opts(**kw)
        mp, keep = _vec_ptr(m)
        if isinstance(keep, np.ndarray):
            keep = keep.copy()
            mp = C.c_void_p(keep.ctypes.data)
        F = _host_f64(fields_T, (-1, 3))
        nf = F.shape[0]
        mavg = np.zeros((nf, 3))
        Et = np.zeros(nf)
        st = (Stats * nf)()
        acc = np.zeros(nf, dtype=np.int32)
        hp = None if h_prev_T is None else _host_f64(h_prev_T, (3,))
        rc = self._check(self._L.mm_demag_curve_learned(
            self.h, net.h if net else None, graph.h if graph else None, int(mode), mp,
            None if hp is None else hp.ctypes.data_as(_dp), F.ctypes.data_as(_dp), nf,
            C.byref(o), mavg.ctypes.data_as(_dp), Et.ctypes.data_as(_dp), st, acc.ctypes.data_as(_ip)))
        return dict(m=keep, m_avg=mavg, E=Et, stats=[s.as_dict() for s in st], rc=rc, accepted=acc)


def gnn_param_count():
    return int(lib().mm_gnn_param_count())


class Graph:
    """Magnet-node graph of a single-instance context (mm_graph)."""

    def __init__(self, ctx):
        self.ctx = ctx
        self._L = ctx._L
        h = C.c_void_p()
        ctx._check(self._L.mm_graph_create(ctx.h, C.byref(h)))
        self.h = h
        n, e = C.c_long(), C.c_long()
        self._L.mm_graph_size(h, C.byref(n), C.byref(e))
        self.n, self.n_edges = n.value, e.value
        _LIVE_NETS.add(self)

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self._L.mm_graph_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def features(self, m, h_prev_T, h_next_T, out=None):
        """Node features (n x 32 float32) for (m, h_prev -> h_next)."""
        mp, keep = _vec_ptr(m)
        hp = _host_f64(h_prev_T, (3,))
        hn = _host_f64(h_next_T, (3,))
        X = np.zeros((self.n, 32), dtype=np.float32) if out is None else out
        xp, xk = _vec_ptr(X, np.float32)
        self.ctx._check(self._L.mm_gnn_features(self.h, mp, hp.ctypes.data_as(_dp), hn.ctypes.data_as(_dp), xp))
        return X

    def targets(self, m, m_next, diag3, dm_out=None, s_out=None):
        """Training targets of one field step (mm_gnn_targets): the
        tangent step dm* (n x 3) and the Jacobi factor s* (n); outputs may be
        given (numpy or device tensors)."""
        mp, k1 = _vec_ptr(m)
        np_, k2 = _vec_ptr(m_next)
        dp_, k3 = _vec_ptr(diag3)
        dm = np.zeros((self.n, 3)) if dm_out is None else dm_out
        sv = np.zeros(self.n) if s_out is None else s_out
        dmp, k4 = _vec_ptr(dm)
        svp, k5 = _vec_ptr(sv)
        self.ctx._check(self._L.mm_gnn_targets(self.h, mp, np_, dp_, dmp, svp))
        return dm, sv

    def moments(self, X):
        """Column sums and sums of squares of features X (mm_gnn_moments)."""
        xp, xk = _vec_ptr(X, np.float32)
        s1, s2 = np.zeros(32), np.zeros(32)
        self.ctx._check(self._L.mm_gnn_moments(self.h, xp, s1.ctypes.data_as(_dp), s2.ctypes.data_as(_dp)))
        return s1, s2


class Gnn:
    """Graph network of the learned warm start / scaling (mm_gnn)."""

    def __init__(self, ctx):
        self.ctx = ctx
        self._L = ctx._L
        h = C.c_void_p()
        ctx._check(self._L.mm_gnn_create(ctx.h, C.byref(h)))
        self.h = h
        self.n_params = gnn_param_count()
        _LIVE_NETS.add(self)

    def close(self):
        if getattr(self, "h", None):
            self._L.mm_gnn_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc < 0:
            raise MMError(rc, self._L.mm_gnn_last_error(self.h).decode())
        return rc

    def set_precision(self, fp32):
        """Dense layers in FP32 (debug mode) or BF16 on the matrix cores."""
        self._chk(self._L.mm_gnn_set_precision(self.h, MM_GNN_FP32 if fp32 else MM_GNN_BF16))

    def set_params(self, theta):
        tp, keep = _vec_ptr(theta)
        self._chk(self._L.mm_gnn_set_params(self.h, tp))

    def set_input_norm(self, mu, sd):
        a = _host_f64(mu, (32,))
        b = _host_f64(sd, (32,))
        self._chk(self._L.mm_gnn_set_input_norm(self.h, a.ctypes.data_as(_dp), b.ctypes.data_as(_dp)))

    def get_params(self):
        out = np.zeros(self.n_params)
        self._chk(self._L.mm_gnn_get_params(self.h, C.c_void_p(out.ctypes.data)))
        return out

    def forward(self, graph, X, m):
        xp, xk = (None, None) if X is None else _vec_ptr(X, np.float32)
        mp, mk = _vec_ptr(m)
        dm = np.zeros((graph.n, 3))
        s = np.zeros(graph.n)
        self._chk(self._L.mm_gnn_forward(self.h, graph.h, xp, mp, C.c_void_p(dm.ctypes.data),
                                         C.c_void_p(s.ctypes.data)))
        return dm, s

    def loss_grad(self, graph, X, m, dm_target, s_target, inv_dm2=1.0, w_s=1.0, want_grad=True):
        xp, xk = (None, None) if X is None else _vec_ptr(X, np.float32)
        mp, mk = _vec_ptr(m)
        tp, tk = _vec_ptr(dm_target)
        sp, sk = _vec_ptr(s_target)
        loss = C.c_double()
        grad = np.zeros(self.n_params) if want_grad else None
        self._chk(self._L.mm_gnn_loss_grad(self.h, graph.h, xp, mp, tp, sp, float(inv_dm2), float(w_s),
                                           C.byref(loss), None if grad is None else C.c_void_p(grad.ctypes.data)))
        return loss.value, grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._chk(self._L.mm_gnn_adam(self.h, float(lr), float(beta1), float(beta2), float(eps)))

    def train(self, samples, epochs, lr, w_s=1.0, seed=0):
        """mm_gnn_train over samples [(graph, X, m, dm_target, s_target,
        inv_dm2)], the arrays device tensors; returns the mean loss per
        epoch."""
        import torch
        torch.cuda.current_stream().synchronize()
        n = len(samples)
        P = C.c_void_p * n
        g = P(*[s[0].h for s in samples])
        cols = [P(*[C.c_void_p(s[q].data_ptr()) for s in samples]) for q in range(1, 5)]
        w = np.array([float(s[5]) for s in samples])
        out = np.zeros(max(epochs, 1))
        self._chk(self._L.mm_gnn_train(self.h, n, g, cols[0], cols[1], cols[2], cols[3], w.ctypes.data_as(_dp),
                                       float(w_s), int(epochs), float(lr), int(seed), out.ctypes.data_as(_dp)))
        return out[:epochs]

    def save(self, path):
        """Parameters and input standardization to a file (mm_gnn_save)."""
        self._chk(self._L.mm_gnn_save(self.h, os.fsencode(path)))

    def load(self, path):
        """Parameters and input standardization from mm_gnn_save's file."""
        self._chk(self._L.mm_gnn_load(self.h, os.fsencode(path)))
        return self
