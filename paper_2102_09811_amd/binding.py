"""Thin ctypes binding of libheatbem.so (the C ABI declared in include/heatbem.h).

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
PyTorch supplies device memory and the current stream.  The library must be built
(``__graft_entry__.build()``); importing this module without it raises immediately.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libheatbem.so")

HB_OK, HB_EINVAL, HB_EMESH, HB_EORIENT, HB_ENOMEM, HB_EHIP, HB_ENOCONV, HB_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
HB_OP_V, HB_OP_K, HB_OP_D, HB_OP_KT, HB_OP_V11 = 1, 2, 4, 8, 16
HB_PREC_FP64, HB_PREC_MIXED = 0, 1
HB_DTYPE_F64, HB_DTYPE_F32 = 0, 1
HB_SOLVE_GMRES, HB_SOLVE_TIMEMARCH, HB_SOLVE_MIXED_IR = 0, 1, 2

EXPORTED = sorted(["hb_default_options", "hb_check_mesh", "hb_create", "hb_destroy",
                   "hb_create_nonuniform", "hb_is_nonuniform",
                   "hb_last_error", "hb_sizes", "hb_assemble", "hb_get_blocks", "hb_apply",
                   "hb_apply_noalloc",
                   "hb_rhs_dirichlet", "hb_rhs_neumann", "hb_solve", "hb_solve_neumann",
                   "hb_nearfield_pattern", "hb_assemble_nearfield",
                   "hb_eval_repr", "hb_last_assembly_ms", "hb_measure_peaks",
                   "hb_precond_pattern", "hb_precond_features", "hb_precond_spai",
                   "hb_precond_set", "hb_mlp_num_params", "hb_mlp_work_floats", "hb_mlp_forward",
                   "hb_mlp_backward", "hb_precond_loss", "hb_adam_step",
                   "hb_default_train_opts", "hb_precond_train", "hb_pcnet_create", "hb_pcnet_get",
                   "hb_pcnet_save", "hb_pcnet_load", "hb_pcnet_destroy", "hb_precond_install"])
HB_PC_SLOTS = 16
HB_PC_SLOT_FEATURES = 8
HB_PC_FEATURES = HB_PC_SLOTS * HB_PC_SLOT_FEATURES + 4


class HBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("heatbem error %d: %s" % (code, msg))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("ss_order", ctypes.c_int32), ("d_switch", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("mixed_d_min", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 12)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("precond", ctypes.c_int32), ("precond_max_iter", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]


class MLPDims(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("n_hidden", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("reserved", ctypes.c_int32 * 8)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("refinements", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


_lib = None


def lib():
    """Load libheatbem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libheatbem.so not built: run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.hb_default_options.argtypes = [ctypes.POINTER(Options)]
    L.hb_default_options.restype = None
    L.hb_check_mesh.argtypes = [vp, i64, vp, i64, vp]
    L.hb_create.argtypes = [ctypes.POINTER(vp), vp, i64, vp, i64, f64, f64, i32, ctypes.POINTER(Options)]
    L.hb_create_nonuniform.argtypes = [ctypes.POINTER(vp), vp, i64, vp, i64, f64, vp, i32,
                                       ctypes.POINTER(Options)]
    L.hb_is_nonuniform.argtypes = [vp]
    L.hb_destroy.argtypes = [vp]
    L.hb_destroy.restype = None
    L.hb_last_error.argtypes = [vp]
    L.hb_last_error.restype = ctypes.c_char_p
    L.hb_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.hb_assemble.argtypes = [vp, ctypes.c_uint32, i32, vp]
    L.hb_get_blocks.argtypes = [vp, ctypes.c_uint32, i32, i32, vp, i32, i32, vp]
    L.hb_apply.argtypes = [vp, ctypes.c_uint32, vp, vp, vp]
    L.hb_apply_noalloc.argtypes = [vp, ctypes.c_uint32, vp, vp, vp]
    L.hb_rhs_dirichlet.argtypes = [vp, vp, vp, vp]
    L.hb_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    L.hb_rhs_neumann.argtypes = [vp, vp, vp, vp]
    L.hb_nearfield_pattern.argtypes = [vp, f64, ctypes.POINTER(i64), vp, vp]
    L.hb_assemble_nearfield.argtypes = [vp, vp, vp, vp]
    L.hb_solve_neumann.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    L.hb_eval_repr.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
    L.hb_last_assembly_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.hb_measure_peaks.argtypes = [ctypes.POINTER(ctypes.c_double), vp]
    L.hb_precond_pattern.argtypes = [vp, vp, vp, vp]
    L.hb_precond_features.argtypes = [vp, vp, vp]
    L.hb_precond_spai.argtypes = [vp, vp, vp, vp, vp]
    L.hb_precond_set.argtypes = [vp, vp, vp]
    pd = ctypes.POINTER(MLPDims)
    L.hb_mlp_num_params.argtypes = [pd]
    L.hb_mlp_num_params.restype = i64
    L.hb_mlp_work_floats.argtypes = [pd, i64]
    L.hb_mlp_work_floats.restype = i64
    L.hb_mlp_forward.argtypes = [pd, vp, vp, i64, vp, vp, vp]
    L.hb_mlp_backward.argtypes = [pd, vp, vp, i64, vp, vp, vp, vp]
    L.hb_precond_loss.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.hb_adam_step.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, i32, vp]
    L.hb_default_train_opts.argtypes = [ctypes.POINTER(TrainOpts)]
    L.hb_default_train_opts.restype = None
    L.hb_precond_train.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(TrainOpts),
                                   ctypes.POINTER(vp), vp, vp]
    L.hb_pcnet_create.argtypes = [pd, vp, ctypes.POINTER(vp)]
    L.hb_pcnet_get.argtypes = [vp, pd, vp]
    L.hb_pcnet_save.argtypes = [vp, ctypes.c_char_p]
    L.hb_pcnet_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    L.hb_pcnet_destroy.argtypes = [vp]
    L.hb_pcnet_destroy.restype = None
    L.hb_precond_install.argtypes = [vp, vp, vp]
    for name in EXPORTED:
        fn = getattr(L, name)
        if fn.restype is ctypes.c_int:   # default restype
            fn.restype = ctypes.c_int
    _lib = L
    return L


def default_options(**kw):
    o = Options()
    lib().hb_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def measure_peaks(stream=None):
    """Measured vector-ALU ceilings of the current device (hb_measure_peaks): FP64 FMA TFLOP/s,
    v_rsq_f64 G/s, FP32 FMA TFLOP/s as the library is built."""
    out = (ctypes.c_double * 3)()
    rc = lib().hb_measure_peaks(out, _stream(stream))
    if rc != HB_OK:
        raise HBError(rc, "hb_measure_peaks failed")
    return {"fp64_fma_tflops": out[0], "fp64_rsq_gops": out[1], "fp32_fma_tflops": out[2]}


def _mesh_arrays(verts, tris):
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
        raise ValueError("verts must be (N, 3) float64 and tris (E, 3) int32")
    return v, t


def check_mesh(verts, tris):
    """(status code, class counts [separated, vertex, edge, identical]) -- host only, no GPU."""
    v, t = _mesh_arrays(verts, tris)
    counts = np.zeros(4, dtype=np.int64)
    rc = lib().hb_check_mesh(v.ctypes.data, len(v), t.ctypes.data, len(t), counts.ctypes.data)
    return rc, counts, lib().hb_last_error(None).decode()


def _ptr(tensor):
    import torch
    if not isinstance(tensor, torch.Tensor) or not tensor.is_cuda:
        raise TypeError("expected a device tensor")
    if not tensor.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(tensor.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class PCNet:
    """A trained learned-preconditioner network (hb_pcnet): parameters in device memory."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def create(cls, params, n_hidden):
        """From host parameters (the layout of hb_mlp_forward) of a (HB_PC_FEATURES, n_hidden,
        HB_PC_SLOTS) network."""
        d = MLPDims()
        d.n_in, d.n_hidden, d.n_out = HB_PC_FEATURES, int(n_hidden), HB_PC_SLOTS
        p = np.ascontiguousarray(params, dtype=np.float32)
        h = ctypes.c_void_p()
        rc = lib().hb_pcnet_create(ctypes.byref(d), p.ctypes.data, ctypes.byref(h))
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(None).decode())
        return cls(h)

    @classmethod
    def load(cls, path):
        h = ctypes.c_void_p()
        rc = lib().hb_pcnet_load(os.fsencode(path), ctypes.byref(h))
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(None).decode())
        return cls(h)

    def save(self, path):
        rc = lib().hb_pcnet_save(self._h, os.fsencode(path))
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(None).decode())

    def params(self):
        """(n_in, n_hidden, n_out), host float32 parameters."""
        d = MLPDims()
        rc = lib().hb_pcnet_get(self._h, ctypes.byref(d), None)
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(None).decode())
        n = lib().hb_mlp_num_params(ctypes.byref(d))
        p = np.empty(n, dtype=np.float32)
        rc = lib().hb_pcnet_get(self._h, None, p.ctypes.data)
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(None).decode())
        return (d.n_in, d.n_hidden, d.n_out), p

    def close(self):
        if getattr(self, "_h", None):
            lib().hb_pcnet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def precond_train(contexts, epochs=30, batch=2048, lr=1e-3, n_hidden=256, seed=0, stream=None):
    """hb_precond_train over the contexts (V assembled): (PCNet, per-epoch mean row losses)."""
    o = TrainOpts()
    lib().hb_default_train_opts(ctypes.byref(o))
    o.epochs, o.batch, o.lr, o.n_hidden, o.seed = int(epochs), int(batch), float(lr), int(n_hidden), int(seed)
    arr = (ctypes.c_void_p * len(contexts))(*[c._h for c in contexts])
    h = ctypes.c_void_p()
    loss = np.zeros(int(epochs), dtype=np.float32)
    rc = lib().hb_precond_train(arr, len(contexts), ctypes.byref(o), ctypes.byref(h),
                                loss.ctypes.data, _stream(stream))
    if rc != HB_OK:
        raise HBError(rc, lib().hb_last_error(contexts[0]._h).decode())
    return PCNet(h), loss.astype(np.float64).tolist()


def _info_dict(info, rc):
    return {"iterations": info.iterations, "rel_residual": info.rel_residual,
            "seconds": info.seconds, "refinements": info.refinements,
            "fallback": bool(info.fallback), "restarts": info.restarts,
            "converged": rc == HB_OK}


class Context:
    """One mesh / time grid on the current device; owns the assembled blocks."""

    def __init__(self, verts, tris, alpha, T, n_t, **opts):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("heatbem needs a HIP device")
        v, t = _mesh_arrays(verts, tris)
        self.n_tris, self.n_verts, self.n_t = len(t), len(v), int(n_t)
        self.alpha, self.T = float(alpha), float(T)
        o = default_options(**opts)
        self.storage = o.storage
        h = ctypes.c_void_p()
        rc = lib().hb_create(ctypes.byref(h), v.ctypes.data, len(v), t.ctypes.data, len(t),
                             self.alpha, self.T, self.n_t, ctypes.byref(o))
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(None).decode())
        self._h = h
        self.n_blocks = self.n_t

    def _check(self, rc):
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().hb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        a, b, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        c = ctypes.c_int32()
        self._check(lib().hb_sizes(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def assemble(self, ops=HB_OP_V | HB_OP_K, precision=HB_PREC_FP64, stream=None):
        self._check(lib().hb_assemble(self._h, ops, precision, _stream(stream)))

    def last_assembly_ms(self):
        ms = (ctypes.c_double * 3)()
        self._check(lib().hb_last_assembly_ms(self._h, ms))
        return list(ms)

    def blocks(self, op, d0=0, nd=None, dtype=None, device=True, stream=None):
        """Blocks d0 .. d0+nd-1 of op as a (nd, rows, cols) tensor (device) or ndarray (host):
        rows E_x (V, K) or N_x (D, V11), cols E_x (V) or N_x (K, D, V11)."""
        import torch
        nd = self.n_blocks - d0 if nd is None else nd
        rows = self.n_verts if op in (HB_OP_D, HB_OP_V11) else self.n_tris
        cols = self.n_tris if op == HB_OP_V else self.n_verts
        if dtype is None:
            dtype = HB_DTYPE_F32 if self.storage == HB_DTYPE_F32 else HB_DTYPE_F64
        if device:
            out = torch.empty((nd, rows, cols), dtype=torch.float64 if dtype == HB_DTYPE_F64 else torch.float32, device="cuda")
            self._check(lib().hb_get_blocks(self._h, op, d0, nd, _ptr(out), dtype, 1, _stream(stream)))
            return out
        out = np.empty((nd, rows, cols), dtype=np.float64 if dtype == HB_DTYPE_F64 else np.float32)
        self._check(lib().hb_get_blocks(self._h, op, d0, nd, ctypes.c_void_p(out.ctypes.data), dtype, 0, _stream(stream)))
        return out

    def apply(self, op, x, y=None, stream=None):
        import torch
        if y is None:
            rows = self.n_verts if op in (HB_OP_D, HB_OP_KT, HB_OP_V11) else self.n_tris
            y = torch.empty((self.n_t, rows), dtype=torch.float64, device="cuda")
        self._check(lib().hb_apply(self._h, op, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def apply_noalloc(self, op, x, y, stream=None):
        """hb_apply_noalloc: the product of apply() with the library's fixed scratch (y given)."""
        self._check(lib().hb_apply_noalloc(self._h, op, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def rhs_dirichlet(self, g, b=None, stream=None):
        import torch
        if b is None:
            b = torch.empty((self.n_t, self.n_tris), dtype=torch.float64, device="cuda")
        self._check(lib().hb_rhs_dirichlet(self._h, _ptr(g), _ptr(b), _stream(stream)))
        return b

    def nearfield_pattern(self, radius):
        """(row_start (E_x + 1,) int64, cols (nnz,) int32): near-field pairs within `radius`
        (centroid distance) plus every touching pair; kept for assemble_nearfield."""
        nnz = ctypes.c_int64()
        self._check(lib().hb_nearfield_pattern(self._h, float(radius), ctypes.byref(nnz), None, None))
        start = np.empty(self.n_tris + 1, dtype=np.int64)
        cols = np.empty(max(nnz.value, 1), dtype=np.int32)
        self._check(lib().hb_nearfield_pattern(self._h, float(radius), ctypes.byref(nnz),
                                               start.ctypes.data, cols.ctypes.data))
        self._near_nnz = nnz.value
        return start, cols[:nnz.value]

    def assemble_nearfield(self, stream=None):
        """(V (E_t, nnz), K (E_t, nnz, 3)) device float64 for the last near-field pattern."""
        import torch
        nnz = getattr(self, "_near_nnz", 0)
        V = torch.empty((self.n_t, max(nnz, 1)), dtype=torch.float64, device="cuda")
        K = torch.empty((self.n_t, max(nnz, 1), 3), dtype=torch.float64, device="cuda")
        self._check(lib().hb_assemble_nearfield(self._h, _ptr(V), _ptr(K), _stream(stream)))
        return V[:, :nnz], K[:, :nnz]

    def rhs_neumann(self, psi, b=None, stream=None):
        """b = (1/2 M_h^T - K_h^T) psi; psi: (E_t, E_x), b: (E_t, N_x)."""
        import torch
        if b is None:
            b = torch.empty((self.n_t, self.n_verts), dtype=torch.float64, device="cuda")
        self._check(lib().hb_rhs_neumann(self._h, _ptr(psi), _ptr(b), _stream(stream)))
        return b

    def solve_neumann(self, b, tol=1e-8, max_iter=500, u=None, precond=False,
                      precond_max_iter=0, stream=None):
        """D_h u = b by GMRES; b, u: (E_t, N_x); precond: the operator preconditioner
        M_h^{-1} V_h^{11} M_h^{-1} (needs HB_OP_V11 assembled)."""
        import torch
        if u is None:
            u = torch.empty((self.n_t, self.n_verts), dtype=torch.float64, device="cuda")
        o = SolveOpts()
        o.method, o.tol, o.max_iter, o.precond = HB_SOLVE_GMRES, tol, max_iter, int(bool(precond))
        o.precond_max_iter = precond_max_iter
        info = SolveInfo()
        rc = lib().hb_solve_neumann(self._h, _ptr(b), _ptr(u), ctypes.byref(o), ctypes.byref(info),
                                    _stream(stream))
        if rc not in (HB_OK, HB_ENOCONV):
            self._check(rc)
        return u, _info_dict(info, rc)

    def solve(self, b, method=HB_SOLVE_GMRES, tol=1e-8, max_iter=500, w=None, precond=False,
              precond_max_iter=0, stream=None):
        """V_h w = b; converged means ||b - V_h w|| / ||b|| <= tol recomputed in double."""
        import torch
        if w is None:
            w = torch.empty((self.n_t, self.n_tris), dtype=torch.float64, device="cuda")
        o = SolveOpts()
        o.method, o.tol, o.max_iter, o.precond = method, tol, max_iter, int(bool(precond))
        o.precond_max_iter = precond_max_iter
        info = SolveInfo()
        rc = lib().hb_solve(self._h, _ptr(b), _ptr(w), ctypes.byref(o), ctypes.byref(info), _stream(stream))
        if rc not in (HB_OK, HB_ENOCONV):
            self._check(rc)
        return w, _info_dict(info, rc)

    # ---- learned preconditioner ----
    def precond_pattern(self, stream=None):
        import torch
        cols = torch.empty((self.n_tris, HB_PC_SLOTS), dtype=torch.int32, device="cuda")
        cls = torch.empty((self.n_tris, HB_PC_SLOTS), dtype=torch.int8, device="cuda")
        self._check(lib().hb_precond_pattern(self._h, _ptr(cols), _ptr(cls), _stream(stream)))
        return cols, cls

    def precond_features(self, stream=None):
        import torch
        f = torch.empty((self.n_tris, HB_PC_FEATURES), dtype=torch.float32, device="cuda")
        self._check(lib().hb_precond_features(self._h, _ptr(f), _stream(stream)))
        return f

    def precond_spai(self, exact=True, stream=None):
        import torch
        G = torch.empty((self.n_tris, HB_PC_SLOTS, HB_PC_SLOTS), dtype=torch.float32, device="cuda")
        a = torch.empty((self.n_tris, HB_PC_SLOTS), dtype=torch.float32, device="cuda")
        y = torch.empty_like(a) if exact else None
        self._check(lib().hb_precond_spai(self._h, _ptr(G), _ptr(a), _ptr(y) if exact else None,
                                          _stream(stream)))
        return G, a, y

    def precond_install(self, net, stream=None):
        """Predict and install the learned preconditioner of this context (hb_precond_install)."""
        self._check(lib().hb_precond_install(self._h, net._h, _stream(stream)))

    def precond_set(self, weights, stream=None):
        self._check(lib().hb_precond_set(self._h, _ptr(weights) if weights is not None else None,
                                         _stream(stream)))

    def eval_repr(self, pts, w, g, stream=None, parts=False):
        import torch
        P = pts.shape[0]
        u = torch.empty(P, dtype=torch.float64, device="cuda")
        sl = torch.empty_like(u) if parts else None
        dl = torch.empty_like(u) if parts else None
        self._check(lib().hb_eval_repr(self._h, _ptr(pts), P, _ptr(w), _ptr(g), _ptr(u),
                                       _ptr(sl) if parts else None, _ptr(dl) if parts else None,
                                       _stream(stream)))
        return (u, sl, dl) if parts else u


class NonuniformContext(Context):
    """A mesh with the non-uniform time grid t_nodes (0 = t_0 < ... < t_{E_t}): block
    lower-triangular V_h and K_h with blocks (k, i), i <= k, at index k (k + 1) / 2 + i
    (hb_create_nonuniform)."""

    def __init__(self, verts, tris, alpha, t_nodes, **opts):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("heatbem needs a HIP device")
        v, t = _mesh_arrays(verts, tris)
        tn = np.ascontiguousarray(t_nodes, dtype=np.float64)
        self.n_tris, self.n_verts, self.n_t = len(t), len(v), len(tn) - 1
        self.alpha, self.T = float(alpha), float(tn[-1])
        self.t_nodes = tn
        o = default_options(**opts)
        self.storage = o.storage
        h = ctypes.c_void_p()
        rc = lib().hb_create_nonuniform(ctypes.byref(h), v.ctypes.data, len(v), t.ctypes.data,
                                        len(t), self.alpha, tn.ctypes.data, self.n_t, ctypes.byref(o))
        if rc != HB_OK:
            raise HBError(rc, lib().hb_last_error(None).decode())
        self._h = h
        self.n_blocks = self.n_t * (self.n_t + 1) // 2
