"""Python binding of libdgmg (ctypes): argument marshalling only.

Every computation runs in the HIP library; torch provides device memory (the
workspace and the vectors) and the current stream.  There is no fallback: if
the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int64, c_size_t, c_void_p
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgmg.so")

OK, NOT_CONVERGED, FELLBACK = 0, 1, 2
F64, F32 = 0, 1

_FLUX = {"ip": 0, "ldg": 1}
_SMOOTHER = {"EA": 0, "FA": 1, "EM": 2, "FM": 3}
_ORDER = {"lex": 0, "colour": 1}
_DISC = {"dg": 0, "se": 1}
_WEIGHT = {"quintic": 0, "cubic": 1, "arith": 2, "none": 3}
_VCYCLE = {"classical": 0, "variable": 1}
_PREC = {"fp64": 0, "mixed": 1}


class DgmgGrid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n_elem", c_int * 3), ("dx", POINTER(c_double) * 3),
                ("periodic", c_int * 3)]


class DgmgOpts(ctypes.Structure):
    _fields_ = [("P", c_int), ("flux", c_int), ("beta", c_double * 3), ("mu_star", c_double),
                ("smoother", c_int), ("overlap", c_int), ("weighting", c_int), ("vcycle", c_int),
                ("ns_pre", c_int), ("ns_post", c_int), ("precision", c_int), ("max_iter", c_int),
                ("order", c_int), ("disc", c_int)]


class DgmgStats(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("converged", c_int), ("r0", c_double),
                ("r_final", c_double), ("rho", c_double), ("history", c_double * 256),
                ("r_true", c_double), ("replacements", c_int)]


# (name, restype, argtypes) of every exported entry point of include/dgmg.h
SIGNATURES = [
    ("dgmg_opts_default", c_int, [POINTER(DgmgOpts)]),
    ("dgmg_setup", c_int, [POINTER(DgmgGrid), POINTER(DgmgOpts), POINTER(c_void_p)]),
    ("dgmg_workspace_bytes", c_int, [c_void_p, POINTER(c_size_t)]),
    ("dgmg_bind_workspace", c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    ("dgmg_set_stream", c_int, [c_void_p, c_void_p]),
    ("dgmg_num_levels", c_int, [c_void_p]),
    ("dgmg_level_info", c_int, [c_void_p, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int64)]),
    ("dgmg_node_coords", c_int, [c_void_p, c_int, c_int, POINTER(c_double)]),
    ("dgmg_apply", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int]),
    ("dgmg_residual", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int]),
    ("dgmg_smooth", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int, c_int]),
    ("dgmg_sweep", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int, c_int]),
    ("dgmg_restrict", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int]),
    ("dgmg_prolong", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int]),
    ("dgmg_coarse_solve", c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    ("dgmg_vcycle", c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    ("dgmg_solve", c_int, [c_void_p, c_void_p, c_void_p, c_double, POINTER(DgmgStats)]),
    ("dgmg_mass", c_int, [c_void_p, c_void_p, c_void_p]),
    ("dgmg_kernel_timing", c_int, [c_void_p, c_int]),
    ("dgmg_kernel_time", c_int, [c_void_p, POINTER(c_double), POINTER(c_int64), POINTER(c_double),
                                 POINTER(c_double)]),
    ("dgmg_use_graphs", c_int, [c_void_p, c_int]),
    ("dgmg_autotune", c_int, [c_void_p]),
    ("dgmg_tune_get", c_int, [c_void_p, c_int, c_int, POINTER(c_int), POINTER(c_double)]),
    ("dgmg_tune_set", c_int, [c_void_p, c_int, c_int, c_int]),
    ("dgmg_destroy", None, [c_void_p]),
    ("dgmg_last_error", ctypes.c_char_p, [c_void_p]),
    ("dgmg_face_count", c_int, [c_void_p]),
    ("dgmg_face_features", c_int, [c_void_p, POINTER(ctypes.c_float)]),
    ("dgmg_set_face_params", c_int, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    ("dgmg_get_face_params", c_int, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    ("dgmg_mlp_param_count", c_int, []),
    ("dgmg_mlp_forward", c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    ("dgmg_mlp_forward_noalloc", c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    ("dgmg_mlp_backward", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p]),
    ("dgmg_mlp_adam", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, ctypes.c_float, c_void_p]),
    ("dgmg_mlp_work_bytes", c_int, [c_void_p, POINTER(c_size_t)]),
    ("dgmg_apply_mlp", c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_int, POINTER(c_double)]),
    ("dgmg_batch_setup", c_int, [c_int, POINTER(DgmgGrid), POINTER(DgmgOpts), POINTER(c_void_p)]),
    ("dgmg_batch_workspace_bytes", c_int, [c_void_p, POINTER(c_size_t)]),
    ("dgmg_batch_plan_info", c_int, [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
    ("dgmg_batch_bind_workspace", c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    ("dgmg_batch_offsets", c_int, [c_void_p, POINTER(c_int64)]),
    ("dgmg_batch_handle", c_int, [c_void_p, c_int, POINTER(c_void_p)]),
    ("dgmg_batch_autotune", c_int, [c_void_p]),
    ("dgmg_batch_use_graphs", c_int, [c_void_p, c_int]),
    ("dgmg_batch_solve", c_int, [c_void_p, c_void_p, c_void_p, c_double, POINTER(DgmgStats)]),
    ("dgmg_batch_last_error", ctypes.c_char_p, [c_void_p]),
    ("dgmg_batch_destroy", None, [c_void_p]),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdgmg.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise OSError(f"{path} not found: build it with `python -m paper_1603_02524_amd.build_lib`")
        # torch first: the HIP runtime it loads then serves the library too (loaded
        # the other way round, the two can end up with separate runtimes, and the
        # library's finds no device)
        try:
            import torch  # noqa: F401
        except ImportError:  # host-only use (setup, tables) needs no torch
            pass
        lib = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class DgmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dgmg error {code}: {msg}")
        self.code = code


def make_structs(grid, method, max_iter: int = 100):
    """Translate synth.Grid / synth.Method into the C structs (kept alive by the caller)."""
    g = DgmgGrid()
    g.dim = grid.dim
    keep = []
    for d in range(3):
        if d < grid.dim:
            arr = np.ascontiguousarray(np.asarray(grid.dx[d], dtype=np.float64))
            keep.append(arr)
            g.n_elem[d] = len(arr)
            g.dx[d] = arr.ctypes.data_as(POINTER(c_double))
            g.periodic[d] = int(bool(grid.periodic[d]))
        else:
            g.n_elem[d] = 1
            g.dx[d] = None
            g.periodic[d] = 0
    o = DgmgOpts()
    o.P = int(method.P)
    o.flux = _FLUX[method.flux]
    for d in range(3):
        o.beta[d] = float(method.beta[d]) if d < len(method.beta) else 0.0
    o.mu_star = float(method.mu_star)
    o.smoother = _SMOOTHER[method.smoother]
    ov = method.overlap
    o.overlap = {"level": -1, "level_floor": -2, "zero": 0}.get(ov, ov) if isinstance(ov, str) else int(ov)
    o.weighting = _WEIGHT[method.weighting]
    o.vcycle = _VCYCLE[method.vcycle]
    o.ns_pre, o.ns_post = int(method.ns[0]), int(method.ns[1])
    o.precision = _PREC[method.precision]
    o.max_iter = int(max_iter)
    o.order = _ORDER[getattr(method, "order", "lex")]
    o.disc = _DISC[getattr(method, "disc", "dg")]
    return g, o, keep


def setup_handle(grid, method, max_iter: int = 100):
    """dgmg_setup only (host work); returns (handle, keepalive)."""
    lib = load_library()
    g, o, keep = make_structs(grid, method, max_iter)
    h = c_void_p()
    rc = lib.dgmg_setup(ctypes.byref(g), ctypes.byref(o), ctypes.byref(h))
    if rc != 0:
        raise DgmgError(rc, lib.dgmg_last_error(None).decode())
    return h, keep


class Solver:
    """Handle wrapper: tables built at construction, workspace from torch on `device`."""

    def __init__(self, grid, method, max_iter: int = 100, device: str = "cuda"):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.grid, self.method = grid, method
        self.h, self._keep = setup_handle(grid, method, max_iter)
        nbytes = c_size_t()
        self._check(self.lib.dgmg_workspace_bytes(self.h, ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self._ws.device)
        self._check(self.lib.dgmg_bind_workspace(self.h, c_void_p(aligned), self.ws_bytes,
                                                 c_void_p(self.stream.cuda_stream)))
        self.device = self._ws.device
        self.mixed = method.precision == "mixed"

    # ------------------------------------------------------------------ helpers
    def _check(self, rc, allow=(0,)):
        if rc not in allow:
            msg = self.lib.dgmg_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise DgmgError(rc, msg)
        return rc

    @staticmethod
    def _dtype_code(t):
        import torch
        if t.dtype == torch.float64:
            return F64
        if t.dtype == torch.float32:
            return F32
        raise TypeError("vectors must be float64 or float32")

    def _ptr(self, t):
        if not t.is_contiguous():
            raise ValueError("vectors must be contiguous")
        if t.device != self.device:
            raise ValueError("vector on the wrong device")
        return c_void_p(t.data_ptr())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dgmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ queries
    @property
    def num_levels(self):
        return self.lib.dgmg_num_levels(self.h)

    def level_info(self, level):
        P, no, nd = c_int(), c_int(), c_int64()
        self._check(self.lib.dgmg_level_info(self.h, level, ctypes.byref(P), ctypes.byref(no), ctypes.byref(nd)))
        return P.value, no.value, nd.value

    def n_dof(self, level=-1):
        if level < 0:
            level = self.num_levels + level
        return self.level_info(level)[2]

    def node_coords(self, level, d):
        P, _, _ = self.level_info(level)
        N = len(self.grid.dx[d])
        if getattr(self.method, "disc", "dg") == "se":  # stored lattice nodes
            out = np.zeros(N * P - (0 if self.grid.periodic[d] else 1))
        else:
            out = np.zeros(N * (P + 1))
        self._check(self.lib.dgmg_node_coords(self.h, level, d, out.ctypes.data_as(POINTER(c_double))))
        return out

    # ------------------------------------------------------------------ operations
    def apply(self, level, x, y=None):
        y = self.torch.empty_like(x) if y is None else y
        self._check(self.lib.dgmg_apply(self.h, level, self._ptr(x), self._ptr(y), self._dtype_code(x)))
        return y

    def residual(self, level, f, x, r=None):
        r = self.torch.empty_like(x) if r is None else r
        self._check(self.lib.dgmg_residual(self.h, level, self._ptr(f), self._ptr(x), self._ptr(r),
                                           self._dtype_code(x)))
        return r

    def smooth(self, level, u, f, nsteps=1):
        self._check(self.lib.dgmg_smooth(self.h, level, self._ptr(u), self._ptr(f), nsteps,
                                         self._dtype_code(u)))
        return u

    def sweep(self, level, u, f, normal=-1):
        """One Schwarz sweep in place on u (normal -1: element-centred); multiplicative
        handles sweep their own partition forwards."""
        self._check(self.lib.dgmg_sweep(self.h, level, self._ptr(u), self._ptr(f), int(normal),
                                        self._dtype_code(u)))
        return u

    def restrict(self, level, r_fine, f_coarse=None):
        if f_coarse is None:
            f_coarse = self.torch.empty(self.n_dof(level - 1), dtype=r_fine.dtype, device=self.device)
        self._check(self.lib.dgmg_restrict(self.h, level, self._ptr(r_fine), self._ptr(f_coarse),
                                           self._dtype_code(r_fine)))
        return f_coarse

    def prolong(self, level, u_coarse, u_fine):
        self._check(self.lib.dgmg_prolong(self.h, level, self._ptr(u_coarse), self._ptr(u_fine),
                                          self._dtype_code(u_coarse)))
        return u_fine

    def coarse_solve(self, f0, u0=None):
        u0 = self.torch.empty_like(f0) if u0 is None else u0
        self._check(self.lib.dgmg_coarse_solve(self.h, self._ptr(f0), self._ptr(u0), self._dtype_code(f0)))
        return u0

    def vcycle(self, r, z=None):
        z = self.torch.empty_like(r) if z is None else z
        self._check(self.lib.dgmg_vcycle(self.h, self._ptr(r), self._ptr(z), self._dtype_code(r)))
        return z

    def mass(self, f_nodal, g=None):
        g = self.torch.empty_like(f_nodal) if g is None else g
        self._check(self.lib.dgmg_mass(self.h, self._ptr(f_nodal), self._ptr(g)))
        return g

    def solve(self, rhs, x, tol=1e-10):
        st = DgmgStats()
        rc = self._check(self.lib.dgmg_solve(self.h, self._ptr(rhs), self._ptr(x), float(tol),
                                             ctypes.byref(st)), allow=(0, 1))
        return _stats_dict(st, rc)

    def use_graphs(self, enable=True):
        self._check(self.lib.dgmg_use_graphs(self.h, int(enable)))

    def autotune(self):
        """Time the patch-solve block shapes of every sweep and keep the fastest."""
        self._check(self.lib.dgmg_autotune(self.h))
        return self.tuning()

    def tuning(self):
        out = {}
        for l in range(1, self.num_levels):
            for kind in range(4):
                w, ms = c_int(), c_double()
                self._check(self.lib.dgmg_tune_get(self.h, l, kind, ctypes.byref(w), ctypes.byref(ms)))
                if w.value:
                    out[(l, kind)] = (w.value, ms.value)
        return out

    def set_tuning(self, level, kind, waves):
        self._check(self.lib.dgmg_tune_set(self.h, level, kind, int(waves)))

    def kernel_timing(self, enable=True, stride=1):
        """Start (every stride-th top-level patch-solve launch timed) or stop."""
        if enable and stride < 1:
            raise ValueError("kernel_timing: stride must be >= 1")
        self._check(self.lib.dgmg_kernel_timing(self.h, int(stride) if enable else 0))

    def kernel_time(self):
        ms, n, fl, by = c_double(), c_int64(), c_double(), c_double()
        self._check(self.lib.dgmg_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl),
                                              ctypes.byref(by)))
        return {"ms": ms.value, "launches": n.value, "flops": fl.value, "bytes": by.value}

    # ------------------------------------------------------------------ learned face weights
    def face_count(self):
        return self._check(self.lib.dgmg_face_count(self.h), allow=range(0, 1 << 30))

    def face_features(self):
        return _face_features(self.lib, self.h)

    def set_face_params(self, theta=None, omega=None):
        """Impose (theta, omega) per face (host arrays), or restore the fixed weights."""
        if theta is None:
            self._check(self.lib.dgmg_set_face_params(self.h, None, None))
            return
        n = self.face_count()
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(n)
        om = np.ascontiguousarray(omega, dtype=np.float64).reshape(n)
        self._check(self.lib.dgmg_set_face_params(self.h, th.ctypes.data_as(POINTER(c_double)),
                                                  om.ctypes.data_as(POINTER(c_double))))

    def face_params(self):
        n = self.face_count()
        th, om = np.zeros(n), np.zeros(n)
        rc = self.lib.dgmg_get_face_params(self.h, th.ctypes.data_as(POINTER(c_double)),
                                           om.ctypes.data_as(POINTER(c_double)))
        self._check(rc, allow=(0, 1))
        return th, om, bool(rc)

    def apply_mlp(self, params, probe_iters=3):
        """Learned weights from the MLP (FP32 device params) with the probe fallback.

        Returns (kept, ratio_learned, ratio_fixed)."""
        nb = c_size_t()
        self._check(self.lib.dgmg_mlp_work_bytes(self.h, ctypes.byref(nb)))
        work = self.torch.empty(int(nb.value) + 256, dtype=self.torch.uint8, device=self.device)
        aligned = (work.data_ptr() + 255) // 256 * 256
        ratios = (c_double * 2)()
        rc = self._check(self.lib.dgmg_apply_mlp(self.h, self._ptr(params), c_void_p(aligned), int(nb.value),
                                                 int(probe_iters), ratios), allow=(0, FELLBACK))
        return rc == 0, ratios[0], ratios[1]


def _face_features(lib, h):
    n = lib.dgmg_face_count(h)
    if n < 0:
        raise DgmgError(n, "face count")
    X = np.zeros((n, MLP_IN), dtype=np.float32)
    rc = lib.dgmg_face_features(h, X.ctypes.data_as(POINTER(ctypes.c_float)))
    if rc:
        raise DgmgError(rc, "face features")
    return X


def face_features(grid, method):
    """Per-face MLP features of a problem (host only: no device needed)."""
    lib = load_library()
    h, keep = setup_handle(grid, method)
    try:
        return _face_features(lib, h)
    finally:
        lib.dgmg_destroy(h)


MLP_IN, MLP_HIDDEN, MLP_OUT = 6, 64, 2
MLP_NOALLOC_MAX_ROWS = 8192


def mlp_param_count():
    return load_library().dgmg_mlp_param_count()


def _dptr(t):
    if not t.is_contiguous() or not t.is_cuda:
        raise ValueError("MLP arrays must be contiguous device tensors")
    return c_void_p(t.data_ptr())


def _stream(t):
    import torch
    return c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_forward(params, X):
    """Y [B][OUT] and the hidden activations [B][2 HIDDEN] (float32 device tensors)."""
    import torch
    lib = load_library()
    B = X.shape[0]
    Y = torch.empty((B, MLP_OUT), dtype=torch.float32, device=X.device)
    work = torch.empty((B, 2 * MLP_HIDDEN), dtype=torch.float32, device=X.device)
    rc = lib.dgmg_mlp_forward(_dptr(params), _dptr(X), B, _dptr(Y), _dptr(work), _stream(X))
    if rc:
        raise DgmgError(rc, "mlp forward")
    return Y, work


def mlp_forward_noalloc(params, X, Y=None):
    """Y = MLP(X) with the library's static work area (no device allocation by the
    library; X rows <= MLP_NOALLOC_MAX_ROWS)."""
    import torch
    lib = load_library()
    B = X.shape[0]
    if Y is None:
        Y = torch.empty((B, MLP_OUT), dtype=torch.float32, device=X.device)
    rc = lib.dgmg_mlp_forward_noalloc(_dptr(params), _dptr(X), B, _dptr(Y), _stream(X))
    if rc:
        raise DgmgError(rc, lib.dgmg_last_error(None).decode())
    return Y


def mlp_backward(params, X, T, Y, work):
    """Gradient of (1/B) sum (Y - T)^2 with respect to the parameters."""
    import torch
    lib = load_library()
    B = X.shape[0]
    grad = torch.empty_like(params)
    scratch = torch.empty(B * (2 * MLP_HIDDEN + MLP_OUT), dtype=torch.float32, device=X.device)
    rc = lib.dgmg_mlp_backward(_dptr(params), _dptr(X), _dptr(T), B, _dptr(Y), _dptr(work), _dptr(grad),
                               _dptr(scratch), _stream(X))
    if rc:
        raise DgmgError(rc, "mlp backward")
    return grad


def mlp_adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One in-place Adam step on params (m, v: moment tensors, updated in place)."""
    lib = load_library()
    rc = lib.dgmg_mlp_adam(_dptr(params), _dptr(grad), _dptr(m), _dptr(v), params.numel(), int(t), lr, b1, b2,
                           eps, _stream(params))
    if rc:
        raise DgmgError(rc, "mlp adam")


def _stats_dict(st, rc):
    n = st.iterations
    return {"rc": rc, "iterations": n, "converged": bool(st.converged), "r0": st.r0,
            "r_final": st.r_final, "rho": st.rho, "r_true": st.r_true, "replacements": st.replacements,
            "history": [st.history[i] for i in range(min(n, 255) + 1)]}


class BatchSolver:
    """Many independent grids solved in lock step (hipGraph replay per MGCG phase)."""

    def __init__(self, problems, max_iter: int = 100, device: str = "cuda"):
        import torch
        self.torch = torch
        self.lib = load_library()
        n = len(problems)
        grids = (DgmgGrid * n)()
        opts = (DgmgOpts * n)()
        self._keep = []
        for i, (g, m) in enumerate(problems):
            gg, oo, keep = make_structs(g, m, max_iter)
            grids[i] = gg
            opts[i] = oo
            self._keep.append(keep)
        self._grids, self._opts = grids, opts
        self.b = c_void_p()
        rc = self.lib.dgmg_batch_setup(n, grids, opts, ctypes.byref(self.b))
        if rc != 0:
            raise DgmgError(rc, self.lib.dgmg_batch_last_error(None).decode())
        self.count = n
        nbytes = c_size_t()
        self._check(self.lib.dgmg_batch_workspace_bytes(self.b, ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self._ws.device)
        self._check(self.lib.dgmg_batch_bind_workspace(self.b, c_void_p(aligned), self.ws_bytes,
                                                       c_void_p(self.stream.cuda_stream)))
        off = (c_int64 * (n + 1))()
        self._check(self.lib.dgmg_batch_offsets(self.b, off))
        self.offsets = [int(off[i]) for i in range(n + 1)]
        self.device = self._ws.device

    def _check(self, rc, allow=(0,)):
        if rc not in allow:
            raise DgmgError(rc, self.lib.dgmg_batch_last_error(self.b).decode())
        return rc

    def plan_info(self):
        """(planned, batched kernel launches per iteration, per-grid operations per iteration)."""
        p, k, g = c_int(), c_int(), c_int()
        self._check(self.lib.dgmg_batch_plan_info(self.b, ctypes.byref(p), ctypes.byref(k), ctypes.byref(g)))
        return bool(p.value), k.value, g.value

    @property
    def n_dof(self):
        return self.offsets[-1]

    def use_graphs(self, enable=True):
        self._check(self.lib.dgmg_batch_use_graphs(self.b, int(enable)))

    def autotune(self):
        self._check(self.lib.dgmg_batch_autotune(self.b))

    def solve(self, rhs, x, tol=1e-10):
        for t in (rhs, x):
            if t.dtype != self.torch.float64 or not t.is_contiguous() or t.numel() != self.n_dof:
                raise ValueError("rhs and x must be contiguous float64 vectors of all grids")
        st = (DgmgStats * self.count)()
        rc = self._check(self.lib.dgmg_batch_solve(self.b, c_void_p(rhs.data_ptr()), c_void_p(x.data_ptr()),
                                                   float(tol), st), allow=(0, 1))
        return [_stats_dict(st[i], rc) for i in range(self.count)]

    def close(self):
        if getattr(self, "b", None):
            self.lib.dgmg_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
