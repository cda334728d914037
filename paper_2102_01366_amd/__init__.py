"""MI355X (gfx950) implementation of the third-order compact gas-kinetic scheme
on tetrahedral meshes (Ji, Zhao, Shyy & Xu, arXiv:2102.01366).

The computation lives in ``libgks.so`` (HIP kernels behind the C interface of
``include/gks.h``).  This package only marshals arguments: ``Solver`` wraps
one library context, takes device memory and the stream from PyTorch, and
mirrors the C entry points one to one.  There is no CPU fallback: if the
library is missing, importing the binding raises.

``paper_2102_01366_amd.inputs`` (meshes and initial fields) can be imported
without the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgks.so")

GKS_OK = 0
GKS_E_INVAL = -1
GKS_E_MESH = -2
GKS_E_NONPHYSICAL = -3
GKS_E_ORDER = -4
GKS_E_DEVICE = -5
GKS_E_STATE = -6
GKS_E_NOMEM = -7

GKS_FP64 = 0
GKS_FP32_BULK = 1
GKS_FLUX_FULL = 0    # eq. 2nd-flux
GKS_FLUX_SMOOTH = 1  # eq. 2nd-smooth-flux

# names of every function the C interface declares (include/gks.h)
EXPORTS = ("gks_default_config", "gks_create", "gks_destroy", "gks_set_stream",
           "gks_mesh_upload", "gks_workspace_bytes", "gks_bind_workspace", "gks_init",
           "gks_compute_dt", "gks_stage", "gks_step", "gks_step_cfl", "gks_last_dt",
           "gks_adjoint_workspace_bytes", "gks_bind_adjoint_workspace", "gks_step_adjoint",
           "gks_read_state", "gks_conservation_sums_noalloc",
           "gks_conservation_sums", "gks_debug_reconstruct", "gks_debug_face_terms", "gks_debug_flux_integrals",
           "gks_timing_enable", "gks_timing_read", "gks_flux_op_count", "gks_flux_point_check",
           "gks_flux_face_check", "gks_weno_check", "gks_wall_ghost_check", "gks_last_error",
           "gks_strerror")

KERNELS = ("slopes", "reconstruct", "flux_stage1", "flux_stage2", "update_stage1",
           "update_stage2", "dt")


class GksError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("prandtl", ctypes.c_double), ("eps_tau", ctypes.c_double),
                ("c_tau", ctypes.c_double), ("eps_weno", ctypes.c_double),
                ("lw2", ctypes.c_double * 3), ("lw1", ctypes.c_double * 2),
                ("viscous", ctypes.c_int32), ("nonlinear", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("order", ctypes.c_int32),
                ("flux", ctypes.c_int32), ("wall_T", ctypes.c_double),
                ("farfield", ctypes.c_double * 5)]


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vert", ctypes.c_int64), ("xyz", ctypes.c_void_p),
                ("n_cell", ctypes.c_int64), ("tet", ctypes.c_void_p),
                ("n_face", ctypes.c_int64), ("face_vert", ctypes.c_void_p),
                ("face_cell", ctypes.c_void_p), ("face_tag", ctypes.c_void_p),
                ("face_shift", ctypes.c_void_p), ("face_wall_u", ctypes.c_void_p),
                ("tet_mid", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgks.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libgks.so not found at {path}; build it with "
                          "`python -m paper_2102_01366_amd.build`")
    import torch  # noqa: F401  (loads the HIP runtime the library links against)
    L = ctypes.CDLL(path)
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    S = ctypes.c_int32
    sig = {
        "gks_default_config": (None, [P]),
        "gks_create": (S, [P, P]),
        "gks_destroy": (None, [P]),
        "gks_set_stream": (S, [P, P]),
        "gks_mesh_upload": (S, [P, P]),
        "gks_workspace_bytes": (S, [P, P]),
        "gks_bind_workspace": (S, [P, P, ctypes.c_size_t]),
        "gks_init": (S, [P, P, P, I32]),
        "gks_compute_dt": (S, [P, D, P]),
        "gks_stage": (S, [P, I32, D]),
        "gks_step": (S, [P, D]),
        "gks_step_cfl": (S, [P, D]),
        "gks_adjoint_workspace_bytes": (S, [P, P]),
        "gks_bind_adjoint_workspace": (S, [P, P, ctypes.c_size_t]),
        "gks_step_adjoint": (S, [P, D, P, P, P, P, P, P]),
        "gks_last_dt": (S, [P, P]),
        "gks_read_state": (S, [P, P, P, I32]),
        "gks_conservation_sums": (S, [P, P]),
        "gks_conservation_sums_noalloc": (S, [P, P]),
        "gks_debug_reconstruct": (S, [P, P, P, P, I32]),
        "gks_debug_face_terms": (S, [P, D, P, I32]),
        "gks_debug_flux_integrals": (S, [P, D, P, I32]),
        "gks_timing_enable": (S, [P, I32]),
        "gks_timing_read": (S, [P, P, P, I32]),
        "gks_flux_op_count": (S, [P, P]),
        "gks_flux_point_check": (S, [P, D, P, P, P, P, P, P]),
        "gks_flux_face_check": (S, [P, D, P, P, P, P, P, P, P]),
        "gks_weno_check": (S, [P, P, I32, P, P, P, P, P, P]),
        "gks_wall_ghost_check": (S, [P, I32, P, P, P, P, P, P, P]),
        "gks_last_error": (ctypes.c_char_p, [P]),
        "gks_strerror": (ctypes.c_char_p, [S]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def default_config(**kw) -> Config:
    """The paper's defaults (gks_default_config), overridden by keywords;
    ``lw2``/``lw1`` take ratios."""
    L = load_library()
    c = Config()
    L.gks_default_config(ctypes.byref(c))
    names = {f[0] for f in Config._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown configuration field {k!r}")
        if k in ("lw2", "lw1", "farfield"):
            arr = getattr(c, k)
            for i, x in enumerate(v):
                arr[i] = float(x)
        elif k in ("viscous", "nonlinear"):
            setattr(c, k, 1 if v else 0)
        else:
            setattr(c, k, v)
    return c


def flux_op_count(config: Config | None = None) -> dict:
    """Algorithmic operations of the flux kernel per face (host-side count)."""
    L = load_library()
    c = config if config is not None else default_config()
    out = (ctypes.c_double * 4)()
    st = L.gks_flux_op_count(ctypes.byref(c), out)
    if st != GKS_OK:
        raise GksError(st, "gks_flux_op_count failed")
    d = {"add": out[0], "mul": out[1], "div": out[2], "special": out[3]}
    d["total"] = sum(out)
    return d


def flux_point_check(config: Config, dt: float, x, v, ybar):
    """Host check of the interface-point flux: (y, J v, J^T ybar), see gks.h."""
    L = load_library()
    x, v, yb = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, v, ybar))
    assert x.shape == (40,) and v.shape == (40,) and yb.shape == (20,)
    y, jv, xb = np.zeros(20), np.zeros(20), np.zeros(40)
    st = L.gks_flux_point_check(ctypes.byref(config), float(dt), _ptr(x), _ptr(v), _ptr(yb),
                                _ptr(y), _ptr(jv), _ptr(xb))
    if st != GKS_OK:
        raise GksError(st, "gks_flux_point_check failed")
    return y, jv, xb


def flux_face_check(config: Config, dt: float, geo, coef, v, accbar):
    """Host check of one Gauss point's face terms: (acc, J v, J^T accbar), see gks.h."""
    L = load_library()
    geo, coef, v, ab = (np.ascontiguousarray(a, dtype=np.float64) for a in (geo, coef, v, accbar))
    assert geo.shape == (10,) and coef.shape == (100,) and v.shape == (100,) and ab.shape == (20,)
    acc, jv, cb = np.zeros(20), np.zeros(20), np.zeros(100)
    st = L.gks_flux_face_check(ctypes.byref(config), float(dt), _ptr(geo), _ptr(coef), _ptr(v), _ptr(ab),
                               _ptr(acc), _ptr(jv), _ptr(cb))
    if st != GKS_OK:
        raise GksError(st, "gks_flux_face_check failed")
    return acc, jv, cb


def weno_check(config: Config, geo, has_mask: int, x, v, rbar):
    """Host check of the step-2 nonlinear combination: (r, J v, J^T rbar), see gks.h."""
    L = load_library()
    geo, x, v, rb = (np.ascontiguousarray(a, dtype=np.float64) for a in (geo, x, v, rbar))
    assert geo.shape == (8,) and x.shape == (25,) and v.shape == (25,) and rb.shape == (10,)
    r, jv, xb = np.zeros(10), np.zeros(10), np.zeros(25)
    st = L.gks_weno_check(ctypes.byref(config), _ptr(geo), int(has_mask), _ptr(x), _ptr(v), _ptr(rb),
                          _ptr(r), _ptr(jv), _ptr(xb))
    if st != GKS_OK:
        raise GksError(st, "gks_weno_check failed")
    return r, jv, xb


def wall_ghost_check(config: Config, tag: int, uw, x, v, ybar):
    """Host check of the no-slip ghost state: (y, J v, J^T ybar), see gks.h."""
    L = load_library()
    uw, x, v, yb = (np.ascontiguousarray(a, dtype=np.float64) for a in (uw, x, v, ybar))
    assert uw.shape == (3,) and x.shape == (20,) and v.shape == (20,) and yb.shape == (20,)
    y, jv, xb = np.zeros(20), np.zeros(20), np.zeros(20)
    st = L.gks_wall_ghost_check(ctypes.byref(config), int(tag), _ptr(uw), _ptr(x), _ptr(v), _ptr(yb),
                                _ptr(y), _ptr(jv), _ptr(xb))
    if st != GKS_OK:
        raise GksError(st, "gks_wall_ghost_check failed")
    return y, jv, xb


def _ptr(a) -> int:
    """Address of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class Solver:
    """One libgks context bound to a mesh, a torch-allocated workspace and the
    current torch stream of ``device``."""

    def __init__(self, mesh, config: Config | None = None, device="cuda", stream=None):
        import torch
        self._torch = torch
        self.L = load_library()
        self.config = config if config is not None else default_config()
        self.device = torch.device(device)
        self._h = ctypes.c_void_p()
        self._check(self.L.gks_create(ctypes.byref(self.config), ctypes.byref(self._h)), "create")
        self.nc = int(mesh.n_cell)
        self.nf = int(mesh.n_face)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.L.gks_set_stream(self._h, ctypes.c_void_p(self.stream.cuda_stream)),
                    "set_stream")
        keep = [np.ascontiguousarray(mesh.xyz, np.float64),
                np.ascontiguousarray(mesh.tet, np.int64),
                np.ascontiguousarray(mesh.face_vert, np.int64),
                np.ascontiguousarray(mesh.face_cell, np.int64),
                np.ascontiguousarray(mesh.face_tag, np.int32),
                np.ascontiguousarray(mesh.face_shift, np.float64)]
        wu = getattr(mesh, "face_wall_u", None)
        tm = getattr(mesh, "tet_mid", None)
        keep.append(None if wu is None else np.ascontiguousarray(wu, np.float64))
        keep.append(None if tm is None else np.ascontiguousarray(tm, np.float64))
        m = _Mesh(mesh.n_vert, keep[0].ctypes.data, self.nc, keep[1].ctypes.data, self.nf,
                  keep[2].ctypes.data, keep[3].ctypes.data, keep[4].ctypes.data,
                  keep[5].ctypes.data, keep[6].ctypes.data if wu is not None else None,
                  keep[7].ctypes.data if tm is not None else None)
        self._check(self.L.gks_mesh_upload(self._h, ctypes.byref(m)), "mesh_upload")
        nbytes = ctypes.c_size_t()
        self._check(self.L.gks_workspace_bytes(self._h, ctypes.byref(nbytes)), "workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self._check(self.L.gks_bind_workspace(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                              self.workspace_bytes), "bind_workspace")

    # -- plumbing ----------------------------------------------------------
    def _check(self, status, what):
        if status != GKS_OK:
            msg = self.L.gks_last_error(self._h) if self._h else b""
            name = self.L.gks_strerror(status).decode()
            raise GksError(status, f"gks_{what}: {name}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_h", None):
            self.L.gks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        return (not isinstance(a, np.ndarray)) and a.is_cuda

    def _enter(self):
        """Device inputs were produced on torch's current stream: the
        library's stream waits for it before its work is enqueued."""
        cur = self._torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        return cur

    def _leave(self, cur, tensors):
        """The library's work on device tensors is enqueued on its own stream:
        the caching allocator keeps them until that work ends, and torch's
        current stream waits for it before the tensors are used there."""
        if cur != self.stream:
            for t in tensors:
                t.record_stream(self.stream)
            cur.wait_stream(self.stream)

    # -- the C interface -----------------------------------------------------
    def init(self, W, gW):
        """W[5, n], gW[15, n]: float64 numpy arrays or CUDA tensors."""
        on_dev = self._dev(W)
        if on_dev:
            W = W.contiguous().to(self._torch.float64)
            gW = gW.contiguous().to(self._torch.float64)
        else:
            W = np.ascontiguousarray(W, np.float64)
            gW = np.ascontiguousarray(gW, np.float64)
        if tuple(W.shape) != (5, self.nc) or tuple(gW.shape) != (15, self.nc):
            raise ValueError("W must be [5, n_cell] and gW [15, n_cell]")
        cur = self._enter() if on_dev else None
        self._check(self.L.gks_init(self._h, ctypes.c_void_p(_ptr(W)), ctypes.c_void_p(_ptr(gW)),
                                    1 if on_dev else 0), "init")
        if on_dev:
            self._leave(cur, (W, gW))

    def bind_adjoint(self):
        """Allocate and bind the adjoint workspace (once)."""
        if getattr(self, "adjoint_workspace", None) is not None:
            return
        nbytes = ctypes.c_size_t()
        self._check(self.L.gks_adjoint_workspace_bytes(self._h, ctypes.byref(nbytes)), "adjoint_workspace_bytes")
        self.adjoint_workspace = self._torch.empty(int(nbytes.value), dtype=self._torch.uint8, device=self.device)
        self._check(self.L.gks_bind_adjoint_workspace(self._h, ctypes.c_void_p(self.adjoint_workspace.data_ptr()),
                                                      int(nbytes.value)), "bind_adjoint_workspace")

    def step_adjoint(self, dt: float, W, gW, Wbar, gWbar):
        """Adjoints of (W, gW) before a step of size dt, given the state (W, gW)
        before it and the adjoints (Wbar, gWbar) of the state after it (CUDA
        float64 tensors [5, n] and [15, n]).  Returns new tensors."""
        t = self._torch
        self.bind_adjoint()
        args = []
        for a, rows in ((W, 5), (gW, 15), (Wbar, 5), (gWbar, 15)):
            if not self._dev(a) or tuple(a.shape) != (rows, self.nc):
                raise ValueError("step_adjoint takes CUDA tensors [5, n] and [15, n]")
            args.append(a.contiguous().to(t.float64))
        Wo = t.empty((5, self.nc), dtype=t.float64, device=self.device)
        Go = t.empty((15, self.nc), dtype=t.float64, device=self.device)
        cur = self._enter()
        self._check(self.L.gks_step_adjoint(self._h, float(dt), *(ctypes.c_void_p(a.data_ptr()) for a in args),
                                            ctypes.c_void_p(Wo.data_ptr()), ctypes.c_void_p(Go.data_ptr())),
                    "step_adjoint")
        self._leave(cur, args + [Wo, Go])
        return Wo, Go

    def compute_dt(self, cfl: float) -> float:
        dt = ctypes.c_double()
        self._check(self.L.gks_compute_dt(self._h, float(cfl), ctypes.byref(dt)), "compute_dt")
        return float(dt.value)

    def stage(self, stage: int, dt: float):
        self._check(self.L.gks_stage(self._h, int(stage), float(dt)), "stage")

    def step(self, dt: float):
        self._check(self.L.gks_step(self._h, float(dt)), "step")

    def step_cfl(self, cfl: float):
        """One step with dt = cfl x the CFL bound, computed and used on the device."""
        self._check(self.L.gks_step_cfl(self._h, float(cfl)), "step_cfl")

    def last_dt(self) -> float:
        dt = ctypes.c_double()
        self._check(self.L.gks_last_dt(self._h, ctypes.byref(dt)), "last_dt")
        return float(dt.value)

    def read_state(self, device: bool = False):
        if device:
            t = self._torch
            W = t.empty((5, self.nc), dtype=t.float64, device=self.device)
            gW = t.empty((15, self.nc), dtype=t.float64, device=self.device)
        else:
            W = np.empty((5, self.nc))
            gW = np.empty((15, self.nc))
        cur = self._enter() if device else None
        self._check(self.L.gks_read_state(self._h, ctypes.c_void_p(_ptr(W)),
                                          ctypes.c_void_p(_ptr(gW)), 1 if device else 0),
                    "read_state")
        if device:
            self._leave(cur, (W, gW))
        return W, gW

    def conservation_sums(self):
        out = np.empty(5)
        self._check(self.L.gks_conservation_sums(self._h, ctypes.c_void_p(out.ctypes.data)),
                    "conservation_sums")
        return out

    def debug_reconstruct(self):
        b = np.empty((15, self.nc))
        coef = np.empty((50, self.nc))
        flag = np.empty(self.nc, np.int32)
        self._check(self.L.gks_debug_reconstruct(self._h, ctypes.c_void_p(b.ctypes.data),
                                                 ctypes.c_void_p(coef.ctypes.data),
                                                 ctypes.c_void_p(flag.ctypes.data), 0),
                    "debug_reconstruct")
        return b, coef, flag

    def timing_enable(self, on: bool = True):
        self._check(self.L.gks_timing_enable(self._h, 1 if on else 0), "timing_enable")

    def timing_read(self, reset: bool = True):
        """{kernel: (total ms, launches)} accumulated since the last reset."""
        ms = np.zeros(len(KERNELS))
        cnt = np.zeros(len(KERNELS), np.int64)
        self._check(self.L.gks_timing_read(self._h, ctypes.c_void_p(ms.ctypes.data),
                                           ctypes.c_void_p(cnt.ctypes.data), 1 if reset else 0),
                    "timing_read")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNELS)}

    def debug_face_terms(self, dt: float):
        out = np.empty((20, self.nf))
        self._check(self.L.gks_debug_face_terms(self._h, float(dt),
                                                ctypes.c_void_p(out.ctypes.data), 0),
                    "debug_face_terms")
        return out

    def debug_flux_integrals(self, dt: float):
        """[20, n_face]: |Gamma| sum_k w_k of F_k(dt), F_k(dt/2), W_k(0), W_k(dt)."""
        out = np.empty((20, self.nf))
        self._check(self.L.gks_debug_flux_integrals(self._h, float(dt),
                                                    ctypes.c_void_p(out.ctypes.data), 0),
                    "debug_flux_integrals")
        return out
