"""FP64 CPU oracle of the compact third-order gas-kinetic scheme (test infrastructure).

A plain C implementation (``gks_oracle.c``) of one time step of the scheme,
written from the paper (Ji, Zhao, Shyy & Xu, compact GKS on tetrahedra) and
sharing no code with the HIP library.  Only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg may import this package.

``build()`` compiles ``libgks_oracle.so`` next to this file with gcc
(``-O2``, OpenMP, no fast-math); ``Oracle`` wraps a mesh and exposes the
per-kernel and per-step entry points as numpy functions.

``build()`` also compiles the tangent build ``libgks_oracle_tangent.so``: the
same source compiled as C++ over the forward-mode dual numbers of
``or_dual.hpp`` (value plus 16 directional derivatives).  ``TangentOracle``
runs its steps and returns exact Jacobian-vector products of the step map
(time steps held fixed), and counts how often a kink of the scheme lies
within a given distance along each direction.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gks_oracle.c")
_LIB = os.path.join(_HERE, "libgks_oracle.so")
_TLIB = os.path.join(_HERE, "libgks_oracle_tangent.so")
_DUAL = os.path.join(_HERE, "or_dual.hpp")
# the tangent build keeps ~3 MB of dual-number polynomials on each OpenMP
# thread's stack; libgomp reads this when the first OpenMP library loads
os.environ.setdefault("OMP_STACKSIZE", "64M")


def build(force: bool = True) -> str:
    """Compile the oracle library (serial-order arithmetic, OpenMP loops)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_DUAL))
    if force or not os.path.exists(_TLIB) or os.path.getmtime(_TLIB) < newest:
        cmd = ["g++", "-O2", "-x", "c++", "-std=gnu++17", "-DOR_TANGENT", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-Wall", "-Wno-class-memaccess", "-Wl,-Bsymbolic", "-o", _TLIB + ".tmp",
               _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_TLIB + ".tmp", _TLIB)
    return _LIB


class Config(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("K", ctypes.c_double), ("mu", ctypes.c_double),
                ("prandtl", ctypes.c_double), ("eps_tau", ctypes.c_double),
                ("c_tau", ctypes.c_double), ("eps_weno", ctypes.c_double),
                ("lw2", ctypes.c_double * 3), ("lw1", ctypes.c_double * 2),
                ("viscous", ctypes.c_int32), ("nonlinear", ctypes.c_int32), ("order", ctypes.c_int32),
                ("flux", ctypes.c_int32), ("wall_T", ctypes.c_double),
                ("farfield", ctypes.c_double * 5), ("weno_reading", ctypes.c_int32)]


def make_config(gamma=1.4, mu=0.0, prandtl=1.0, viscous=False, nonlinear=True,
                eps_tau=0.01, c_tau=1.0, eps_weno=1e-8, lw2=(100.0, 10.0, 1.0),
                lw1=(10.0, 1.0), K=None, order=3, flux=0, wall_T=1.0,
                farfield=(1.0, 0.0, 0.0, 0.0, 2.5), weno_reading=0) -> Config:
    """Scheme parameters; linear weights are given as ratios and normalised.
    flux: 0 for eq. 2nd-flux, 1 for the smooth-flow form eq. 2nd-smooth-flux.
    weno_reading: 0, or bits of READ_* selecting alternative readings of the
    nonlinear weights (only for comparisons with the paper's Tables 2-3)."""
    c = Config()
    c.weno_reading = weno_reading
    c.order = order
    c.flux = flux
    c.wall_T = wall_T
    for q in range(5):
        c.farfield[q] = farfield[q]
    c.gamma = gamma
    c.K = (5.0 - 3.0 * gamma) / (gamma - 1.0) if K is None else K
    c.mu = mu
    c.prandtl = prandtl
    c.eps_tau = eps_tau
    c.c_tau = c_tau
    c.eps_weno = eps_weno
    s2 = sum(lw2)
    s1 = sum(lw1)
    for i in range(3):
        c.lw2[i] = lw2[i] / s2
    for i in range(2):
        c.lw1[i] = lw1[i] / s1
    c.viscous = 1 if viscous else 0
    c.nonlinear = 1 if nonlinear else 0
    return c


# alternative readings of the nonlinear weights (gks_oracle.h, OR_READ_*)
READ_POW1, READ_POW1ST2, READ_B0VOL, READ_MIXED2, READ_BETA_LOWER, READ_SIGMA1 = 1, 2, 4, 8, 16, 32

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I64 = ctypes.c_int64
        L.or_create.restype = P
        L.or_create.argtypes = [ctypes.POINTER(Config), I64, P, I64, P, I64, P, P, P, P, P]
        L.or_create_quadratic.restype = P
        L.or_create_quadratic.argtypes = [ctypes.POINTER(Config), I64, P, I64, P, I64, P, P, P, P, P, P]
        L.or_wall_ghost.argtypes = [ctypes.POINTER(Config), ctypes.c_int32, P, P, P, P, P, P]
        L.or_destroy.argtypes = [P]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = ctypes.c_int
        for name in ("or_geometry",):
            getattr(L, name).argtypes = [P, P, P, P, P]
        L.or_face_geometry.argtypes = [P, P, P, P]
        L.or_face_points.argtypes = [P, P, P]
        L.or_slopes.argtypes = [P, P, P, P]
        L.or_reconstruct.argtypes = [P, P, P, P, P, P]
        L.or_face_terms.argtypes = [P, P, P, D, P]
        L.or_face_integrals.argtypes = [P, P, P, D, P]
        L.or_last_face_terms.argtypes = [P, P]
        L.or_stage.argtypes = [P, ctypes.c_int, D, P, P]
        L.or_step.argtypes = [P, D, P, P]
        L.or_compute_dt.argtypes = [P, P, D]
        L.or_compute_dt.restype = D
        L.or_conservation_sums.argtypes = [P, P, P]
        L.or_point_flux.argtypes = [ctypes.POINTER(Config), P, P, P, P, P, D, P]
        L.or_point_flux_density.argtypes = [ctypes.POINTER(Config), P, P, P, P, P, D, D, P]
        L.or_maxwell_moments.argtypes = [ctypes.POINTER(Config), P, P]
        L.or_volume_rule.argtypes = [P, P]
        L.or_face_rule.argtypes = [P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> int:
    return _load().or_set_threads(int(n))


class Oracle:
    """The oracle bound to one mesh and one configuration."""

    def __init__(self, mesh, cfg: Config):
        L = _load()
        self.cfg = cfg
        self.nc = mesh.n_cell
        self.nf = mesh.n_face
        self._keep = [np.ascontiguousarray(mesh.xyz, np.float64),
                      np.ascontiguousarray(mesh.tet, np.int64),
                      np.ascontiguousarray(mesh.face_vert, np.int64),
                      np.ascontiguousarray(mesh.face_cell, np.int64),
                      np.ascontiguousarray(mesh.face_tag, np.int32),
                      np.ascontiguousarray(mesh.face_shift, np.float64)]
        wu = getattr(mesh, "face_wall_u", None)
        self._keep.append(None if wu is None else np.ascontiguousarray(wu, np.float64))
        tm = getattr(mesh, "tet_mid", None)
        self._keep.append(None if tm is None else np.ascontiguousarray(tm, np.float64))
        xyz, tet, fv, fc, ft, fs, fw, tmid = self._keep
        self._h = L.or_create_quadratic(ctypes.byref(cfg), mesh.n_vert, _p(xyz), self.nc, _p(tet),
                                        self.nf, _p(fv), _p(fc), _p(ft), _p(fs),
                                        None if fw is None else _p(fw), None if tmid is None else _p(tmid))
        if not self._h:
            raise ValueError("oracle rejected the mesh")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    def geometry(self):
        n = self.nc
        vol, cen, m2, dr = np.empty(n), np.empty((3, n)), np.empty((6, n)), np.empty(n)
        _load().or_geometry(self._h, _p(vol), _p(cen), _p(m2), _p(dr))
        return vol, cen, m2, dr

    def face_geometry(self):
        nf = self.nf
        area, nrm, gp = np.empty(nf), np.empty((3, nf)), np.empty((3, 3, nf))
        _load().or_face_geometry(self._h, _p(area), _p(nrm), _p(gp))
        return area, nrm, gp

    def face_points(self):
        """Per Gauss point: unit normals [3 points][3][nf] and weights [3][nf]
        (the face area included)."""
        nf = self.nf
        nrm, w = np.empty((3, 3, nf)), np.empty((3, nf))
        _load().or_face_points(self._h, _p(nrm), _p(w))
        return nrm, w

    def slopes(self, W, gW=None):
        W = _f64(W)
        g = _f64(gW) if gW is not None else None
        b = np.empty((15, self.nc))
        _load().or_slopes(self._h, _p(W), _p(g) if g is not None else None, _p(b))
        return b

    def reconstruct(self, W, gW, with_p2=False):
        W, gW = _f64(W), _f64(gW)
        coef = np.empty((50, self.nc))
        flag = np.empty(self.nc, np.int32)
        p2 = np.empty((50, self.nc)) if with_p2 else None
        _load().or_reconstruct(self._h, _p(W), _p(gW), _p(coef), _p(flag),
                               _p(p2) if with_p2 else None)
        return (coef, flag, p2) if with_p2 else (coef, flag)

    def face_terms(self, W, gW, dt):
        W, gW = _f64(W), _f64(gW)
        out = np.empty((20, self.nf))
        rc = _load().or_face_terms(self._h, _p(W), _p(gW), float(dt), _p(out))
        if rc:
            raise RuntimeError("oracle face terms failed")
        return out

    def face_integrals(self, W, gW, dt):
        """[20, nf]: |Gamma| sum_k w_k of F_k(dt), F_k(dt/2), W_k(0), W_k(dt)."""
        W, gW = _f64(W), _f64(gW)
        out = np.empty((20, self.nf))
        rc = _load().or_face_integrals(self._h, _p(W), _p(gW), float(dt), _p(out))
        if rc:
            raise RuntimeError("oracle face integrals failed")
        return out

    def last_face_terms(self):
        """[20, nf]: the face terms (as face_terms) of the last stage run."""
        out = np.empty((20, self.nf))
        _load().or_last_face_terms(self._h, _p(out))
        return out

    def gradient_bound(self, stage, ft1=None):
        """Per cell, component and direction, the sum of the magnitudes of the
        terms of the Gauss-theorem gradient (eq. gauss-formula) of the last
        stage run, (1/|Omega_i|) sum over the cell's faces of |W_f| |n_d|
        (interface values weighted by |Gamma|; on a quadratic face the largest
        |n_d| of its Gauss points): stage 1 sums (W_k(0) +
        W_k(dt)) / 2, stage 2 sums W1_k(0) + W2_k(dt) - W2_k(0), ft1 the face
        terms of stage 1.  The momentum components share one bound (the face
        frame mixes them), which also counts the thermal momentum scale
        sqrt(|rho| |rho E|): the interface momentum is a sum of the two
        half-space momenta of the kinetic weighting (eq. new-equ-part), of
        that size and opposite signs, so its rounding is relative to them even
        where the gas is at rest.  Two correct FP64 evaluations of the
        gradient differ by rounding relative to this bound, not to the
        gradient."""
        ft = self.last_face_terms()
        if stage == 1:
            a = 0.5 * (np.abs(ft[10:15]) + np.abs(ft[15:20]))
        else:
            a = np.abs(ft1[10:15]) + np.abs(ft[15:20]) + np.abs(ft[10:15])
        a[1:4] = a[1:4].sum(axis=0) + np.sqrt(a[0] * a[4])
        vol = self.geometry()[0]
        # the largest |n_d| over the face's Gauss points (one normal on a flat face)
        nrm = np.abs(self.face_points()[0]).max(axis=0)
        fc = self._keep[3].reshape(-1, 2)
        B = np.zeros((15, self.nc))
        for side in (0, 1):
            cells = fc[:, side]
            ok = cells >= 0
            for q in range(5):
                for d in range(3):
                    B[3 * q + d] += np.bincount(cells[ok], weights=a[q, ok] * nrm[d, ok], minlength=self.nc)
        return B / vol

    def stage(self, stage, dt, W, gW):
        W, gW = _f64(W).copy(), _f64(gW).copy()
        rc = _load().or_stage(self._h, int(stage), float(dt), _p(W), _p(gW))
        if rc:
            raise RuntimeError(f"oracle stage {stage} failed ({rc})")
        return W, gW

    def step(self, dt, W, gW):
        W, gW = _f64(W).copy(), _f64(gW).copy()
        rc = _load().or_step(self._h, float(dt), _p(W), _p(gW))
        if rc:
            raise RuntimeError(f"oracle step failed ({rc})")
        return W, gW

    def compute_dt(self, W, cfl):
        W = _f64(W)
        return float(_load().or_compute_dt(self._h, _p(W), float(cfl)))

    def conservation_sums(self, W):
        W = _f64(W)
        out = np.empty(5)
        _load().or_conservation_sums(self._h, _p(W), _p(out))
        return out


def wall_ghost(cfg: Config, tag, n, uw, W, gW):
    """Ghost state (W, gW[15], component c direction d at 3c+d) of a wall
    point: tag 2 slip, 3 no-slip adiabatic, 4 no-slip isothermal, 5 far field."""
    Wg, gWg = np.empty(5), np.empty(15)
    rc = _load().or_wall_ghost(ctypes.byref(cfg), int(tag), _p(_f64(n)), _p(_f64(uw)), _p(_f64(W)),
                               _p(_f64(gW)), _p(Wg), _p(gWg))
    if rc != 0:
        raise ValueError("unknown wall tag")
    return Wg, gWg


def point_flux(cfg: Config, n, Wl, gWl, Wr, gWr, dt):
    """F(dt), F(dt/2), W(0), W(dt) at one interface point (global frame)."""
    args = [_f64(x) for x in (n, Wl, gWl, Wr, gWr)]
    out = np.empty(20)
    rc = _load().or_point_flux(ctypes.byref(cfg), *[_p(a) for a in args], float(dt), _p(out))
    if rc:
        raise RuntimeError("oracle point flux failed")
    return out.reshape(4, 5)


def point_flux_density(cfg: Config, n, Wl, gWl, Wr, gWr, dt, t):
    args = [_f64(x) for x in (n, Wl, gWl, Wr, gWr)]
    out = np.empty(5)
    rc = _load().or_point_flux_density(ctypes.byref(cfg), *[_p(a) for a in args], float(dt),
                                       float(t), _p(out))
    if rc:
        raise RuntimeError("oracle point flux density failed")
    return out


def maxwell_moments(cfg: Config, W):
    W = _f64(W)
    out = np.empty(54)
    rc = _load().or_maxwell_moments(ctypes.byref(cfg), _p(W), _p(out))
    if rc:
        raise RuntimeError("non-physical state")
    return {"u": out[0:10], "u_pos": out[10:20], "u_neg": out[20:30], "v": out[30:40],
            "w": out[40:50], "xi2": out[50:54]}


def volume_rule():
    p, w = np.empty(15), np.empty(5)
    _load().or_volume_rule(_p(p), _p(w))
    return p.reshape(5, 3), w


def face_rule():
    p, w = np.empty(6), np.empty(3)
    _load().or_face_rule(_p(p), _p(w))
    return p.reshape(3, 2), w


_tlib = None


def _load_tangent():
    global _tlib
    if _tlib is None:
        if not os.path.exists(_TLIB):
            build(force=False)
        L = ctypes.CDLL(_TLIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I64 = ctypes.c_int64
        L.or_create.restype = P
        L.or_create.argtypes = [ctypes.POINTER(Config), I64, P, I64, P, I64, P, P, P, P, P]
        L.or_create_quadratic.restype = P
        L.or_create_quadratic.argtypes = [ctypes.POINTER(Config), I64, P, I64, P, I64, P, P, P, P, P, P]
        L.or_destroy.argtypes = [P]
        L.or_step.argtypes = [P, D, P, P]
        L.or_tangent_ndir.restype = ctypes.c_int
        L.or_tangent_set_kink_eps.argtypes = [D]
        L.or_tangent_kinks.argtypes = [P, ctypes.c_int]
        _tlib = L
    return _tlib


class TangentOracle:
    """The oracle's tangent build bound to one mesh and configuration.

    States are arrays of shape (rows, n_cell, 1 + ndir): the value, then its
    derivatives along ``ndir`` directions.  ``step`` advances them by one
    step of the scheme with the time step held fixed, so the derivative part
    of the result is the exact Jacobian-vector product of the step map."""

    def __init__(self, mesh, cfg: Config):
        L = _load_tangent()
        self.cfg = cfg
        self.nc = mesh.n_cell
        self.ndir = L.or_tangent_ndir()
        self._keep = [np.ascontiguousarray(mesh.xyz, np.float64),
                      np.ascontiguousarray(mesh.tet, np.int64),
                      np.ascontiguousarray(mesh.face_vert, np.int64),
                      np.ascontiguousarray(mesh.face_cell, np.int64),
                      np.ascontiguousarray(mesh.face_tag, np.int32),
                      np.ascontiguousarray(mesh.face_shift, np.float64)]
        wu = getattr(mesh, "face_wall_u", None)
        self._keep.append(None if wu is None else np.ascontiguousarray(wu, np.float64))
        tm = getattr(mesh, "tet_mid", None)
        self._keep.append(None if tm is None else np.ascontiguousarray(tm, np.float64))
        xyz, tet, fv, fc, ft, fs, fw, tmid = self._keep
        self._h = L.or_create_quadratic(ctypes.byref(cfg), mesh.n_vert, _p(xyz), self.nc, _p(tet),
                                        mesh.n_face, _p(fv), _p(fc), _p(ft), _p(fs),
                                        None if fw is None else _p(fw), None if tmid is None else _p(tmid))
        if not self._h:
            raise ValueError("oracle rejected the mesh")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _tlib is not None:
            _tlib.or_destroy(h)
            self._h = None

    def pack(self, X, dX):
        """value X[rows][n] and derivatives dX[ndir][rows][n] -> dual array"""
        out = np.empty(X.shape + (1 + self.ndir,))
        out[..., 0] = X
        out[..., 1:] = np.moveaxis(np.asarray(dX, np.float64), 0, -1)
        return out

    @staticmethod
    def unpack(Xd):
        """dual array -> value [rows][n], derivatives [ndir][rows][n]"""
        return Xd[..., 0].copy(), np.ascontiguousarray(np.moveaxis(Xd[..., 1:], -1, 0))

    def step(self, dt, Wd, gWd):
        Wd = np.ascontiguousarray(Wd, np.float64).copy()
        gWd = np.ascontiguousarray(gWd, np.float64).copy()
        assert Wd.shape == (5, self.nc, 1 + self.ndir) and gWd.shape == (15, self.nc, 1 + self.ndir)
        rc = _tlib.or_step(self._h, float(dt), _p(Wd), _p(gWd))
        if rc:
            raise RuntimeError(f"tangent oracle step failed ({rc})")
        return Wd, gWd

    @staticmethod
    def set_kink_eps(eps):
        _load_tangent().or_tangent_set_kink_eps(float(eps))

    def kinks(self, reset=True):
        """counts [2][ndir]: jump-term and WENO-indicator kinks within the
        set distance along each direction, since the last reset"""
        out = np.zeros(2 * self.ndir, np.int64)
        _tlib.or_tangent_kinks(_p(out), 1 if reset else 0)
        return out.reshape(2, self.ndir)
