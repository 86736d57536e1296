"""ctypes binding of the FP64 CPU oracle (oracle/pabd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and by
the CPU-baseline leg of bench.py -- never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pabd_oracle.c")
LIB_PATH = os.path.join(_HERE, "libpabd_oracle.so")
# a library built elsewhere from a copy of the source, used as it is; the test
# that plants mistakes in such copies sets it, nothing else does
_LIB_OVERRIDE = os.environ.get("PABD_ORACLE_LIB")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, -O2, no fast-math)."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    stale = not os.path.exists(LIB_PATH) or any(
        os.path.getmtime(src) > os.path.getmtime(LIB_PATH) for src in (_SRC, _SRC[:-2] + ".h"))
    if force or stale:
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_P = C.POINTER
_d = _P(C.c_double)
_i = _P(C.c_int32)


class _Desc(C.Structure):
    _fields_ = [
        ("n_bodies", C.c_int32), ("shape", _i), ("shape_param", _d), ("density", _d),
        ("flags", _P(C.c_uint8)), ("group", _i), ("c0", _d), ("A0", _d), ("v0", _d), ("w0", _d),
        ("n_bonds", C.c_int32), ("bond_i", _i), ("bond_j", _i), ("bond_type", _i),
        ("x_i", _d), ("x_j", _d), ("kappa", _d), ("rest_len", _d), ("drive", _d),
        ("gravity", C.c_double * 3), ("h", C.c_double), ("t0", C.c_double), ("iters", C.c_int32),
        ("contact_enable", C.c_int32), ("mu", C.c_double), ("contact_kappa_scale", C.c_double),
        ("contact_margin", C.c_double), ("n_planes", C.c_int32), ("planes", _d),
        ("al_beta", C.c_double), ("al_alpha", C.c_double), ("al_gamma", C.c_double),
        ("order", _i), ("mass", _d), ("Pi0", _d),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.pabd_oracle_create.restype = C.c_void_p
        L.pabd_oracle_create.argtypes = [_P(_Desc)]
        L.pabd_oracle_destroy.argtypes = [C.c_void_p]
        L.pabd_oracle_step.argtypes = [C.c_void_p, C.c_int32]
        L.pabd_oracle_read_state.argtypes = [C.c_void_p, _d, _d, _d, _d]
        L.pabd_oracle_residuals.argtypes = [C.c_void_p, _d, C.c_int32]
        L.pabd_oracle_set_debug.argtypes = [C.c_void_p, C.c_int32]
        L.pabd_oracle_last_iterates.argtypes = [C.c_void_p, _d, _d]
        L.pabd_oracle_body_mass.argtypes = [C.c_int32, _d, C.c_double, _d, _d]
        L.pabd_oracle_polar.argtypes = [_d, _d]
        L.pabd_oracle_dense_H.argtypes = [C.c_void_p, C.c_int32, _d]
        L.pabd_oracle_contacts.argtypes = [C.c_void_p, C.c_int32, _i, _i, _i, _d, _d, _d, _d]
        L.pabd_oracle_detect.argtypes = [C.c_void_p]
        L.pabd_oracle_detect_body.argtypes = [C.c_void_p, C.c_int32]
        L.pabd_oracle_bond_state.argtypes = [C.c_void_p, _d, _d]
        L.pabd_oracle_poly_split.argtypes = [C.c_double, C.c_int32, C.c_double, C.c_double, _d, _d]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(_P(t)) if a is not None and a.size else None


def poly_split(kappa: float, p: int, l: float, d: float):
    """(w, phim) of a polynomial bond: implicit weight phi^+ / d and explicit phi^-."""
    w, pm = C.c_double(), C.c_double()
    lib().pabd_oracle_poly_split(kappa, p, l, d, C.byref(w), C.byref(pm))
    return w.value, pm.value


def body_mass(shape: int, param, density: float):
    p = np.ascontiguousarray(np.asarray(param, dtype=np.float64).reshape(3))
    m = np.zeros(1)
    Pi = np.zeros(9)
    lib().pabd_oracle_body_mass(shape, _ptr(p, C.c_double), float(density), _ptr(m, C.c_double),
                                _ptr(Pi, C.c_double))
    return float(m[0]), Pi.reshape(3, 3)


def polar(A) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(9))
    r = np.zeros(9)
    lib().pabd_oracle_polar(_ptr(a, C.c_double), _ptr(r, C.c_double))
    return r.reshape(3, 3)


class Oracle:
    """One scene simulated by the FP64 oracle."""

    def __init__(self, scene):
        s = scene.normalized()
        self._keep = s  # arrays must outlive create (they are copied there, but be safe)
        d = _Desc()
        d.n_bodies = s.n_bodies
        d.shape = _ptr(s.shape, C.c_int32)
        d.shape_param = _ptr(s.shape_param, C.c_double)
        d.density = _ptr(s.density, C.c_double)
        d.flags = _ptr(s.flags, C.c_uint8)
        d.group = _ptr(s.group, C.c_int32)
        d.c0 = _ptr(s.c0, C.c_double)
        d.A0 = _ptr(s.A0, C.c_double)
        d.v0 = _ptr(s.v0, C.c_double)
        d.w0 = _ptr(s.w0, C.c_double)
        d.n_bonds = s.n_bonds
        d.bond_i = _ptr(s.bond_i, C.c_int32)
        d.bond_j = _ptr(s.bond_j, C.c_int32)
        d.bond_type = _ptr(s.bond_type, C.c_int32)
        d.x_i = _ptr(s.x_i, C.c_double)
        d.x_j = _ptr(s.x_j, C.c_double)
        d.kappa = _ptr(s.kappa, C.c_double)
        d.rest_len = _ptr(s.rest_len, C.c_double)
        d.drive = _ptr(s.drive, C.c_double)
        d.gravity = (C.c_double * 3)(*s.gravity.tolist())
        d.h = s.h
        d.t0 = s.t0
        d.iters = s.iters
        d.contact_enable = s.contact_enable
        d.mu = s.mu
        d.contact_kappa_scale = s.contact_kappa_scale
        d.contact_margin = s.contact_margin
        d.n_planes = s.planes.shape[0]
        d.planes = _ptr(s.planes, C.c_double)
        d.al_beta = s.al_beta
        d.al_alpha = s.al_alpha
        d.al_gamma = s.al_gamma
        d.order = _ptr(s.order, C.c_int32)
        d.mass = _ptr(s.mass, C.c_double)
        d.Pi0 = _ptr(s.Pi0, C.c_double)
        self.n = s.n_bodies
        self.n_bonds = s.n_bonds
        self.iters = s.iters
        self._h = lib().pabd_oracle_create(C.byref(d))
        if not self._h:
            raise ValueError("oracle rejected the scene description")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().pabd_oracle_destroy(h)
            self._h = None

    def step(self, nsteps: int = 1) -> None:
        if lib().pabd_oracle_step(self._h, int(nsteps)) != 0:
            raise FloatingPointError("oracle state became non-finite")

    def state(self):
        c = np.zeros((self.n, 3)); A = np.zeros((self.n, 3, 3))
        v = np.zeros((self.n, 3)); w = np.zeros((self.n, 3))
        lib().pabd_oracle_read_state(self._h, _ptr(c, C.c_double), _ptr(A, C.c_double),
                                     _ptr(v, C.c_double), _ptr(w, C.c_double))
        return c, A, v, w

    def residuals(self) -> np.ndarray:
        r = np.zeros(self.iters)
        lib().pabd_oracle_residuals(self._h, _ptr(r, C.c_double), self.iters)
        return r

    def set_debug(self, flags: int) -> None:
        lib().pabd_oracle_set_debug(self._h, int(flags))

    def last_iterates(self):
        a = np.zeros((self.n, 12)); b = np.zeros((self.n, 12))
        lib().pabd_oracle_last_iterates(self._h, _ptr(a, C.c_double), _ptr(b, C.c_double))
        return a, b

    def dense_H(self, body: int) -> np.ndarray:
        H = np.zeros(144)
        lib().pabd_oracle_dense_H(self._h, int(body), _ptr(H, C.c_double))
        return H.reshape(12, 12)

    def bond_state(self):
        """(kappa_j, lambda_j) of every bond after the last step (augmented bonds;
        others report kappa and 0)."""
        k = np.zeros(self.n_bonds)
        lam = np.zeros(self.n_bonds)
        if self.n_bonds:
            lib().pabd_oracle_bond_state(self._h, _ptr(k, C.c_double), _ptr(lam, C.c_double))
        return k, lam

    def detect(self) -> int:
        return int(lib().pabd_oracle_detect(self._h))

    def detect_body(self, body: int) -> int:
        """Contacts involving one body on the current state (O(N)); read them with
        contacts().  Replaces the stored contact set."""
        n = int(lib().pabd_oracle_detect_body(self._h, int(body)))
        if n < 0:
            raise IndexError(body)
        return n

    def contacts(self):
        """Contact bonds of the last detection: dict of arrays."""
        n = lib().pabd_oracle_contacts(self._h, 0, None, None, None, None, None, None, None)
        ci = np.zeros(n, np.int32); cj = np.zeros(n, np.int32); ft = np.zeros(n, np.int32)
        xi = np.zeros((n, 3)); xj = np.zeros((n, 3)); nn = np.zeros((n, 3)); kk = np.zeros(n)
        if n:
            lib().pabd_oracle_contacts(self._h, n, _ptr(ci, C.c_int32), _ptr(cj, C.c_int32),
                                       _ptr(ft, C.c_int32), _ptr(xi, C.c_double),
                                       _ptr(xj, C.c_double), _ptr(nn, C.c_double),
                                       _ptr(kk, C.c_double))
        return dict(i=ci, j=cj, feature=ft, x_i=xi, x_j=xj, normal=nn, kappa=kk)


def run(scene, steps: int):
    """Convenience: simulate ``steps`` steps and return the final state."""
    o = Oracle(scene)
    o.step(steps)
    return o.state()
