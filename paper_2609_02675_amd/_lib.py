"""ctypes binding of libpabd.so (include/pabd.h): argument marshalling only.

Every step of the simulation runs in the HIP library; this module converts
numpy scene descriptions into the C descriptor and arrays back.  It raises
immediately when the built library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional

import numpy as np

from .scenes import SceneDesc

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpabd.so")

PABD_OK, PABD_E_INVALID, PABD_E_OOM, PABD_E_DEVICE, PABD_E_DIVERGED, PABD_E_BUSY, PABD_E_NOTFOUND = (
    0, -1, -2, -3, -4, -5, -6)

SYMBOLS = [
    "pabd_last_error", "pabd_device_count", "pabd_scene_create", "pabd_scene_destroy",
    "pabd_scene_step", "pabd_scene_read_state", "pabd_scene_residuals", "pabd_scene_contacts",
    "pabd_scene_bytes", "pabd_scene_set_debug", "pabd_scene_poke", "pabd_scene_stream",
    "pabd_batch_create", "pabd_batch_destroy", "pabd_batch_admit", "pabd_batch_step",
    "pabd_batch_steps",
    "pabd_batch_poll", "pabd_batch_read_state", "pabd_batch_residual", "pabd_batch_release",
    "pabd_batch_steps_done", "pabd_batch_autotune", "pabd_batch_set_tile", "pabd_batch_stream",
    "pabd_batch_memory", "pabd_batch_time_tile_kernel", "pabd_batch_layout",
    "pabd_hbm_copy_probe", "pabd_batch_sync", "pabd_scene_bond_state", "pabd_set_allocator",
    "pabd_scene_residual", "pabd_debug_poke", "pabd_scene_polar_fallbacks", "pabd_batch_faults",
    "pabd_batch_poke", "pabd_batch_polar_fallbacks", "pabd_scene_run_noalloc",
    "pabd_batch_tune", "pabd_batch_set_schedule", "pabd_batch_get_schedule", "pabd_scene_tune",
    "pabd_scene_set_schedule", "pabd_scene_get_schedule", "pabd_tune_cache_clear",
    "pabd_tune_cache_size",
]

TUNE_FORCE = 1

_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class PabdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pabd status {status}: {msg}")
        self.status = status


class Busy(PabdError):
    pass


class Diverged(PabdError):
    pass


_P = C.POINTER
_d = _P(C.c_double)
_i = _P(C.c_int32)


class _Schedule(C.Structure):
    _fields_ = [("tile_bodies", C.c_int32), ("contact_lanes", C.c_int32),
                ("group_waves", C.c_int32), ("from_cache", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def _schedule(tile_bodies: int = 0, contact_lanes: int = 4, group_waves: int = 1) -> _Schedule:
    return _Schedule(int(tile_bodies), int(contact_lanes), int(group_waves), 0)


class _Desc(C.Structure):
    _fields_ = [
        ("n_bodies", C.c_int32), ("shape", _i), ("shape_param", _d), ("density", _d),
        ("flags", _P(C.c_uint8)), ("group", _i), ("c0", _d), ("A0", _d), ("v0", _d), ("w0", _d),
        ("n_bonds", C.c_int32), ("bond_i", _i), ("bond_j", _i), ("bond_type", _i),
        ("x_i", _d), ("x_j", _d), ("kappa", _d), ("rest_len", _d), ("drive", _d),
        ("gravity", C.c_double * 3), ("h", C.c_double), ("t0", C.c_double), ("iters", C.c_int32),
        ("contact_enable", C.c_int32), ("mu", C.c_double), ("contact_kappa_scale", C.c_double),
        ("contact_margin", C.c_double), ("n_planes", C.c_int32), ("planes", _d),
        ("max_contacts_per_body", C.c_int32), ("precision", C.c_int32),
        ("al_beta", C.c_double), ("al_alpha", C.c_double), ("al_gamma", C.c_double),
        ("order", _i), ("mass", _d), ("Pi0", _d),
    ]


_lib = None


def lib():
    """Load the built library; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run python paper_2609_02675_amd/build.py first")
    # PyTorch ships its own HIP runtime and exports its symbols globally; loading it
    # first makes the library bind to that same runtime, so a process that also
    # uses torch (streams, events, its allocator) has one HIP runtime, not two
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.pabd_last_error.restype = C.c_char_p
    L.pabd_device_count.restype = C.c_int32
    L.pabd_scene_create.argtypes = [_P(_Desc), _P(vp)]
    L.pabd_scene_destroy.argtypes = [vp]
    L.pabd_scene_step.argtypes = [vp, C.c_int32, vp]
    L.pabd_scene_read_state.argtypes = [vp, _d, _d, _d, _d]
    L.pabd_scene_residuals.argtypes = [vp, _d, C.c_int32, _i]
    L.pabd_scene_contacts.argtypes = [vp, C.c_int32, _i, _i, _i, _d, _d, _d, _d, _i]
    L.pabd_scene_bond_state.argtypes = [vp, _d, _d]
    L.pabd_set_allocator.argtypes = [_ALLOC_T, _FREE_T, vp]
    L.pabd_scene_bytes.argtypes = [_P(_Desc)]
    L.pabd_scene_bytes.restype = C.c_size_t
    L.pabd_scene_set_debug.argtypes = [vp, C.c_int32]
    L.pabd_scene_poke.argtypes = [vp, C.c_int32, C.c_int32, C.c_double]
    L.pabd_scene_stream.argtypes = [vp]
    L.pabd_scene_stream.restype = vp
    L.pabd_batch_create.argtypes = [C.c_int32, C.c_size_t, C.c_int32, _P(vp)]
    L.pabd_batch_destroy.argtypes = [vp]
    L.pabd_batch_admit.argtypes = [vp, _P(_Desc), C.c_int32, _i]
    L.pabd_batch_step.argtypes = [vp, vp]
    L.pabd_batch_steps.argtypes = [vp, C.c_int32, vp]
    L.pabd_batch_poll.argtypes = [vp, _i, C.c_int32, _i]
    L.pabd_batch_read_state.argtypes = [vp, C.c_int32, _d, _d, _d, _d]
    L.pabd_batch_residual.argtypes = [vp, C.c_int32, _d]
    L.pabd_batch_release.argtypes = [vp, C.c_int32]
    L.pabd_batch_steps_done.argtypes = [vp, C.c_int32, _i]
    L.pabd_batch_autotune.argtypes = [vp, _i]
    L.pabd_batch_set_tile.argtypes = [vp, C.c_int32]
    L.pabd_batch_stream.argtypes = [vp]
    L.pabd_batch_stream.restype = vp
    L.pabd_batch_memory.argtypes = [vp, _P(C.c_size_t), _P(C.c_size_t)]
    L.pabd_batch_time_tile_kernel.argtypes = [vp, C.c_int32, C.c_int32, _d]
    L.pabd_batch_layout.argtypes = [vp, _i, _i, _i]
    L.pabd_hbm_copy_probe.argtypes = [C.c_size_t, C.c_int32, _d, _d]
    L.pabd_batch_sync.argtypes = [vp]
    L.pabd_scene_residual.argtypes = [vp, _d]
    L.pabd_debug_poke.argtypes = [vp, C.c_int32, C.c_int32, C.c_double]
    _i64 = _P(C.c_int64)
    L.pabd_scene_polar_fallbacks.argtypes = [vp, _i64, _i64]
    L.pabd_batch_faults.argtypes = [vp, _i, _i, C.c_int32, _i]
    L.pabd_batch_poke.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double]
    L.pabd_batch_polar_fallbacks.argtypes = [vp, C.c_int32, _i64, _i64]
    L.pabd_scene_run_noalloc.argtypes = [_P(_Desc), C.c_int32, _d, _d, _d, _d, vp]
    for name in ("pabd_batch_tune", "pabd_scene_tune"):
        getattr(L, name).argtypes = [vp, C.c_int32, _P(_Schedule)]
    for name in ("pabd_batch_set_schedule", "pabd_batch_get_schedule", "pabd_scene_set_schedule",
                 "pabd_scene_get_schedule"):
        getattr(L, name).argtypes = [vp, _P(_Schedule)]
    L.pabd_tune_cache_clear.restype = None
    L.pabd_tune_cache_size.restype = C.c_int32
    _lib = L
    return L


def _check(status: int):
    if status == PABD_OK:
        return
    msg = lib().pabd_last_error().decode(errors="replace")
    if status == PABD_E_BUSY:
        raise Busy(status, msg)
    if status == PABD_E_DIVERGED:
        raise Diverged(status, msg)
    raise PabdError(status, msg)


def _ptr(a, t):
    return a.ctypes.data_as(_P(t)) if a is not None and a.size else None


class _Marshalled:
    """The C descriptor plus the numpy arrays it points into (kept alive)."""

    def __init__(self, scene: SceneDesc):
        s = scene.normalized()
        self.s = s
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
        d.max_contacts_per_body = s.max_contacts_per_body if s.contact_enable else 0
        d.precision = s.precision
        d.al_beta = s.al_beta
        d.al_alpha = s.al_alpha
        d.al_gamma = s.al_gamma
        d.order = _ptr(s.order, C.c_int32)
        d.mass = _ptr(s.mass, C.c_double)
        d.Pi0 = _ptr(s.Pi0, C.c_double)
        self.desc = d


_allocator_refs = None  # the callbacks must outlive every handle that uses them


def use_torch_allocator(enable: bool = True):
    """Route the device memory of scenes and batches created from now on through
    PyTorch's caching allocator (enable=False restores hipMalloc).  Handles keep
    the allocator they were created with."""
    global _allocator_refs
    if not enable:
        _check(lib().pabd_set_allocator(_ALLOC_T(), _FREE_T(), None))
        return
    import torch

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:  # out of memory: the library reports PABD_E_OOM
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    refs = (_ALLOC_T(_alloc), _FREE_T(_free))
    _check(lib().pabd_set_allocator(refs[0], refs[1], None))
    keep = [] if _allocator_refs is None else list(_allocator_refs)
    _allocator_refs = keep + [refs]


def device_count() -> int:
    return int(lib().pabd_device_count())


def tune_cache_clear():
    lib().pabd_tune_cache_clear()


def tune_cache_size() -> int:
    return int(lib().pabd_tune_cache_size())


def hbm_copy_probe(nbytes: int, reps: int = 20):
    """(GB/s of read + write traffic, average ms) of a device-wide streaming copy."""
    g, ms = np.zeros(1), np.zeros(1)
    _check(lib().pabd_hbm_copy_probe(int(nbytes), int(reps), _ptr(g, C.c_double), _ptr(ms, C.c_double)))
    return float(g[0]), float(ms[0])


def scene_bytes(scene: SceneDesc) -> int:
    m = _Marshalled(scene)
    return int(lib().pabd_scene_bytes(C.byref(m.desc)))


def _state_arrays(n):
    return np.zeros((n, 3)), np.zeros((n, 3, 3)), np.zeros((n, 3)), np.zeros((n, 3))


def run_noalloc(scene: SceneDesc, nsteps: int, stream: Optional[int] = None):
    """pabd_scene_run_noalloc: create, nsteps steps and read-back in one call,
    with no device allocation (the library's static scratch); returns (c, A, v, w)."""
    m = _Marshalled(scene)
    c, A, v, w = _state_arrays(scene.n_bodies)
    _check(lib().pabd_scene_run_noalloc(C.byref(m.desc), int(nsteps), _ptr(c, C.c_double), _ptr(A, C.c_double),
                                        _ptr(v, C.c_double), _ptr(w, C.c_double),
                                        C.c_void_p(stream) if stream else None))
    return c, A, v, w


class Scene:
    """One scene on the plain path (one kernel launch per iteration)."""

    def __init__(self, scene: SceneDesc):
        self.n = scene.n_bodies
        self.iters = scene.iters
        self._nb = scene.n_bonds
        m = _Marshalled(scene)
        h = C.c_void_p()
        _check(lib().pabd_scene_create(C.byref(m.desc), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pabd_scene_destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def stream(self) -> int:
        return int(lib().pabd_scene_stream(self._h) or 0)

    def step(self, nsteps: int = 1, stream: Optional[int] = None):
        _check(lib().pabd_scene_step(self._h, int(nsteps), C.c_void_p(stream) if stream else None))

    def state(self, check: bool = True):
        c, A, v, w = _state_arrays(self.n)
        st = lib().pabd_scene_read_state(self._h, _ptr(c, C.c_double), _ptr(A, C.c_double),
                                         _ptr(v, C.c_double), _ptr(w, C.c_double))
        if check:
            _check(st)
        return c, A, v, w

    def residuals(self) -> np.ndarray:
        out = np.zeros(self.iters)
        k = C.c_int32()
        _check(lib().pabd_scene_residuals(self._h, _ptr(out, C.c_double), self.iters, C.byref(k)))
        return out

    def residual(self) -> float:
        """FP64 residual of the last iteration of the last step."""
        r = np.zeros(1)
        _check(lib().pabd_scene_residual(self._h, _ptr(r, C.c_double)))
        return float(r[0])

    def polar_fallbacks(self):
        """(body-iterations whose local step took the SVD, those with det <= 0)."""
        a, b = C.c_int64(), C.c_int64()
        _check(lib().pabd_scene_polar_fallbacks(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_debug(self, flags: int):
        _check(lib().pabd_scene_set_debug(self._h, int(flags)))

    def poke(self, body: int, field: int, value: float):
        _check(lib().pabd_debug_poke(self._h, int(body), int(field), float(value)))

    def bond_state(self):
        """(kappa_j, lambda_j) of every bond after the last step."""
        k = np.zeros(self._nb)
        lam = np.zeros(self._nb)
        if self._nb:
            _check(lib().pabd_scene_bond_state(self._h, _ptr(k, C.c_double), _ptr(lam, C.c_double)))
        return k, lam

    def contacts(self):
        n = C.c_int32()
        _check(lib().pabd_scene_contacts(self._h, 0, None, None, None, None, None, None, None,
                                         C.byref(n)))
        k = n.value
        ci = np.zeros(k, np.int32); cj = np.zeros(k, np.int32); ft = np.zeros(k, np.int32)
        xi = np.zeros((k, 3)); xj = np.zeros((k, 3)); nn = np.zeros((k, 3)); kk = np.zeros(k)
        if k:
            _check(lib().pabd_scene_contacts(self._h, k, _ptr(ci, C.c_int32), _ptr(cj, C.c_int32),
                                             _ptr(ft, C.c_int32), _ptr(xi, C.c_double),
                                             _ptr(xj, C.c_double), _ptr(nn, C.c_double),
                                             _ptr(kk, C.c_double), C.byref(n)))
        return dict(i=ci, j=cj, feature=ft, x_i=xi, x_j=xj, normal=nn, kappa=kk)

    def schedule(self) -> dict:
        """Flat-path schedule in force (contact_lanes, group_waves; tile_bodies 0)."""
        sc = _Schedule()
        _check(lib().pabd_scene_get_schedule(self._h, C.byref(sc)))
        return sc.as_dict()

    def set_schedule(self, contact_lanes: int = 4, group_waves: int = 1):
        sc = _schedule(0, contact_lanes, group_waves)
        _check(lib().pabd_scene_set_schedule(self._h, C.byref(sc)))

    def tune(self, force: bool = False) -> dict:
        """Time the flat-path schedules from the saved state and keep the fastest."""
        sc = _Schedule()
        _check(lib().pabd_scene_tune(self._h, TUNE_FORCE if force else 0, C.byref(sc)))
        return sc.as_dict()


class Batch:
    """Many resident scenes advanced together, one graph replay per step."""

    def __init__(self, max_slots: int, hbm_budget: int, precision: int):
        h = C.c_void_p()
        _check(lib().pabd_batch_create(int(max_slots), int(hbm_budget), int(precision), C.byref(h)))
        self._h = h
        self._n = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().pabd_batch_destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def stream(self) -> int:
        return int(lib().pabd_batch_stream(self._h) or 0)

    def admit(self, scene: SceneDesc, nsteps: int) -> Optional[int]:
        """Slot of the admitted scene, or None if no slot / budget is free now."""
        m = _Marshalled(scene)
        slot = C.c_int32(-1)
        st = lib().pabd_batch_admit(self._h, C.byref(m.desc), int(nsteps), C.byref(slot))
        if st == PABD_E_BUSY:
            return None
        _check(st)
        self._n[slot.value] = scene.n_bodies
        return slot.value

    def step(self, stream: Optional[int] = None, nsteps: int = 1):
        """nsteps steps of every resident scene (pabd_batch_steps; one tile
        kernel launch runs all of them)."""
        s = C.c_void_p(stream) if stream else None
        if nsteps == 1:
            _check(lib().pabd_batch_step(self._h, s))
        else:
            _check(lib().pabd_batch_steps(self._h, int(nsteps), s))

    def sync(self):
        _check(lib().pabd_batch_sync(self._h))

    def poll(self) -> List[int]:
        cap = max(1, len(self._n))
        out = np.zeros(cap, np.int32)
        n = C.c_int32()
        _check(lib().pabd_batch_poll(self._h, _ptr(out, C.c_int32), cap, C.byref(n)))
        return out[: min(n.value, cap)].tolist()

    def state(self, slot: int, check: bool = True):
        c, A, v, w = _state_arrays(self._n[slot])
        st = lib().pabd_batch_read_state(self._h, int(slot), _ptr(c, C.c_double), _ptr(A, C.c_double),
                                         _ptr(v, C.c_double), _ptr(w, C.c_double))
        if check:
            _check(st)
        return c, A, v, w

    def residual(self, slot: int) -> float:
        r = np.zeros(1)
        _check(lib().pabd_batch_residual(self._h, int(slot), _ptr(r, C.c_double)))
        return float(r[0])

    def steps_done(self, slot: int) -> int:
        k = C.c_int32()
        _check(lib().pabd_batch_steps_done(self._h, int(slot), C.byref(k)))
        return k.value

    def release(self, slot: int):
        _check(lib().pabd_batch_release(self._h, int(slot)))
        self._n.pop(slot, None)

    def faults(self) -> dict:
        """{slot: health bits} of the resident scenes that failed (bit0 non-finite
        state, bit1 contact capacity overflow)."""
        cap = max(1, len(self._n))
        sl = np.zeros(cap, np.int32)
        co = np.zeros(cap, np.int32)
        n = C.c_int32()
        _check(lib().pabd_batch_faults(self._h, _ptr(sl, C.c_int32), _ptr(co, C.c_int32), cap, C.byref(n)))
        k = min(n.value, cap)
        return {int(a): int(b) for a, b in zip(sl[:k], co[:k])}

    def poke(self, slot: int, body: int, field: int, value: float):
        _check(lib().pabd_batch_poke(self._h, int(slot), int(body), int(field), float(value)))

    def polar_fallbacks(self, slot: int):
        a, b = C.c_int64(), C.c_int64()
        _check(lib().pabd_batch_polar_fallbacks(self._h, int(slot), C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self) -> int:
        t = C.c_int32()
        _check(lib().pabd_batch_autotune(self._h, C.byref(t)))
        return t.value

    def set_tile(self, tile_bodies: int):
        _check(lib().pabd_batch_set_tile(self._h, int(tile_bodies)))

    def schedule(self) -> dict:
        """Schedule in force: tile_bodies, contact_lanes, group_waves."""
        sc = _Schedule()
        _check(lib().pabd_batch_get_schedule(self._h, C.byref(sc)))
        return sc.as_dict()

    def set_schedule(self, tile_bodies: int = 0, contact_lanes: int = 4, group_waves: int = 1):
        sc = _schedule(tile_bodies, contact_lanes, group_waves)
        _check(lib().pabd_batch_set_schedule(self._h, C.byref(sc)))

    def tune(self, force: bool = False) -> dict:
        """Time tile sizes, then flat-path lanes and workgroup shapes, from the
        saved state; keep the fastest (cached per architecture, precision and
        size bucket)."""
        sc = _Schedule()
        _check(lib().pabd_batch_tune(self._h, TUNE_FORCE if force else 0, C.byref(sc)))
        return sc.as_dict()

    def time_tile_kernel(self, reps: int, nsteps: int = 1) -> float:
        """Average ms of one tile-kernel launch running nsteps steps."""
        ms = np.zeros(1)
        _check(lib().pabd_batch_time_tile_kernel(self._h, int(reps), int(nsteps), _ptr(ms, C.c_double)))
        return float(ms[0])

    def layout(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().pabd_batch_layout(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(bodies=a.value, tiles=b.value, tile_bodies=c.value)

    def memory(self):
        u, b = C.c_size_t(), C.c_size_t()
        _check(lib().pabd_batch_memory(self._h, C.byref(u), C.byref(b)))
        return u.value, b.value
