"""Error metric for GPU-vs-oracle parity (shared by the GPU tests and bench).

Relative position error: max over bodies of |c - c_ref| / L, L the diagonal of
the initial bounding box of the body centres (at least 1 m); rotation error:
max over bodies of |A - A_ref|_F / sqrt(3); velocity errors relative to the
largest reference speed (at least 1 m/s or 1 rad/s)."""
import numpy as np


def scale_of(scene) -> float:
    c = np.asarray(scene.c0)
    if len(c) == 0:
        return 1.0
    return max(1.0, float(np.linalg.norm(c.max(0) - c.min(0))))


def errors(state, ref, L: float):
    c, A, v, w = state
    cr, Ar, vr, wr = ref
    if len(c) == 0:
        return dict(pos=0.0, rot=0.0, vel=0.0, omega=0.0)
    pos = float(np.linalg.norm(c - cr, axis=1).max() / L)
    rot = float(np.linalg.norm((A - Ar).reshape(len(A), 9), axis=1).max() / np.sqrt(3.0))
    vs = max(1.0, float(np.linalg.norm(vr, axis=1).max()))
    ws = max(1.0, float(np.linalg.norm(wr, axis=1).max()))
    vel = float(np.linalg.norm(v - vr, axis=1).max() / vs)
    om = float(np.linalg.norm(w - wr, axis=1).max() / ws)
    return dict(pos=pos, rot=rot, vel=vel, omega=om)


def worst(e) -> float:
    return max(e.values())


def fp64_ok(e, pos_tol: float = 1e-9, vel_tol: float = 1e-6) -> bool:
    """FP64 bar: positions and rotations to 1e-9 relative; velocities, which are
    difference quotients (c^{n+1} - c^n)/h and lose digits to that division, to
    1e-6 relative."""
    return e["pos"] <= pos_tol and e["rot"] <= pos_tol and e["vel"] <= vel_tol and e["omega"] <= vel_tol
