"""Seeded synthetic scene generators.

This module builds scene descriptions only: body shapes, densities, initial
poses and velocities, bond anchors and stiffnesses, contact settings.  It holds
none of the method's arithmetic (no mass or inertia, no dynamics); the HIP
library and the test oracle each derive everything else from these inputs.

The paper's own scenes (meshes, sand, water) are not available, so these
synthetic workloads stand in for them.  All randomness is NumPy PCG64 with an
explicit seed.

Shapes: 0 = box (shape_param = half extents), 1 = sphere (shape_param[0] = radius).
Body flags: bit0 = pinned (kinematic, infinite mass), bit1 = no contact.
Bond types: 0 = quadratic (rest length l; l = 0 is a ball joint),
            1 = driven ball joint (j-side anchor follows a target angle),
            3 = augmented Lagrangian, 4 = polynomial,
            5 = slider (point of i on a line of j; drive[0:3] is the line's axis).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SHAPE_BOX = 0
SHAPE_SPHERE = 1
FLAG_PINNED = 1
FLAG_NO_CONTACT = 2
BOND_QUADRATIC = 0
BOND_DRIVEN = 1
BOND_AUGMENTED = 3  # augmented Lagrangian (Sec. 5.2.2); kappa is kappa_start
BOND_POLYNOMIAL = 4  # Psi = kappa / p (d - l)^p, p = order (even >= 2)
# point-on-line bond: x_i of body i held on the line through x_j along the axis
# drive[0:3] (both in j's material frame, world if j = -1); rest length 0
BOND_SLIDER = 5

PREC_FP32 = 0
PREC_FP64 = 1


@dataclasses.dataclass
class SceneDesc:
    """Arrays are float64 / int32 / uint8 numpy arrays, row-major."""

    shape: np.ndarray          # [N] int32
    shape_param: np.ndarray    # [N,3]
    density: np.ndarray        # [N]
    flags: np.ndarray          # [N] uint8
    group: np.ndarray          # [N] int32
    c0: np.ndarray             # [N,3]
    A0: np.ndarray             # [N,3,3]
    v0: np.ndarray             # [N,3]
    w0: np.ndarray             # [N,3]
    bond_i: np.ndarray         # [B] int32
    bond_j: np.ndarray         # [B] int32 (-1 = world)
    bond_type: np.ndarray      # [B] int32
    x_i: np.ndarray            # [B,3]
    x_j: np.ndarray            # [B,3]
    kappa: np.ndarray          # [B]
    rest_len: np.ndarray       # [B]
    drive: np.ndarray          # [B,13]
    order: Optional[np.ndarray] = None  # [B] int32 polynomial order (polynomial bonds)
    # optional generalised mass replacing what density and shape give: mass [N],
    # Pi0 [N,6] packed symmetric (00, 01, 02, 11, 12, 22) in the material frame
    mass: Optional[np.ndarray] = None
    Pi0: Optional[np.ndarray] = None
    gravity: np.ndarray = dataclasses.field(default_factory=lambda: np.array([0.0, -9.81, 0.0]))
    h: float = 1.0 / 60.0
    t0: float = 0.0
    iters: int = 20
    contact_enable: int = 0
    mu: float = 0.5
    contact_kappa_scale: float = 0.3
    contact_margin: float = 0.01
    planes: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 4)))
    precision: int = PREC_FP64
    max_contacts_per_body: int = 64
    # augmented-Lagrangian constants (the paper's values, Sec. 5.2.2)
    al_beta: float = 1e4
    al_alpha: float = 0.99
    al_gamma: float = 0.999
    name: str = ""

    @property
    def n_bodies(self) -> int:
        return int(self.shape.shape[0])

    @property
    def n_bonds(self) -> int:
        return int(self.bond_i.shape[0])

    def copy(self, **changes) -> "SceneDesc":
        d = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}
        for k, v in d.items():
            if isinstance(v, np.ndarray):
                d[k] = v.copy()
        d.update(changes)
        return SceneDesc(**d)

    def with_state(self, c, A, v, w, t0: Optional[float] = None) -> "SceneDesc":
        """Same scene restarted from another state (e.g. a checkpoint)."""
        out = self.copy(c0=np.array(c, dtype=np.float64).reshape(-1, 3),
                        A0=np.array(A, dtype=np.float64).reshape(-1, 3, 3),
                        v0=np.array(v, dtype=np.float64).reshape(-1, 3),
                        w0=np.array(w, dtype=np.float64).reshape(-1, 3))
        if t0 is not None:
            out.t0 = float(t0)
        return out

    def normalized(self) -> "SceneDesc":
        """Contiguous arrays of the dtypes the C interfaces expect."""
        f64 = lambda a, shp: np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shp))
        i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))
        n, b = self.n_bodies, self.n_bonds
        return dataclasses.replace(
            self,
            shape=i32(self.shape), shape_param=f64(self.shape_param, (n, 3)),
            density=f64(self.density, (n,)),
            flags=np.ascontiguousarray(np.asarray(self.flags, dtype=np.uint8).reshape(-1)),
            group=i32(self.group), c0=f64(self.c0, (n, 3)), A0=f64(self.A0, (n, 3, 3)),
            v0=f64(self.v0, (n, 3)), w0=f64(self.w0, (n, 3)),
            bond_i=i32(self.bond_i), bond_j=i32(self.bond_j), bond_type=i32(self.bond_type),
            x_i=f64(self.x_i, (b, 3)), x_j=f64(self.x_j, (b, 3)), kappa=f64(self.kappa, (b,)),
            rest_len=f64(self.rest_len, (b,)), drive=f64(self.drive, (b, 13)),
            order=i32(self.order if self.order is not None else np.full(b, 2)),
            mass=None if self.mass is None else f64(self.mass, (n,)),
            Pi0=None if self.Pi0 is None else f64(self.Pi0, (n, 6)),
            gravity=f64(self.gravity, (3,)), planes=f64(self.planes, (-1, 4)))


def _empty_bonds(b: int):
    return dict(bond_i=np.zeros(b, np.int32), bond_j=np.zeros(b, np.int32),
                bond_type=np.zeros(b, np.int32), x_i=np.zeros((b, 3)), x_j=np.zeros((b, 3)),
                kappa=np.zeros(b), rest_len=np.zeros(b), drive=np.zeros((b, 13)))


def _bodies(n: int):
    return dict(shape=np.zeros(n, np.int32), shape_param=np.zeros((n, 3)), density=np.ones(n),
                flags=np.zeros(n, np.uint8), group=np.zeros(n, np.int32), c0=np.zeros((n, 3)),
                A0=np.tile(np.eye(3), (n, 1, 1)), v0=np.zeros((n, 3)), w0=np.zeros((n, 3)))


def rot_z(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_axis(axis, theta: float) -> np.ndarray:
    u = np.asarray(axis, dtype=np.float64)
    u = u / np.linalg.norm(u)
    K = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return np.eye(3) + math.sin(theta) * K + (1 - math.cos(theta)) * (K @ K)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed rotations (normalised Gaussian quaternions)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    x, y, z, w = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


# ---------------------------------------------------------------------------
# joint chains (the 8-body chain and the batched chains)
# ---------------------------------------------------------------------------

def chain(n: int, *, tilt_deg: float = 45.0, joint_angles_deg=None, kappa: float = 1e5,
          iters: int = 20, h: float = 1.0 / 60.0, origin=(0.0, 0.0, 0.0),
          precision: int = PREC_FP64, pin_top: bool = True, name: str = "") -> SceneDesc:
    """Chain of n unit cubes (1 kg: density 1) joined by ball joints at the face
    centres (0, -0.5, 0) of body k and (0, +0.5, 0) of body k+1, body 0 pinned.

    Body 0's axis is tilted by ``tilt_deg`` from the downward vertical in the x-y
    plane; joint k additionally turns body k+1 by ``joint_angles_deg[k]`` about z.
    """
    bd = _bodies(n)
    bd["shape_param"][:] = 0.5
    if pin_top:
        bd["flags"][0] = FLAG_PINNED
    bd["flags"] |= FLAG_NO_CONTACT
    ang = np.zeros(max(n - 1, 0)) if joint_angles_deg is None else np.asarray(joint_angles_deg, float)
    # every joint turns about z, so body k is turned by tilt + sum of the first k joint angles
    th = np.radians(tilt_deg + np.concatenate([[0.0], np.cumsum(ang)]))[:n]
    cth, sth = np.cos(th), np.sin(th)
    R = np.zeros((n, 3, 3))
    R[:, 0, 0], R[:, 0, 1], R[:, 1, 0], R[:, 1, 1], R[:, 2, 2] = cth, -sth, sth, cth, 1.0
    xa, xb = np.array([0.0, -0.5, 0.0]), np.array([0.0, 0.5, 0.0])
    # c_{k+1} = c_k + R_k x_a - R_{k+1} x_b
    step = (R[:-1] @ xa) - (R[1:] @ xb)
    c = np.zeros((n, 3))
    c[0] = np.asarray(origin, dtype=np.float64)
    if n > 1:
        c[1:] = c[0] + np.cumsum(step, axis=0)
    bd["c0"][:] = c
    bd["A0"][:] = R
    b = max(n - 1, 0)
    bonds = _empty_bonds(b)
    bonds["bond_i"][:] = np.arange(b, dtype=np.int32)
    bonds["bond_j"][:] = np.arange(1, b + 1, dtype=np.int32)
    bonds["x_i"][:] = xa
    bonds["x_j"][:] = xb
    bonds["kappa"][:] = kappa
    return SceneDesc(**bd, **bonds, h=h, iters=iters, precision=precision, name=name or f"chain{n}")


def mass_ratio_chain(n: int = 19, ratio: float = 1000.0, augmented: bool = True,
                     kappa: float = 1e4, rest: float = 0.1, iters: int = 10,
                     tilt_deg: float = 30.0, precision: int = PREC_FP64) -> SceneDesc:
    """The paper's mass-ratio chain (Sec. 5.2.2, Table 2): n unit cubes hanging
    from a pinned top cube by n - 1 distance constraints between face centres
    (rest length `rest`), the bottom cube `ratio` times heavier than the others,
    released at rest, the chain tilted `tilt_deg` from vertical.  With `augmented`
    the constraints are augmented-Lagrangian bonds with kappa_start = `kappa`;
    otherwise quadratic bonds of stiffness `kappa`.  Neither the mass ratio nor
    the rest length is printed in the paper (1000 and 0.1 m here)."""
    sc = chain(n, tilt_deg=tilt_deg, kappa=kappa, iters=iters, precision=precision,
               name=f"massratio{n}_{'al' if augmented else 'quad'}")
    # open every joint to its rest length along the chain axis
    axis = sc.A0[0] @ np.array([0.0, -1.0, 0.0])
    c0 = sc.c0 + rest * np.arange(n)[:, None] * axis[None, :]
    dens = sc.density.copy()
    dens[-1] = ratio
    bt = np.full(sc.n_bonds, BOND_AUGMENTED if augmented else BOND_QUADRATIC, np.int32)
    return sc.copy(c0=c0, density=dens, bond_type=bt, rest_len=np.full(sc.n_bonds, rest))


def spring_pair(order: int = 2, stretch: float = 2.0, rest: float = 1.0, kappa: float = 1e4,
                iters: int = 20, precision: int = PREC_FP64) -> SceneDesc:
    """Two unit cubes (1 kg) joined centre to centre by one spring of rest length
    `rest`, stretched to `stretch` times it, at rest, no gravity (the paper's
    two-box spring, Sec. 5.2.2): order 2 is the quadratic bond, higher even orders
    the polynomial bond kappa / p (d - l)^p."""
    bd = _bodies(2)
    bd["shape_param"][:] = 0.5
    bd["flags"][:] = FLAG_NO_CONTACT
    bd["c0"][0] = (-stretch * rest / 2, 0.0, 0.0)
    bd["c0"][1] = (stretch * rest / 2, 0.0, 0.0)
    bonds = _empty_bonds(1)
    bonds["bond_i"][0], bonds["bond_j"][0] = 0, 1
    bonds["kappa"][0] = kappa
    bonds["rest_len"][0] = rest
    bonds["bond_type"][0] = BOND_QUADRATIC if order == 2 else BOND_POLYNOMIAL
    return SceneDesc(**bd, **bonds, order=np.array([order], np.int32), gravity=np.zeros(3),
                     iters=iters, precision=precision, name=f"springpair_p{order}")


def spring_net(n: int = 11, order: int = 2, spacing: float = 1.0, size: float = 0.5,
               kappa: float = 1e4, pull: float = 0.3, iters: int = 20,
               precision: int = PREC_FP64) -> SceneDesc:
    """The paper's net (Sec. 5.2.2): an n x n grid of cubes (side `size`, 1000
    kg/m^3) in the x-y plane joined to their four neighbours by centre-to-centre
    springs of rest length `spacing` (2 n (n - 1) springs, 220 for n = 11).  Every
    cube starts pulled a fraction `pull` of the way towards the centre of the
    bottom edge, so the springs start stretched or compressed; the two top corners
    are pinned; gravity on.  The pull and the pins are readings (the paper shows
    the scene but does not list its parameters)."""
    ix, iy = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    grid = np.stack([ix.ravel(), iy.ravel()], axis=1).astype(np.float64)
    m = grid.shape[0]
    bd = _bodies(m)
    bd["shape_param"][:] = size / 2
    bd["density"][:] = 1000.0
    bd["flags"][:] = FLAG_NO_CONTACT
    rest_xy = np.stack([(grid[:, 0] - (n - 1) / 2) * spacing, grid[:, 1] * spacing], axis=1)
    target = np.array([0.0, 0.0])
    xy = rest_xy + pull * (target - rest_xy)
    top = grid[:, 1] == n - 1
    corner = top & ((grid[:, 0] == 0) | (grid[:, 0] == n - 1))
    xy[corner] = rest_xy[corner]
    bd["c0"][:, :2] = xy
    bd["flags"][corner] |= FLAG_PINNED
    idx = lambda a, b: a * n + b
    pairs = [(idx(a, b), idx(a + 1, b)) for a in range(n - 1) for b in range(n)] + \
            [(idx(a, b), idx(a, b + 1)) for a in range(n) for b in range(n - 1)]
    bonds = _empty_bonds(len(pairs))
    bonds["bond_i"][:] = [p[0] for p in pairs]
    bonds["bond_j"][:] = [p[1] for p in pairs]
    bonds["kappa"][:] = kappa
    bonds["rest_len"][:] = spacing
    bonds["bond_type"][:] = BOND_QUADRATIC if order == 2 else BOND_POLYNOMIAL
    return SceneDesc(**bd, **bonds, order=np.full(len(pairs), order, np.int32), iters=iters,
                     precision=precision, name=f"net{n}_p{order}")


def chain8(precision: int = PREC_FP64, tilt_deg: float = 45.0) -> SceneDesc:
    """8 unit cubes, 7 ball joints (kappa 1e5), body 0 pinned, g = 9.81, h = 1/60,
    20 iterations per step.  ``tilt_deg=10`` is the gentle, non-chaotic variant."""
    return chain(8, tilt_deg=tilt_deg, kappa=1e5, iters=20, precision=precision,
                 name=f"chain8_tilt{tilt_deg:g}")


def batched_chain_lengths(n_scenes: int, seed: int = 2, lo: int = 4, hi: int = 64) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=n_scenes)


def batched_chains(n_scenes: int = 4096, seed: int = 2, iters: int = 20,
                   precision: int = PREC_FP32, lo: int = 4, hi: int = 64,
                   max_angle_deg: float = 30.0) -> List[SceneDesc]:
    """Independent chains of U{lo..hi} unit cubes with ball joints at the face
    centres; every joint turned by U[-30, 30] degrees about z; top body pinned."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = rng.integers(lo, hi + 1, size=n_scenes)
    out = []
    for s, n in enumerate(lengths):
        ang = rng.uniform(-max_angle_deg, max_angle_deg, size=int(n) - 1)
        out.append(chain(int(n), tilt_deg=0.0, joint_angles_deg=ang, kappa=1e5, iters=iters,
                         precision=precision, name=f"chain{n}_s{s}"))
    return out


def merge(scenes: List[SceneDesc], name: str = "merged") -> SceneDesc:
    """Concatenate independent scenes into one scene (same h, iters, gravity)."""
    off = np.cumsum([0] + [s.n_bodies for s in scenes])
    cat = lambda k: np.concatenate([getattr(s, k) for s in scenes], axis=0)
    bi = np.concatenate([s.bond_i + off[i] for i, s in enumerate(scenes)])
    bj = np.concatenate([np.where(s.bond_j >= 0, s.bond_j + off[i], -1) for i, s in enumerate(scenes)])
    first = scenes[0]
    extra = {}
    for k in ("mass", "Pi0"):
        given = [getattr(s, k) is not None for s in scenes]
        if any(given):
            if not all(given):
                raise ValueError(f"merge: {k} given for some scenes only")
            extra[k] = cat(k)
    return first.copy(**extra,
        shape=cat("shape"), shape_param=cat("shape_param"), density=cat("density"),
        flags=cat("flags"), group=cat("group"), c0=cat("c0"), A0=cat("A0"), v0=cat("v0"),
        w0=cat("w0"), bond_i=bi.astype(np.int32), bond_j=bj.astype(np.int32),
        bond_type=cat("bond_type"), x_i=cat("x_i"), x_j=cat("x_j"), kappa=cat("kappa"),
        rest_len=cat("rest_len"), drive=cat("drive"),
        order=np.concatenate([s.order if s.order is not None else np.full(s.n_bonds, 2, np.int32)
                              for s in scenes]).astype(np.int32), name=name)


# ---------------------------------------------------------------------------
# box piles with contact and friction
# ---------------------------------------------------------------------------

def box_drop(n_side: int = 10, layers: Optional[int] = None, seed: int = 0, mu: float = 0.5,
             iters: int = 30, h: float = 1.0 / 60.0, spacing: float = 2.7,
             base_height: float = 2.0, precision: int = PREC_FP32, jitter: float = 0.1,
             max_contacts_per_body: int = 256, name: str = "") -> SceneDesc:
    """Boxes with side lengths U[0.5, 1.5] per axis, density 1000, on an
    n_side x layers x n_side lattice at ``spacing`` with +-jitter, uniformly random
    orientation, at rest, every box's lowest point at least ``base_height``
    above the ground plane y = 0.  n_side = 10, layers = 10 is the 1,000-box drop.

    Contact capacity: when such a pile lands, its boxes sink into each other and
    the speculative margin of the impact step (h |v|, about 0.25 m at 15 m/s)
    brings many vertices of neighbours into range; measured on the GPU over the
    landing of piles of 10 to 5,000 boxes, the most contact ends one box held
    grew with the pile, to 82 at 1,000 boxes and 217 at 4,200, hence 256."""
    layers = n_side if layers is None else layers
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_side * n_side * layers
    bd = _bodies(n)
    bd["shape"][:] = SHAPE_BOX
    bd["shape_param"][:] = 0.5 * rng.uniform(0.5, 1.5, size=(n, 3))
    bd["density"][:] = 1000.0
    bd["A0"][:] = random_rotations(rng, n)
    ix, iy, iz = np.meshgrid(np.arange(n_side), np.arange(layers), np.arange(n_side), indexing="ij")
    grid = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    lift = base_height + math.sqrt(3.0) * 0.75
    centre = np.array([(n_side - 1) * spacing / 2, 0.0, (n_side - 1) * spacing / 2])
    bd["c0"][:] = grid * spacing - centre + np.array([0.0, lift, 0.0])
    bd["c0"][:] += rng.uniform(-jitter, jitter, size=(n, 3))
    return SceneDesc(**bd, **_empty_bonds(0), h=h, iters=iters, contact_enable=1, mu=mu,
                     contact_kappa_scale=0.3, contact_margin=0.01,
                     planes=np.array([[0.0, 1.0, 0.0, 0.0]]), precision=precision,
                     max_contacts_per_body=max_contacts_per_body, name=name or f"boxdrop{n}")


def box_stack(n: int = 6, mass_ratio: float = 10.0, size: float = 1.0, gap: float = 0.0,
              mu: float = 0.5, iters: int = 30, precision: int = PREC_FP64,
              name: str = "") -> SceneDesc:
    """Axis-aligned stack of n cubes resting on the ground plane y = 0, each box
    ``mass_ratio`` times heavier than the one below it (bottom box density 100)."""
    bd = _bodies(n)
    bd["shape"][:] = SHAPE_BOX
    bd["shape_param"][:] = size / 2
    bd["density"][:] = 100.0 * mass_ratio ** np.arange(n)
    bd["c0"][:, 1] = size / 2 + np.arange(n) * (size + gap)
    return SceneDesc(**bd, **_empty_bonds(0), iters=iters, contact_enable=1, mu=mu,
                     planes=np.array([[0.0, 1.0, 0.0, 0.0]]), precision=precision,
                     name=name or f"stack{n}x{mass_ratio:g}")


def single_body(shape: int = SHAPE_BOX, half=(0.5, 0.5, 0.5), density: float = 1.0,
                c=(0.0, 0.0, 0.0), A=None, v=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0),
                gravity=(0.0, -9.81, 0.0), iters: int = 20, h: float = 1.0 / 60.0,
                precision: int = PREC_FP64) -> SceneDesc:
    bd = _bodies(1)
    bd["shape"][0] = shape
    bd["shape_param"][0] = half
    bd["density"][0] = density
    bd["c0"][0] = c
    if A is not None:
        bd["A0"][0] = A
    bd["v0"][0] = v
    bd["w0"][0] = w
    return SceneDesc(**bd, **_empty_bonds(0), gravity=np.asarray(gravity, float), iters=iters, h=h,
                     precision=precision, name="single")


def world_pendulum(ell: float = 0.5, theta0_deg: float = 0.0, kappa: float = 1e5,
                   h: float = 1.0 / 60.0, iters: int = 20, precision: int = PREC_FP64) -> SceneDesc:
    """Unit cube hung from the world point (0, 0, 0) by a ball joint at the
    material point (0, ell, 0), swung by theta0 about z."""
    bd = _bodies(1)
    bd["shape_param"][0] = 0.5
    R = rot_z(math.radians(theta0_deg))
    x = np.array([0.0, ell, 0.0])
    bd["A0"][0] = R
    bd["c0"][0] = -(R @ x)
    bonds = _empty_bonds(1)
    bonds["bond_i"][0], bonds["bond_j"][0] = 0, -1
    bonds["x_i"][0] = x
    bonds["kappa"][0] = kappa
    return SceneDesc(**bd, **bonds, h=h, iters=iters, precision=precision, name="pendulum")


def _slider_scene(bd, rows, gravity, iters, precision, name):
    bonds = _empty_bonds(len(rows))
    for e, (i, j, xi, xj, axis, kappa) in enumerate(rows):
        bonds["bond_i"][e], bonds["bond_j"][e], bonds["bond_type"][e] = i, j, BOND_SLIDER
        bonds["x_i"][e], bonds["x_j"][e], bonds["kappa"][e] = xi, xj, kappa
        bonds["drive"][e][:3] = axis
    return SceneDesc(**bd, **bonds, gravity=np.asarray(gravity, float), iters=iters,
                     precision=precision, name=name)


def slider_rail(kappa: float = 1e5, deg: float = 30.0, iters: int = 20,
                precision: int = PREC_FP64) -> SceneDesc:
    """A 1 kg cube (half extent 5 cm) on a world rail down a `deg` incline in
    the x-y plane (gravity -y): its points +-5 cm along the rail held on the
    rail's line through the origin, its point 5 cm along z on the parallel line
    through (0, 0, 5 cm).  Returns the scene; the rail's direction is
    (cos deg, -sin deg, 0)."""
    u = np.array([math.cos(math.radians(deg)), -math.sin(math.radians(deg)), 0.0])
    bd = _bodies(1)
    bd["shape_param"][0] = 0.05
    bd["density"][0] = 1000.0
    rows = [(0, -1, 0.05 * u, (0, 0, 0), u, kappa), (0, -1, -0.05 * u, (0, 0, 0), u, kappa),
            (0, -1, (0, 0, 0.05), (0, 0, 0.05), u, kappa)]
    return _slider_scene(bd, rows, (0.0, -9.81, 0.0), iters, precision, "slider_rail")


def slider_rod(kappa: float = 1e7, turn=None, iters: int = 100,
               precision: int = PREC_FP64) -> SceneDesc:
    """A 20 kg rod (2 m x 10 cm x 10 cm, centre at 0.25 m on x) threaded over
    two fixed points of a pinned body at x = -0.25 m and x = 1 m: slider bonds
    whose line is the rod's axis (material x through its centre), so the line
    side is the free body.  `turn` = (axis, angle) turns the whole scene (both
    frames and gravity) by one rotation."""
    R = np.eye(3) if turn is None else rot_axis(turn[0], turn[1])
    bd = _bodies(2)
    bd["flags"][0] = FLAG_PINNED
    bd["shape_param"][0] = 0.05
    bd["shape_param"][1] = (1.0, 0.05, 0.05)
    bd["density"][1] = 1000.0
    bd["c0"][1] = R @ np.array([0.25, 0.0, 0.0])
    bd["A0"][:] = R
    ex = (1.0, 0.0, 0.0)
    rows = [(0, 1, (-0.25, 0, 0), (0, 0, 0), ex, kappa), (0, 1, (1.0, 0, 0), (0, 0, 0), ex, kappa)]
    return _slider_scene(bd, rows, R @ np.array([0.0, -9.81, 0.0]), iters, precision, "slider_rod")


def slider_pair(kappa: float = 1e5, moving_along: bool = False, iters: int = 20,
                precision: int = PREC_FP64) -> SceneDesc:
    """Two free bodies and no gravity: a 1 kg cube whose point (2, 1, 0) cm is
    held on the axis (1, 0.2, 0) through the centre of a 10 kg rod (1 m x 10 cm x
    10 cm) turned by 0.4 rad about (0.2, 0.3, 1), starting on that axis 0.3 m
    from the rod's centre; both move and spin.  With
    `moving_along`, the cube instead sits on the unturned rod's axis at -0.6 m,
    sliding along it at 2 m/s with the rod at rest."""
    bd = _bodies(2)
    bd["shape_param"][0] = 0.05
    bd["shape_param"][1] = (0.5, 0.05, 0.05)
    bd["density"][:] = 1000.0
    if moving_along:
        bd["c0"][0] = (-0.6, 0.0, 0.0)
        bd["v0"][0] = (2.0, 0.0, 0.0)
        rows = [(0, 1, (0, 0, 0), (0, 0, 0), (1.0, 0.0, 0.0), kappa)]
    else:
        bd["A0"][1] = rot_axis((0.2, 0.3, 1.0), 0.4)
        u = np.array([1.0, 0.2, 0.0]) / math.hypot(1.0, 0.2)
        bd["c0"][0] = 0.3 * (bd["A0"][1] @ u) - np.array([0.02, 0.01, 0.0])
        bd["v0"][0] = (0.5, 1.0, -0.3)
        bd["w0"][0] = (0.2, -0.1, 0.4)
        bd["v0"][1] = (0.0, -0.1, 0.05)
        bd["w0"][1] = (0.0, 0.1, 0.3)
        rows = [(0, 1, (0.02, 0.01, 0), (0, 0, 0), (1.0, 0.2, 0.0), kappa)]
    return _slider_scene(bd, rows, (0.0, 0.0, 0.0), iters, precision, "slider_pair")


def linkage(kind: str = "slider", *, kappa: float = 1e5, crank: float = 0.2, rod: float = 0.6,
            theta0_deg: float = 60.0, rocker: float = 1.0, drive_amp_deg: Optional[float] = None,
            drive_freq: float = 0.5, iters: int = 20, h: float = 1.0 / 60.0,
            precision: int = PREC_FP64) -> SceneDesc:
    """The four-body linkage of Sec. 5.1 (Table 2): a pinned ground (body 0), a
    crank (1) hinged to the ground at the origin, a connecting rod (2) hinged to
    the crank's tip, and a 1 kg block (3) hinged to the rod's far end, all in the
    x-y plane with hinge axes along z and gravity along -y.  Each hinge is two
    ball bonds 5 cm either side of the axis point.

    kind "slider": the block slides on the ground's x axis (a slider crank),
    held by three slider bonds from its points (+-5 cm, 0, 0) and (0, 0, 5 cm)
    to lines along x.  kind "four_bar": the block is replaced by a rocker of
    the same mass hinged to the ground `rocker` below the rod's end (the slider
    crank is the four-bar linkage whose rocker is infinitely long).

    Crank and rod are boxes 4 cm thick of density 1000 (0.32 kg and 0.96 kg at
    the default lengths); the crank starts at theta0 from the x axis, every body
    at rest.  With drive_amp_deg, a driven bond turns the crank's tip about the
    pivot by amp sin(2 pi f t) from its start (stiffness kappa)."""
    th = math.radians(theta0_deg)
    p1 = crank * np.array([math.cos(th), math.sin(th), 0.0])
    p2 = np.array([crank * math.cos(th) + math.sqrt(rod * rod - (crank * math.sin(th)) ** 2), 0.0, 0.0])
    bd = _bodies(4)
    bd["flags"][:] = FLAG_NO_CONTACT
    bd["flags"][0] |= FLAG_PINNED
    bd["shape_param"][0] = 0.1
    bd["density"][:] = 1000.0

    def link(b, a, z, half):
        d = z - a
        bd["c0"][b] = 0.5 * (a + z)
        bd["A0"][b] = rot_z(math.atan2(d[1], d[0]))
        bd["shape_param"][b] = (half, 0.02, 0.02)

    link(1, np.zeros(3), p1, crank / 2)
    link(2, p1, p2, rod / 2)
    rows = []

    def hinge(i, j, xi, xj):
        for dz in (-0.05, 0.05):
            rows.append((i, j, BOND_QUADRATIC, np.add(xi, (0, 0, dz)), np.add(xj, (0, 0, dz)), np.zeros(13)))

    hinge(1, 0, (-crank / 2, 0, 0), (0, 0, 0))
    hinge(2, 1, (-rod / 2, 0, 0), (crank / 2, 0, 0))
    if kind == "slider":
        bd["c0"][3] = p2
        bd["shape_param"][3] = 0.05
        hinge(3, 2, (0, 0, 0), (rod / 2, 0, 0))
        axis = np.r_[1.0, 0.0, 0.0, np.zeros(10)]
        for xi, xj in (((0.05, 0, 0), (0, 0, 0)), ((-0.05, 0, 0), (0, 0, 0)),
                       ((0, 0, 0.05), (0, 0, 0.05))):
            rows.append((3, 0, BOND_SLIDER, np.asarray(xi, float), np.asarray(xj, float), axis))
    elif kind == "four_bar":
        pg = p2 - np.array([0.0, rocker, 0.0])
        link(3, pg, p2, rocker / 2)
        bd["density"][3] = 1.0 / (rocker * 0.04 * 0.04)  # 1 kg, as the block
        hinge(3, 2, (rocker / 2, 0, 0), (rod / 2, 0, 0))
        hinge(3, 0, (-rocker / 2, 0, 0), pg)
    else:
        raise ValueError(kind)
    if drive_amp_deg is not None:
        drive = np.r_[0.0, 0.0, 1.0, 0.0, 0.0, 0.0, p1, 0.0, math.radians(drive_amp_deg), drive_freq, 0.0]
        rows.append((1, 0, BOND_DRIVEN, np.array([crank / 2, 0.0, 0.0]), p1, drive))
    bonds = _empty_bonds(len(rows))
    for e, (i, j, t, xi, xj, dr) in enumerate(rows):
        bonds["bond_i"][e], bonds["bond_j"][e], bonds["bond_type"][e] = i, j, t
        bonds["x_i"][e], bonds["x_j"][e], bonds["drive"][e] = xi, xj, dr
    bonds["kappa"][:] = kappa
    return SceneDesc(**bd, **bonds, h=h, iters=iters, precision=precision, name=f"linkage_{kind}")


# ---------------------------------------------------------------------------
# serving requests (Poisson arrivals of chains and box piles)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    arrival_s: float
    scene: SceneDesc
    steps: int


def pile(n: int, seed: int, precision: int = PREC_FP32, iters: int = 30) -> SceneDesc:
    """A box pile of about n boxes as in the box drop, on a near-square lattice."""
    side = max(1, int(round(n ** (1.0 / 3.0))))
    layers = max(1, int(math.ceil(n / (side * side))))
    # contact capacity grows with the pile (the landing compresses taller piles
    # more, at higher impact speeds): at most 217 ends per body were measured on
    # piles of up to 4,200 boxes, but single piles of 1,900 to 4,900 boxes went
    # beyond 256
    ccap = 128 if n < 200 else (256 if n < 1000 else 512)
    full = box_drop(n_side=side, layers=layers, seed=seed, iters=iters, precision=precision,
                    max_contacts_per_body=ccap)
    keep = np.arange(n)
    return full.copy(shape=full.shape[keep], shape_param=full.shape_param[keep],
                     density=full.density[keep], flags=full.flags[keep], group=full.group[keep],
                     c0=full.c0[keep], A0=full.A0[keep], v0=full.v0[keep], w0=full.w0[keep],
                     name=f"pile{n}_s{seed}")


def block_pile(n_side: int = 50, layers: int = 50, size: float = 1.0, gap: float = 1e-3,
               seed: int = 0, mu: float = 0.5, iters: int = 20, tilt_deg: float = 0.5,
               precision: int = PREC_FP32) -> SceneDesc:
    """n_side x n_side x layers cubes of side `size` (density 1000) stacked on the
    plane y = 0 with `gap` between neighbours, each turned by a seeded random angle
    below `tilt_deg` about a random axis (so faces are not exactly parallel), at
    rest: every cube starts in resting contact with its neighbours.  50^3 = 125,000
    cubes stand in for the paper's 50^3 block pile (Table 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sp = size + gap
    ix, iy, iz = np.meshgrid(np.arange(n_side), np.arange(layers), np.arange(n_side), indexing="ij")
    grid = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    n = grid.shape[0]
    bd = _bodies(n)
    bd["shape"][:] = SHAPE_BOX
    bd["shape_param"][:] = size / 2
    bd["density"][:] = 1000.0
    bd["c0"][:, 0] = (grid[:, 0] - (n_side - 1) / 2) * sp
    bd["c0"][:, 1] = size / 2 + gap + grid[:, 1] * sp
    bd["c0"][:, 2] = (grid[:, 2] - (n_side - 1) / 2) * sp
    axes = rng.normal(size=(n, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    ang = np.radians(tilt_deg) * rng.uniform(0.0, 1.0, size=n)
    K = np.zeros((n, 3, 3))
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -axes[:, 2], axes[:, 1], -axes[:, 0]
    K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = axes[:, 2], -axes[:, 1], axes[:, 0]
    sa, ca = np.sin(ang)[:, None, None], np.cos(ang)[:, None, None]
    bd["A0"][:] = np.eye(3)[None] + sa * K + (1 - ca) * (K @ K)  # Rodrigues
    return SceneDesc(**bd, **_empty_bonds(0), iters=iters, contact_enable=1, mu=mu,
                     contact_kappa_scale=0.3, contact_margin=0.01,
                     planes=np.array([[0.0, 1.0, 0.0, 0.0]]), precision=precision,
                     max_contacts_per_body=96, name=f"blockpile{n}")


def serving_requests(rate_hz: float = 200.0, duration_s: float = 60.0, seed: int = 3,
                     n_lo: int = 8, n_hi: int = 5000, steps_lo: int = 60, steps_hi: int = 600,
                     precision: int = PREC_FP32, max_requests: Optional[int] = None) -> List[Request]:
    """Poisson arrivals; body counts log-uniform in [n_lo, n_hi]; half random
    chains (K = 20), half box piles (K = 30); U{steps_lo..steps_hi} steps each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s or (max_requests is not None and len(out) >= max_requests):
            break
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        sub = int(rng.integers(0, 2**31 - 1))
        if rng.uniform() < 0.5:
            r2 = np.random.Generator(np.random.PCG64(sub))
            ang = r2.uniform(-30.0, 30.0, size=n - 1)
            sc = chain(n, tilt_deg=0.0, joint_angles_deg=ang, iters=20, precision=precision,
                       name=f"req{len(out)}_chain{n}")
        else:
            sc = pile(n, seed=sub, precision=precision)
            sc.name = f"req{len(out)}_pile{n}"
        out.append(Request(arrival_s=t, scene=sc, steps=steps))
    return out


# ---------------------------------------------------------------------------
# legged robot on a granular bed
# ---------------------------------------------------------------------------

def granular_bed_quadruped(nx: int = 50, nz: int = 50, ny: int = 20, r: float = 0.01,
                           seed: int = 1, mu: float = 0.6, iters: int = 20,
                           precision: int = PREC_FP32, with_robot: bool = True,
                           gait_amp_deg: float = 20.0, gait_hz: float = 1.0,
                           joint_kappa: float = 2e4, drive_kappa: float = 5e3,
                           name: str = "") -> SceneDesc:
    """Spheres of radius r (density 1000) on an nx x ny x nz lattice at spacing
    2r(1 + 1e-3) with 1e-4 m jitter, inside a box of walls around the nx x nz
    footprint (1 x 1 m for 50 x 50 at r = 0.01) on the floor y = 0, plus a 13-body
    quadruped: torso box 0.6 x 0.15 x 0.3 m and four legs of three 0.05 x 0.15 x
    0.05 m links.  Each of the 12 revolute joints is two ball bonds at +-0.025 m on
    its hinge axis (z) plus a driven bond that pulls the child's centre to the
    parent point turned by theta(t) = amp sin(2 pi f t + phase) (trot phases).

    Under the method as read this bed does not stand: a body resting on a contact
    settles a gap of g h^2 (1/scale + m l^2/Pi) below it (the local step keeps the
    centre solved together with the stretched A), which for a sphere (l = r,
    Pi = m r^2/5) is g h^2 (1/scale + 5) = 22.7 mm at h = 1/60 and scale 0.3 --
    more than the radius.  The spheres sink through the floor and each other and
    the bed churns, so contact counts grow with time; the capacity is sized for
    the first tens of steps, which is the horizon it serves (parity and timing)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sp = 2 * r * (1 + 1e-3)
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    grid = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    ns = grid.shape[0]
    half_x, half_z = nx * sp / 2, nz * sp / 2
    cs = np.empty((ns, 3))
    cs[:, 0] = -half_x + sp / 2 + grid[:, 0] * sp
    cs[:, 1] = sp / 2 + grid[:, 1] * sp
    cs[:, 2] = -half_z + sp / 2 + grid[:, 2] * sp
    cs += rng.uniform(-1e-4, 1e-4, size=cs.shape)
    bodies = _bodies(ns)
    bodies["shape"][:] = SHAPE_SPHERE
    bodies["shape_param"][:, 0] = r
    bodies["density"][:] = 1000.0
    bodies["c0"][:] = cs
    bond_rows = []
    if with_robot:
        top = ny * sp
        th_, tw, td = 0.15, 0.6, 0.3
        link = np.array([0.025, 0.075, 0.025])
        leg_len = 3 * 0.15
        y_torso = top + leg_len + th_ / 2 + 0.01
        rb = _bodies(13)
        rb["shape"][:] = SHAPE_BOX
        rb["group"][:] = 1
        rb["density"][:] = 1000.0
        rb["shape_param"][0] = (tw / 2, th_ / 2, td / 2)
        rb["c0"][0] = (0.0, y_torso, 0.0)
        corners = [(0.25, 0.12), (0.25, -0.12), (-0.25, 0.12), (-0.25, -0.12)]  # FL FR BL BR
        phases = [0.0, math.pi, math.pi, 0.0]
        b = 1
        for leg, ((cx, cz), ph) in enumerate(zip(corners, phases)):
            parent, p_joint_local = 0, np.array([cx, -th_ / 2, cz])
            p_center = np.array([0.0, y_torso, 0.0])
            for seg in range(3):
                joint_world = p_center + p_joint_local
                child_center = joint_world - np.array([0.0, 0.075, 0.0])
                rb["shape_param"][b] = link
                rb["c0"][b] = child_center
                child_joint_local = np.array([0.0, 0.075, 0.0])
                for dz in (-0.025, 0.025):
                    bond_rows.append(dict(i=ns + b, j=ns + parent, type=BOND_QUADRATIC,
                                          xi=child_joint_local + [0, 0, dz],
                                          xj=p_joint_local + [0, 0, dz], kappa=joint_kappa))
                # driven bond: child centre to the parent point turned about z through the joint
                base = (child_center - p_center)
                drive = np.concatenate([[0.0, 0.0, 1.0], p_joint_local, base,
                                        [0.0, math.radians(gait_amp_deg) * (1.0 if seg < 2 else 0.5),
                                         gait_hz, ph + (math.pi / 2 if seg == 1 else 0.0)]])
                bond_rows.append(dict(i=ns + b, j=ns + parent, type=BOND_DRIVEN, xi=np.zeros(3),
                                      xj=base, kappa=drive_kappa, drive=drive))
                parent, p_center, p_joint_local = b, child_center, np.array([0.0, -0.075, 0.0])
                b += 1
        for k in bodies:
            bodies[k] = np.concatenate([bodies[k], rb[k]], axis=0)
    nb = len(bond_rows)
    bonds = _empty_bonds(nb)
    for e, row in enumerate(bond_rows):
        bonds["bond_i"][e], bonds["bond_j"][e], bonds["bond_type"][e] = row["i"], row["j"], row["type"]
        bonds["x_i"][e], bonds["x_j"][e], bonds["kappa"][e] = row["xi"], row["xj"], row["kappa"]
        if "drive" in row:
            bonds["drive"][e] = row["drive"]
    planes = np.array([[0.0, 1.0, 0.0, 0.0],
                       [1.0, 0.0, 0.0, -half_x], [-1.0, 0.0, 0.0, -half_x],
                       [0.0, 0.0, 1.0, -half_z], [0.0, 0.0, -1.0, -half_z]])
    return SceneDesc(**bodies, **bonds, iters=iters, contact_enable=1, mu=mu,
                     contact_kappa_scale=0.3, contact_margin=0.2 * r, planes=planes,
                     precision=precision, max_contacts_per_body=256,
                     name=name or f"bed{ns}{'_quadruped' if with_robot else ''}")


# ---------------------------------------------------------------------------
# cases of the local step's fallback and of a general generalised mass
# ---------------------------------------------------------------------------

def polar_fallback_body(kind: str = "flip", kappa: float = 1e7, iters: int = 2,
                        precision: int = PREC_FP64) -> SceneDesc:
    """One box (half extents 0.5, 0.4, 0.3; 0.48 kg) at rest, turned 0.7 rad about
    (0.3, -0.5, 0.8), no gravity, held by four stiff world bonds from the centres
    of its x and y faces.  "flip": the x anchors sit 2 m beyond the opposite
    faces and the y anchors 0.8 m beyond their own, so the global step turns A
    inside out along x and stretches it along y (det A^{k+1/2} < 0, singular
    values near 4, 3, 1).  "flat": both x anchors sit at the centre and the y
    anchors 0.1 m out, so A^{k+1/2} is nearly rank two (smallest singular value
    about 3e-7 at kappa = 1e9)."""
    bd = _bodies(1)
    bd["shape_param"][0] = (0.5, 0.4, 0.3)
    R = rot_axis((0.3, -0.5, 0.8), 0.7)
    bd["A0"][0] = R
    if kind == "flip":
        pairs = [((0.5, 0, 0), (-2.0, 0, 0)), ((-0.5, 0, 0), (2.0, 0, 0)),
                 ((0, 0.4, 0), (0, 1.2, 0)), ((0, -0.4, 0), (0, -1.2, 0))]
    elif kind == "flat":
        pairs = [((0.5, 0, 0), (0.0, 0, 0)), ((-0.5, 0, 0), (0.0, 0, 0)),
                 ((0, 0.4, 0), (0, 0.5, 0)), ((0, -0.4, 0), (0, -0.5, 0))]
    else:
        raise ValueError(kind)
    bonds = _empty_bonds(len(pairs))
    for e, (xi, yw) in enumerate(pairs):
        bonds["bond_i"][e], bonds["bond_j"][e] = 0, -1
        bonds["x_i"][e] = xi
        bonds["x_j"][e] = R @ np.asarray(yw, dtype=np.float64)
        bonds["kappa"][e] = kappa
    return SceneDesc(**bd, **bonds, gravity=np.zeros(3), iters=iters, precision=precision,
                     name=f"polar_{kind}")


def general_inertia_chain(n: int = 6, seed: int = 5, precision: int = PREC_FP64,
                          iters: int = 20) -> SceneDesc:
    """The chain of ``chain`` (top body pinned, 45 degrees) whose bodies carry an
    explicit mass and an affine moment Pi0 that no box or sphere has: a seeded
    symmetric positive definite matrix with off-diagonal terms (principal axes
    turned away from the material frame, moments in [0.02, 0.2] kg m^2) and
    masses in [0.5, 2] kg."""
    sc = chain(n, tilt_deg=45.0, kappa=1e5, iters=iters, precision=precision,
               name=f"geninertia{n}")
    rng = np.random.Generator(np.random.PCG64(seed))
    Q = random_rotations(rng, n)
    lam = rng.uniform(0.02, 0.2, size=(n, 3))
    P = np.einsum("nij,nj,nkj->nik", Q, lam, Q)
    pi0 = np.stack([P[:, 0, 0], P[:, 0, 1], P[:, 0, 2], P[:, 1, 1], P[:, 1, 2], P[:, 2, 2]], axis=1)
    return sc.copy(mass=rng.uniform(0.5, 2.0, size=n), Pi0=pi0)
