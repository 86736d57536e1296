"""Invariants of the oracle's contact bonds.  The paper's own contact and
friction energies are in its (unavailable) supplement, so the contact model is a
reading (contact bond with a stick anchor, normal gate and Coulomb clamp); these
tests pin what that reading must satisfy geometrically and physically.  Parity
with the paper's own contact model is unpinned."""
import math

import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S


def _verts(he):
    return np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)]) * he


def test_box_plane_contacts_are_the_vertices_within_the_margin():
    rng = np.random.default_rng(1)
    R = S.random_rotations(rng, 1)[0]
    sc = S.box_stack(n=1).copy(A0=R[None], c0=np.array([[0.2, 0.62, -0.1]]))
    o = oracle.Oracle(sc)
    o.detect()
    ct = o.contacts()
    y = sc.c0[0] + _verts(sc.shape_param[0]) @ R.T
    expect = sorted(np.nonzero(y[:, 1] < sc.contact_margin)[0].tolist())
    assert sorted(ct["feature"].tolist()) == expect
    assert np.all(ct["j"] == -1)
    for k, f in enumerate(ct["feature"]):
        np.testing.assert_allclose(ct["x_i"][k], _verts(sc.shape_param[0])[f], atol=1e-15)
        np.testing.assert_allclose(ct["x_j"][k], [y[f, 0], 0.0, y[f, 2]], atol=1e-14)


def _on_plane(shape, half, gap, v=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0)):
    """One body above the plane y = 0 with its lowest point at height gap."""
    sc = S.single_body(shape=shape, half=half, v=v, w=w, c=(0.0, half[0 if shape == S.SHAPE_SPHERE else 1] + gap, 0.0))
    return sc.copy(contact_enable=1, planes=np.array([[0.0, 1.0, 0.0, 0.0]]))


def _detected(sc):
    o = oracle.Oracle(sc)
    o.detect()
    return sorted(o.contacts()["feature"].tolist())


def test_detection_margin_grows_with_the_motion_of_the_step():
    """Detection on q^n looks ahead by the distance the surface can travel in the
    step, h (|v| + |w| R): a box whose bottom face is 0.04 above the margin is
    found when it falls at 3 m/s (h |v| = 0.05) or spins at 10 rad/s about y
    (h |w| R = 0.144 with R = |half extents|), not at rest; a sphere spinning in
    place is not found (its distance to the plane does not change)."""
    half = (0.5, 0.5, 0.5)
    m = S.SceneDesc.contact_margin
    gap = m + 0.04
    bottom = [0, 1, 4, 5]  # vertices with -half along y
    assert _detected(_on_plane(S.SHAPE_BOX, half, gap)) == []
    assert _detected(_on_plane(S.SHAPE_BOX, half, gap, v=(0.0, -3.0, 0.0))) == bottom
    assert _detected(_on_plane(S.SHAPE_BOX, half, gap, v=(0.0, 3.0, 0.0))) == bottom
    assert _detected(_on_plane(S.SHAPE_BOX, half, gap, w=(0.0, 10.0, 0.0))) == bottom
    assert _detected(_on_plane(S.SHAPE_BOX, half, m + 0.06, v=(0.0, -3.0, 0.0))) == []
    assert _detected(_on_plane(S.SHAPE_SPHERE, (0.5, 0.0, 0.0), gap, w=(0.0, 10.0, 0.0))) == []
    assert len(_detected(_on_plane(S.SHAPE_SPHERE, (0.5, 0.0, 0.0), gap, v=(0.0, -3.0, 0.0)))) == 1


def test_box_box_contacts_stop_at_the_lateral_extent_of_the_face():
    """Two unit cubes, the upper one 5 mm above the lower one's top face and
    shifted 0.9 m along x: its bottom face overlaps the lower top face over
    x in [0.4, 0.5] only, so of its four bottom vertices within the margin only
    the two at x = 0.4 become contacts, on the lower box's face with normal +y."""
    lo = S.single_body(c=(0.0, 0.0, 0.0))
    up = S.single_body(c=(0.9, 1.005, 0.0))
    sc = S.merge([lo, up]).copy(contact_enable=1)
    o = oracle.Oracle(sc)
    o.detect()
    ct = o.contacts()
    assert sorted(ct["feature"].tolist()) == [0, 4]  # -x and -y in the upper box's frame
    assert np.all(ct["i"] == 1) and np.all(ct["j"] == 0)
    np.testing.assert_allclose(ct["normal"], [[0.0, 1.0, 0.0]] * 2, atol=1e-15)


def test_sphere_sphere_contact_geometry():
    sc = S.single_body(shape=S.SHAPE_SPHERE, half=(0.3, 0, 0), density=500.0)
    sc = S.merge([sc, sc.copy(c0=np.array([[0.35, 0.4, 0.1]]), shape_param=np.array([[0.25, 0, 0]]))])
    sc = sc.copy(contact_enable=1, A0=np.stack([S.rot_z(0.3), S.rot_axis((1, 2, 3), 1.0)]))
    o = oracle.Oracle(sc)
    o.detect()
    ct = o.contacts()
    assert len(ct["i"]) == 1 and ct["i"][0] == 0 and ct["j"][0] == 1
    d = sc.c0[1] - sc.c0[0]
    n = -d / np.linalg.norm(d)
    np.testing.assert_allclose(ct["normal"][0], n, atol=1e-15)
    yi = sc.c0[0] + sc.A0[0] @ ct["x_i"][0]
    yj = sc.c0[1] + sc.A0[1] @ ct["x_j"][0]
    np.testing.assert_allclose(yi, sc.c0[0] - 0.3 * n, atol=1e-15)
    np.testing.assert_allclose(yj, sc.c0[1] + 0.25 * n, atol=1e-15)
    assert n @ (yi - yj) == pytest.approx(np.linalg.norm(d) - 0.55, abs=1e-14)


def test_aligned_box_stack_contacts_use_face_normals():
    sc = S.box_stack(n=2, mass_ratio=1.0)
    o = oracle.Oracle(sc)
    o.detect()
    ct = o.contacts()
    pair = ct["j"] >= 0
    assert pair.sum() == 4 and (~pair).sum() == 4
    for k in np.nonzero(pair)[0]:
        # vertex of the incident box on the reference face, normal along +-y
        assert abs(abs(ct["normal"][k][1]) - 1.0) < 1e-15


def test_box_at_rest_on_plane_stays_at_rest():
    sc = S.box_stack(n=1)
    o = oracle.Oracle(sc)
    o.step(240)
    c, A, v, w = o.state()
    assert np.abs(v).max() < 1e-6 and np.abs(w).max() < 1e-6
    np.testing.assert_allclose(A[0], np.eye(3), atol=1e-9)
    # Resting fixed point, in closed form.  With v = 0 the prediction is
    # s = (c + h^2 g, I); the global step gives m (c_hat - s_c) = h^2 f_total, so the
    # four vertex forces carry the weight (f_k = m g / 4 each), and
    # Pi_y (a2_hat - e2) = h^2 sum_k x_k,y f_k with x_k,y = -a and Pi_y = m a^2 / 3,
    # which stretches a2_hat by 3 h^2 g / a (a1, a3 stay: the vertex sums cancel).
    # The projection returns A = I and keeps c_hat, and each stick force
    # kappa_c (0 - y_k) = m g / 4 with kappa_c = scale m / h^2 fixes
    # c_y = a - 3 h^2 g - h^2 g / (4 scale).
    a, h, g, sc_k = 0.5, 1.0 / 60.0, 9.81, 0.3
    assert sc.contact_kappa_scale == sc_k and sc.h == h
    assert abs(c[0, 1] - (a - 3 * h * h * g - h * h * g / (4 * sc_k))) < 1e-9
    o.step(60)
    assert abs(o.state()[0][0, 1] - c[0, 1]) < 1e-7


def test_sphere_at_rest_on_plane_settles_at_the_closed_form_gap():
    """One contact at the sphere's lowest point x = (0, -r, 0): the weight m g is
    carried by the stick force, the column a2_hat is stretched by
    h^2 r m g / Pi = 5 h^2 g / r (Pi = m r^2 / 5), and the projection keeps c_hat,
    so the centre rests at r - g h^2 (1 / scale + 5).  At r = 1 cm and h = 1/60
    that is below the floor: the reason 1 cm spheres sink under the method."""
    r, h, g, k = 0.01, 1.0 / 60.0, 9.81, 0.3
    sc = S.single_body(shape=S.SHAPE_SPHERE, half=(r, 0, 0), density=1000.0,
                       c=(0, 0.95 * r, 0), h=h)
    sc = sc.copy(contact_enable=1, mu=0.5, planes=np.array([[0.0, 1.0, 0.0, 0.0]]),
                 max_contacts_per_body=8, contact_kappa_scale=k, contact_margin=0.2 * r)
    o = oracle.Oracle(sc)
    o.step(800)
    c, A, v, w = o.state()
    assert np.abs(v).max() < 1e-12
    assert abs(c[0, 1] - (r - g * h * h * (1.0 / k + 5.0))) < 1e-12


def _incline(theta_deg, mu):
    th = math.radians(theta_deg)
    n = np.array([-math.sin(th), math.cos(th), 0.0])
    R = S.rot_z(th)
    sc = S.box_stack(n=1, mu=mu).copy(planes=np.array([[n[0], n[1], n[2], 0.0]]),
                                      A0=R[None], c0=(R @ np.array([0, 0.5, 0]))[None])
    t_dir = np.array([math.cos(th), math.sin(th), 0.0])
    o = oracle.Oracle(sc)
    o.step(60)
    v1 = o.state()[2][0] @ t_dir
    o.step(60)
    v2 = o.state()[2][0] @ t_dir
    return (v2 - v1) / 1.0, v2


def test_incline_slip_accelerates_at_coulomb_rate():
    acc, _ = _incline(35.0, 0.5)
    th = math.radians(35.0)
    assert -acc == pytest.approx(9.81 * (math.sin(th) - 0.5 * math.cos(th)), rel=0.1)


def test_incline_below_friction_angle_does_not_accelerate():
    acc, v = _incline(20.0, 0.5)
    assert abs(acc) < 0.02 * 9.81 * math.sin(math.radians(20.0))
    assert abs(v) < 0.5  # bounded creep from the per-step anchor reset


def test_mass_ratio_stack_is_stable():
    """Six boxes, each ten times heavier than the one below (the paper's mass-ratio
    stack): it stays upright and settles."""
    sc = S.box_stack(n=6, mass_ratio=10.0)
    o = oracle.Oracle(sc)
    o.step(180)
    c, A, v, w = o.state()
    assert np.abs(v).max() < 0.2
    assert np.all(np.diff(c[:, 1]) > 0.8)
    assert np.abs(c[:, [0, 2]]).max() < 1e-6
    assert c[0, 1] > 0.4


def test_per_body_detection_is_the_full_detection_restricted_to_the_body():
    """The O(N) per-body query (used for sampled parity on large scenes) must
    return exactly the full brute-force contacts that involve the body."""
    sc = S.block_pile(n_side=4, layers=3, precision=S.PREC_FP64, tilt_deg=3.0)
    o = oracle.Oracle(sc)
    o.detect()
    full = o.contacts()
    assert len(full["i"]) > 0
    for b in range(sc.n_bodies):
        o.detect_body(b)
        mine = o.contacts()
        sel = (full["i"] == b) | (full["j"] == b)
        key_full = sorted(zip(full["i"][sel], full["j"][sel], full["feature"][sel]))
        key_mine = sorted(zip(mine["i"], mine["j"], mine["feature"]))
        assert key_full == key_mine
        order_f = np.lexsort((full["feature"][sel], full["j"][sel], full["i"][sel]))
        order_m = np.lexsort((mine["feature"], mine["j"], mine["i"]))
        np.testing.assert_array_equal(full["x_j"][sel][order_f], mine["x_j"][order_m])


_HE = np.array([0.3, 0.5, 0.7])
_RB = S.rot_axis((1.0, -0.4, 0.7), 0.9)
_RS = S.rot_axis((-0.3, 1.0, 0.2), 2.1)
_CB = np.array([0.4, 1.3, -0.2])
_R = 0.2


def _sphere_box(local_centre, box_first):
    """A sphere of radius 0.2 whose centre sits at `local_centre` in the material
    frame of a turned box with half extents (0.3, 0.5, 0.7); both at rest, so the
    detection margin of the pair is twice the base margin."""
    box = S.single_body(half=tuple(_HE), c=tuple(_CB), A=_RB)
    sph = S.single_body(shape=S.SHAPE_SPHERE, half=(_R, 0.0, 0.0), density=700.0,
                        c=tuple(_CB + _RB @ np.asarray(local_centre, float)), A=_RS)
    sc = S.merge([box, sph] if box_first else [sph, box]).copy(contact_enable=1)
    o = oracle.Oracle(sc)
    o.detect()
    return o.contacts(), (1 if box_first else 0), (0 if box_first else 1)


def _expect_contact(local_centre, closest, normal_local, box_first):
    ct, s, b = _sphere_box(local_centre, box_first)
    assert len(ct["i"]) == 1 and ct["i"][0] == s and ct["j"][0] == b
    n = _RB @ (np.asarray(normal_local, float) / np.linalg.norm(normal_local))
    np.testing.assert_allclose(ct["normal"][0], n, atol=1e-14)
    np.testing.assert_allclose(ct["x_j"][0], closest, atol=1e-14)
    # the sphere's point is its surface point facing the box: -r n in the world,
    # stored in the sphere's material frame
    np.testing.assert_allclose(_RS @ ct["x_i"][0], -_R * n, atol=1e-14)
    assert ct["feature"][0] == 8


@pytest.mark.parametrize("box_first", [True, False])
def test_sphere_box_contact_geometry_face_edge_corner(box_first):
    """Closed-form geometry of a sphere outside a box, 5 mm from its surface
    (inside the margin 2 x 0.01): against a face the closest point is the foot of
    the perpendicular and the normal the face normal; against an edge and a corner
    the closest point is the edge point or the vertex and the normal points from
    it to the sphere's centre."""
    g = 0.005
    _expect_contact((_HE[0] + _R + g, 0.1, -0.2), (_HE[0], 0.1, -0.2), (1, 0, 0), box_first)
    e = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    _expect_contact(np.array([_HE[0], _HE[1], 0.1]) + (_R + g) * e, (_HE[0], _HE[1], 0.1), e, box_first)
    k = np.array([1.0, -1.0, 1.0]) / math.sqrt(3.0)
    corner = np.array([_HE[0], -_HE[1], _HE[2]])
    _expect_contact(corner + (_R + g) * k, corner, k, box_first)


@pytest.mark.parametrize("box_first", [True, False])
def test_sphere_box_contact_inside_uses_the_nearest_face(box_first):
    """A sphere whose centre is inside the box, 0.05 from the +x face and further
    from every other face: the contact goes to that face (its foot point, its
    outward normal), although the centre is only 0.05 deep and the sphere's
    radius is 0.2."""
    _expect_contact((_HE[0] - 0.05, 0.1, -0.2), (_HE[0], 0.1, -0.2), (1, 0, 0), box_first)
    # just inside the -z face
    _expect_contact((0.05, -0.1, -_HE[2] + 0.02), (0.05, -0.1, -_HE[2]), (0, 0, -1), box_first)


def test_sphere_box_beyond_the_margin_has_no_contact():
    """3 cm from a face, an edge or a corner (beyond the pair's 2 cm margin) the
    sphere has no contact; 1.5 cm from them it has one."""
    for g, n_expect in ((0.03, 0), (0.015, 1)):
        assert len(_sphere_box((_HE[0] + _R + g, 0.1, -0.2), True)[0]["i"]) == n_expect
        e = np.array([0.0, 1.0, -1.0]) / math.sqrt(2.0)
        assert len(_sphere_box(np.array([0.1, _HE[1], -_HE[2]]) + (_R + g) * e, True)[0]["i"]) == n_expect
        k = np.array([-1.0, -1.0, -1.0]) / math.sqrt(3.0)
        assert len(_sphere_box(-_HE + (_R + g) * k, False)[0]["i"]) == n_expect
