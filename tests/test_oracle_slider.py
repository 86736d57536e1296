"""Pins of the oracle's slider (point-on-line) bond, a reading of the slider
joints of Sec. 5.1 (the paper names them but prints no energy): the bond holds
a point of body i on a line of body j, and each iteration re-projects the
line-side anchor to the foot of the perpendicular from the point.

Held to what mechanics fixes: a block on a frictionless world rail falls along
it exactly as a free body falls along the rail's direction and settles at the
static sag of its two rail supports; a free rod resting on two fixed points
takes the lever-rule sag and tilt; a point slides freely along a free body's
line; the same scene turned as a whole turns its result; and the driven slider
crank of Table 2 follows its converged trajectory within the twenty iterations
the paper gives it."""
import math

import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S


@pytest.mark.parametrize("iters", [1, 20])
def test_block_on_an_incline_rail_falls_along_it_as_a_free_body(iters):
    # along the rail only g.u acts, and the prediction already has it, so each
    # step's axial position is that of a free fall along u (symplectic Euler from
    # rest: c_n.u = h^2 (g.u) n (n + 1) / 2) after any number of iterations
    sc = S.slider_rail(iters=iters)
    u = sc.drive[0, :3]
    o = oracle.Oracle(sc)
    g_ax = float(np.dot(sc.gravity, u))
    for n in range(1, 61):
        o.step(1)
        c, A, v, w = o.state()
        assert abs(c[0] @ u - sc.h ** 2 * g_ax * n * (n + 1) / 2) <= 1e-12 * max(1.0, n * n * sc.h ** 2 * g_ax)
        assert abs(v[0] @ u - n * sc.h * g_ax) <= 1e-11


def test_block_on_an_incline_rail_settles_at_the_static_sag():
    # across the rail: the two rail supports share the weight's normal part
    # m g_perp (the third support is offset along z, so balancing torques about
    # the centre leaves it unloaded), each sagging by delta = m |g_perp| / (2 kappa);
    # the block turns about the rail until the third point is back on its line
    kappa = 1e5
    sc = S.slider_rail(kappa=kappa, iters=60)
    u = sc.drive[0, :3]
    o = oracle.Oracle(sc)
    o.step(120)
    c, A, v, w = o.state()
    g = np.asarray(sc.gravity)
    g_perp = g - (g @ u) * u
    m = 1000.0 * 0.1 ** 3
    delta = m * np.linalg.norm(g_perp) / (2 * kappa)
    off = c[0] - (c[0] @ u) * u  # the centre's offset from the rail line
    np.testing.assert_allclose(off, delta * g_perp / np.linalg.norm(g_perp), rtol=0, atol=1e-4 * delta)

    def dist(x_mat, through):
        y = c[0] + A[0] @ np.asarray(x_mat, float) - np.asarray(through, float)
        return np.linalg.norm(y - (y @ u) * u)

    assert abs(dist(0.05 * u, (0, 0, 0)) - delta) <= 2e-3 * delta
    assert abs(dist(-0.05 * u, (0, 0, 0)) - delta) <= 2e-3 * delta
    assert dist((0, 0, 0.05), (0, 0, 0.05)) <= 2e-3 * delta
    assert np.linalg.norm(v[0] - (v[0] @ u) * u) <= 1e-6


@pytest.mark.parametrize("turned", [False, True])
def test_rod_on_two_fixed_points_takes_the_lever_rule_sag(turned):
    # a 20 kg rod (2 m long) resting through two fixed points at material
    # t1 = -0.5 and t2 = 0.75 along its axis: the supports' forces kappa
    # (delta - phi t_k) carry the weight with no net moment about the centre,
    #   2 delta - (t1 + t2) phi = m g / kappa,  (t1 + t2) delta - (t1^2 + t2^2) phi = 0,
    # for the centre's sag delta and the axis' tilt phi about z (small angles);
    # the line of this bond is the rod's, so this holds the line side's foot
    # point as the place where the force acts.  Turned: the whole scene (both
    # bodies' frames and gravity) turned by one rotation, whose result is the
    # same one turned (the axis lives in the rod's material frame)
    kappa = 1e7
    turn = ((0.3, -0.8, 0.5), 1.1) if turned else None
    R = S.rot_axis(*turn) if turned else np.eye(3)
    sc = S.slider_rod(kappa=kappa, turn=turn)
    o = oracle.Oracle(sc)
    o.step(60)
    c, A, v, w = o.state()
    c = c @ R  # back in the unturned frame: R^T c, R^T A
    A = np.einsum("ji,bjk->bik", R, A)
    m, g = 20.0, 9.81
    t1, t2 = -0.5, 0.75
    M = np.array([[2.0, -(t1 + t2)], [t1 + t2, -(t1 * t1 + t2 * t2)]])
    delta, phi = np.linalg.solve(M, [m * g / kappa, 0.0])
    assert abs(-c[1][1] - delta) <= 1e-3 * delta
    assert abs(math.atan2(A[1][1, 0], A[1][0, 0]) - phi) <= 1e-3 * abs(phi)
    # the rod slides down its tilt (g sin phi along the axis) by well under the
    # spacing of the supports
    assert abs(c[1][0] - 0.25) < 1e-3


def test_point_slides_freely_along_a_free_bodys_line():
    # no gravity, rod at rest, a block on the rod's axis moving along it: the
    # bond exerts nothing, the block keeps its speed and the rod stays put (a
    # ball joint in its place would drag the two together)
    sc = S.slider_pair(moving_along=True)
    o = oracle.Oracle(sc)
    o.step(30)
    c, A, v, w = o.state()
    np.testing.assert_allclose(c[0], (-0.6 + 30 * sc.h * 2.0, 0, 0), atol=1e-12)
    np.testing.assert_allclose(c[1], (0, 0, 0), atol=1e-12)
    np.testing.assert_allclose(v[1], 0, atol=1e-12)


def test_driven_slider_crank_follows_its_converged_trajectory_at_twenty_iterations():
    # Table 2 runs the linkage at 20 iterations.  With the crank driven
    # (60 degrees amplitude at 0.5 Hz, block stroke about 33 cm), the block at
    # K = 20 stays within 0.6 mm of the K = 1000 trajectory once the start from
    # rest has passed, and within 1.5 mm at its start; on the converged
    # trajectory it sits within 2 mm of the rigid linkage's kinematics
    sc = S.linkage("slider", drive_amp_deg=60.0)
    a = oracle.Oracle(sc.copy(iters=20))
    b = oracle.Oracle(sc.copy(iters=1000))
    r, L = 0.2, 0.6
    worst_late = worst_early = worst_kin = 0.0
    for n in range(120):
        a.step(1)
        b.step(1)
        ca, cb = a.state()[0], b.state()[0]
        Ab = b.state()[1]
        d = np.abs(ca - cb).max()
        if n < 10:
            worst_early = max(worst_early, d)
        else:
            worst_late = max(worst_late, d)
        th = math.atan2(Ab[1][1, 0], Ab[1][0, 0])
        worst_kin = max(worst_kin, abs(cb[3, 0] - (r * math.cos(th) + math.sqrt(L * L - (r * math.sin(th)) ** 2))))
    assert worst_late < 6e-4
    assert worst_early < 1.5e-3
    assert worst_kin < 2e-3
