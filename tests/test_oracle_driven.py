"""Pins of the oracle's driven joint (a reading: the paper drives hinge angles
with a periodic function of time, Sec. 5.3.3, without printing the joint's
energy).  As read, a driven bond is a ball joint whose j-side anchor is a base
point turned about an axis through a pivot by theta(t) = theta0 + a sin(2 pi f t
+ phi), with t the time at the end of the step being taken.  So one step of a
driven bond must equal one step of a plain ball joint whose anchor is that
turned point, computed here with an independent rotation routine (scipy's
rotation vectors); the ball joint itself is pinned by the closed forms of
test_oracle_dynamics.py."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from paper_2609_02675_amd import scenes as S

AXIS = np.array([0.3, 0.8, -0.5]) / np.linalg.norm([0.3, 0.8, -0.5])
PIVOT = np.array([0.1, 0.2, -0.3])
BASE = np.array([0.6, 0.45, 0.1])
THETA0, AMP, FREQ, PHASE = 0.2, 0.35, 1.3, 0.4


def _target(t):
    th = THETA0 + AMP * math.sin(2.0 * math.pi * FREQ * t + PHASE)
    return PIVOT + Rotation.from_rotvec(th * AXIS).apply(BASE - PIVOT)


def _scene(world: bool, driven: bool, xj=None, kappa=2e4, iters=3):
    """A box (body 0) joined at a material point to the driven anchor: in the
    world (world=True), or in the material frame of a second, heavier box
    (body 1) that swings freely."""
    n = 1 if world else 2
    bd = S._bodies(n)
    bd["shape_param"][0] = (0.2, 0.3, 0.25)
    bd["density"][0] = 800.0
    bd["c0"][0] = (0.4, -0.2, 0.15)
    bd["A0"][0] = S.rot_axis((1, -2, 0.5), 0.6)
    bd["v0"][0] = (0.3, -0.1, 0.2)
    bd["w0"][0] = (0.5, 1.1, -0.7)
    if not world:
        bd["shape_param"][1] = (0.4, 0.4, 0.4)
        bd["density"][1] = 2000.0
        bd["c0"][1] = (-0.3, 0.5, 0.0)
        bd["A0"][1] = S.rot_axis((0.2, 1, 0.3), -0.4)
        bd["w0"][1] = (-0.2, 0.3, 0.6)
    bonds = S._empty_bonds(1)
    bonds["bond_i"][0] = 0
    bonds["bond_j"][0] = -1 if world else 1
    bonds["x_i"][0] = (0.1, 0.2, -0.05)
    bonds["kappa"][0] = kappa
    if driven:
        bonds["bond_type"][0] = S.BOND_DRIVEN
        bonds["drive"][0] = np.concatenate([AXIS, PIVOT, BASE, [THETA0, AMP, FREQ, PHASE]])
        bonds["x_j"][0] = BASE
    else:
        bonds["x_j"][0] = xj
    return S.SceneDesc(**bd, **bonds, iters=iters, precision=S.PREC_FP64)


def _check_steps_follow_the_target(world: bool):
    drv = oracle.Oracle(_scene(world, True))
    h = S.SceneDesc.h
    for n in range(6):
        t_end = (n + 1) * h
        # the same step with a ball joint to the turned point, from the same state
        ball = _scene(world, False, xj=_target(t_end)).with_state(*drv.state(), t0=n * h)
        ob = oracle.Oracle(ball)
        ob.step(1)
        drv.step(1)
        for x, y in zip(drv.state(), ob.state()):
            np.testing.assert_allclose(x, y, rtol=0, atol=1e-12)


def test_driven_world_anchor_is_a_ball_joint_to_the_turned_point():
    _check_steps_follow_the_target(world=True)


def test_driven_body_anchor_is_a_ball_joint_to_the_turned_material_point():
    _check_steps_follow_the_target(world=False)


def test_driven_anchor_moves_the_body():
    """The target moves by several centimetres over the steps checked, so the
    pins above compare states that the drive actually changes."""
    h = S.SceneDesc.h
    assert np.linalg.norm(_target(6 * h) - _target(h)) > 0.03
    still = oracle.Oracle(_scene(True, False, xj=_target(h)))
    drv = oracle.Oracle(_scene(True, True))
    still.step(6)
    drv.step(6)
    assert np.abs(still.state()[0] - drv.state()[0]).max() > 1e-3
