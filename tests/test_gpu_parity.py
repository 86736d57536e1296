"""GPU parity of the plain path (one launch per iteration) against the FP64
oracle, through the C ABI.  FP64 mode: <= 1e-9 relative (position and rotation,
C-12 metric in tests/parity.py); FP32 mode: <= 1e-4 after one step, <= 1e-3
after 100 steps on non-chaotic scenes."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S
from parity import errors, fp64_ok, scale_of, worst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def run_both(P, sc, steps):
    print(f"[case] {sc.name} n={sc.n_bodies} steps={steps} prec={sc.precision}", flush=True)
    g = P.Scene(sc)
    g.step(steps)
    st = g.state()
    o = oracle.Oracle(sc)
    o.step(steps)
    return st, o.state(), g, o


def test_chain8_fp64_100_steps(P):
    sc = S.chain8(precision=S.PREC_FP64)
    st, ref, g, o = run_both(P, sc, 100)
    e = errors(st, ref, scale_of(sc))
    print("chain8 fp64", e)
    assert e["pos"] <= 1e-9 and e["rot"] <= 1e-9
    assert e["vel"] <= 1e-7 and e["omega"] <= 1e-7


@pytest.mark.parametrize("steps,tol", [(1, 1e-4), (100, 1e-3)])
def test_chain8_gentle_fp32(P, steps, tol):
    sc = S.chain8(precision=S.PREC_FP32, tilt_deg=10.0)
    st, ref, g, o = run_both(P, sc, steps)
    e = errors(st, ref, scale_of(sc))
    print(f"chain8 gentle fp32 after {steps}", e)
    assert e["pos"] <= tol and e["rot"] <= tol


def test_chain8_fp32_45deg_one_step(P):
    sc = S.chain8(precision=S.PREC_FP32)
    st, ref, g, o = run_both(P, sc, 1)
    e = errors(st, ref, scale_of(sc))
    print("chain8 fp32 one step", e)
    assert e["pos"] <= 1e-4 and e["rot"] <= 1e-4


def test_free_rotation_and_fall_fp64(P):
    sc = S.single_body(half=(0.2, 0.5, 0.3), w=(0.4, -3.0, 1.2), v=(1.0, 2.0, 0.0),
                       A=S.rot_axis((1, 1, 0), 0.7))
    st, ref, g, o = run_both(P, sc, 50)
    e = errors(st, ref, 1.0)
    assert worst(e) <= 1e-12


def test_springs_world_bonds_and_spin_fp64(P):
    rng = np.random.default_rng(3)
    sc = S.chain(4, tilt_deg=20.0, joint_angles_deg=[30.0, -40.0, 10.0], kappa=1e4, iters=7,
                 pin_top=False)
    sc = sc.copy(w0=rng.normal(0, 1.5, (4, 3)), v0=rng.normal(0, 1.0, (4, 3)))
    sc = sc.copy(bond_i=np.r_[sc.bond_i, 0, 3].astype(np.int32),
                 bond_j=np.r_[sc.bond_j, 2, -1].astype(np.int32),
                 bond_type=np.r_[sc.bond_type, 0, 0].astype(np.int32),
                 x_i=np.r_[sc.x_i, [[0.3, 0.1, -0.2], [0.1, -0.5, 0.2]]],
                 x_j=np.r_[sc.x_j, [[-0.2, 0.4, 0.1], sc.c0[3] + [0.1, -0.6, 0.2]]],
                 kappa=np.r_[sc.kappa, 2e3, 5e3], rest_len=np.r_[sc.rest_len, 0.7, 0.0],
                 drive=np.zeros((sc.n_bonds + 2, 13)))
    st, ref, g, o = run_both(P, sc, 40)
    e = errors(st, ref, scale_of(sc))
    print("springs fp64", e)
    assert worst(e) <= 1e-9


def test_global_step_only_fp64(P):
    """Local step switched off: one step only, since without rigidification A
    leaves SO(3) and the two sides' rotation handling (quaternion read-off and
    explicit inverse in the oracle, rotation update and transpose on the GPU)
    is defined for rotations only."""
    sc = S.chain(4, tilt_deg=30.0, joint_angles_deg=[10.0, -20.0, 15.0], kappa=3e3, iters=50)
    g = P.Scene(sc)
    g.set_debug(1)
    g.step(1)
    o = oracle.Oracle(sc)
    o.set_debug(1)
    o.step(1)
    e = errors(g.state(), o.state(), scale_of(sc))
    assert e["pos"] <= 1e-9 and e["rot"] <= 1e-9


def test_residual_history_fp64(P):
    sc = S.chain8(precision=S.PREC_FP64)
    g = P.Scene(sc)
    g.set_debug(2)  # record rho_k of every iteration
    g.step(5)
    o = oracle.Oracle(sc)
    o.step(5)
    np.testing.assert_allclose(g.residuals(), o.residuals(), rtol=1e-6)


def test_residual_last_iteration_fp64(P):
    sc = S.chain8(precision=S.PREC_FP64)
    g = P.Scene(sc)
    g.step(5)
    o = oracle.Oracle(sc)
    o.step(5)
    assert g.residuals()[-1] == pytest.approx(o.residuals()[-1], rel=1e-6)


def test_driven_joint_fp64(P):
    """A box hung from the world by a ball joint whose world anchor is driven
    around a circle: the j-side anchor follows theta(t)."""
    sc = S.world_pendulum(ell=0.5, theta0_deg=0.0, kappa=1e5)
    drive = np.zeros((1, 13))
    drive[0, :3] = (0, 0, 1)        # axis
    drive[0, 3:6] = (0.2, 0, 0)     # pivot
    drive[0, 6:9] = (0.0, 0, 0)     # base (initial anchor)
    drive[0, 9:] = (0.0, 0.6, 1.0, 0.3)
    sc = sc.copy(bond_type=np.array([S.BOND_DRIVEN], np.int32), drive=drive)
    st, ref, g, o = run_both(P, sc, 60)
    assert fp64_ok(errors(st, ref, 1.0))


def test_empty_and_all_pinned_scenes(P):
    empty = S.chain(1, pin_top=False).copy(
        shape=np.zeros(0, np.int32), shape_param=np.zeros((0, 3)), density=np.zeros(0),
        flags=np.zeros(0, np.uint8), group=np.zeros(0, np.int32), c0=np.zeros((0, 3)),
        A0=np.zeros((0, 3, 3)), v0=np.zeros((0, 3)), w0=np.zeros((0, 3)))
    g = P.Scene(empty)
    g.step(3)
    assert g.state()[0].shape == (0, 3)
    pinned = S.chain(3).copy(flags=np.full(3, S.FLAG_PINNED | S.FLAG_NO_CONTACT, np.uint8))
    g = P.Scene(pinned)
    g.step(5)
    c, A, v, w = g.state()
    np.testing.assert_array_equal(c, pinned.c0)
    assert np.all(v == 0) and np.all(w == 0)


def test_invalid_descriptions_are_rejected(P):
    bad = S.chain8().copy(h=-1.0)
    with pytest.raises(P.PabdError):
        P.Scene(bad)
    bad = S.chain8()
    bad.bond_j[0] = 99
    with pytest.raises(P.PabdError):
        P.Scene(bad)
    bad = S.chain8().copy(iters=0)
    with pytest.raises(P.PabdError):
        P.Scene(bad)


def test_fault_injection_reports_divergence(P):
    sc = S.chain8(precision=S.PREC_FP32)
    g = P.Scene(sc)
    g.step(2)
    g.poke(3, 0, float("nan"))
    g.step(1)
    with pytest.raises(P.Diverged):
        g.state()


def test_chain_ragged_sizes_fp64(P):
    """Chains of sizes around the 256-thread block boundary (ragged tails)."""
    for n in (1, 2, 255, 257):
        sc = S.chain(n, tilt_deg=30.0, joint_angles_deg=np.linspace(-20, 20, max(n - 1, 0)),
                     precision=S.PREC_FP64, iters=10)
        st, ref, g, o = run_both(P, sc, 3)
        assert fp64_ok(errors(st, ref, scale_of(sc))), n
