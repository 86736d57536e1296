"""Pins of the oracle's time step against closed forms, brute-force dense solves
and exact identities of the method (prediction, global step, local step,
velocity recovery of Algorithm 1)."""
import math

import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S

G = np.array([0.0, -9.81, 0.0])


def test_free_fall_is_symplectic_euler():
    """No bonds: q = s every step; c_n = c_0 + n h v_0 + g h^2 n(n+1)/2 exactly."""
    v0 = np.array([1.0, 2.0, -0.5])
    sc = S.single_body(c=(0.3, 4.0, -1.0), v=v0)
    o = oracle.Oracle(sc)
    h = sc.h
    for n in (1, 7, 30):
        o2 = oracle.Oracle(sc)
        o2.step(n)
        c, A, v, w = o2.state()
        exp = np.array([0.3, 4.0, -1.0]) + n * h * v0 + G * h * h * n * (n + 1) / 2
        np.testing.assert_allclose(c[0], exp, atol=1e-13)
        np.testing.assert_allclose(v[0], v0 + n * h * G, atol=1e-12)
        np.testing.assert_allclose(A[0], np.eye(3), atol=1e-15)


def test_free_rotation_per_step_angle_and_omega_decay():
    """Quaternion prediction then velocity recovery: rotation by 2 atan(h|w|/2)
    about the fixed axis and |w_{n+1}| = |w_n| / (1 + h^2 |w_n|^2 / 4)."""
    w0 = np.array([0.4, -3.0, 1.2])
    R0 = S.rot_axis((1, 1, 0), 0.7)
    sc = S.single_body(half=(0.2, 0.5, 0.3), w=w0, A=R0, gravity=(0, 0, 0))
    o = oracle.Oracle(sc)
    h = sc.h
    R = R0.copy()
    wn = np.linalg.norm(w0)
    for _ in range(25):
        o.step(1)
        R = S.rot_axis(w0, 2 * math.atan(h * wn / 2)) @ R
        wn = wn / (1 + h * h * wn * wn / 4)
    c, A, v, w = o.state()
    np.testing.assert_allclose(A[0], R, atol=1e-13)
    assert np.linalg.norm(w[0]) == pytest.approx(wn, rel=1e-12)
    np.testing.assert_allclose(w[0] / np.linalg.norm(w[0]), w0 / np.linalg.norm(w0), atol=1e-12)


@pytest.mark.parametrize("kappa,ell", [(1e5, 0.5), (1e6, 0.5), (1e5, 0.3)])
def test_hanging_body_gap_closed_form(kappa, ell):
    """One body hanging at rest from a world point by a ball joint at offset ell:
    the fixed point of global + local keeps the translation solved together with a
    stretched A, so the joint gap is m g (1/kappa + h^2 ell^2 / Pi_ll), not m g/kappa."""
    sc = S.world_pendulum(ell=ell, kappa=kappa)
    o = oracle.Oracle(sc)
    o.step(900)
    c, A, v, w = o.state()
    y = c[0] + A[0] @ np.array([0.0, ell, 0.0])
    Pi_ll = 1.0 / 12.0
    gap = 9.81 * (1 / kappa + sc.h ** 2 * ell ** 2 / Pi_ll)
    assert np.linalg.norm(y) == pytest.approx(gap, rel=1e-9)
    np.testing.assert_allclose(A[0], np.eye(3), atol=1e-12)


def test_body_bonded_only_to_fixed_partners_converges_in_one_iteration():
    """The right-hand side of the body-wise update does not depend on the body's own
    q^k, so K = 1 and K = 20 give the same step."""
    sc = S.world_pendulum(ell=0.5, theta0_deg=25.0, kappa=1e5)
    sc = sc.copy(w0=np.array([[0.3, -0.2, 1.0]]), v0=np.array([[0.5, 0.0, 0.1]]))
    a = oracle.Oracle(sc.copy(iters=1)); a.step(5)
    b = oracle.Oracle(sc.copy(iters=20)); b.step(5)
    for x, y in zip(a.state(), b.state()):
        np.testing.assert_allclose(x, y, atol=1e-12)


def _jac(x):
    J = np.zeros((3, 12))
    J[:, :3] = np.eye(3)
    for r in range(3):
        J[r, 3 + 3 * r:6 + 3 * r] = x
    return J


def test_global_step_alone_converges_to_dense_solve():
    """With the local step switched off, the body-wise Jacobi update converges to
    the solution of the square 12N x 12N linear system of the semi-implicit global
    equation (ball joints: phi^- = 0), assembled densely here."""
    sc = S.chain(4, tilt_deg=30.0, joint_angles_deg=[10.0, -20.0, 15.0], kappa=3e3, iters=3000)
    o = oracle.Oracle(sc)
    o.set_debug(1)
    o.step(1)
    c, A, v, w = o.state()
    h2 = sc.h ** 2
    free = [b for b in range(sc.n_bodies) if not (sc.flags[b] & S.FLAG_PINNED)]
    idx = {b: k for k, b in enumerate(free)}
    n = len(free)
    K = np.zeros((12 * n, 12 * n))
    rhs = np.zeros(12 * n)
    q0 = np.concatenate([sc.c0, sc.A0.reshape(-1, 9)], axis=1)
    for b in free:
        m, Pi = oracle.body_mass(sc.shape[b], sc.shape_param[b], sc.density[b])
        M = np.zeros((12, 12))
        M[:3, :3] = m * np.eye(3)
        for k in range(3):
            M[3 + 3 * k:6 + 3 * k, 3 + 3 * k:6 + 3 * k] = Pi
        s = q0[b].copy()
        s[:3] += h2 * G  # at rest: s = (c + h^2 g, A)
        i = idx[b]
        K[12 * i:12 * i + 12, 12 * i:12 * i + 12] += M
        rhs[12 * i:12 * i + 12] += M @ s
    for e in range(sc.n_bonds):
        bi, bj, kap = sc.bond_i[e], sc.bond_j[e], sc.kappa[e]
        for self_, other, xs, xo in ((bi, bj, sc.x_i[e], sc.x_j[e]), (bj, bi, sc.x_j[e], sc.x_i[e])):
            if self_ not in idx:
                continue
            i = idx[self_]
            Js = _jac(xs)
            K[12 * i:12 * i + 12, 12 * i:12 * i + 12] += h2 * kap * Js.T @ Js
            if other in idx:
                j = idx[other]
                K[12 * i:12 * i + 12, 12 * j:12 * j + 12] -= h2 * kap * Js.T @ _jac(xo)
            else:
                y = xo if other < 0 else _jac(xo) @ q0[other]
                rhs[12 * i:12 * i + 12] += h2 * kap * Js.T @ y
    q = np.linalg.solve(K, rhs).reshape(n, 12)
    for b in free:
        np.testing.assert_allclose(c[b], q[idx[b], :3], atol=1e-11)
        np.testing.assert_allclose(A[b].reshape(9), q[idx[b], 3:], atol=1e-11)


def test_compound_pendulum_period():
    """Small swings of a unit cube hung from a face centre: T = 2 pi sqrt(I/(m g l)),
    I = 1/6 + 1/4 = 5/12 -> T = 1.8313 s.  Implicit Euler damps the swing, so the
    amplitude decreases monotonically."""
    sc = S.world_pendulum(ell=0.5, theta0_deg=5.0, kappa=1e6)
    o = oracle.Oracle(sc)
    h = sc.h
    th = []
    for _ in range(int(12.0 / h)):
        o.step(1)
        A = o.state()[1][0]
        th.append(math.atan2(A[1, 0], A[0, 0]))
    th = np.array(th)
    up = np.nonzero((th[:-1] < 0) & (th[1:] >= 0))[0]
    tz = (up + th[up] / (th[up] - th[up + 1])) * h  # linear interpolation
    T = np.diff(tz).mean()
    T_exact = 2 * math.pi * math.sqrt((5.0 / 12.0) / (9.81 * 0.5))
    assert T_exact == pytest.approx(1.8313, abs=1e-4)
    assert T == pytest.approx(T_exact, rel=0.01)
    peaks = [np.abs(th[a:b]).max() for a, b in zip(up[:-1], up[1:])]
    assert all(p1 < p0 for p0, p1 in zip(peaks, peaks[1:]))


def test_momentum_balance_identity():
    """Summing the translational rows of the last global update over all bodies:
    sum m (v^{n+1} - v^n - h g) = h sum_bonds [w (y_o^{K-1} - y_s^{K-1/2}) + phi^- n^{K-1}]
    over both ends of every bond (free ends only).  Holds to rounding for any K."""
    rng = np.random.default_rng(3)
    sc = S.chain(4, tilt_deg=20.0, joint_angles_deg=[30.0, -40.0, 10.0], kappa=1e4, iters=7,
                 pin_top=False)
    sc = sc.copy(w0=rng.normal(0, 1.5, (4, 3)), v0=rng.normal(0, 1.0, (4, 3)))
    # add a spring (l > 0) between bodies 0 and 2 and a ball joint of body 3 to the world
    sc = sc.copy(bond_i=np.r_[sc.bond_i, 0, 3].astype(np.int32),
                 bond_j=np.r_[sc.bond_j, 2, -1].astype(np.int32),
                 bond_type=np.r_[sc.bond_type, 0, 0].astype(np.int32),
                 x_i=np.r_[sc.x_i, [[0.3, 0.1, -0.2], [0.1, -0.5, 0.2]]],
                 x_j=np.r_[sc.x_j, [[-0.2, 0.4, 0.1], sc.c0[3] + [0.1, -0.6, 0.2]]],
                 kappa=np.r_[sc.kappa, 2e3, 5e3], rest_len=np.r_[sc.rest_len, 0.7, 0.0],
                 drive=np.zeros((sc.n_bonds + 2, 13)))
    o = oracle.Oracle(sc)
    o.step(3)
    c0, A0, v0, w0 = o.state()
    o.step(1)
    c1, A1, v1, w1 = o.state()
    qp, qh = o.last_iterates()
    h = sc.h
    m = np.array([oracle.body_mass(sc.shape[b], sc.shape_param[b], sc.density[b])[0]
                  for b in range(sc.n_bodies)])
    lhs = (m[:, None] * (v1 - v0 - h * G)).sum(0)
    y = lambda q, x: q[:3] + q[3:].reshape(3, 3) @ x
    rhs = np.zeros(3)
    for e in range(sc.n_bonds):
        bi, bj, kap, l = sc.bond_i[e], sc.bond_j[e], sc.kappa[e], sc.rest_len[e]
        for s_, o_, xs, xo in ((bi, bj, sc.x_i[e], sc.x_j[e]), (bj, bi, sc.x_j[e], sc.x_i[e])):
            if s_ < 0:
                continue
            yo_prev = xo if o_ < 0 else y(qp[o_], xo)
            ys_half = y(qh[s_], xs)
            rhs += h * kap * (yo_prev - ys_half)
            if l > 0:
                dv = yo_prev - y(qp[s_], xs)
                rhs += h * (-kap * l) * dv / np.linalg.norm(dv)
    np.testing.assert_allclose(lhs, rhs, atol=1e-9 * max(1.0, np.abs(lhs).max()))


def test_momentum_conserved_for_com_anchored_springs_at_convergence():
    """Springs anchored at the centres of mass, no gravity: at the fixed point of
    the iteration the bond forces cancel pairwise and momentum is conserved."""
    rng = np.random.default_rng(5)
    n = 5
    sc = S.chain(n, kappa=50.0, iters=400, pin_top=False)
    sc = sc.copy(x_i=np.zeros((n - 1, 3)), x_j=np.zeros((n - 1, 3)), rest_len=np.full(n - 1, 0.8),
                 v0=rng.normal(0, 1, (n, 3)), w0=rng.normal(0, 1, (n, 3)), gravity=np.zeros(3))
    m = 1.0
    o = oracle.Oracle(sc)
    p0 = (m * sc.v0).sum(0)
    o.step(30)
    p1 = (m * o.state()[2]).sum(0)
    np.testing.assert_allclose(p1, p0, atol=1e-11)


def test_spring_split_fixed_point_is_implicit_euler():
    """Two 1 kg bodies joined at their centres by a spring of rest length l
    stretched to 2 l: with phi^+ = kappa d, phi^- = -kappa l the converged step is
    the implicit Euler step m (x - x0)/h^2 = -kappa (2 x - l) of each half."""
    l, kap, h = 1.0, 300.0, 1.0 / 60.0
    sc = S.chain(2, kappa=kap, iters=300, pin_top=False)
    sc = sc.copy(c0=np.array([[-l, 0, 0], [l, 0, 0.0]]), A0=np.tile(np.eye(3), (2, 1, 1)),
                 x_i=np.zeros((1, 3)), x_j=np.zeros((1, 3)), rest_len=np.array([l]),
                 gravity=np.zeros(3))
    o = oracle.Oracle(sc)
    o.step(1)
    c = o.state()[0]
    x = (1.0 * l / h ** 2 + kap * l) / (1.0 / h ** 2 + 2 * kap)
    np.testing.assert_allclose(c[1], [x, 0, 0], atol=1e-12)
    np.testing.assert_allclose(c[0], [-x, 0, 0], atol=1e-12)


def test_residual_decreases_geometrically_on_chain():
    """rho_k = ||q^{k+1} - q^k||_M / ||q^k||_M falls geometrically with k on the
    8-body chain; the joint gap converges to the fixed point, not to zero."""
    sc = S.chain8()
    o = oracle.Oracle(sc.copy(iters=60))
    o.step(5)
    rho = o.residuals()
    assert np.all(np.diff(rho[5:]) < 0)
    ratios = rho[21:60] / rho[20:59]
    assert ratios.max() < 0.99 and ratios.max() - ratios.min() < 0.1
    assert rho[-1] < 1e-2 * rho[0]


@pytest.mark.parametrize("axis", [(1, 0, 0), (0, 1, 0), (0, 0, 1)], ids=["x", "y", "z"])
def test_free_rotation_from_a_large_turn_takes_each_quaternion_branch(axis):
    """The prediction of Algorithm 1 reads the quaternion of A^n off the rotation
    matrix by Shepperd's rule, which picks the largest of (A00, A11, A22, trace).
    A turn of 150 degrees about x, y or z makes that diagonal entry the largest,
    so each of the three non-trace branches is taken; a free body must still turn
    by 2 atan(h|w|/2) per step about the fixed axis w (P-5), with
    |w_{n+1}| = |w_n| / (1 + h^2 |w_n|^2 / 4)."""
    R0 = S.rot_axis(axis, math.radians(150.0))
    diag = [R0[0, 0], R0[1, 1], R0[2, 2], np.trace(R0)]
    assert int(np.argmax(diag)) == int(np.argmax(axis))
    w0 = np.array([0.9, -2.3, 1.4])
    sc = S.single_body(half=(0.2, 0.5, 0.3), w=w0, A=R0, gravity=(0, 0, 0))
    o = oracle.Oracle(sc)
    h = sc.h
    R = R0.copy()
    wn = np.linalg.norm(w0)
    for _ in range(8):
        o.step(1)
        R = S.rot_axis(w0, 2 * math.atan(h * wn / 2)) @ R
        wn = wn / (1 + h * h * wn * wn / 4)
        c, A, v, w = o.state()
        np.testing.assert_allclose(A[0], R, atol=1e-13)
        # still in the same branch of the read-off at the next step
        assert int(np.argmax([A[0][0, 0], A[0][1, 1], A[0][2, 2], np.trace(A[0])])) == int(np.argmax(axis))
    assert np.linalg.norm(w[0]) == pytest.approx(wn, rel=1e-12)
    np.testing.assert_allclose(w[0] / np.linalg.norm(w[0]), w0 / np.linalg.norm(w0), atol=1e-12)
