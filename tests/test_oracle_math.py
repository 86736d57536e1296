"""Pins of the oracle's building blocks against closed forms and independent
routes (quadrature, LAPACK, the paper's sparse inverse written out here).

The oracle is test infrastructure; these tests are what make it trustworthy.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S


def _gauss_box(he, f, n=4):
    """Gauss-Legendre quadrature of f(x) over the box [-he, he]^3 (exact for
    polynomials of degree <= 2n-1 per axis)."""
    t, w = np.polynomial.legendre.leggauss(n)
    tot = 0.0
    for a, wa in zip(t, w):
        for b, wb in zip(t, w):
            for c, wc in zip(t, w):
                x = np.array([a * he[0], b * he[1], c * he[2]])
                tot = tot + wa * wb * wc * f(x)
    return tot * he[0] * he[1] * he[2]


def _jac(x):
    J = np.zeros((3, 12))
    J[:, :3] = np.eye(3)
    for r in range(3):
        J[r, 3 + 3 * r:6 + 3 * r] = x
    return J


@pytest.mark.parametrize("he,rho", [((0.5, 0.5, 0.5), 1.0), ((0.3, 0.7, 0.45), 1000.0)])
def test_box_mass_and_affine_moment_match_quadrature(he, rho):
    """Theorem of Sec. 4.1.1: Pi = int rho x x^T dV (COM origin)."""
    m, Pi = oracle.body_mass(S.SHAPE_BOX, he, rho)
    mq = _gauss_box(he, lambda x: rho)
    Piq = _gauss_box(he, lambda x: rho * np.outer(x, x))
    assert m == pytest.approx(mq, rel=1e-13)
    np.testing.assert_allclose(Pi, Piq, rtol=1e-12, atol=1e-14 * m)


def test_sphere_mass_and_affine_moment_match_quadrature():
    r, rho = 0.37, 800.0
    m, Pi = oracle.body_mass(S.SHAPE_SPHERE, (r, 0, 0), rho)
    # spherical coordinates, Gauss-Legendre in radius and cos(polar), uniform in azimuth
    tr, wr = np.polynomial.legendre.leggauss(6)
    tu, wu = np.polynomial.legendre.leggauss(6)
    nphi = 16
    mq, Pq = 0.0, np.zeros((3, 3))
    for a, wa in zip(tr, wr):
        rr = 0.5 * r * (a + 1)
        for u, wuu in zip(tu, wu):
            s = math.sqrt(1 - u * u)
            for k in range(nphi):
                ph = 2 * math.pi * k / nphi
                x = rr * np.array([s * math.cos(ph), s * math.sin(ph), u])
                wgt = wa * 0.5 * r * wuu * (2 * math.pi / nphi) * rr * rr
                mq += rho * wgt
                Pq += rho * wgt * np.outer(x, x)
    assert m == pytest.approx(mq, rel=1e-12)
    np.testing.assert_allclose(Pi, Pq, rtol=1e-11, atol=1e-14 * m)


def test_generalised_mass_is_integral_of_JtJ():
    """M_i = int rho J^T J dV = diag(m I, Pi, Pi, Pi) (proof of the mass theorem);
    with no bonds the oracle's H_i is exactly M_i."""
    he, rho = (0.4, 0.25, 0.6), 500.0
    sc = S.single_body(half=he, density=rho, gravity=(0, 0, 0))
    o = oracle.Oracle(sc)
    o.step(1)
    Mq = _gauss_box(he, lambda x: rho * _jac(x).T @ _jac(x))
    np.testing.assert_allclose(o.dense_H(0), Mq, rtol=1e-12, atol=1e-12)


def _body_with_bonds(seed=0, nb=5):
    """One free body tied to the world by nb bonds at random anchors."""
    rng = np.random.default_rng(seed)
    sc = S.single_body(half=(0.3, 0.5, 0.4), density=700.0, gravity=(0, 0, 0))
    sc = sc.copy(bond_i=np.zeros(nb, np.int32), bond_j=-np.ones(nb, np.int32),
                 bond_type=np.zeros(nb, np.int32), x_i=rng.uniform(-0.5, 0.5, (nb, 3)),
                 x_j=rng.uniform(-1, 1, (nb, 3)), kappa=rng.uniform(1e3, 1e6, nb),
                 rest_len=np.zeros(nb), drive=np.zeros((nb, 13)))
    return sc


def test_dense_H_has_the_sparse_structure_and_closed_form_inverse():
    """Sec. 4.3: H_i = [[a I, e_k b^T], [b e_k^T, D]] with a = m + h^2 sum w,
    b = h^2 sum w x, D = Pi + h^2 sum w x x^T, and its inverse has the same
    structure with (1/a + a~), -g, D~^{-1}, g = D~^{-1} b~ (checked against LAPACK)."""
    sc = _body_with_bonds()
    o = oracle.Oracle(sc)
    o.step(1)
    H = o.dense_H(0)
    h2 = sc.h ** 2
    m, Pi = oracle.body_mass(S.SHAPE_BOX, sc.shape_param[0], sc.density[0])
    w, x = sc.kappa, sc.x_i
    a = m + h2 * w.sum()
    b = h2 * (w[:, None] * x).sum(0)
    D = Pi + h2 * np.einsum("k,ki,kj->ij", w, x, x)
    Hs = np.zeros((12, 12))
    Hs[:3, :3] = a * np.eye(3)
    for k in range(3):
        Hs[k, 3 + 3 * k:6 + 3 * k] = b
        Hs[3 + 3 * k:6 + 3 * k, k] = b
        Hs[3 + 3 * k:6 + 3 * k, 3 + 3 * k:6 + 3 * k] = D
    np.testing.assert_allclose(H, Hs, rtol=1e-13, atol=1e-12)
    bt = b / a
    Dt = D - np.outer(b, b) / a
    Dti = np.linalg.inv(Dt)
    g = Dti @ bt
    at = bt @ Dti @ bt
    Hi = np.zeros((12, 12))
    Hi[:3, :3] = (1 / a + at) * np.eye(3)
    for k in range(3):
        Hi[k, 3 + 3 * k:6 + 3 * k] = -g
        Hi[3 + 3 * k:6 + 3 * k, k] = -g
        Hi[3 + 3 * k:6 + 3 * k, 3 + 3 * k:6 + 3 * k] = Dti
    ref = np.linalg.inv(H)
    assert np.abs(Hi - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("seed", range(6))
def test_polar_matches_lapack_svd(seed):
    """Sec. 4.2.2: the local step keeps the rotation factor of A; for det <= 0 the
    nearest proper rotation U diag(1, 1, det(U V^T)) V^T."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3))
    if seed % 2:
        A = S.random_rotations(rng, 1)[0] @ (np.eye(3) + 0.05 * rng.standard_normal((3, 3)))
    if seed == 4:
        A[:, 2] *= -1  # improper
    U, s, Vt = np.linalg.svd(A)
    d = np.sign(np.linalg.det(U @ Vt))
    R = U @ np.diag([1, 1, d]) @ Vt
    Ro = oracle.polar(A)
    np.testing.assert_allclose(Ro, R, atol=2e-14)
    np.testing.assert_allclose(Ro @ Ro.T, np.eye(3), atol=1e-14)
    assert np.linalg.det(Ro) == pytest.approx(1.0, abs=1e-14)


def test_polar_of_near_singular_and_rotation():
    rng = np.random.default_rng(7)
    R0 = S.random_rotations(rng, 1)[0]
    np.testing.assert_allclose(oracle.polar(R0), R0, atol=1e-15)
    A = R0 @ np.diag([1.0, 0.5, 1e-14])
    Ro = oracle.polar(A)
    np.testing.assert_allclose(Ro @ Ro.T, np.eye(3), atol=1e-13)
    assert np.linalg.det(Ro) == pytest.approx(1.0, abs=1e-13)
    # maximises tr(R^T A) over rotations: better than random rotations
    best = np.trace(Ro.T @ A)
    for Q in S.random_rotations(rng, 200):
        assert np.trace(Q.T @ A) <= best + 1e-12


def test_given_affine_moment_is_frame_invariant():
    """A body's material frame is a choice: re-expressing a box in a frame turned
    by Q (x' = Q^T x) gives A' = A Q, Pi0' = Q^T Pi0 Q (off-diagonal in general)
    and anchors Q^T x, and must leave every world trajectory unchanged
    (Sec. 4.1.1: M = diag(m I, Pi0, Pi0, Pi0) acts on the rows of A).  The box
    moments come from density and shape in one run and are given explicitly,
    turned, in the other."""
    from paper_2609_02675_amd import scenes as S
    sc = S.chain(5, tilt_deg=35.0, kappa=1e5, iters=20).copy(
        w0=np.array([[0, 0, 0], [0.3, -0.2, 0.5], [0, 0.4, 0], [-0.6, 0, 0.1], [0.2, 0.2, 0.2]], float))
    sc.shape_param[:] = (0.5, 0.3, 0.2)
    rng = np.random.default_rng(7)
    Q = S.random_rotations(rng, sc.n_bodies)
    m = np.zeros(sc.n_bodies)
    pi = np.zeros((sc.n_bodies, 6))
    A1 = sc.A0.copy()
    for b in range(sc.n_bodies):
        mb, Pb = oracle.body_mass(S.SHAPE_BOX, sc.shape_param[b], sc.density[b])
        Pq = Q[b].T @ Pb @ Q[b]
        m[b], pi[b] = mb, (Pq[0, 0], Pq[0, 1], Pq[0, 2], Pq[1, 1], Pq[1, 2], Pq[2, 2])
        A1[b] = sc.A0[b] @ Q[b]
    xi = np.einsum("eji,ej->ei", Q[sc.bond_i], sc.x_i)
    xj = np.einsum("eji,ej->ei", Q[sc.bond_j], sc.x_j)
    turned = sc.copy(A0=A1, mass=m, Pi0=pi, x_i=xi, x_j=xj)
    assert np.abs(pi[:, [1, 2, 4]]).max() > 1e-3
    a, b = oracle.Oracle(sc), oracle.Oracle(turned)
    a.step(30)
    b.step(30)
    ca, Aa, va, wa = a.state()
    cb, Ab, vb, wb = b.state()
    np.testing.assert_allclose(cb, ca, atol=1e-12)
    np.testing.assert_allclose(Ab, Aa @ Q, atol=1e-12)
    np.testing.assert_allclose(vb, va, atol=1e-10)
    np.testing.assert_allclose(wb, wa, atol=1e-10)
