"""Pins of the oracle's polynomial bonds Psi = kappa / p (d - l)^p (the nonlinear
bonds of Sec. 4.2.1 and the spring experiments of Sec. 5.2.2)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_2609_02675_amd import scenes as S


def test_split_is_exact_and_sign_definite():
    """w d + phi^- = kappa (d - l)^{p-1} with w >= 0 and phi^- <= 0 for d, l >= 0
    (the split condition of Sec. 4.2.1); p = 2 is the quadratic split w = kappa,
    phi^- = -kappa l."""
    rng = np.random.default_rng(3)
    for p in (2, 4, 6, 8):
        for d, l in rng.uniform(0.0, 3.0, size=(50, 2)):
            w, pm = oracle.poly_split(2.5, p, l, d)
            assert w >= 0.0 and pm <= 0.0
            # exact up to the rounding of a sum of terms as large as kappa (d + l)^{p-1}
            scale = 2.5 * (d + l) ** (p - 1)
            assert abs(w * d + pm - 2.5 * (d - l) ** (p - 1)) <= 1e-14 * p * scale
    w, pm = oracle.poly_split(7.0, 2, 0.3, 1.9)
    assert (w, pm) == (7.0, -7.0 * 0.3)


def test_order_two_polynomial_is_the_quadratic_bond():
    quad = S.spring_net(order=2, iters=20)
    poly = quad.copy(bond_type=np.full(quad.n_bonds, S.BOND_POLYNOMIAL, np.int32))
    a, b = oracle.Oracle(quad), oracle.Oracle(poly)
    a.step(5)
    b.step(5)
    for x, y in zip(a.state(), b.state()):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-12)


@pytest.mark.parametrize("p,iters,tol", [(2, 400, 1e-12), (4, 400, 1e-12), (6, 4000, 1e-10)])
def test_spring_pair_converges_to_implicit_euler(p, iters, tol):
    """Two boxes on a centre-to-centre spring stretched to twice its rest length
    (the paper's two-box spring): with enough iterations the first step equals
    the implicit-Euler solution of the 1-D problem, found here by bracketing:
    each box moves by (d0 - d)/2, so m (d - d0) / (2 h^2) + kappa (d - l)^{p-1} = 0."""
    sc = S.spring_pair(order=p, iters=iters)
    o = oracle.Oracle(sc)
    o.step(1)
    c = o.state()[0]
    h, m, k, l, d0 = sc.h, 1.0, 1e4, 1.0, 2.0
    d_ref = brentq(lambda d: m * (d - d0) / (2 * h * h) + k * (d - l) ** (p - 1), 0.5, 3.0, xtol=1e-15)
    assert abs((c[1, 0] - c[0, 0]) - d_ref) < tol
    np.testing.assert_allclose(c[:, 1:], 0.0, atol=1e-14)


def test_net_first_step_converges_linearly():
    """The 11 x 11 net (220 springs): the relative error of the first step falls
    by more than six orders within 20 iterations, order 2 and order 4."""
    for p in (2, 4):
        sc = S.spring_net(order=p, iters=40)
        o = oracle.Oracle(sc)
        o.step(1)
        rho = o.residuals()
        assert rho[19] < 1e-6 * rho[0]
        assert np.all(np.diff(np.log(rho[:15] + 1e-300)) < 0.5)  # no growth beyond noise


def test_polynomial_needs_an_even_order():
    sc = S.spring_pair(order=4).copy(order=np.array([3], np.int32))
    with pytest.raises(ValueError):
        oracle.Oracle(sc)
