"""Pins of the oracle's augmented-Lagrangian bonds (Sec. 5.2.2): the multiplier
and stiffness updates on a case with a closed form, the hard-constraint behaviour
the formulation exists for, and the mass-ratio chain the paper shows it on."""
import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S


def _hanging(iters, rest=0.1, density=1.0, kappa=1e4, augmented=True, beta=1e4):
    """A unit cube hanging at rest from the world point (0, 0, 0) by one bond from
    its top face centre, stretched to exactly its rest length."""
    bd = S._bodies(1)
    bd["shape_param"][:] = 0.5
    bd["density"][:] = density
    bd["c0"][0] = (0.0, -0.5 - rest, 0.0)
    bonds = S._empty_bonds(1)
    bonds["bond_i"][0], bonds["bond_j"][0] = 0, -1
    bonds["x_i"][0] = (0.0, 0.5, 0.0)
    bonds["kappa"][0] = kappa
    bonds["rest_len"][0] = rest
    bonds["bond_type"][0] = S.BOND_AUGMENTED if augmented else S.BOND_QUADRATIC
    return S.SceneDesc(**bd, **bonds, iters=iters, al_beta=beta, precision=S.PREC_FP64)


def _joint_error(sc, state):
    c, A = state[0], state[1]
    err = []
    for e in range(sc.n_bonds):
        i, j = sc.bond_i[e], sc.bond_j[e]
        yi = A[i] @ sc.x_i[e] + c[i]
        yj = sc.x_j[e] if j < 0 else A[j] @ sc.x_j[e] + c[j]
        err.append(np.linalg.norm(yi - yj) - sc.rest_len[e])
    return np.array(err)


def test_first_iteration_updates_from_the_predicted_stretch():
    """One step with one iteration from rest at the rest length: the iteration's
    elongation is that of the prediction, C = h^2 g (the free fall of the step),
    so lambda = kappa_start h^2 g and kappa = kappa_start + beta h^2 g."""
    sc = _hanging(iters=1)
    o = oracle.Oracle(sc)
    o.step(1)
    kap, lam = o.bond_state()
    C0 = sc.h * sc.h * 9.81
    assert lam[0] == pytest.approx(1e4 * C0, rel=1e-12)
    assert kap[0] == pytest.approx(1e4 + 1e4 * C0, rel=1e-12)


def test_first_iteration_updates_from_a_compression():
    """Without gravity, from rest with the bond compressed by 0.02: the first
    elongation is C = -0.02, so lambda = kappa_start C < 0 and the stiffness still
    grows by beta |C|."""
    sc = _hanging(iters=1).copy(gravity=np.zeros(3), c0=np.array([[0.0, -0.5 - 0.08, 0.0]]))
    o = oracle.Oracle(sc)
    o.step(1)
    kap, lam = o.bond_state()
    assert lam[0] == pytest.approx(1e4 * -0.02, rel=1e-9)
    assert kap[0] == pytest.approx(1e4 + 1e4 * 0.02, rel=1e-9)


def test_augmented_bond_closes_the_joint_that_a_quadratic_bond_leaves_open():
    """At rest the quadratic bond keeps the compliance gap m g / kappa plus the
    projection offset (about 9e-3 m here); the multiplier drives the elongation
    of the iterate to zero, since lambda only stops changing when C = 0."""
    quad = oracle.Oracle(_hanging(iters=30, augmented=False))
    quad.step(400)
    gap_q = abs(_joint_error(quad._keep, quad.state())[0])
    al = oracle.Oracle(_hanging(iters=30))
    al.step(400)
    gap_a = abs(_joint_error(al._keep, al.state())[0])
    assert gap_q > 5e-3
    assert gap_a < 1e-6
    kap, lam = al.bond_state()
    assert lam[0] > 0.0 and kap[0] >= 1e4  # a tension; stiffness never below kappa_start


def test_augmented_bond_needs_a_rest_length():
    sc = _hanging(iters=10, rest=0.0)
    with pytest.raises(ValueError):
        oracle.Oracle(sc)


def test_mass_ratio_chain_keeps_its_joints_with_augmented_bonds():
    """The paper's observation on the chain with a heavy bottom box: without the
    augmented Lagrangian the distance constraints stretch by metres, with it they
    hold to centimetres (under 0.1 m at every sampled step, 20x below the
    quadratic bonds' worst)."""
    quad = S.mass_ratio_chain(augmented=False)
    aug = S.mass_ratio_chain(augmented=True)
    oq, oa = oracle.Oracle(quad), oracle.Oracle(aug)
    worst_q = worst_a = 0.0
    for _ in range(6):
        oq.step(50)
        oa.step(50)
        eq = np.abs(_joint_error(quad, oq.state())).max()
        ea = np.abs(_joint_error(aug, oa.state())).max()
        worst_q, worst_a = max(worst_q, eq), max(worst_a, ea)
        assert ea < eq
    assert worst_q > 1.0 and worst_a < 0.1 and worst_a < worst_q / 20


def test_warm_start_scales_the_multiplier_by_alpha_gamma():
    """Warm start of Sec. 5.2.2: each step begins from lambda^0 = alpha gamma
    lambda^n.  With one iteration per step and beta = 0 the stiffness stays
    kappa_start and the step's elongation C is measured at the prediction, which
    does not depend on the multiplier carried over; so after two steps lambda
    differs between two values alpha, alpha' of the factor by exactly
    (alpha - alpha') gamma lambda_1, lambda_1 being the multiplier after the first
    step (the same for both, since the first step starts from lambda = 0)."""
    gamma = 0.9
    base = _hanging(iters=1, beta=0.0).copy(al_gamma=gamma, c0=np.array([[0.05, -0.5 - 0.13, 0.02]]),
                                           w0=np.array([[0.4, -0.2, 0.9]]))
    lam1, lam2 = {}, {}
    for alpha in (0.99, 0.5, 0.0):
        o = oracle.Oracle(base.copy(al_alpha=alpha))
        o.step(1)
        lam1[alpha] = o.bond_state()[1][0]
        o.step(1)
        lam2[alpha] = o.bond_state()[1][0]
        assert o.bond_state()[0][0] == pytest.approx(1e4, rel=1e-15)
    assert lam1[0.99] == lam1[0.5] == lam1[0.0] != 0.0
    l1 = lam1[0.99]
    assert lam2[0.99] - lam2[0.5] == pytest.approx((0.99 - 0.5) * gamma * l1, rel=1e-9)
    assert lam2[0.5] - lam2[0.0] == pytest.approx(0.5 * gamma * l1, rel=1e-9)
