"""Descriptor validation at the boundary, on the CPU: the library (through
pabd_scene_bytes, which returns 0 for a descriptor it rejects and touches no
device) and the oracle reject the same malformed scenes and accept the same
well-formed ones, including a generalised mass given directly (Sec. 4.1.1)."""
import numpy as np
import pytest

import oracle
import paper_2609_02675_amd as P
from paper_2609_02675_amd import scenes as S


def _both_accept(sc):
    ok_lib = P.scene_bytes(sc) > 0
    try:
        oracle.Oracle(sc)
        ok_ora = True
    except ValueError:
        ok_ora = False
    assert ok_lib == ok_ora, (ok_lib, ok_ora)
    return ok_lib


def test_given_mass_and_pi0_are_accepted_without_density():
    sc = S.general_inertia_chain()
    assert _both_accept(sc)
    assert _both_accept(sc.copy(density=np.zeros(sc.n_bodies)))


def test_a0_must_be_a_rotation():
    sc = S.chain8()
    assert _both_accept(sc)
    A = sc.A0.copy()
    A[3] = A[3] * 1.01  # scaled
    assert not _both_accept(sc.copy(A0=A))
    A = sc.A0.copy()
    A[3] = A[3] @ np.diag([1.0, 1.0, -1.0])  # reflection
    assert not _both_accept(sc.copy(A0=A))
    A = sc.A0.copy()
    A[3, 0, 1] += 1e-8  # within rounding of a rotation
    assert _both_accept(sc.copy(A0=A))


@pytest.mark.parametrize("bad", ["negative_mass", "indefinite", "singular"])
def test_free_bodies_need_positive_mass_and_definite_pi0(bad):
    sc = S.general_inertia_chain()
    m, pi = sc.mass.copy(), sc.Pi0.copy()
    if bad == "negative_mass":
        m[2] = -1.0
    elif bad == "indefinite":
        pi[2] = (0.1, 0.2, 0.0, 0.1, 0.0, 0.1)  # 2 x 2 minor negative
    else:
        pi[2] = (0.1, 0.1, 0.0, 0.1, 0.0, 0.1)  # 2 x 2 minor zero
    assert not _both_accept(sc.copy(mass=m, Pi0=pi))
    # the pinned top body's mass never enters a step: anything goes
    m, pi = sc.mass.copy(), sc.Pi0.copy()
    m[0] = 0.0
    pi[0] = 0.0
    assert _both_accept(sc.copy(mass=m, Pi0=pi))


def test_polar_fallback_scenes_are_valid():
    for kind in ("flip", "flat"):
        assert _both_accept(S.polar_fallback_body(kind))


def test_slider_bonds_need_an_axis_and_no_rest_length():
    for sc in (S.slider_rail(), S.slider_rod(), S.slider_pair(), S.linkage("slider", drive_amp_deg=60.0)):
        assert _both_accept(sc)
    sc = S.slider_rail()
    assert not _both_accept(sc.copy(drive=np.zeros_like(sc.drive)))
    assert not _both_accept(sc.copy(rest_len=np.full(sc.n_bonds, 0.1)))
    assert _both_accept(sc.copy(drive=3.0 * sc.drive))  # the axis need not be unit
