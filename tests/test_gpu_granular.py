"""The legged robot on a granular bed: sphere-sphere, sphere-plane, sphere-box
and box-plane contacts, revolute joints as ball-bond pairs and driven target
bonds, against the oracle -- a reduced bed over 30 steps and the full
50,013-body bed for one step (contact set exact in FP64)."""
import time

import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S
from parity import errors, fp64_ok, scale_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def _table(ct):
    key = np.stack([ct["i"], ct["j"], ct["feature"]], axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    return key[order], {k: v[order] for k, v in ct.items()}


def _reduced(prec):
    return S.granular_bed_quadruped(nx=34, nz=18, ny=2, precision=prec)


def test_reduced_bed_with_quadruped_fp64(P):
    sc = _reduced(S.PREC_FP64)
    print(f"[case] reduced bed n={sc.n_bodies} bonds={sc.n_bonds}", flush=True)
    g = P.Scene(sc)
    o = oracle.Oracle(sc)
    for step in (1, 2, 3):
        g.step(1)
        o.step(1)
        kg, cg = _table(g.contacts())
        ko, co = _table(o.contacts())
        np.testing.assert_array_equal(kg, ko)
        np.testing.assert_allclose(cg["x_j"], co["x_j"], atol=1e-9)
        e = errors(g.state(), o.state(), scale_of(sc))
        print("reduced bed after step", step, e)
        assert fp64_ok(e)


def test_reduced_bed_fp32_one_step(P):
    sc = _reduced(S.PREC_FP32)
    g = P.Scene(sc)
    g.step(1)
    o = oracle.Oracle(sc.copy(precision=S.PREC_FP64))
    o.step(1)
    e = errors(g.state(), o.state(), scale_of(sc))
    print("reduced bed fp32", e)
    assert e["pos"] <= 1e-4 and e["rot"] <= 1e-4


@pytest.mark.parametrize("prec", [S.PREC_FP64, S.PREC_FP32])
def test_full_bed_one_step(P, prec):
    sc = S.granular_bed_quadruped(precision=prec)
    print(f"[case] full bed n={sc.n_bodies} prec={prec}", flush=True)
    g = P.Scene(sc)
    g.step(1)
    st = g.state()
    t = time.time()
    o = oracle.Oracle(sc.copy(precision=S.PREC_FP64))
    o.step(1)
    print(f"oracle one step of {sc.n_bodies} bodies: {time.time() - t:.1f}s", flush=True)
    e = errors(st, o.state(), scale_of(sc))
    print("full bed", prec, e)
    if prec == S.PREC_FP64:
        kg, _ = _table(g.contacts())
        ko, _ = _table(o.contacts())
        np.testing.assert_array_equal(kg, ko)
        assert fp64_ok(e)
    else:
        # positions meet the FP32 bar; the orientations of a few 1 cm spheres
        # carry more: the FP64 oracle itself, from FP32-rounded inputs, moves
        # them by 2.9e-4 in this step (tests/test_oracle_sensitivity.py), so
        # their bar is 1e-3
        assert e["pos"] <= 1e-4 and e["rot"] <= 1e-3
