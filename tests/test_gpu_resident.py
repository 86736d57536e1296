"""The resident step kernel (a single scene that fits one workgroup: the whole
step, with q^k in LDS, in one launch after its contact construction) against
the flat path's kernels, which a batch uses for the same scene, and against the
oracle.  The body iteration is the same code in both, so the states agree bit
for bit."""
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


def _cases(prec):
    return [S.chain(150, tilt_deg=25.0, precision=prec, name="chain150"),     # one lane per body
            S.pile(120, seed=7, precision=prec),                             # contacts, four lanes per body
            S.mass_ratio_chain(augmented=True, precision=prec),              # augmented bonds
            S.spring_net(order=4, precision=prec),                           # polynomial bonds
            S.linkage("slider", drive_amp_deg=60.0, precision=prec),         # slider and driven bonds
            S.slider_pair(precision=prec),                                   # slider line side on a free body
            S.granular_bed_quadruped(nx=6, nz=6, ny=2, precision=prec)]      # contacts and driven bonds


@pytest.mark.parametrize("prec", [S.PREC_FP32, S.PREC_FP64], ids=["fp32", "fp64"])
def test_resident_step_equals_the_flat_kernels_bit_for_bit(P, prec):
    for sc in _cases(prec):
        steps = 70 if "pile" in sc.name else 25  # the pile lands from step 40 on
        print(f"[case] resident vs flat {sc.name} prec={prec}", flush=True)
        g = P.Scene(sc)          # resident kernel
        g.step(steps)
        b = P.Batch(4, 1 << 30, prec)  # flat kernels
        slot = b.admit(sc, steps)
        for _ in range(steps):
            b.step()
        for x, y in zip(g.state(), b.state(slot)):
            assert np.array_equal(x, y), sc.name
        assert g.residual() == pytest.approx(b.residual(slot), rel=1e-12)


def test_recording_every_residual_switches_to_the_flat_kernels(P):
    """Debug bit1 (residual of every iteration) runs the flat kernels; the states
    stay the same bits and the recorded last residual is the resident one's."""
    sc = S.chain(100, tilt_deg=30.0, precision=S.PREC_FP64)
    a = P.Scene(sc)
    a.step(5)
    h = P.Scene(sc)
    h.set_debug(2)
    h.step(5)
    for x, y in zip(a.state(), h.state()):
        assert np.array_equal(x, y)
    assert h.residuals()[-1] == pytest.approx(a.residual(), rel=1e-12)


def test_resident_step_matches_the_oracle_fp64(P):
    for sc in _cases(S.PREC_FP64):
        steps = 3
        g = P.Scene(sc)
        g.step(steps)
        o = oracle.Oracle(sc)
        o.step(steps)
        e = errors(g.state(), o.state(), scale_of(sc))
        print(sc.name, e)
        assert fp64_ok(e), sc.name
