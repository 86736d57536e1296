"""How far FP32-sized changes of the inputs move the FP64 oracle itself: the bar
that an FP32 GPU result can be held to is no tighter than this spread.  On the
CPU, with the oracle alone."""
import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S
from parity import errors, scale_of


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _rounded(sc):
    return sc.copy(c0=_f32(sc.c0), A0=_f32(sc.A0), v0=_f32(sc.v0), w0=_f32(sc.w0), x_i=_f32(sc.x_i),
                   x_j=_f32(sc.x_j), rest_len=_f32(sc.rest_len), shape_param=_f32(sc.shape_param),
                   drive=_f32(sc.drive))


def _spread(sc, steps):
    a = oracle.Oracle(sc)
    a.step(steps)
    b = oracle.Oracle(_rounded(sc))
    b.step(steps)
    return errors(b.state(), a.state(), scale_of(sc))


@pytest.mark.slow
def test_full_bed_one_step_spread_from_fp32_rounded_inputs():
    """The robot on the 50,013-sphere bed, one step: rounding the inputs to FP32
    moves the orientations of a few spheres by about 3e-4 (the largest moves
    are 40 % of those spheres' turn in the step) while positions move by about
    3e-6.  The FP32 GPU bar on this scene's rotations
    (1e-3, with positions at 1e-4) is set from this spread."""
    e = _spread(S.granular_bed_quadruped(precision=S.PREC_FP64), 1)
    print(e)
    assert 1e-4 < e["rot"] < 1e-3
    assert e["pos"] < 1e-5


def test_mass_ratio_chain_spread_from_fp32_rounded_inputs():
    """The augmented mass-ratio chain stays insensitive over 40 steps (positions
    and rotations move by less than 2e-7), so its FP32 GPU results are held to
    the 1e-3 bar over that horizon."""
    for steps in (10, 40):
        e = _spread(S.mass_ratio_chain(augmented=True, precision=S.PREC_FP64), steps)
        assert e["pos"] < 2e-7 and e["rot"] < 2e-7, (steps, e)
