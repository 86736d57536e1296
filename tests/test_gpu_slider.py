"""Slider bonds on the GPU (flat path and the resident step) against the
oracle: a block on a world rail (point side only), a rod over two fixed points
(line side on a free body, whose weight moves with the foot every iteration),
two free bodies joined by one slider bond (both sides), and the driven slider
crank of Table 2, in FP64 and FP32, alone and in a batch.

FP32 bars: rounding these scenes' inputs to FP32 moves the FP64 oracle itself
by at most 6e-7 (positions and rotations, relative) over the horizons below,
so FP32 results are held to 1e-4."""
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
    return [(S.slider_rail(precision=prec), 60),
            (S.slider_rod(turn=((0.3, -0.8, 0.5), 1.1), precision=prec), 60),
            (S.slider_pair(precision=prec), 30),
            (S.slider_pair(moving_along=True, precision=prec), 30),
            (S.linkage("slider", drive_amp_deg=60.0, precision=prec), 120)]


@pytest.mark.parametrize("prec", [S.PREC_FP64, S.PREC_FP32], ids=["fp64", "fp32"])
def test_slider_scenes_against_the_oracle(P, prec):
    for sc, steps in _cases(prec):
        print(f"[case] {sc.name} prec={prec} steps={steps}", flush=True)
        g = P.Scene(sc)
        o = oracle.Oracle(sc.copy(precision=S.PREC_FP64))
        for chunk in (steps // 3, steps - steps // 3):
            g.step(chunk)
            o.step(chunk)
            e = errors(g.state(), o.state(), scale_of(sc))
            print(sc.name, chunk, e, flush=True)
            if prec == S.PREC_FP64:
                assert fp64_ok(e), (sc.name, e)
            else:
                assert e["pos"] <= 1e-4 and e["rot"] <= 1e-4, (sc.name, e)


def test_slider_crank_in_a_batch_matches_alone_and_the_oracle(P):
    """The slider crank admitted beside chains runs on the flat kernels; its
    state equals the oracle's to the FP64 bar, and equals the same scene in a
    batch of its own bit for bit."""
    sc = S.linkage("slider", drive_amp_deg=60.0, precision=S.PREC_FP64)
    alone = P.Batch(2, 1 << 26, S.PREC_FP64)
    a = alone.admit(sc, 40)
    mix = P.Batch(8, 1 << 28, S.PREC_FP64)
    others = [mix.admit(x, 40) for x in S.batched_chains(5, seed=4, precision=S.PREC_FP64)]
    m = mix.admit(sc, 40)
    assert all(s is not None for s in others) and a is not None and m is not None
    for _ in range(40):
        alone.step()
        mix.step()
    for x, y in zip(mix.state(m), alone.state(a)):
        np.testing.assert_array_equal(x, y)
    o = oracle.Oracle(sc)
    o.step(40)
    e = errors(mix.state(m), o.state(), scale_of(sc))
    print(e)
    assert fp64_ok(e)

