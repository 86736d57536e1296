"""Checkpoint and resume through the C ABI: read_state after n steps, create (or
admit) the scene again from that state, step m more times, and compare with n +
m uninterrupted steps.  FP64 states are read back as the doubles the device
holds, so an FP64 resume repeats the uninterrupted run bit for bit (scenes
without augmented, driven or slider bonds carry nothing else from step to
step).  An FP32 position is an unevaluated sum of two floats that a round trip
through one double need not reproduce, so an FP32 resume is held to the FP32
one-step bar (1e-4) instead; the box pile after landing amplifies that first
rounding."""
import numpy as np
import pytest

from paper_2609_02675_amd import scenes as S
from parity import errors, scale_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def _cases(prec):
    return [(S.chain(150, tilt_deg=25.0, precision=prec, name="chain150"), 9, 7),
            (S.box_drop(n_side=4, layers=3, seed=5, precision=prec), 45, 15)]


def _plain(P, sc, n, m):
    full = P.Scene(sc)
    full.step(n + m)
    first = P.Scene(sc)
    first.step(n)
    c, A, v, w = first.state()
    rest = P.Scene(sc.with_state(c, A, v, w, t0=sc.t0 + n * sc.h))
    rest.step(m)
    return rest.state(), full.state()


def test_plain_scene_resumes_bit_for_bit_fp64(P):
    for sc, n, m in _cases(S.PREC_FP64):
        print(f"[case] plain resume {sc.name} n={n} m={m}", flush=True)
        got, want = _plain(P, sc, n, m)
        for x, y in zip(got, want):
            assert np.array_equal(x, y), sc.name


def test_batch_slot_resumes_bit_for_bit_fp64(P):
    for sc, n, m in _cases(S.PREC_FP64):
        print(f"[case] batch resume {sc.name} n={n} m={m}", flush=True)
        b = P.Batch(4, 1 << 28, S.PREC_FP64)
        full = b.admit(sc, n + m)
        first = b.admit(sc, n)
        for _ in range(n):
            b.step()
        c, A, v, w = b.state(first)
        b.release(first)
        rest = b.admit(sc.with_state(c, A, v, w, t0=sc.t0 + n * sc.h), m)
        for _ in range(m):
            b.step()
        for x, y in zip(b.state(rest), b.state(full)):
            assert np.array_equal(x, y), sc.name


def test_plain_scene_resumes_within_the_fp32_bar(P):
    for sc, n, m in _cases(S.PREC_FP32):
        print(f"[case] plain resume fp32 {sc.name}", flush=True)
        got, want = _plain(P, sc, n, m)
        e = errors(got, want, scale_of(sc))
        assert e["pos"] <= 1e-4 and e["rot"] <= 1e-4, (sc.name, e)
