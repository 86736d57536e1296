"""The allocation-free entry point pabd_scene_run_noalloc against the plain
path's create + step + read_state, through the C ABI: bit for bit, on calls in
a row that reuse the library's static scratch array (the second with a smaller
scene), and a scene too large for the array turned away with PABD_E_OOM before
the device is touched."""
import numpy as np
import pytest

from paper_2609_02675_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def _plain(P, sc, steps):
    g = P.Scene(sc)
    g.step(steps)
    return g.state()


def _same(a, b, name):
    for x, y in zip(a, b):
        assert np.array_equal(x, y), name


def test_noalloc_equals_the_plain_path_on_calls_in_a_row(P):
    from paper_2609_02675_amd._lib import run_noalloc
    # a landing pile (contacts, FP32), then a smaller chain (FP64), then the pile again
    pile = S.box_drop(n_side=6, layers=6, seed=4, precision=S.PREC_FP32)
    chain = S.chain8(precision=S.PREC_FP64)
    print(f"[case] noalloc pile {pile.n_bodies} bodies, 50 steps", flush=True)
    first = run_noalloc(pile, 50)
    _same(first, _plain(P, pile, 50), pile.name)
    assert np.isfinite(first[0]).all() and first[0][:, 1].min() < 1.5  # it landed
    print("[case] noalloc chain8 fp64, 20 steps", flush=True)
    second = run_noalloc(chain, 20)
    _same(second, _plain(P, chain, 20), chain.name)
    print("[case] noalloc pile again", flush=True)
    _same(run_noalloc(pile, 50), first, pile.name)


def test_noalloc_rejects_a_scene_beyond_the_scratch(P):
    from paper_2609_02675_amd import _lib
    big = S.box_drop(n_side=20, layers=10, seed=1, precision=S.PREC_FP32)  # 4,000 boxes x 256 contact slots
    print(f"[case] noalloc oversize {big.n_bodies} bodies", flush=True)
    with pytest.raises(_lib.PabdError) as ei:
        _lib.run_noalloc(big, 1)
    assert ei.value.status == _lib.PABD_E_OOM and "static scratch" in str(ei.value)
    # the next call still works
    small = S.chain(5, precision=S.PREC_FP32)
    _same(_lib.run_noalloc(small, 3), _plain(P, small, 3), small.name)
