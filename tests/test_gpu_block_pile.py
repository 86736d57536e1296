"""Contact construction at the paper's largest scale: 50^3 = 125,000 stacked
cubes, every cube in resting contact with its neighbours.  The full contact set
is too large for the oracle's all-pairs detection, so sampled bodies are checked:
for each, the oracle's O(N) per-body query must return exactly the contacts the
GPU built for that body (FP64, bit-exact keys and anchors)."""
import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def _by_body(ct, b):
    sel = (ct["i"] == b) | (ct["j"] == b)
    key = np.stack([ct["i"][sel], ct["j"][sel], ct["feature"][sel]], axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    return key[order], {k: v[sel][order] for k, v in ct.items()}


def test_block_pile_125k_sampled_contacts_fp64(P):
    sc = S.block_pile(precision=S.PREC_FP64)
    print(f"[case] block pile n={sc.n_bodies} fp64", flush=True)
    g = P.Scene(sc)
    g.step(1)
    g.state()  # raises on capacity overflow or a non-finite state
    ct = g.contacts()
    assert len(ct["i"]) > 20 * sc.n_bodies
    o = oracle.Oracle(sc)  # the initial state, which the step's detection used
    rng = np.random.default_rng(0)
    n_side, layers = 50, 50
    corner = 0
    top_centre = (25 * layers + (layers - 1)) * n_side + 25
    samples = [corner, top_centre, sc.n_bodies - 1] + list(rng.choice(sc.n_bodies, 45, replace=False))
    for b in samples:
        o.detect_body(int(b))
        ko, co = _by_body(o.contacts(), b)
        kg, cg = _by_body(ct, b)
        np.testing.assert_array_equal(kg, ko)
        for f in ("x_i", "x_j", "normal", "kappa"):
            np.testing.assert_allclose(cg[f], co[f], rtol=1e-12, atol=1e-12)


def test_block_pile_125k_fp32_steps(P):
    sc = S.block_pile(precision=S.PREC_FP32)
    print(f"[case] block pile n={sc.n_bodies} fp32", flush=True)
    g = P.Scene(sc)
    g.step(10)
    c, A, v, w = g.state()
    assert np.all(np.isfinite(c)) and np.all(np.isfinite(v))
    # the stack settles under gravity: nothing rises far above its start or leaves the floor
    assert c[:, 1].max() < sc.c0[:, 1].max() + 0.5 and c[:, 1].min() > 0.0
