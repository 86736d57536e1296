"""Device memory from a caller's allocator (pabd_set_allocator), here PyTorch's
caching allocator: the memory is taken from it and returned to it, and the
results are the same bits as with the library's own allocations."""
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


def _run_scene(P, sc, steps):
    g = P.Scene(sc)
    g.step(steps)
    st = g.state()
    return g, st


def test_scene_and_batch_on_torch_allocator(P):
    import torch
    torch.cuda.init()
    sc = S.box_drop(n_side=3, layers=2, precision=S.PREC_FP32)
    ref_g, ref = _run_scene(P, sc, 30)
    ref_g.close()
    chains = S.batched_chains(6, seed=5, precision=S.PREC_FP32)
    rb = P.Batch(8, 1 << 27, S.PREC_FP32)
    rslots = [rb.admit(c, 10) for c in chains]
    for _ in range(10):
        rb.step()
    ref_batch = [rb.state(s) for s in rslots]
    rb.close()
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    P.use_torch_allocator(True)
    try:
        g, st = _run_scene(P, sc, 30)
        assert torch.cuda.memory_allocated() > m0
        for x, y in zip(st, ref):
            np.testing.assert_array_equal(x, y)
        b = P.Batch(8, 1 << 27, S.PREC_FP32)
        slots = [b.admit(c, 10) for c in chains]
        for _ in range(10):
            b.step()
        for s, r in zip(slots, ref_batch):
            for x, y in zip(b.state(s), r):
                np.testing.assert_array_equal(x, y)
        g.close()
        b.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == m0
    finally:
        P.use_torch_allocator(False)
    g2, st2 = _run_scene(P, sc, 1)  # the library's own allocations again
    g2.close()
