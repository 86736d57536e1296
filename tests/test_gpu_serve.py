"""Serving on the GPU: continuous batching under an HBM budget; every result is
the same alone and in the mix (bit for bit: per-body sums run in a fixed order
that does not depend on the other resident scenes)."""
import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S
from parity import errors, scale_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def _requests(prec, n=20, seed=3):
    return S.serving_requests(rate_hz=2000.0, duration_s=1.0, seed=seed, n_lo=8, n_hi=400,
                              steps_lo=5, steps_hi=25, precision=prec, max_requests=n)


@pytest.mark.parametrize("prec", [S.PREC_FP32, S.PREC_FP64])
def test_served_results_equal_alone_and_in_the_mix(P, prec):
    from paper_2609_02675_amd.serve import Server
    reqs = _requests(prec)
    print(f"[case] serve mix prec={prec} sizes={[r.scene.n_bodies for r in reqs]}", flush=True)
    need = [P.scene_bytes(r.scene) for r in reqs]
    budget = max(max(need), sum(need) // 4)
    srv = Server(budget, 32, prec)
    res, st = srv.run(reqs, realtime=False)
    assert st.rejected == 0 and st.diverged == 0 and st.completed == len(reqs)
    assert st.peak_bytes <= budget
    # every result, piles included, was read back healthy (a non-finite state or
    # a contact overflow would have evicted it) and is finite
    for r in res.values():
        assert r.status == "ok", (r.scene_name, r.reason)
        assert all(np.isfinite(x).all() for x in r.state), r.scene_name
    assert st.max_resident < len(reqs)
    for k in (0, 5, 11, len(reqs) - 1):
        alone = Server(1 << 28, 4, prec)
        ra, _ = alone.run([reqs[k]], realtime=False)
        for a, b in zip(res[k].state, ra[0].state):
            np.testing.assert_array_equal(a, b)
        o = oracle.Oracle(reqs[k].scene)
        o.step(reqs[k].steps)
        e = errors(res[k].state, o.state(), scale_of(reqs[k].scene))
        tol = 1e-9 if prec == S.PREC_FP64 else 1e-4
        assert e["pos"] <= tol and e["rot"] <= tol, (reqs[k].scene.name, e)


def test_served_mix_full_size_fp32(P):
    """The served workload at its full shape: one second of Poisson arrivals at
    200 req/s, 8 to 5,000 bodies, 60 to 600 steps, FP32, 8 GiB budget, all queued
    at once. Every request completes within the budget; the cheapest chains with
    at most 100 steps match the oracle within the FP32 bar (piles are chaotic over
    these horizons)."""
    from paper_2609_02675_amd.serve import Server
    reqs = S.serving_requests(rate_hz=200.0, duration_s=1.0, seed=3, precision=S.PREC_FP32)
    print(f"[case] full served mix: {len(reqs)} requests, "
          f"{sum(r.scene.n_bodies for r in reqs)} bodies", flush=True)
    budget = 8 << 30
    srv = Server(budget, 512, S.PREC_FP32)
    res, st = srv.run(reqs, realtime=False)
    assert st.rejected == 0 and st.diverged == 0 and st.completed == len(reqs)
    assert st.peak_bytes <= budget
    # every result, piles included, was read back healthy (a non-finite state or
    # a contact overflow would have evicted it) and is finite
    for r in res.values():
        assert r.status == "ok", (r.scene_name, r.reason)
        assert all(np.isfinite(x).all() for x in r.state), r.scene_name
    chains = [k for k, r in enumerate(reqs) if "chain" in r.scene.name and r.steps <= 100]
    chains.sort(key=lambda k: reqs[k].scene.n_bodies * reqs[k].steps)
    assert chains
    for k in chains[:3]:
        sc64 = reqs[k].scene.copy(precision=S.PREC_FP64)
        o = oracle.Oracle(sc64)
        o.step(reqs[k].steps)
        e = errors(res[k].state, o.state(), scale_of(sc64))
        print(reqs[k].scene.name, reqs[k].steps, e)
        assert e["pos"] <= 1e-3 and e["rot"] <= 1e-3, (reqs[k].scene.name, e)
