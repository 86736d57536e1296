"""Launch schedules of the flat path and the tuner.

Every schedule (lanes per contact body, wavefronts per workgroup, tile size)
must give the oracle's result within the FP64 bar; a schedule repeats its own
bits; the tuner leaves the scenes exactly where they were and caches its pick
per (architecture, precision, size bucket)."""
import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S
from parity import errors, fp64_ok, scale_of

pytestmark = pytest.mark.gpu

LANES = (1, 2, 4, 8, 16)
WAVES = (1, 2, 4)


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def settled_drop(n_side, layers, steps, seed, precision=S.PREC_FP64):
    """A box drop advanced by the oracle until its boxes touch."""
    sc = S.box_drop(n_side=n_side, layers=layers, seed=seed, precision=S.PREC_FP64)
    o = oracle.Oracle(sc)
    o.step(steps)
    c, A, v, w = o.state()
    return sc.with_state(c, A, v, w, t0=steps * sc.h).copy(precision=precision)


@pytest.fixture(scope="module")
def pile_fp64():
    # 324 boxes: more than the resident kernel takes, so a plain scene iterates
    # on the flat path
    return settled_drop(9, 4, 60, seed=7)


@pytest.fixture(scope="module")
def small_piles():
    return [settled_drop(3, 1, 60, seed=s) for s in (5, 6)]


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("lanes", LANES)
def test_plain_scene_every_contact_lane_count_matches_the_oracle_fp64(P, pile_fp64, lanes):
    sc = pile_fp64
    ref = oracle.Oracle(sc)
    ref.step(3)
    for waves in WAVES:
        print(f"[case] plain pile n={sc.n_bodies} lanes {lanes} waves {waves}", flush=True)
        g = P.Scene(sc)
        g.set_schedule(contact_lanes=lanes, group_waves=waves)
        assert g.schedule() == dict(tile_bodies=0, contact_lanes=lanes, group_waves=waves, from_cache=0)
        g.step(3)
        e = errors(g.state(), ref.state(), scale_of(sc))
        assert fp64_ok(e), (lanes, waves, e)
        again = P.Scene(sc)
        again.set_schedule(contact_lanes=lanes, group_waves=waves)
        again.step(3)
        _same(g.state(), again.state())


@pytest.mark.parametrize("lanes", LANES)
def test_batch_every_schedule_matches_the_oracle_fp64(P, small_piles, lanes):
    """Two piles on the flat path's contact waves, a 100-body chain on its plain
    waves and three short chains in tiles, under each schedule."""
    chains = S.batched_chains(3, seed=4, precision=S.PREC_FP64)
    long_chain = S.chain(100, tilt_deg=20.0, joint_angles_deg=np.linspace(-5, 5, 99),
                         precision=S.PREC_FP64, iters=12)
    scs = small_piles + chains + [long_chain]
    refs = []
    for sc in scs:
        o = oracle.Oracle(sc)
        o.step(6)
        refs.append(o.state())
    for waves, tile in ((1, 64), (4, 32), (2, 128)):
        print(f"[case] batch lanes {lanes} waves {waves} tile {tile}", flush=True)
        b = P.Batch(8, 1 << 28, S.PREC_FP64)
        b.set_schedule(tile_bodies=tile, contact_lanes=lanes, group_waves=waves)
        slots = [b.admit(s, 6) for s in scs]
        for _ in range(6):
            b.step()
        assert b.schedule() == dict(tile_bodies=tile, contact_lanes=lanes, group_waves=waves,
                                    from_cache=0)
        for sc, sl, r in zip(scs, slots, refs):
            e = errors(b.state(sl), r, scale_of(sc))
            assert fp64_ok(e), (sc.name, lanes, waves, tile, e)


def test_schedule_values_outside_the_sets_are_rejected(P, small_piles):
    b = P.Batch(2, 1 << 26, S.PREC_FP32)
    for bad in (dict(contact_lanes=3), dict(contact_lanes=32), dict(group_waves=3),
                dict(group_waves=8), dict(tile_bodies=48)):
        with pytest.raises(P.PabdError) as ex:
            b.set_schedule(**bad)
        assert ex.value.status == -1  # PABD_E_INVALID
    g = P.Scene(small_piles[0])
    with pytest.raises(P.PabdError):
        g.set_schedule(contact_lanes=0)
    assert b.schedule()["contact_lanes"] == 4 and g.schedule()["contact_lanes"] == 4


def _served_like_batch(P):
    """FP32 chains (tiled and flat), an augmented chain (flat, bond states that
    change every iteration) and box piles (flat, contacts)."""
    b = P.Batch(16, 1 << 28, S.PREC_FP32)
    scs = (S.batched_chains(6, seed=9)
           + [S.chain(150, tilt_deg=10.0, joint_angles_deg=np.linspace(-8, 8, 149), iters=20,
                      precision=S.PREC_FP32)]
           + [S.mass_ratio_chain(precision=S.PREC_FP32)]
           + [S.pile(n, seed=s) for n, s in ((60, 1), (200, 2))])
    slots = [b.admit(s, 400) for s in scs]
    return b, slots


def test_batch_tune_restores_the_scenes_and_caches_its_pick(P):
    P.tune_cache_clear()
    b, slots = _served_like_batch(P)
    for _ in range(4):
        b.step()
    before = [b.state(s) for s in slots]
    done = [b.steps_done(s) for s in slots]
    print("[case] batch tune", flush=True)
    sch = b.tune()
    assert sch["from_cache"] == 0
    assert sch["tile_bodies"] in (32, 64, 128, 256)
    assert sch["contact_lanes"] in LANES and sch["group_waves"] in WAVES
    assert P.tune_cache_size() == 1
    # the scenes are where they were
    for s, st, d in zip(slots, before, done):
        _same(b.state(s), st)
        assert b.steps_done(s) == d
    # and continue as a batch that never tuned but runs the same schedule
    twin, tslots = _served_like_batch(P)
    for _ in range(4):
        twin.step()
    twin.set_schedule(**{k: sch[k] for k in ("tile_bodies", "contact_lanes", "group_waves")})
    for _ in range(5):
        b.step()
        twin.step()
    for s, t in zip(slots, tslots):
        _same(b.state(s), twin.state(t))
    # the same workload shape takes the cached schedule without timing
    again = twin.tune()
    assert again["from_cache"] == 1
    assert {k: again[k] for k in ("tile_bodies", "contact_lanes", "group_waves")} == \
        {k: sch[k] for k in ("tile_bodies", "contact_lanes", "group_waves")}
    forced = twin.tune(force=True)
    assert forced["from_cache"] == 0
    P.tune_cache_clear()
    assert P.tune_cache_size() == 0


def test_scene_tune_restores_the_scene(P, pile_fp64):
    P.tune_cache_clear()
    sc = pile_fp64.copy(precision=S.PREC_FP32)
    g = P.Scene(sc)
    g.step(2)
    before = g.state()
    rho = g.residual()
    print("[case] scene tune", flush=True)
    sch = g.tune()
    assert sch["from_cache"] == 0 and sch["tile_bodies"] == 0
    assert sch["contact_lanes"] in LANES and sch["group_waves"] in WAVES
    _same(g.state(), before)
    assert g.residual() == rho
    twin = P.Scene(sc)
    twin.step(2)
    twin.set_schedule(contact_lanes=sch["contact_lanes"], group_waves=sch["group_waves"])
    g.step(3)
    twin.step(3)
    _same(g.state(), twin.state())
    assert P.Scene(sc).tune()["from_cache"] == 1
    # a scene the resident kernel runs whole has nothing to time
    small = P.Scene(S.chain8(precision=S.PREC_FP32))
    assert small.tune()["from_cache"] == 0
    assert P.tune_cache_size() == 1
    P.tune_cache_clear()


def test_tile_change_keeps_the_augmented_bond_state_fp64(P):
    """Changing the tile size re-places every scene; the augmented chain's
    multipliers and stiffnesses move with it, so after 5 + 5 steps it still
    matches the oracle's 10."""
    al = S.mass_ratio_chain(precision=S.PREC_FP64)
    chains = S.batched_chains(3, seed=3, precision=S.PREC_FP64)
    b = P.Batch(8, 1 << 28, S.PREC_FP64)
    sa = b.admit(al, 10)
    for c in chains:
        b.admit(c, 10)
    for _ in range(5):
        b.step()
    b.set_tile(32 if b.layout()["tile_bodies"] != 32 else 128)
    print("[case] augmented chain across a tile change", flush=True)
    for _ in range(5):
        b.step()
    o = oracle.Oracle(al)
    o.step(10)
    e = errors(b.state(sa), o.state(), scale_of(al))
    assert fp64_ok(e), e
