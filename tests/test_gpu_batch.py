"""GPU tests of the batched path (tile kernel + flat kernels in one captured
graph per step): parity with the oracle per scene, invariance of every scene's
result alone vs in the mix and across tile sizes, admission by HBM budget."""
import numpy as np
import pytest

import oracle
from paper_2609_02675_amd import scenes as S
from parity import errors, fp64_ok, scale_of, worst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        pytest.fail("no HIP device visible")
    return P


def _oracle_state(sc, steps):
    o = oracle.Oracle(sc)
    o.step(steps)
    return o.state()


def _run_batch(P, scenes, steps, prec, tile=None, budget=1 << 30):
    b = P.Batch(len(scenes) + 2, budget, prec)
    if tile:
        b.set_tile(tile)
    slots = [b.admit(s, steps) for s in scenes]
    assert all(x is not None for x in slots)
    for _ in range(steps):
        b.step()
    return b, slots, [b.state(s) for s in slots]


def test_batched_chains_fp64_match_oracle(P):
    scs = S.batched_chains(48, seed=2, precision=S.PREC_FP64)
    print(f"[case] 48 chains fp64 sizes {[s.n_bodies for s in scs][:8]}...", flush=True)
    b, slots, states = _run_batch(P, scs, 30, S.PREC_FP64)
    for sc, st in zip(scs, states):
        e = errors(st, _oracle_state(sc, 30), scale_of(sc))
        assert e["pos"] <= 1e-9 and e["rot"] <= 1e-9, (sc.name, e)


@pytest.mark.parametrize("steps,tol", [(1, 1e-4), (100, 1e-3)])
def test_batched_chains_fp32_match_oracle(P, steps, tol):
    scs = S.batched_chains(32, seed=7, precision=S.PREC_FP32)
    print(f"[case] 32 chains fp32 steps {steps}", flush=True)
    b, slots, states = _run_batch(P, scs, steps, S.PREC_FP32)
    worst_e = 0.0
    for sc, st in zip(scs, states):
        e = errors(st, _oracle_state(sc, steps), scale_of(sc))
        worst_e = max(worst_e, e["pos"], e["rot"])
        assert e["pos"] <= tol and e["rot"] <= tol, (sc.name, e)
    print(f"fp32 worst error after {steps} steps: {worst_e:.3e}")


def test_each_scene_same_alone_and_in_the_mix(P):
    """Per-body sums run in a fixed (bond id) order, so a scene's bits do not
    depend on its neighbours in the batch."""
    scs = S.batched_chains(40, seed=11, precision=S.PREC_FP32)
    b, slots, mixed = _run_batch(P, scs, 20, S.PREC_FP32)
    for k in (0, 13, 39):
        b1, s1, alone = _run_batch(P, [scs[k]], 20, S.PREC_FP32)
        for x, y in zip(mixed[k], alone[0]):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("tile", [32, 128, 256])
def test_tile_size_does_not_change_results(P, tile):
    scs = [s for s in S.batched_chains(24, seed=5, precision=S.PREC_FP32) if s.n_bodies <= 32]
    b, slots, ref = _run_batch(P, scs, 10, S.PREC_FP32, tile=64)
    b2, slots2, got = _run_batch(P, scs, 10, S.PREC_FP32, tile=tile)
    for x, y in zip(ref, got):
        for a, c in zip(x, y):
            np.testing.assert_array_equal(a, c)


def test_flat_path_scenes_in_a_batch(P):
    """Scenes too large for a tile (300 bodies) and driven scenes go through the
    flat kernels of the same graph; mixed with tiled chains."""
    big = S.chain(300, tilt_deg=20.0, joint_angles_deg=np.linspace(-5, 5, 299),
                  precision=S.PREC_FP64, iters=12)
    small = S.batched_chains(5, seed=3, precision=S.PREC_FP64)
    scs = [big] + small
    b, slots, states = _run_batch(P, scs, 15, S.PREC_FP64)
    for sc, st in zip(scs, states):
        assert fp64_ok(errors(st, _oracle_state(sc, 15), scale_of(sc))), sc.name


def test_scenes_with_different_step_budgets_freeze(P):
    scs = S.batched_chains(3, seed=1, precision=S.PREC_FP64)
    b = P.Batch(4, 1 << 28, S.PREC_FP64)
    slots = [b.admit(s, n) for s, n in zip(scs, (5, 10, 15))]
    for _ in range(15):
        b.step()
    assert sorted(b.poll()) == sorted(slots)
    for sc, sl, n in zip(scs, slots, (5, 10, 15)):
        assert b.steps_done(sl) == n
        assert fp64_ok(errors(b.state(sl), _oracle_state(sc, n), scale_of(sc)))


def test_admission_respects_budget_and_release_frees_it(P):
    sc = S.chain(64, tilt_deg=0.0, precision=S.PREC_FP32)
    need = P.scene_bytes(sc)
    b = P.Batch(16, 3 * need + need // 2, S.PREC_FP32)
    slots = [b.admit(sc, 10) for _ in range(4)]
    assert slots[3] is None and all(s is not None for s in slots[:3])
    b.release(slots[0])
    assert b.admit(sc, 10) is not None


def test_autotune_picks_a_tile_and_keeps_state(P):
    scs = S.batched_chains(64, seed=9, precision=S.PREC_FP32)
    b = P.Batch(70, 1 << 28, S.PREC_FP32)
    slots = [b.admit(s, 20) for s in scs]
    for _ in range(5):
        b.step()
    tile = b.autotune()
    assert tile in (64, 128, 256)
    for _ in range(15):
        b.step()
    ref_b, ref_slots, ref = _run_batch(P, scs, 20, S.PREC_FP32)
    for sl, r in zip(slots, ref):
        for x, y in zip(b.state(sl), r):
            np.testing.assert_array_equal(x, y)


def test_full_size_batched_chains_sampled(P):
    """4096 chains of 4..64 bodies (the batched workload) in one batch, FP32,
    20 iterations, 100 steps in the benchmark's launch configuration (tiles of
    64 bodies, 10 steps per launch); sampled scenes checked against the oracle."""
    scs = S.batched_chains(4096, seed=2, precision=S.PREC_FP32)
    print(f"[case] 4096 chains, {sum(s.n_bodies for s in scs)} bodies", flush=True)
    b = P.Batch(len(scs) + 2, 2 << 30, S.PREC_FP32)
    b.set_tile(64)
    slots = [b.admit(s, 100) for s in scs]
    assert all(x is not None for x in slots)
    for _ in range(10):
        b.step(nsteps=10)
    rng = np.random.default_rng(0)
    for k in rng.choice(len(scs), 8, replace=False):
        e = errors(b.state(slots[k]), _oracle_state(scs[k], 100), scale_of(scs[k]))
        print(scs[k].name, e)
        assert e["pos"] <= 1e-3 and e["rot"] <= 1e-3


def test_many_scenes_without_planes_or_driven_bonds_all_admit(P):
    """Scenes without planes or driven bonds take no space in those tables, so the
    number of resident scenes is not capped by their size (20,000 small chains
    in a batch whose driven-bond table holds about 15,000 entries)."""
    scs = S.batched_chains(20000, seed=11, lo=4, hi=6, precision=S.PREC_FP32)
    print(f"[case] {len(scs)} small chains", flush=True)
    b = P.Batch(len(scs) + 8, 1 << 30, S.PREC_FP32)
    slots = [b.admit(s, 3) for s in scs]
    assert all(x is not None for x in slots)
    for _ in range(3):
        b.step()
    b.sync()
    assert sorted(b.poll()) == sorted(slots)


@pytest.mark.parametrize("prec", [S.PREC_FP32, S.PREC_FP64])
def test_several_steps_per_launch_equal_single_steps(P, prec):
    """pabd_batch_steps runs nsteps steps of every tile in one launch: the same
    bits as nsteps single-step calls, for scenes that run through the launch,
    scenes whose step budget ends inside it, and flat-path scenes beside them."""
    tiled = S.batched_chains(30, seed=13, precision=prec)
    big = S.chain(300, tilt_deg=20.0, joint_angles_deg=np.linspace(-5, 5, 299),
                  precision=prec, iters=12)
    scs = tiled + [big]
    budgets = [7 if k % 3 else 3 for k in range(len(tiled))] + [7]
    print(f"[case] several steps per launch, prec {prec}", flush=True)

    def run(launch_steps):
        b = P.Batch(len(scs) + 2, 1 << 30, prec)
        slots = [b.admit(s, n) for s, n in zip(scs, budgets)]
        done = 0
        for n in launch_steps:
            b.step(nsteps=n)
            done += n
        assert done == 7
        return b, slots

    b1, s1 = run([1] * 7)
    b2, s2 = run([5, 2])
    for k, (x, y) in enumerate(zip(s1, s2)):
        assert b2.steps_done(y) == budgets[k]
        for u, w in zip(b1.state(x), b2.state(y)):
            np.testing.assert_array_equal(u, w)
        assert b1.residual(x) == b2.residual(y)
    assert sorted(b2.poll()) == sorted(s2)
    # and against the oracle
    for k in (0, 1, len(scs) - 1):
        e = errors(b2.state(s2[k]), _oracle_state(scs[k], budgets[k]), scale_of(scs[k]))
        if prec == S.PREC_FP64:
            assert fp64_ok(e), (scs[k].name, e)
        else:
            assert e["pos"] <= 1e-3 and e["rot"] <= 1e-3, (scs[k].name, e)


@pytest.mark.parametrize("prec", [S.PREC_FP32, S.PREC_FP64])
def test_largest_steps_per_launch_equal_single_steps(P, prec):
    """256 steps in one launch, the largest count allowed: the same bits as 256
    single steps, for scenes that run through the launch and scenes whose budget
    ends inside it; in FP64 the early-ending scenes also match the oracle."""
    scs = S.batched_chains(12, seed=21, precision=prec)
    budgets = [256 if k % 2 else 97 for k in range(len(scs))]
    print(f"[case] 256 steps per launch, prec {prec}", flush=True)

    def run(launch_steps):
        b = P.Batch(len(scs) + 2, 1 << 30, prec)
        slots = [b.admit(s, n) for s, n in zip(scs, budgets)]
        for n in launch_steps:
            b.step(nsteps=n)
        return b, slots

    b1, s1 = run([1] * 256)
    b2, s2 = run([256])
    for k, (x, y) in enumerate(zip(s1, s2)):
        assert b2.steps_done(y) == budgets[k]
        for u, w in zip(b1.state(x), b2.state(y)):
            np.testing.assert_array_equal(u, w)
    assert sorted(b2.poll()) == sorted(s2)
    if prec != S.PREC_FP64:
        return
    for k in (0, 2):
        e = errors(b2.state(s2[k]), _oracle_state(scs[k], budgets[k]), scale_of(scs[k]))
        assert fp64_ok(e), (scs[k].name, e)


def test_steps_per_launch_out_of_range_is_rejected(P):
    b = P.Batch(2, 1 << 26, S.PREC_FP32)
    b.admit(S.chain8(precision=S.PREC_FP32), 5)
    for n in (0, 257):
        with pytest.raises(P.PabdError):
            b.step(nsteps=n)


def test_batched_residuals_match_oracle_fp64(P):
    """The per-scene residual of the last iteration (summed in FP64 inside the
    tile kernel) against the oracle's."""
    scs = S.batched_chains(12, seed=4, precision=S.PREC_FP64)
    print("[case] batched residuals fp64", flush=True)
    b, slots, _ = _run_batch(P, scs, 6, S.PREC_FP64)
    for sc, sl in zip(scs, slots):
        o = oracle.Oracle(sc)
        o.step(6)
        assert b.residual(sl) == pytest.approx(o.residuals()[-1], rel=1e-6), sc.name
