"""GPU tests of the batched tile path on bond layouts other than plain chains:
two bonds between the same pair of bodies (the mirror end of each is found by
the order of the bonds), bodies with more than two ends (ends past the second,
and ends whose mirror is past the partner's second, take the partner's q from
LDS), ends anchored in the world, and springs with a rest length.  Every scene
here is tiled (it fits the tile size set), and is checked against the oracle."""
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


def _hinge_chain(n, prec, interleave, seed):
    """A chain whose neighbours are joined by two ball joints, 0.3 m either side
    of the face centre along z (a hinge about z, the axis the chain's joints turn
    about, so the start is consistent).  interleave: the two bonds of a joint are
    listed next to each other; else all first bonds, then all second bonds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = S.chain(n, tilt_deg=20.0, joint_angles_deg=rng.uniform(-20, 20, n - 1),
                   precision=prec, name=f"hinge{n}")
    b = base.n_bonds
    off = np.array([0.0, 0.0, 0.3])
    if interleave:
        pick = np.repeat(np.arange(b), 2)
        sign = np.tile([1.0, -1.0], b)
    else:
        pick = np.concatenate([np.arange(b), np.arange(b)])
        sign = np.concatenate([np.ones(b), -np.ones(b)])
    return base.copy(
        bond_i=base.bond_i[pick], bond_j=base.bond_j[pick], bond_type=base.bond_type[pick],
        x_i=base.x_i[pick] + sign[:, None] * off, x_j=base.x_j[pick] + sign[:, None] * off,
        kappa=base.kappa[pick], rest_len=base.rest_len[pick], drive=base.drive[pick],
        order=None)


def _world_chain(n, prec):
    """A chain hung from the world by a ball joint at body 0's top face centre,
    nothing pinned."""
    base = S.chain(n, tilt_deg=35.0, precision=prec, pin_top=False, name=f"worldchain{n}")
    A0 = np.asarray(base.A0[0])
    xw = np.asarray(base.c0[0]) + A0 @ np.array([0.0, 0.5, 0.0])
    return base.copy(
        bond_i=np.concatenate([[0], base.bond_i]).astype(np.int32),
        bond_j=np.concatenate([[-1], base.bond_j]).astype(np.int32),
        bond_type=np.concatenate([[0], base.bond_type]).astype(np.int32),
        x_i=np.concatenate([[[0.0, 0.5, 0.0]], base.x_i]),
        x_j=np.concatenate([[xw], base.x_j]),
        kappa=np.concatenate([[1e5], base.kappa]),
        rest_len=np.concatenate([[0.0], base.rest_len]),
        drive=np.concatenate([np.zeros((1, 13)), base.drive]), order=None)


def _scenes(prec):
    return ([_hinge_chain(n, prec, True, seed=n) for n in (3, 9, 20)] +
            [_hinge_chain(n, prec, False, seed=n + 1) for n in (5, 17)] +
            [_world_chain(n, prec) for n in (1, 6, 30)] +
            [S.world_pendulum(theta0_deg=40.0, precision=prec)])


def _run(P, scenes, steps, prec, tile):
    b = P.Batch(len(scenes) + 2, 1 << 30, prec)
    b.set_tile(tile)
    slots = [b.admit(s, steps) for s in scenes]
    assert all(x is not None for x in slots)
    for _ in range(steps):
        b.step()
    return [b.state(s) for s in slots]


def _ref(sc, steps):
    o = oracle.Oracle(sc)
    o.step(steps)
    return o.state()


def test_hinges_and_world_anchors_fp64(P):
    scs = _scenes(S.PREC_FP64)
    print(f"[case] tile 64 fp64 {[s.name for s in scs]}", flush=True)
    got = _run(P, scs, 25, S.PREC_FP64, 64)
    for sc, st in zip(scs, got):
        e = errors(st, _ref(sc, 25), scale_of(sc))
        assert fp64_ok(e), (sc.name, e)


@pytest.mark.parametrize("steps,tol", [(1, 1e-4), (40, 1e-3)])
def test_hinges_and_world_anchors_fp32(P, steps, tol):
    scs = _scenes(S.PREC_FP32)
    print(f"[case] tile 64 fp32 steps {steps}", flush=True)
    got = _run(P, scs, steps, S.PREC_FP32, 64)
    for sc, st in zip(scs, got):
        e = errors(st, _ref(sc, steps), scale_of(sc))
        assert e["pos"] <= tol and e["rot"] <= tol, (sc.name, e)


def test_hinge_chain_same_in_every_tile_size(P):
    """The mirror pairing and the long way give the same bits whatever the tile."""
    scs = [_hinge_chain(n, S.PREC_FP32, k % 2 == 0, seed=k) for k, n in enumerate((4, 11, 29))]
    ref = _run(P, scs, 8, S.PREC_FP32, 32)
    for tile in (64, 128, 256):
        got = _run(P, scs, 8, S.PREC_FP32, tile)
        for x, y in zip(ref, got):
            for a, c in zip(x, y):
                np.testing.assert_array_equal(a, c)


@pytest.mark.parametrize("prec,steps,tol,tile", [(S.PREC_FP64, 10, None, 128),
                                                 (S.PREC_FP64, 10, None, 256),
                                                 (S.PREC_FP32, 1, 1e-4, 128),
                                                 (S.PREC_FP32, 1, 1e-4, 256)])
def test_spring_net_in_a_tile(P, prec, steps, tol, tile):
    """The 11 x 11 net (121 bodies, four springs with rest lengths per inner body)
    in one tile of 128 or 256 bodies."""
    sc = S.spring_net(11, order=2, precision=prec)
    print(f"[case] net tile {tile} prec {prec}", flush=True)
    (st,) = _run(P, [sc], steps, prec, tile)
    e = errors(st, _ref(sc, steps), scale_of(sc))
    if tol is None:
        assert fp64_ok(e), e
    else:
        assert e["pos"] <= tol and e["rot"] <= tol, e


@pytest.mark.parametrize("prec", [S.PREC_FP32, S.PREC_FP64])
def test_mixed_tiles_same_bits_in_every_grouping(P, prec):
    """Chains whose every end pairs with a mirror end beside hinge chains (more
    ends per body than a lane keeps in registers) and a chain hung from the
    world (an end taken the long way): a workgroup holding any of the latter
    publishes q^k in every iteration, one of chains alone only in a step's
    first.  Every tile size (so every grouping of scenes into workgroups) and
    each scene alone give the same bits, over three launches of five steps."""
    scs = (S.batched_chains(6, seed=8, precision=prec, hi=30) +
           [_hinge_chain(9, prec, True, seed=3), _world_chain(6, prec)] +
           S.batched_chains(5, seed=9, precision=prec, hi=30))

    def run(scenes, tile):
        b = P.Batch(len(scenes) + 2, 1 << 28, prec)
        b.set_tile(tile)
        slots = [b.admit(s, 15) for s in scenes]
        for _ in range(3):
            b.step(nsteps=5)
        out = [b.state(s) for s in slots]
        b.close()
        return out

    ref = run(scs, 64)
    for tile in (32, 128, 256):
        print(f"[case] mixed tiles, prec {prec}, tile {tile}", flush=True)
        for x, y in zip(ref, run(scs, tile)):
            for a, c in zip(x, y):
                np.testing.assert_array_equal(a, c)
    for k in (0, 6, 7, 12):
        print(f"[case] mixed tiles, prec {prec}, {scs[k].name} alone", flush=True)
        (alone,) = run([scs[k]], 64)
        for a, c in zip(ref[k], alone):
            np.testing.assert_array_equal(a, c)
