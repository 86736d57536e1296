"""GPU contact-bond construction and contact dynamics against the oracle.

The discrete contact set (which point of which body touches which surface) is
compared exactly in FP64 mode; the states within the FP64/FP32 tolerances.
Contact-rich starting states are made by the oracle alone."""
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


def settled_drop(n_side=4, layers=2, steps=90, seed=0):
    """A small box drop advanced by the oracle until many contacts exist."""
    sc = S.box_drop(n_side=n_side, layers=layers, seed=seed, precision=S.PREC_FP64)
    o = oracle.Oracle(sc)
    o.step(steps)
    c, A, v, w = o.state()
    return sc.with_state(c, A, v, w, t0=steps * sc.h)


def _contact_table(ct):
    key = np.stack([ct["i"], ct["j"], ct["feature"]], axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    return key[order], {k: v[order] for k, v in ct.items()}


def _compare_contacts(g, o):
    kg, cg = _contact_table(g.contacts())
    ko, co = _contact_table(o.contacts())
    assert len(kg) > 0
    np.testing.assert_array_equal(kg, ko)
    for f in ("x_i", "x_j", "normal", "kappa"):
        np.testing.assert_allclose(cg[f], co[f], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_contact_set_matches_oracle_fp64(P, seed):
    sc = settled_drop(seed=seed)
    print(f"[case] contact set seed {seed} n={sc.n_bodies}", flush=True)
    g = P.Scene(sc)
    g.step(1)
    o = oracle.Oracle(sc)
    o.step(1)
    _compare_contacts(g, o)
    assert fp64_ok(errors(g.state(), o.state(), scale_of(sc)))


def test_contact_dynamics_fp64_several_steps(P):
    sc = settled_drop(seed=2)
    g = P.Scene(sc)
    g.step(10)
    o = oracle.Oracle(sc)
    o.step(10)
    e = errors(g.state(), o.state(), scale_of(sc))
    print("contact fp64 10 steps", e)
    assert e["pos"] <= 1e-9 and e["rot"] <= 1e-9


def test_contact_dynamics_fp32_one_step(P):
    sc = settled_drop(seed=3).copy(precision=S.PREC_FP32)
    g = P.Scene(sc)
    g.step(1)
    o = oracle.Oracle(sc)
    o.step(1)
    e = errors(g.state(), o.state(), scale_of(sc))
    print("contact fp32 1 step", e)
    assert e["pos"] <= 1e-4 and e["rot"] <= 1e-4


def test_mass_ratio_stack_fp64(P):
    sc = S.box_stack(n=6, mass_ratio=10.0)
    g = P.Scene(sc)
    g.step(60)
    o = oracle.Oracle(sc)
    o.step(60)
    assert fp64_ok(errors(g.state(), o.state(), scale_of(sc)))


def test_spheres_and_boxes_fp64(P):
    """Sphere-sphere, sphere-plane, sphere-box and box-plane contacts."""
    rng = np.random.default_rng(4)
    n = 40
    sc = S.box_drop(n_side=2, layers=1, seed=4, precision=S.PREC_FP64)
    sp = S.single_body(shape=S.SHAPE_SPHERE, half=(0.2, 0, 0), density=800.0)
    spheres = []
    for k in range(n):
        spheres.append(sp.copy(c0=np.array([[rng.uniform(-2, 2), 0.25 + 0.45 * k / 4, rng.uniform(-2, 2)]]),
                               shape_param=np.array([[rng.uniform(0.15, 0.3), 0, 0]])))
    sc = S.merge([sc] + spheres).copy(contact_enable=1, planes=np.array([[0.0, 1.0, 0.0, 0.0]]),
                                      precision=S.PREC_FP64)
    o = oracle.Oracle(sc)
    o.step(40)
    c, A, v, w = o.state()
    sc = sc.with_state(c, A, v, w, t0=40 * sc.h)
    g = P.Scene(sc)
    g.step(1)
    o = oracle.Oracle(sc)
    o.step(1)
    _compare_contacts(g, o)
    g.step(9)
    o.step(9)
    assert fp64_ok(errors(g.state(), o.state(), scale_of(sc)))


def test_contact_capacity_overflow_is_reported(P):
    sc = settled_drop(seed=0).copy(max_contacts_per_body=2)
    g = P.Scene(sc)
    g.step(1)
    with pytest.raises(P.Diverged):
        g.state()


def test_contact_scenes_in_a_batch_fp64(P):
    scs = [settled_drop(n_side=3, layers=1, steps=60, seed=s) for s in (5, 6)]
    b = P.Batch(8, 1 << 28, S.PREC_FP64)
    slots = [b.admit(s, 8) for s in scs]
    chains = S.batched_chains(3, seed=4, precision=S.PREC_FP64)
    cslots = [b.admit(s, 8) for s in chains]
    for _ in range(8):
        b.step()
    for sc, sl in zip(scs + chains, slots + cslots):
        o = oracle.Oracle(sc)
        o.step(8)
        assert fp64_ok(errors(b.state(sl), o.state(), scale_of(sc))), sc.name


def test_body_with_more_ends_than_a_wave_holds_fp64(P):
    """A wide plate resting on an 18 x 18 grid of spheres holds 324 contact ends,
    more than the sort keeps in registers (256 per body): its ends take the
    sort's path through memory, and the contact set and state still match."""
    r, n = 0.1, 18
    sp = S.single_body(shape=S.SHAPE_SPHERE, half=(r, 0, 0), density=1000.0)
    xs = (np.arange(n) - (n - 1) / 2) * 2.2 * r
    balls = [sp.copy(c0=np.array([[x, r - 1e-4, z]])) for x in xs for z in xs]
    half = 0.5 * n * 2.2 * r
    plate = S.single_body(shape=S.SHAPE_BOX, half=(half, 0.05, half), density=200.0,
                          c=(0.0, 2 * r + 0.05 - 2e-4, 0.0))
    sc = S.merge([plate] + balls).copy(contact_enable=1, planes=np.array([[0.0, 1.0, 0.0, 0.0]]),
                                       max_contacts_per_body=512, precision=S.PREC_FP64)
    print(f"[case] plate on {n * n} spheres, n={sc.n_bodies}", flush=True)
    g = P.Scene(sc)
    g.step(1)
    o = oracle.Oracle(sc)
    o.step(1)
    _compare_contacts(g, o)
    ct = g.contacts()  # every bond gives an end to each of its two bodies
    assert np.count_nonzero((ct["i"] == 0) | (ct["j"] == 0)) > 256
    g.step(2)
    o.step(2)
    assert fp64_ok(errors(g.state(), o.state(), scale_of(sc)))


@pytest.mark.parametrize("prec", [S.PREC_FP64, S.PREC_FP32])
def test_contact_and_plain_flat_scenes_share_a_batch(P, prec):
    """A 300-body chain (flat path, no contacts) beside two box piles in one batch:
    the chain's waves take one lane per body as they do alone, so its result is
    the same alone and in the mix bit for bit; the chain matches the oracle
    (FP64 bar, or FP32 within 1e-4 after 8 steps), and so do the piles in FP64
    (box piles are chaotic under FP32 rounding, so they are not held to the
    oracle over 8 steps in FP32)."""
    big = S.chain(300, tilt_deg=20.0, joint_angles_deg=np.linspace(-5, 5, 299),
                  precision=prec, iters=12)
    piles = [settled_drop(n_side=3, layers=1, steps=60, seed=s).copy(precision=prec) for s in (5, 6)]
    print(f"[case] chain 300 beside two piles prec {prec}", flush=True)
    b = P.Batch(8, 1 << 28, prec)
    sb = b.admit(big, 8)
    sp = [b.admit(p, 8) for p in piles]
    for _ in range(8):
        b.step()
    alone = P.Batch(4, 1 << 28, prec)
    sa = alone.admit(big, 8)
    for _ in range(8):
        alone.step()
    for x, y in zip(b.state(sb), alone.state(sa)):
        np.testing.assert_array_equal(x, y)

    def ok(e):
        if prec == S.PREC_FP64:
            return fp64_ok(e)
        return e["pos"] <= 1e-4 and e["rot"] <= 1e-4

    o = oracle.Oracle(big)
    o.step(8)
    e = errors(b.state(sb), o.state(), scale_of(big))
    assert ok(e), e
    if prec != S.PREC_FP64:
        return
    for pl, s in zip(piles, sp):
        o = oracle.Oracle(pl)
        o.step(8)
        e = errors(b.state(s), o.state(), scale_of(pl))
        assert ok(e), (pl.name, e)


def test_box_drop_1000_full_size_from_a_landing_state(P):
    """The 1,000-box drop at full size, from the oracle's state at step 60 (the
    lowest boxes landing, about 600 contact bonds): one GPU step in FP64 has the
    oracle's contact set and state; in FP32, positions and rotations within 1e-4."""
    sc = S.box_drop(precision=S.PREC_FP64)
    o = oracle.Oracle(sc)
    o.step(60)
    c, A, v, w = o.state()
    st = sc.with_state(c, A, v, w, t0=60 * sc.h)
    print(f"[case] box drop n={st.n_bodies} from step 60", flush=True)
    ref = oracle.Oracle(st)
    ref.step(1)
    g = P.Scene(st)
    g.step(1)
    _compare_contacts(g, ref)
    assert fp64_ok(errors(g.state(), ref.state(), scale_of(st)))
    g32 = P.Scene(st.copy(precision=S.PREC_FP32))
    g32.step(1)
    e = errors(g32.state(), ref.state(), scale_of(st))
    print("box drop fp32 one step", e)
    assert e["pos"] <= 1e-4 and e["rot"] <= 1e-4


def test_empty_and_single_body_contact_scenes(P):
    """The all-pairs broad phase at its smallest: a contact scene with no body,
    and one box (no pair at all) coming to rest on the plane, against the oracle."""
    drop = S.box_drop(n_side=2, layers=1, precision=S.PREC_FP64)
    empty = drop.copy(shape=np.zeros(0, np.int32), shape_param=np.zeros((0, 3)), density=np.zeros(0),
                      flags=np.zeros(0, np.uint8), group=np.zeros(0, np.int32), c0=np.zeros((0, 3)),
                      A0=np.zeros((0, 3, 3)), v0=np.zeros((0, 3)), w0=np.zeros((0, 3)))
    print("[case] empty contact scene", flush=True)
    g = P.Scene(empty)
    g.step(3)
    assert g.state()[0].shape == (0, 3)
    keep = [0]
    one = drop.copy(shape=drop.shape[keep], shape_param=drop.shape_param[keep], density=drop.density[keep],
                    flags=drop.flags[keep], group=drop.group[keep], A0=drop.A0[keep], v0=drop.v0[keep],
                    w0=drop.w0[keep], c0=np.array([[0.0, 0.9, 0.0]]))
    print("[case] one box on the plane", flush=True)
    g = P.Scene(one)
    o = oracle.Oracle(one)
    for _ in range(3):
        g.step(10)
        o.step(10)
    _compare_contacts(g, o)
    assert fp64_ok(errors(g.state(), o.state(), scale_of(one)))


def test_fp32_contact_records_decode_to_the_fp64_ones(P):
    """The FP32 contact record keeps the normal in octahedral form and takes the
    stiffness from the two bodies' q records.  On the same settled state, every
    contact the FP32 and FP64 scenes both find must read back the FP64 record's
    points and normal to float rounding, and its stiffness as the FP64 one
    rounded to float (the larger of the two rounded body shares is the rounded
    larger share)."""
    sc = settled_drop(seed=4)
    print(f"[case] fp32 contact records n={sc.n_bodies}", flush=True)
    g64 = P.Scene(sc)
    g64.step(1)
    g32 = P.Scene(sc.copy(precision=S.PREC_FP32))
    g32.step(1)
    k64, c64 = _contact_table(g64.contacts())
    k32, c32 = _contact_table(g32.contacts())
    pos = {tuple(k): n for n, k in enumerate(map(tuple, k64))}
    both = [(pos[tuple(k)], n) for n, k in enumerate(map(tuple, k32)) if tuple(k) in pos]
    assert len(both) >= 0.9 * max(len(k64), len(k32)) and len(both) > 50
    a = np.array([x for x, _ in both])
    b = np.array([y for _, y in both])
    n64, n32 = c64["normal"][a], c32["normal"][b]
    assert np.abs(np.linalg.norm(n32, axis=1) - 1.0).max() < 1e-6
    assert np.abs(n32 - n64).max() < 1e-6
    for f in ("x_i", "x_j"):
        assert np.abs(c32[f][b] - c64[f][a]).max() < 1e-5
    h2 = sc.h * sc.h
    want = (np.float32(c64["kappa"][a] * h2)).astype(np.float64) / h2
    np.testing.assert_allclose(c32["kappa"][b], want, rtol=1e-12)
