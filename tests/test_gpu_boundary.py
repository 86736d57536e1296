"""The boundary's calls that follow the problem statement (Sec. 4.1.1, Algorithm
1), through the C ABI on the GPU: a generalised mass given directly with an
affine moment that no box or sphere has, the last-iteration residual, fault
injection, and the local step's SVD fallback (Sec. 4.2.2: det A^{k+1/2} <= 0 or
nearly singular) against the oracle's SVD with the determinant fix."""
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


def _oracle(sc, steps):
    o = oracle.Oracle(sc)
    o.step(steps)
    return o


def test_general_inertia_plain_path_fp64(P):
    sc = S.general_inertia_chain(precision=S.PREC_FP64)
    print(f"[case] {sc.name} plain fp64", flush=True)
    g = P.Scene(sc)
    g.step(60)
    e = errors(g.state(), _oracle(sc, 60).state(), scale_of(sc))
    print(e)
    assert fp64_ok(e)


def test_general_inertia_batched_tile_path_fp64(P):
    sc = S.general_inertia_chain(precision=S.PREC_FP64)
    print(f"[case] {sc.name} batched fp64", flush=True)
    b = P.Batch(4, 64 << 20, S.PREC_FP64)
    other = S.chain(12, tilt_deg=30.0, precision=S.PREC_FP64)
    s0 = b.admit(sc, 60)
    s1 = b.admit(other, 60)
    assert b.layout()["tiles"] == 1  # both in one tile
    for _ in range(6):
        b.step(nsteps=10)
    assert fp64_ok(errors(b.state(s0), _oracle(sc, 60).state(), scale_of(sc)))
    assert fp64_ok(errors(b.state(s1), _oracle(other, 60).state(), scale_of(other)))


def test_general_inertia_fp32_one_step(P):
    sc = S.general_inertia_chain(precision=S.PREC_FP32)
    g = P.Scene(sc)
    g.step(1)
    e = errors(g.state(), _oracle(sc, 1).state(), scale_of(sc))
    assert e["pos"] <= 1e-4 and e["rot"] <= 1e-4, e


def test_scene_residual_is_the_last_iteration_residual(P):
    sc = S.chain8(precision=S.PREC_FP64)
    g = P.Scene(sc)
    assert g.residual() == 0.0
    g.step(5)
    o = _oracle(sc, 5)
    assert g.residual() == pytest.approx(o.residuals()[-1], rel=1e-6)
    assert g.residual() == g.residuals()[-1]


def test_debug_poke_overwrites_one_component(P):
    sc = S.chain8(precision=S.PREC_FP64)
    g = P.Scene(sc)
    g.poke(3, 1, 7.25)      # c_y of body 3
    g.poke(5, 3 + 4, 0.5)   # A_11 of body 5
    g.poke(2, 15, -1.5)     # w_x of body 2
    c, A, v, w = g.state()
    assert c[3, 1] == 7.25 and A[5, 1, 1] == 0.5 and w[2, 0] == -1.5
    with pytest.raises(P.PabdError):
        g.poke(8, 0, 1.0)
    with pytest.raises(P.PabdError):
        g.poke(0, 18, 1.0)


# (kind, kappa, precision, bar on A and c after one step)
POLAR_CASES = [("flip", 1e7, S.PREC_FP64, 1e-12), ("flip", 1e7, S.PREC_FP32, 1e-6),
               ("flat", 1e9, S.PREC_FP64, 1e-12), ("flat", 1e9, S.PREC_FP32, 1e-6)]


def _polar_errors(st, ref):
    return (float(np.abs(st[1] - ref[1]).max()), float(np.abs(st[0] - ref[0]).max()))


@pytest.mark.parametrize("kind,kappa,prec,tol", POLAR_CASES,
                         ids=[f"{c[0]}-{'fp64' if c[2] else 'fp32'}" for c in POLAR_CASES])
def test_local_step_fallback_plain_path(P, kind, kappa, prec, tol):
    """One step of two iterations of a body whose global step gives A^{k+1/2}
    with det < 0 ("flip") or a tiny singular value ("flat"): the rotation is the
    nearest proper rotation, as the oracle's SVD with the determinant fix gives
    it.  The fallback counter shows the branch ran: in "flip" every iteration
    (both with det <= 0); in "flat" FP32 falls back (det below its floor of
    1e-6) while FP64 Newton still converges (det above 1e-12)."""
    sc = S.polar_fallback_body(kind, kappa=kappa, precision=prec)
    print(f"[case] polar {kind} plain prec={prec}", flush=True)
    g = P.Scene(sc)
    g.step(1)
    o = _oracle(sc, 1)
    _, qh = o.last_iterates()
    det = np.linalg.det(qh[0, 3:].reshape(3, 3))
    assert (det < 0) if kind == "flip" else (0 < det < 1e-6)
    ea, ec = _polar_errors(g.state(check=False), o.state())
    print(f"A err {ea:.3e} c err {ec:.3e}", g.polar_fallbacks())
    assert ea <= tol and ec <= tol
    svd, neg = g.polar_fallbacks()
    if kind == "flip":
        assert (svd, neg) == (2, 2)
    elif prec == S.PREC_FP32:
        assert svd == 2 and neg == 0
    else:
        assert (svd, neg) == (0, 0)


@pytest.mark.parametrize("kind,kappa,prec,tol", POLAR_CASES,
                         ids=[f"{c[0]}-{'fp64' if c[2] else 'fp32'}" for c in POLAR_CASES])
def test_local_step_fallback_tile_path(P, kind, kappa, prec, tol):
    """The same in a batch, where the body is tiled beside a chain: the tile
    kernel's continuation of the polar iteration (through LDS) and its counter."""
    sc = S.polar_fallback_body(kind, kappa=kappa, precision=prec)
    other = S.chain(10, tilt_deg=25.0, precision=prec)
    print(f"[case] polar {kind} tile prec={prec}", flush=True)
    b = P.Batch(4, 64 << 20, prec)
    s0 = b.admit(sc, 1)
    s1 = b.admit(other, 1)
    assert b.layout()["tiles"] == 1
    b.step()
    ea, ec = _polar_errors(b.state(s0, check=False), _oracle(sc, 1).state())
    assert ea <= tol and ec <= tol
    svd, neg = b.polar_fallbacks(s0)
    if kind == "flip":
        assert (svd, neg) == (2, 2)
    elif prec == S.PREC_FP32:
        assert svd == 2 and neg == 0
    assert b.polar_fallbacks(s1) == (0, 0)
    # the chain beside it is unaffected
    e = errors(b.state(s1), _oracle(other, 1).state(), scale_of(other))
    assert e["pos"] <= (1e-9 if prec == S.PREC_FP64 else 1e-4)


def _mixed_batch(P, prec):
    scs = S.batched_chains(5, seed=6, precision=prec)
    big = S.chain(80, tilt_deg=20.0, precision=prec, name="chain80")  # flat path (too long for a tile)
    pile = S.pile(60, seed=2, precision=prec)
    all_ = scs + [big, pile]
    b = P.Batch(16, 256 << 20, prec)
    slots = [b.admit(s, 40) for s in all_]
    return b, slots, all_


@pytest.mark.parametrize("victim", [1, 5, 6], ids=["tiled", "flat", "contact"])
def test_a_diverged_scene_is_reported_alone_and_neighbours_are_unchanged(P, victim):
    """A non-finite value poked into one resident scene: that slot, and only it,
    reports PABD_E_DIVERGED (pabd_batch_faults lists it, its read-back raises),
    and every other scene ends bit for bit where it ends in a batch without the
    poke."""
    prec = S.PREC_FP32
    print(f"[case] batch fault victim={victim}", flush=True)
    ref, ref_slots, scs = _mixed_batch(P, prec)
    bad, bad_slots, _ = _mixed_batch(P, prec)
    for b in (ref, bad):
        b.step(nsteps=5)
    bad.poke(bad_slots[victim], 1, 0, float("nan"))
    for b in (ref, bad):
        for _ in range(3):
            b.step(nsteps=5)
        b.sync()
    faults = bad.faults()
    assert list(faults) == [bad_slots[victim]] and faults[bad_slots[victim]] & 1
    assert ref.faults() == {}
    with pytest.raises(P.Diverged):
        bad.state(bad_slots[victim])
    for k, (a, b_) in enumerate(zip(ref_slots, bad_slots)):
        if k == victim:
            continue
        for x, y in zip(ref.state(a), bad.state(b_)):
            assert np.array_equal(x, y), scs[k].name
