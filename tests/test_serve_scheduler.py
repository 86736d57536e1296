"""The serving loop's scheduling on the CPU: the device batch is replaced by an
executor with the same interface that runs every scene on the FP64 oracle, so
admission order, HBM-budget accounting, step counting and completion can be
checked without a GPU."""
import numpy as np

import oracle
from paper_2609_02675_amd import scenes as S
from paper_2609_02675_amd.serve import Server


def fake_bytes(sc):
    return 1000 * sc.n_bodies + 100 * sc.n_bonds


class OracleBatch:
    def __init__(self, budget, max_slots):
        self.budget, self.max_slots, self.used = budget, max_slots, 0
        self.slots = {}
        self.admitted = []
        self.admit_calls = 0
        self.releases = 0

    def admit(self, scene, steps):
        self.admit_calls += 1
        need = fake_bytes(scene)
        if self.used + need > self.budget or len(self.slots) >= self.max_slots:
            return None
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = dict(o=oracle.Oracle(scene), steps=steps, done=0, bytes=need)
        self.used += need
        self.admitted.append(scene.name)
        return slot

    def step(self):
        for s in self.slots.values():
            if s["done"] < s["steps"]:
                s["o"].step(1)
                s["done"] += 1

    def sync(self):
        pass

    def poll(self):
        return [k for k, s in self.slots.items() if s["done"] >= s["steps"]]

    def faults(self):
        # a scene whose oracle state is no longer finite has failed
        return {k: 1 for k, s in self.slots.items() if not np.isfinite(s["o"].state()[0]).all()}

    def state(self, slot, check=True):
        return self.slots[slot]["o"].state()

    def residual(self, slot):
        return float(self.slots[slot]["o"].residuals()[-1])

    def release(self, slot):
        self.releases += 1
        self.used -= self.slots.pop(slot)["bytes"]

    def memory(self):
        return self.used, self.budget

    def close(self):
        pass


def small_requests(n=14, seed=5):
    reqs = S.serving_requests(rate_hz=1000.0, duration_s=1.0, seed=seed, n_lo=4, n_hi=40,
                              steps_lo=3, steps_hi=12, precision=S.PREC_FP64, max_requests=n)
    return reqs


def test_scheduler_admits_in_order_within_budget_and_completes_all():
    reqs = small_requests()
    budget = sum(fake_bytes(r.scene) for r in reqs) // 3
    fb = OracleBatch(budget, max_slots=6)
    srv = Server(budget, 6, S.PREC_FP64, batch=fb)
    results, st = srv.run(reqs, realtime=False)
    order = sorted(range(len(reqs)), key=lambda k: reqs[k].arrival_s)
    fits = [k for k in order if fake_bytes(reqs[k].scene) <= budget]
    assert fb.admitted == [reqs[k].scene.name for k in fits]  # FIFO
    assert st.peak_bytes <= budget
    assert st.max_resident < len(reqs)  # requests had to wait for room
    # a request that found no room is tried again only after a scene left: at
    # most one failed admission per release (plus the ones that were admitted)
    assert fb.admit_calls <= len(fits) + fb.releases
    for k in fits:
        assert results[k].steps == reqs[k].steps
        o = oracle.Oracle(reqs[k].scene)
        o.step(reqs[k].steps)
        for a, b in zip(results[k].state, o.state()):
            np.testing.assert_array_equal(a, b)
    # scenes larger than the whole budget are rejected, not left waiting
    for k in set(order) - set(fits):
        assert results[k].admitted_s < 0


def test_step_latency_and_throughput_accounting():
    reqs = small_requests(6, seed=9)
    fb = OracleBatch(1 << 40, max_slots=8)
    srv = Server(1 << 40, 8, S.PREC_FP64, batch=fb)
    results, st = srv.run(reqs, realtime=False)
    assert st.replays == max(r.steps for r in reqs)
    assert len(st.step_latency_ms) == sum(r.steps for r in reqs)
    assert st.body_iterations == sum(r.scene.n_bodies * r.scene.iters * r.steps for r in reqs)


def test_inadmissible_request_is_rejected_and_serving_continues():
    """A request the batch refuses outright (here: a PabdError for one scene, as
    the library raises for a scene with more contact ends per body than the batch
    holds) is rejected with its reason; every other request still completes."""
    from paper_2609_02675_amd import _lib
    reqs = small_requests(n=8)
    bad_name = reqs[3].scene.name

    class Refusing(OracleBatch):
        def admit(self, scene, steps):
            if scene.name == bad_name:
                raise _lib.PabdError(-1, "the scene needs more contact slots than the batch holds (capacity)")
            return super().admit(scene, steps)

    srv = Server(0, 0, S.PREC_FP64, batch=Refusing(1 << 30, 4))
    res, st = srv.run(reqs, realtime=False)
    assert res[3].status == "rejected" and "capacity" in res[3].reason
    assert st.rejected == 1 and st.completed == len(reqs) - 1 and st.diverged == 0
    assert all(res[k].status == "ok" and res[k].state is not None for k in range(len(reqs)) if k != 3)


def test_diverged_scene_is_evicted_and_left_out_of_the_throughput():
    """A scene whose state turns non-finite while resident is found by the
    periodic fault check, evicted with status "diverged", and its iterations are
    taken out of the throughput; the other scenes complete."""
    reqs = small_requests(n=6)
    victim = 2

    class Poisoning(OracleBatch):
        def step(self):
            super().step()
            for s in self.slots.values():
                if s["o"].n and s["done"] == 2 and s.get("name") == reqs[victim].scene.name:
                    c = s["o"]
                    st = list(c.state())
                    # restart that scene from a non-finite state
                    st[0] = st[0] * np.nan
                    s["o"] = oracle.Oracle(reqs[victim].scene.with_state(*st))

        def admit(self, scene, steps):
            slot = super().admit(scene, steps)
            if slot is not None:
                self.slots[slot]["name"] = scene.name
            return slot

    batch = Poisoning(1 << 30, 8)
    srv = Server(0, 0, S.PREC_FP64, batch=batch, fault_check_every=1)
    res, st = srv.run(reqs, realtime=False)
    assert res[victim].status == "diverged" and res[victim].state is None
    assert st.diverged == 1 and st.completed == len(reqs) - 1
    expect = sum(r.scene.n_bodies * r.scene.iters * r.steps for k, r in enumerate(reqs) if k != victim)
    assert st.body_iterations == expect


def test_server_applies_a_given_schedule_to_its_batch():
    calls = []

    class Scheduled(OracleBatch):
        def set_schedule(self, **kw):
            calls.append(kw)

    sch = dict(tile_bodies=128, contact_lanes=8, group_waves=2, from_cache=1)
    Server(1 << 30, 4, S.PREC_FP64, batch=Scheduled(1 << 30, 4), schedule=sch)
    assert calls == [dict(tile_bodies=128, contact_lanes=8, group_waves=2)]
    Server(1 << 30, 4, S.PREC_FP64, batch=Scheduled(1 << 30, 4))
    assert len(calls) == 1
