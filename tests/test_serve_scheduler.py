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

    def admit(self, scene, steps):
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

    def state(self, slot, check=True):
        return self.slots[slot]["o"].state()

    def residual(self, slot):
        return float(self.slots[slot]["o"].residuals()[-1])

    def release(self, slot):
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
