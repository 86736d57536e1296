"""Serving loop: continuous batching of simulation requests on one GPU.

Requests (a scene description and a number of steps) arrive over time.  The
server keeps one batch resident on the device; every iteration of its loop it
admits waiting requests in arrival order while a slot and enough of the HBM
budget are free (admission is a copy into the batch's arrays -- the captured
step graph is rebuilt only when the set of resident scenes changed), advances
every resident scene one step with a single graph replay, and hands back the
scenes that have taken all their steps, freeing their slot and memory for the
next arrivals.  Work of scenes admitted at different times overlaps on the
device within each replay.

Failures stay with their scene: a request the batch cannot take at all (a
descriptor it rejects, or one larger than the whole budget) is rejected with
the reason and the loop goes on; every few replays the batch's fault list is
read, and a scene that diverged (non-finite state, or contact capacity
exceeded) is evicted at once.  Such scenes are reported with their status and
count neither as completed nor in the throughput.

Reported: per-step latency (wall time of the replay that advanced a scene, as
seen by that scene), aggregate body-iterations per second, queueing delay.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import _lib
from .scenes import Request


@dataclasses.dataclass
class Result:
    index: int
    scene_name: str
    n_bodies: int
    steps: int
    arrival_s: float
    admitted_s: float
    finished_s: float
    state: tuple
    residual: float
    status: str = "ok"  # "ok", "diverged" (evicted, state dropped) or "rejected"
    reason: str = ""


@dataclasses.dataclass
class ServeStats:
    wall_s: float
    body_iterations: float
    body_its_per_s: float
    step_latency_ms: np.ndarray
    p50_step_ms: float
    p99_step_ms: float
    queue_wait_ms_p50: float
    queue_wait_ms_p99: float
    completed: int
    rejected: int
    diverged: int
    replays: int
    max_resident: int
    peak_bytes: int

    def summary(self) -> dict:
        return dict(wall_s=self.wall_s, body_its_per_s=self.body_its_per_s,
                    body_iterations=self.body_iterations, p50_step_ms=self.p50_step_ms,
                    p99_step_ms=self.p99_step_ms, queue_wait_ms_p50=self.queue_wait_ms_p50,
                    queue_wait_ms_p99=self.queue_wait_ms_p99, completed=self.completed,
                    rejected=self.rejected, diverged=self.diverged, replays=self.replays,
                    max_resident=self.max_resident,
                    peak_bytes=self.peak_bytes)


# Launch schedule of a server's own batch: eight lanes per contact body, so that
# a pile body's contact ends take half as many rounds of dependent loads per
# iteration.  A served step waits on its slowest body's chain, so this lowers the
# step latency at a given load, at the cost of some throughput at saturation (the
# per-body solve runs on one lane of eight instead of one of four).  Every scene
# of a server runs under it, alone or in the mix, so its results keep their bits
# either way.
SERVE_SCHEDULE = dict(tile_bodies=64, contact_lanes=8, group_waves=1)


class Server:
    """Continuous-batching server over one pabd batch (or any object with the
    same admit / step / sync / poll / state / residual / release / memory
    methods)."""

    def __init__(self, hbm_budget: int, max_slots: int, precision: int,
                 clock: Callable[[], float] = time.perf_counter, batch=None,
                 fault_check_every: int = 8, schedule: Optional[dict] = None):
        if batch is None:
            batch = _lib.Batch(max_slots, hbm_budget, precision)
            if schedule is None:
                schedule = SERVE_SCHEDULE
        self.batch = batch
        if schedule:  # e.g. a pick of Batch.tune on a sample of the load
            self.batch.set_schedule(**{k: int(schedule[k]) for k in
                                       ("tile_bodies", "contact_lanes", "group_waves")})
        self.precision = precision
        self.clock = clock
        # replays between two reads of the batch's fault list (each read waits
        # for the device and copies one word per slot)
        self.fault_check_every = max(1, int(fault_check_every))

    def close(self):
        self.batch.close()

    def run(self, requests: List[Request], realtime: bool = True,
            keep_state: bool = True, max_wall_s: Optional[float] = None) -> tuple:
        """Serve ``requests`` (sorted by arrival).  With ``realtime`` the arrival
        times are honoured against the wall clock; otherwise every request is
        available at once.  Returns (results by request index, ServeStats)."""
        b = self.batch
        pending = collections.deque()
        nxt = 0
        resident: Dict[int, dict] = {}
        results: Dict[int, Result] = {}
        lat = []
        waits = []
        body_its = 0.0
        replays = 0
        max_res = 0
        peak = 0
        t0 = self.clock()
        order = sorted(range(len(requests)), key=lambda k: requests[k].arrival_s)
        # set when the head of the queue found no room: room appears only when a
        # scene leaves, so admission is not tried again until one does (a failed
        # admission costs a host-side scene build)
        blocked = False

        def reject(k, reason):
            req = requests[k]
            results[k] = Result(index=k, scene_name=req.scene.name, n_bodies=req.scene.n_bodies,
                                steps=0, arrival_s=req.arrival_s, admitted_s=-1.0,
                                finished_s=self.clock() - t0, state=None, residual=float("nan"),
                                status="rejected", reason=reason)

        def evict(slot, reason):
            # a diverged scene: its work leaves the throughput, its slot is freed
            nonlocal body_its, blocked
            r = resident.pop(slot)
            req = requests[r["k"]]
            body_its -= r["done"] * r["n"] * r["iters"]
            results[r["k"]] = Result(index=r["k"], scene_name=req.scene.name, n_bodies=r["n"],
                                     steps=r["done"], arrival_s=req.arrival_s,
                                     admitted_s=r["admitted"], finished_s=self.clock() - t0,
                                     state=None, residual=float("nan"), status="diverged",
                                     reason=reason)
            b.release(slot)
            blocked = False

        while nxt < len(order) or pending or resident:
            now = self.clock() - t0
            if max_wall_s is not None and now > max_wall_s:
                break
            while nxt < len(order) and (not realtime or requests[order[nxt]].arrival_s <= now):
                pending.append(order[nxt])
                nxt += 1
            # admit in arrival order while room is free
            while pending and not (blocked and resident):
                k = pending[0]
                req = requests[k]
                try:
                    slot = b.admit(req.scene, req.steps)
                except _lib.PabdError as e:
                    # the batch can never take this scene (e.g. more contact ends
                    # per body than it holds): reject it, keep serving the rest
                    pending.popleft()
                    reject(k, str(e))
                    continue
                if slot is None:
                    if not resident:
                        # nothing resident and still no room: the request can
                        # never fit this server's budget; reject it
                        pending.popleft()
                        reject(k, "larger than the HBM budget")
                        continue
                    blocked = True
                    break
                pending.popleft()
                t_adm = self.clock() - t0
                waits.append(1e3 * max(0.0, t_adm - (req.arrival_s if realtime else 0.0)))
                resident[slot] = dict(k=k, admitted=t_adm, n=req.scene.n_bodies,
                                      iters=req.scene.iters, steps=req.steps, done=0)
            if not resident:
                if nxt < len(order) and realtime:
                    time.sleep(max(0.0, min(0.001, requests[order[nxt]].arrival_s - now)))
                continue
            max_res = max(max_res, len(resident))
            peak = max(peak, b.memory()[0])
            ts = self.clock()
            b.step()
            b.sync()
            dt = self.clock() - ts
            replays += 1
            for slot, r in resident.items():
                if r["done"] < r["steps"]:
                    r["done"] += 1
                    lat.append(1e3 * dt)
                    body_its += r["n"] * r["iters"]
            finished = b.poll()
            if finished or replays % self.fault_check_every == 0:
                for slot, code in b.faults().items():
                    if slot in resident:
                        evict(slot, f"health bits {code}: " +
                              ("non-finite state" if code & 1 else "contact capacity exceeded"))
            for slot in finished:
                if slot not in resident:
                    continue
                r = resident.pop(slot)
                req = requests[r["k"]]
                st = b.state(slot) if keep_state else None
                rho = b.residual(slot)
                results[r["k"]] = Result(index=r["k"], scene_name=req.scene.name, n_bodies=r["n"],
                                         steps=r["steps"], arrival_s=req.arrival_s,
                                         admitted_s=r["admitted"], finished_s=self.clock() - t0,
                                         state=st, residual=rho)
                b.release(slot)
                blocked = False
        wall = self.clock() - t0
        lat = np.asarray(lat) if lat else np.zeros(1)
        waits = np.asarray(waits) if waits else np.zeros(1)
        stats = ServeStats(wall_s=wall, body_iterations=body_its, body_its_per_s=body_its / max(wall, 1e-9),
                           step_latency_ms=lat, p50_step_ms=float(np.percentile(lat, 50)),
                           p99_step_ms=float(np.percentile(lat, 99)),
                           queue_wait_ms_p50=float(np.percentile(waits, 50)),
                           queue_wait_ms_p99=float(np.percentile(waits, 99)),
                           completed=sum(1 for r in results.values() if r.status == "ok"),
                           rejected=sum(1 for r in results.values() if r.status == "rejected"),
                           diverged=sum(1 for r in results.values() if r.status == "diverged"),
                           replays=replays, max_resident=max_res, peak_bytes=peak)
        return results, stats


