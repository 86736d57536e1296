#!/usr/bin/env python3
"""Benchmark: affine-body SSM iterations per second on one MI355X.

Default workload: 4,096 independent joint chains of 4..64 unit cubes (ball joints,
+-30 degree random joint angles, top body pinned), FP32, 20 iterations per step,
all advanced together by the batched path (one captured-graph replay per 10
steps: one tile-kernel launch running every scene's steps from registers and
LDS).  Also reported on the same accuracy bar: the plain single-scene path (one kernel launch per
iteration) on a sample of the same scenes, the served mix (continuous
batching, see paper_2609_02675_amd/serve.py), and the FP64 CPU oracle on a
bounded sample (the CPU baseline).

Prints ONE JSON line.  `python bench.py --gpus N` with N > 1 exits: the library
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "affine-body SSM iterations/s (served/batched vs plain); p50/p99 step ms"
HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
# published MI355X vector FP32 peak: 256 CU x 128 lanes x 2 (FMA) x 2.4 GHz, which
# counts two-wide packed FMAs; every HIP source here is compiled without packed
# FP32 instructions, whose issue rate is half of it (78.6 TFLOP/s), reported beside
FP32_PEAK = 157.3e12
FP32_UNPACKED_PEAK = 78.6e12
# algorithmic bytes the tile kernel moves per body: once per launch it reads q
# (16 floats: c_hi, A, c_lo), v/w (8), mass (8), H^-1 factor (12), two bond ends
# (8 floats + partner id each), scene id, flags and end range; after every step
# it writes q and v/w
TILE_LOAD_BYTES_PER_BODY = 64 + 32 + 32 + 48 + 2 * (32 + 4) + 4 + 1 + 8
TILE_STORE_BYTES_PER_BODY_STEP = 64 + 32


def tile_bytes(n_bodies, steps_per_launch):
    return n_bodies * (TILE_LOAD_BYTES_PER_BODY + steps_per_launch * TILE_STORE_BYTES_PER_BODY_STEP)


# algorithmic flops of one body-iteration of a two-bond chain body, counted by
# hand from the operations the method needs (an estimate of the work, not a
# hardware count): bond terms (2 x 63), inertia term M (s - q) (81), closed-form
# block solve (84), increment (12), two Newton polar steps (2 x 90)
FLOPS_PER_BODY_ITER = 2 * 63 + 81 + 84 + 12 + 2 * 90


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TILE_SOURCES = ["common.h", "device_math.h", "kernels_step.h", "kernels_tile.h"]
# counter profile of the tile kernel, one file per workload
TILE_PROFILE = os.path.join(ROOT, "profiles", "k_tile_step_{workload}.md")


def tile_traffic(steps_per_launch, tile_bodies, workload):
    """HBM bytes per tile-kernel launch from the committed counter profile, if the
    kernel sources still hash to what was profiled and the profile ran the same
    workload, tile size and steps per launch; else None."""
    return tile_profile_value("traffic_bytes_per_launch", steps_per_launch, tile_bodies, workload)


def tile_valu(steps_per_launch, tile_bodies, workload):
    """VALU instructions (wave64) per tile-kernel launch, SQ_INSTS_VALU from the
    committed counter profile, under the same conditions as tile_traffic."""
    return tile_profile_value("valu_insts_per_launch", steps_per_launch, tile_bodies, workload)


def tile_profile_value(key, steps_per_launch, tile_bodies, workload):
    import hashlib
    h = hashlib.sha256()
    for f in TILE_SOURCES:
        with open(os.path.join(ROOT, "paper_2609_02675_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        text = open(TILE_PROFILE.format(workload=workload)).read()
    except OSError:
        return None
    import re
    m = re.search(r"kernel-source-sha256-16:\s*([0-9a-f]{16})", text)
    t = re.search(key + r":\s*(\d+)", text)
    n = re.search(r"steps_per_launch:\s*(\d+)", text)
    tb = re.search(r"tile_bodies:\s*(\d+)", text)
    w = re.search(r"workload:\s*(\S+)", text)
    if not (m and t and n and tb and w):
        return None
    if (m.group(1) != h.hexdigest()[:16] or int(n.group(1)) != steps_per_launch
            or int(tb.group(1)) != tile_bodies or w.group(1) != workload):
        return None
    return float(t.group(1))


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands, one scene per task
# ---------------------------------------------------------------------------

_SCENES = None


def _oracle_worker(args):
    k, steps = args
    import oracle
    sc = _SCENES[k]
    o = oracle.Oracle(sc)
    t = time.perf_counter()
    o.step(steps)
    return sc.n_bodies * sc.iters * steps, time.perf_counter() - t


def _pool_timing(scenes, n_sample, steps, cores):
    global _SCENES
    _SCENES = scenes[:n_sample]
    work = [(k, steps) for k in range(len(_SCENES))]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, work, chunksize=4)
    wall = time.perf_counter() - t0
    body_its = sum(r[0] for r in res)
    cpu_s = sum(r[1] for r in res)
    return dict(value=body_its / wall, unit="body-iterations/s", cores=cores, kind="oracle",
                per_core=body_its / cpu_s,
                sample=f"first {len(_SCENES)} of the batched chains, {steps} steps each, FP64 "
                       f"oracle, one scene per task on a {cores}-process pool "
                       f"({body_its:.3g} body-iterations, {wall:.1f} s wall)")


def cpu_baseline_leg(args, S, scenes, plan):
    """The CPU leg, run before the GPU is touched (so that fork is safe): the FP64
    oracle as it stands, timed on a bounded sample of the batched chains (the
    cpu_baseline) and on the single-scene workloads, and the oracle's results
    that the GPU legs state their error against. It is the only part of this
    script that runs the oracle."""
    import oracle
    oracle.build()
    cpu = None
    if not args.no_cpu_baseline:
        cores = min(16, os.cpu_count() or 1)
        sc64 = [s.copy(precision=S.PREC_FP64) for s in scenes[: args.cpu_sample]]
        cpu = _pool_timing(sc64, len(sc64), args.cpu_steps, cores)
        cpu["host"] = host_info()
        log("cpu baseline", cpu)

    def run(sc, steps):
        o = oracle.Oracle(sc.copy(precision=S.PREC_FP64))
        o.step(steps)
        return o.state()

    refs = {"batched": {k: run(scenes[k], plan["total_steps"]) for k in plan["batched_sample"]},
            "plain": {k: run(scenes[k], plan["plain_steps"]) for k in plan["plain_sample"]}}
    if plan["big_scenes"] is not None:
        refs["big"] = {k: run(plan["big_scenes"][k], plan["big_steps"]) for k in plan["big_sample"]}
    if plan["requests"]:
        refs["served"] = {k: run(plan["requests"][k].scene, plan["requests"][k].steps)
                          for k in plan["served_sample"]}
        refs["pile_mid"], refs["pile_next"] = {}, {}
        for k in plan["pile_sample"]:
            sc = plan["requests"][k].scene
            mid = sc.with_state(*run(sc, 60), t0=60 * sc.h)
            refs["pile_mid"][k] = mid
            refs["pile_next"][k] = run(mid, 1)
    if not args.no_scenes:
        # the box drop from the oracle's own state after 60 steps (contacts
        # active), and the oracle's next step from there
        drop = S.box_drop(precision=S.PREC_FP64)
        mid = drop.with_state(*run(drop, 60), t0=60 * drop.h)
        refs["drop_mid"] = mid
        refs["drop_next"] = run(mid, 1)
        refs["mass_ratio"] = {aug: run(S.mass_ratio_chain(augmented=aug), 110) for aug in (True, False)}
        refs["linkage"] = run(S.linkage("slider", drive_amp_deg=60.0), 120)
        # the oracle's own spread: the same chain from FP32-rounded inputs
        f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
        refs["mass_ratio_f32_inputs"] = {}
        for aug in (True, False):
            mc = S.mass_ratio_chain(augmented=aug)
            mc = mc.copy(c0=f32(mc.c0), x_i=f32(mc.x_i), x_j=f32(mc.x_j), rest_len=f32(mc.rest_len))
            refs["mass_ratio_f32_inputs"][aug] = run(mc, 110)
    if cpu is not None and not args.no_oracle_single:
        cpu["single_core_single_scene"] = oracle_single_core(oracle, S, refs.get("drop_mid"))
    return cpu, refs


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(logical_cpus=os.cpu_count(), model=model)


def big_batch_leg(P, S, torch, plan, refs):
    """The batched chains at 16x the default count (about 2.2M bodies, a working
    set well beyond the 256 MB last-level cache), tile 64, FP32, spl steps per
    tile-kernel launch."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import errors, scale_of
    spl = plan["spl"]
    scs = plan["big_scenes"]
    n_scenes = len(scs)
    t = time.perf_counter()
    nb = sum(x.n_bodies for x in scs)
    b = P.Batch(n_scenes + 8, 16 << 30, S.PREC_FP32)
    slots = [b.admit(x, 1 << 30) for x in scs]
    assert all(x is not None for x in slots)
    b.set_tile(64)
    log(f"big batch: {n_scenes} scenes, {nb} bodies admitted in {time.perf_counter() - t:.1f}s")
    stream = torch.cuda.Stream()
    sptr = stream.cuda_stream
    b.step(stream=sptr, nsteps=spl)  # warm-up and graph capture
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(BIG_TIMED_LAUNCHES):
        b.step(stream=sptr, nsteps=spl)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (BIG_TIMED_LAUNCHES * spl)
    iters = scs[0].iters
    launch_ms = b.time_tile_kernel(BIG_REPS, spl)
    tile_ms = launch_ms / spl
    flops = nb * iters * FLOPS_PER_BODY_ITER
    acc = 0.0
    for k in plan["big_sample"]:  # every scene has now taken plan["big_steps"] steps
        e = errors(b.state(slots[k]), refs["big"][k], scale_of(scs[k]))
        acc = max(acc, e["pos"], e["rot"])
    b.close()
    out = dict(scenes=n_scenes, bodies=nb, iters=iters, steps_per_launch=spl, ms_per_step=ms,
               body_its_per_s=nb * iters / (ms / 1e3), tile_kernel_ms_per_launch=launch_ms,
               tile_kernel_ms_per_step=tile_ms,
               alu_frac=flops / (tile_ms / 1e3) / FP32_PEAK,
               alu_frac_of_unpacked_peak=flops / (tile_ms / 1e3) / FP32_UNPACKED_PEAK,
               hbm_GBs_algorithmic=tile_bytes(nb, spl) / (launch_ms / 1e3) / 1e9,
               load_bytes_per_launch=nb * TILE_LOAD_BYTES_PER_BODY,
               max_rel_err_vs_fp64_oracle=acc, tile_bodies=64)
    log("big batch", out)
    return out


def oracle_single_core(oracle, S, drop_mid=None):
    """The FP64 oracle, one thread, on the single-scene workloads: the 8-chain
    (100 steps), the 1,000-box drop (5 steps with contacts active, from the
    oracle's own state at step 60) and the granular bed with the robot (1 step)."""
    out = {}
    sc = S.chain8(precision=S.PREC_FP64)
    o = oracle.Oracle(sc)
    t = time.perf_counter()
    o.step(100)
    dt = time.perf_counter() - t
    out["chain8"] = dict(body_its_per_s=sc.n_bodies * sc.iters * 100 / dt, steps=100, seconds=dt)
    drop = drop_mid if drop_mid is not None else S.box_drop(precision=S.PREC_FP64)
    o = oracle.Oracle(drop)
    t = time.perf_counter()
    o.step(5)
    dt = time.perf_counter() - t
    out["box_drop_1000"] = dict(body_its_per_s=drop.n_bodies * drop.iters * 5 / dt, steps=5,
                                seconds=dt, start="step 60" if drop_mid is not None else "step 0")
    bed = S.granular_bed_quadruped(precision=S.PREC_FP64)
    o = oracle.Oracle(bed)
    t = time.perf_counter()
    o.step(1)
    dt = time.perf_counter() - t
    out["granular_bed_quadruped"] = dict(body_its_per_s=bed.n_bodies * bed.iters / dt, steps=1, seconds=dt)
    out["threads"] = 1
    log("oracle single core", out)
    return out


# the big batch leg: one warm-up launch, BIG_TIMED_LAUNCHES timed launches, then
# the tile kernel alone BIG_REPS times (each after a warm launch)
BIG_TIMED_LAUNCHES, BIG_REPS = 2, 2
# the plain leg: untimed and timed steps of each scene
PLAIN_WARM, PLAIN_STEPS = 2, 10


def _plan(args, S, scenes):
    """What the GPU legs will run and which of their results the oracle checks,
    fixed before either side runs."""
    spl = args.steps_per_launch
    if spl < 1 or args.steps % spl:
        raise SystemExit("--steps must be a multiple of --steps-per-launch")
    warm_launches = max(1, -(-args.warmup // spl))
    rng = np.random.default_rng(1)
    plan = dict(spl=spl, launches=args.steps // spl, warm_launches=warm_launches,
                total_steps=warm_launches * spl + args.steps,
                batched_sample=[int(k) for k in rng.choice(len(scenes), 4, replace=False)],
                requests=[], served_sample=[], pile_sample=[], big_scenes=None, big_sample=(),
                big_steps=0, plain_steps=PLAIN_WARM + PLAIN_STEPS,
                plain_sample=list(range(min(3, args.plain_sample))))
    if args.serve_seconds > 0:
        reqs = S.serving_requests(rate_hz=200.0, duration_s=args.serve_seconds, seed=3,
                                  precision=S.PREC_FP32)
        plan["requests"] = reqs
        # chains: box piles are chaotic over hundreds of steps (FP32-rounded inputs
        # move the FP64 oracle itself by O(1)), so they are checked at short
        # horizons in the tests
        plan["served_sample"] = [k for k in range(len(reqs))
                                 if "chain" in reqs[k].scene.name and reqs[k].scene.n_bodies <= 80][:3]
        # piles over one step from the oracle's own state at step 60 (landing,
        # contacts active), served through the same loop
        plan["pile_sample"] = [k for k in range(len(reqs))
                               if "pile" in reqs[k].scene.name and 100 <= reqs[k].scene.n_bodies <= 400][:2]
    if args.big_scenes > 0:
        n = args.big_scenes
        plan["big_scenes"] = S.batched_chains(n, seed=2, precision=S.PREC_FP32)
        plan["big_sample"] = (0, n // 2, n - 1)
        plan["big_steps"] = (1 + BIG_TIMED_LAUNCHES + 1 + BIG_REPS) * spl
    return plan


# ---------------------------------------------------------------------------

def tile_occupancy_sweep(steps_per_launch=10):
    """The tile kernel alone on n identical tiles (one FP32 chain of 64 bodies
    each, K = 20, joints turned by -20..20 degrees), n = 1 to 6 tiles per SIMD,
    one 64-lane wave per tile: launch time against waves per SIMD.  Each point
    is the best of three means over five launches (HIP events)."""
    import torch
    import paper_2609_02675_amd as P
    from paper_2609_02675_amd import scenes as S
    if P.device_count() < 1:
        raise SystemExit("no HIP device visible")
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    base = S.chain(64, tilt_deg=0.0, joint_angles_deg=np.linspace(-20, 20, 63), kappa=1e5, iters=20,
                   precision=S.PREC_FP32, name="chain64")
    for per in (1.0, 2.0, 2.18, 3.0, 3.5, 4.5, 6.0):
        nt = int(round(per * simds))
        b = P.Batch(nt + 2, 4 << 30, S.PREC_FP32)
        b.set_tile(64)
        for _ in range(nt):
            assert b.admit(base, 1 << 30) is not None
        assert b.layout()["tiles"] == nt
        b.step(nsteps=steps_per_launch)
        b.sync()
        ms = min(b.time_tile_kernel(5, nsteps=steps_per_launch) for _ in range(3))
        print(json.dumps({"tiles_per_simd": per, "tiles": nt, "simds": simds,
                          "steps_per_launch": steps_per_launch, "ms_per_launch": ms,
                          "us_per_step": 1e3 * ms / steps_per_launch}), flush=True)
        b.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--steps-per-launch", type=int, default=10,
                    help="batched leg: steps one tile-kernel launch (one graph replay) runs")
    ap.add_argument("--scenes", type=int, default=4096)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of Poisson arrivals (200 req/s) in the served leg; 0 = skip")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--only-scene", default="",
                    choices=["", "box_drop", "granular_bed", "mass_ratio_chain", "linkage", "spring_net",
                             "block_pile"],
                    help="run only this one of the single-scene legs (for profiling it alone)")
    ap.add_argument("--no-scenes", action="store_true",
                    help="skip the single-scene legs (1,000-box drop, granular bed)")
    ap.add_argument("--big-scenes", type=int, default=65536,
                    help="scenes in the cache-exceeding batched leg (0 = skip)")
    ap.add_argument("--no-oracle-single", action="store_true",
                    help="skip the single-core oracle timings of the single-scene workloads")
    ap.add_argument("--probe-only", action="store_true",
                    help="run only the 1 GiB HBM copy probe (counter calibration)")
    ap.add_argument("--tile-occupancy-sweep", action="store_true",
                    help="run only the tile kernel on identical 64-body tiles at 1 to 6 tiles per "
                         "SIMD (one JSON line per point), to separate a wave's step latency from "
                         "the SIMDs' issue rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.probe_only:
        import paper_2609_02675_amd as P
        gbs, ms = P.hbm_copy_probe(1 << 30, 10)
        print(json.dumps({"probe": "hbm_copy", "bytes_per_direction": 1 << 30, "GBs": gbs, "ms": ms}))
        return
    if args.tile_occupancy_sweep:
        tile_occupancy_sweep()
        return

    from paper_2609_02675_amd import scenes as S
    scenes = S.batched_chains(args.scenes, seed=2, precision=S.PREC_FP32)
    n_bodies = sum(s.n_bodies for s in scenes)
    iters = scenes[0].iters

    # the CPU leg first (before the GPU is touched): oracle timings and the
    # oracle's reference results for every error the GPU legs report
    plan = _plan(args, S, scenes)
    cpu, refs = cpu_baseline_leg(args, S, scenes, plan)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import errors, scale_of

    import torch
    import paper_2609_02675_amd as P
    if P.device_count() < 1:
        raise SystemExit("no HIP device visible")
    spl, launches, warm_launches = plan["spl"], plan["launches"], plan["warm_launches"]
    total_steps = plan["total_steps"]
    b = P.Batch(len(scenes) + 8, 4 << 30, S.PREC_FP32)
    t = time.perf_counter()
    slots = [b.admit(s, 1 << 30) for s in scenes]
    assert all(x is not None for x in slots)
    log(f"admitted {len(scenes)} scenes ({n_bodies} bodies) in {time.perf_counter() - t:.1f}s")
    if args.tile:
        b.set_tile(args.tile)
    elif not args.no_autotune:
        t = time.perf_counter()
        sch = b.tune()
        log(f"tuner picked {sch} in {time.perf_counter() - t:.1f}s")
    lay = b.layout()

    # timed: `launches` graph replays of spl steps each (one tile-kernel launch
    # runs all spl steps of every tile), an event after every replay
    stream = torch.cuda.Stream()
    sptr = stream.cuda_stream
    for _ in range(warm_launches):
        b.step(stream=sptr, nsteps=spl)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(launches + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(launches):
        b.step(stream=sptr, nsteps=spl)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(launches)])
    step_ms = launch_ms / spl
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps
    body_its = n_bodies * iters * args.steps
    value = body_its / (total_ms / 1e3)
    log(f"batched: {ms_per_step:.4f} ms/step, {value:.4g} body-it/s, {spl} steps per launch "
        f"(host wall {wall:.3f}s)")

    # accuracy of the benchmarked run on sampled scenes vs the FP64 oracle
    acc = 0.0
    for k in plan["batched_sample"]:
        e = errors(b.state(slots[k]), refs["batched"][k], scale_of(scenes[k]))
        acc = max(acc, e["pos"], e["rot"])
    log(f"accuracy vs oracle after {total_steps} steps: {acc:.3e}")

    # dominant kernel: the tile kernel alone (spl steps per launch), timed with
    # HIP events on its stream
    tile_launch_ms = b.time_tile_kernel(max(2, 20 // spl), spl)
    tile_ms = tile_launch_ms / spl
    tbytes = tile_bytes(n_bodies, spl)
    tile_flops = n_bodies * iters * spl * FLOPS_PER_BODY_ITER
    hbm_ach = tbytes / (tile_launch_ms / 1e3)
    alu_ach = tile_flops / (tile_launch_ms / 1e3)
    traffic = tile_traffic(spl, lay["tile_bodies"], f"batched_chains_{len(scenes)}")
    # counter figure beside the flop estimate: wave64 VALU instructions of the
    # profiled launch (SQ_INSTS_VALU) and the flops the estimate gives each of
    # their lane-operations
    valu = tile_valu(spl, lay["tile_bodies"], f"batched_chains_{len(scenes)}")
    common = dict(traffic=traffic, traffic_unit="bytes/launch", valu_insts_per_launch=valu,
                  est_flops_per_valu_lane_op=None if valu is None else tile_flops / (64.0 * valu),
                  kernel="k_tile_step<float>",
                  steps_per_launch=spl, kernel_ms_per_launch=tile_launch_ms, kernel_ms_per_step=tile_ms,
                  flops_per_launch=tile_flops, bytes_per_launch=tbytes)
    if alu_ach / FP32_PEAK >= hbm_ach / HBM_PEAK:
        roof = dict(bound="alu", achieved=alu_ach / 1e12, peak=FP32_PEAK / 1e12, unit="TFLOP/s",
                    frac=alu_ach / FP32_PEAK, frac_of_unpacked_fp32_peak=alu_ach / FP32_UNPACKED_PEAK,
                    flops_per_body_iter_estimate=FLOPS_PER_BODY_ITER,
                    hbm_achieved_GBs=hbm_ach / 1e9, **common)
    else:
        roof = dict(bound="hbm", achieved=hbm_ach / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=hbm_ach / HBM_PEAK, **common)
    log(f"tile kernel {tile_launch_ms:.4f} ms per launch of {spl} steps ({tile_ms:.4f} ms per step); "
        f"roofline {roof['bound']} frac {roof['frac']:.3f}")

    # achievable HBM bandwidth: device-wide streaming copy of 1 GiB
    probe_gbs, _ = P.hbm_copy_probe(1 << 30, 10)
    log(f"hbm copy probe: {probe_gbs:.1f} GB/s")

    # plain path (one kernel launch per iteration, one scene at a time)
    plain = None
    if not args.no_plain:
        sample = scenes[: args.plain_sample]
        objs = [P.Scene(s) for s in sample]
        for o_ in objs:
            o_.step(PLAIN_WARM)
        torch.cuda.synchronize()
        # one scene at a time: each scene's steps run and finish before the next
        # scene's start
        t = time.perf_counter()
        for o_ in objs:
            o_.step(PLAIN_STEPS)
            torch.cuda.synchronize()
        dt = time.perf_counter() - t
        its = sum(s.n_bodies for s in sample) * iters * PLAIN_STEPS
        acc_p = 0.0
        for k in plan["plain_sample"]:
            e = errors(objs[k].state(), refs["plain"][k], scale_of(sample[k]))
            acc_p = max(acc_p, e["pos"], e["rot"])
        plain = dict(value=its / dt, unit="body-iterations/s",
                     ms_per_scene_step=1e3 * dt / (PLAIN_STEPS * len(sample)),
                     sample=f"{len(sample)} of the chains, {PLAIN_STEPS} steps each, one scene at a time "
                            f"(each scene's steps synchronised before the next scene starts)",
                     max_rel_err_vs_fp64_oracle=acc_p,
                     accuracy_checked=f"first {len(plan['plain_sample'])} scenes after "
                                      f"{plan['plain_steps']} steps")
        del objs
        log(f"plain: {plain['value']:.4g} body-it/s, err {acc_p:.2e}")

    # served mix: Poisson arrivals of chains and box piles, continuous batching
    served = served_sat = None
    if args.serve_seconds > 0:
        from paper_2609_02675_amd.serve import Server
        reqs = plan["requests"]
        log(f"{len(reqs)} requests")
        budget = int(args.serve_budget_gib * (1 << 30))
        # the server's own schedule (serve.SERVE_SCHEDULE: eight lanes per
        # contact body), the same for the real-time and the saturated run
        srv = Server(budget, 512, S.PREC_FP32)
        res, st = srv.run(reqs, realtime=True, keep_state=False)
        served = st.summary()
        served.update(requests=len(reqs), rate_hz=200.0, arrivals_s=args.serve_seconds,
                      budget_bytes=budget, mode="Poisson arrivals in real time",
                      schedule=srv.batch.schedule())
        srv.close()
        log("served", served)
        srv = Server(budget, 512, S.PREC_FP32)
        res, st = srv.run(reqs, realtime=False, keep_state=True)
        served_sat = st.summary()
        served_sat.update(requests=len(reqs), budget_bytes=budget,
                          mode="same requests all queued at t=0 (capacity)",
                          schedule=srv.batch.schedule())
        # accuracy of served results against the oracle, on sampled chains
        acc_s = 0.0
        small = plan["served_sample"]
        for k in small:
            e = errors(res[k].state, refs["served"][k], scale_of(reqs[k].scene))
            acc_s = max(acc_s, e["pos"], e["rot"])
        served_sat["max_rel_err_vs_fp64_oracle"] = acc_s
        served_sat["checked"] = [reqs[k].scene.name for k in small]
        srv.close()
        # piles: one served step from the oracle's landing state at step 60
        from paper_2609_02675_amd.scenes import Request
        pk = plan["pile_sample"]
        if pk:
            preq = [Request(arrival_s=0.0, scene=refs["pile_mid"][k].copy(precision=S.PREC_FP32), steps=1)
                    for k in pk]
            srv = Server(budget, 16, S.PREC_FP32)
            pres, _ = srv.run(preq, realtime=False, keep_state=True)
            srv.close()
            acc_pile = 0.0
            for j, k in enumerate(pk):
                e = errors(pres[j].state, refs["pile_next"][k], scale_of(refs["pile_mid"][k]))
                acc_pile = max(acc_pile, e["pos"], e["rot"])
            served_sat["pile_one_step_err_vs_fp64_oracle"] = acc_pile
            served_sat["piles_checked"] = [f"{reqs[k].scene.name} from step 60" for k in pk]
        log("served (saturated)", served_sat)

    # single-scene legs on the plain path: the 1,000-box drop (contact and
    # friction; FP32 and FP64) and the legged robot on a 50,000-sphere bed
    scene_legs = None
    if not args.no_scenes:
        scene_legs = {}

        schedules = {}

        def time_scene(sc, warm, steps, tune_on=None):
            """ms per step over `steps` steps after `warm`, under the schedule the
            tuner picks on the state after the warm-up (or on `tune_on`, a state of
            the same scene with its contacts formed, whose pick the cache then
            hands to the timed scene)."""
            if tune_on is not None and not args.no_autotune:
                gt = P.Scene(tune_on)
                gt.step(1)
                gt.tune(force=True)
                del gt
            g = P.Scene(sc)
            g.step(warm)
            if not args.no_autotune:
                schedules[sc.name] = g.tune()
            torch.cuda.synchronize()
            t = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            return g, sc.n_bodies * sc.iters * steps / dt, 1e3 * dt / steps

        def want(leg):
            return not args.only_scene or args.only_scene == leg

        for prec, tag in ((S.PREC_FP32, "fp32"), (S.PREC_FP64, "fp64")) if want("box_drop") else ():
            sc = S.box_drop(precision=prec)
            # accuracy: one step from the oracle's state after 60 steps (contacts active)
            mid = refs["drop_mid"].copy(precision=prec)
            g, rate, ms = time_scene(sc, 40, 60, tune_on=mid)
            gm = P.Scene(mid)
            gm.step(1)
            e = errors(gm.state(check=False), refs["drop_next"], scale_of(mid))
            scene_legs[f"box_drop_1000_{tag}"] = dict(
                body_its_per_s=rate, ms_per_step=ms, steps_timed="40..100 (falling, then landing)",
                one_step_err_vs_oracle=max(e["pos"], e["rot"]), iters=sc.iters,
                schedule=schedules.get(sc.name))
            log(f"box drop {tag}: {rate:.3g} body-it/s, {ms:.3f} ms/step, 1-step err {max(e['pos'], e['rot']):.2e}")
        if want("granular_bed"):
            bed = S.granular_bed_quadruped(precision=S.PREC_FP32)
            # the bed churns as it sinks (a property of the method as read for 1 cm
            # spheres at h = 1/60), so the timed window is its first steps
            g, rate, ms = time_scene(bed, 1, 5)
            ct = g.contacts()
            scene_legs["granular_bed_quadruped_fp32"] = dict(
                body_its_per_s=rate, ms_per_step=ms, bodies=bed.n_bodies, iters=bed.iters,
                steps_timed="2..6", contacts_after=int(len(ct["i"])), schedule=schedules.get(bed.name))
            log(f"granular bed: {rate:.3g} body-it/s, {ms:.3f} ms/step")
        # the paper's mass-ratio chain, augmented-Lagrangian joints on and off
        for aug, tag in ((True, "al"), (False, "quadratic")) if want("mass_ratio_chain") else ():
            mc = S.mass_ratio_chain(augmented=aug, precision=S.PREC_FP32)
            g, rate, ms = time_scene(mc, 10, 100)
            joint = lambda c, A: max(abs(np.linalg.norm(A[mc.bond_i[e]] @ mc.x_i[e] + c[mc.bond_i[e]]
                                                     - A[mc.bond_j[e]] @ mc.x_j[e] - c[mc.bond_j[e]])
                                         - mc.rest_len[e]) for e in range(mc.n_bonds))
            st = g.state(check=False)
            scene_legs[f"mass_ratio_chain_19_{tag}_fp32"] = dict(
                body_its_per_s=rate, ms_per_step=ms, iters=mc.iters, steps_timed="11..110",
                max_joint_error_m=float(joint(st[0], st[1])),
                max_joint_error_oracle_m=float(joint(*refs["mass_ratio"][aug][:2])),
                # the oracle itself from FP32-rounded inputs: how far rounding the
                # inputs alone moves this chain after 110 steps
                max_joint_error_oracle_fp32_inputs_m=float(joint(*refs["mass_ratio_f32_inputs"][aug][:2])),
                oracle_state_spread_from_fp32_inputs=float(
                    max(np.abs(refs["mass_ratio_f32_inputs"][aug][0] - refs["mass_ratio"][aug][0]).max(),
                        np.abs(refs["mass_ratio_f32_inputs"][aug][1] - refs["mass_ratio"][aug][1]).max())),
                paper_context="Table 2, mass-ratio chain (19 bodies, 10 iterations) on an RTX 3080: "
                              "t_solve 1.28 ms (AL on) / 1.25 ms (off) per frame")
            log(f"mass-ratio chain {tag}: {ms:.3f} ms/step, joint error {joint(st[0], st[1]):.3g} m")
        # the paper's four-body linkage (three hinges and a slider), crank driven
        if want("linkage"):
            lk = S.linkage("slider", drive_amp_deg=60.0, precision=S.PREC_FP32)
            g, rate, ms = time_scene(lk, 10, 110)
            e = errors(g.state(check=False), refs["linkage"], scale_of(lk))
            scene_legs["linkage_slider_crank_fp32"] = dict(
                body_its_per_s=rate, ms_per_step=ms, bodies=lk.n_bodies, bonds=lk.n_bonds, iters=lk.iters,
                steps_timed="11..120", err_vs_fp64_oracle_after_120_steps=max(e["pos"], e["rot"]),
                paper_context="Table 2, linkage (a) (4 bodies, 4 joints, 20 iterations) on an RTX 3080: "
                              "t_solve 2.37 ms per frame")
            log(f"linkage: {ms:.4f} ms/step, err {max(e['pos'], e['rot']):.2e}")
        # the paper's 11 x 11 net of 220 springs, quadratic and quartic bonds:
        # convergence of the first step (relative error per iteration) and step time
        for p_ in (2, 4) if want("spring_net") else ():
            net = S.spring_net(order=p_, iters=20, precision=S.PREC_FP32)
            if p_ == 2:
                net = net.copy(bond_type=np.full(net.n_bonds, S.BOND_POLYNOMIAL, np.int32))
            gn = P.Scene(net)
            gn.set_debug(2)
            gn.step(1)
            rho = gn.residuals()
            gn.set_debug(0)
            _, rate, ms = time_scene(net, 10, 100)
            scene_legs[f"spring_net_11_p{p_}_fp32"] = dict(
                body_its_per_s=rate, ms_per_step=ms, bonds=net.n_bonds, iters=net.iters,
                first_step_residual_rho_k=[float(x) for x in rho[:20]])
            log(f"net p={p_}: {ms:.3f} ms/step, first-step rho {rho[0]:.2e} -> {rho[19]:.2e}")
        # 50^3 stacked cubes in resting contact (the paper's largest scene size)
        if want("block_pile"):
            pile = S.block_pile(precision=S.PREC_FP32)
            g, rate, ms = time_scene(pile, 1, 10)
            ct = g.contacts()
            scene_legs["block_pile_125k_fp32"] = dict(
                body_its_per_s=rate, ms_per_step=ms, bodies=pile.n_bodies, iters=pile.iters,
                steps_timed="2..11", contacts_after=int(len(ct["i"])), schedule=schedules.get(pile.name),
                paper_context="Table 2, 50^3 block pile on an RTX 3080: 72.56 ms collision + 87.55 ms "
                              "solve per frame at 20 iterations (2.9e7 body-iterations/s for the solve)")
            del g
            log(f"block pile: {rate:.3g} body-it/s, {ms:.3f} ms/step, {len(ct['i'])} contacts")

    # the batched chains at 16x the count: a working set beyond the last-level cache
    big = None
    if args.big_scenes > 0:
        del b
        big = big_batch_leg(P, S, torch, plan, refs)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "body-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched_chains_{len(scenes)}", "scenes": len(scenes),
                   "bodies": n_bodies, "iters": iters, "dt": scenes[0].h,
                   "tile_bodies": lay["tile_bodies"], "tiles": lay["tiles"],
                   "steps_per_launch": spl,
                   "mode": f"batched, one graph replay (one tile-kernel launch) per {spl} steps"},
        # per step: each replay's event-timed duration divided by its steps
        "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "p50_launch_ms": float(np.percentile(launch_ms, 50)),
        "accuracy": {"max_rel_err_vs_fp64_oracle": acc, "after_steps": total_steps,
                     "tolerance": 1e-3},
        "hbm_copy_probe_GBs": probe_gbs,
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "served": served,
        "served_saturated": served_sat,
        "roofline": roof,
        "single_scene": scene_legs,
        "batched_beyond_cache": big,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
