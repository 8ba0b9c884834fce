#!/usr/bin/env python3
"""Benchmark: syndrome rounds/s and measurements/s of a rotated surface-code memory workload on
one MI355X, batched (all shots in one launch sequence) and plain (one shot at a time).

A step is one pass of the whole hot path over the workload: reset every shot to |0...0>, then
every gate layer, noise channel and measurement layer of the circuit for all shots, and the
measurement record copied to the host.  The value is whole-job throughput: shots * rounds / time.

With --workload random_batch it times the uneven multi-circuit batch instead: 4096
independent random layered Clifford circuits of n ~ U{64..2048} qubits run by one launch; a
step resets and runs every circuit once, and the value is measurements/s over the batch.

Usage: python bench.py [--workload surface_d25|surface_d71|surface_d3|random_batch]
                       [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure
METRIC = "syndrome rounds/sec & measurements/sec at d=25/71, batched vs plain, bit-exact"

DEFAULTS = {  # steps, warmup, shots (circuits) timed in the plain form
    "surface_d3": (20, 2, 200),
    "surface_d25": (50, 2, 10),
    "surface_d71": (10, 1, 2),
    "random_batch": (3, 1, 64),
    "commute": (20, 2, 0),
    "surface_d25_t1t2": (3, 1, 0),
    "serve": (1, 0, 0),
}
COMMUTE_METRIC = "Pauli-string pairs/sec, group-wise and qubit-wise commutation matrices, bit-exact"
# int32 VALU operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (the fp32 vector
# figure of 157.3 TFLOP/s counts a fused multiply-add as two and packs two fp32 per lane)
VALU_INT32_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
BATCH_METRIC = "measurements/sec of an uneven multi-circuit batch (random Clifford circuits), bit-exact"


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2507_03092_amd", "csrc")
    for f in sorted(os.listdir(src)):
        h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()[:16]


def seg_bytes_per_launch(n: int, shots: int, mode: str, K: int, write_back: bool) -> int:
    """Algorithmic HBM bytes of one segment-kernel launch: every 64-row band of every tableau
    copy read once (and written once when a gate changes x|z), plus the x and z column words
    extracted for the K targets of the next measurement layer."""
    wc = (n + 63) // 64
    rs, nb = 2 * wc, 2 * wc
    copies = 1 if mode == "shared" else shots
    band = 64 * rs * 8
    return copies * nb * (band * (2 if write_back else 1) + 2 * K * 8)


def load_pmc(workload: str, mode: str, tile=None) -> dict:
    """HBM bytes per launch of each kernel from the committed rocprofv3 counter summary of this
    workload (FETCH_SIZE and WRITE_SIZE, scaled by what they read for a plain copy of known
    size), if it was taken from the current kernel sources (and, for the batch, the same launch
    configuration); else {}."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.json")
    if not os.path.exists(path):
        return {}
    p = json.load(open(path))
    if p.get("source_digest") != kernel_source_digest() or p.get("mode") != mode:
        return {}
    if tile is not None and p.get("tile") != tile:
        return {}
    fs, ws = p["fetch_scale"], p["write_scale"]
    return {k: (v["fetch_kib"] * fs + v["write_kib"] * ws) * 1024.0 for k, v in p["kernels"].items()}


def cpu_host() -> dict:
    """Host CPU model and the cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable}


def surface_alg_bytes(n, d, rounds, shots, mode, work, per_step) -> dict:
    """Algorithmic bytes per step of each surface-code kernel: the per-unit figures of the
    kernels (one band, one target, one rowsum row) times the work counters of a step."""
    wc = (n + 63) // 64
    row_b, nb = 2 * wc * 8, 2 * wc
    return {
        # one segment per round (gates change x|z) plus the noise-only segment before the final
        # data readout; K = d*d-1 ancillas, then d*d data qubits
        "segment": rounds * seg_bytes_per_launch(n, shots, mode, d * d - 1, True)
        + seg_bytes_per_launch(n, shots, mode, d * d, False),
        # per random measurement: the stabilizer half of its column, the pivot row read, logged
        # and replaced; per stabilizer rowsum row a read and a write
        "chain": work[4] * (wc * 8 + 3 * row_b) + work[5] * 2 * row_b,
        # per walked destabilizer a read and a write, per applied pivot its logged row read
        "replay": work[9] * 2 * row_b + work[8] * row_b,
        # the final tableau read and the columns of every target written (about d*d targets)
        "extract": per_step.get("extract", (0, 0))[1] * seg_bytes_per_launch(n, shots, mode, d * d, False),
        # layer start: every target's column read, and every stabilizer row multiplied by a
        # deterministic reduction (both passes; the second pass reduces few)
        "classify": (work[2] + work[4] + work[6]) * nb * 8 + work[3] * row_b,
        # after the chain: the columns of the targets it left deterministic
        "det": work[6] * nb * 8,
    }


ROOF_KERNELS = ("segment", "classify", "chain")


def run_surface(workload: str, mode: str, steps: int, warmup: int, graph: bool, plain_shots: int, log) -> dict:
    """Time `steps` steps of a surface-code workload in one storage mode.  Returns the step
    times, the record, the per-kernel breakdown, the work counters and rooflines of the dominant
    kernel and of the segment, classify and chain kernels."""
    import numpy as np
    import torch

    from paper_2507_03092_amd import circuits as Cc
    from paper_2507_03092_amd import stab

    w = Cc.WORKLOADS[workload]
    circ, lay, seed, shots = Cc.workload(workload)
    d, rounds = w["d"], w["rounds"]
    nmeas = circ.num_measurements()
    n = circ.n
    log(f"{workload}: n={n} rounds={rounds} shots={shots} mode={mode}")
    ctx = stab.Context(n, shots, mode=mode, seed=seed)
    prog = ctx.compile(circ)
    for _ in range(warmup):
        ctx.reset(seed)
        ctx.execute(prog)
    # per-kernel breakdown from one untimed step with every launch bracketed by events; the
    # timed eager steps then bracket only the kernels whose rooflines are reported (each
    # event pair costs a few microseconds of the step)
    ctx.set_timing(True)
    ctx.reset(seed)
    ctx.execute(prog)
    full = ctx.kernel_times()
    breakdown = {k: v[0] for k, v in full.items() if v[1] > 0}
    dom = max(breakdown, key=breakdown.get)
    timed = sorted(set(ROOF_KERNELS) | {dom})
    ctx.set_timing(True, kernels=timed)
    cnt0 = ctx.counters().astype(np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.reset(seed)
        rec = ctx.execute(prog)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimes = ctx.kernel_times()
    ctx.set_timing(False)
    work = (ctx.counters().astype(np.int64) - cnt0) / steps     # per step
    eager_ms_step = (t1 - t0) * 1000.0 / steps
    if graph:
        # the same steps replayed as one captured graph each, no events: the throughput (the
        # capture happens in an untimed step first)
        ctx.set_graph(True)
        ctx.reset(seed)
        ctx.execute(prog)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.reset(seed)
            grec = ctx.execute(prog)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.set_graph(False)
        if not np.array_equal(grec, rec):
            raise AssertionError("graph replay record differs from the eager record")
    ms_step = (t1 - t0) * 1000.0 / steps
    rounds_s = shots * rounds / ((t1 - t0) / steps)
    meas_s = shots * nmeas / ((t1 - t0) / steps)
    log(f"{workload} batched-{mode}: {ms_step:.3f} ms/step, {rounds_s:.1f} rounds/s, {meas_s:.3e} meas/s")

    per_step = {k: (v[0] / steps, v[1] / steps) for k, v in ktimes.items()}
    alg = surface_alg_bytes(n, d, rounds, shots, mode, work, per_step)
    pmc = load_pmc(workload, mode)

    def roof(kernel):
        ms, launches = per_step[kernel]
        if not launches or kernel not in alg:
            return None
        per_launch = alg[kernel] / launches
        achieved = per_launch / (ms / launches / 1000.0) / 1e9
        t = pmc.get(kernel)
        return {"kernel": kernel, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": int(t) if t is not None else None, "bytes_per_launch": int(per_launch),
                "avg_launch_us": round(ms * 1000.0 / launches, 2), "launches_per_step": launches,
                "share_of_step": round(ms / eager_ms_step, 3)}

    rooflines = {k: roof(k) for k in timed if k in alg}
    roofline = dict(rooflines[dom]) if rooflines.get(dom) else None
    if roofline is not None:
        roofline["timed_in"] = "eager steps (the same count, right before the graph-replayed ones)"

    plain = None
    if plain_shots > 0:
        ctx1 = stab.Context(n, 1, mode="shared", seed=seed)
        prog1 = ctx1.compile(circ)
        ctx1.reset(seed, first_shot=0)
        ctx1.execute(prog1)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        ok = True
        for b in range(plain_shots):
            ctx1.reset(seed, first_shot=b)
            r1 = ctx1.execute(prog1)
            ok &= bool(np.array_equal(r1[0], rec[b]))
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        plain = {"rounds_per_s": round(plain_shots * rounds / (p1 - p0), 2),
                 "meas_per_s": round(plain_shots * nmeas / (p1 - p0), 1),
                 "ms_per_shot": round((p1 - p0) * 1000.0 / plain_shots, 3),
                 "shots_timed": plain_shots, "matches_batched": ok}
        log(f"{workload} plain: {plain}")
        ctx1.close()
    ctx.close()
    return {
        "workload": workload, "mode": mode, "circ": circ, "seed": seed, "shots": shots, "d": d,
        "rounds": rounds, "n": n, "nmeas": nmeas, "w": w, "rec": rec, "steps": steps,
        "ms_step": ms_step, "eager_ms_step": eager_ms_step, "rounds_s": rounds_s, "meas_s": meas_s,
        "breakdown": breakdown, "roofline": roofline, "rooflines": rooflines, "work": work, "plain": plain,
        "graph": graph,
    }


def surface_cpu_baseline(r: dict, log) -> dict:
    """The oracle on the host, bit-exact against the GPU record: all cores (one thread per
    shot) and one core.  d=71 runs the first two rounds of the workload's op stream (an exact
    prefix, so its records are a prefix of the GPU's); the smaller workloads run whole."""
    import numpy as np

    from oracle import oracle as O
    from paper_2507_03092_amd import circuits as Cc

    circ, seed, shots, rec = r["circ"], r["seed"], r["shots"], r["rec"]
    if r["workload"] == "surface_d71":
        ins, tg = circ.arrays()
        k = int(np.nonzero(ins["kind"] == Cc.MR)[0][1]) + 1            # through syndrome round 2's MR
        sc = Cc.PackedCircuit(circ.n, ins[:k].copy(), tg[:int(ins["ntargets"][:k].sum())].copy())
        srounds, one_shots = 2, 1
        desc = "the first 2 rounds of the d=71 op stream (round 1 holds the random X-ancilla measurements)"
    else:
        sc, srounds = circ, r["rounds"]
        one_shots = min(shots, 4)
        desc = f"the whole {r['workload']} workload"
    nrec = sc.num_measurements()
    c0 = time.perf_counter()
    orec = O.run(sc, shots, seed)
    c1 = time.perf_counter()
    ok_all = bool(np.array_equal(orec, rec[:, :nrec]))
    o0 = time.perf_counter()
    ok_one = True
    for s in range(one_shots):
        o = O.run(sc, 1, seed, first_shot=s)        # one shot: one thread
        ok_one &= bool(np.array_equal(o[0], rec[s, :nrec]))
    o1 = time.perf_counter()
    cpu = {"value": round(shots * srounds / (c1 - c0), 4), "unit": "rounds/s",
           "cores": min(O.threads(), shots), "kind": "oracle",
           "sample": f"{desc}; all {shots} shots, one host thread per shot", "seconds": round(c1 - c0, 2),
           "bit_exact_vs_gpu": ok_all and ok_one,
           "one_core": {"value": round(one_shots * srounds / (o1 - o0), 4), "unit": "rounds/s", "cores": 1,
                        "sample": f"{one_shots} shot(s) of the same, one after another",
                        "seconds": round(o1 - o0, 2)}}
    cpu.update(cpu_host())
    log(f"{r['workload']} cpu baseline: {cpu}")
    return cpu


def surface_summary(r: dict) -> dict:
    """The fields of a timed surface-code run that go into the JSON line."""
    work = r["work"]
    return {
        "ms_per_step": round(r["ms_step"], 4), "eager_ms_per_step": round(r["eager_ms_step"], 4),
        "rounds_per_s": round(r["rounds_s"], 2), "measurements_per_s": round(r["meas_s"], 1),
        "launch": "captured graph" if r["graph"] else "eager",
        "kernel_ms_per_step": {k: round(v, 4) for k, v in r["breakdown"].items()},
        "roofline": r["roofline"],
        "rooflines": r["rooflines"],
        "work_per_step": {"random_measurements": int(work[4]), "rowsum_rows": int(work[5]),
                          "replay_rowsum_rows": int(work[8]), "replay_walked_rows": int(work[9]),
                          "replay_rows_by_testing": int(work[10]), "replay_events_by_testing": int(work[11]),
                          "deterministic_measurements": int(work[2] + work[6]),
                          "multiplied_rows": int(work[3]), "chain_rounds": int(work[0]),
                          "noise_events": int(work[7])},
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="surface_d71", choices=sorted(DEFAULTS))
    ap.add_argument("--mode", default="shared", choices=["shared", "full"])
    ap.add_argument("--plain-shots", type=int, default=None)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-companions", action="store_true",
                    help="surface_d71: skip the batched-full form and the d=25 workload that the "
                         "default line carries beside the headline")
    ap.add_argument("--no-graph", action="store_true",
                    help="surface workloads: launch every kernel eagerly in the timed steps")
    ap.add_argument("--tile", default="auto",
                    help="random_batch launch configuration: 'auto' (autotuner, first two measurement "
                         "instructions of every circuit) or a configuration number")
    ap.add_argument("--tune-quota", type=int, default=6, help="measurement instructions the autotuner times")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrival window of the serving workload")
    ap.add_argument("--serve-rate", type=float, default=None, help="arrival rate of the serving workload (1/s)")
    ap.add_argument("--serve-arena-gb", type=float, default=200.0, help="device arena of the server (GB)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates HBM byte "
                         "counters of a profiler against a known size) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: only one GPU is supported (--gpus 1); sharding across GPUs is a design, "
              "not implemented here", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nbytes}))
        return 0
    if args.workload == "random_batch":
        return bench_batch(args)
    if args.workload == "commute":
        return bench_commute(args)
    if args.workload == "surface_d25_t1t2":
        return bench_exact_noise(args)
    if args.workload == "serve":
        return bench_serve(args)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def knobs(workload):
        steps0, warm0, plain0 = DEFAULTS[workload]
        steps = args.steps if args.steps is not None else steps0
        warmup = args.warmup if args.warmup is not None else warm0
        plain = 0 if args.no_plain else (args.plain_shots if args.plain_shots is not None else plain0)
        return steps, warmup, plain

    steps, warmup, plain_shots = knobs(args.workload)
    head = run_surface(args.workload, args.mode, steps, warmup, not args.no_graph, plain_shots, log)
    w = head["w"]
    line = {
        "metric": METRIC, "value": round(head["rounds_s"], 2), "unit": "rounds/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(head["ms_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "code": "rotated surface code, Z memory", "d": head["d"],
                   "qubits": head["n"], "rounds": head["rounds"], "shots": head["shots"], "p_depolarizing": w["p"],
                   "idle_pauli": list(w["idle"]) if w["idle"] else None, "seed": head["seed"],
                   "form": f"batched-{args.mode}", "launch": "eager" if args.no_graph else "captured graph"},
    }
    summ = surface_summary(head)
    for k in ("eager_ms_per_step", "measurements_per_s", "kernel_ms_per_step", "roofline", "rooflines",
              "work_per_step"):
        line[k] = summ[k]
    line["plain"] = head["plain"]
    companions = args.workload == "surface_d71" and args.mode == "shared" and not args.no_companions
    if companions:
        # the same workload with one tableau per shot (records must equal the shared form's)
        full = run_surface("surface_d71", "full", steps, warmup, not args.no_graph, 0, log)
        fs = surface_summary(full)
        fs["matches_shared"] = bool(np.array_equal(full["rec"], head["rec"]))
        if not fs["matches_shared"]:
            raise AssertionError("batched-full record differs from batched-shared")
        line["full"] = fs
        del full
        # d=25, shared, with its plain form and its own CPU baseline
        s25, w25, p25 = knobs("surface_d25")
        r25 = run_surface("surface_d25", "shared", s25, w25, not args.no_graph, p25, log)
        line["d25"] = {"config": {"workload": "surface_d25", "d": 25, "qubits": r25["n"], "rounds": r25["rounds"],
                                  "shots": r25["shots"], "seed": r25["seed"], "form": "batched-shared",
                                  "steps": s25},
                       **surface_summary(r25), "plain": r25["plain"]}
        if not args.no_cpu_baseline:
            line["d25"]["cpu_baseline"] = surface_cpu_baseline(r25, log)
    line["cpu_baseline"] = None if args.no_cpu_baseline else surface_cpu_baseline(head, log)
    print(json.dumps(line))
    return 0


def bench_batch(args) -> int:
    """The uneven multi-circuit batch: one persistent launch runs every circuit."""
    import numpy as np
    import torch

    from paper_2507_03092_amd import circuits as Cc
    from paper_2507_03092_amd import stab

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    steps0, warm0, plain0 = DEFAULTS["random_batch"]
    steps = args.steps if args.steps is not None else steps0
    warmup = args.warmup if args.warmup is not None else warm0
    plain_n = args.plain_shots if args.plain_shots is not None else plain0
    w = Cc.RANDOM_BATCH
    g0 = time.perf_counter()
    ns, circs = Cc.random_batch(w["ncirc"], w["n_lo"], w["n_hi"], w["layers"], w["seed"], w["meas_every"],
                                w["meas_frac"])
    nmeas = int(sum(c.num_measurements() for c in circs))
    log(f"random_batch: {len(circs)} circuits, n {ns.min()}..{ns.max()}, {nmeas} measurements, "
        f"generated in {time.perf_counter() - g0:.1f} s")
    seed = w["seed"]
    b = stab.Batch(ns, seed=seed)
    prog = b.compile(circs)
    tune_s = None
    if args.tile == "auto":
        a0 = time.perf_counter()
        b.autotune(prog, meas_quota=args.tune_quota, force=True)
        tune_s = time.perf_counter() - a0
        log(f"autotuner: tile {prog.tile:#x} in {tune_s:.2f} s")
    else:
        prog.tile = int(args.tile, 0)
    for _ in range(warmup):
        b.reset(seed)
        b.execute(prog)
    torch.cuda.synchronize()
    c_before = b.counters().astype(np.int64)
    kms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        b.reset(seed)
        rec, ms = b.execute(prog, timed=True)
        kms += ms
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c_after = b.counters().astype(np.int64)
    ms_step = (t1 - t0) * 1000.0 / steps
    meas_s = nmeas / ((t1 - t0) / steps)
    log(f"batched: {ms_step:.2f} ms/step, {meas_s:.4e} meas/s, kernel {kms / steps:.2f} ms")
    dc = (c_after - c_before) / steps
    bytes_launch = float(dc[6] + dc[7])
    k_avg_ms = kms / steps
    achieved = bytes_launch / (k_avg_ms / 1000.0) / 1e9
    traffic = load_pmc("random_batch", "batch", prog.tile).get("batch")
    roofline = {"kernel": "batch", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": int(traffic) if traffic is not None else None,
                "bytes_per_launch": int(bytes_launch), "avg_launch_us": round(k_avg_ms * 1000.0, 1),
                "random_measurements": int(dc[4]), "deterministic_measurements": int(dc[2]),
                "rowsum_rows": int(dc[5])}
    b.close()

    # plain: a sample of circuits, one launch each
    plain = None
    if not args.no_plain and plain_n > 0:
        rng = np.random.default_rng(1)
        pick = [int(c) for c in rng.choice(len(circs), size=min(plain_n, len(circs)), replace=False)]
        batches = []
        for c in pick:
            bc = stab.Batch(ns[c:c + 1], seed=seed)
            batches.append((bc, bc.compile([circs[c]]), c))
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for bc, pc, c in batches:
            bc.execute(pc)
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        pm = sum(circs[c].num_measurements() for c in pick)
        plain = {"meas_per_s": round(pm / (p1 - p0), 1), "circuits_timed": len(pick),
                 "ms_per_circuit": round((p1 - p0) * 1000.0 / len(pick), 3)}
        for bc, _, _ in batches:
            bc.close()
        log(f"plain: {plain}")

    cpu = None
    if not args.no_cpu_baseline:
        from concurrent.futures import ThreadPoolExecutor

        from oracle import oracle as O

        rng = np.random.default_rng(2)
        small = np.nonzero(ns <= 512)[0]
        pick = [int(c) for c in rng.choice(small, size=min(160, len(small)), replace=False)]
        cores = O.threads()
        c0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            outs = list(ex.map(lambda c: O.run(circs[c], 1, seed, c), pick))
        c1 = time.perf_counter()
        ok = all(np.array_equal(o[0], rec[c]) for o, c in zip(outs, pick))
        pm = sum(circs[c].num_measurements() for c in pick)
        cpu = {"value": round(pm / (c1 - c0), 1), "unit": "meas/s", "cores": cores, "kind": "oracle",
               "sample": f"{len(pick)} circuits of the batch drawn at random among those with n <= 512 "
                         f"(cheaper per measurement than the batch average), one circuit per host thread",
               "seconds": round(c1 - c0, 2), "bit_exact_vs_gpu": bool(ok)}
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": BATCH_METRIC, "value": round(meas_s, 1), "unit": "meas/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "random_batch", "circuits": int(w["ncirc"]), "n_range": [w["n_lo"], w["n_hi"]],
                   "layers": w["layers"], "measure_every": w["meas_every"], "measure_fraction": w["meas_frac"],
                   "measurements": nmeas, "seed": seed, "form": "batched (one launch)",
                   "tile": prog.tile, "tuned": tune_s is not None,
                   "tune_seconds": None if tune_s is None else round(tune_s, 2)},
        "circuits_per_s": round(len(circs) / ((t1 - t0) / steps), 2),
        "plain": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


def bench_serve(args) -> int:
    """Continuous batching: Poisson arrivals of surface-code memory requests (d ~ U{3,...,31},
    d rounds, p = 1e-3, shots ~ U{1..100}) served by one server on a 200 GB arena; latency from
    arrival to records.  A fixed sample of the served requests is checked afterwards against the
    same request run alone (stab_sample), and its small ones against the oracle."""
    import numpy as np
    import torch

    from paper_2507_03092_amd import circuits as Cc
    from paper_2507_03092_amd import stab

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    w = dict(Cc.SERVING)
    rate = args.serve_rate if args.serve_rate is not None else w["rate"]
    times, ds, shots, seeds = Cc.serving_requests(rate, args.serve_seconds, w["seed"], w["d_lo"], w["d_hi"],
                                                  w["shots_hi"])
    m = len(times)
    circs = {int(d): Cc.surface_code_memory(int(d), int(d), w["p"])[0] for d in np.unique(ds)}
    arena = (int(args.serve_arena_gb * 1e9) // 256) * 256
    srv = stab.Server(arena)
    prog = {d: srv.program(c) for d, c in circs.items()}
    # the requests whose records are kept and checked: every 25th, and every 5th one with d >= 25
    keep = {j for j in range(m) if j % 25 == 0 or (ds[j] >= 25 and j % 5 == 0)}
    log(f"serve: {m} requests over {args.serve_seconds} s at {rate}/s, arena {arena / 1e9:.0f} GB")
    torch.cuda.synchronize()
    arrival, lat, kept = {}, [], {}
    done_work = 0
    i = 0
    steps = 0
    busy_sum = 0
    t0 = time.perf_counter()
    drain_limit = args.serve_seconds + 120.0
    last_log = 0.0
    while True:
        now = time.perf_counter() - t0
        while i < m and times[i] <= now:
            d = int(ds[i])
            rid = srv.submit(prog[d], int(shots[i]), int(seeds[i]))
            arrival[rid] = (times[i], i)
            i += 1
        st = srv.stats()
        if st["queued"] == 0 and st["resident_requests"] == 0:
            if i == m:
                break
            time.sleep(max(0.0, min(times[i] - now, 0.001)))
            continue
        if now > drain_limit:
            break
        nf = srv.step()
        steps += 1
        busy_sum += st["resident_shots"]
        tdone = time.perf_counter() - t0
        for rid in srv.poll():
            ta, j = arrival.pop(rid)
            lat.append(tdone - ta)
            done_work += int(shots[j]) * int(ds[j])
            rec = srv.result(rid, int(shots[j]))
            if j in keep:
                kept[j] = rec
        if now - last_log > 10.0:
            last_log = now
            log(f"t={now:.0f} s: {len(lat)} served, {st['in_flight']} in flight, {st['queued']} queued")
        if nf == 0 and (i == m or times[i] > tdone + 0.0002):
            time.sleep(0.0001)
    wall = time.perf_counter() - t0
    unfinished = len(arrival) + (m - i)
    lat_ms = np.array(lat) * 1000.0
    p50 = float(np.percentile(lat_ms, 50)) if len(lat) else None
    p99 = float(np.percentile(lat_ms, 99)) if len(lat) else None
    st = srv.stats()
    log(f"served {len(lat)} of {m} in {wall:.1f} s, p50 {p50} ms, p99 {p99} ms, {steps} steps, "
        f"{st['steps']} batch launches")
    srv.close()
    # parity of the kept sample: the same request alone, and the oracle for the small ones
    bad = [j for j, rec in kept.items()
           if not np.array_equal(rec, stab.sample(circs[int(ds[j])], int(shots[j]), int(seeds[j]))[0])]
    small = sorted(j for j in kept if ds[j] <= 7)[:24]
    from oracle import oracle as O

    bad_oracle = [j for j in small
                  if not np.array_equal(kept[j], O.run(circs[int(ds[j])], int(shots[j]), int(seeds[j])))]
    parity = {"checked_alone": len(kept), "checked_alone_d_ge_25": int(sum(1 for j in kept if ds[j] >= 25)),
              "equal_alone": len(kept) - len(bad), "checked_oracle": len(small),
              "equal_oracle": len(small) - len(bad_oracle)}
    log(f"parity of served requests: {parity}")
    cpu = None
    if not args.no_cpu_baseline:
        from concurrent.futures import ThreadPoolExecutor

        pick = np.random.default_rng(3).choice(m, size=min(16, m), replace=False)
        c0 = time.perf_counter()
        with ThreadPoolExecutor(4) as ex:
            list(ex.map(lambda j: O.run(circs[int(ds[j])], int(shots[j]), int(seeds[j])), pick))
        c1 = time.perf_counter()
        work = int(sum(int(shots[j]) * int(ds[j]) for j in pick))
        cpu = {"value": round(work / (c1 - c0), 1), "unit": "shot-rounds/s", "cores": O.threads(), "kind": "oracle",
               "sample": f"{len(pick)} requests drawn from the stream (4 at a time, each over its shots)",
               "seconds": round(c1 - c0, 2)}
        log(f"cpu baseline: {cpu}")
    line = {
        "metric": "continuous-batching sampling service: shot-rounds/sec served, p50/p99 request latency",
        "value": round(done_work / wall, 1), "unit": "shot-rounds/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(wall * 1000.0 / max(steps, 1), 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serve", "rate_per_s": rate, "seconds": args.serve_seconds, "requests": m,
                   "d_range": [w["d_lo"], w["d_hi"]], "shots_max": w["shots_hi"], "p": w["p"], "seed": w["seed"],
                   "arena_bytes": arena, "lanes": "auto (every request Pauli-noise: shared lane)"},
        "latency_ms": {"p50": p50, "p99": p99, "max": float(lat_ms.max()) if len(lat) else None},
        "served": len(lat), "unfinished": unfinished, "wall_s": round(wall, 2),
        "batch_launches": st["steps"], "mean_resident_shots": round(busy_sum / max(steps, 1), 1),
        "parity": parity,
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0 if not bad and not bad_oracle else 1


def bench_exact_noise(args) -> int:
    """The d=25 memory experiment with the exact (composite, not twirled) T1/T2 idle channel:
    resets make every shot's tableau its own, so the shots run as a batch of circuits."""
    import numpy as np
    import torch

    from paper_2507_03092_amd import circuits as Cc
    from paper_2507_03092_amd import stab

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    steps0, warm0, _ = DEFAULTS[args.workload]
    steps = args.steps if args.steps is not None else steps0
    warmup = args.warmup if args.warmup is not None else warm0
    w = Cc.WORKLOADS[args.workload]
    circ, lay, seed, shots = Cc.workload(args.workload)
    rounds, nmeas = w["rounds"], circ.num_measurements()
    b = stab.Batch(np.full(shots, circ.n, dtype=np.int32), seed=seed)
    prog = b.compile([circ] * shots)
    if args.tile == "auto":
        a0 = time.perf_counter()
        b.autotune(prog, meas_quota=args.tune_quota, force=True)
        log(f"autotuner: tile {prog.tile:#x} in {time.perf_counter() - a0:.2f} s")
    else:
        prog.tile = int(args.tile, 0)
    for _ in range(warmup):
        b.reset(seed)
        b.execute(prog)
    c_before = b.counters().astype(np.int64)
    torch.cuda.synchronize()
    kms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        b.reset(seed)
        rec, ms = b.execute(prog, timed=True)
        kms += ms
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dc = (b.counters().astype(np.int64) - c_before) / steps
    ms_step = (t1 - t0) * 1000.0 / steps
    k_ms = kms / steps
    bytes_launch = float(dc[6] + dc[7])
    achieved = bytes_launch / (k_ms / 1000.0) / 1e9
    log(f"{args.workload}: {ms_step:.2f} ms/step, {shots * rounds / (ms_step / 1000.0):.1f} rounds/s")
    traffic = load_pmc(args.workload, "batch", prog.tile).get("batch")
    roofline = {"kernel": "batch", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": int(traffic) if traffic is not None else None,
                "bytes_per_launch": int(bytes_launch), "avg_launch_us": round(k_ms * 1000.0, 1),
                "random_measurements": int(dc[4]), "deterministic_measurements": int(dc[2])}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        ss = shots
        c0 = time.perf_counter()
        orec = O.run(circ, ss, seed)
        c1 = time.perf_counter()
        ok = all(np.array_equal(orec[s], rec[s]) for s in range(ss))
        cpu = {"value": round(ss * rounds / (c1 - c0), 3), "unit": "rounds/s", "cores": O.threads(),
               "kind": "oracle", "sample": f"the whole workload ({ss} shots)", "seconds": round(c1 - c0, 2),
               "bit_exact_vs_gpu": bool(ok)}
        log(f"cpu baseline: {cpu}")
    b.close()
    line = {
        "metric": "syndrome rounds/sec with the exact T1/T2 idle channel (stochastic reset + Z), bit-exact",
        "value": round(shots * rounds / (ms_step / 1000.0), 2), "unit": "rounds/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "d": w["d"], "qubits": circ.n, "rounds": rounds, "shots": shots,
                   "p_depolarizing": w["p"], "idle_exact": list(w["idle_exact"]), "seed": seed,
                   "form": "batch of per-shot tableaux (one launch)", "tile": prog.tile,
                   "tuned": args.tile == "auto"},
        "measurements_per_s": round(shots * nmeas / (ms_step / 1000.0), 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


def bench_commute(args) -> int:
    """Pairwise commutation of 32768 Pauli strings on 256 qubits against themselves."""
    import numpy as np
    import torch

    from paper_2507_03092_amd import circuits as Cc
    from paper_2507_03092_amd import stab

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    steps0, warm0, _ = DEFAULTS["commute"]
    steps = args.steps if args.steps is not None else steps0
    warmup = args.warmup if args.warmup is not None else warm0
    w = Cc.COMMUTE
    m, n = w["m"], w["n"]
    x, z = Cc.random_paulis(m, n, w["seed"])
    P = torch.from_numpy(stab.pack_paulis(x, z).view(np.int64)).cuda()
    nbw = (m + 63) // 64
    gc = torch.empty((m, nbw), dtype=torch.int64, device="cuda")
    qw = torch.empty_like(gc)
    L = stab.lib()
    stream = torch.cuda.current_stream()
    import ctypes as C

    def launch():
        stab._check(L.stab_commute(C.c_void_p(P.data_ptr()), m, C.c_void_p(P.data_ptr()), m, n,
                                   C.c_void_p(gc.data_ptr()), C.c_void_p(qw.data_ptr()),
                                   C.c_void_p(stream.cuda_stream)))

    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        launch()
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms = e0.elapsed_time(e1) / steps
    ms_step = (t1 - t0) * 1000.0 / steps
    pairs = float(m) * m
    W = (n + 63) // 64
    ops = pairs * W * 10          # per pair and 64-bit word: 2 AND, 3 XOR/OR on 32-bit halves x 2
    achieved = ops / (k_ms / 1000.0) / 1e12
    log(f"commute: {ms_step:.3f} ms/step, kernel {k_ms:.3f} ms, {pairs / (ms_step / 1000.0):.4e} pairs/s")
    roofline = {"kernel": "commute", "bound": "alu", "achieved": round(achieved, 2),
                "peak": round(VALU_INT32_PEAK_TOPS, 2), "unit": "Tops/s (int32 VALU)",
                "frac": round(achieved / VALU_INT32_PEAK_TOPS, 4), "traffic": None,
                "ops_per_launch": int(ops), "avg_launch_us": round(k_ms * 1000.0, 2)}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import commute as OC

        rows = np.random.default_rng(0).choice(m, size=256, replace=False)
        c0 = time.perf_counter()
        wg, wq = OC.commute_matrix(x[rows], z[rows], x, z)
        c1 = time.perf_counter()
        g = gc.cpu().numpy().view(np.uint64)[rows]
        bits = np.unpackbits(g.view(np.uint8).reshape(len(rows), nbw * 8), axis=1, bitorder="little")[:, :m]
        cpu = {"value": round(len(rows) * m / (c1 - c0), 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": "256 random strings against all 32768 (numpy integer matrix products)",
               "seconds": round(c1 - c0, 2), "bit_exact_vs_gpu": bool(np.array_equal(bits, wg))}
        log(f"cpu baseline: {cpu}")
    line = {
        "metric": COMMUTE_METRIC, "value": round(pairs / (ms_step / 1000.0), 1), "unit": "pairs/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "commute", "strings": m, "qubits": n, "seed": w["seed"],
                   "identity_probability": 0.25},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
