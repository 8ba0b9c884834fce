#!/usr/bin/env python3
"""Benchmark: syndrome rounds/s and measurements/s of a rotated surface-code memory workload on
one MI355X, batched (all shots in one launch sequence) and plain (one shot at a time).

A step is one pass of the whole hot path over the workload: reset every shot to |0...0>, then
every gate layer, noise channel and measurement layer of the circuit for all shots, and the
measurement record copied to the host.  The value is whole-job throughput: shots * rounds / time.

Usage: python bench.py [--workload surface_d25|surface_d71|surface_d3] [--steps K] [--warmup W]
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

DEFAULTS = {  # steps, warmup, shots timed in the plain form
    "surface_d3": (20, 2, 200),
    "surface_d25": (10, 1, 10),
    "surface_d71": (3, 1, 2),
}


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("stab_kernels.hip", "stab_api.hip", "stab_device.h"):
        h.update(open(os.path.join(ROOT, "paper_2507_03092_amd", "csrc", f), "rb").read())
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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="surface_d25", choices=sorted(DEFAULTS))
    ap.add_argument("--mode", default="shared", choices=["shared", "full"])
    ap.add_argument("--plain-shots", type=int, default=None)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (--gpus 1); multi-GPU sharding is "
              "described in DESIGN.md but not implemented", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2507_03092_amd import circuits as Cc
    from paper_2507_03092_amd import stab

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    steps0, warm0, plain0 = DEFAULTS[args.workload]
    steps = args.steps if args.steps is not None else steps0
    warmup = args.warmup if args.warmup is not None else warm0
    plain_shots = args.plain_shots if args.plain_shots is not None else plain0

    w = Cc.WORKLOADS[args.workload]
    circ, lay, seed, shots = Cc.workload(args.workload)
    d, rounds = w["d"], w["rounds"]
    nmeas = circ.num_measurements()
    n = circ.n

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # ---------------- batched: all shots, one launch sequence ----------------
    log(f"{args.workload}: n={n} rounds={rounds} shots={shots} mode={args.mode}")
    ctx = stab.Context(n, shots, mode=args.mode, seed=seed)
    prog = ctx.compile(circ)
    for _ in range(warmup):
        ctx.reset(seed)
        ctx.execute(prog)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.reset(seed)
        rec = ctx.execute(prog)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimes = ctx.kernel_times()
    ctx.set_timing(False)
    ms_step = (t1 - t0) * 1000.0 / steps
    rounds_s = shots * rounds / ((t1 - t0) / steps)
    meas_s = shots * nmeas / ((t1 - t0) / steps)
    log(f"batched: {ms_step:.3f} ms/step, {rounds_s:.1f} rounds/s, {meas_s:.3e} meas/s")

    # ---------------- roofline of the dominant kernel ----------------
    per_step = {k: (v[0] / steps, v[1] / steps) for k, v in ktimes.items()}
    dom = max(per_step, key=lambda k: per_step[k][0])
    roofline = None
    launches = ktimes["segment"][1]
    if launches:
        # surface-code stream: one segment per round (gates change x|z) plus the noise-only
        # segment before the final data readout; K = d*d-1 ancillas, then d*d data qubits
        nseg_wb = rounds
        tot = nseg_wb * seg_bytes_per_launch(n, shots, args.mode, d * d - 1, True) + \
            seg_bytes_per_launch(n, shots, args.mode, d * d, False)
        tot_steps = tot * steps
        seg_ms = ktimes["segment"][0]
        achieved = tot_steps / (seg_ms / 1000.0) / 1e9
        traffic = None
        pmc = os.path.join(ROOT, "profiles", f"segment_{args.workload}_pmc.json")
        if os.path.exists(pmc):
            p = json.load(open(pmc))
            if p.get("source_digest") == kernel_source_digest() and p.get("mode") == args.mode:
                traffic = p.get("bytes_per_launch")
        roofline = {"kernel": "segment", "bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "bytes_per_launch": int(tot / (nseg_wb + 1)),
                    "avg_launch_us": round(seg_ms * 1000.0 / launches, 2),
                    "dominant_kernel": dom}

    # ---------------- plain: one shot at a time ----------------
    plain = None
    if not args.no_plain and plain_shots > 0:
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
        log(f"plain: {plain}")
        ctx1.close()

    # ---------------- CPU baseline: the oracle on a bounded sample ----------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        if args.workload == "surface_d71":
            sc, _ = Cc.surface_code_memory(d, 2, w["p"], w["idle"])
            sshots, srounds, desc = 1, 2, "1 shot of the d=71 circuit truncated to its first 2 rounds"
        elif args.workload == "surface_d25":
            sc, sshots, srounds, desc = circ, shots, rounds, "the whole d=25 workload (100 shots x 25 rounds)"
        else:
            sc, sshots, srounds, desc = circ, shots, rounds, "the whole d=3 workload (1000 shots x 3 rounds)"
        c0 = time.perf_counter()
        orec = O.run(sc, sshots, seed)
        c1 = time.perf_counter()
        bit_exact = None
        if sc is circ:
            bit_exact = bool(np.array_equal(orec, rec[:sshots]))
        cpu = {"value": round(sshots * srounds / (c1 - c0), 3), "unit": "rounds/s",
               "cores": O.threads(), "kind": "oracle", "sample": desc,
               "seconds": round(c1 - c0, 2), "bit_exact_vs_gpu": bit_exact}
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": METRIC, "value": round(rounds_s, 2), "unit": "rounds/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "code": "rotated surface code, Z memory", "d": d,
                   "qubits": n, "rounds": rounds, "shots": shots, "p_depolarizing": w["p"],
                   "idle_pauli": list(w["idle"]) if w["idle"] else None, "seed": seed,
                   "form": f"batched-{args.mode}"},
        "measurements_per_s": round(meas_s, 1),
        "plain": plain,
        "kernel_ms_per_step": {k: round(v[0], 4) for k, v in per_step.items() if v[1] > 0},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
