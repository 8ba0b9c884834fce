"""Write per-shot record digests of a surface-code workload, computed by the CPU oracle only.

Usage: python tests/golden/make_surface_golden.py surface_d71
Writes tests/golden/<workload>_oracle.json: sha256 of each shot's packed record (LSB-first
bits), its number of ones, and the workload parameters.  No value here comes from the GPU.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2507_03092_amd import circuits as Cc  # noqa: E402


def main(name: str):
    circ, lay, seed, shots = Cc.workload(name)
    t0 = time.time()
    rec = O.run(circ, shots, seed)
    dt = time.time() - t0
    out = {
        "workload": name, "seed": seed, "shots": shots, "n": circ.n,
        "measurements": circ.num_measurements(),
        "sha256": [hashlib.sha256(np.packbits(r, bitorder="little").tobytes()).hexdigest() for r in rec],
        "ones": [int(r.sum()) for r in rec],
        "oracle_seconds": round(dt, 1), "oracle_threads": O.threads(),
    }
    det, obs = Cc.surface_detectors(lay, Cc.WORKLOADS[name]["rounds"], rec)
    out["detector_rate"] = float(det.mean())
    out["observable_flips"] = [int(v) for v in obs]
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "sha256"}))


if __name__ == "__main__":
    main(sys.argv[1])
