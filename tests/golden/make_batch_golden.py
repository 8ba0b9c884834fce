"""Write record digests for the largest circuits of the 4096-circuit random batch, computed by
the CPU oracle only.

Usage: python tests/golden/make_batch_golden.py
Writes tests/golden/random_batch_large_oracle.json: for the largest circuit of the batch and
five others drawn (numpy seed 1) from those with n >= 1500, the circuit index, n, the sha256 of
its packed record (LSB-first bits) and its number of ones.  Circuit c runs alone in the oracle
with RNG key (batch seed, c), which is its key inside the batch.  No value here comes from the
GPU.
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2507_03092_amd import circuits as Cc  # noqa: E402


def pick(ns: np.ndarray) -> list:
    """The largest circuit, then five drawn from those with n >= 1500."""
    big = np.nonzero(ns >= 1500)[0]
    top = int(np.argmax(ns))
    rng = np.random.default_rng(1)
    rest = [int(c) for c in rng.choice(big[big != top], size=5, replace=False)]
    return [top] + sorted(rest)


def main():
    w = Cc.RANDOM_BATCH
    ns, circs = Cc.random_batch(w["ncirc"], w["n_lo"], w["n_hi"], w["layers"], w["seed"], w["meas_every"],
                                w["meas_frac"])
    idx = pick(ns)
    t0 = time.time()
    with ThreadPoolExecutor(len(idx)) as ex:
        futs = {c: ex.submit(O.run, circs[c], 1, w["seed"], c) for c in idx}
        recs = {c: f.result()[0] for c, f in futs.items()}
    out = {
        "workload": "random_batch", "seed": w["seed"], "ncirc": w["ncirc"],
        "circuits": [{"index": c, "n": int(ns[c]), "measurements": int(circs[c].num_measurements()),
                      "sha256": hashlib.sha256(np.packbits(recs[c], bitorder="little").tobytes()).hexdigest(),
                      "ones": int(recs[c].sum())} for c in idx],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "random_batch_large_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
