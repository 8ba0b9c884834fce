"""Determinism of the HIP path: the same seed gives the same records across repeated runs, and
running every kernel with its workgroups taken in reverse order (STAB_REVERSE_BLOCKS=1, in a
child process) changes neither the records nor the exported tableaux.  A result that depended on
the order in which workgroups run (a race) would show here; the oracle checks of the other GPU
tests fix what the results must be."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2507_03092_amd import circuits as Cc

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases():
    """(name, circuit, shots, seed, mode): noisy surface codes in both storage modes and random
    Clifford circuits with M/MR/R layers whose measurements are mostly random and dense."""
    return [
        ("surface_d5", Cc.surface_code_memory(5, 5, 1e-2)[0], 64, 3, "shared"),
        ("surface_d7_full", Cc.surface_code_memory(7, 4, 1e-2)[0], 6, 4, "full"),
        ("surface_d11", Cc.surface_code_memory(11, 6, 5e-3, idle=(1e-3, 1e-3, 1e-3))[0], 33, 5, "shared"),
        ("random_130", Cc.random_clifford_measure(130, 30, seed=21, noise=1e-2), 40, 6, "shared"),
        ("random_300_full", Cc.random_clifford_measure(300, 12, seed=22, p_meas=0.5), 3, 7, "full"),
    ]


def run_all(stab) -> dict:
    """Records and a tableau export of every case, and the records of an uneven batch."""
    out = {}
    for name, circ, shots, seed, mode in _cases():
        ctx = stab.Context(circ.n, shots, mode=mode, seed=seed)
        out[name] = ctx.run(circ)
        x, z, r = ctx.get_tableau(shots - 1)
        out[name + "_tab"] = np.concatenate([x.ravel(), z.ravel(), r.ravel()])
        ctx.close()
    ns = [17, 130, 64, 257, 9]
    circs = [Cc.random_clifford_measure(n, 20, seed=100 + i, noise=1e-2) for i, n in enumerate(ns)]
    b = stab.Batch(ns, seed=9)
    recs = b.execute(b.compile(circs))
    for i, rec in enumerate(recs):
        out[f"batch_{i}"] = rec
    b.close()
    return out


@pytest.fixture(scope="module")
def stab():
    import torch

    assert torch.cuda.is_available(), "no GPU"
    from paper_2507_03092_amd import stab as S

    S.lib()
    return S


def test_same_seed_same_records_ten_runs(stab):
    for name, circ, shots, seed, mode in _cases()[:4]:
        say(f"case {name}: 10 executions from |0...0>")
        ctx = stab.Context(circ.n, shots, mode=mode, seed=seed)
        prog = ctx.compile(circ)
        first = ctx.execute(prog)
        for rep in range(9):
            ctx.reset(seed)
            assert np.array_equal(ctx.execute(prog), first), f"{name}: execution {rep + 2} differs"
        ctx.close()


def test_reversed_workgroup_order_same_results(stab, tmp_path):
    say("cases in this process (workgroups in dispatch order)")
    here = run_all(stab)
    path = tmp_path / "reversed.npz"
    script = ("import sys; sys.path.insert(0, %r); import numpy as np; "
              "from paper_2507_03092_amd import stab; from tests.test_gpu_determinism import run_all; "
              "np.savez(%r, **run_all(stab))" % (ROOT, str(path)))
    env = dict(os.environ, STAB_REVERSE_BLOCKS="1")
    say("the same cases in a child process with STAB_REVERSE_BLOCKS=1")
    res = subprocess.run([sys.executable, "-c", script], env=env, cwd=ROOT, capture_output=True, text=True,
                         timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    there = np.load(path)
    assert sorted(there.files) == sorted(here)
    for k, v in here.items():
        assert np.array_equal(there[k], v), f"{k} differs with reversed workgroup order"
