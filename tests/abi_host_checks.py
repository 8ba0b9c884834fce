"""Host-only calls of the C ABI, run in a child process by test_sanitizers_cpu.py against a
build of the library whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer.
Every call returns before the library makes a HIP call (sizes, stream validation and
compilation planning, argument errors).  Usage: python abi_host_checks.py <libstab.so>"""
from __future__ import annotations

import ctypes as C
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2507_03092_amd import circuits as Cc  # noqa: E402
from paper_2507_03092_amd import stab  # noqa: E402


def main(path: str) -> int:
    stab.LIB_PATH = path
    L = stab.lib()
    out = C.c_uint64(0)
    for n, shots, mode in ((1, 1, 0), (1249, 100, 0), (10081, 10, 1), (10240, 2, 0)):
        assert L.stab_tableau_bytes(n, shots, mode, C.byref(out)) == 0 and out.value > 0
    assert L.stab_tableau_bytes(0, 1, 0, C.byref(out)) == stab.EINVAL
    assert L.stab_tableau_bytes(stab.max_qubits() + 1, 1, 0, C.byref(out)) == stab.ERANGE
    assert L.stab_tableau_bytes(5, 1, 0, None) == stab.EINVAL
    # stream validation and planning over every kind of stream
    circs = [Cc.surface_code_memory(d, d, 1e-3)[0] for d in (3, 5, 11)]
    circs.append(Cc.workload("surface_d71", rounds=2)[0])
    circs += [Cc.random_clifford_measure(n, depth=10, seed=n, p_meas=0.3, noise=0.05) for n in (1, 64, 65, 300)]
    for c in circs:
        p = stab.plan_describe(c, shots=7)
        assert p["records"] == c.num_measurements()
    base = Cc.Circuit(n=5)
    base.gate(Cc.H, [0])
    base.gate(Cc.CX, [0, 1])
    base.append(Cc.M, [0, 1, 0])
    for bad in ("kind", "range", "neg", "odd", "cx_same", "short", "long"):
        instr, tg = base.arrays()
        instr, tg = instr.copy(), tg.copy()
        if bad == "kind":
            instr["kind"][0] = 99
        elif bad == "range":
            tg[0] = 5
        elif bad == "neg":
            tg[0] = -1
        elif bad == "odd":
            instr["ntargets"][1] = 1
            tg = np.concatenate([tg[:2], tg[3:]])
        elif bad == "cx_same":
            tg[2] = tg[1]
        elif bad == "short":
            tg = tg[:2]
        elif bad == "long":
            tg = np.concatenate([tg, np.array([1], dtype=np.int32)])
        o = np.zeros(8, dtype=np.int64)
        rc = L.stab_plan_describe(5, 1, 0, instr.ctypes.data_as(C.c_void_p), len(instr),
                                  tg.ctypes.data_as(C.c_void_p), len(tg), o.ctypes.data_as(C.c_void_p), 8)
        assert rc == stab.EINVAL and L.stab_last_error(), bad
    t = Cc.Circuit(n=3)
    t.t1t2(1e-6, 100e-6, 100e-6, [0, 1])
    try:
        stab.plan_describe(t)
        raise AssertionError("T1T2 accepted by a single context")
    except stab.StabError as e:
        assert e.code == stab.EINVAL
    # batches: sizes and argument errors
    ns = np.array([1, 64, 65, 2048, 8192], dtype=np.int32)
    assert stab.batch_bytes(ns) > 0
    bad_n = np.array([5, 8193], dtype=np.int32)
    assert L.stab_batch_bytes(2, bad_n.ctypes.data_as(C.c_void_p), C.byref(out)) == stab.ERANGE
    h = C.c_void_p(None)
    p = ns.ctypes.data_as(C.c_void_p)
    assert L.stab_batch_create(5, p, 0, None, 1 << 20, None, C.byref(h)) == stab.EINVAL
    assert L.stab_batch_create(5, p, 0, C.c_void_p(0x100000), 16, None, C.byref(h)) == stab.ENOMEM
    assert L.stab_batch_execute(None, None, None, None) == stab.EINVAL
    assert L.stab_batch_program_records(None, 0) == -1
    L.stab_batch_destroy(None)
    L.stab_batch_program_destroy(None)
    L.stab_destroy(None)
    L.stab_program_destroy(None)
    L.stab_server_destroy(None)
    print("abi host checks ok", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
