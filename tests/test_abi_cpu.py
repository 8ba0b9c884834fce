"""The C-ABI library loads and exports what include/stab.h declares; host-only argument checks.

No GPU is touched: every call here returns before the library makes a HIP call.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2507_03092_amd import build as hipbuild
from paper_2507_03092_amd import circuits as Cc
from paper_2507_03092_amd import stab

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    hipbuild.build(force=False)
    return stab.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "stab.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stab_[a-z_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert declared_functions() == sorted(stab.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_instruction_record_is_32_bytes():
    assert Cc.INSTR_DTYPE.itemsize == 32
    # kinds match the header's enum
    src = open(os.path.join(ROOT, "include", "stab.h")).read()
    for name, code in Cc.NAME_TO_KIND.items():
        m = re.search(r"STAB_%s = (\d+)" % name, src)
        assert m and int(m.group(1)) == code, name


def test_max_qubits(L):
    # 2 * ceil(n/64) band words of a target column over one wave (5 per lane)
    assert stab.max_qubits() == 160 * 64


def _bytes(n, shots, mode):
    wc = (n + 63) // 64
    nr = 64 * wc
    s = 1 if mode == 0 else shots
    a = lambda v: (v + 255) & ~255
    tab = s * 2 * nr * 2 * wc * 8
    rs = a(tab) + s * 2 * wc * 8
    rd = a(rs) + shots * 2 * wc * 8
    return a(rd)


@pytest.mark.parametrize("n,shots,mode", [(1, 1, 0), (17, 1000, 0), (1249, 100, 0), (1249, 100, 1),
                                          (10081, 10, 0), (10240, 2, 0), (64, 3, 1), (65, 3, 1)])
def test_tableau_bytes(L, n, shots, mode):
    assert stab.tableau_bytes(n, shots, mode) == _bytes(n, shots, mode)


def test_argument_errors_without_gpu(L):
    out = C.c_uint64(0)
    assert L.stab_tableau_bytes(0, 1, 0, C.byref(out)) == stab.EINVAL
    assert L.stab_tableau_bytes(5, 0, 0, C.byref(out)) == stab.EINVAL
    assert L.stab_tableau_bytes(5, 1, 7, C.byref(out)) == stab.EINVAL
    assert L.stab_tableau_bytes(stab.max_qubits() + 1, 1, 0, C.byref(out)) == stab.ERANGE
    assert L.stab_tableau_bytes(5, 70000, 0, C.byref(out)) == stab.ERANGE
    assert L.stab_tableau_bytes(5, 1, 0, None) == stab.EINVAL
    h = C.c_void_p(None)
    assert L.stab_create(5, 1, 0, 0, 0, None, 1 << 20, None, C.byref(h)) == stab.EINVAL
    assert L.stab_create(5, 1, 0, 0, 0, C.c_void_p(0x1001), 1 << 20, None, C.byref(h)) == stab.EINVAL
    assert L.stab_create(5, 1, 0, 0, 0, C.c_void_p(0x100000), 16, None, C.byref(h)) == stab.ENOMEM
    assert b"stab_tableau_bytes" in L.stab_last_error()
    assert L.stab_create(5, 1, 0, 0, 0, None, 0, None, None) == stab.EINVAL
    # NULL handles are rejected or ignored
    assert L.stab_run(None, None, 0, None, 0, None) == stab.EINVAL
    assert L.stab_reset(None, 0, 0) == stab.EINVAL
    assert L.stab_get_tableau(None, 0, None, None, None) == stab.EINVAL
    L.stab_destroy(None)
    L.stab_program_destroy(None)
    assert L.stab_program_records(None) == -1


def test_sample_noalloc_host_checks(L):
    """stab_sample_noalloc checks its arguments and its scratch need before touching a device."""
    circ = Cc.Circuit(4)
    circ.append(Cc.H, [0])
    circ.append(Cc.CX, [0, 1])
    circ.append(Cc.M, [0, 1, 2, 3])
    instr, tg = circ.arrays()
    out = np.zeros(16, dtype=np.uint8)
    big = C.c_void_p(0x100000)

    def call(c, shots, buf, nbytes, instr=instr, tg=tg):
        return L.stab_sample_noalloc(stab._ptr(instr), len(instr), stab._ptr(tg), len(tg), c.n, shots, 0, 1,
                                     buf, nbytes, None, stab._ptr(out))

    assert call(circ, 1, None, 1 << 20) == stab.EINVAL
    assert call(circ, 1, C.c_void_p(0x1001), 1 << 20) == stab.EINVAL
    assert call(circ, 1, big, 16) == stab.ENOMEM
    bt = tg.copy()
    bt[-1] = 4
    assert call(circ, 1, big, 1 << 20, instr, bt) == stab.EINVAL
    assert b"out of range" in L.stab_last_error()
    # one Z measurement of all 10240 qubits needs two 26 MB target-column arrays and a 26 MB
    # pivot log: more than the static scratch holds
    wide = Cc.Circuit(stab.max_qubits())
    wide.append(Cc.M, range(wide.n))
    wi, wt = wide.arrays()
    assert stab.NOALLOC_SCRATCH_BYTES == 64 << 20
    assert call(wide, 1, big, 1 << 40, wi, wt) == stab.ERANGE
    msg = L.stab_last_error().decode()
    assert "stab_sample_noalloc" in msg and str(stab.NOALLOC_SCRATCH_BYTES) in msg


def test_record_unpacking_layout():
    # shot b's bits start at byte b*ceil(nrec/8), LSB first
    rec = np.array([[1, 0, 1, 1, 0, 0, 0, 0, 1], [0, 1, 0, 0, 0, 0, 0, 1, 1]], dtype=np.uint8)
    packed = np.packbits(rec, axis=1, bitorder="little").reshape(-1)
    assert list(packed) == [0b00001101, 1, 0b10000010, 1]
    assert np.array_equal(stab.unpack_record(packed, 2, 9), rec)


# ---------------------------------------------------------------- host-side stream compilation ---
def _c(n):
    return Cc.Circuit(n=n)


def test_plan_splits_layers_and_segments(L):
    c = _c(4)
    c.gate(Cc.H, [0, 1])
    c.gate(Cc.S, [2])            # disjoint: same layer as the H's
    c.gate(Cc.H, [0])            # repeats qubit 0: new layer ...
    c.gate(Cc.CX, [1, 2, 2, 3])  # ... which CX(1,2) joins; CX(2,3) repeats 2: new layer
    c.dep1(0.1, [0, 0])          # noise closes the layer; repeated targets allowed
    c.gate(Cc.X, [1])
    c.append(Cc.M, [0, 1, 0])    # repeat splits the measurement into two layers
    c.append(Cc.R, [2])
    c.append(Cc.MR, [3])
    p = stab.plan_describe(c)
    # layers: [H0 H1 S2] [H0 CX12] [CX23] [X1]
    assert p["gate_layers"] == 4 and p["gates"] == 7
    assert p["noise_instructions"] == 1 and p["noise_units"] == 2
    assert p["measurement_layers"] == 4 and p["records"] == 4 and p["max_layer"] == 2
    assert p["segments"] == 5      # one before each measurement layer + the trailing one


def test_plan_surface_code_counts(L):
    for d, rounds in ((3, 3), (25, 25)):
        circ, lay = Cc.surface_code_memory(d, rounds, 1e-3)
        p = stab.plan_describe(circ, shots=100)
        assert p["measurement_layers"] == rounds + 1
        assert p["gate_layers"] == 6 * rounds
        assert p["gates"] == rounds * (4 * d * (d - 1) + 2 * (d * d - 1) // 2)
        assert p["records"] == circ.num_measurements() == rounds * (d * d - 1) + d * d
        assert p["max_layer"] == d * d


@pytest.mark.parametrize("bad", ["kind", "range", "neg", "odd", "cx_same", "short", "long"])
def test_plan_rejects_malformed_streams(L, bad):
    c = _c(5)
    c.gate(Cc.H, [0])
    c.gate(Cc.CX, [0, 1])
    instr, tg = c.arrays()
    if bad == "kind":
        instr["kind"][0] = 99
    elif bad == "range":
        tg[0] = 5
    elif bad == "neg":
        tg[0] = -1
    elif bad == "odd":
        instr["ntargets"][1] = 1
        tg = tg[:2]
    elif bad == "cx_same":
        tg[2] = tg[1]
    elif bad == "short":
        tg = tg[:2]
    elif bad == "long":
        tg = np.concatenate([tg, np.array([1], dtype=np.int32)])
    out = np.zeros(8, dtype=np.int64)
    rc = L.stab_plan_describe(5, 1, 0, instr.ctypes.data_as(C.c_void_p), len(instr),
                              tg.ctypes.data_as(C.c_void_p), len(tg), out.ctypes.data_as(C.c_void_p), 8)
    assert rc == stab.EINVAL
    assert L.stab_last_error()


# ------------------------------------------------------------------ multi-circuit batches ---
def _batch_bytes(ns):
    a = lambda v: (v + 255) & ~255
    tot = 0
    for n in ns:
        wc = (n + 63) // 64
        tot += a(2 * 64 * wc * 2 * wc * 8)
    for n in ns:
        tot += a(2 * ((n + 63) // 64) * 8)
    return tot


@pytest.mark.parametrize("ns", [[1], [64, 65, 2048], [1, 8192], list(range(1, 300, 7))])
def test_batch_bytes(L, ns):
    assert stab.batch_bytes(ns) == _batch_bytes(ns)


def test_batch_argument_errors_without_gpu(L):
    out = C.c_uint64(0)
    n = np.array([5, 0], dtype=np.int32)
    assert L.stab_batch_bytes(2, n.ctypes.data_as(C.c_void_p), C.byref(out)) == stab.EINVAL
    n = np.array([5, 8193], dtype=np.int32)
    assert L.stab_batch_bytes(2, n.ctypes.data_as(C.c_void_p), C.byref(out)) == stab.ERANGE
    assert L.stab_batch_bytes(0, n.ctypes.data_as(C.c_void_p), C.byref(out)) == stab.EINVAL
    assert L.stab_batch_bytes(1, None, C.byref(out)) == stab.EINVAL
    h = C.c_void_p(None)
    n = np.array([5, 7], dtype=np.int32)
    p = n.ctypes.data_as(C.c_void_p)
    assert L.stab_batch_create(2, p, 0, None, 1 << 20, None, C.byref(h)) == stab.EINVAL
    assert L.stab_batch_create(2, p, 0, C.c_void_p(0x1001), 1 << 20, None, C.byref(h)) == stab.EINVAL
    assert L.stab_batch_create(2, p, 0, C.c_void_p(0x100000), 16, None, C.byref(h)) == stab.ENOMEM
    assert L.stab_batch_create(2, p, 0, C.c_void_p(0x100000), 1 << 20, None, None) == stab.EINVAL
    assert L.stab_batch_reset(None, 0) == stab.EINVAL
    assert L.stab_batch_execute(None, None, None, None) == stab.EINVAL
    assert L.stab_batch_get_tableau(None, 0, None, None, None) == stab.EINVAL
    assert L.stab_batch_program_records(None, 0) == -1
    t = C.c_int32(-7)
    assert L.stab_batch_autotune(None, None, 0, 0, C.byref(t)) == stab.EINVAL and t.value == -7
    assert L.stab_batch_program_set_tile(None, 0) == stab.EINVAL
    assert L.stab_batch_program_tile(None) == -1
    L.stab_batch_destroy(None)
    L.stab_batch_program_destroy(None)


def test_random_batch_generator_shapes():
    ns, circs = Cc.random_batch(6, 64, 300, layers=20, seed=4)
    assert len(circs) == 6 and all(64 <= n <= 300 for n in ns)
    for n, c in zip(ns, circs):
        instr, tg = c.arrays()
        assert c.n == n and int(instr["ntargets"].sum()) == len(tg)
        assert c.num_measurements() == 2 * max(1, round(0.1 * n))
        # every gate layer (H, S, CX between measurements) touches each qubit at most once
        off = 0
        seen = set()
        for k, nt in zip(instr["kind"], instr["ntargets"]):
            t = tg[off:off + nt]
            off += nt
            if k == Cc.M:
                assert len(set(t.tolist())) == nt
                continue
            if k == Cc.H:
                seen = set()
            assert not (seen & set(t.tolist()))
            seen |= set(t.tolist())
    # deterministic in the seed
    ns2, circs2 = Cc.random_batch(6, 64, 300, layers=20, seed=4)
    assert np.array_equal(ns, ns2) and all(np.array_equal(a.targets, b.targets) for a, b in zip(circs, circs2))


def test_single_context_rejects_t1t2(L):
    c = Cc.Circuit(n=3)
    c.t1t2(1e-6, 100e-6, 100e-6, [0, 1])
    with pytest.raises(stab.StabError) as e:
        stab.plan_describe(c)
    assert e.value.code == stab.EINVAL and "batch" in str(e.value)


def test_server_argument_errors_without_gpu(L):
    """Server calls that fail before any HIP call: NULL handles and arguments."""
    null = C.c_void_p(None)
    out = C.c_void_p(None)
    assert L.stab_server_create(null, 1 << 20, null, C.byref(out)) == stab.EINVAL
    assert L.stab_server_create(C.c_void_p(4096 + 8), 1 << 20, null, C.byref(out)) == stab.EINVAL  # misaligned
    assert L.stab_server_set_lane(null, 0, stab.LANE_SHARED) == stab.EINVAL
    assert L.stab_set_rng(null, 1, 0) == stab.EINVAL
    assert L.stab_server_cancel(null, 1) == stab.EINVAL
    assert L.stab_server_step(null, None) == stab.EINVAL
    assert L.stab_server_poll(null, None, 0) == stab.EINVAL
    assert L.stab_server_records(null, 1) == -1
    assert L.stab_server_program_records(null, 0) == -1
    v = np.zeros(9, dtype=np.int64)
    assert L.stab_server_stats(null, v.ctypes.data_as(C.c_void_p), 9) == stab.EINVAL
    L.stab_server_destroy(null)                 # a no-op
