"""Sanitizer builds of host code.

* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc) runs every
  instruction kind, both measurement branches, noise and T1T2 without a report, and gives the
  same records and tableaux as the ordinary build.
* The library's host code built with the same sanitizers (hipcc, host compilation only; the
  device code is built as usual) runs the host-only ABI calls of abi_host_checks.py, in a child
  process that preloads the sanitizer runtime, without a report."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_03092_amd import circuits as Cc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("san") / "oracle_san")
    flags = ["-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-Wall", "-Wextra"]
    subprocess.check_call(["gcc", *flags, "-o", out, os.path.join(ORACLE, "chp_oracle.c"),
                           os.path.join(ORACLE, "sanitize_driver.c")])
    return out


def _run(driver, tmp_path, circ, shots, seed, first_shot=0):
    instr, tg = circ.arrays()
    nrec = circ.num_measurements()
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(inp, "wb") as f:
        np.array([circ.n, shots, first_shot, seed, len(instr), len(tg), nrec], dtype=np.int64).tofile(f)
        np.ascontiguousarray(instr).tofile(f)
        np.ascontiguousarray(tg, dtype=np.int32).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, inp, outp], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    raw = np.fromfile(outp, dtype=np.uint8)
    n = circ.n
    rec = raw[: shots * nrec].reshape(shots, nrec)
    sq = shots * 2 * n * n
    o = shots * nrec
    tx = raw[o: o + sq].reshape(shots, 2 * n, n)
    tz = raw[o + sq: o + 2 * sq].reshape(shots, 2 * n, n)
    tr = raw[o + 2 * sq:].reshape(shots, 2 * n)
    return rec, tx, tz, tr


def _cases():
    yield Cc.random_clifford_measure(7, depth=12, seed=3, p_meas=0.3, noise=0.05)
    yield Cc.random_clifford_measure(130, depth=8, seed=4, p_meas=0.25, noise=0.02)
    c = Cc.random_layered_clifford(65, layers=30, seed=5, meas_every=5, meas_frac=0.3)
    c.append(Cc.M, list(range(65)))
    yield c
    yield Cc.surface_code_memory(3, 3, 0.01)[0]
    t = Cc.Circuit(n=6)
    t.gate(Cc.H, [0, 2, 4])
    t.gate(Cc.CX, [0, 1, 2, 3, 4, 5])
    t.append(Cc.T1T2, [0, 2, 4], (int(0.35 * 2 ** 64), int(0.7 * 2 ** 64), 0))
    t.append(Cc.R, [1])
    t.append(Cc.MR, [3, 5])
    t.append(Cc.M, list(range(6)))
    yield t


@pytest.mark.parametrize("k", range(5))
def test_oracle_under_asan_ubsan_matches_plain_build(driver, tmp_path, k):
    circ = list(_cases())[k]
    shots, seed = 3, 40 + k
    rec, tx, tz, tr = _run(driver, tmp_path, circ, shots, seed)
    want, (wx, wz, wr) = O.run(circ, shots, seed, want_tableau=True)
    assert np.array_equal(rec, want)
    assert np.array_equal(tx, wx) and np.array_equal(tz, wz) and np.array_equal(tr, wr)


def test_sanitized_driver_rejects_malformed_stream(driver, tmp_path):
    c = Cc.Circuit(n=4)
    c.append(Cc.M, [0, 1])
    instr, tg = c.arrays()
    tg = tg.copy()
    tg[1] = 9                                   # out of range: the oracle refuses the stream
    inp, outp = str(tmp_path / "bad.bin"), str(tmp_path / "bad_out.bin")
    with open(inp, "wb") as f:
        np.array([4, 1, 0, 1, len(instr), len(tg), 2], dtype=np.int64).tofile(f)
        np.ascontiguousarray(instr).tofile(f)
        tg.astype(np.int32).tofile(f)
    r = subprocess.run([driver, inp, outp], capture_output=True, text=True, timeout=60)
    assert r.returncode == 3 and "Sanitizer" not in r.stderr and "runtime error" not in r.stderr


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _asan_runtime():
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_library_host_code_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no sanitizer runtime next to hipcc")
    so = str(tmp_path / "libstab_san.so")
    pkg = os.path.join(ROOT, "paper_2507_03092_amd")
    # host-side sanitizers only: each -fsanitize option is scoped to the host compilation
    host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host, "-shared-libsan",
           "-I", os.path.join(ROOT, "include"), "-o", so, os.path.join(pkg, "csrc", "stab_api.hip")]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "abi_host_checks.py"), so],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "abi host checks ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
