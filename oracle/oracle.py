"""Python access to the plain CPU oracle (chp_oracle.c).  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this.
The HIP product path never loads it.  The oracle follows the CHP formalism as the paper
restates it (Sec. 2.3-2.4, Table 1, rowsum of Appendix A.2); see the header of chp_oracle.c
for the readings taken where the paper is incomplete.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chp_oracle.c")
LIB = os.path.join(HERE, "libchp_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over shots)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.oracle_tab_new.restype = P
        L.oracle_tab_new.argtypes = [C.c_int]
        L.oracle_tab_free.argtypes = [P]
        L.oracle_g.restype = C.c_int
        L.oracle_g.argtypes = [C.c_int] * 4
        L.oracle_rowsum.argtypes = [P, C.c_int, C.c_int]
        L.oracle_exec.restype = C.c_long
        L.oracle_exec.argtypes = [P, P, C.c_long, P, C.c_long, C.c_uint64, C.c_uint64,
                                  C.c_uint64, P, P, P]
        L.oracle_tab_get.argtypes = [P, P, P, P]
        L.oracle_tab_set_row.argtypes = [P, C.c_int, P, P, C.c_int]
        L.oracle_tab_get_row.argtypes = [P, C.c_int, P, P, P]
        L.oracle_run.restype = C.c_long
        L.oracle_run.argtypes = [P, C.c_long, P, C.c_long, C.c_int, C.c_long, C.c_uint64,
                                 C.c_uint64, P, C.c_long, P, P, P]
        L.oracle_philox4x64_10.argtypes = [P, P, P]
        L.oracle_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def g(x1, z1, x2, z2) -> int:
    return lib().oracle_g(x1, z1, x2, z2)


class Tableau:
    """One CHP tableau (rows 0..n-1 destabilizers, n..2n-1 stabilizers, 2n scratch)."""

    def __init__(self, n: int):
        self.n = n
        self.h = lib().oracle_tab_new(n)
        if not self.h:
            raise MemoryError("oracle_tab_new failed")
        self.instr_index = 0

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_tab_free(self.h)
            self.h = None

    def execute(self, instr: np.ndarray, targets: np.ndarray, seed: int = 0, shot: int = 0,
                want_flags: bool = False):
        """Run instructions; the RNG instruction index continues from earlier calls."""
        instr = np.ascontiguousarray(instr)
        targets = np.ascontiguousarray(targets, dtype=np.int32)
        nmeas = int(sum(int(i["ntargets"]) for i in instr if int(i["kind"]) in (7, 8, 9)))
        rec = np.zeros(max(nmeas, 1), dtype=np.uint8)
        flags = np.zeros(max(nmeas, 1), dtype=np.uint8)
        nfl = C.c_long(0)
        got = lib().oracle_exec(self.h, _p(instr), len(instr), _p(targets), len(targets),
                                seed, shot, self.instr_index, _p(rec), _p(flags), C.byref(nfl))
        if got < 0:
            raise ValueError("malformed op stream")
        self.instr_index += len(instr)
        if want_flags:
            return rec[:got].copy(), flags[: nfl.value].copy()
        return rec[:got].copy()

    def get(self):
        n = self.n
        x = np.zeros((2 * n, n), dtype=np.uint8)
        z = np.zeros((2 * n, n), dtype=np.uint8)
        r = np.zeros(2 * n, dtype=np.uint8)
        lib().oracle_tab_get(self.h, _p(x), _p(z), _p(r))
        return x, z, r

    def set_row(self, i, x, z, r):
        x = np.ascontiguousarray(x, dtype=np.uint8)
        z = np.ascontiguousarray(z, dtype=np.uint8)
        lib().oracle_tab_set_row(self.h, i, _p(x), _p(z), int(r))

    def get_row(self, i):
        x = np.zeros(self.n, dtype=np.uint8)
        z = np.zeros(self.n, dtype=np.uint8)
        r = np.zeros(1, dtype=np.uint8)
        lib().oracle_tab_get_row(self.h, i, _p(x), _p(z), _p(r))
        return x, z, int(r[0])

    def rowsum(self, h, i):
        lib().oracle_rowsum(self.h, h, i)


def run(circ, shots: int, seed: int, first_shot: int = 0, want_tableau: bool = False):
    """Sample ``shots`` shots of a circuit.  Returns record [shots, M] (uint8) and optionally
    the final tableaux (x, z: [shots, 2n, n]; r: [shots, 2n])."""
    instr, targets = circ.arrays()
    n = circ.n
    nrec = circ.num_measurements()
    rec = np.zeros((shots, max(nrec, 1)), dtype=np.uint8)
    tx = tz = tr = None
    if want_tableau:
        tx = np.zeros((shots, 2 * n, n), dtype=np.uint8)
        tz = np.zeros((shots, 2 * n, n), dtype=np.uint8)
        tr = np.zeros((shots, 2 * n), dtype=np.uint8)
    got = lib().oracle_run(_p(instr), len(instr), _p(targets), len(targets), n, shots,
                           first_shot, seed, _p(rec), nrec, _p(tx), _p(tz), _p(tr))
    if got < 0:
        raise ValueError("oracle_run failed")
    rec = rec[:, :nrec]
    if want_tableau:
        return rec, (tx, tz, tr)
    return rec


def threads() -> int:
    return lib().oracle_threads()
