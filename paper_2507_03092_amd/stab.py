"""Python binding of libstab (include/stab.h): argument marshalling only.

Every step of the simulation runs in the HIP kernels behind the C ABI; torch provides the
device buffer that holds the tableaux and the HIP stream.  There is no CPU fallback: if the
library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import circuits as _circ

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libstab.so")

OK, EINVAL, ENOMEM, EDEVICE, ERANGE, EINTERNAL = 0, -1, -2, -3, -4, -5
MODE_SHARED, MODE_FULL = 0, 1
_MODES = {"shared": MODE_SHARED, "full": MODE_FULL, MODE_SHARED: MODE_SHARED, MODE_FULL: MODE_FULL}

# every function declared in include/stab.h
EXPORTS = ("stab_max_qubits", "stab_tableau_bytes", "stab_create", "stab_destroy", "stab_run",
           "stab_apply_layer", "stab_measure", "stab_get_tableau", "stab_compile", "stab_execute",
           "stab_program_records", "stab_program_destroy", "stab_reset", "stab_sample", "stab_sample_noalloc",
           "stab_get_counters", "stab_set_timing", "stab_set_graph", "stab_get_kernel_times", "stab_plan_describe",
           "stab_batch_bytes", "stab_batch_create", "stab_batch_destroy", "stab_batch_reset",
           "stab_batch_compile", "stab_batch_program_records", "stab_batch_program_destroy",
           "stab_batch_execute", "stab_batch_autotune", "stab_batch_program_set_tile", "stab_batch_program_tile",
           "stab_batch_get_tableau", "stab_batch_get_counters",
           "stab_commute", "stab_server_request_bytes", "stab_server_create", "stab_server_destroy",
           "stab_server_program", "stab_server_program_records", "stab_server_submit", "stab_server_step",
           "stab_server_poll", "stab_server_records", "stab_server_result", "stab_server_stats",
           "stab_server_set_lane", "stab_server_cancel", "stab_set_rng",
           "stab_last_error")
PLAN_FIELDS = ("segments", "measurement_layers", "gate_layers", "gates", "noise_instructions",
               "noise_units", "records", "max_layer")
TILE_WHOLE_WAVE = 0x100   # STAB_TILE_WHOLE_WAVE
TILE_ONE_BLOCK = 0x200    # STAB_TILE_ONE_BLOCK
TUNE_FORCE = 1            # STAB_TUNE_FORCE
KERNELS = ("init", "noise_draw", "segment", "classify", "det", "chain", "reset_record", "pack", "replay",
           "extract")


class StabError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libstab error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libstab.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2507_03092_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U32, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
    sig = {
        "stab_max_qubits": (I32, []),
        "stab_tableau_bytes": (C.c_int, [I32, I32, I32, C.POINTER(U64)]),
        "stab_create": (C.c_int, [I32, I32, I32, U64, U64, P, U64, P, C.POINTER(P)]),
        "stab_destroy": (None, [P]),
        "stab_run": (C.c_int, [P, P, I32, P, I64, P]),
        "stab_apply_layer": (C.c_int, [P, P, I32, P, I64]),
        "stab_measure": (C.c_int, [P, U32, P, I32, P]),
        "stab_get_tableau": (C.c_int, [P, I32, P, P, P]),
        "stab_compile": (C.c_int, [P, P, I32, P, I64, C.POINTER(P)]),
        "stab_execute": (C.c_int, [P, P, P, C.POINTER(C.c_float)]),
        "stab_program_records": (I64, [P]),
        "stab_program_destroy": (None, [P]),
        "stab_reset": (C.c_int, [P, U64, U64]),
        "stab_sample": (C.c_int, [P, I32, P, I64, I32, I32, I32, U64, P, U64, P, P, C.POINTER(C.c_float)]),
        "stab_sample_noalloc": (C.c_int, [P, I32, P, I64, I32, I32, I32, U64, P, U64, P, P]),
        "stab_get_counters": (C.c_int, [P, P, I32]),
        "stab_set_timing": (C.c_int, [P, I32]),
        "stab_set_graph": (C.c_int, [P, I32]),
        "stab_get_kernel_times": (C.c_int, [P, P, P, I32]),
        "stab_plan_describe": (C.c_int, [I32, I32, I32, P, I32, P, I64, P, I32]),
        "stab_batch_bytes": (C.c_int, [I32, P, C.POINTER(U64)]),
        "stab_batch_create": (C.c_int, [I32, P, U64, P, U64, P, C.POINTER(P)]),
        "stab_batch_destroy": (None, [P]),
        "stab_batch_reset": (C.c_int, [P, U64]),
        "stab_batch_compile": (C.c_int, [P, P, P, P, P, C.POINTER(P)]),
        "stab_batch_program_records": (I64, [P, I32]),
        "stab_batch_program_destroy": (None, [P]),
        "stab_batch_execute": (C.c_int, [P, P, P, C.POINTER(C.c_float)]),
        "stab_batch_autotune": (C.c_int, [P, P, I32, I32, C.POINTER(I32)]),
        "stab_batch_program_set_tile": (C.c_int, [P, I32]),
        "stab_batch_program_tile": (I32, [P]),
        "stab_batch_get_tableau": (C.c_int, [P, I32, P, P, P]),
        "stab_batch_get_counters": (C.c_int, [P, P, I32]),
        "stab_commute": (C.c_int, [P, I32, P, I32, I32, P, P, P]),
        "stab_server_request_bytes": (C.c_int, [P, I32, I32, C.POINTER(U64)]),
        "stab_server_create": (C.c_int, [P, U64, P, C.POINTER(P)]),
        "stab_server_destroy": (None, [P]),
        "stab_server_program": (C.c_int, [P, P, I32, P, I64, I32, C.POINTER(I32)]),
        "stab_server_program_records": (I64, [P, I32]),
        "stab_server_submit": (C.c_int, [P, I32, I32, U64, C.POINTER(I64)]),
        "stab_server_step": (C.c_int, [P, C.POINTER(I32)]),
        "stab_server_poll": (C.c_int, [P, P, I32]),
        "stab_server_records": (I64, [P, I64]),
        "stab_server_result": (C.c_int, [P, I64, P]),
        "stab_server_stats": (C.c_int, [P, P, I32]),
        "stab_server_set_lane": (C.c_int, [P, I32, I32]),
        "stab_server_cancel": (C.c_int, [P, I64]),
        "stab_set_rng": (C.c_int, [P, U64, U64]),
        "stab_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise StabError(rc, lib().stab_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def unpack_record(bits: np.ndarray, shots: int, nrec: int) -> np.ndarray:
    nbytes = (nrec + 7) // 8
    b = bits.reshape(shots, nbytes)
    return np.unpackbits(b, axis=1, bitorder="little")[:, :nrec]


def tableau_bytes(n: int, shots: int, mode="shared") -> int:
    out = C.c_uint64(0)
    _check(lib().stab_tableau_bytes(n, shots, _MODES[mode], C.byref(out)))
    return out.value


def plan_describe(circ: _circ.Circuit, shots: int = 1, mode="shared") -> dict:
    """Host-only: how the library splits a stream into segments and layers (no GPU used)."""
    instr, tg = circ.arrays()
    out = np.zeros(len(PLAN_FIELDS), dtype=np.int64)
    _check(lib().stab_plan_describe(circ.n, shots, _MODES[mode], _ptr(instr), len(instr), _ptr(tg), len(tg),
                                    _ptr(out), len(PLAN_FIELDS)))
    return dict(zip(PLAN_FIELDS, (int(v) for v in out)))


def max_qubits() -> int:
    return lib().stab_max_qubits()


class Program:
    def __init__(self, ctx: "Context", handle, nrec: int, ninstr: int):
        self.ctx, self.h, self.nrec, self.ninstr = ctx, handle, nrec, ninstr

    def __del__(self):
        try:
            if getattr(self, "h", None) and _lib is not None:
                _lib.stab_program_destroy(self.h)
        except Exception:   # interpreter shutdown
            pass
        self.h = None


class Context:
    """`shots` tableaux of n qubits on one GPU (stab_create)."""

    def __init__(self, n: int, shots: int = 1, mode="shared", seed: int = 0, first_shot: int = 0,
                 device: str = "cuda:0"):
        import torch

        self.n, self.shots, self.mode = n, shots, _MODES[mode]
        nbytes = tableau_bytes(n, shots, mode)
        self.device = torch.device(device)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p(None)
        _check(lib().stab_create(n, shots, self.mode, seed, first_shot, C.c_void_p(self.buf.data_ptr()),
                                 nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().stab_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown
            pass

    def compile(self, circ: _circ.Circuit) -> Program:
        instr, tg = circ.arrays()
        h = C.c_void_p(None)
        _check(lib().stab_compile(self.h, _ptr(instr), len(instr), _ptr(tg), len(tg), C.byref(h)))
        return Program(self, h, lib().stab_program_records(h), len(instr))

    def execute(self, prog: Program, timed: bool = False):
        nbytes = (prog.nrec + 7) // 8
        out = np.zeros(max(self.shots * nbytes, 1), dtype=np.uint8)
        ms = C.c_float(0.0)
        _check(lib().stab_execute(self.h, prog.h, _ptr(out), C.byref(ms)))
        rec = unpack_record(out[: self.shots * nbytes], self.shots, prog.nrec)
        return (rec, ms.value) if timed else rec

    def run(self, circ: _circ.Circuit) -> np.ndarray:
        instr, tg = circ.arrays()
        nrec = circ.num_measurements()
        nbytes = (nrec + 7) // 8
        out = np.zeros(max(self.shots * nbytes, 1), dtype=np.uint8)
        _check(lib().stab_run(self.h, _ptr(instr), len(instr), _ptr(tg), len(tg), _ptr(out)))
        return unpack_record(out[: self.shots * nbytes], self.shots, nrec)

    def apply_layer(self, circ: _circ.Circuit) -> None:
        instr, tg = circ.arrays()
        _check(lib().stab_apply_layer(self.h, _ptr(instr), len(instr), _ptr(tg), len(tg)))

    def measure(self, qubits, kind: int = _circ.M) -> np.ndarray:
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        nbytes = (len(q) + 7) // 8
        out = np.zeros(max(self.shots * nbytes, 1), dtype=np.uint8)
        _check(lib().stab_measure(self.h, kind, _ptr(q), len(q), _ptr(out)))
        if kind == _circ.R:
            return np.zeros((self.shots, 0), dtype=np.uint8)
        return unpack_record(out[: self.shots * nbytes], self.shots, len(q))

    def get_tableau(self, shot: int = 0):
        n = self.n
        x = np.zeros((2 * n, n), dtype=np.uint8)
        z = np.zeros((2 * n, n), dtype=np.uint8)
        r = np.zeros(2 * n, dtype=np.uint8)
        _check(lib().stab_get_tableau(self.h, shot, _ptr(x), _ptr(z), _ptr(r)))
        return x, z, r

    def reset(self, seed: int, first_shot: int = 0) -> None:
        _check(lib().stab_reset(self.h, seed, first_shot))

    def set_rng(self, seed: int, first_shot: int = 0) -> None:
        """Key of later draws (stab_set_rng); the tableaux and the instruction counter stay."""
        _check(lib().stab_set_rng(self.h, seed, first_shot))

    def set_timing(self, enable: bool, kernels=None) -> None:
        """Time every kernel (kernels=None) or the named ones, with HIP events on the stream."""
        if not enable:
            mask = 0
        elif kernels is None:
            mask = (1 << len(KERNELS)) - 1
        else:
            mask = sum(1 << KERNELS.index(k) for k in kernels)
        _check(lib().stab_set_timing(self.h, mask))

    def set_graph(self, enable: bool) -> None:
        """Replay a program's launches as a captured hipGraph while its key is unchanged."""
        _check(lib().stab_set_graph(self.h, 1 if enable else 0))

    def kernel_times(self) -> dict:
        """{kernel name: (total ms, launches)} since set_timing(True)."""
        ms = np.zeros(len(KERNELS), dtype=np.float64)
        n = np.zeros(len(KERNELS), dtype=np.uint64)
        _check(lib().stab_get_kernel_times(self.h, _ptr(ms), _ptr(n), len(KERNELS)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}

    def counters(self) -> np.ndarray:
        c = np.zeros(12, dtype=np.uint64)
        _check(lib().stab_get_counters(self.h, _ptr(c), 12))
        return c


def sample(circ: _circ.Circuit, shots: int, seed: int, mode="shared", device: str = "cuda:0"):
    """stab_sample: returns (record [shots, nrec] uint8, device milliseconds)."""
    import torch

    instr, tg = circ.arrays()
    nrec = circ.num_measurements()
    nbytes = tableau_bytes(circ.n, shots, mode)
    buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    out = np.zeros(max(shots * ((nrec + 7) // 8), 1), dtype=np.uint8)
    ms = C.c_float(0.0)
    _check(lib().stab_sample(_ptr(instr), len(instr), _ptr(tg), len(tg), circ.n, shots, _MODES[mode],
                             seed, C.c_void_p(buf.data_ptr()), nbytes, C.c_void_p(stream.cuda_stream),
                             _ptr(out), C.byref(ms)))
    return unpack_record(out[: shots * ((nrec + 7) // 8)], shots, nrec), ms.value


NOALLOC_SCRATCH_BYTES = 64 << 20   # STAB_NOALLOC_SCRATCH_BYTES


def sample_noalloc(circ: _circ.Circuit, shots: int, seed: int, mode="shared", device: str = "cuda:0",
                   buf=None):
    """stab_sample_noalloc: the record [shots, nrec] uint8.  buf (optional): a caller-owned
    torch uint8 device tensor of at least tableau_bytes() bytes for the tableaux."""
    import torch

    instr, tg = circ.arrays()
    nrec = circ.num_measurements()
    nbytes = tableau_bytes(circ.n, shots, mode)
    if buf is None:
        buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    out = np.zeros(max(shots * ((nrec + 7) // 8), 1), dtype=np.uint8)
    _check(lib().stab_sample_noalloc(_ptr(instr), len(instr), _ptr(tg), len(tg), circ.n, shots, _MODES[mode],
                                     seed, C.c_void_p(buf.data_ptr()), buf.numel(), C.c_void_p(stream.cuda_stream),
                                     _ptr(out)))
    return unpack_record(out[: shots * ((nrec + 7) // 8)], shots, nrec)


# ------------------------------------------------------------------ multi-circuit batches ---
def batch_bytes(ns) -> int:
    n = np.ascontiguousarray(ns, dtype=np.int32)
    out = C.c_uint64(0)
    _check(lib().stab_batch_bytes(len(n), _ptr(n), C.byref(out)))
    return out.value


class BatchProgram:
    def __init__(self, batch: "Batch", handle, nrec):
        self.batch, self.h, self.nrec = batch, handle, nrec
        self.rec_byte = np.concatenate([[0], np.cumsum((np.asarray(nrec, dtype=np.int64) + 7) // 8)])

    @property
    def tile(self) -> int:
        """Launch configuration (stab_batch_program_tile)."""
        return int(lib().stab_batch_program_tile(self.h))

    @tile.setter
    def tile(self, value: int) -> None:
        _check(lib().stab_batch_program_set_tile(self.h, int(value)))

    def __del__(self):
        try:
            if getattr(self, "h", None) and _lib is not None:
                _lib.stab_batch_program_destroy(self.h)
        except Exception:   # interpreter shutdown
            pass
        self.h = None


class Batch:
    """Independent circuits of different sizes in one device buffer (stab_batch_create);
    circuit c draws its randomness with key (seed, c)."""

    def __init__(self, ns, seed: int = 0, device: str = "cuda:0"):
        import torch

        self.ns = np.ascontiguousarray(ns, dtype=np.int32)
        nbytes = batch_bytes(self.ns)
        self.device = torch.device(device)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p(None)
        _check(lib().stab_batch_create(len(self.ns), _ptr(self.ns), seed, C.c_void_p(self.buf.data_ptr()), nbytes,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().stab_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown
            pass

    def compile(self, circs) -> BatchProgram:
        if len(circs) != len(self.ns):
            raise ValueError("one circuit per batch slot")
        arrs = [c.arrays() for c in circs]
        instr = np.concatenate([a[0] for a in arrs]) if arrs else np.zeros(0, dtype=_circ.INSTR_DTYPE)
        tg = np.concatenate([a[1] for a in arrs]).astype(np.int32)
        ioff = np.concatenate([[0], np.cumsum([len(a[0]) for a in arrs])]).astype(np.int64)
        toff = np.concatenate([[0], np.cumsum([len(a[1]) for a in arrs])]).astype(np.int64)
        instr = np.ascontiguousarray(instr)
        tg = np.ascontiguousarray(tg)
        if len(tg) == 0:
            tg = np.zeros(1, dtype=np.int32)
        h = C.c_void_p(None)
        _check(lib().stab_batch_compile(self.h, _ptr(instr), _ptr(ioff), _ptr(tg), _ptr(toff), C.byref(h)))
        nrec = [int(lib().stab_batch_program_records(h, c)) for c in range(len(circs))]
        return BatchProgram(self, h, nrec)

    def execute(self, prog: BatchProgram, timed: bool = False):
        """Run every circuit once; returns a list of per-circuit records (uint8 arrays)."""
        total = int(prog.rec_byte[-1])
        out = np.zeros(max(total, 1), dtype=np.uint8)
        ms = C.c_float(0.0)
        _check(lib().stab_batch_execute(self.h, prog.h, _ptr(out), C.byref(ms)))
        recs = [np.unpackbits(out[prog.rec_byte[c]:prog.rec_byte[c + 1]], bitorder="little")[: prog.nrec[c]]
                for c in range(len(prog.nrec))]
        return (recs, ms.value) if timed else recs

    def autotune(self, prog: BatchProgram, meas_quota: int = 0, force: bool = False) -> int:
        """Time every launch configuration on prog from the current state and keep the fastest
        (stab_batch_autotune); the batch's state is left as it was.  Returns the choice."""
        t = C.c_int32(0)
        _check(lib().stab_batch_autotune(self.h, prog.h, int(meas_quota), TUNE_FORCE if force else 0, C.byref(t)))
        return t.value

    def reset(self, seed: int) -> None:
        _check(lib().stab_batch_reset(self.h, seed))

    def get_tableau(self, c: int):
        n = int(self.ns[c])
        x = np.zeros((2 * n, n), dtype=np.uint8)
        z = np.zeros((2 * n, n), dtype=np.uint8)
        r = np.zeros(2 * n, dtype=np.uint8)
        _check(lib().stab_batch_get_tableau(self.h, c, _ptr(x), _ptr(z), _ptr(r)))
        return x, z, r

    def counters(self) -> np.ndarray:
        c = np.zeros(8, dtype=np.uint64)
        _check(lib().stab_batch_get_counters(self.h, _ptr(c), 8))
        return c


# ------------------------------------------------------------------ Pauli commutation ---
def pack_paulis(x: np.ndarray, z: np.ndarray) -> np.ndarray:
    """[m, n] 0/1 x and z bits -> [m, 2*ceil(n/64)] uint64 rows (x words, then z words)."""
    m, n = x.shape
    W = (n + 63) // 64

    def words(bits):
        pad = np.zeros((m, W * 64), dtype=np.uint8)
        pad[:, :n] = bits
        return np.packbits(pad.reshape(m, W, 64), axis=2, bitorder="little").reshape(m, W, 8).view("<u8")[:, :, 0]

    return np.ascontiguousarray(np.concatenate([words(x), words(z)], axis=1))


def commute(A, B, n: int, device: str = "cuda:0", qubitwise: bool = True):
    """stab_commute on packed strings (numpy [na, 2W] or device tensors).  Returns
    (gc, qwc) as [na, nb] uint8 numpy arrays (qwc None unless qubitwise)."""
    import torch

    dev = torch.device(device)
    tA = A if isinstance(A, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(A).view(np.int64)).to(dev)
    tB = B if isinstance(B, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(B).view(np.int64)).to(dev)
    na, nb = tA.shape[0], tB.shape[0]
    nbw = (nb + 63) // 64
    gc = torch.empty((na, nbw), dtype=torch.int64, device=dev)
    qw = torch.empty((na, nbw), dtype=torch.int64, device=dev) if qubitwise else None
    stream = torch.cuda.current_stream(dev)
    _check(lib().stab_commute(C.c_void_p(tA.data_ptr()), na, C.c_void_p(tB.data_ptr()), nb, n,
                              C.c_void_p(gc.data_ptr()), C.c_void_p(qw.data_ptr() if qw is not None else 0),
                              C.c_void_p(stream.cuda_stream)))

    def unpack(t):
        h = t.cpu().numpy().view(np.uint64)
        bits = np.unpackbits(h.view(np.uint8).reshape(na, nbw * 8), axis=1, bitorder="little")
        return bits[:, :nb]

    return unpack(gc), (unpack(qw) if qw is not None else None)


# ------------------------------------------------------------ continuous-batching server ---
SERVER_STATS = ("queued", "resident_requests", "resident_shots", "bytes_in_use", "arena_bytes", "steps",
                "finished", "in_flight", "cancelled")
LANE_AUTO, LANE_BATCH, LANE_SHARED = 0, 1, 2


class Server:
    """stab_server_*: requests admitted by arena bytes; batch-lane shots advance one round per
    step, shared-lane requests run whole on the server's streams."""

    def __init__(self, arena_bytes: int, device: str = "cuda:0"):
        import torch

        self.device = torch.device(device)
        self.buf = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p(None)
        _check(lib().stab_server_create(C.c_void_p(self.buf.data_ptr()), arena_bytes,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.nrec = {}

    def close(self):
        if getattr(self, "h", None):
            lib().stab_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown
            pass

    def program(self, circ) -> int:
        instr, tg = circ.arrays()
        tg = np.ascontiguousarray(tg, dtype=np.int32)
        pid = C.c_int32(0)
        _check(lib().stab_server_program(self.h, _ptr(instr), len(instr), _ptr(tg), len(tg), circ.n,
                                         C.byref(pid)))
        return pid.value

    def set_lane(self, prog: int, lane: int):
        _check(lib().stab_server_set_lane(self.h, prog, lane))

    def cancel(self, rid: int):
        _check(lib().stab_server_cancel(self.h, rid))

    def request_bytes(self, prog: int, shots: int) -> int:
        out = C.c_uint64(0)
        _check(lib().stab_server_request_bytes(self.h, prog, shots, C.byref(out)))
        return out.value

    def submit(self, prog: int, shots: int, seed: int) -> int:
        rid = C.c_int64(0)
        _check(lib().stab_server_submit(self.h, prog, shots, seed, C.byref(rid)))
        return rid.value

    def step(self) -> int:
        nf = C.c_int32(0)
        _check(lib().stab_server_step(self.h, C.byref(nf)))
        return nf.value

    def poll(self, max_ids: int = 4096) -> list:
        ids = np.zeros(max_ids, dtype=np.int64)
        k = lib().stab_server_poll(self.h, _ptr(ids), max_ids)
        if k < 0:
            _check(k)
        return [int(v) for v in ids[:k]]

    def result(self, rid: int, shots: int) -> np.ndarray:
        nrec = lib().stab_server_records(self.h, rid)
        if nrec < 0:
            raise StabError(EINVAL, f"request {rid} is not finished")
        nbytes = (nrec + 7) // 8
        out = np.zeros(max(shots * nbytes, 1), dtype=np.uint8)
        _check(lib().stab_server_result(self.h, rid, _ptr(out)))
        return unpack_record(out[: shots * nbytes], shots, nrec)

    def stats(self) -> dict:
        v = np.zeros(len(SERVER_STATS), dtype=np.int64)
        _check(lib().stab_server_stats(self.h, _ptr(v), len(SERVER_STATS)))
        return dict(zip(SERVER_STATS, (int(x) for x in v)))
