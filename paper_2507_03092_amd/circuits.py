"""Seeded circuit inputs for the tableau simulator: the op-stream format and its generators.

This module holds no tableau arithmetic.  It only describes circuits (which gate, measurement
or noise channel acts on which qubits) and produces seeded synthetic workloads.  Both the CPU
oracle (``oracle/``) and the HIP library consume the arrays built here.

Op-stream format
----------------
A circuit is a list of *instructions*.  Each instruction has a kind, a count of int32 targets
that it consumes from one flat target array (in order), and three uint64 noise thresholds.
Two-qubit kinds (CX, DEP2) consume targets in pairs ``(a0, b0, a1, b1, ...)``.  Targets of one
instruction act one after another, in order, exactly as if each were its own instruction; the
simulators may run them together only where that gives the same result.

Randomness is counter-based: every random draw is the Philox4x64-10 block (Salmon et al.,
SC'11) with key ``(seed, shot)`` and counter ``(instruction_index, target_position, 0, 0)``,
where ``instruction_index`` is the 0-based position of the instruction in the stream (TICK
included) and ``target_position`` is the index of the target (or pair) within it.  The four
64-bit words of that block are ``u0..u3``:

* DEP1 (single-qubit depolarizing, probability p): an error happens iff ``u0 < t0`` with
  ``t0 = floor(p * 2**64)``; the Pauli is ``1 + mulhi64(u1, 3)`` -> 1=X, 2=Y, 3=Z.
* DEP2 (two-qubit depolarizing on a pair (a, b)): error iff ``u0 < t0``; ``k = 1 + mulhi64(u1, 15)``,
  Pauli on a = ``k >> 2``, on b = ``k & 3`` (0=I, 1=X, 2=Y, 3=Z).
* PAULI1 (px, py, pz): X iff ``u0 < t0``, else Y iff ``u0 < t1``, else Z iff ``u0 < t2``, with
  the cumulative thresholds ``t0 = floor(px 2^64)``, ``t1 = floor((px+py) 2^64)``,
  ``t2 = floor((px+py+pz) 2^64)`` computed exactly from the float64 probabilities.
* M / MR / R: a Z measurement whose outcome is not fixed by the state takes ``u0 >> 63``.
  MR and R then apply X to the qubit when the outcome is 1 (reset to |0>); R records nothing.

Measurement records hold one bit per M/MR target, in stream order (1 = eigenvalue -1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

# ---- instruction kinds (numeric codes are part of the input format) -----------------------------
TICK, H, S, X, Y, Z, CX, M, MR, R, DEP1, DEP2, PAULI1, T1T2 = range(14)

KIND_NAMES = {
    TICK: "TICK", H: "H", S: "S", X: "X", Y: "Y", Z: "Z", CX: "CX", M: "M", MR: "MR", R: "R",
    DEP1: "DEP1", DEP2: "DEP2", PAULI1: "PAULI1", T1T2: "T1T2",
}
NAME_TO_KIND = {v: k for k, v in KIND_NAMES.items()}
TWO_QUBIT = (CX, DEP2)
GATES = (H, S, X, Y, Z, CX)
MEASURES = (M, MR, R)
NOISE = (DEP1, DEP2, PAULI1)
RECORDED = (M, MR)

# 32-byte instruction record, identical to ``stab_instr`` in include/stab.h
INSTR_DTYPE = np.dtype([("kind", "<u4"), ("ntargets", "<u4"),
                        ("t0", "<u8"), ("t1", "<u8"), ("t2", "<u8")])

TWO64 = 1 << 64


def threshold(p: float) -> int:
    """floor(p * 2^64), exact for the float64 value of ``p``; clamped to [0, 2^64-1]."""
    if not (0.0 <= p <= 1.0):
        raise ValueError(f"probability out of range: {p}")
    t = math.floor(Fraction(p) * TWO64)
    return min(t, TWO64 - 1)


def pauli1_thresholds(px: float, py: float, pz: float) -> tuple[int, int, int]:
    """Cumulative thresholds (X, X+Y, X+Y+Z) for a PAULI1 channel, exact in rational arithmetic."""
    fx, fy, fz = Fraction(px), Fraction(py), Fraction(pz)
    if min(fx, fy, fz) < 0 or fx + fy + fz > 1:
        raise ValueError("invalid Pauli channel")
    cum = [fx, fx + fy, fx + fy + fz]
    return tuple(min(math.floor(c * TWO64), TWO64 - 1) for c in cum)  # type: ignore[return-value]


def twirled_t1t2(t: float, t1: float, t2: float) -> tuple[float, float, float]:
    """Pauli-twirl of amplitude damping (T1) followed by pure dephasing (T2) for a duration t.

    The paper builds stochastic Pauli channels by Pauli twirling (Stabilizer Noise Modeling,
    Sec. 2.7).  For relaxation with gamma = 1 - exp(-t/T1) and total coherence decay
    exp(-t/T2), the twirled channel is p_x = p_y = gamma/4 and p_z = (1 - exp(-t/T2))/2 - gamma/4.
    (Requires T2 <= 2 T1.)
    """
    gamma = 1.0 - math.exp(-t / t1)
    px = py = gamma / 4.0
    pz = (1.0 - math.exp(-t / t2)) / 2.0 - gamma / 4.0
    if pz < 0:
        raise ValueError("T2 > 2*T1 is unphysical")
    return px, py, pz


def t1t2_composite(t: float, t1: float, t2: float) -> tuple[float, float]:
    """Relaxation for a duration t (amplitude damping, gamma = 1 - exp(-t/T1)) followed by
    dephasing to a total coherence decay exp(-t/T2), written as a mixture of stochastic
    Clifford+reset operations (Sec. 2.7 and Sec. 4.2: the composite distribution, positive
    when T1 >= T2).  A qubit channel is fixed by its action on the Bloch vector; this one maps
    (x, y, z) to (e2 x, e2 y, e1 z + 1 - e1) with e1 = exp(-t/T1), e2 = exp(-t/T2).  The
    mixture a*I + b*Z(.)Z + c*Reset maps it to ((a - b) x, (a - b) y, (a + b) z + c), so
    c = 1 - e1 and b = (e1 - e2) / 2.  Returns (c, b): the reset and Z probabilities."""
    if t < 0 or t1 <= 0 or t2 <= 0:
        raise ValueError("need t >= 0 and positive T1, T2")
    if t2 > t1:
        raise ValueError("T2 > T1: the composite distribution has a negative weight")
    e1, e2 = math.exp(-t / t1), math.exp(-t / t2)
    return 1.0 - e1, (e1 - e2) / 2.0


def t1t2_thresholds(t: float, t1: float, t2: float) -> tuple[int, int, int]:
    """Cumulative thresholds (reset, reset + Z, 0) of a T1T2 instruction, exact in rational
    arithmetic from the float64 probabilities."""
    c, b = t1t2_composite(t, t1, t2)
    fc, fb = Fraction(c), Fraction(b)
    return (min(math.floor(fc * TWO64), TWO64 - 1), min(math.floor((fc + fb) * TWO64), TWO64 - 1), 0)


@dataclass
class Circuit:
    """An op stream: instructions plus one flat int32 target array."""

    n: int
    kinds: list = field(default_factory=list)
    ntargets: list = field(default_factory=list)
    thresholds: list = field(default_factory=list)
    targets: list = field(default_factory=list)

    def append(self, kind: int, targets=(), t=(0, 0, 0)) -> None:
        targets = [int(q) for q in targets]
        if kind in TWO_QUBIT and len(targets) % 2:
            raise ValueError("two-qubit instruction needs an even target count")
        for q in targets:
            if not (0 <= q < self.n):
                raise ValueError(f"target {q} out of range for n={self.n}")
        self.kinds.append(kind)
        self.ntargets.append(len(targets))
        t = tuple(int(v) for v in t) + (0,) * (3 - len(t))
        self.thresholds.append(t)
        self.targets.extend(targets)

    # convenience builders
    def gate(self, kind, targets):
        self.append(kind, targets)

    def dep1(self, p, targets):
        self.append(DEP1, targets, (threshold(p), 0, 0))

    def dep2(self, p, pairs):
        self.append(DEP2, pairs, (threshold(p), 0, 0))

    def pauli1(self, px, py, pz, targets):
        self.append(PAULI1, targets, pauli1_thresholds(px, py, pz))

    def t1t2(self, t, t1, t2, targets):
        self.append(T1T2, targets, t1t2_thresholds(t, t1, t2))

    def tick(self):
        self.append(TICK, ())

    def __len__(self):
        return len(self.kinds)

    def arrays(self) -> tuple[np.ndarray, np.ndarray]:
        instr = np.zeros(len(self.kinds), dtype=INSTR_DTYPE)
        instr["kind"] = self.kinds
        instr["ntargets"] = self.ntargets
        if self.thresholds:
            th = np.array(self.thresholds, dtype=np.uint64).reshape(-1, 3)
            instr["t0"], instr["t1"], instr["t2"] = th[:, 0], th[:, 1], th[:, 2]
        tg = np.asarray(self.targets, dtype=np.int32)
        return instr, tg

    def num_measurements(self) -> int:
        return sum(nt for k, nt in zip(self.kinds, self.ntargets) if k in RECORDED)

    def counts(self) -> dict:
        out: dict = {}
        for k, nt in zip(self.kinds, self.ntargets):
            name = KIND_NAMES[k]
            units = nt // 2 if k in TWO_QUBIT else nt
            out[name] = out.get(name, 0) + units
        return out


# ---- rotated surface code (Z-memory) --------------------------------------------------------------
@dataclass
class SurfaceLayout:
    d: int
    n: int
    data: list            # data qubit index by (r, c): r*d + c
    x_anc: list           # X-check ancilla qubit indices (in ancilla index order)
    z_anc: list
    anc: list             # all ancillas, in measurement order
    support: dict         # ancilla -> list of data qubits it checks
    is_x: dict            # ancilla -> bool
    cx_layers: list       # 4 lists of (control, target) pairs
    logical_z: list       # data qubits of the logical Z string


def rotated_layout(d: int) -> SurfaceLayout:
    """Rotated surface code of odd distance d: d*d data qubits and d*d-1 check ancillas.

    Data (r, c) is qubit r*d + c.  A plaquette with top-left data corner (r, c) covers the data
    qubits NW=(r,c), NE=(r,c+1), SW=(r+1,c), SE=(r+1,c+1) that exist.  Interior plaquettes
    (0 <= r, c <= d-2) are X-type when (r + c) is even, Z-type otherwise; weight-2 X plaquettes
    sit on the top/bottom boundary and weight-2 Z plaquettes on the left/right boundary.
    Ancillas are numbered d*d + k in row-major scan order of their plaquette position.
    The CNOT order is NW, NE, SW, SE for X checks and NW, SW, NE, SE for Z checks, so each of
    the four layers touches every qubit at most once.
    """
    if d < 3 or d % 2 == 0:
        raise ValueError("d must be odd and >= 3")
    plaq = []
    for r in range(-1, d):
        for c in range(-1, d):
            is_x = (r + c) % 2 == 0
            interior = 0 <= r <= d - 2 and 0 <= c <= d - 2
            top_bot = (r == -1 or r == d - 1) and 0 <= c <= d - 2
            left_right = (c == -1 or c == d - 1) and 0 <= r <= d - 2
            if interior or (top_bot and is_x) or (left_right and not is_x):
                plaq.append((r, c, is_x))
    assert len(plaq) == d * d - 1
    n = 2 * d * d - 1

    def dq(r, c):
        return r * d + c if (0 <= r < d and 0 <= c < d) else None

    support, isx, x_anc, z_anc, anc = {}, {}, [], [], []
    layers = [[], [], [], []]
    for k, (r, c, is_x) in enumerate(plaq):
        a = d * d + k
        anc.append(a)
        isx[a] = is_x
        (x_anc if is_x else z_anc).append(a)
        nw, ne, sw, se = dq(r, c), dq(r, c + 1), dq(r + 1, c), dq(r + 1, c + 1)
        order = (nw, ne, sw, se) if is_x else (nw, sw, ne, se)
        support[a] = [q for q in (nw, ne, sw, se) if q is not None]
        for li, q in enumerate(order):
            if q is None:
                continue
            layers[li].append((a, q) if is_x else (q, a))
    for li in range(4):
        used = [q for pair in layers[li] for q in pair]
        assert len(used) == len(set(used)), "CNOT layer touches a qubit twice"
    return SurfaceLayout(d=d, n=n, data=list(range(d * d)), x_anc=x_anc, z_anc=z_anc, anc=anc,
                         support=support, is_x=isx, cx_layers=layers,
                         logical_z=[dq(0, c) for c in range(d)])


def surface_code_memory(d: int, rounds: int, p: float = 0.0, idle: tuple | None = None,
                        idle_exact: tuple | None = None) -> tuple[Circuit, SurfaceLayout]:
    """Rotated surface-code Z-memory experiment (the paper's QEC workload, Sec. 4.1).

    Each round: H on X ancillas, four CNOT layers, H on X ancillas, MR on every ancilla.
    With p > 0, DEP1(p) follows each H and DEP2(p) each CNOT pair.  With ``idle=(px,py,pz)``
    a PAULI1 channel acts on every qubit after each of the seven layers of a round; with
    ``idle_exact=(t, T1, T2)`` the exact relaxation/dephasing composite (T1T2) acts there
    instead.  After the last round every data qubit is measured (M).  All qubits start in |0>.
    """
    lay = rotated_layout(d)
    c = Circuit(n=lay.n)
    allq = list(range(lay.n))

    def idle_noise():
        if idle is not None:
            c.pauli1(*idle, allq)
        if idle_exact is not None:
            c.t1t2(*idle_exact, allq)

    for _ in range(rounds):
        c.tick()
        c.gate(H, lay.x_anc)
        if p > 0:
            c.dep1(p, lay.x_anc)
        idle_noise()
        for li in range(4):
            flat = [q for pair in lay.cx_layers[li] for q in pair]
            c.gate(CX, flat)
            if p > 0:
                c.dep2(p, flat)
            idle_noise()
        c.gate(H, lay.x_anc)
        if p > 0:
            c.dep1(p, lay.x_anc)
        idle_noise()
        c.append(MR, lay.anc)
        idle_noise()
    c.tick()
    c.append(M, lay.data)
    return c, lay


def surface_detectors(lay: SurfaceLayout, rounds: int, record: np.ndarray):
    """Detector and observable bits of a Z-memory record (uint8 array [shots, measurements]).

    Detectors: round-1 Z checks; every check against its previous round (rounds >= 2);
    each Z check against the parity of its data qubits in the final readout.  Observable:
    parity of the final readout on the logical-Z data string.  All are 0 without noise.
    """
    na = len(lay.anc)
    rec = np.asarray(record, dtype=np.uint8)
    anc_pos = {a: i for i, a in enumerate(lay.anc)}
    rounds_rec = rec[:, : rounds * na].reshape(rec.shape[0], rounds, na)
    final = rec[:, rounds * na:]
    dets = []
    z_idx = [anc_pos[a] for a in lay.z_anc]
    dets.append(rounds_rec[:, 0, z_idx])
    if rounds > 1:
        dets.append((rounds_rec[:, 1:, :] ^ rounds_rec[:, :-1, :]).reshape(rec.shape[0], -1))
    fin = []
    for a in lay.z_anc:
        par = np.bitwise_xor.reduce(final[:, lay.support[a]], axis=1)
        fin.append(par ^ rounds_rec[:, -1, anc_pos[a]])
    dets.append(np.stack(fin, axis=1))
    obs = np.bitwise_xor.reduce(final[:, lay.logical_z], axis=1)
    return np.concatenate(dets, axis=1), obs


# ---- random circuits ------------------------------------------------------------------------------
def random_clifford_measure(n: int, depth: int, seed: int, p_meas: float = 0.2,
                            noise: float = 0.0, resets: bool = True) -> Circuit:
    """Random Clifford+measurement circuit for parity tests.

    Each layer is a random perfect matching: a pair gets a CX (random orientation) with
    probability 0.5, otherwise each qubit gets H, S, X, Y, Z or nothing.  After a layer, a
    random subset of qubits is measured with M, MR or R.  Optional DEP1/DEP2 noise.
    """
    rng = np.random.default_rng(seed)
    c = Circuit(n=n)
    for _ in range(depth):
        perm = rng.permutation(n)
        pairs, singles = [], {H: [], S: [], X: [], Y: [], Z: []}
        for i in range(0, n - 1, 2):
            a, b = int(perm[i]), int(perm[i + 1])
            if rng.random() < 0.5:
                pairs += [a, b] if rng.random() < 0.5 else [b, a]
            else:
                for q in (a, b):
                    k = int(rng.integers(0, 6))
                    if k < 5:
                        singles[(H, S, X, Y, Z)[k]].append(q)
        if n % 2:
            q = int(perm[-1])
            k = int(rng.integers(0, 6))
            if k < 5:
                singles[(H, S, X, Y, Z)[k]].append(q)
        for kind in (H, S, X, Y, Z):
            if singles[kind]:
                c.gate(kind, singles[kind])
        if pairs:
            c.gate(CX, pairs)
            if noise > 0:
                c.dep2(noise, pairs)
        if noise > 0:
            c.dep1(noise, list(range(n)))
        mq = [int(q) for q in np.nonzero(rng.random(n) < p_meas)[0]]
        rng.shuffle(mq)
        if mq:
            kinds = (M, MR, R) if resets else (M,)
            c.append(kinds[int(rng.integers(0, len(kinds)))], mq)
    c.append(M, list(range(n)))
    return c


class PackedCircuit:
    """An op stream already in array form (instruction records + int32 targets), for
    generated workloads too large to build target by target."""

    def __init__(self, n: int, instr: np.ndarray, targets: np.ndarray):
        self.n = n
        self.instr = np.ascontiguousarray(instr, dtype=INSTR_DTYPE)
        self.targets = np.ascontiguousarray(targets, dtype=np.int32)
        if int(self.instr["ntargets"].sum()) != len(self.targets):
            raise ValueError("target count does not match the instructions")

    def append(self, kind: int, targets=(), t=(0, 0, 0)) -> None:
        tg = np.asarray(targets, dtype=np.int64).reshape(-1)
        if kind in TWO_QUBIT and len(tg) % 2:
            raise ValueError("two-qubit instruction needs an even target count")
        if len(tg) and (tg.min() < 0 or tg.max() >= self.n):
            raise ValueError(f"target out of range for n={self.n}")
        rec = np.zeros(1, dtype=INSTR_DTYPE)
        rec["kind"], rec["ntargets"] = kind, len(tg)
        t = tuple(int(v) for v in t) + (0,) * (3 - len(t))
        rec["t0"], rec["t1"], rec["t2"] = t
        self.instr = np.concatenate([self.instr, rec])
        self.targets = np.concatenate([self.targets, tg.astype(np.int32)])

    def gate(self, kind, targets):
        self.append(kind, targets)

    def arrays(self) -> tuple[np.ndarray, np.ndarray]:
        return self.instr, self.targets

    def num_measurements(self) -> int:
        rec = np.isin(self.instr["kind"], list(RECORDED))
        return int(self.instr["ntargets"][rec].sum())

    def __len__(self):
        return len(self.instr)


def random_layered_clifford(n: int, layers: int, seed, meas_every: int = 10,
                            meas_frac: float = 0.1) -> PackedCircuit:
    """The batched random-Clifford workload: ``layers`` random perfect-matching layers over
    {H, S, CX} (a pair gets CX with probability 0.5, random orientation; otherwise each of
    its qubits gets H, S or nothing with probability 1/3 each; with odd n the unmatched qubit
    idles), and M on a random ``meas_frac`` subset (in random order) after every
    ``meas_every``-th layer.  Noiseless."""
    rng = np.random.default_rng(seed)
    h = n // 2
    perm = np.argsort(rng.random((layers, n)), axis=1).astype(np.int32)
    a, b = perm[:, 0:2 * h:2], perm[:, 1:2 * h:2]
    cx = rng.random((layers, h)) < 0.5
    flip = rng.random((layers, h)) < 0.5
    ctrl, targ = np.where(flip, b, a), np.where(flip, a, b)
    single = np.concatenate([a, b], axis=1)
    free = np.concatenate([~cx, ~cx], axis=1)
    k = rng.integers(0, 3, size=(layers, 2 * h))
    hm, sm = free & (k == 0), free & (k == 1)
    parts = [(H, single[hm], hm.sum(axis=1)), (S, single[sm], sm.sum(axis=1)),
             (CX, np.stack([ctrl[cx], targ[cx]], axis=1).reshape(-1), 2 * cx.sum(axis=1))]
    k_meas = max(1, int(round(meas_frac * n)))
    mlayers = [li for li in range(layers) if (li + 1) % meas_every == 0]
    meas = {li: rng.choice(n, size=k_meas, replace=False).astype(np.int32) for li in mlayers}
    offs = [np.concatenate([[0], np.cumsum(cnt)]) for _, _, cnt in parts]
    kinds, counts, chunks = [], [], []
    for li in range(layers):
        for (kind, arr, cnt), off in zip(parts, offs):
            if cnt[li]:
                kinds.append(kind)
                counts.append(int(cnt[li]))
                chunks.append(arr[off[li]:off[li + 1]])
        if li in meas:
            kinds.append(M)
            counts.append(k_meas)
            chunks.append(meas[li])
    instr = np.zeros(len(kinds), dtype=INSTR_DTYPE)
    instr["kind"] = kinds
    instr["ntargets"] = counts
    tg = np.concatenate(chunks).astype(np.int32) if chunks else np.zeros(0, dtype=np.int32)
    return PackedCircuit(n, instr, tg)


def random_batch(ncirc: int, n_lo: int, n_hi: int, layers: int, seed: int, meas_every: int = 10,
                 meas_frac: float = 0.1):
    """Uneven batch of independent random layered Clifford circuits: sizes n ~ U{n_lo..n_hi}
    drawn from ``seed``, circuit c generated from the seed pair (seed, c).
    Returns (sizes, circuits)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=ncirc)
    circs = [random_layered_clifford(int(ns[c]), layers, (seed, c), meas_every, meas_frac) for c in range(ncirc)]
    return ns.astype(np.int32), circs


# ---- Pauli strings (the grouping check) ---------------------------------------------------------------
def random_paulis(m: int, n: int, seed, p_identity: float = 0.25):
    """m random Pauli strings on n qubits as 0/1 arrays (x, z) [m, n]: each qubit is I with
    probability p_identity, else X, Y or Z with equal probability."""
    rng = np.random.default_rng(seed)
    ident = rng.random((m, n)) < p_identity
    k = rng.integers(1, 4, size=(m, n))          # 1 X, 2 Z, 3 Y
    x = ((k & 1) == 1) & ~ident
    z = ((k & 2) == 2) & ~ident
    return x.astype(np.uint8), z.astype(np.uint8)


# Pauli-string commutation workload: 32768 strings against themselves on 256 qubits
COMMUTE = dict(m=32768, n=256, seed=6)


# ---- serving workload (continuous batching) -------------------------------------------------------
# Poisson arrivals of memory-experiment requests: d ~ U{3, 5, ..., 31}, d rounds, DEP1/DEP2
# p = 1e-3, shots ~ U{1..100}
SERVING = dict(rate=200.0, duration=60.0, d_lo=3, d_hi=31, shots_hi=100, p=1e-3, seed=5)


def serving_requests(rate: float, duration: float, seed: int, d_lo: int = 3, d_hi: int = 31,
                     shots_hi: int = 100):
    """Arrival times (seconds), distances, shot counts and request seeds of a Poisson stream."""
    rng = np.random.default_rng(seed)
    times = []
    t = rng.exponential(1.0 / rate)
    while t < duration:
        times.append(t)
        t += rng.exponential(1.0 / rate)
    m = len(times)
    ds = rng.choice(np.arange(d_lo, d_hi + 1, 2), size=m)
    shots = rng.integers(1, shots_hi + 1, size=m)
    seeds = rng.integers(0, 2 ** 62, size=m)
    return np.array(times), ds.astype(np.int32), shots.astype(np.int32), seeds.astype(np.uint64)


# ---- the surface-code workloads -----------------------------------------------------------------
IDLE_T1T2 = twirled_t1t2(1e-6, 100e-6, 100e-6)

# uneven multi-circuit batch: 4096 random layered Clifford circuits, n ~ U{64..2048},
# 200 layers, M on 10% of the qubits every 10 layers, noiseless
RANDOM_BATCH = dict(ncirc=4096, n_lo=64, n_hi=2048, layers=200, seed=4, meas_every=10, meas_frac=0.1)

WORKLOADS = {
    "surface_d3": dict(d=3, rounds=3, p=1e-3, idle=None, seed=1, shots=1000),
    "surface_d25": dict(d=25, rounds=25, p=1e-3, idle=None, seed=2, shots=100),
    "surface_d71": dict(d=71, rounds=71, p=1e-3, idle=IDLE_T1T2, seed=3, shots=10),
    # the exact (not twirled) T1/T2 idle: per-shot tableaux, run as a batch of shots
    "surface_d25_t1t2": dict(d=25, rounds=25, p=1e-3, idle=None, idle_exact=(1e-6, 100e-6, 100e-6),
                             seed=7, shots=100),
}


def workload(name: str, rounds: int | None = None):
    """(circuit, layout, seed, shots) for a named surface-code workload."""
    w = WORKLOADS[name]
    r = w["rounds"] if rounds is None else rounds
    circ, lay = surface_code_memory(w["d"], r, w["p"], w["idle"], w.get("idle_exact"))
    return circ, lay, w["seed"], w["shots"]
