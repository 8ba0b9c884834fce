"""Oracle (test infrastructure only): commutation of Pauli strings, written from its
definition (Sec. 3.2).  Pauli strings are 0/1 arrays x[m, n], z[m, n] (X = (1,0), Z = (0,1),
Y = (1,1), I = (0,0)).  At one qubit two single-qubit Paulis anticommute iff
x1 z2 + z1 x2 is odd; two strings anticommute (group-wise) iff the number of anticommuting
qubits is odd, and conflict qubit-wise iff that number is non-zero.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline may use this module.
"""
from __future__ import annotations

import numpy as np


def anticommuting_qubits(ax, az, bx, bz) -> np.ndarray:
    """[na, nb] number of qubits whose single-qubit factors anticommute:
    sum_q (ax bz + az bx - 2 ax az bx bz) (the per-qubit XOR of the two AND terms)."""
    ax, az, bx, bz = (np.asarray(v, dtype=np.int64) for v in (ax, az, bx, bz))
    return ax @ bz.T + az @ bx.T - 2 * ((ax & az) @ (bx & bz).T)


def commute_matrix(ax, az, bx, bz):
    """(gc, qwc) as uint8 [na, nb]: gc = 1 iff the strings anticommute, qwc = 1 iff some qubit
    anticommutes."""
    cnt = anticommuting_qubits(ax, az, bx, bz)
    return (cnt % 2).astype(np.uint8), (cnt > 0).astype(np.uint8)
