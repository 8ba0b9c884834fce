"""The kernels' rowsum phase bookkeeping against the g-function of the rowsum algorithm
(Appendix A.2; Alg. 1).  The replay and the deterministic reduction do not sum g qubit by qubit:
they use that multiplying Paulis with canonical phase, P_i P_h, raises i to
|P_i| + |P_h| + 2 z_i.x_h - |P_i P_h| (mod 4), |u| = number of qubits where u has both x and z,
so that over a chain of left multiplications D <- P D the powers telescope to
sum|P| + |D_0| - |D_n| + 2 sum z_P.x_D, of which only the parity of the last sum matters.
These tests check that identity exhaustively on one qubit and on random chains, against the
oracle's g (itself pinned by matrix products in test_oracle_pins)."""
from __future__ import annotations

import itertools

import numpy as np

from oracle import oracle as O


def _xz(u):
    return int(np.count_nonzero(u[0] & u[1]))


def test_single_qubit_identity_exhaustive():
    for x1, z1, x2, z2 in itertools.product((0, 1), repeat=4):
        lhs = O.g(x1, z1, x2, z2) % 4
        rhs = (x1 * z1 + x2 * z2 + 2 * z1 * x2 - (x1 ^ x2) * (z1 ^ z2)) % 4
        assert lhs == rhs, (x1, z1, x2, z2)


def test_telescoped_chain_matches_stepwise_g():
    rng = np.random.default_rng(11)
    for trial in range(300):
        n = int(rng.integers(1, 70))
        steps = int(rng.integers(1, 12))
        D = [rng.integers(0, 2, n).astype(np.uint8) for _ in range(2)]
        Ps = [[rng.integers(0, 2, n).astype(np.uint8) for _ in range(2)] for _ in range(steps)]
        # stepwise: sum over steps and qubits of g(P, D) with D updated after each step
        stepwise = 0
        cur = [D[0].copy(), D[1].copy()]
        for P in Ps:
            stepwise += sum(O.g(int(P[0][q]), int(P[1][q]), int(cur[0][q]), int(cur[1][q])) for q in range(n))
            cur = [cur[0] ^ P[0], cur[1] ^ P[1]]
        # telescoped: sum|P| + |D0| - |Dn| + 2 * parity(XOR of z_P & x_D)
        acc = np.zeros(n, dtype=np.uint8)
        tel = _xz(D)
        cur = [D[0].copy(), D[1].copy()]
        for P in Ps:
            acc ^= P[1] & cur[0]
            tel += _xz(P)
            cur = [cur[0] ^ P[0], cur[1] ^ P[1]]
        tel += 2 * (int(np.count_nonzero(acc)) & 1) - _xz(cur)
        assert (stepwise - tel) % 4 == 0, trial
