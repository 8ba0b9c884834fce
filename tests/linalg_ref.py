"""Dense linear-algebra references for pinning the oracle (test helpers only).

Everything here is textbook quantum mechanics in numpy complex128: Pauli and gate matrices,
conjugation, and a brute-force state-vector simulator.  None of it uses the tableau method.
Qubit q is bit q of the basis-state index.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
HAD = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
SPH = np.array([[1, 0], [0, 1j]], dtype=complex)


def sigma(x: int, z: int) -> np.ndarray:
    """Hermitian single-qubit Pauli from its (x, z) bits: I, X, Z, Y."""
    return {(0, 0): I2, (1, 0): PX, (0, 1): PZ, (1, 1): PY}[(int(x), int(z))]


def pauli_matrix(x, z, r: int = 0) -> np.ndarray:
    """(-1)^r * tensor product of sigma(x_j, z_j); qubit j is bit j of the index."""
    m = np.array([[1.0 + 0j]])
    for j in range(len(x)):
        m = np.kron(sigma(x[j], z[j]), m)   # qubit j is the j-th least significant factor
    return (-1) ** int(r) * m


def decompose(mat: np.ndarray, n: int):
    """Write a matrix that is +-1 times a Hermitian Pauli as (x, z, r); None if it is not."""
    import itertools
    for bits in itertools.product((0, 1), repeat=2 * n):
        x, z = bits[:n], bits[n:]
        p = pauli_matrix(x, z)
        c = np.trace(p.conj().T @ mat) / (2 ** n)
        if abs(abs(c) - 1) < 1e-9:
            if np.allclose(mat, c * p, atol=1e-9):
                if abs(c - 1) < 1e-9:
                    return list(x), list(z), 0
                if abs(c + 1) < 1e-9:
                    return list(x), list(z), 1
                return None
    return None


def op_on(n: int, u: np.ndarray, q: int) -> np.ndarray:
    """Embed a single-qubit unitary on qubit q of n."""
    m = np.array([[1.0 + 0j]])
    for j in range(n):
        m = np.kron(u if j == q else I2, m)
    return m


def cx_matrix(n: int, c: int, t: int) -> np.ndarray:
    dim = 2 ** n
    m = np.zeros((dim, dim), dtype=complex)
    for b in range(dim):
        b2 = b ^ (1 << t) if (b >> c) & 1 else b
        m[b2, b] = 1
    return m


class StateVector:
    """Brute-force state vector (2^n amplitudes) for n <= ~12."""

    def __init__(self, n: int):
        self.n = n
        self.psi = np.zeros(2 ** n, dtype=complex)
        self.psi[0] = 1.0

    def _apply1(self, u, q):
        # C-order reshape puts the most significant bit first, so qubit q is axis n-1-q
        psi = self.psi.reshape([2] * self.n)
        ax = self.n - 1 - q
        psi = np.moveaxis(psi, ax, 0)
        psi = np.tensordot(u, psi, axes=([1], [0]))
        psi = np.moveaxis(psi, 0, ax)
        self.psi = psi.reshape(-1)

    def h(self, q):
        self._apply1(HAD, q)

    def s(self, q):
        self._apply1(SPH, q)

    def x(self, q):
        self._apply1(PX, q)

    def y(self, q):
        self._apply1(PY, q)

    def z(self, q):
        self._apply1(PZ, q)

    def cx(self, c, t):
        idx = np.arange(2 ** self.n)
        mask = ((idx >> c) & 1) == 1
        perm = idx.copy()
        perm[mask] = idx[mask] ^ (1 << t)
        new = np.empty_like(self.psi)
        new[perm] = self.psi
        self.psi = new

    def prob_one(self, q) -> float:
        idx = np.arange(2 ** self.n)
        return float(np.sum(np.abs(self.psi[((idx >> q) & 1) == 1]) ** 2))

    def project(self, q, outcome):
        idx = np.arange(2 ** self.n)
        keep = ((idx >> q) & 1) == outcome
        self.psi = np.where(keep, self.psi, 0)
        nrm = np.linalg.norm(self.psi)
        self.psi /= nrm

    def expect(self, x, z, r) -> complex:
        """<psi| (-1)^r P(x,z) |psi>, applying the Pauli factor by factor (no 4^n matrix)."""
        phi = self.psi.copy()
        saved = self.psi
        self.psi = phi
        for j in range(self.n):
            if x[j] and z[j]:
                self.y(j)
            elif x[j]:
                self.x(j)
            elif z[j]:
                self.z(j)
        out = np.vdot(saved, self.psi) * (-1) ** int(r)
        self.psi = saved
        return out
