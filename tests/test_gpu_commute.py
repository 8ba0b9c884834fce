"""GPU parity of stab_commute (Pauli-string commutation, group-wise and qubit-wise) against
the oracle's definition-level matrices, bit for bit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import commute as OC
from paper_2507_03092_amd import circuits as Cc

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stab():
    import torch

    assert torch.cuda.is_available(), "no GPU"
    from paper_2507_03092_amd import stab as S

    S.lib()
    return S


@pytest.mark.parametrize("n", [1, 63, 64, 65, 130, 256, 1000])
@pytest.mark.parametrize("na,nb", [(1, 1), (63, 65), (64, 64), (200, 129)])
def test_commute_random(stab, n, na, nb):
    say(f"commute n={n} na={na} nb={nb}")
    ax, az = Cc.random_paulis(na, n, (1, n, na))
    bx, bz = Cc.random_paulis(nb, n, (2, n, nb))
    gc, qwc = stab.commute(stab.pack_paulis(ax, az), stab.pack_paulis(bx, bz), n)
    wg, wq = OC.commute_matrix(ax, az, bx, bz)
    assert np.array_equal(gc, wg)
    assert np.array_equal(qwc, wq)


def test_commute_structured(stab):
    # identities, single-qubit strings and a string against itself
    n = 70
    x = np.zeros((4 * n + 1, n), dtype=np.uint8)
    z = np.zeros_like(x)
    for q in range(n):
        x[1 + 4 * q, q] = 1                   # X_q
        z[2 + 4 * q, q] = 1                   # Z_q
        x[3 + 4 * q, q] = z[3 + 4 * q, q] = 1  # Y_q
        x[4 + 4 * q, :q + 1] = 1              # X...X on 0..q
    P = stab.pack_paulis(x, z)
    gc, qwc = stab.commute(P, P, n)
    wg, wq = OC.commute_matrix(x, z, x, z)
    assert np.array_equal(gc, wg) and np.array_equal(qwc, wq)
    assert not gc[0].any() and not qwc[0].any()
    assert np.array_equal(gc, gc.T)


def test_commute_outputs_optional_and_errors(stab):
    import torch
    import ctypes as C

    ax, az = Cc.random_paulis(100, 90, 3)
    A = stab.pack_paulis(ax, az)
    gc, qwc = stab.commute(A, A, 90, qubitwise=False)
    assert qwc is None and np.array_equal(gc, OC.commute_matrix(ax, az, ax, az)[0])
    L = stab.lib()
    t = torch.zeros(8, dtype=torch.int64, device="cuda")
    p = C.c_void_p(t.data_ptr())
    assert L.stab_commute(p, 1, p, 1, 64, None, None, None) == stab.EINVAL
    assert L.stab_commute(p, 1, p, 1, 0, p, None, None) == stab.EINVAL
    assert L.stab_commute(None, 1, p, 1, 64, p, None, None) == stab.EINVAL
    assert L.stab_commute(p, 0, p, 1, 64, p, None, None) == stab.OK


def test_commute_full_size_sampled(stab):
    """The benchmark's 32768 x 32768 strings on 256 qubits, in the benchmark's launch; the
    oracle checks 48 random rows against every column."""
    import torch

    w = Cc.COMMUTE
    x, z = Cc.random_paulis(w["m"], w["n"], w["seed"])
    P = stab.pack_paulis(x, z)
    tP = torch.from_numpy(P.view(np.int64)).cuda()
    gc, qwc = stab.commute(tP, tP, w["n"])
    rows = np.random.default_rng(0).choice(w["m"], size=48, replace=False)
    wg, wq = OC.commute_matrix(x[rows], z[rows], x, z)
    assert np.array_equal(gc[rows], wg) and np.array_equal(qwc[rows], wq)
    assert np.array_equal(gc[rows][:, rows], gc[rows][:, rows].T)
