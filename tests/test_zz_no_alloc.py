"""stab_sample_noalloc against stab_sample through the C ABI, bit for bit: two calls in a row,
the second with a smaller input (the static scratch keeps the first call's contents), plus the
oracle on the smaller case.  The first call's noise does not fit the scratch in one draw, so it
also runs the segment-by-segment draws."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import oracle as O
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


def _same(got, want, what):
    assert got.shape == want.shape, what
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert len(bad) == 0, f"{what}: record differs in shots {bad[:10]}"


def test_noalloc_matches_sample_two_calls(stab):
    import torch

    big, _ = Cc.surface_code_memory(25, 25, 1e-3)
    small = Cc.random_clifford_measure(70, 40, seed=11, noise=1e-2)
    # one caller-owned tableau buffer, large enough for both calls
    nbytes = max(stab.tableau_bytes(big.n, 100, "shared"), stab.tableau_bytes(small.n, 24, "full"))
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")

    say("case 1: surface d=25, 25 rounds, p=1e-3, 100 shots, shared, seed 2")
    got1 = stab.sample_noalloc(big, 100, 2, mode="shared", buf=buf)
    torch.cuda.synchronize()
    want1, _ = stab.sample(big, 100, 2, mode="shared")
    _same(got1, want1, "d=25 shared")

    say("case 2: random Clifford+M/MR/R n=70 depth 40, 24 shots, full, seed 5")
    got2 = stab.sample_noalloc(small, 24, 5, mode="full", buf=buf)
    torch.cuda.synchronize()
    want2, _ = stab.sample(small, 24, 5, mode="full")
    _same(got2, want2, "n=70 full")
    _same(got2, O.run(small, 24, 5), "n=70 full vs oracle")


def test_noalloc_rejects_oversize_before_the_device(stab):
    wide = Cc.Circuit(stab.max_qubits())
    wide.append(Cc.M, range(wide.n))
    with pytest.raises(stab.StabError) as e:
        stab.sample_noalloc(wide, 1, 0)
    assert e.value.code == stab.ERANGE
