"""GPU tests of the continuous-batching server (stab_server_*): every request's records equal
the oracle's for that request alone, whatever else is resident; admission by arena bytes."""
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


def _drain(srv, limit=100000):
    out = []
    for _ in range(limit):
        srv.step()
        out += srv.poll()
        st = srv.stats()
        if st["queued"] == 0 and st["resident_requests"] == 0:
            return out + srv.poll()
    raise AssertionError("server did not drain")


def test_server_mixed_requests_match_oracle_alone_and_in_the_mix(stab):
    circs = {d: Cc.surface_code_memory(d, d, 3e-3)[0] for d in (3, 5, 7)}
    rnd = Cc.random_clifford_measure(20, depth=8, seed=3, p_meas=0.3, noise=0.02)
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(14):
        kind = int(rng.integers(0, 4))
        circ = rnd if kind == 3 else circs[(3, 5, 7)[kind]]
        reqs.append((circ, int(rng.integers(1, 12)), int(rng.integers(0, 2 ** 40))))
    srv = stab.Server(1 << 30)
    progs = {}
    ids = []
    for circ, shots, seed in reqs:
        if id(circ) not in progs:
            progs[id(circ)] = srv.program(circ)
        ids.append(srv.submit(progs[id(circ)], shots, seed))
        if len(ids) % 4 == 0:
            srv.step()                      # later requests join while earlier ones run
    done = set(_drain(srv)) | set()
    got = {rid: srv.result(rid, shots) for rid, (c, shots, seed) in zip(ids, reqs)}
    for rid, (circ, shots, seed) in zip(ids, reqs):
        want = O.run(circ, shots, seed)
        assert np.array_equal(got[rid], want), f"request {rid} (n={circ.n}, shots={shots})"
    # the same request alone on a fresh server
    alone = stab.Server(1 << 28)
    circ, shots, seed = reqs[5]
    rid = alone.submit(alone.program(circ), shots, seed)
    _drain(alone)
    assert np.array_equal(alone.result(rid, shots), got[ids[5]])
    srv.close()
    alone.close()


def test_server_admission_by_bytes(stab):
    circ = Cc.surface_code_memory(5, 5, 2e-3)[0]
    probe = stab.Server(1 << 20)
    per = probe.request_bytes(probe.program(circ), 8)
    probe.close()
    srv = stab.Server(2 * per + 4096)          # room for two requests at a time
    prog = srv.program(circ)
    ids = [srv.submit(prog, 8, 100 + i) for i in range(5)]
    srv.step()
    st = srv.stats()
    assert st["resident_requests"] == 2 and st["queued"] == 3 and st["bytes_in_use"] <= st["arena_bytes"]
    _drain(srv)
    for i, rid in enumerate(ids):
        assert np.array_equal(srv.result(rid, 8), O.run(circ, 8, 100 + i))
    with pytest.raises(stab.StabError):
        srv.submit(prog, 100, 1)                # larger than the whole arena
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_server_edge_requests(stab):
    srv = stab.Server(1 << 26)
    empty = Cc.Circuit(n=4)
    gates_only = Cc.Circuit(n=70)
    gates_only.gate(Cc.H, list(range(70)))
    meas_only = Cc.Circuit(n=9)
    meas_only.append(Cc.MR, list(range(9)))
    meas_only.append(Cc.M, [0, 0, 3])
    ids = [(srv.submit(srv.program(c), s, 7), c, s) for c, s in ((empty, 3), (gates_only, 2), (meas_only, 5))]
    _drain(srv)
    for rid, c, s in ids:
        assert np.array_equal(srv.result(rid, s), O.run(c, s, 7)[:, :c.num_measurements()])
    srv.close()
