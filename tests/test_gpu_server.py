"""GPU tests of the continuous-batching server (stab_server_*): every request's records equal
the oracle's for that request alone, whatever else is resident and in whichever lane it runs;
admission by arena bytes; cancellation."""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_03092_amd import circuits as Cc

pytestmark = pytest.mark.gpu

LANES = {"batch": 1, "shared": 2}


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


def _drain(srv, seconds=120.0):
    out = []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        nf = srv.step()
        out += srv.poll()
        st = srv.stats()
        if st["queued"] == 0 and st["resident_requests"] == 0:
            return out + srv.poll()
        if nf == 0 and st["in_flight"] > 0:
            time.sleep(0.0005)
    raise AssertionError("server did not drain")


def _program(srv, circ, lane):
    p = srv.program(circ)
    if lane is not None:
        srv.set_lane(p, LANES[lane])
    return p


@pytest.mark.parametrize("lane", ["batch", "shared"])
def test_server_mixed_requests_match_oracle_alone_and_in_the_mix(stab, lane):
    say(f"[server] mixed requests, {lane} lane")
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
            progs[id(circ)] = _program(srv, circ, lane)
        ids.append(srv.submit(progs[id(circ)], shots, seed))
        if len(ids) % 4 == 0:
            srv.step()                      # later requests join while earlier ones run
    done = set(_drain(srv))
    assert done == set(ids)
    got = {rid: srv.result(rid, shots) for rid, (c, shots, seed) in zip(ids, reqs)}
    for rid, (circ, shots, seed) in zip(ids, reqs):
        want = O.run(circ, shots, seed)
        assert np.array_equal(got[rid], want), f"request {rid} (n={circ.n}, shots={shots})"
    # the same request alone on a fresh server, in the other lane too
    for other in LANES:
        alone = stab.Server(1 << 28)
        circ, shots, seed = reqs[5]
        rid = alone.submit(_program(alone, circ, other), shots, seed)
        _drain(alone)
        assert np.array_equal(alone.result(rid, shots), got[ids[5]]), other
        alone.close()
    srv.close()


def test_server_both_lanes_and_exact_t1t2_in_one_mix(stab):
    """Automatic lanes: Pauli-noise streams run shared, the exact T1/T2 stream runs batched; a
    d=25 request rides along with small ones."""
    say("[server] both lanes in one mix, d=25 included")
    d25 = Cc.surface_code_memory(25, 3, 1e-3)[0]
    d5 = Cc.surface_code_memory(5, 5, 3e-3)[0]
    t1t2 = Cc.surface_code_memory(3, 3, 1e-3, None, (1e-6, 20e-6, 20e-6))[0]
    srv = stab.Server(1 << 31)
    p25, p5, pt = srv.program(d25), srv.program(d5), srv.program(t1t2)
    reqs = [(pt, t1t2, 6, 9), (p25, d25, 3, 21), (p5, d5, 17, 4), (pt, t1t2, 2, 33), (p5, d5, 64, 8),
            (p25, d25, 1, 5), (p5, d5, 1, 77)]
    ids = []
    for k, (p, c, shots, seed) in enumerate(reqs):
        ids.append(srv.submit(p, shots, seed))
        if k == 2:
            srv.step()
            st = srv.stats()
            assert st["in_flight"] >= 1 and st["steps"] == 1     # both lanes busy at once
    with pytest.raises(stab.StabError):
        srv.set_lane(pt, 2)                  # T1T2 changes x|z shot by shot
    assert set(_drain(srv)) == set(ids)
    for rid, (p, c, shots, seed) in zip(ids, reqs):
        assert np.array_equal(srv.result(rid, shots), O.run(c, shots, seed)), f"request {rid} (n={c.n})"
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


@pytest.mark.parametrize("lane", ["batch", "shared"])
def test_server_admission_by_bytes(stab, lane):
    say(f"[server] admission by bytes, {lane} lane")
    circ = Cc.surface_code_memory(5, 5, 2e-3)[0]
    probe = stab.Server(1 << 20)
    per = probe.request_bytes(_program(probe, circ, lane), 8)
    probe.close()
    srv = stab.Server(2 * per + 4096)          # room for two requests at a time
    prog = _program(srv, circ, lane)
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


@pytest.mark.parametrize("lane", ["batch", "shared"])
def test_server_cancel(stab, lane):
    say(f"[server] cancellation, {lane} lane")
    circ = Cc.surface_code_memory(7, 7, 2e-3)[0]
    per = None
    srv = stab.Server(1 << 30)
    prog = _program(srv, circ, lane)
    per = srv.request_bytes(prog, 10)
    srv.close()
    srv = stab.Server(3 * per + 4096)          # three resident, the rest queued
    prog = _program(srv, circ, lane)
    ids = [srv.submit(prog, 10, 500 + i) for i in range(6)]
    srv.cancel(ids[5])                          # queued
    srv.step()
    srv.cancel(ids[1])                          # resident
    with pytest.raises(stab.StabError):
        srv.cancel(ids[1])                      # twice
    done = _drain(srv)
    assert set(done) == {ids[0], ids[2], ids[3], ids[4]}
    srv.cancel(ids[4])                          # finished, not taken
    with pytest.raises(stab.StabError):
        srv.result(ids[4], 10)
    for i in (0, 2, 3):
        assert np.array_equal(srv.result(ids[i], 10), O.run(circ, 10, 500 + i))
    st = srv.stats()
    assert st["cancelled"] == 3 and st["bytes_in_use"] == 0 and st["in_flight"] == 0
    with pytest.raises(stab.StabError):
        srv.cancel(12345)
    srv.close()


@pytest.mark.parametrize("lane", ["batch", "shared"])
def test_server_edge_requests(stab, lane):
    say(f"[server] edge requests, {lane} lane")
    srv = stab.Server(1 << 26)
    empty = Cc.Circuit(n=4)
    gates_only = Cc.Circuit(n=70)
    gates_only.gate(Cc.H, list(range(70)))
    meas_only = Cc.Circuit(n=9)
    meas_only.append(Cc.MR, list(range(9)))
    meas_only.append(Cc.M, [0, 0, 3])
    ids = [(srv.submit(_program(srv, c, lane), s, 7), c, s) for c, s in ((empty, 3), (gates_only, 2), (meas_only, 5))]
    _drain(srv)
    for rid, c, s in ids:
        assert np.array_equal(srv.result(rid, s), O.run(c, s, 7)[:, :c.num_measurements()])
    srv.close()
