"""GPU tests of the continuous-batching server: admission by HBM budget and
slots, requests arriving while others run, and results that are the same
bits alone and in the mix (and match the oracle)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2304_06586_amd as pkg
    pkg.load_library()
    return pkg


def _mix(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nz = int(rng.integers(200, 6000))
        steps = int(rng.integers(1, 1500))
        beta = float(rng.uniform(-0.45, 0.45))
        kind = W.MATTER if rng.uniform() < 0.3 else W.MODULATION
        prec = W.F64 if rng.uniform() < 0.5 else W.F32
        st = ["slab", "random", "crystal", "uniform"][int(rng.integers(0, 4))]
        out.append(W.small_case(nz, steps, beta, kind=kind, precision=prec,
                                structure=st, seed=seed * 100 + i, nprobe=3))
    return out


def _same(a, b):
    for k in ("trace", "dft", "d", "b"):
        assert np.array_equal(a[k], b[k]), k


def test_served_equals_alone_under_a_tight_budget(P):
    probs = _mix(1, 14)
    alone = [P.gfdtd_solve(p) for p in probs]
    big = max(P.gfdtd_workspace_bytes(p) for p in probs)
    # room for only a few runs at a time: admission must wait for memory
    with P.Server(pool_bytes=3 * big + (8 << 20), max_slots=4) as srv:
        ids = [srv.submit(p, record_trace=True, keep_fields=True) for p in probs]
        done = {}
        max_live = 0
        for _ in range(100000):
            live, queued = srv.progress(max_blocks=3)
            max_live = max(max_live, live)
            for i, rid in enumerate(ids):
                if i not in done:
                    r = srv.poll(rid)
                    if r is not None:
                        done[i] = r
            if len(done) == len(ids):
                break
        assert len(done) == len(ids)
        assert 1 <= max_live <= 4
    for i, p in enumerate(probs):
        _same(done[i], alone[i])
        assert done[i]["status"] == 0


def test_requests_arriving_while_others_run(P):
    probs = _mix(2, 10)
    alone = [P.gfdtd_solve(p) for p in probs]
    with P.Server(pool_bytes=1 << 30, max_slots=64, block_steps=16) as srv:
        ids = {}
        done = {}
        pending = list(range(len(probs)))
        while pending or len(done) < len(probs):
            if pending:                        # one new arrival per round
                i = pending.pop(0)
                ids[i] = srv.submit(probs[i], record_trace=True, keep_fields=True)
            srv.progress(max_blocks=2)
            for i, rid in ids.items():
                if i not in done:
                    r = srv.poll(rid)
                    if r is not None:
                        done[i] = r
    for i, p in enumerate(probs):
        _same(done[i], alone[i])
        tol = 1e-12 if p.precision == W.F64 else 1e-5
        want = oracle.solve(p)
        num = np.linalg.norm(done[i]["trace"] - want["trace"])
        den = np.linalg.norm(want["trace"])
        assert num <= tol * den


def test_poll_not_ready_and_budget_errors(P):
    p = W.small_case(3000, 500, 0.3, seed=4)
    need = P.gfdtd_workspace_bytes(p)
    with P.Server(pool_bytes=need + (8 << 20), max_slots=2) as srv:
        rid = srv.submit(p, record_trace=True)
        assert srv.poll(rid) is None
        big = W.small_case(400000, 10, 0.3, seed=5)
        with pytest.raises(P.GfdtdError) as e:
            srv.submit(big)
        assert e.value.status == P.gfdtd.GFDTD_E_NOMEM
        while srv.poll(rid) is None:
            srv.progress(max_blocks=8)
    with pytest.raises(P.GfdtdError) as e:
        P.Server(pool_bytes=4096, max_slots=8)
    assert e.value.status == P.gfdtd.GFDTD_E_NOMEM


def test_zero_step_request(P):
    p = W.small_case(500, 0, 0.2, seed=6)
    import torch
    with P.Server(pool_bytes=64 << 20, max_slots=2) as srv:
        rid = srv.submit(p, record_trace=True, keep_fields=True)
        srv.progress(max_blocks=1)
        torch.cuda.synchronize()        # progress returns without waiting
        r = srv.poll(rid)
        assert r is not None and r["steps_done"] == 0
        assert np.all(r["d"] == 0)
