"""GPU parity of the served form: every request's result equals the oracle's
and the plain isprime_u64 result, whether it runs alone or packed with other
requests (tolerance: zero mismatching bytes)."""
import os
import threading

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def isp():
    import paper_2108_04791_amd as isp
    isp.init()
    return isp


def request_mix(k, max_len, seed):
    rng = np.random.default_rng(seed)
    lens = np.floor(np.exp2(rng.random(k) * np.log2(max_len + 1))).astype(int)
    reqs = []
    for i, L in enumerate(lens):
        cls = int(rng.integers(0, 4))
        idx = np.arange(i * max_len, i * max_len + L, dtype=np.uint64)
        reqs.append(W.class_values(seed, idx, cls))
    return reqs


def test_served_mix_equals_oracle_and_alone(isp):
    reqs = request_mix(120, 1 << 15, 5)
    exp = [oracle.isprime_array(r, nthreads=NTHREADS, use_table=True)[0] for r in reqs]
    # in a mix: everything submitted at once, packed into shared batches
    with isp.Server(max_inflight=3, max_batch_elems=1 << 16) as srv:
        outs = [np.zeros(r.size, np.uint8) for r in reqs]
        tickets = [srv.submit(r, o) for r, o in zip(reqs, outs)]
        for t in tickets:
            srv.wait(t)
    # alone: one request in the server at a time
    with isp.Server(max_inflight=1) as srv:
        alone = []
        for r in reqs:
            o = np.zeros(r.size, np.uint8)
            srv.wait(srv.submit(r, o))
            alone.append(o)
    for r, o, a, e in zip(reqs, outs, alone, exp):
        assert np.array_equal(o, e)
        assert np.array_equal(a, o)
    # and the plain device call on the same bytes
    for r, o in zip(reqs[:20], outs[:20]):
        t = torch.from_numpy(r.view(np.int64)).cuda()
        p = isp.isprime(t).cpu().numpy().astype(np.uint8)
        assert np.array_equal(p, o)


def test_served_split_request_and_threads(isp):
    big = W.c3_mixed(300001, start=77)
    exp_big = oracle.isprime_array(big, nthreads=NTHREADS, use_table=True)[0]
    with isp.Server(max_inflight=2, max_batch_elems=65536, mem_budget_bytes=9 * 200000) as srv:
        out = np.zeros(big.size, np.uint8)
        t = srv.submit(big, out)  # larger than the budget: admitted alone, 5 pieces
        errors = []

        def client(seed):
            for r in request_mix(15, 4096, seed):
                o = np.zeros(r.size, np.uint8)
                srv.wait(srv.submit(r, o))
                if not np.array_equal(o, oracle.isprime_array(r, nthreads=2, use_table=True)[0]):
                    errors.append(seed)

        th = [threading.Thread(target=client, args=(s,)) for s in (11, 12, 13, 14)]
        for x in th:
            x.start()
        srv.wait(t)
        for x in th:
            x.join()
        assert not errors
        assert np.array_equal(out, exp_big)


def test_served_at_the_benchmarked_configuration(isp):
    """The server as the benchmark runs it (the defaults: 8 slots of 2^18
    elements, requests of up to 2^20 split over several) on the first 300 requests of the
    benchmark's own stream (lengths log-uniform in [1, 2^20]): every result
    equals the oracle's, submitted all at once (packed into shared batches)
    and one at a time."""
    reqs = [r for _, r, _ in W.c5_requests(300, qps=1.0)]
    assert max(r.size for r in reqs) > (1 << 19)
    exp = [oracle.isprime_array(r, nthreads=NTHREADS, use_table=True)[0] for r in reqs]
    with isp.Server() as srv:
        # the fixed footprint: 8 slots, each a workspace for 2^18 elements
        # and 9 pinned bytes per element
        dev_b, pin_b = srv.footprint()
        assert dev_b == 8 * isp.workspace_bytes(1 << 18) and pin_b == 8 * 9 * (1 << 18)
        mixed = [np.full(r.size, 2, np.uint8) for r in reqs]
        tickets = [srv.submit(r, o) for r, o in zip(reqs, mixed)]
        for t in tickets:
            srv.wait(t)
        alone = []
        for r in reqs[:60]:
            o = np.full(r.size, 2, np.uint8)
            srv.wait(srv.submit(r, o))
            alone.append(o)
    for i, (o, e) in enumerate(zip(mixed, exp)):
        bad = np.nonzero(o != e)[0]
        assert bad.size == 0, "request %d (%d values): mismatch at %s" % (i, e.size, bad[:10].tolist())
    for o, m in zip(alone, mixed):
        assert np.array_equal(o, m)

