"""The request server's host logic, exercised without a GPU: test mode runs
each batch on the server's own thread and writes n & 1 (a stand-in that makes
routing errors visible), with injected delays and failures.  Checks
admission by memory, splitting into pieces, packing many requests per batch,
ordering, error isolation, and the ticket API."""
import threading
import time

import numpy as np
import pytest

import paper_2108_04791_amd as isp


def rand_req(rng, n):
    return rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=n, dtype=np.uint64)


def test_results_routed_to_their_requests():
    rng = np.random.default_rng(0)
    with isp.Server(test_mode=1, max_batch_elems=1000, max_inflight=2) as srv:
        reqs = [rand_req(rng, int(k)) for k in rng.integers(0, 3000, size=60)]
        outs = [np.full(r.size, 7, dtype=np.uint8) for r in reqs]
        tickets = [srv.submit(r, o) for r, o in zip(reqs, outs)]
        for t in tickets:
            srv.wait(t)
        for r, o in zip(reqs, outs):
            assert np.array_equal(o, (r & np.uint64(1)).astype(np.uint8))


def test_large_batches_staged_by_several_threads():
    """Batches above a few hundred KB are staged by the server's copy
    threads in byte ranges that cut across pieces: every request, split
    over pieces and packed with others, still gets exactly its own bytes."""
    rng = np.random.default_rng(4)
    with isp.Server(test_mode=1, max_batch_elems=(1 << 20) + 12345, max_inflight=3) as srv:
        lens = [int(k) for k in rng.integers(1, 700000, size=24)] + [3 << 20, 1, 999999]
        reqs = [rand_req(rng, k) for k in lens]
        outs = [np.full(r.size, 7, dtype=np.uint8) for r in reqs]
        tickets = [srv.submit(r, o) for r, o in zip(reqs, outs)]
        for t in tickets:
            srv.wait(t)
        for r, o in zip(reqs, outs):
            assert np.array_equal(o, (r & np.uint64(1)).astype(np.uint8))


def test_ticket_api():
    with isp.Server(test_mode=1, test_delay_us=20000) as srv:
        a = np.arange(10, dtype=np.uint64)
        o = np.zeros(10, dtype=np.uint8)
        t = srv.submit(a, o)
        assert srv.poll(t) is False
        with pytest.raises(isp.IsprimeError) as e:
            srv.wait(t, timeout_us=100)
        assert e.value.status == isp.ISP_ETIMEDOUT
        srv.wait(t)
        with pytest.raises(isp.IsprimeError) as e:
            srv.poll(t)  # consumed by wait
        assert e.value.status == isp.ISP_ENOENT
        t0 = srv.submit(np.zeros(0, np.uint64), np.zeros(0, np.uint8))
        assert srv.poll(t0) is True
        srv.wait(t0)


def test_admission_refuses_when_full_and_nonblocking():
    budget = 9 * 1000
    with isp.Server(test_mode=1, mem_budget_bytes=budget, block_on_full=False,
                    test_delay_us=50000) as srv:
        a = np.arange(800, dtype=np.uint64)
        oa = np.zeros(800, np.uint8)
        ta = srv.submit(a, oa)
        b = np.arange(300, dtype=np.uint64)
        ob = np.zeros(300, np.uint8)
        with pytest.raises(isp.IsprimeError) as e:
            srv.submit(b, ob)
        assert e.value.status == isp.ISP_EBUSY
        srv.wait(ta)
        tb = srv.submit(b, ob)  # budget released
        srv.wait(tb)
        assert np.array_equal(ob, (b & np.uint64(1)).astype(np.uint8))
        # larger than the whole budget: admitted when nothing else holds any
        c = np.arange(5000, dtype=np.uint64)
        oc = np.zeros(5000, np.uint8)
        srv.wait(srv.submit(c, oc))
        assert np.array_equal(oc, (c & np.uint64(1)).astype(np.uint8))


def test_admission_blocks_until_space():
    budget = 9 * 2000
    with isp.Server(test_mode=1, mem_budget_bytes=budget, block_on_full=True,
                    test_delay_us=5000, max_batch_elems=500) as srv:
        rng = np.random.default_rng(1)
        reqs = [rand_req(rng, 900) for _ in range(12)]
        outs = [np.zeros(900, np.uint8) for _ in reqs]
        t0 = time.perf_counter()
        tickets = [srv.submit(r, o) for r, o in zip(reqs, outs)]  # blocks as needed
        for t in tickets:
            srv.wait(t)
        assert time.perf_counter() - t0 > 0.01
        for r, o in zip(reqs, outs):
            assert np.array_equal(o, (r & np.uint64(1)).astype(np.uint8))


def test_failures_only_fail_their_batch():
    # one request per batch (max_batch_reqs=1), every 3rd batch fails
    with isp.Server(test_mode=1, test_fail_every=3, max_batch_reqs=1, max_inflight=1) as srv:
        reqs = [np.arange(i, i + 50, dtype=np.uint64) for i in range(9)]
        outs = [np.zeros(50, np.uint8) for _ in reqs]
        tickets = [srv.submit(r, o) for r, o in zip(reqs, outs)]
        status = []
        for t in tickets:
            try:
                srv.wait(t)
                status.append(0)
            except isp.IsprimeError as e:
                status.append(e.status)
        assert status == [0, 0, isp.ISP_EDEVICE] * 3
        for r, o, st in zip(reqs, outs, status):
            if st == 0:
                assert np.array_equal(o, (r & np.uint64(1)).astype(np.uint8))


def test_split_request_fails_if_any_piece_fails():
    with isp.Server(test_mode=1, test_fail_every=2, max_batch_elems=100, max_batch_reqs=1,
                    max_inflight=1) as srv:
        a = np.arange(350, dtype=np.uint64)  # 4 pieces, the 2nd and 4th fail
        with pytest.raises(isp.IsprimeError) as e:
            srv.wait(srv.submit(a, np.zeros(350, np.uint8)))
        assert e.value.status == isp.ISP_EDEVICE


def test_many_client_threads():
    rng = np.random.default_rng(2)
    with isp.Server(test_mode=1, max_batch_elems=4096, max_inflight=3,
                    mem_budget_bytes=9 * 20000) as srv:
        errors = []

        def client(seed):
            r = np.random.default_rng(seed)
            for _ in range(40):
                a = rand_req(r, int(r.integers(1, 3000)))
                o = np.zeros(a.size, np.uint8)
                srv.wait(srv.submit(a, o))
                if not np.array_equal(o, (a & np.uint64(1)).astype(np.uint8)):
                    errors.append(seed)

        th = [threading.Thread(target=client, args=(int(s),)) for s in rng.integers(0, 1 << 30, 6)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors


def test_destroy_finishes_queued_work():
    srv = isp.Server(test_mode=1, test_delay_us=2000, max_batch_reqs=2)
    reqs = [np.arange(i * 100, i * 100 + 100, dtype=np.uint64) for i in range(10)]
    outs = [np.zeros(100, np.uint8) for _ in reqs]
    for r, o in zip(reqs, outs):
        srv.submit(r, o)
    srv.close()  # drains
    for r, o in zip(reqs, outs):
        assert np.array_equal(o, (r & np.uint64(1)).astype(np.uint8))


def test_bad_arguments():
    with pytest.raises(isp.IsprimeError):
        isp.Server(test_mode=1, max_inflight=9)
    with pytest.raises(isp.IsprimeError):
        isp.Server(test_mode=2)
    with isp.Server(test_mode=1) as srv:
        with pytest.raises(TypeError):
            srv.submit(np.zeros(3, np.int32), np.zeros(3, np.uint8))
        assert isp.lib().isp_submit(srv._h, None, None, 5, None) == isp.ISP_EINVAL


def test_submit_rejects_impossible_lengths():
    """A length whose byte count cannot be represented is refused before
    anything is queued (the pointers are never read)."""
    import ctypes
    with isp.Server(test_mode=1, max_batch_elems=1000) as srv:
        t = ctypes.c_uint64()
        for n in (1 << 61, (1 << 64) - 1):
            st = isp.lib().isp_submit(srv._h, ctypes.c_void_p(8), ctypes.c_void_p(8), n,
                                      ctypes.byref(t))
            assert st == isp.ISP_EINVAL, n
        r = np.arange(5, dtype=np.uint64)
        o = np.zeros(5, dtype=np.uint8)
        srv.wait(srv.submit(r, o))
        assert np.array_equal(o, (r & np.uint64(1)).astype(np.uint8))
