"""GPU parity of the batched (graph-replayed, persistent) entry point: equal to
the oracle and to per-array plain calls, byte for byte, on every replay."""
import os

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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def test_batched_c4_against_oracle_and_plain(isp, oracle_table):
    arrs = W.c4_batched()
    flat = np.concatenate([a for a, _ in arrs])
    exp, _ = oracle.isprime_array(flat, nthreads=NTHREADS, use_table=True)
    dev = [to_dev(a) for a, _ in arrs]
    outs = isp.isprime_batched(dev)
    torch.cuda.synchronize()
    got = np.concatenate([o.cpu().numpy().astype(np.uint8) for o in outs])
    assert np.array_equal(got, exp), np.nonzero(got != exp)[0][:10]
    # plain calls, one per array, give the same bytes
    plain = [isp.isprime(d) for d in dev[:256]]
    torch.cuda.synchronize()
    for p, o in zip(plain, outs[:256]):
        assert torch.equal(p, o)


def test_batched_replays_and_eager_work_between(isp):
    """The graph is replayed; every replay must equal the eager result, with
    the program's own work and synchronisations between replays."""
    rng = np.random.default_rng(1)
    arrays = [W.c3_mixed(int(L), start=int(s)) for L, s in
              zip(rng.integers(1, 20000, size=64), rng.integers(0, 1 << 30, size=64))]
    exp = [oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)[0] for a in arrays]
    dev = [to_dev(a) for a in arrays]
    for rep in range(5):
        outs = isp.isprime_batched(dev)
        torch.cuda.synchronize()
        junk = isp.isprime(dev[rep])  # eager plain work between replays
        torch.cuda.synchronize()
        assert np.array_equal(junk.cpu().numpy().astype(np.uint8), exp[rep])
        for o, e in zip(outs, exp):
            assert np.array_equal(o.cpu().numpy().astype(np.uint8), e), rep


def test_batched_back_to_back_calls(isp):
    """Calls issued back to back with no synchronisation between them (the
    library alternates two descriptor buffers and graphs): every call's
    outputs are its own, for two input sets taken in turn and for a prepared
    Batch run repeatedly."""
    rng = np.random.default_rng(3)
    sets = []
    for _ in range(2):
        arrays = [W.c3_mixed(int(L), start=int(st)) for L, st in
                  zip(rng.integers(1, 5000, size=40), rng.integers(0, 1 << 30, size=40))]
        sets.append(([to_dev(a) for a in arrays],
                     [oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)[0] for a in arrays]))
    runs = []
    for r in range(6):
        dev, exp = sets[r % 2]
        outs = [torch.full((d.numel(),), 7, dtype=torch.uint8, device="cuda") for d in dev]
        isp.Batch(dev, outs).run()
        runs.append((outs, exp))
    prepared = isp.Batch(sets[0][0])
    for _ in range(3):
        prepared.run()
    torch.cuda.synchronize()
    runs.append((prepared.outs, sets[0][1]))
    for r, (outs, exp) in enumerate(runs):
        for o, e in zip(outs, exp):
            assert np.array_equal(o.cpu().numpy().astype(np.uint8), e), r


def test_batched_growing_and_empty_arrays(isp):
    rng = np.random.default_rng(2)
    for k in (1, 3, 1500, 5000):
        lens = rng.integers(0, 300, size=k)
        lens[::7] = 0
        arrays = [W.c2_mr64(int(L), start=int(i) * 1000) for i, L in enumerate(lens)]
        dev = [to_dev(a) for a in arrays]
        outs = isp.isprime_batched(dev)
        torch.cuda.synchronize()
        flat = np.concatenate(arrays) if arrays else np.zeros(0, np.uint64)
        exp, _ = oracle.isprime_array(flat, nthreads=NTHREADS, use_table=False)
        got = np.concatenate([o.cpu().numpy().astype(np.uint8) for o in outs])
        assert np.array_equal(got, exp), k


def test_batched_grids(isp):
    arrays = [W.c3_mixed(L, start=L) for L in (1, 255, 256, 257, 70000, 3, 0, 5)]
    exp = [oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)[0] for a in arrays]
    dev = [to_dev(a) for a in arrays]
    for cfg in (dict(classify_blocks_per_cu=1), dict(classify_blocks_per_cu=16, classify_ept=1),
                dict(mr_blocks_per_cu=1, mr_block=64), dict(sort_survivors=-1)):
        prev = isp.set_config(**cfg)
        try:
            outs = isp.isprime_batched(dev)
            torch.cuda.synchronize()
        finally:
            isp.set_config(**prev)
        for o, e in zip(outs, exp):
            assert np.array_equal(o.cpu().numpy().astype(np.uint8), e), cfg


def test_batched_invalid(isp):
    import ctypes
    L = isp.lib()
    NP = ctypes.c_uint64 * 1
    z = NP(0)
    five = NP(5)
    assert L.isprime_u64_batched(ctypes.cast(z, ctypes.c_void_p), ctypes.cast(z, ctypes.c_void_p),
                                 ctypes.cast(five, ctypes.c_void_p), 1, None) == isp.ISP_EINVAL
    assert L.isprime_u64_batched(None, None, None, 0, None) == isp.ISP_OK


def test_offsets_form_against_oracle(isp):
    """The arrays of C4 laid end to end in one buffer with an offsets table
    (on the device, then on the host): equal to the oracle; bytes outside
    [offsets[0], offsets[-1]) untouched; decreasing offsets refused."""
    arrs = [a for a, _ in W.c4_batched(num_arrays=512)]
    flat = np.concatenate(arrs)
    exp, _ = oracle.isprime_array(flat, nthreads=NTHREADS, use_table=False)
    offs = np.concatenate([[0], np.cumsum([a.size for a in arrs])]).astype(np.int64)
    dev = to_dev(np.concatenate([flat, np.array([2, 3], dtype=np.uint64)]))  # 2 extra at the end
    for where in ("cuda", "cpu"):
        out = torch.full((dev.numel(),), 7, dtype=torch.uint8, device="cuda")
        isp.isprime_batched_offsets(dev, torch.from_numpy(offs).to(where), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got[:flat.size], exp), where
        assert got[flat.size:].tolist() == [7, 7]  # outside the arrays: not written
    # a sub-range: arrays 10 .. 20 only
    out = torch.full((dev.numel(),), 7, dtype=torch.uint8, device="cuda")
    sub = torch.from_numpy(offs[10:21].copy()).cuda()
    isp.isprime_batched_offsets(dev, sub, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    lo, hi = offs[10], offs[20]
    assert np.array_equal(got[lo:hi], exp[lo:hi])
    assert (got[:lo] == 7).all() and (got[hi:] == 7).all()
    bad = torch.tensor([0, 5, 3], dtype=torch.int64, device="cuda")
    with pytest.raises(isp.IsprimeError) as e:
        isp.isprime_batched_offsets(dev, bad, out)
    assert e.value.status == isp.ISP_EINVAL
