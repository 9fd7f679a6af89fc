"""Seeded input generators: determinism, chunk independence, value classes."""
import numpy as np

import workloads as W


def test_splitmix_counter_matches_sequential():
    """Draw k of the counter form equals output k of the sequential generator."""
    seed = 0x2108047900000001
    M = (1 << 64) - 1
    state, seq = seed, []
    for _ in range(16):
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        seq.append(z ^ (z >> 31))
    assert W.draws(seed, np.arange(16)).tolist() == seq


def test_deterministic_and_chunk_independent():
    a = W.c2_mr64(5000)
    assert np.array_equal(a, W.c2_mr64(5000))
    assert np.array_equal(a[1234:2345], W.c2_mr64(2345 - 1234, start=1234))
    c = W.c3_mixed(3000)
    assert np.array_equal(c[100:200], W.c3_mixed(100, start=100))
    assert W.digest(a) == W.digest(W.c2_mr64(5000))


def test_value_classes():
    c1 = W.c1_uniform20()
    assert c1.size == 65536 and int(c1.max()) < (1 << 20)
    c2 = W.c2_mr64(1 << 16)
    assert int(c2.min()) >= (1 << 49)
    odd = float((c2 & np.uint64(1)).mean())
    assert 0.73 < odd < 0.77  # half forced odd, the other half odd by chance
    c3 = W.c3_mixed(1 << 18)
    cher = set(W.chernick_values().tolist())
    frac_ch = np.isin(c3, np.array(sorted(cher), dtype=np.uint64)).mean()
    frac_fx = np.isin(c3, W.C3_FIXED).mean()
    assert 0.045 < frac_ch < 0.056 and 0.008 < frac_fx < 0.013
    assert int(c3.min()) >= 1
    bl = np.floor(np.log2(c3.astype(np.float64))).astype(int)
    counts = np.bincount(bl, minlength=64)
    assert counts[:60].min() > 0.6 * counts[:60].mean()


def test_batched_and_requests_shapes():
    arrs = W.c4_batched(256)
    assert len(arrs) == 256
    lens = [a.size for a, _ in arrs]
    assert min(lens) >= 1 and max(lens) <= 1 << 16
    bounds = [(0, 1 << 20), (1 << 20, 1 << 32), (1 << 32, 1 << 49), (1 << 49, 1 << 64)]
    for a, c in arrs:
        lo, hi = bounds[c]
        assert int(a.min()) >= lo and int(a.max()) < hi
    reqs = W.c5_requests(50, qps=100.0)
    ts = [t for t, _, _ in reqs]
    assert ts == sorted(ts) and all(1 <= r.size <= 1 << 20 for _, r, _ in reqs)


def test_odd_band_octaves():
    """Odd values inside one octave, spread over all of it, chunk independent."""
    for bits in (2, 33, 40, 64):
        a = W.odd_band(20000, bits)
        lo, hi = 1 << (bits - 1), 1 << bits
        assert int(a.min()) >= lo and int(a.max()) < hi, bits
        assert bool(((a & np.uint64(1)) == 1).all()), bits
    a = W.odd_band(20000, 40)
    frac = (a.astype(np.float64) - 2.0 ** 39) / 2.0 ** 39
    counts = np.histogram(frac, bins=16, range=(0, 1))[0]
    assert counts.min() > 0.8 * counts.mean()
    assert np.array_equal(a[500:900], W.odd_band(400, 40, start=500))
    assert not np.array_equal(W.odd_band(100, 39), W.odd_band(100, 40) >> np.uint64(1))
