"""CPU-side checks of the C ABI library: it loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "isprime.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*\b((?:isp|isprime)_[a-z_0-9]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def isp():
    import paper_2108_04791_amd as isp
    if not os.path.exists(isp.LIB_PATH):
        from paper_2108_04791_amd import _build
        _build.build()
    return isp


def test_header_parses():
    names = declared_functions()
    for n in ("isprime_u64", "isprime_u64_batched", "isp_init", "isp_server_create"):
        assert n in names


def test_library_exports_every_declared_symbol(isp):
    L = ctypes.CDLL(isp.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(isp.SIGNATURES)


def test_argument_errors_without_device(isp):
    L = isp.lib()
    assert L.isprime_u64(None, None, 0, None) == isp.ISP_OK
    assert L.isprime_u64(None, None, 7, None) == isp.ISP_EINVAL
    assert L.isp_montmul_u64(None, None, None, None, 3, None) == isp.ISP_EINVAL
    assert L.isp_init(-1) == isp.ISP_EINVAL
    assert L.isprime_u64_batched(None, None, None, 0, None) == isp.ISP_OK
    # more than 2^30 elements in one batched call, also through a wrapping sum
    ptrs = (ctypes.c_void_p * 2)(8, 8)
    for lens in ((1 << 30, 1), ((1 << 64) - 1, 2), (1 << 63, 1 << 63)):
        ls = (ctypes.c_uint64 * 2)(*lens)
        assert L.isprime_u64_batched(ptrs, ptrs, ls, 2, None) == isp.ISP_EINVAL, lens
    # the allocation-free entry point refuses before any HIP call
    cap = L.isp_noalloc_max_len()
    assert cap == 1 << 20
    assert L.isprime_u64_noalloc(None, None, 0, None) == isp.ISP_OK
    assert L.isprime_u64_noalloc(None, None, 5, None) == isp.ISP_EINVAL
    assert L.isprime_u64_noalloc(8, 8, cap + 1, None) == isp.ISP_ERANGE
    assert "isp_init" in L.isp_strerror(isp.ISP_ENOINIT).decode()
    assert L.isp_strerror(isp.ISP_EBUSY).decode().startswith("busy")
    assert L.isp_workspace_bytes(1 << 20) >= 32 * (1 << 20)


def test_range_workspace_by_mode(isp):
    """An interval call holds survivor workspace only for pieces that go to
    Miller-Rabin, and bucket workspace only for bucket-mode pieces; above
    2^32 also one 12-byte entry per interval prime: the prime, its 32-bit
    reciprocal and the piece's residue (2,063,688 odd primes below 2^25, one
    entry to spare)."""
    W = isp.lib().isp_range_workspace_bytes
    res = 12 * 2063689
    assert W(0, 1 << 20) == 0                      # below 2^32: the table
    assert W(1 << 34, 1 << 28) == res              # complete segment sieve
    assert W(1 << 44, 1 << 30) == res
    assert W((1 << 32) - 10, 20) == res            # crosses 2^32
    assert W(1 << 63, 1 << 24) == isp.workspace_bytes(1 << 24) + res  # short: Miller-Rabin
    b = W(1 << 62, 1 << 30)                        # bucket mode, no survivors
    assert res < b < 3 << 30 and b < isp.workspace_bytes(1 << 28)
    assert W((1 << 64) - 5, 10) == 0                # passes 2^64 - 1
    assert W(5, 0) == 0


def test_config_validation(isp):
    prev = isp.get_config()
    try:
        for bad in (dict(classify_block=100), dict(classify_ept=3), dict(filter_primes=300),
                    dict(filter_primes=12),
                    dict(mr_window=5), dict(sort_survivors=2), dict(classify_blocks_per_cu=17),
                    dict(mr_block=2048), dict(mr_block=96), dict(mr_blocks_per_cu=0 - 1),
                    dict(wheel_log2=32), dict(wheel_log2=41), dict(wheel_log2=-2)):
            with pytest.raises(isp.IsprimeError):
                isp.set_config(**bad)
        isp.set_config(mr_window=4)
        assert isp.get_config()["mr_window"] == 4
        assert prev["wheel_log2"] == -1  # the wheel stage is off by default
        for b in (33, 40):
            isp.set_config(wheel_log2=b)
            assert isp.get_config()["wheel_log2"] == b
    finally:
        isp.set_config(**prev)
    assert isp.get_config() == prev


def test_no_oracle_in_product_path():
    """The product package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2108_04791_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text, f
