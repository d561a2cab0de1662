"""The library's radix sort (tree build, ray order, image-source collection,
IR assembly) against numpy's stable sort, through its test hook: sizes that
end inside a tile and span many tiles, bit ranges of one to eight digits,
keys with long runs of equal digits (every tile's digit counts and their
prefix over the tiles must be exact), a last digit narrower than 8 bits, and
a device-side count below the capacity."""
import ctypes
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_1811_05784_amd as rt
    return rt.load()


def _keys(n, seed, kind):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(0, 2 ** 63, size=n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=n).astype(np.uint64)
    if kind == "few":      # a handful of distinct keys: long runs of one digit across many tiles
        return rng.choice(np.array([0, 7, 255, 1 << 20, (1 << 40) + 3, 2 ** 64 - 1], dtype=np.uint64), size=n)
    if kind == "sorted":
        return np.sort(rng.integers(0, 1 << 30, size=n).astype(np.uint64))
    raise ValueError(kind)


def _run(lib, keys, begin, end, n=None, cap=None):
    cap = len(keys) if cap is None else cap
    k = torch.zeros(cap, dtype=torch.int64, device="cuda:0")
    k[:len(keys)] = torch.from_numpy(keys.view(np.int64)).to("cuda:0")
    order = torch.full((cap,), -1, dtype=torch.int32, device="cuda:0")
    n_dev = None if n is None else torch.tensor([n], dtype=torch.int64, device="cuda:0")
    rc = lib.rt_debug_radix_sort(ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(order.data_ptr()), cap,
                                 None if n_dev is None else ctypes.c_void_p(n_dev.data_ptr()), begin, end,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.rt_last_error()
    torch.cuda.synchronize()
    return k.cpu().numpy().view(np.uint64), order.cpu().numpy().astype(np.int64)


def _expect(keys, begin, end):
    w = end - begin
    mask = np.uint64((1 << w) - 1) if w < 64 else np.uint64(2 ** 64 - 1)
    d = (keys >> np.uint64(begin)) & mask
    perm = np.argsort(d, kind="stable")
    return keys[perm], perm


@pytest.mark.parametrize("n", [1, 5, 1023, 1024, 1025, 12_305, 300_001, 1_000_000])
@pytest.mark.parametrize("bits", [(0, 64), (0, 30), (0, 16), (8, 24), (3, 11)])
def test_sort_matches_stable_sort(lib, n, bits):
    for kind, seed in (("uniform", n + bits[0]), ("few", 7 * n + 1)):
        _say("sort n=%d bits=%s keys=%s" % (n, bits, kind))
        keys = _keys(n, seed, kind)
        got_k, got_o = _run(lib, keys, *bits)
        want_k, want_o = _expect(keys, *bits)
        assert np.array_equal(got_o, want_o), "order differs"
        assert np.array_equal(got_k, want_k), "keys differ"


def test_sort_with_a_device_count_below_the_capacity(lib):
    cap = 50_000
    for n in (0, 1, 999, 31_337, cap):
        _say("device count n=%d of cap %d" % (n, cap))
        keys = _keys(cap, n + 11, "uniform")
        got_k, got_o = _run(lib, keys, 0, 40, n=n, cap=cap)
        want_k, want_o = _expect(keys[:n], 0, 40)
        assert np.array_equal(got_o[:n], want_o) and np.array_equal(got_k[:n], want_k)


def test_sort_of_sorted_and_constant_keys(lib):
    for kind in ("sorted", "few"):
        keys = _keys(200_000, 3, kind)
        if kind == "few":
            keys[:] = keys[0]
        _say("sort of %s keys" % kind)
        got_k, got_o = _run(lib, keys, 0, 64)
        want_k, want_o = _expect(keys, 0, 64)
        assert np.array_equal(got_o, want_o) and np.array_equal(got_k, want_k)


def test_sort_rejects_bad_bit_ranges(lib):
    k = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    o = torch.zeros(4, dtype=torch.int32, device="cuda:0")
    for b, e in ((0, 0), (5, 3), (0, 65), (-1, 8)):
        assert lib.rt_debug_radix_sort(ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(o.data_ptr()), 4, None, b, e,
                                       None) == -1
