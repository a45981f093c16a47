"""The start search's last step (the lower bound inside the window that the
run index leaves, probed line by line from an interpolated first line) run
on the CPU with the device code: equal to the plain lower bound whatever the
interpolation bounds say, on runs with duplicates, gaps and extreme keys."""
import numpy as np
import pytest

import paper_1207_0145_amd as mpsm

U64 = (1 << 64) - 1


def _window_cases(rng, keys, n_cases):
    n = len(keys)
    for _ in range(n_cases):
        key = int(keys[rng.integers(0, n)]) + int(rng.integers(-2, 3)) if rng.random() < 0.7 \
            else int(rng.integers(0, U64, dtype=np.uint64, endpoint=True))
        key = min(max(key, 0), U64)
        lb = int(np.searchsorted(keys, np.uint64(key), side="left"))
        # any window [a, b] around the bound: a <= lb <= b
        a = int(rng.integers(0, lb + 1))
        b = int(rng.integers(lb, n + 1))
        yield key, lb, a, b


@pytest.mark.parametrize("kind", ["uniform", "dups", "clustered", "tiny"])
def test_window_lower_bound_equals_searchsorted(kind):
    rng = np.random.default_rng({"uniform": 1, "dups": 2, "clustered": 3, "tiny": 4}[kind])
    if kind == "uniform":
        keys = np.sort(rng.integers(0, U64, 4096, dtype=np.uint64, endpoint=True))
    elif kind == "dups":
        keys = np.sort(rng.integers(0, 40, 3000).astype(np.uint64))
    elif kind == "clustered":
        keys = np.sort(np.concatenate([rng.integers(c, c + 50, 300, dtype=np.uint64)
                                       for c in rng.integers(0, U64 - 100, 8, dtype=np.uint64)]))
    else:
        keys = np.array([0, 0, 5, U64, U64], np.uint64)
    for key, lb, a, b in _window_cases(rng, keys, 400):
        # interpolation bounds: the true neighbours, or nonsense
        for klo, khi in [(int(keys[a - 1]) if a else 0, int(keys[b]) if b < len(keys) else U64),
                         (0, U64), (U64, 0), (key, key), (int(rng.integers(0, U64, dtype=np.uint64)), 7)]:
            got, probes = mpsm.lower_bound_window_host(keys, a, b, klo, khi, key)
            assert got == lb, (kind, key, a, b, klo, khi)
            # the interpolated line, a gallop, then a bisection of what is left
            assert probes <= 3 + 2 * int(np.ceil(np.log2(b - a + 1))), (kind, key, a, b, probes)


def test_window_probes_one_line_on_uniform_keys():
    """With the true index keys around a 256-key window of uniform keys, the
    interpolated first line is the right one, or a neighbour, in most cases
    (lines read: against about five for a bisection of the window)."""
    rng = np.random.default_rng(5)
    keys = np.sort(rng.integers(0, 1 << 60, 1 << 16, dtype=np.uint64))
    probes = []
    for _ in range(2000):
        w = int(rng.integers(1, (1 << 16) // 256 - 1))
        a, b = (w - 1) * 256 + 1, w * 256
        key = int(rng.integers(int(keys[a - 1]) + 1, int(keys[b]) + 1))
        got, pr = mpsm.lower_bound_window_host(keys, a, b, int(keys[a - 1]), int(keys[b]), key)
        assert got == int(np.searchsorted(keys, np.uint64(key), side="left"))
        probes.append(pr)
    assert np.mean(probes) < 2.0


def test_window_rejects_null():
    L = mpsm.lib()
    out = mpsm.ctypes.c_uint32(0)
    assert L.mpsm_lower_bound_window_host(None, 0, 4, 0, 0, 1, mpsm.ctypes.byref(out), None) == 1   # no keys
    assert L.mpsm_lower_bound_window_host(None, 3, 3, 0, 0, 1, None, None) == 1                      # no out
    assert L.mpsm_lower_bound_window_host(None, 3, 3, 0, 0, 1, mpsm.ctypes.byref(out), None) == 0    # empty window
    assert out.value == 3
