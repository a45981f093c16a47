"""CPU oracle for the P-MPSM equi-join -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it,
and it imports nothing from the product package.

Thin ctypes wrapper around ``oracle.c`` (plain, sequential C; integer
arithmetic in every join result, floating point only in the Section 4
estimates).  Arrays are numpy ``uint64`` of shape ``[n, 2]``
(key, payload).  See ``oracle.c`` for the paper passage each function
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    src = os.path.join(_HERE, "oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", src, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        u64, u32, i32, p, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_double
        sig = {
            "orc_mix64": ([u64], u64),
            "orc_splitmix_at": ([u64, u64], u64),
            "orc_pair_hash": ([u64, u64, u64], u64),
            "orc_sort_by_key": ([p, u64], i32),
            "orc_sort_pairs": ([p, u64], None),
            "orc_join": ([p, u64, p, u64, p, p, u64], i32),
            "orc_join_nested": ([p, u64, p, u64, p, p, u64], i32),
            "orc_join_key_range": ([p, u64, p, u64, u64, u64, i32, p], i32),
            "orc_join_hash": ([p, u64, p, u64, p, p], i32),
            "orc_fk_closed_form": ([p, p, p, u64, p], i32),
            "orc_sort_runs": ([p, u64, u64, p], i32),
            "orc_radix_partition": ([p, u64, u64, i32, i32, p, u32, p, p, p, p], i32),
            "orc_sample_splitters": ([p, u64, u32, u32, u64, p], i32),
            "orc_cdf_knots": ([p, u64, u32, u32, u64, p], i32),
            "orc_bucket_of": ([p, u32, u64], u32),
            "orc_bucket_partition": ([p, u64, p, u32, p, p], i32),
            "orc_lower_bound": ([p, u64, u64], u64),
            "orc_interp_search": ([p, u64, u64, p], u64),
            "orc_equi_height": ([p, u64, u64, p], u64),
            "orc_s_cdf": ([p, p, u32, u64, p, u64, p], i32),
            "orc_split_cost": ([u64, u32, u64], dbl),
            "orc_cost_splitters_dp": ([p, p, u32, u32, u32, p], dbl),
            "orc_pmpsm_join": ([p, u64, p, u64, u32, i32, i32, p, p], i32),
            "orc_bmpsm_join": ([p, u64, p, u64, u32, p], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _tuples(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if a.ndim != 2 or a.shape[1] != 2:
        raise ValueError("tuples must have shape [n, 2]")
    return a


class JoinResult(NamedTuple):
    count: int
    checksum: int
    maxsum: int        # max(R.payload + S.payload), wrapping uint64 sum
    nonempty: bool
    pairs: np.ndarray | None = None


def _result(out4, pairs=None) -> JoinResult:
    return JoinResult(int(out4[0]), int(out4[1]), int(out4[2]), bool(out4[3]), pairs)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed ({rc})")


def mix64(z: int) -> int:
    return int(lib().orc_mix64(z))


def splitmix_at(seed: int, i: int) -> int:
    return int(lib().orc_splitmix_at(seed, i))


def pair_hash(k: int, rp: int, sp: int) -> int:
    return int(lib().orc_pair_hash(k, rp, sp))


def join(R, S, pairs: bool = False, cap: int | None = None) -> JoinResult:
    """The join by definition: sort both inputs, textbook merge."""
    R, S = _tuples(R), _tuples(S)
    out4 = np.zeros(4, np.uint64)
    pbuf = None
    if pairs:
        cap = cap if cap is not None else max(1, len(R) * len(S) if len(R) * len(S) < (1 << 24) else (1 << 24))
        pbuf = np.zeros((cap, 3), np.uint64)
    _check(lib().orc_join(_p(R), len(R), _p(S), len(S), _p(out4), _p(pbuf), cap or 0), "join")
    if pairs:
        pbuf = pbuf[: min(int(out4[0]), cap)]
    return _result(out4, pbuf)


def join_key_range(R, S, lo: int, hi: int | None) -> JoinResult:
    """The join restricted to keys in [lo, hi) (hi None: up to 2^64 - 1)."""
    R, S = _tuples(R), _tuples(S)
    out4 = np.zeros(4, np.uint64)
    _check(lib().orc_join_key_range(_p(R), len(R), _p(S), len(S), lo, 0 if hi is None else hi,
                                    1 if hi is None else 0, _p(out4)), "join_key_range")
    return _result(out4)


def join_sliced(R, S, bounds, threads: int = 1) -> JoinResult:
    """The join as the sum of its key-range slices [b_i, b_{i+1}) over the
    sorted inner bounds (first slice from 0, last to 2^64 - 1), each slice
    joined by join_key_range, the slices spread over `threads` threads."""
    from concurrent.futures import ThreadPoolExecutor
    edges = [0] + [int(b) for b in bounds] + [None]
    parts = [(edges[i], edges[i + 1]) for i in range(len(edges) - 1)]
    with ThreadPoolExecutor(max(1, threads)) as ex:
        res = list(ex.map(lambda ab: join_key_range(R, S, ab[0], ab[1]), parts))
    M = (1 << 64) - 1
    count = sum(r.count for r in res)
    checksum = sum(r.checksum for r in res) & M
    nonempty = any(r.nonempty for r in res)
    maxsum = max((r.maxsum for r in res if r.nonempty), default=0)
    return JoinResult(count, checksum, maxsum, nonempty)


def join_nested(R, S, pairs: bool = False) -> JoinResult:
    R, S = _tuples(R), _tuples(S)
    out4 = np.zeros(4, np.uint64)
    cap = len(R) * len(S) if pairs else 0
    pbuf = np.zeros((max(cap, 1), 3), np.uint64) if pairs else None
    _check(lib().orc_join_nested(_p(R), len(R), _p(S), len(S), _p(out4), _p(pbuf), cap), "join_nested")
    return _result(out4, pbuf[: int(out4[0])] if pairs else None)


def join_hash(R, S):
    """Hash join result and the key-count invariant sum_k cntR(k)*cntS(k)."""
    R, S = _tuples(R), _tuples(S)
    out4 = np.zeros(4, np.uint64)
    inv = ctypes.c_uint64(0)
    _check(lib().orc_join_hash(_p(R), len(R), _p(S), len(S), _p(out4), ctypes.byref(inv)), "join_hash")
    return _result(out4), int(inv.value)


def fk_closed_form(R, S, partner) -> JoinResult:
    R, S = _tuples(R), _tuples(S)
    partner = np.ascontiguousarray(partner, dtype=np.uint32)
    out4 = np.zeros(4, np.uint64)
    _check(lib().orc_fk_closed_form(_p(R), _p(S), _p(partner), len(S), _p(out4)), "fk_closed_form")
    return _result(out4)


def sort_by_key(T) -> np.ndarray:
    T = _tuples(T).copy()
    _check(lib().orc_sort_by_key(_p(T), len(T)), "sort_by_key")
    return T


def sort_runs(S, run_len: int) -> np.ndarray:
    S = _tuples(S)
    out = np.empty_like(S)
    _check(lib().orc_sort_runs(_p(S), len(S), run_len, _p(out)), "sort_runs")
    return out


def radix_partition(C, chunk_len: int, B: int, shift: int, sp, P: int):
    """Returns (hist[nchunk,P], ps[nchunk,P], base[P+1], out)."""
    C = _tuples(C)
    sp = np.ascontiguousarray(sp, dtype=np.uint32)
    n = len(C)
    nchunk = (n + chunk_len - 1) // chunk_len
    hist = np.zeros((max(nchunk, 1), P), np.uint64)
    ps = np.zeros((max(nchunk, 1), P), np.uint64)
    base = np.zeros(P + 1, np.uint64)
    out = np.empty_like(C)
    _check(lib().orc_radix_partition(_p(C), n, chunk_len, B, shift, _p(sp), P, _p(hist), _p(ps), _p(base), _p(out)),
           "radix_partition")
    return hist[:nchunk], ps[:nchunk], base, out


def sample_splitters(T, nbucket: int, oversample: int, seed: int) -> np.ndarray:
    T = _tuples(T)
    spl = np.zeros(max(nbucket - 1, 1), np.uint64)
    _check(lib().orc_sample_splitters(_p(T), len(T), nbucket, oversample, seed, _p(spl)), "sample_splitters")
    return spl[: max(nbucket - 1, 0)]


def cdf_knots(T, m: int, k: int, seed: int) -> np.ndarray:
    T = _tuples(T)
    out = np.zeros(k, np.uint64)
    _check(lib().orc_cdf_knots(_p(T), len(T), m, k, seed, _p(out)), "cdf_knots")
    return out


def bucket_of(spl, nbucket: int, key: int) -> int:
    spl = np.ascontiguousarray(spl, dtype=np.uint64)
    return int(lib().orc_bucket_of(_p(spl) if len(spl) else None, nbucket, key))


def bucket_partition(T, spl, nbucket: int):
    T = _tuples(T)
    spl = np.ascontiguousarray(spl, dtype=np.uint64)
    out = np.empty_like(T)
    bstart = np.zeros(nbucket + 1, np.uint64)
    _check(lib().orc_bucket_partition(_p(T), len(T), _p(spl) if len(spl) else None, nbucket, _p(out), _p(bstart)),
           "bucket_partition")
    return out, bstart


def lower_bound(run, key: int) -> int:
    run = _tuples(run)
    return int(lib().orc_lower_bound(_p(run), len(run), key))


def interp_search(run, key: int):
    run = _tuples(run)
    probes = ctypes.c_uint32(0)
    pos = int(lib().orc_interp_search(_p(run), len(run), key, ctypes.byref(probes)))
    return pos, int(probes.value)


def equi_height(run, stride: int) -> np.ndarray:
    """Bounds of the run's equi-height histogram: its key at every
    stride-th position from 0 (Section 4.1)."""
    run = _tuples(run)
    out = np.zeros(max(1, (len(run) + stride - 1) // stride), np.uint64)
    m = int(lib().orc_equi_height(_p(run), len(run), stride, _p(out)))
    return out[:m]


def s_cdf(S_runs, run_start, stride: int, keys) -> np.ndarray:
    """Estimated number of S tuples below each key, from the runs' merged
    equi-height bounds with equal step heights and linear interpolation
    (Section 4.1, Fig. 8).  S_runs: the sorted runs concatenated; run_start:
    Q + 1 run boundaries."""
    S_runs = _tuples(S_runs)
    rs = np.ascontiguousarray(run_start, dtype=np.uint64)
    x = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(max(1, len(x)), np.float64)
    _check(lib().orc_s_cdf(_p(S_runs), _p(rs), len(rs) - 1, stride, _p(x), len(x), _p(out)), "s_cdf")
    return out[:len(x)]


def split_cost(r_size: int, T: int, s_tuples: int) -> float:
    return float(lib().orc_split_cost(r_size, T, s_tuples))


def cost_splitters_dp(h, s, P: int, T: int):
    h = np.ascontiguousarray(h, dtype=np.uint64)
    s = np.ascontiguousarray(s, dtype=np.uint64)
    first = np.zeros(P, np.uint32)
    opt = float(lib().orc_cost_splitters_dp(_p(h), _p(s), len(h), P, T, _p(first)))
    return opt, first


def bmpsm_join(R, S, T: int) -> JoinResult:
    """B-MPSM (Section 2.1): T sorted runs of each input, every R run
    merge-joined with every S run."""
    R, S = _tuples(R), _tuples(S)
    out4 = np.zeros(4, np.uint64)
    _check(lib().orc_bmpsm_join(_p(R), len(R), _p(S), len(S), T, _p(out4)), "bmpsm_join")
    return _result(out4)


def pmpsm_join(R, S, T: int, B: int, shift: int = 0, sp=None) -> JoinResult:
    R, S = _tuples(R), _tuples(S)
    out4 = np.zeros(4, np.uint64)
    spa = None if sp is None else np.ascontiguousarray(sp, dtype=np.uint32)
    _check(lib().orc_pmpsm_join(_p(R), len(R), _p(S), len(S), T, B, shift, _p(spa), _p(out4)), "pmpsm_join")
    return _result(out4)
