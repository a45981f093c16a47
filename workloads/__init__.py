"""Seeded synthetic inputs for the MPSM join (host side, shared by the oracle
checks and the GPU tests/bench).

Arrays are numpy ``uint64`` of shape ``[n, 2]``: column 0 is the join key,
column 1 the payload (the paper's ``{joinkey: 64-bit, payload: 64-bit}``
relations, Section 5.1).  Nothing here computes any part of the join.

The five named workloads:

* ``fk_small``   |R|=2^20 keys = permutation of [0,2^20), |S|=2^22 uniform
  foreign keys.
* ``fk_uniform`` |R|=2^26 keys = permutation of [0,2^26) mixed into 64-bit
  space by a keyed bijection, |S|=2^28 uniform foreign keys.
* ``skewed``     |R|=2^26 distinct keys from 64 Gaussian blobs, |S|=2^28
  Zipf(1.0) foreign keys over R's key set.
* ``lognormal``  |R|=2^28 keys floor(exp(2Z) 2^28) with duplicates,
  |S|=2^30 with 1..16 copies of every distinct R key.
* ``batch``      256 joins, |R_b| log-uniform in [2^12, 2^22],
  |S_b| = k_b |R_b|, k_b in {1..8}, half uniform, half Zipf(0.5..1.2).

Workloads of the paper's other experiments: ``negcorr`` (negatively
correlated 80:20 skew, Section 5.6), ``location_skew`` (S ordered small to
large in clusters, Section 5.5) and foreign-key joins of multiplicity m for
role reversal (Section 5.4, ``fk_uniform`` with |S| = m |R|).

``scale_shift`` shrinks every size by 2^scale_shift for tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libworkloads.so")
_lib = None

SEED_BASE = 0x1207014500000000
WORKLOAD_SEEDS = {"fk_small": SEED_BASE + 1, "fk_uniform": SEED_BASE + 2, "skewed": SEED_BASE + 3,
                  "lognormal": SEED_BASE + 4, "batch": SEED_BASE + 5}


def build() -> str:
    """Compile gen.c into libworkloads.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", src, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        u64, i32, p = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        L.wl_gen_fk_uniform.argtypes = [u64, u64, u64, i32, p, p, p]
        L.wl_gen_zipf_partner.argtypes = [u64, u64, ctypes.c_double, u64, p]
        L.wl_gen_clustered_r.argtypes = [u64, u64, i32, p]
        L.wl_gen_s_from_partner.argtypes = [p, u64, u64, p, p]
        L.wl_gen_lognormal.argtypes = [u64, u64, u64, ctypes.c_double, p, p, p, p]
        L.wl_batch_sizes.argtypes = [i32, u64, i32, i32, p, p, p, p, ctypes.c_double, ctypes.c_double]
        L.wl_batch_fill.argtypes = [i32, u64, u64, u64, i32, ctypes.c_double, p, p, p]
        L.wl_gen_uniform_keys.argtypes = [u64, u64, u64, u64, p]
        L.wl_splitmix_at.argtypes = [u64, u64]
        L.wl_splitmix_at.restype = u64
        for f in (L.wl_gen_fk_uniform, L.wl_gen_zipf_partner, L.wl_gen_clustered_r, L.wl_gen_s_from_partner,
                  L.wl_gen_lognormal, L.wl_batch_sizes, L.wl_batch_fill, L.wl_gen_uniform_keys):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"workload generator {what} failed with code {rc}")


@dataclass
class Workload:
    name: str
    R: np.ndarray
    S: np.ndarray
    partner: np.ndarray | None = None   # S[j].key == R[partner[j]].key (foreign-key workloads)
    expected_count: int | None = None   # join size known by construction
    meta: dict = field(default_factory=dict)


def fk_uniform(nR: int, nS: int, seed: int, spread: bool) -> Workload:
    R = np.empty((nR, 2), np.uint64)
    S = np.empty((nS, 2), np.uint64)
    partner = np.empty(nS, np.uint32)
    _check(lib().wl_gen_fk_uniform(nR, nS, seed, int(spread), _ptr(R), _ptr(S), _ptr(partner)), "fk_uniform")
    return Workload("fk_uniform", R, S, partner, nS, {"spread": spread})


def zipf_partner(nR: int, nS: int, theta: float, seed: int) -> np.ndarray:
    partner = np.empty(nS, np.uint32)
    _check(lib().wl_gen_zipf_partner(nR, nS, theta, seed, _ptr(partner)), "zipf")
    return partner


def skewed(nR: int, nS: int, seed: int, theta: float = 1.0, nblob: int = 64) -> Workload:
    R = np.empty((nR, 2), np.uint64)
    _check(lib().wl_gen_clustered_r(nR, seed, nblob, _ptr(R)), "clustered")
    partner = zipf_partner(nR, nS, theta, seed)
    S = np.empty((nS, 2), np.uint64)
    _check(lib().wl_gen_s_from_partner(_ptr(R), nS, seed, _ptr(partner), _ptr(S)), "s_from_partner")
    return Workload("skewed", R, S, partner, nS, {"theta": theta, "nblob": nblob})


def lognormal(nR: int, nS: int, seed: int, sigma: float = 2.0) -> Workload:
    R = np.empty((nR, 2), np.uint64)
    S = np.empty((nS, 2), np.uint64)
    D = ctypes.c_uint64(0)
    pairs = ctypes.c_uint64(0)
    _check(lib().wl_gen_lognormal(nR, nS, seed, sigma, _ptr(R), _ptr(S), ctypes.byref(D), ctypes.byref(pairs)),
           "lognormal")
    return Workload("lognormal", R, S, None, int(pairs.value), {"distinct": int(D.value), "sigma": sigma})


def batch(n_join: int, seed: int, lo_log2: int = 12, hi_log2: int = 22,
          zlo: float = 0.5, zhi: float = 1.2) -> list[Workload]:
    nR = np.empty(n_join, np.uint64)
    nS = np.empty(n_join, np.uint64)
    zf = np.empty(n_join, np.int32)
    th = np.empty(n_join, np.float64)
    _check(lib().wl_batch_sizes(n_join, seed, lo_log2, hi_log2, _ptr(nR), _ptr(nS), _ptr(zf), _ptr(th), zlo, zhi),
           "batch_sizes")
    out = []
    for b in range(n_join):
        R = np.empty((int(nR[b]), 2), np.uint64)
        S = np.empty((int(nS[b]), 2), np.uint64)
        partner = np.empty(int(nS[b]), np.uint32)
        _check(lib().wl_batch_fill(b, seed, int(nR[b]), int(nS[b]), int(zf[b]), float(th[b]),
                                   _ptr(R), _ptr(S), _ptr(partner)), "batch_fill")
        out.append(Workload(f"batch[{b}]", R, S, partner, int(nS[b]),
                            {"zipf": bool(zf[b]), "theta": float(th[b])}))
    return out


def uniform_keys(n: int, domain: int, seed: int, tag: int = 0) -> np.ndarray:
    """n tuples with keys uniform in [0, domain) (domain 0 = all of uint64)."""
    T = np.empty((n, 2), np.uint64)
    _check(lib().wl_gen_uniform_keys(n, domain, seed, tag, _ptr(T)), "uniform_keys")
    return T


def splitmix_at(seed: int, i: int) -> int:
    return int(lib().wl_splitmix_at(seed, i))


def negcorr(nR: int, nS: int, seed: int, domain: int | None = None, hot: float = 0.8, span: float = 0.2) -> Workload:
    """Negatively correlated skew (the paper's Section 5.6 data set): 80% of
    R's keys uniform in the top 20% of the key domain, the rest uniform
    below it; 80% of S's keys uniform in the bottom 20%, the rest above it.
    Keys are drawn independently (duplicates kept; no foreign-key relation).
    The paper draws 1600 M keys from [0, 2^32), about 0.37 keys per domain
    value; the default domain here is 4 x the power of two at or above |R|
    (0.25 per value at |R| = 2^24)."""
    D = domain or 4 * (1 << max(0, (nR - 1).bit_length()))
    cut_r, cut_s = int(D * (1 - span)), int(D * span)
    rng = np.random.default_rng(seed)
    hr = rng.random(nR) < hot
    rk = np.where(hr, rng.integers(cut_r, D, nR, dtype=np.uint64), rng.integers(0, cut_r, nR, dtype=np.uint64))
    hs = rng.random(nS) < hot
    sk = np.where(hs, rng.integers(0, cut_s, nS, dtype=np.uint64), rng.integers(cut_s, D, nS, dtype=np.uint64))
    pr = rng.integers(0, (1 << 64) - 1, nR, dtype=np.uint64, endpoint=True)
    ps = rng.integers(0, (1 << 64) - 1, nS, dtype=np.uint64, endpoint=True)
    return Workload("negcorr", np.stack([rk, pr], 1), np.stack([sk, ps], 1), None, None,
                    {"domain": D, "hot": hot, "span": span})


def location_skew(w: Workload, clusters: int, seed: int) -> Workload:
    """S arranged small to large in `clusters` consecutive clusters of equal
    size, each in random order inside (the paper's Section 5.5: no total
    order, so the clusters still need sorting); R unchanged."""
    rng = np.random.default_rng(seed)
    order = np.argsort(w.S[:, 0], kind="stable")
    n = len(order)
    bounds = [(c * n) // clusters for c in range(clusters + 1)]
    for a, b in zip(bounds[:-1], bounds[1:]):
        rng.shuffle(order[a:b])
    S = np.ascontiguousarray(w.S[order])
    partner = None if w.partner is None else np.ascontiguousarray(w.partner[order])
    return Workload(w.name + "+location_skew", w.R, S, partner, w.expected_count, {**w.meta, "clusters": clusters})


def make(name: str, scale_shift: int = 0, seed: int | None = None):
    """The named workload at its full size shrunk by 2^scale_shift."""
    s = WORKLOAD_SEEDS[name] if seed is None else seed
    k = scale_shift
    if name == "fk_small":
        return fk_uniform(1 << (20 - k), 1 << (22 - k), s, spread=False)
    if name == "fk_uniform":
        w = fk_uniform(1 << (26 - k), 1 << (28 - k), s, spread=True)
        w.name = name
        return w
    if name == "skewed":
        return skewed(1 << (26 - k), 1 << (28 - k), s)
    if name == "lognormal":
        return lognormal(1 << (28 - k), 1 << (30 - k), s)
    if name == "batch":
        return batch(256 >> min(k, 7), s, 12 - min(k, 6), 22 - k)
    raise KeyError(name)
