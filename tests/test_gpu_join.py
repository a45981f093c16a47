"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Join results (count, checksum, sorted pair lists) must be bit-identical.
Intermediate results are compared where they are unique: sorted key
sequences, the multiset of tuples per run/bucket, splitters (same seeded
sample on both sides), bucket boundaries, and merge-start offsets (unique
lower bounds)."""
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_1207_0145_amd as mpsm
import workloads

pytestmark = pytest.mark.gpu
U64 = (1 << 64) - 1


def _dev(a):
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1, 2)
    return torch.from_numpy(a.view(np.int64)).to("cuda")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def gpu_join(R, S, cfg=None, pairs=False, workspace=None, stats=False):
    _say(f"mpsm_join nR={len(R)} nS={len(S)} pairs={pairs} "
         f"cfg={None if cfg is None else {k: getattr(cfg, k) for k, _ in cfg._fields_}}")
    return mpsm.join(_dev(R), _dev(S), cfg=cfg, pairs=pairs, workspace=workspace, with_stats=stats)


def check(R, S, cfg=None, pairs=False):
    want = oracle.join(R, S)
    got = gpu_join(R, S, cfg, pairs=pairs)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    if pairs:
        wp = oracle.join(R, S, pairs=True, cap=max(1, want.count)).pairs
        assert np.array_equal(got["pairs"], wp)
    return got


def rel(rng, n, domain):
    k = (rng.integers(0, domain, size=n, dtype=np.uint64) if domain
         else rng.integers(0, U64, size=n, dtype=np.uint64, endpoint=True))
    p = rng.integers(0, U64, size=n, dtype=np.uint64, endpoint=True)
    return np.stack([k, p], axis=1)


# ------------------------------------------------------------- small cases

def test_worked_example():
    R = np.array([(1, 10), (2, 20), (2, 21), (5, 50)], np.uint64)
    S = np.array([(2, 200), (2, 201), (3, 300), (5, 500), (7, 1)], np.uint64)
    got = check(R, S, pairs=True)
    assert got["count"] == 5 and got["checksum"] == 0x680EDA8D7152D3C9


@pytest.mark.parametrize("nR,nS", [(0, 0), (0, 7), (7, 0), (1, 1)])
def test_empty_and_single(nR, nS):
    rng = np.random.default_rng(nR + 10 * nS)
    check(rel(rng, nR, 3), rel(rng, nS, 3))


@pytest.mark.parametrize("nR,nS,domain", [(100, 300, 50), (1000, 3000, 100), (3000, 1000, 100), (5000, 20000, 0),
                                          (777, 7777, 7), (4097, 8193, 4096)])
def test_random_small_with_pairs(nR, nS, domain):
    rng = np.random.default_rng(nR * 31 + nS + domain)
    check(rel(rng, nR, domain), rel(rng, nS, domain), pairs=True)


def test_extreme_keys():
    rng = np.random.default_rng(8)
    keys = np.array([0, 1, U64 - 1, U64, 1 << 63], np.uint64)
    R = np.stack([keys[rng.integers(0, 5, 2000)], rng.integers(0, U64, 2000, dtype=np.uint64)], 1)
    S = np.stack([keys[rng.integers(0, 5, 3000)], rng.integers(0, U64, 3000, dtype=np.uint64)], 1)
    check(R, S)
    check(R[:40], S[:60], pairs=True)


def test_all_equal_keys():
    rng = np.random.default_rng(9)
    R = rel(rng, 300, 1)
    S = rel(rng, 1000, 1)
    check(R, S, pairs=True)
    R = rel(rng, 20000, 1)
    S = rel(rng, 30000, 1)
    check(R, S)                        # 6e8 pairs, count and checksum


def test_partitions_beyond_the_lds_tile_at_scale():
    """|R| = 2^21 with 64 keys of 12000 copies each (join units larger than
    the 8192-tuple LDS tile, joined from global memory) among distinct keys,
    |S| = 2^23 drawn from R's distinct keys: count and checksum against the
    oracle, which also counts the heavy keys' pairs one by one."""
    rng = np.random.default_rng(2112)
    n = 1 << 21
    heavy = rng.integers(0, U64, 64, dtype=np.uint64)
    k = rng.integers(0, U64, n, dtype=np.uint64)
    k[: 64 * 12000] = np.repeat(heavy, 12000)
    R = np.stack([k[rng.permutation(n)], rng.integers(0, U64, n, dtype=np.uint64, endpoint=True)], 1)
    u = np.unique(R[:, 0])
    S = np.stack([u[rng.integers(0, len(u), 1 << 23)], rng.integers(0, U64, 1 << 23, dtype=np.uint64, endpoint=True)], 1)
    want = oracle.join(R, S)
    assert np.isin(S[:, 0], heavy).sum() >= 64   # the heavy keys meet S
    got = gpu_join(R, S, stats=True)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    assert got["stats"]["max_partition"] >= 12000


def test_disjoint_ranges():
    rng = np.random.default_rng(10)
    R = rel(rng, 5000, 1000)
    S = rel(rng, 9000, 1000)
    S[:, 0] += np.uint64(5000)
    got = check(R, S)
    assert got["count"] == 0 and got["checksum"] == 0


def test_ragged_sizes():
    rng = np.random.default_rng(11)
    check(rel(rng, 70001, 1 << 20), rel(rng, 300007, 1 << 20))


def _spaced_keys(kind, n, rng):
    """R key sets whose partitions span key ranges around the bounds of the
    cell maps (splitter directory, sort sub-buckets, join directory): narrower
    than the directory (a dense range far from 0), partitions about 2^42 and
    2^51 wide (keys 2^31 + 7 and 2^40 + 12345 apart), the top of the 64-bit
    range, and dense and sparse partitions side by side."""
    i = rng.permutation(n).astype(np.uint64)
    if kind == "dense_high_base":
        return np.uint64(1 << 40) + i
    if kind == "step_2p31":
        return i * np.uint64((1 << 31) + 7)
    if kind == "step_2p40":
        return i * np.uint64((1 << 40) + 12345)
    if kind == "top_of_range":
        return np.uint64(U64) - i * np.uint64(3)
    if kind == "dense_and_sparse":
        half = n // 2
        sparse = rng.integers(1 << 20, U64, size=n - half, dtype=np.uint64, endpoint=True)
        return np.concatenate([i[:half] % np.uint64(half), sparse])
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["dense_high_base", "step_2p31", "step_2p40", "top_of_range", "dense_and_sparse"])
@pytest.mark.parametrize("kw", [dict(), dict(search=mpsm.SEARCH_BINARY), dict(splitter=mpsm.SPLIT_LEARNED)],
                         ids=["default", "binary", "learned"])
def test_key_ranges_around_the_cell_maps(kind, kw):
    rng = np.random.default_rng(zlib.crc32(kind.encode()))
    nR, nS = 1 << 17, 1 << 19
    rk = _spaced_keys(kind, nR, rng)
    R = np.stack([rk, rng.integers(0, U64, nR, dtype=np.uint64, endpoint=True)], 1)
    # foreign keys, plus keys just beside R's (absent unless R has them)
    sk = rk[rng.integers(0, nR, nS)]
    nudge = rng.integers(0, 4, nS) == 0
    sk[nudge] = sk[nudge] + np.uint64(1)
    S = np.stack([sk, rng.integers(0, U64, nS, dtype=np.uint64, endpoint=True)], 1)
    check(R, S, mpsm.config(**kw))
    check(R[:3000], S[:9000], mpsm.config(**kw), pairs=True)


CONFIGS = [
    dict(role=mpsm.ROLE_AS_GIVEN), dict(role=mpsm.ROLE_SWAP), dict(search=mpsm.SEARCH_BINARY),
    dict(search=mpsm.SEARCH_INTERP), dict(log2_run_len=12), dict(log2_run_len=16, bucket_target=256),
    dict(bucket_target=1024, join_chunk=1024), dict(seed=12345), dict(want_max=1),
    dict(splitter=mpsm.SPLIT_LEARNED), dict(search=mpsm.SEARCH_LEARNED),
    dict(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED, bucket_target=1024),
    dict(splitter=mpsm.SPLIT_COST), dict(splitter=mpsm.SPLIT_COST, bucket_target=1024, search=mpsm.SEARCH_INTERP),
    dict(splitter=mpsm.SPLIT_NONE), dict(splitter=mpsm.SPLIT_NONE, log2_run_len=14, search=mpsm.SEARCH_INTERP),
    dict(splitter=mpsm.SPLIT_NONE, log2_run_len=13, role=mpsm.ROLE_SWAP, want_max=1),
]


@pytest.mark.parametrize("kw", CONFIGS, ids=[str(c) for c in CONFIGS])
def test_result_independent_of_config(kw):
    rng = np.random.default_rng(12)
    R = rel(rng, 60000, 200000)
    S = rel(rng, 250000, 200000)
    check(R, S, cfg=mpsm.config(**kw))


def test_want_max_matches_query_aggregate():
    rng = np.random.default_rng(13)
    R = rel(rng, 20000, 30000)
    S = rel(rng, 50000, 30000)
    want = oracle.join(R, S)
    got = gpu_join(R, S, mpsm.config(want_max=1), stats=True)
    assert got["count"] == want.count and got["stats"]["max_payload_sum"] == want.maxsum
    assert got["stats"]["nonempty"] == int(want.nonempty)


@pytest.mark.parametrize("workload,shift", [("fk_uniform", 8), ("skewed", 8), ("lognormal", 10)])
def test_learned_modes_exact_and_model_sane(workload, shift):
    w = workloads.make(workload, scale_shift=shift)
    want, _ = oracle.join_hash(w.R, w.S)
    for kw in (dict(), dict(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED)):
        got = gpu_join(w.R, w.S, mpsm.config(**kw), stats=True)
        assert (got["count"], got["checksum"]) == (want.count, want.checksum), kw
        st = got["stats"]
        if kw:
            # the model is fitted to its own sample; a continuous fit cannot follow a
            # jump of the CDF, so its error there is about the heaviest key's share
            top_s = np.unique(w.S[:, 0], return_counts=True)[1].max() / len(w.S)
            top_r = np.unique(w.R[:, 0], return_counts=True)[1].max() / len(w.R)
            assert 0.0 <= st["cdf_eps_r"] < 0.02 + 1.5 * top_r, st
            assert 0.0 <= st["cdf_eps_s"] < 0.02 + 1.5 * top_s, st
            assert st["search_fallbacks"] <= st["partitions"] * st["runs"]
        else:
            assert st["cdf_eps_r"] == -1.0 and st["search_fallbacks"] == 0


@pytest.mark.parametrize("name,shift", [("skewed", 6), ("lognormal", 8)])
def test_learned_cdf_knots_against_the_oracle(name, shift):
    """The learned models' piecewise-linear part: every knot of R's model
    (learned splitters) and of S's model (learned search) equals the
    oracle's knot of the same seeded sample of the same relation; the join
    stays exact."""
    w = workloads.make(name, scale_shift=shift)
    cfg = mpsm.config(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED)
    lay = mpsm.layout(len(w.R), len(w.S), cfg)
    assert lay["swapped"] == 0
    ws = mpsm.alloc_workspace(len(w.R), len(w.S), cfg)
    got = gpu_join(w.R, w.S, cfg, workspace=ws)
    want, _ = oracle.join_hash(w.R, w.S)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    torch.cuda.synchronize()
    m, k = lay["cdf_sample"], lay["cdf_knots"]
    for T, off, seed in ((w.R, lay["off_cdf_model_r"], lay["cdf_seed_r"]),
                         (w.S, lay["off_cdf_model_s"], lay["cdf_seed_s"])):
        assert np.array_equal(_ws_view(ws, off, k, np.uint64), oracle.cdf_knots(T, m, k, seed))


def test_learned_search_with_bad_window_falls_back():
    # tiny R with a handful of distinct keys: the model sees a step function;
    # whatever it predicts, the bracket check keeps the offsets exact
    rng = np.random.default_rng(21)
    R = rel(rng, 3000, 7)
    S = rel(rng, 200000, 7)
    check(R, S, cfg=mpsm.config(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED))


def test_oversize_bucket_fallback():
    # one sample key per bucket makes some buckets far larger than an LDS tile
    rng = np.random.default_rng(14)
    R = rel(rng, 200000, 0)
    S = rel(rng, 400000, 0)
    S[: len(S) // 2, 0] = R[rng.integers(0, len(R), len(S) // 2), 0]
    cfg = mpsm.config(oversample=1, bucket_target=4096)
    want = oracle.join(R, S)
    lay = mpsm.layout(len(R), len(S), cfg)
    ws = mpsm.alloc_workspace(len(R), len(S), cfg)
    got = gpu_join(R, S, cfg, workspace=ws, stats=True)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    assert got["stats"]["oversize_buckets"] > 0
    torch.cuda.synchronize()
    # the buckets sorted by the multi-pass sort are sorted like the rest
    L = lay["run_len"]
    Ssorted = _ws_view(ws, lay["off_s_sorted"], 2 * len(S), np.uint64).reshape(-1, 2)
    ref = oracle.sort_runs(S, L)
    assert np.array_equal(Ssorted[:, 0], ref[:, 0])
    for j in range(lay["runs"]):
        x, y = Ssorted[j * L:(j + 1) * L], ref[j * L:(j + 1) * L]
        assert np.array_equal(x[np.lexsort((x[:, 1], x[:, 0]))], y[np.lexsort((y[:, 1], y[:, 0]))])
    Rsorted = _ws_view(ws, lay["off_r_sorted"], 2 * len(R), np.uint64).reshape(-1, 2)
    assert np.array_equal(Rsorted[np.lexsort((Rsorted[:, 1], Rsorted[:, 0]))], R[np.lexsort((R[:, 1], R[:, 0]))])
    assert np.array_equal(Rsorted[:, 0], np.sort(R[:, 0]))


def test_few_distinct_keys_oversize_equal_buckets():
    rng = np.random.default_rng(15)
    keys = np.array([3, 1 << 40, U64], np.uint64)
    R = np.stack([keys[rng.integers(0, 3, 30000)], rng.integers(0, U64, 30000, dtype=np.uint64)], 1)
    S = np.stack([keys[rng.integers(0, 3, 40000)], rng.integers(0, U64, 40000, dtype=np.uint64)], 1)
    check(R, S)


def _dup_pattern(name, rng, n):
    """Key columns that stress the one-pass bucket sort: duplicates inside
    interpolation cells, clusters inside a bucket, heavy keys with light
    neighbours, and two heavy neighbours (which must fall back)."""
    if name == "zipf_copies":          # many keys with tens to thousands of copies
        base = rng.integers(0, U64, 1 << 16, dtype=np.uint64)
        return base[(len(base) * rng.random(n) ** 2).astype(np.int64)]
    if name == "two_clusters":         # two narrow clusters far apart, some repeats
        k = rng.integers(0, 1 << 30, n, dtype=np.uint64)
        k[rng.random(n) < 0.5] += np.uint64(1 << 62)
        k[: n // 8] = k[n // 8: n // 4]
        return k
    if name == "heavy_with_neighbours":  # heavy keys with light keys right next to them
        h = rng.integers(1 << 20, 1 << 60, 512, dtype=np.uint64)
        k = h[rng.integers(0, len(h), n)]
        light = rng.random(n) < 0.3
        k[light] += rng.integers(1, 2000, int(light.sum()), dtype=np.uint64)
        return k
    if name == "geometric":            # distinct-ish keys packed towards zero
        return np.floor(np.exp2(rng.random(n) * 60.0)).astype(np.uint64)
    if name in ("mid_groups", "mid_cells"):
        # run by run (runs of 2^17): keys with 9 to 32 copies, some copies
        # moved a little above their key, so that an interpolation cell
        # holds one frequent key and a few strays; mid_cells puts three such
        # keys next to each other, so that they share a first-level cell and
        # part in second-level cells
        out = []
        for _ in range((n + (1 << 17) - 1) >> 17):
            m = 1 << 17
            h = rng.integers(1 << 20, 1 << 62, m // 12, dtype=np.uint64)
            if name == "mid_cells":
                h = (h[:, None] + np.arange(3, dtype=np.uint64) * np.uint64(4096)).ravel()
            k = np.repeat(h, rng.integers(9, 33, len(h)))[:m]
            k = np.concatenate([k, rng.integers(0, U64, m - len(k), dtype=np.uint64)])
            stray = rng.random(m) < 0.06
            k[stray] += rng.integers(1, 256, int(stray.sum()), dtype=np.uint64)
            out.append(k[rng.permutation(m)])
        return np.concatenate(out)[:n]
    if name == "heavy_pairs":          # adjacent heavy keys share every cell: fallback path
        h = rng.integers(1 << 20, 1 << 60, 256, dtype=np.uint64)
        k = h[rng.integers(0, len(h), n)]
        k[rng.random(n) < 0.5] += np.uint64(1)
        return k
    raise ValueError(name)


@pytest.mark.parametrize("pattern", ["zipf_copies", "two_clusters", "heavy_with_neighbours", "geometric",
                                     "mid_groups", "mid_cells", "heavy_pairs"])
def test_bucket_sort_duplicates_and_clusters(pattern):
    rng = np.random.default_rng(zlib.crc32(pattern.encode()))
    nS = 1 << 20
    S = np.stack([_dup_pattern(pattern, rng, nS), rng.integers(0, U64, nS, dtype=np.uint64, endpoint=True)], 1)
    rk = np.unique(S[:, 0])
    rk = rk[rng.random(len(rk)) < 0.7]
    R = np.stack([np.concatenate([rk, rk[: len(rk) // 4]]),
                  rng.integers(0, U64, len(rk) + len(rk) // 4, dtype=np.uint64, endpoint=True)], 1)
    R = R[rng.permutation(len(R))]
    cfg = mpsm.config(log2_run_len=17)
    lay = mpsm.layout(len(R), nS, cfg)
    ws = mpsm.alloc_workspace(len(R), nS, cfg)
    got = gpu_join(R, S, cfg, workspace=ws, stats=True)
    want = oracle.join(R, S)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    torch.cuda.synchronize()
    L = lay["run_len"]
    Ssorted = _ws_view(ws, lay["off_s_sorted"], 2 * nS, np.uint64).reshape(-1, 2)
    ref = oracle.sort_runs(S, L)
    assert np.array_equal(Ssorted[:, 0], ref[:, 0])
    for j in range(lay["runs"]):
        x, y = Ssorted[j * L:(j + 1) * L], ref[j * L:(j + 1) * L]
        assert np.array_equal(x[np.lexsort((x[:, 1], x[:, 0]))], y[np.lexsort((y[:, 1], y[:, 0]))])
    Rsorted = _ws_view(ws, lay["off_r_sorted"], 2 * len(R), np.uint64).reshape(-1, 2)
    assert np.array_equal(Rsorted[:, 0], np.sort(R[:, 0]))
    st = got["stats"]
    _say(f"{pattern}: resorted buckets {st['resorted_buckets']} of {lay['runs'] * lay['s_buckets']} S buckets, "
         f"oversize {st['oversize_buckets']}")
    if pattern == "heavy_pairs":
        assert st["resorted_buckets"] > 0


def test_r_bucket_retry_over_own_range():
    """R made of blocks of 1500 consecutive keys plus 1500 keys spread over
    the next 2^20, far from both ends of the key space.  The first and last
    R buckets take their outer bounds from the key space itself (0 and
    2^64 - 1); interpolated over those, their keys fall into one cell whose
    second-level cells still hold hundreds of distinct keys, so the one-pass
    sort gives up on them and they are sorted again over their own key
    range (what is still left would go to the LSD sort)."""
    rng = np.random.default_rng(0x7E7)
    blocks = []
    for k in range(88):
        base = np.uint64((1 << 40) + (k << 20))
        tail = rng.choice((1 << 20) - 1500, 1500, replace=False).astype(np.uint64) + np.uint64(1500)
        blocks.append(base + np.concatenate([np.arange(1500, dtype=np.uint64), tail]))
    rk = np.concatenate(blocks)
    assert len(np.unique(rk)) == len(rk)
    R = np.stack([rk, rng.integers(0, U64, len(rk), dtype=np.uint64, endpoint=True)], 1)
    R = R[rng.permutation(len(R))]
    nS = 1 << 19
    S = np.stack([rk[rng.integers(0, len(rk), nS)], rng.integers(0, U64, nS, dtype=np.uint64, endpoint=True)], 1)
    cfg = mpsm.config()
    lay = mpsm.layout(len(R), nS, cfg)
    ws = mpsm.alloc_workspace(len(R), nS, cfg)
    got = gpu_join(R, S, cfg, workspace=ws, stats=True)
    want = oracle.join(R, S)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    torch.cuda.synchronize()
    Rsorted = _ws_view(ws, lay["off_r_sorted"], 2 * len(R), np.uint64).reshape(-1, 2)
    assert np.array_equal(Rsorted[:, 0], np.sort(R[:, 0]))
    assert np.array_equal(Rsorted[np.lexsort((Rsorted[:, 1], Rsorted[:, 0]))], R[np.lexsort((R[:, 1], R[:, 0]))])
    st = got["stats"]
    _say(f"retried R buckets {st['retried_buckets']}, LSD re-sorts {st['resorted_buckets']}")
    assert st["retried_buckets"] >= 1


# ------------------------------------------------------- named workloads

def test_fk_small_full_size():
    w = workloads.make("fk_small")                # |R| = 2^20, |S| = 2^22
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    got = check(w.R, w.S)
    assert got["count"] == len(w.S) and got["checksum"] == fk.checksum


def test_skewed_reduced():
    w = workloads.make("skewed", scale_shift=6)   # |R| = 2^20, |S| = 2^22, Zipf(1)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    got = gpu_join(w.R, w.S)
    assert (got["count"], got["checksum"]) == (fk.count, fk.checksum)


def test_lognormal_reduced():
    w = workloads.make("lognormal", scale_shift=8)   # |R| = 2^20, |S| = 2^22, duplicates
    want, inv = oracle.join_hash(w.R, w.S)
    got = gpu_join(w.R, w.S)
    assert got["count"] == w.expected_count == inv
    assert got["checksum"] == want.checksum


# ------------------------------------------------- B-MPSM (no range partitioning)

BMPSM = dict(splitter=mpsm.SPLIT_NONE)


@pytest.mark.parametrize("nR,nS,domain", [(0, 10, 5), (10, 0, 5), (1, 1, 2), (3000, 9000, 500),
                                          (70000, 5000, 0), (5000, 70001, 1 << 40)])
def test_bmpsm_small_with_pairs(nR, nS, domain):
    """B-MPSM: every R run against every S run; pair lists equal the oracle's."""
    rng = np.random.default_rng(nR * 7 + nS)
    check(rel(rng, nR, domain), rel(rng, nS, domain), cfg=mpsm.config(log2_run_len=12, **BMPSM), pairs=True)


@pytest.mark.parametrize("name,shift", [("skewed", 8), ("lognormal", 10)])
def test_bmpsm_skewed_and_duplicates(name, shift):
    """B-MPSM on Zipf(1) foreign keys and on log-normal keys with duplicates
    in R, with several R runs (run length 2^14)."""
    w = workloads.make(name, scale_shift=shift)
    want = oracle.join(w.R, w.S)
    for kw in (dict(log2_run_len=14), dict(log2_run_len=14, search=mpsm.SEARCH_LEARNED)):
        got = gpu_join(w.R, w.S, mpsm.config(**BMPSM, **kw), stats=True)
        assert (got["count"], got["checksum"]) == (want.count, want.checksum), kw
        lay = mpsm.layout(len(w.R), len(w.S), mpsm.config(**BMPSM, **kw))
        assert lay["runs"] > 1


def test_batch_members_reduced():
    for w in workloads.make("batch", scale_shift=5)[:4]:
        fk = oracle.fk_closed_form(w.R, w.S, w.partner)
        got = gpu_join(w.R, w.S)
        assert (got["count"], got["checksum"]) == (fk.count, fk.checksum), w.name


# ------------------------------------------------ intermediate results

def _check_splitters(got, quantiles):
    """GPU splitters against the oracle's equi-depth quantiles of the same
    seeded sample: each is its quantile, or (a frequent key isolated in its
    own bucket) the previous quantile + 1; non-decreasing."""
    got = np.asarray(got, np.uint64)
    q = np.asarray(quantiles, np.uint64)
    assert len(got) == len(q)
    moved = np.zeros(len(q), bool)
    moved[1:] = got[1:] == q[:-1] + np.uint64(1)
    assert np.all((got == q) | moved)
    assert np.all(got[1:] >= got[:-1])


def _bucket_starts_with_rule(keys, spl, nb):
    """Bucket starts of a stable partition of keys by the oracle's bucket
    function (the number of splitters <= key) with the kernel's documented
    exception: a key equal to two or more splitters goes to the bucket below
    (which those splitters leave empty), so that it has a bucket to itself."""
    b = np.array([oracle.bucket_of(spl, nb, int(k)) for k in np.unique(keys)], np.int64)
    u = np.unique(keys)
    sp = np.concatenate([[np.uint64(0)], spl])   # sp[b] = spl[b-1]
    twice = (b >= 2) & (sp[np.maximum(b, 1)] == u) & (sp[np.maximum(b - 1, 0)] == u)
    b = b - twice
    per_key = b[np.searchsorted(u, keys)]
    cnt = np.bincount(per_key, minlength=nb)
    return np.concatenate([[0], np.cumsum(cnt)[:-1]])


def _ws_view(ws, off, n, dtype):
    b = ws[off: off + n * np.dtype(dtype).itemsize].cpu().numpy()
    return b.view(dtype)


@pytest.mark.parametrize("nR,nS,bt,skew", [(1 << 17, 1 << 19, 1024, False), (1 << 19, 1 << 20, 256, False),
                                          (1 << 17, 1 << 19, 4096, True), (1 << 17, 1 << 19, 2048, "lognormal")])
def test_intermediate_results(nR, nS, bt, skew):
    rng = np.random.default_rng(nR + bt)
    R = rel(rng, nR, 1 << 24)
    S = rel(rng, nS, 1 << 24)
    if skew == "lognormal":   # heavy-tailed keys: the splitter directories take logarithmic cells
        R[:, 0] = np.floor(np.exp(2.0 * rng.standard_normal(nR)) * 2.0 ** 28).astype(np.uint64)
        S[:, 0] = R[rng.integers(0, nR, nS), 0]
    elif skew:   # S keys with a heavy head: frequent keys of one splitter get their own bucket
        base = np.unique(R[:, 0])
        S[:, 0] = base[(len(base) * rng.random(nS) ** 4).astype(np.int64)]
    cfg = mpsm.config(bucket_target=bt, log2_run_len=17)
    lay = mpsm.layout(nR, nS, cfg)
    ws = mpsm.alloc_workspace(nR, nS, cfg)
    got = gpu_join(R, S, cfg, workspace=ws)
    want = oracle.join(R, S)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    torch.cuda.synchronize()
    Q, L, NB = lay["runs"], lay["run_len"], lay["s_buckets"]
    Ssorted = _ws_view(ws, lay["off_s_sorted"], 2 * nS, np.uint64).reshape(-1, 2)
    ref_runs = oracle.sort_runs(S, L)
    # phase 1: every run sorted, same keys as the oracle's run sort, same tuples
    assert np.array_equal(Ssorted[:, 0], ref_runs[:, 0])
    for j in range(Q):
        a, b = j * L, min((j + 1) * L, nS)
        x = Ssorted[a:b]
        y = ref_runs[a:b]
        assert np.array_equal(x[np.lexsort((x[:, 1], x[:, 0]))], y[np.lexsort((y[:, 1], y[:, 0]))])
    # S splitters: valid splitters of the same seeded sample (the oracle's plain
    # equi-depth quantiles, or a quantile's predecessor + 1 where the kernel gave
    # a frequent key its own bucket), non-decreasing
    spl = _ws_view(ws, lay["off_s_splitters"], Q * (NB - 1), np.uint64).reshape(Q, NB - 1)
    for j in range(Q):
        seed = oracle.splitmix_at(lay["s_level_seed"], j)
        a, b = j * L, min((j + 1) * L, nS)
        _check_splitters(spl[j], oracle.sample_splitters(S[a:b], NB, lay["s_oversample"], seed))
    if skew is True:   # the frequent-key rule has fired: some splitter is its predecessor + 1
        assert np.count_nonzero(spl[:, 1:] == spl[:, :-1] + np.uint64(1)) > 0
    # S bucket boundaries: the oracle's stable partition of each run under the
    # GPU's own splitters, with the kernel's rule for keys equal to two or more
    # splitters applied here; every bucket boundary falls between distinct keys
    bst = _ws_view(ws, lay["off_s_bucket_start"], Q * NB + 1, np.uint32)
    for j in range(Q):
        a, b = j * L, min((j + 1) * L, nS)
        want = _bucket_starts_with_rule(S[a:b, 0], spl[j], NB)
        got = bst[j * NB:(j + 1) * NB].astype(np.int64) - a
        assert np.array_equal(got, want)
        inner = got[(got > 0) & (got < b - a)]
        assert np.all(ref_runs[a + inner - 1, 0] < ref_runs[a + inner, 0])
    # R level-1 splitters: valid splitters of R's seeded sample
    NB1 = lay["r_buckets1"]
    spl1 = _ws_view(ws, lay["off_r_splitters1"], NB1 - 1, np.uint64)
    _check_splitters(spl1, oracle.sample_splitters(R, NB1, lay["r_oversample1"],
                                                   oracle.splitmix_at(lay["r_level_seed1"], 0)))
    # R level-2 splitters (two levels): each level-1 bucket's first nb - 1
    # (nb: its length over 3/4 of the bucket target, rounded up, within
    # [1, r_buckets2]) are non-decreasing, inside the bucket's key range, and
    # each an R key or one above an R key (a splitter moved past a frequent
    # key).  They come from a sample of the bucket in the order the first
    # level's scatter left it, a buffer the join reuses, so they are judged by
    # these properties, not against the oracle's quantiles.
    NB2 = lay["r_buckets2"]
    if NB2 > 1:
        bst1 = _ws_view(ws, lay["off_r_bucket_start1"], NB1 + 1, np.uint32).astype(np.int64)
        spl2 = _ws_view(ws, lay["off_r_splitters2"], NB1 * (NB2 - 1), np.uint64).reshape(NB1, NB2 - 1)
        rkeys = np.unique(R[:, 0])
        bt2 = bt * 3 // 4
        for s1 in range(NB1):
            ln = int(bst1[s1 + 1] - bst1[s1])
            nb = min(max(-(-ln // bt2), 1), NB2)
            sp = spl2[s1, :nb - 1]
            lo = spl1[s1 - 1] if s1 > 0 else np.uint64(0)
            hi = spl1[s1] if s1 < NB1 - 1 else np.uint64(U64)
            assert np.all(sp[1:] >= sp[:-1]), s1
            assert np.all((sp >= lo) & (sp <= hi)), s1
            assert np.all(np.isin(sp, rkeys) | np.isin(sp - np.uint64(1), rkeys)), s1
    # phase 2+3: R sorted, partitions contiguous, first keys
    Rsorted = _ws_view(ws, lay["off_r_sorted"], 2 * nR, np.uint64).reshape(-1, 2)
    ref_R = oracle.sort_by_key(R)
    assert np.array_equal(Rsorted[:, 0], ref_R[:, 0])
    P = int(_ws_view(ws, lay["off_partitions"], 1, np.uint32)[0])
    pstart = _ws_view(ws, lay["off_part_start"], P, np.uint32).astype(np.int64)
    plen = _ws_view(ws, lay["off_part_len"], P, np.uint32).astype(np.int64)
    pkey = _ws_view(ws, lay["off_part_key"], P, np.uint64)
    assert pstart[0] == 0 and np.all(pstart[1:] == pstart[:-1] + plen[:-1]) and pstart[-1] + plen[-1] == nR
    assert np.array_equal(pkey, Rsorted[pstart, 0])
    assert np.all(Rsorted[pstart[1:] - 1, 0] < pkey[1:])          # key-disjoint partitions
    # join units: pairs (2i, 2i+1) that fit one LDS tile together, else singles
    span = _ws_view(ws, lay["off_join_span"], P, np.uint8).astype(np.int64)
    for p in range(P):
        pair = p % 2 == 0 and p + 1 < P and plen[p] + plen[p + 1] <= 8192
        second = p % 2 == 1 and plen[p - 1] + plen[p] <= 8192
        assert span[p] == (2 if pair else (0 if second else 1)), p
    heads = np.nonzero(span > 0)[0]
    # phase 4: start offsets are lower bounds of the first key of every unit's first partition
    o = _ws_view(ws, lay["off_offsets"], (P + 1) * Q, np.uint32).reshape(P + 1, Q)
    for j in range(Q):
        a, b = j * L, min((j + 1) * L, nS)
        ref = np.searchsorted(ref_runs[a:b, 0], pkey[heads], side="left")
        assert np.array_equal(o[heads, j], ref)
        assert o[P, j] == b - a
    # equi-height index: every idx_stride-th key of each run
    st, ipr = lay["idx_stride"], lay["idx_per_run"]
    idx = _ws_view(ws, lay["off_run_index"], Q * ipr, np.uint64).reshape(Q, ipr)
    for j in range(Q):
        a, b = j * L, min((j + 1) * L, nS)
        keys = ref_runs[a:b:st, 0]
        assert np.array_equal(idx[j, :len(keys)], keys)


# --------------------------------------------------- full-size workload

def test_fk_uniform_full_size_sampled():
    """The benchmark workload (|R| = 2^26, |S| = 2^28) in the benchmark's
    configuration: exact count and checksum from the foreign-key closed form,
    plus sampled runs and offsets against the oracle."""
    w = workloads.make("fk_uniform")
    nR, nS = len(w.R), len(w.S)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    cfg = mpsm.config()
    lay = mpsm.layout(nR, nS, cfg)
    ws = mpsm.alloc_workspace(nR, nS, cfg)
    got = gpu_join(w.R, w.S, cfg, workspace=ws)
    assert got["count"] == nS == fk.count
    assert got["checksum"] == fk.checksum
    torch.cuda.synchronize()
    Q, L = lay["runs"], lay["run_len"]
    rng = np.random.default_rng(1)
    for j in sorted(set([0, Q - 1] + rng.integers(0, Q, 2).tolist())):
        a, b = j * L, min((j + 1) * L, nS)
        x = _ws_view_range(ws, lay["off_s_sorted"], a, b)
        ref = oracle.sort_by_key(w.S[a:b])
        assert np.array_equal(x[:, 0], ref[:, 0])
        assert np.array_equal(x[np.lexsort((x[:, 1], x[:, 0]))], ref[np.lexsort((ref[:, 1], ref[:, 0]))])
        P = int(_ws_view(ws, lay["off_partitions"], 1, np.uint32)[0])
        pkey = _ws_view(ws, lay["off_part_key"], P, np.uint64)
        heads = np.nonzero(_ws_view(ws, lay["off_join_span"], P, np.uint8))[0]
        ps = heads[rng.integers(0, len(heads), 64)]
        o = _ws_view(ws, lay["off_offsets"], (P + 1) * Q, np.uint32).reshape(P + 1, Q)
        assert np.array_equal(o[ps, j], np.searchsorted(ref[:, 0], pkey[ps], side="left"))


def _ws_view_range(ws, off, a, b):
    return ws[off + 16 * a: off + 16 * b].cpu().numpy().view(np.uint64).reshape(-1, 2)


# ----------------------------------------- the two large workloads at full size

def _golden_full(name):
    import json
    import os
    from conftest import GOLDEN
    with open(os.path.join(GOLDEN, "full_size.json")) as f:
        return json.load(f)[name]


def _fingerprint(w):
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w.R[::4097]).tobytes())
    h.update(np.ascontiguousarray(w.S[::4099]).tobytes())
    return h.hexdigest()


def _sampled_runs_and_offsets(ws, lay, S_host, nS, seed, nruns=2):
    """Sampled S runs against the oracle's sort of the same chunk, and 64
    sampled start offsets per run against lower bounds in the oracle's run."""
    Q, L = lay["runs"], lay["run_len"]
    rng = np.random.default_rng(seed)
    P = int(_ws_view(ws, lay["off_partitions"], 1, np.uint32)[0])
    pkey = _ws_view(ws, lay["off_part_key"], P, np.uint64)
    heads = np.nonzero(_ws_view(ws, lay["off_join_span"], P, np.uint8))[0]
    o = _ws_view(ws, lay["off_offsets"], (P + 1) * Q, np.uint32).reshape(P + 1, Q)
    for j in sorted(set([0, Q - 1] + rng.integers(0, Q, nruns).tolist())):
        a, b = j * L, min((j + 1) * L, nS)
        x = _ws_view_range(ws, lay["off_s_sorted"], a, b)
        ref = oracle.sort_by_key(S_host[a:b])
        assert np.array_equal(x[:, 0], ref[:, 0])
        assert np.array_equal(x[np.lexsort((x[:, 1], x[:, 0]))], ref[np.lexsort((ref[:, 1], ref[:, 0]))])
        ps = heads[rng.integers(0, len(heads), 64)]
        assert np.array_equal(o[ps, j], np.searchsorted(ref[:, 0], pkey[ps], side="left"))
        _say(f"run {j}: sorted keys, tuples and 64 start offsets match the oracle")


@pytest.mark.timeout(900)
def test_skewed_full_size():
    """|R| = 2^26 keys from 64 Gaussian blobs, |S| = 2^28 Zipf(1.0) foreign
    keys, at full size in the plain and the learned form: count and checksum
    against the foreign-key closed form (computed here, and stored by the
    oracle-only script), plus sampled runs and start offsets."""
    g = _golden_full("skewed")
    w = workloads.make("skewed")
    assert _fingerprint(w) == g["inputs_sha256"], "the generator differs on this host"
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    assert (fk.count, fk.checksum) == (g["count"], int(g["checksum_hex"], 16))
    _say("skewed full: generated, closed form computed")
    nR, nS = len(w.R), len(w.S)
    R, S = _dev(w.R), _dev(w.S)
    cfg = mpsm.config()
    lay = mpsm.layout(nR, nS, cfg)
    ws = mpsm.alloc_workspace(nR, nS, cfg)
    got = mpsm.join(R, S, cfg, workspace=ws)
    assert (got["count"], got["checksum"]) == (fk.count, fk.checksum)
    torch.cuda.synchronize()
    _sampled_runs_and_offsets(ws, lay, w.S, nS, seed=2)
    learned = mpsm.join(R, S, mpsm.config(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED), workspace=ws)
    assert (learned["count"], learned["checksum"]) == (fk.count, fk.checksum)
    _say("skewed full: plain and learned equal the closed form")


@pytest.mark.timeout(900)
def test_lognormal_full_size():
    """|R| = 2^28 log-normal keys with duplicates, |S| = 2^30 (1..16 copies
    of every distinct key), at full size in the plain and the learned form
    and with bisection search: the count against the generator (exact by
    construction) and the checksum against the oracle's sort-merge join over
    key-range slices (stored by the oracle-only script), plus sampled runs
    and start offsets."""
    g = _golden_full("lognormal")
    w = workloads.make("lognormal")
    assert _fingerprint(w) == g["inputs_sha256"], "the generator differs on this host"
    assert w.expected_count == g["count"]
    want = (g["count"], int(g["checksum_hex"], 16))
    nR, nS = len(w.R), len(w.S)
    _say(f"lognormal full: generated |R|={nR} |S|={nS}, expected pairs {w.expected_count}")
    R, S = _dev(w.R), _dev(w.S)
    cfg = mpsm.config()
    lay = mpsm.layout(nR, nS, cfg)
    ws = mpsm.alloc_workspace(nR, nS, cfg)
    got = mpsm.join(R, S, cfg, workspace=ws)
    assert (got["count"], got["checksum"]) == want
    torch.cuda.synchronize()
    _sampled_runs_and_offsets(ws, lay, w.S, nS, seed=3)
    for kw in (dict(search=mpsm.SEARCH_BINARY), dict(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED)):
        other = mpsm.join(R, S, mpsm.config(**kw), workspace=ws)
        assert (other["count"], other["checksum"]) == want, kw
        _say(f"lognormal full: {kw} equals the oracle")


def test_lognormal_eighth_scale_against_oracle():
    """|R| = 2^25, |S| = 2^27 log-normal keys with duplicates: count and
    checksum against the oracle's join over key-range slices, computed here."""
    w = workloads.make("lognormal", scale_shift=3)
    got = gpu_join(w.R, w.S)
    assert got["count"] == w.expected_count
    smp = np.sort(w.R[np.random.default_rng(0).integers(0, len(w.R), 1 << 14), 0])
    want = oracle.join_sliced(w.R, w.S, np.unique(smp[(np.arange(1, 16) * len(smp)) // 16]), threads=16)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)


def test_pair_capacity_truncation():
    """Pairs asked for with too small a buffer: the count and checksum stay
    exact, the call reports MPSM_ECAPACITY through its status word, and the
    pairs written are capacity many of the oracle's pairs."""
    import collections
    rng = np.random.default_rng(31)
    R = rel(rng, 5000, 3000)
    S = rel(rng, 20000, 3000)
    want = oracle.join(R, S, pairs=True, cap=1 << 20)
    have = collections.Counter(map(tuple, want.pairs.tolist()))
    Rd, Sd = _dev(R), _dev(S)
    for cap in (1, 777, want.count - 1):
        got = mpsm.join(Rd, Sd, pairs=True, pairs_capacity=cap)
        assert got["status"] == "MPSM_ECAPACITY" and got["stats"]["pairs_truncated"] == 1
        assert (got["count"], got["checksum"]) == (want.count, want.checksum)
        assert len(got["pairs"]) == cap
        c = collections.Counter(map(tuple, got["pairs"].tolist()))
        assert all(have[p] >= k for p, k in c.items())
    got = mpsm.join(Rd, Sd, pairs=True, pairs_capacity=want.count)
    assert got["status"] == "MPSM_OK" and got["stats"]["pairs_truncated"] == 0
    assert np.array_equal(got["pairs"], want.pairs)


def test_cost_balanced_splitters_negatively_correlated():
    """The paper's hardest skew case (Section 4.3): 80% of R keys in the top
    20% of the key domain, 80% of S tuples in the bottom 20%.  Exact join;
    the GPU's S distribution at the sample keys equals the merge of the runs'
    equi-height bounds; its split reaches the optimum of the oracle's exact
    min-max dynamic program on the same cells (and beats equi-depth)."""
    rng = np.random.default_rng(0x8020)
    nR, nS, D = 1 << 15, 1 << 18, 1 << 32
    top = rng.random(nR) < 0.8
    rk = np.where(top, rng.integers(int(0.8 * D), D, nR), rng.integers(0, int(0.8 * D), nR)).astype(np.uint64)
    rk = np.unique(rk)
    rng.shuffle(rk)
    low = rk[rk < np.uint64(int(0.2 * D))]
    sk = np.where(rng.random(nS) < 0.8, low[rng.integers(0, len(low), nS)], rk[rng.integers(0, len(rk), nS)])
    R = np.stack([rk, rng.integers(0, U64, len(rk), dtype=np.uint64, endpoint=True)], 1)
    S = np.stack([sk.astype(np.uint64), rng.integers(0, U64, nS, dtype=np.uint64, endpoint=True)], 1)
    cfg = mpsm.config(splitter=mpsm.SPLIT_COST, log2_run_len=16)
    lay = mpsm.layout(len(R), nS, cfg)
    assert lay["levels"] == 1
    ws = mpsm.alloc_workspace(len(R), nS, cfg)
    got = gpu_join(R, S, cfg, workspace=ws)
    want = oracle.join(R, S)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    torch.cuda.synchronize()
    M, Q, L, NB = lay["cost_cells"], lay["runs"], lay["run_len"], lay["r_buckets1"]
    sample = _ws_view(ws, lay["off_cost_sample"], M, np.uint64)
    s_below = _ws_view(ws, lay["off_cost_s_below"], M + 1, np.uint64).astype(np.int64)
    best = float(_ws_view(ws, lay["off_cost_best"], 1, np.float64)[0])
    assert np.all(np.diff(sample.astype(np.float64)) >= 0)
    # the S distribution at the sample keys: within half a stride per run of the
    # exact count (each run's every-256th-key index brackets its count to one
    # stride, and the kernel takes the middle), and within the error bounds of
    # both of the oracle's Section 4.1 estimate (merged bounds, equal steps,
    # linear interpolation; Q strides)
    runs = oracle.sort_runs(S, L)
    run_start = [min(j * L, nS) for j in range(Q + 1)]
    exact = np.zeros(M, np.int64)
    for j in range(Q):
        a, b = run_start[j], run_start[j + 1]
        exact += np.searchsorted(runs[a:b, 0], sample, side="left")
    assert np.all(np.abs(s_below[:M] - exact) <= 128 * Q) and s_below[M] == nS
    cdf = oracle.s_cdf(runs, run_start, 256, sample)
    assert np.all(np.abs(s_below[:M] - cdf) <= 128 * Q + 256 * Q)
    # cells and the oracle's exact optimum
    RC = (np.arange(M + 1, dtype=np.uint64) * np.uint64(len(R))) // np.uint64(M)
    SC = np.concatenate([[0], s_below[1:]]).astype(np.uint64)
    h, s = np.diff(RC), np.diff(SC)
    opt, _ = oracle.cost_splitters_dp(h, s, P=NB, T=Q)
    # the kernel takes log2 in single precision (relative error about 2^-22)
    assert opt * (1 - 1e-6) <= best <= opt * 1.001, (best, opt)
    # equi-depth over the same cells (what sampled splitters do) is no better
    OS = M // NB
    equi = max(oracle.split_cost(int(h[g * OS:(g + 1) * OS].sum()), Q, int(s[g * OS:(g + 1) * OS].sum()))
               for g in range(NB))
    assert best <= equi * (1 + 1e-9)
    _say(f"cost split: best {best:.0f}, optimum {opt:.0f}, equi-depth {equi:.0f}")


# ------------------------------------ S runs scattered without a histogram

@pytest.mark.parametrize("oversample,expect_redo", [(0, None), (4, None), (2, True)])
def test_padded_s_scatter_and_its_exact_redo(oversample, expect_redo):
    """|S| = 2^22 takes the bucket pass without a histogram: buckets in
    regions sized from the sample.  With 2 sample keys per bucket the
    bounds are loose, the area scales them down and most runs overflow, so
    the exact path redoes them; with 4 some runs are redone and some not.
    Every run must still equal the oracle's sorted run (keys exactly,
    tuples as a multiset), and the join the foreign-key closed form."""
    w = workloads.fk_uniform(1 << 20, 1 << 22, seed=0x1207014500000a01, spread=True)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    cfg = mpsm.config(oversample=oversample, log2_run_len=16)
    lay = mpsm.layout(len(w.R), len(w.S), cfg)
    ws = mpsm.alloc_workspace(len(w.R), len(w.S), cfg)
    _say(f"padded S scatter: oversample {oversample}, {lay['runs']} runs")
    got = mpsm.join(_dev(w.R), _dev(w.S), cfg, workspace=ws, with_stats=True)
    assert (got["count"], got["checksum"]) == (fk.count, fk.checksum)
    redone = got["stats"]["redone_runs"]
    _say(f"redone runs: {redone} of {lay['runs']}")
    if expect_redo:
        assert redone > 0
    torch.cuda.synchronize()
    L, Q = lay["run_len"], lay["runs"]
    U = _ws_view(ws, lay["off_s_sorted"], 2 * len(w.S), np.uint64).reshape(-1, 2)
    ref = oracle.sort_runs(w.S, L)
    assert np.array_equal(U[:, 0], ref[:, 0])
    for j in range(Q):
        a, b = j * L, (j + 1) * L
        x, y = U[a:b], ref[a:b]
        assert np.array_equal(x[np.lexsort((x[:, 1], x[:, 0]))], y[np.lexsort((y[:, 1], y[:, 0]))]), j


@pytest.mark.parametrize("form,oversample", [("sampled", 0), ("sampled", 2), ("learned", 0), ("learned", 3)])
def test_padded_r_levels_and_their_exact_redo(form, oversample):
    """|R| = 2^23 takes two partitioning levels; the second (one segment
    per first-level bucket) has no histogram.  Few sample keys per bucket
    make regions overflow and segments go through the exact path.  R sorted
    and its partitions must equal the oracle's, and the join the
    foreign-key closed form."""
    w = workloads.fk_uniform(1 << 23, 1 << 24, seed=0x1207014500000b01, spread=True)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    kw = dict(splitter=mpsm.SPLIT_LEARNED) if form == "learned" else {}
    cfg = mpsm.config(oversample=oversample, **kw)
    lay = mpsm.layout(len(w.R), len(w.S), cfg)
    assert lay["levels"] == 2
    assert lay["padded_passes"] == 5
    ws = mpsm.alloc_workspace(len(w.R), len(w.S), cfg)
    _say(f"padded R levels: form {form}, oversample {oversample}")
    got = mpsm.join(_dev(w.R), _dev(w.S), cfg, workspace=ws, with_stats=True)
    assert (got["count"], got["checksum"]) == (fk.count, fk.checksum)
    _say(f"redone: S runs {got['stats']['redone_runs']}, R segments {got['stats']['redone_r_segments']}")
    if oversample == 2:
        assert got["stats"]["redone_r_segments"] > 0
    torch.cuda.synchronize()
    nR = len(w.R)
    Rsorted = _ws_view(ws, lay["off_r_sorted"], 2 * nR, np.uint64).reshape(-1, 2)
    ref_R = oracle.sort_by_key(w.R)
    assert np.array_equal(Rsorted[:, 0], ref_R[:, 0])
    assert np.array_equal(Rsorted[np.lexsort((Rsorted[:, 1], Rsorted[:, 0]))],
                          ref_R[np.lexsort((ref_R[:, 1], ref_R[:, 0]))])
    P = int(_ws_view(ws, lay["off_partitions"], 1, np.uint32)[0])
    pstart = _ws_view(ws, lay["off_part_start"], P, np.uint32).astype(np.int64)
    plen = _ws_view(ws, lay["off_part_len"], P, np.uint32).astype(np.int64)
    assert pstart[0] == 0 and np.all(pstart[1:] == pstart[:-1] + plen[:-1]) and pstart[-1] + plen[-1] == nR
    assert np.all(Rsorted[pstart[1:] - 1, 0] < Rsorted[pstart[1:], 0])
    # level-1 bucket starts (compact positions, whether or not the pass had
    # regions): the sorted R falls into the level-1 buckets in order, each
    # bucket's keys within its splitters
    NB1 = lay["r_buckets1"]
    spl1 = _ws_view(ws, lay["off_r_splitters1"], NB1 - 1, np.uint64)
    bst1 = _ws_view(ws, lay["off_r_bucket_start1"], NB1 + 1, np.uint32).astype(np.int64)
    assert bst1[0] == 0 and bst1[-1] == nR and np.all(np.diff(bst1) >= 0)
    for b in range(NB1):
        keys = Rsorted[bst1[b]:bst1[b + 1], 0]
        if len(keys):
            assert b == 0 or keys[0] >= spl1[b - 1], b
            assert b == NB1 - 1 or keys[-1] <= spl1[b], b


@pytest.mark.parametrize("oversample", [0, 2])
def test_padded_bmpsm_runs(oversample):
    """B-MPSM with |R| = 2^22: R's runs, like S's, without a histogram; with
    2 sample keys per bucket runs of both are redone by the exact path."""
    w = workloads.fk_uniform(1 << 22, 1 << 22, seed=0x1207014500000c01, spread=True)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    cfg = mpsm.config(splitter=mpsm.SPLIT_NONE, role=mpsm.ROLE_AS_GIVEN, oversample=oversample, log2_run_len=20)
    lay = mpsm.layout(len(w.R), len(w.S), cfg)
    assert lay["padded_passes"] == 3
    _say(f"padded B-MPSM runs: oversample {oversample}")
    got = mpsm.join(_dev(w.R), _dev(w.S), cfg, with_stats=True)
    assert (got["count"], got["checksum"]) == (fk.count, fk.checksum)
    st = got["stats"]
    _say(f"redone: S runs {st['redone_runs']}, R runs {st['redone_r_segments']}")
    if oversample == 2:
        assert st["redone_runs"] > 0 and st["redone_r_segments"] > 0


@pytest.mark.parametrize("nR,nS", [((1 << 22) + 777, (1 << 22) + 12345), ((1 << 22) - 1, 1 << 22)])
def test_padded_passes_at_ragged_sizes(nR, nS):
    """Sizes at and around the threshold of the passes without a histogram
    (2^22), with a ragged last run and ragged level-1 buckets: the join
    equals the oracle's, S's runs and R's order equal the oracle's sorts."""
    rng = np.random.default_rng(nR ^ nS)
    R = rel(rng, nR, 1 << 40)
    S = rel(rng, nS, 1 << 40)
    S[: nS // 2, 0] = R[rng.integers(0, nR, nS // 2), 0]
    cfg = mpsm.config()
    lay = mpsm.layout(nR, nS, cfg)
    _say(f"ragged padded sizes nR={nR} nS={nS}: passes {lay['padded_passes']}, levels {lay['levels']}")
    assert lay["padded_passes"] & 1 == (1 if nS >= (1 << 22) else 0)
    assert (lay["padded_passes"] >> 2) & 1 == (1 if nR >= (1 << 22) and lay["levels"] == 2 else 0)
    ws = mpsm.alloc_workspace(nR, nS, cfg)
    got = gpu_join(R, S, cfg, workspace=ws)
    want = oracle.join(R, S)
    assert (got["count"], got["checksum"]) == (want.count, want.checksum)
    torch.cuda.synchronize()
    L = lay["run_len"]
    Ssorted = _ws_view(ws, lay["off_s_sorted"], 2 * nS, np.uint64).reshape(-1, 2)
    assert np.array_equal(Ssorted[:, 0], oracle.sort_runs(S, L)[:, 0])
    Rsorted = _ws_view(ws, lay["off_r_sorted"], 2 * nR, np.uint64).reshape(-1, 2)
    assert np.array_equal(Rsorted[:, 0], np.sort(R[:, 0]))
