"""GPU parity of the batched launch (mpsm_batch_*): every join of a batch
against the CPU oracle, eager and graph-replayed, plus the autotuner."""
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


def _edge_joins(rng):
    """Empty sides, single tuples, one shared key, disjoint key ranges."""
    def rel(n, keys):
        return np.stack([np.asarray(keys, np.uint64), rng.integers(0, U64, n, dtype=np.uint64, endpoint=True)], 1)
    e = np.zeros((0, 2), np.uint64)
    return [
        (e, rel(5, [1, 2, 3, 4, 5])),
        (rel(5, [1, 2, 3, 4, 5]), e),
        (e, e),
        (rel(1, [7]), rel(1, [7])),
        (rel(3000, np.full(3000, 42)), rel(5000, np.full(5000, 42))),
        (rel(4000, np.arange(4000)), rel(4000, np.arange(4000) + 10 ** 6)),
        (rel(2, [0, U64]), rel(4, [U64, 0, U64, 5])),
    ]


def _batch_cases(n_join, seed, lo, hi):
    ws = workloads.batch(n_join, seed, lo, hi)
    rng = np.random.default_rng(seed)
    return [(w.R, w.S) for w in ws] + _edge_joins(rng)


def _check_results(cases, got):
    for i, ((R, S), (c, s)) in enumerate(zip(cases, got)):
        want = oracle.join(R, S)
        assert (c, s) == (want.count, want.checksum), f"join {i}: |R|={len(R)} |S|={len(S)}"


@pytest.mark.parametrize("search", [mpsm.SEARCH_INDEX, mpsm.SEARCH_BINARY, mpsm.SEARCH_INTERP])
def test_batch_matches_oracle(search):
    cases = _batch_cases(40, 0x1207014500000101 + search, 6, 16)
    _say(f"batch of {len(cases)} joins, search {search}, |S| total {sum(len(s) for _, s in cases)}")
    joins = [(_dev(R), _dev(S)) for R, S in cases]
    b = mpsm.Batch(joins, mpsm.config(search=search))
    b.run()
    torch.cuda.synchronize()
    _check_results(cases, b.results())
    t = b.times.cpu().numpy().view(np.uint64)
    assert np.all(t[:, 0] == t[0, 0])
    assert np.all(t[:, 1] >= t[:, 0]) and np.all(t[:, 2] >= t[:, 1])
    b.close()


def test_batch_graph_replays_match_eager():
    """The captured graph is replayed several times with eager work and
    synchronisation in between; every replay must give the oracle's results."""
    cases = _batch_cases(24, 0x1207014500000201, 8, 17)
    joins = [(_dev(R), _dev(S)) for R, S in cases]
    b = mpsm.Batch(joins)
    b.run()
    torch.cuda.synchronize()
    eager = b.results()
    _check_results(cases, eager)
    x = torch.randn(512, 512, device="cuda")
    for rep in range(4):
        b.out.zero_()
        _ = (x @ x).sum().item()            # unrelated eager work between replays
        b.run(use_graph=True)
        torch.cuda.synchronize()
        assert b.results() == eager, f"replay {rep}"
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b.out.zero_()
        b.run(use_graph=True, stream=side)
    side.synchronize()
    assert b.results() == eager
    b.close()


def test_batch_tunings_agree_and_autotune_caches(tmp_path):
    cases = _batch_cases(16, 0x1207014500000301, 8, 18)
    joins = [(_dev(R), _dev(S)) for R, S in cases]
    b = mpsm.Batch(joins)
    want = None
    for lg, bt, jc in [(16, 2048, 16384), (18, 4096, 65536), (20, 2048, 65536)]:
        b.set_tuning(lg, bt, jc)
        b.run()
        torch.cuda.synchronize()
        got = b.results()
        want = want or got
        assert got == want, (lg, bt, jc)
    _check_results(cases, want)
    cache = str(tmp_path / "tune.txt")
    t1 = b.autotune(cache)
    assert t1["from_cache"] == 0 and t1["ms"] > 0
    b.run()
    torch.cuda.synchronize()
    assert b.results() == want
    b2 = mpsm.Batch(joins)
    t2 = b2.autotune(cache)
    assert t2["from_cache"] == 1
    assert (t2["log2_run_len"], t2["bucket_target"], t2["join_chunk"]) == \
        (t1["log2_run_len"], t1["bucket_target"], t1["join_chunk"])
    b.close()
    b2.close()


def test_batch_full_size_config():
    """The 256-join workload at full size: every join's count and checksum
    from the foreign-key closed form."""
    ws = workloads.make("batch")
    _say(f"batch 256 joins: |R| total {sum(len(w.R) for w in ws)}, |S| total {sum(len(w.S) for w in ws)}")
    joins = [(_dev(w.R), _dev(w.S)) for w in ws]
    b = mpsm.Batch(joins)
    b.run(use_graph=True)
    torch.cuda.synchronize()
    got = b.results()
    for i, w in enumerate(ws):
        fk = oracle.fk_closed_form(w.R, w.S, w.partner)
        assert got[i] == (fk.count, fk.checksum), w.name
    b.close()
