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


# ------------------------------------------- device descriptors (mpsm_join_batch)

def _device_batch(cases_list, waves=0):
    """Descriptor array, outputs and workspace sized for every batch in
    cases_list (same number of joins each)."""
    n = len(cases_list[0])
    sums = [(sum(len(R) for R, S in c if len(R) and len(S)), sum(len(S) for R, S in c if len(R) and len(S)),
             max([len(S) for R, S in c if len(R) and len(S)] or [0])) for c in cases_list]
    shape = mpsm.batch_shape(max(s[0] for s in sums), max(s[1] for s in sums), max(s[2] for s in sums))
    cfg = mpsm.config(waves=waves)
    ws = torch.empty(mpsm.join_batch_workspace_bytes(n, shape, cfg), dtype=torch.uint8, device="cuda")
    descs = torch.zeros((n, 7), dtype=torch.int64, device="cuda")
    out = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    times = torch.zeros((n, 3), dtype=torch.int64, device="cuda")
    return shape, cfg, ws, descs, out, times


def _results(out):
    return [(c & U64, s & U64) for c, s in out.cpu().tolist()]


def test_join_batch_device_descriptors_graph_replayed_over_new_batches():
    """One call over a device descriptor array; the call captured once into
    a graph and replayed for other batches written into the same array
    (same count, within the shape's bounds), with eager work and
    synchronisation between replays; every replay against the oracle."""
    n = 20
    rng = np.random.default_rng(11)
    batches = []
    for k, (lo, hi) in enumerate([(8, 16), (10, 17), (6, 15)]):
        c = _batch_cases(n - 7, 0x1207014500000401 + k, lo, hi)
        order = rng.permutation(len(c))        # empty and edge joins at varying places
        batches.append([c[i] for i in order])
    shape, cfg, ws, descs, out, times = _device_batch(batches)
    dev = [[(_dev(R), _dev(S)) for R, S in c] for c in batches]
    # eager, first batch (also creates the library's second stream)
    mpsm.write_descs(descs, dev[0], out, times)
    _say(f"mpsm_join_batch eager: n={n} shape=({shape.max_sum_nR}, {shape.max_sum_nS}, {shape.max_nS})")
    mpsm.join_batch(descs, n, shape, ws, cfg)
    torch.cuda.synchronize()
    assert int(ws[:4].view(torch.int32).item()) == 0
    _check_results(batches[0], _results(out))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mpsm.join_batch(descs, n, shape, ws, cfg, stream=torch.cuda.current_stream())
    x = torch.randn(256, 256, device="cuda")
    for rep, k in enumerate([1, 2, 0, 1]):
        mpsm.write_descs(descs, dev[k], out, times)
        out.fill_(-1)
        _ = (x @ x).sum().item()
        _say(f"graph replay {rep}: batch {k}")
        g.replay()
        torch.cuda.synchronize()
        assert int(ws[:4].view(torch.int32).item()) == 0
        _check_results(batches[k], _results(out))


def test_join_batch_waves_finish_small_joins_first():
    """With four waves the smallest quarter of the joins (by nR + nS)
    finishes before the largest quarter starts its join work."""
    cases = _batch_cases(32, 0x1207014500000501, 6, 18)[:32]
    shape, cfg, ws, descs, out, times = _device_batch([cases], waves=4)
    dev = [(_dev(R), _dev(S)) for R, S in cases]
    mpsm.write_descs(descs, dev, out, times)
    mpsm.join_batch(descs, len(cases), shape, ws, cfg)
    torch.cuda.synchronize()
    _check_results(cases, _results(out))
    t = times.cpu().numpy().view(np.uint64)
    work = np.array([len(R) + len(S) if len(R) and len(S) else 0 for R, S in cases])
    order = [i for i in np.argsort(work, kind="stable") if work[i]]
    q = len(order) // 4
    small, large = order[:q], order[-q:]
    assert t[small, 2].max() < t[large, 1].min()
    assert np.all(t[:, 0] == t[0, 0])


def test_join_batch_device_check_rejects_out_of_bounds_batch():
    """A batch whose join exceeds the shape's per-join bound: status word
    MPSM_EINVAL, no output written."""
    cases = _batch_cases(6, 0x1207014500000601, 8, 12)
    shape, cfg, ws, descs, out, times = _device_batch([cases])
    bad = list(cases)
    rng = np.random.default_rng(5)
    big = int(shape.max_nS) + 1
    bad[0] = (bad[0][0] if len(bad[0][0]) else np.ones((3, 2), np.uint64),
              np.stack([rng.integers(0, 10, big, dtype=np.uint64), np.zeros(big, np.uint64)], 1))
    mpsm.write_descs(descs, [(_dev(R), _dev(S)) for R, S in bad], out, times)
    out.fill_(-7)
    mpsm.join_batch(descs, len(bad), shape, ws, cfg)
    torch.cuda.synchronize()
    assert int(ws[:4].view(torch.int32).item()) == 1
    assert bool((out == -7).all())


@pytest.mark.parametrize("oversample", [0, 2])
def test_batch_passes_without_histogram(oversample):
    """A batch whose S and R sums pass 2^22 takes the passes without a
    histogram over every join's runs and R segment; with 2 sample keys per
    bucket regions overflow and segments are redone by the exact path.  Every
    join against the foreign-key closed form, eager and graph-replayed."""
    ws_ = workloads.batch(24, 0x1207014500000d01 + oversample, 17, 20)
    nS = sum(len(w.S) for w in ws_)
    nR = sum(len(w.R) for w in ws_)
    assert nS >= (1 << 22) and nR >= (1 << 22)
    _say(f"batch without histograms: {len(ws_)} joins, sum |R| {nR}, sum |S| {nS}, oversample {oversample}")
    joins = [(_dev(w.R), _dev(w.S)) for w in ws_]
    b = mpsm.Batch(joins, mpsm.config(oversample=oversample))
    for use_graph in (False, True, True):
        b.out.zero_()
        b.run(use_graph=use_graph)
        torch.cuda.synchronize()
        got = b.results()
        for i, w in enumerate(ws_):
            fk = oracle.fk_closed_form(w.R, w.S, w.partner)
            assert got[i] == (fk.count, fk.checksum), (w.name, use_graph)
    b.close()
