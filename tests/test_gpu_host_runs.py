"""GPU parity of the join with S in host memory (the memory-constrained
variant of Section 3.1, its runs kept in pinned host memory instead of on
disk): count and checksum against the oracle's join, and the runs it leaves
in host memory against the oracle's sorted runs (keys position by position,
tuples as a multiset per run, since equal keys may come in any order).  Its
join phase on its own, over runs already in host memory (sorted by the
oracle, or left by an earlier call), against the oracle's join too."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1207_0145_amd as mpsm
import workloads

pytestmark = pytest.mark.gpu
U64 = (1 << 64) - 1


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _dev(a):
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1, 2)
    return torch.from_numpy(a.view(np.int64)).to("cuda")


def _pinned(a):
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1, 2)
    t = torch.empty((len(a), 2), dtype=torch.int64, pin_memory=True)
    t.copy_(torch.from_numpy(a.view(np.int64)))
    return t


def rel(rng, n, domain):
    k = (rng.integers(0, domain, size=n, dtype=np.uint64) if domain
         else rng.integers(0, U64, size=n, dtype=np.uint64, endpoint=True))
    p = rng.integers(0, U64, size=n, dtype=np.uint64, endpoint=True)
    return np.stack([k, p], axis=1)


def host_join(R, S, chunk, cfg=None, keep_runs=True):
    cfg = cfg if cfg is not None else mpsm.config()
    nR, nS = len(R), len(S)
    _say(f"mpsm_join_host_runs nR={nR} nS={nS} chunk={chunk} L=2^{cfg.log2_run_len or 'default'} "
         f"splitter={cfg.splitter} search={cfg.search}")
    nbytes = mpsm.join_host_runs_workspace_bytes(nR, nS, chunk, cfg)
    assert nbytes > 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    Sh = _pinned(S)
    runs = torch.empty((nS, 2), dtype=torch.int64, pin_memory=True) if keep_runs else None
    mpsm.join_host_runs_into(_dev(R), Sh, runs, out, ws, chunk, cfg)
    torch.cuda.synchronize()
    o = out.cpu().numpy().view(np.uint64)
    return int(o[0]), int(o[1]), runs.numpy().view(np.uint64) if keep_runs else None


def check_runs(S, runs, L):
    want = oracle.sort_runs(S, L)
    assert np.array_equal(runs[:, 0], want[:, 0])
    for q in range(0, len(S), L):
        a, b = runs[q:q + L], want[q:q + L]
        assert np.array_equal(a[np.lexsort((a[:, 1], a[:, 0]))], b[np.lexsort((b[:, 1], b[:, 0]))]), q


@pytest.mark.parametrize("nR,nS,domain,chunk", [
    (5000, 100000, 3000, 3 * 4096),    # 9 chunks, the last one ragged, runs of 2^12
    (5000, 100000, 0, 1 << 30),        # one chunk holds all of S
    (3000, 50001, 500, 1000),          # chunk below a run: one run at a time
    (20000, 4095, 100, 4096),          # S shorter than one run
])
def test_host_runs_small(nR, nS, domain, chunk):
    rng = np.random.default_rng(nR + nS + domain)
    R, S = rel(rng, nR, domain), rel(rng, nS, domain)
    cfg = mpsm.config(log2_run_len=12)
    cnt, chk, runs = host_join(R, S, chunk, cfg)
    want = oracle.join(R, S)
    assert (cnt, chk) == (want.count, want.checksum)
    check_runs(S, runs, 1 << 12)


def test_host_runs_not_kept():
    """No buffer for the runs: the same result, over 9 chunks and one."""
    rng = np.random.default_rng(123)
    R, S = rel(rng, 6000, 2500), rel(rng, 90000, 2500)
    want = oracle.join(R, S)
    for chunk in (10000, 1 << 20):
        cnt, chk, runs = host_join(R, S, chunk, mpsm.config(log2_run_len=12), keep_runs=False)
        assert (cnt, chk) == (want.count, want.checksum) and runs is None


@pytest.mark.parametrize("kw", [dict(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED),
                                dict(search=mpsm.SEARCH_BINARY), dict(search=mpsm.SEARCH_INTERP)])
def test_host_runs_options(kw):
    rng = np.random.default_rng(77)
    R, S = rel(rng, 30000, 20000), rel(rng, 200000, 20000)
    cfg = mpsm.config(log2_run_len=13, **kw)
    cnt, chk, runs = host_join(R, S, 5 * 8192, cfg)
    want = oracle.join(R, S)
    assert (cnt, chk) == (want.count, want.checksum)
    check_runs(S, runs, 1 << 13)


@pytest.mark.parametrize("nR,nS", [(0, 1000), (1000, 0), (0, 0)])
def test_host_runs_empty(nR, nS):
    rng = np.random.default_rng(nR + 3 * nS)
    R, S = rel(rng, nR, 10), rel(rng, nS, 10)
    cnt, chk, _ = host_join(R, S, 4096, mpsm.config(log2_run_len=12))
    assert (cnt, chk) == (0, 0)


@pytest.mark.parametrize("chunk", [1 << 22, 1 << 21])
def test_host_runs_lognormal_reduced(chunk):
    """|R| = 2^20, |S| = 2^22 log-normal keys with duplicates, default runs
    (2^16 tuples): a chunk of all 64 runs (2^22 tuples) takes the pass
    without a histogram, a chunk of 32 the counted one."""
    w = workloads.make("lognormal", scale_shift=8)
    want, inv = oracle.join_hash(w.R, w.S)
    cnt, chk, runs = host_join(w.R, w.S, chunk)
    assert cnt == w.expected_count == inv and chk == want.checksum
    L = 1 << 16
    assert np.array_equal(runs[:, 0], oracle.sort_runs(w.S, L)[:, 0])


def test_host_runs_matches_device_join():
    """fk_uniform at |R| = 2^20, |S| = 2^22 (every S tuple has one partner):
    the same count and checksum as the join with S in device memory and as
    the closed form."""
    w = workloads.make("fk_small")
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    dev = mpsm.join(_dev(w.R), _dev(w.S))
    cnt, chk, _ = host_join(w.R, w.S, 3 << 20)
    assert (cnt, chk) == (dev["count"], dev["checksum"]) == (len(w.S), fk.checksum)


def test_host_runs_rejects():
    """Options that need S's runs before R's partitioning, a swapped role,
    chunk 0 and a host buffer that is not pinned: MPSM_EINVAL before anything
    is enqueued; a join afterwards still runs."""
    L = mpsm.lib()
    rng = np.random.default_rng(5)
    R, S = rel(rng, 1000, 50), rel(rng, 5000, 50)
    Rd, Sh = _dev(R), _pinned(S)
    runs = torch.empty_like(Sh).pin_memory()
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    ws = torch.empty(mpsm.join_host_runs_workspace_bytes(1000, 5000, 4096), dtype=torch.uint8, device="cuda")

    def call(cfg, chunk, s_ptr, runs_ptr):
        return L.mpsm_join_host_runs(ctypes.c_void_p(Rd.data_ptr()), 1000, ctypes.c_void_p(s_ptr), 5000,
                                     ctypes.c_void_p(runs_ptr), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr() + 8), ctypes.byref(cfg), chunk,
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)

    for kw in (dict(splitter=mpsm.SPLIT_COST), dict(splitter=mpsm.SPLIT_NONE), dict(role=mpsm.ROLE_SWAP)):
        assert call(mpsm.config(**kw), 4096, Sh.data_ptr(), runs.data_ptr()) == 1, kw
    assert call(mpsm.config(), 0, Sh.data_ptr(), runs.data_ptr()) == 1
    plain = np.ascontiguousarray(S.copy())
    assert call(mpsm.config(), 4096, plain.ctypes.data, runs.data_ptr()) == 1
    with pytest.raises(TypeError):
        mpsm.join_host_runs_into(Rd, torch.from_numpy(S.view(np.int64)), runs, out, ws, 4096)
    cnt, chk, _ = host_join(R, S, 4096, mpsm.config(log2_run_len=12))
    want = oracle.join(R, S)
    assert (cnt, chk) == (want.count, want.checksum)


def test_host_runs_back_to_back():
    """Two calls on one stream and one workspace with no synchronisation
    between them (the second with fewer tuples and other chunks): both
    results and both sets of runs are the oracle's."""
    rng = np.random.default_rng(99)
    cases = [(rel(rng, 7000, 4000), rel(rng, 120000, 4000), 2 * 4096),
             (rel(rng, 3000, 900), rel(rng, 70001, 900), 5 * 4096)]
    cfg = mpsm.config(log2_run_len=12)
    nbytes = max(mpsm.join_host_runs_workspace_bytes(len(R), len(S), ch, cfg) for R, S, ch in cases)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    outs, runs, keep = [], [], []
    for R, S, ch in cases:
        _say(f"back to back: nR={len(R)} nS={len(S)} chunk={ch}")
        Rd, Sh = _dev(R), _pinned(S)
        rh = torch.empty((len(S), 2), dtype=torch.int64, pin_memory=True)
        out = torch.zeros(2, dtype=torch.int64, device="cuda")
        mpsm.join_host_runs_into(Rd, Sh, rh, out, ws, ch, cfg)
        outs.append(out)
        runs.append(rh)
        keep.append((Rd, Sh))
    torch.cuda.synchronize()
    for (R, S, _), out, rh in zip(cases, outs, runs):
        o = out.cpu().numpy().view(np.uint64)
        want = oracle.join(R, S)
        assert (int(o[0]), int(o[1])) == (want.count, want.checksum)
        check_runs(S, rh.numpy().view(np.uint64), 1 << 12)


def spilled_join(R, runs_host, cfg=None):
    cfg = cfg if cfg is not None else mpsm.config()
    _say(f"mpsm_join_spilled_runs nR={len(R)} nS={runs_host.shape[0]} L=2^{cfg.log2_run_len or 'default'} "
         f"splitter={cfg.splitter} search={cfg.search}")
    ws = torch.empty(mpsm.join_spilled_runs_workspace_bytes(len(R), runs_host.shape[0], cfg), dtype=torch.uint8,
                     device="cuda")
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    mpsm.join_spilled_runs_into(_dev(R), runs_host, out, ws, cfg)
    torch.cuda.synchronize()
    o = out.cpu().numpy().view(np.uint64)
    return int(o[0]), int(o[1])


@pytest.mark.parametrize("kw", [dict(), dict(search=mpsm.SEARCH_BINARY), dict(search=mpsm.SEARCH_INTERP),
                                dict(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED)])
def test_spilled_runs_from_the_oracle(kw):
    """Runs sorted by the oracle (ragged last run) in pinned host memory,
    joined with an R the GPU partitions: the oracle's count and checksum."""
    rng = np.random.default_rng(404)
    R, S = rel(rng, 20000, 9000), rel(rng, 150001, 9000)
    cfg = mpsm.config(log2_run_len=12, **kw)
    runs = _pinned(oracle.sort_runs(S, 1 << 12))
    want = oracle.join(R, S)
    assert spilled_join(R, runs, cfg) == (want.count, want.checksum)


def test_spilled_runs_rejoined():
    """The runs one host-memory join leaves behind, joined again with two
    other R: each the oracle's result against S, with S never sorted again."""
    rng = np.random.default_rng(405)
    S = rel(rng, 300000, 50000)
    R0, R1, R2 = rel(rng, 40000, 50000), rel(rng, 7000, 50000), rel(rng, 90000, 60000)
    cnt, chk, runs = host_join(R0, S, 3 << 16)
    want = oracle.join(R0, S)
    assert (cnt, chk) == (want.count, want.checksum)
    runs_pinned = _pinned(runs)
    for R in (R1, R2):
        want = oracle.join(R, S)
        assert spilled_join(R, runs_pinned) == (want.count, want.checksum)


@pytest.mark.parametrize("nR,nS", [(0, 5000), (5000, 0)])
def test_spilled_runs_empty(nR, nS):
    rng = np.random.default_rng(406)
    R, S = rel(rng, nR, 100), rel(rng, nS, 100)
    runs = _pinned(oracle.sort_runs(S, 1 << 12)) if nS else torch.empty((0, 2), dtype=torch.int64)
    assert spilled_join(R, runs, mpsm.config(log2_run_len=12)) == (0, 0)


def test_host_runs_fk_uniform_full_size():
    """The benchmark's fk_uniform workload (|R| = 2^26, |S| = 2^28) with S in
    pinned host memory, in 2^24-tuple chunks as the bench times it: count and
    checksum from the foreign-key closed form, four of the runs it leaves in
    host memory against the oracle's sort, and the join phase over those runs
    with the same result."""
    w = workloads.make("fk_uniform")
    nR, nS = len(w.R), len(w.S)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    cfg = mpsm.config()
    L = mpsm.layout(nR, nS, mpsm.config(role=mpsm.ROLE_AS_GIVEN))["run_len"]
    _say(f"host runs full size: nR={nR} nS={nS} L={L} chunk=2^24")
    Rd = _dev(w.R)
    Sh = _pinned(w.S)
    runs = torch.empty((nS, 2), dtype=torch.int64, pin_memory=True)
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    ws = torch.empty(mpsm.join_host_runs_workspace_bytes(nR, nS, 1 << 24, cfg), dtype=torch.uint8, device="cuda")
    mpsm.join_host_runs_into(Rd, Sh, runs, out, ws, 1 << 24, cfg)
    torch.cuda.synchronize()
    o = out.cpu().numpy().view(np.uint64)
    assert (int(o[0]), int(o[1])) == (nS, fk.checksum) == (fk.count, fk.checksum)
    rv = runs.numpy().view(np.uint64)
    Q = (nS + L - 1) // L
    for j in sorted({0, 17, Q // 2, Q - 1}):
        a, b = j * L, min((j + 1) * L, nS)
        ref = oracle.sort_by_key(w.S[a:b])
        x = rv[a:b]
        assert np.array_equal(x[:, 0], ref[:, 0])
        assert np.array_equal(x[np.lexsort((x[:, 1], x[:, 0]))], ref[np.lexsort((ref[:, 1], ref[:, 0]))])
    del ws
    _say("host runs full size: the join phase over the spilled runs")
    ws = torch.empty(mpsm.join_spilled_runs_workspace_bytes(nR, nS, cfg), dtype=torch.uint8, device="cuda")
    out.zero_()
    mpsm.join_spilled_runs_into(Rd, runs, out, ws, cfg)
    torch.cuda.synchronize()
    o = out.cpu().numpy().view(np.uint64)
    assert (int(o[0]), int(o[1])) == (fk.count, fk.checksum)
