"""mpsm_join_noalloc (the join with the library's own fixed per-GPU
workspace) against mpsm_join with a caller workspace and against the CPU
oracle: bit-identical count, checksum and pair lists, on two calls in a row
(the second smaller, so that it runs over what the first left in the
array), plus the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1207_0145_amd as mpsm

U64 = (1 << 64) - 1


def _rel(rng, n, domain):
    k = rng.integers(0, domain, size=n, dtype=np.uint64)
    p = rng.integers(0, U64, size=n, dtype=np.uint64, endpoint=True)
    return np.stack([k, p], axis=1)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to("cuda")


def _u64(t):
    return [v & U64 for v in t.cpu().tolist()]


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.mark.gpu
@pytest.mark.parametrize("cfg_kw", [{}, {"splitter": mpsm.SPLIT_LEARNED, "search": mpsm.SEARCH_LEARNED}])
def test_noalloc_two_calls_match_mpsm_join(cfg_kw):
    rng = np.random.default_rng(77)
    cases = [(300_000, 1_000_000, 1 << 20), (20_000, 70_001, 9000)]   # second call smaller
    assert mpsm.workspace_bytes(*cases[0][:2]) <= mpsm.NOALLOC_SCRATCH_BYTES
    cfg = mpsm.config(**cfg_kw)
    for nR, nS, dom in cases:
        _say(f"mpsm_join_noalloc nR={nR} nS={nS} domain={dom} cfg={cfg_kw}")
        R, S = _rel(rng, nR, dom), _rel(rng, nS, dom)
        Rd, Sd = _dev(R), _dev(S)
        out = torch.zeros(2, dtype=torch.int64, device="cuda")
        mpsm.join_noalloc_into(Rd, Sd, out, cfg)
        torch.cuda.synchronize()
        got = _u64(out)
        ref = mpsm.join(Rd, Sd, cfg)
        want = oracle.join(R, S)
        assert got == [ref["count"], ref["checksum"]]
        assert got == [want.count, want.checksum]


@pytest.mark.gpu
def test_noalloc_pairs_and_edge_cases():
    rng = np.random.default_rng(78)
    R, S = _rel(rng, 4000, 3000), _rel(rng, 9000, 3000)
    want = oracle.join(R, S, pairs=True, cap=1 << 20)
    Rd, Sd = _dev(R), _dev(S)
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    pbuf = torch.zeros((want.count, 3), dtype=torch.int64, device="cuda")
    _say(f"mpsm_join_noalloc with pairs: nR={len(R)} nS={len(S)} count={want.count}")
    mpsm.join_noalloc_into(Rd, Sd, out, pairs=pbuf)
    torch.cuda.synchronize()
    assert _u64(out) == [want.count, want.checksum]
    p = pbuf.cpu().numpy().view(np.uint64)
    assert np.array_equal(p[np.lexsort((p[:, 2], p[:, 1], p[:, 0]))], want.pairs)
    # empty and single-tuple inputs after a larger call
    for nR, nS in ((0, 5), (5, 0), (1, 1)):
        _say(f"mpsm_join_noalloc nR={nR} nS={nS}")
        a, b = _rel(rng, nR, 2), _rel(rng, nS, 2)
        out.fill_(-1)
        mpsm.join_noalloc_into(_dev(a).reshape(-1, 2), _dev(b).reshape(-1, 2), out)
        torch.cuda.synchronize()
        w = oracle.join(a.reshape(-1, 2), b.reshape(-1, 2))
        assert _u64(out) == [w.count, w.checksum]


def test_noalloc_refuses_sizes_beyond_its_array():
    """Refused on the host before any device call (no GPU needed): the
    pointers are never dereferenced."""
    L = mpsm.lib()
    fake = ctypes.c_void_p(1 << 20)
    nR, nS = 1 << 20, 1 << 22
    assert mpsm.workspace_bytes(nR, nS) > mpsm.NOALLOC_SCRATCH_BYTES
    rc = L.mpsm_join_noalloc(fake, nR, fake, nS, fake, ctypes.c_void_p((1 << 20) + 8), None, 0, None, None)
    assert mpsm.STATUS[rc] == "MPSM_ENOMEM"
    rc = L.mpsm_join_noalloc(fake, 1 << 32, fake, 10, fake, fake, None, 0, None, None)
    assert mpsm.STATUS[rc] == "MPSM_EINVAL"


def test_noalloc_size_constant_matches_header():
    import os
    import re
    from conftest import ROOT
    with open(os.path.join(ROOT, "include", "mpsm.h")) as f:
        m = re.search(r"#define MPSM_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", f.read())
    assert m and int(m.group(1)) << int(m.group(2)) == mpsm.NOALLOC_SCRATCH_BYTES
