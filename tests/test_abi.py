"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, sizes and layouts are sane, and bad arguments are
rejected on the host before anything touches the device."""
import ctypes
import os
import re

import pytest

import paper_1207_0145_amd as mpsm
from conftest import ROOT


def _declared_functions():
    with open(os.path.join(ROOT, "include", "mpsm.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpsm_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function():
    declared = _declared_functions()
    assert "mpsm_join" in declared and "mpsm_workspace_bytes" in declared
    L = mpsm.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert set(mpsm.EXPORTS) == set(declared)


def test_config_struct_size_matches():
    c = mpsm.config()
    assert c.struct_size == ctypes.sizeof(mpsm.MpsmConfig)
    assert c.search == mpsm.SEARCH_INDEX and c.role == mpsm.ROLE_AUTO


def test_status_strings():
    L = mpsm.lib()
    for code in range(6):
        assert L.mpsm_status_string(code)
    assert L.mpsm_status_string(3) == b"workspace too small"


@pytest.mark.parametrize("nR,nS", [(0, 0), (1, 1), (1 << 20, 1 << 22), (1 << 26, 1 << 28), (1 << 28, 1 << 30),
                                   (12345, 678901), (1 << 22, 1 << 10)])
def test_workspace_and_layout(nR, nS):
    ws = mpsm.workspace_bytes(nR, nS)
    assert ws >= 16 * 2 * (nR + nS)            # two copies of each relation at least
    lay = mpsm.layout(nR, nS)
    assert lay["off_s_sorted"] + 16 * max(nR, nS) <= ws
    if nR > nS:
        assert lay["swapped"] == 1
    nprivate = min(nR, nS) if nR != nS else nR
    assert lay["r_buckets1"] * lay["r_buckets2"] >= (nprivate + 4095) // 4096
    assert lay["runs"] * lay["run_len"] >= max(nR, nS) if nR <= nS else True


def test_unsupported_sizes():
    assert mpsm.workspace_bytes(1 << 32, 10) == 0
    assert mpsm.workspace_bytes(10, 1 << 32) == 0
    assert mpsm.workspace_bytes(10, 10, mpsm.config(search=7)) == 0
    assert mpsm.workspace_bytes(10, 10, mpsm.config(log2_run_len=30)) == 0
    assert mpsm.workspace_bytes(10, 10, mpsm.config(waves=65)) == 0
    assert mpsm.workspace_bytes(10, 10, mpsm.config(join_chunk=1 << 20)) == 0
    assert mpsm.workspace_bytes(10, 10, mpsm.config(join_chunk=261888)) > 0
    bad = mpsm.config()
    bad.struct_size = 4
    assert mpsm.workspace_bytes(10, 10, bad) == 0


def test_host_runs_workspace():
    """The join with S in host memory holds one chunk of S on the device: its
    workspace shrinks by both copies of the rest of S (the bucketed and the
    sorted one); options it does not take and chunk 0 size to 0."""
    nR, nS, chunk = 1 << 20, 1 << 30, 1 << 24
    full = mpsm.workspace_bytes(nR, nS)
    host = mpsm.join_host_runs_workspace_bytes(nR, nS, chunk)
    assert 0 < host and host + 2 * 16 * (nS - chunk) <= full
    assert mpsm.join_host_runs_workspace_bytes(nR, nS, nS) >= full - 1024
    assert mpsm.join_host_runs_workspace_bytes(nR, nS, 1) == mpsm.join_host_runs_workspace_bytes(nR, nS, 1 << 16)
    assert mpsm.join_host_runs_workspace_bytes(nR, nS, 0) == 0
    assert mpsm.join_host_runs_workspace_bytes(nR, 1 << 32, chunk) == 0
    for kw in (dict(splitter=mpsm.SPLIT_COST), dict(splitter=mpsm.SPLIT_NONE), dict(role=mpsm.ROLE_SWAP)):
        assert mpsm.join_host_runs_workspace_bytes(nR, nS, chunk, mpsm.config(**kw)) == 0, kw
    assert mpsm.join_host_runs_workspace_bytes(nR, nS, chunk, mpsm.config(splitter=mpsm.SPLIT_LEARNED)) > 0


def test_host_runs_chunks_are_whole_runs():
    """The chunk is rounded down to whole runs (at least one): the workspace
    is the same for every chunk between k and k+1 runs, and grows with k."""
    nR, nS = 1 << 20, 1 << 26
    L = mpsm.layout(nR, nS, mpsm.config(role=mpsm.ROLE_AS_GIVEN))["run_len"]
    sizes = []
    for k in (1, 2, 3, 8):
        w = {mpsm.join_host_runs_workspace_bytes(nR, nS, c) for c in (k * L, k * L + 1, (k + 1) * L - 1)}
        assert len(w) == 1, k
        sizes.append(w.pop())
    assert sizes == sorted(sizes) and sizes[0] < sizes[-1]
    assert mpsm.join_host_runs_workspace_bytes(nR, nS, L - 1) == sizes[0]


def test_spilled_runs_workspace_and_host_checks():
    """The join over runs already in host memory holds no copy of S: its
    workspace is far below the device-resident join's; refused options size
    to 0; a NULL or misaligned run array is refused before any HIP call."""
    nR, nS = 1 << 20, 1 << 30
    ws = mpsm.join_spilled_runs_workspace_bytes(nR, nS)
    assert 0 < ws and ws + 2 * 16 * (nS - (1 << 24)) <= mpsm.workspace_bytes(nR, nS)
    for kw in (dict(splitter=mpsm.SPLIT_COST), dict(splitter=mpsm.SPLIT_NONE), dict(role=mpsm.ROLE_SWAP)):
        assert mpsm.join_spilled_runs_workspace_bytes(nR, nS, mpsm.config(**kw)) == 0, kw
    L = mpsm.lib()
    good = ctypes.c_void_p(0x100000)
    assert L.mpsm_join_spilled_runs(good, 5, None, 5, good, good, None, good, 1 << 40, None) == 1
    assert L.mpsm_join_spilled_runs(good, 5, ctypes.c_void_p(0x100008), 5, good, good, None, good, 1 << 40,
                                    None) == 1
    assert L.mpsm_join_spilled_runs(good, 5, good, 5, good, good,
                                    ctypes.byref(mpsm.config(splitter=mpsm.SPLIT_COST)), good, 1 << 40, None) == 1


def test_host_runs_bad_arguments_rejected_on_host():
    # rejected before any HIP call: the pointers are never dereferenced
    L = mpsm.lib()
    good = ctypes.c_void_p(0x100000)

    def call(S, runs, chunk, cfg=None):
        return L.mpsm_join_host_runs(good, 5, S, 5, runs, good, good, None if cfg is None else ctypes.byref(cfg),
                                     chunk, good, 1 << 40, None)

    assert call(good, good, 0) == 1
    assert call(None, good, 4096) == 1
    assert call(ctypes.c_void_p(0x100008), good, 4096) == 1
    assert call(good, ctypes.c_void_p(0x100004), 4096) == 1
    assert call(good, good, 4096, mpsm.config(splitter=mpsm.SPLIT_COST)) == 1
    assert call(good, good, 4096, mpsm.config(role=mpsm.ROLE_SWAP)) == 1


def _call(R, nR, S, nS, out_c, out_s, ws, wsb, cfg=None):
    L = mpsm.lib()
    return L.mpsm_join(R, nR, S, nS, out_c, out_s, None, 0, None if cfg is None else ctypes.byref(cfg), ws, wsb,
                       None, None)


def test_bad_arguments_rejected_on_host():
    # pointers below are never dereferenced: validation fails first
    good = ctypes.c_void_p(0x100000)
    assert _call(None, 5, good, 5, good, good, good, 1 << 40) == 1          # NULL R with nR > 0
    assert _call(good, 5, None, 5, good, good, good, 1 << 40) == 1          # NULL S with nS > 0
    assert _call(good, 5, good, 5, None, good, good, 1 << 40) == 1          # NULL output
    assert _call(good, 5, good, 5, good, good, None, 1 << 40) == 1          # NULL workspace
    assert _call(ctypes.c_void_p(0x100008), 5, good, 5, good, good, good, 1 << 40) == 1   # misaligned R
    assert _call(good, 5, good, 5, good, good, ctypes.c_void_p(0x100010), 1 << 40) == 1   # misaligned ws
    assert _call(good, 1 << 32, good, 5, good, good, good, 1 << 60) == 1    # too many tuples
    assert _call(good, 5, good, 5, good, good, good, 1024) == 3             # workspace too small
    assert _call(good, 5, good, 5, good, good, good, 1 << 40, mpsm.config(search=9)) == 1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(mpsm, "_lib", None)
    monkeypatch.setattr(mpsm, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        mpsm.lib()


# ------------------------------------------------------------ batch (host side)

def _descs(sizes):
    """Descriptors with fake, aligned device addresses (never dereferenced:
    batch planning touches no device)."""
    arr = (mpsm.MpsmJoinDesc * len(sizes))()
    for i, (nR, nS) in enumerate(sizes):
        d = arr[i]
        d.d_R = 0x10000000 + 0x1000000 * i if nR else None
        d.nR = nR
        d.d_S = 0x80000000 + 0x1000000 * i if nS else None
        d.nS = nS
        d.d_out_count = 0x200000 + 64 * i
        d.d_out_checksum = 0x200000 + 64 * i + 8
        d.d_out_times = None
    return arr


def _create(sizes, cfg=None):
    h = ctypes.c_void_p()
    rc = mpsm.lib().mpsm_batch_create(_descs(sizes), len(sizes), None if cfg is None else ctypes.byref(cfg),
                                      ctypes.byref(h))
    return rc, h


def test_batch_plan_and_tuning():
    L = mpsm.lib()
    rc, h = _create([(4096, 16384), (1 << 20, 1 << 23), (0, 100), (100, 0), (1, 1)])
    assert rc == 0 and h
    try:
        ws = L.mpsm_batch_workspace_bytes(h)
        assert ws >= 2 * 16 * ((4096 + (1 << 20) + 1) + (16384 + (1 << 23) + 1))
        t = mpsm.MpsmBatchTuning()
        assert L.mpsm_batch_get_tuning(h, ctypes.byref(t)) == 0
        assert 16 <= t.log2_run_len <= 22 and t.bucket_target == 4096 and t.join_chunk == 65536
        bad = mpsm.MpsmBatchTuning(12, 4096, 65536, 0, 0.0)           # run length too short
        assert L.mpsm_batch_set_tuning(h, ctypes.byref(bad)) == 5
        ok = mpsm.MpsmBatchTuning(16, 2048, 16384, 0, 0.0)
        assert L.mpsm_batch_set_tuning(h, ctypes.byref(ok)) == 0
        assert L.mpsm_batch_get_tuning(h, ctypes.byref(t)) == 0 and (t.log2_run_len, t.bucket_target) == (16, 2048)
    finally:
        L.mpsm_batch_destroy(h)


def test_batch_rejects_bad_input():
    L = mpsm.lib()
    h = ctypes.c_void_p()
    assert L.mpsm_batch_create(None, 0, None, ctypes.byref(h)) == 1
    d = _descs([(10, 10)])
    d[0].d_R = None                                                     # NULL R with nR > 0
    assert L.mpsm_batch_create(d, 1, None, ctypes.byref(h)) == 1
    d = _descs([(10, 10)])
    d[0].d_S = 0x80000008                                               # misaligned S
    assert L.mpsm_batch_create(d, 1, None, ctypes.byref(h)) == 1
    assert _create([(10, 10)], mpsm.config(splitter=mpsm.SPLIT_LEARNED))[0] == 5
    assert _create([(10, 10)], mpsm.config(search=mpsm.SEARCH_LEARNED))[0] == 5
    assert _create([(10, 10)], mpsm.config(want_max=1))[0] == 5
    assert _create([(1 << 31, 10), (1 << 31, 10)])[0] == 1             # sum of nR beyond 2^32


def test_join_batch_host_checks():
    """mpsm_join_batch: every host-side check returns before anything is
    enqueued (no GPU needed: the fake pointers are never used)."""
    L = mpsm.lib()
    sh = mpsm.batch_shape(1 << 20, 1 << 22, 1 << 20)
    need = mpsm.join_batch_workspace_bytes(256, sh)
    assert need > 32 * ((1 << 20) + (1 << 22))
    # bounds grow the workspace; more joins need larger tables
    assert mpsm.join_batch_workspace_bytes(256, mpsm.batch_shape(1 << 21, 1 << 22, 1 << 20)) > need
    assert mpsm.join_batch_workspace_bytes(512, sh) > need
    assert mpsm.join_batch_workspace_bytes(0, sh) == 0
    assert mpsm.join_batch_workspace_bytes(256, mpsm.batch_shape(1 << 32, 10)) == 0
    assert mpsm.join_batch_workspace_bytes(256, sh, mpsm.config(splitter=mpsm.SPLIT_LEARNED)) == 0
    # one join of 2^28 S tuples would need 4096 runs of 2^16 (at most 2048)
    assert mpsm.join_batch_workspace_bytes(4, mpsm.batch_shape(1 << 20, 1 << 28, 1 << 28),
                                           mpsm.config(log2_run_len=16)) == 0
    assert mpsm.join_batch_workspace_bytes(4, mpsm.batch_shape(1 << 20, 1 << 28, 1 << 28)) > 0
    d, ws = ctypes.c_void_p(1 << 24), ctypes.c_void_p(1 << 30)
    call = lambda descs, n, shape, cfg, w, nb: L.mpsm_join_batch(descs, n, shape, cfg, w, nb, None)
    assert call(None, 256, ctypes.byref(sh), None, ws, need) == 1                      # no descriptors
    assert call(ctypes.c_void_p((1 << 24) + 4), 256, ctypes.byref(sh), None, ws, need) == 1   # misaligned
    assert call(d, 256, None, None, ws, need) == 1                                     # no shape
    assert call(d, 256, ctypes.byref(sh), None, ctypes.c_void_p((1 << 30) + 64), need) == 1   # workspace alignment
    assert call(d, 256, ctypes.byref(sh), None, ws, need - 1) == 3                     # workspace too small
    assert call(d, 0, ctypes.byref(sh), None, ws, need) == 1                           # no joins
    cfg = mpsm.config(want_max=1)
    assert call(d, 256, ctypes.byref(sh), ctypes.byref(cfg), ws, need) == 5
    cfg = mpsm.config(waves=65)
    assert call(d, 256, ctypes.byref(sh), ctypes.byref(cfg), ws, need) == 1


def test_batch_autotune_cache_hit_and_malformed_entries(tmp_path):
    """A cache entry for the batch's shape is used without touching the GPU;
    malformed or out-of-range lines are skipped."""
    L = mpsm.lib()
    sizes = [(5000, 20000), (70000, 300000)]
    rc, h = _create(sizes)
    assert rc == 0
    try:
        cache = tmp_path / "tune.txt"
        t = mpsm.MpsmBatchTuning()
        # no entry and no workspace: nothing to measure with
        assert L.mpsm_batch_autotune(h, None, 0, None, str(cache).encode(), ctypes.byref(t)) == 1
        # learn the signature from a measured entry format, then plant entries
        sig = "gfx950:n2:R16:S18:maxR16:maxS18:search3:w1"
        cache.write_text("garbage line\n"
                         f"{sig} 40 4096 65536 1.0\n"          # log2 run length out of range
                         f"{sig} 18 999 65536 1.0\n"           # bucket target out of range
                         f"{sig} 16 2048 16384 0.5\n"
                         "other:sig 20 4096 65536 0.1\n")
        assert L.mpsm_batch_autotune(h, None, 0, None, str(cache).encode(), ctypes.byref(t)) == 0
        assert t.from_cache == 1 and (t.log2_run_len, t.bucket_target, t.join_chunk) == (16, 2048, 16384)
    finally:
        L.mpsm_batch_destroy(h)


def test_stats_binding_matches_header():
    """The ctypes MpsmStats mirrors include/mpsm.h field by field."""
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "mpsm.h")).read()
    body = hdr[hdr.index("typedef struct mpsm_stats {"):hdr.index("} mpsm_stats;")]
    fields = re.findall(r"^\s*(uint64_t|double)\s+(\w+);", body, re.M)
    ct = {"uint64_t": ctypes.c_uint64, "double": ctypes.c_double}
    assert [(n, ct[t]) for t, n in fields] == list(mpsm.MpsmStats._fields_)
