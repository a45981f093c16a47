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
    assert mpsm.workspace_bytes(10, 10, mpsm.config(reserved=1)) == 0
    bad = mpsm.config()
    bad.struct_size = 4
    assert mpsm.workspace_bytes(10, 10, bad) == 0


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
