"""bench.py's per-step device times from the join's markers (no GPU).

The markers of R's phase are recorded on a second stream when R's
partitioning runs beside S's bucket sort, so consecutive markers in name
order are not consecutive in time.  These tests feed step_times marker
timestamps of both launch orders and check every step's duration.
"""
import importlib.util
import os

import pytest

import paper_1207_0145_amd as mpsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _Events:
    """Stand-in for an EventSet: elapsed(i, j) from marker timestamps (ms)."""

    def __init__(self, t):
        self.t = t

    def elapsed(self, i, j):
        return self.t[j] - self.t[i]


def _names():
    try:
        return mpsm.marker_names()
    except RuntimeError:
        pytest.skip("library not built (run __graft_entry__.build())")


def _stamps(names, durations, order):
    """Timestamps of the markers when the steps in `order` run one after the
    other, each taking durations[step] (the step ends at its marker)."""
    t, now = {}, 0.0
    t[names[0]] = now
    for step in order:
        now += durations[step]
        t[step] = now
    return [t[n] for n in names]


def test_marker_names_cover_the_steps():
    names = _names()
    assert names[0] == "start" and names[1] == "init" and names[-1] == "finalize"
    for n in ("s_scatter", "s_bucket_sort", "s_oversize_sort", "r1_splitters", "r_oversize_sort", "partitions"):
        assert n in names


def test_one_stream_steps_are_marker_differences():
    names = _names()
    dur = {n: 0.1 * (i + 1) for i, n in enumerate(names[1:])}
    stamps = _stamps(names, dur, names[1:])
    out, overlapped = _bench().step_times(names, [_Events(stamps)], 1)
    assert not overlapped
    for n in names[1:]:
        assert out[n] == pytest.approx(dur[n])


def test_two_stream_steps():
    """S's steps on the first stream; R's from the end of S's scatter on the
    second; the partition step waits for the later of the two ends."""
    names = _names()
    ix = {n: i for i, n in enumerate(names)}
    s_steps = names[1:ix["s_oversize_sort"] + 1]
    r_steps = names[ix["r1_splitters"]:ix["r_oversize_sort"] + 1]
    tail = names[ix["r_oversize_sort"] + 1:]
    dur = {n: 0.05 + 0.01 * i for i, n in enumerate(names[1:])}
    t = {names[0]: 0.0}
    now = 0.0
    for n in s_steps:
        now += dur[n]
        t[n] = now
    # R starts once S's scatter is done
    now = t["s_scatter"]
    for n in r_steps:
        now += dur[n]
        t[n] = now
    for late_r in (False, True):
        tt = dict(t)
        if not late_r:   # make S's sort end after R's phase
            shift = tt["r_oversize_sort"] + 0.3 - tt["s_oversize_sort"]
            for n in ("s_bucket_sort", "s_oversize_sort"):
                tt[n] += shift
        now = max(tt["s_oversize_sort"], tt["r_oversize_sort"])
        for n in tail:
            now += dur[n]
            tt[n] = now
        out, overlapped = _bench().step_times(names, [_Events([tt[n] for n in names])], 1)
        assert overlapped
        assert out["r1_splitters"] == pytest.approx(dur["r1_splitters"])
        for n in r_steps[1:] + names[1:ix["s_scatter"] + 1]:
            assert out[n] == pytest.approx(dur[n]), n
        assert out["partitions"] == pytest.approx(dur["partitions"])
        for n in tail:
            assert out[n] == pytest.approx(dur[n]), n


def _write_csv(path, header, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_host_trace_summary(tmp_path):
    """The hostruns trace summary from a synthetic kernel and memory-copy
    trace: one row per form (the second of its two joins), its span, its
    copies in and out (copy kernels counted as copies out, copies under
    0.05 ms left out) and the sum of its other kernels."""
    b = _bench()
    kt, mc = [], []
    t = 0
    ms = 1_000_000   # ns
    for form in range(len(b.HOSTRUNS_CALLS)):
        for call in range(2):
            kt.append(("k_init_result(Result*)", t, t + 1000))
            kt.append(("void k_join<0, 0, false>(JoinArgs)", t + ms, t + 3 * ms))        # 2 ms
            mc.append(("MEMORY_COPY_HOST_TO_DEVICE", t + ms, t + 5 * ms))               # 4 ms in
            kt.append(("__amd_rocclr_copyBuffer(...)", t + 5 * ms, t + 6 * ms))         # 1 ms out
            mc.append(("MEMORY_COPY_DEVICE_TO_HOST", t + 6 * ms, t + 6 * ms + 10_000))  # 0.01 ms: left out
            t += 10 * ms
    _write_csv(tmp_path / "kt.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], kt)
    _write_csv(tmp_path / "mc.csv", ["Direction", "Start_Timestamp", "End_Timestamp"], mc)
    md = b.summarize_host_trace(str(tmp_path / "kt.csv"), str(tmp_path / "mc.csv"), "cmd")
    rows = [r for r in md.splitlines() if r.startswith("| ") and not r.startswith("| form")]
    assert len(rows) == len(b.HOSTRUNS_CALLS)
    for name, r in zip(b.HOSTRUNS_CALLS, rows):
        cells = [c.strip() for c in r.strip("|").split("|")]
        assert cells[0] == name
        assert cells[1] == "6.01"                    # first kernel start to last end
        assert cells[2] == "1, 4.0, 4.00-4.00"
        assert cells[3] == "1, 1.0, 1.00-1.00"
        assert cells[4] == "2.00"                    # k_init_result (0.001 ms) + k_join
    assert "cmd" in md


def test_host_trace_summary_needs_every_call(tmp_path):
    b = _bench()
    _write_csv(tmp_path / "kt.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [("k_init_result(Result*)", 0, 1000)])
    _write_csv(tmp_path / "mc.csv", ["Direction", "Start_Timestamp", "End_Timestamp"], [])
    with pytest.raises(SystemExit):
        b.summarize_host_trace(str(tmp_path / "kt.csv"), str(tmp_path / "mc.csv"), "cmd")
