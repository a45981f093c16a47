"""The join kernel's slice plan (which S positions a join unit reads), run
on the host through mpsm_join_slices_host: the same per-run code as the
kernel.  Offsets that a correct start search never returns (reversed pairs,
values past the run's end, arbitrary 32-bit garbage) must still keep every
read inside its run.  Runs on the CPU; no GPU."""
import numpy as np
import pytest

import paper_1207_0145_amd as mpsm


def _reads_inside_runs(oa, ob, run_start, run_len):
    cum, sbase = mpsm.join_slices_host(oa, ob, run_start, run_len)
    Q = len(oa)
    assert cum[0] == 0 and np.all(np.diff(cum.astype(np.int64)) >= 0)
    for j in range(Q):
        n = int(run_len[j])
        ln = int(cum[j + 1]) - int(cum[j])
        assert ln <= n
        if ln == 0:
            continue
        first = (int(sbase[j]) + int(cum[j])) % (1 << 32)
        last = (int(sbase[j]) + int(cum[j + 1]) - 1) % (1 << 32)
        assert int(run_start[j]) <= first and last < int(run_start[j]) + n, (j, first, last)
        assert last - first + 1 == ln
    return cum, sbase


def _runs(rng, Q):
    run_len = rng.integers(0, 5000, Q).astype(np.uint32)
    run_start = np.concatenate([[0], np.cumsum(run_len)[:-1]]).astype(np.uint32)
    return run_start, run_len


def test_valid_offsets_read_exactly_the_slices():
    rng = np.random.default_rng(1)
    Q = 37
    run_start, run_len = _runs(rng, Q)
    oa = np.array([rng.integers(0, n + 1) for n in run_len], np.uint32)
    ob = np.array([rng.integers(a, n + 1) for a, n in zip(oa, run_len)], np.uint32)
    cum, sbase = _reads_inside_runs(oa, ob, run_start, run_len)
    assert np.array_equal(np.diff(cum.astype(np.int64)), (ob - oa).astype(np.int64))
    for j in range(Q):
        if ob[j] > oa[j]:
            assert (int(sbase[j]) + int(cum[j])) % (1 << 32) == int(run_start[j]) + int(oa[j])


@pytest.mark.parametrize("seed", range(8))
def test_garbage_offsets_stay_inside_the_runs(seed):
    # the offsets an unsorted run can leave: reversed pairs (the wrap that once
    # made the join read far out of bounds), values past the run, any u32
    rng = np.random.default_rng(100 + seed)
    Q = int(rng.integers(1, 300))
    run_start, run_len = _runs(rng, Q)
    kind = seed % 4
    if kind == 0:     # reversed pairs inside the runs
        ob = np.array([rng.integers(0, n + 1) for n in run_len], np.uint32)
        oa = np.array([rng.integers(b, n + 1) for b, n in zip(ob, run_len)], np.uint32)
    elif kind == 1:   # past the end of the run
        oa = (run_len + rng.integers(0, 100, Q)).astype(np.uint32)
        ob = (oa + rng.integers(0, 100, Q)).astype(np.uint32)
    elif kind == 2:   # arbitrary 32-bit values
        oa = rng.integers(0, 1 << 32, Q, dtype=np.uint64).astype(np.uint32)
        ob = rng.integers(0, 1 << 32, Q, dtype=np.uint64).astype(np.uint32)
    else:             # start inside, end far past
        oa = np.array([rng.integers(0, n + 1) for n in run_len], np.uint32)
        ob = np.full(Q, 0xFFFFFFFF, np.uint32)
    _reads_inside_runs(oa, ob, run_start, run_len)


def test_empty_plan():
    cum, sbase = mpsm.join_slices_host([], [], [], [])
    assert cum.tolist() == [0] and len(sbase) == 0
