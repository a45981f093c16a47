"""Register, scratch and LDS use of the built kernels (compiler report).

A kernel that runs out of registers spills lane values to scratch memory.
Scratch lines are ordinary cached memory: a spill stored once per workgroup
at the start of a one-bucket-per-workgroup kernel is later written back to
HBM, dead, for every workgroup (at |S| = 2^28 that was 2 GB of extra writes
per S-run sort).  These tests keep the hot kernels spill-free and at the
occupancy their LDS tiles are sized for.
"""
import json
import os

import pytest

import paper_1207_0145_amd.build as B

# Kernels allowed to use scratch, with the reason.
ALLOWED_SCRATCH = {
    # batched join: a persistent grid of one workgroup per CU, so its spill
    # is written once per CU per launch, not once per work item
    "_Z6k_joinILi0ELi0ELb1E": 64,
}

HOT = {
    "s_sort": "_Z16k_bucket_sort_csILi1024ELi4ELi2048ELi8ELb0ELb0E",
    "r_sort": "_Z16k_bucket_sort_csILi1024ELi8ELi4096ELi1ELb1ELb0E",
    "r_retry": "_Z16k_bucket_sort_csILi1024ELi8ELi4096ELi1ELb1ELb1E",
    "scatter": "_Z16k_bucket_scatterILb0E",
    "scatter_regions": "_Z16k_bucket_scatterILb1E",
    "hist": "_Z13k_bucket_hist",
    "join": "_Z6k_joinILi0ELi0ELb0E",
    "search": "_Z8k_search",
}


def _report():
    if not os.path.exists(B.RESOURCES):
        pytest.skip("library not built (run __graft_entry__.build())")
    with open(B.RESOURCES) as f:
        return json.load(f)


def _find(rep, prefix):
    hits = [k for k in rep if k.startswith(prefix)]
    assert len(hits) == 1, (prefix, hits)
    return rep[hits[0]]


def test_parse_resource_remarks():
    text = "\n".join([
        "k.h:1:1: remark: Function Name: _Z3fooi [-Rpass-analysis=kernel-resource-usage]",
        "k.h:1:1: remark:     VGPRs: 64 [-Rpass-analysis=kernel-resource-usage]",
        "k.h:1:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]",
        "k.h:1:1: remark:     ScratchSize [bytes/lane]: 20 [-Rpass-analysis=kernel-resource-usage]",
        "k.h:1:1: remark:     Occupancy [waves/SIMD]: 8 [-Rpass-analysis=kernel-resource-usage]",
        "   12 | __global__ void foo(int) {",
        "      | ^",
        "k.h:1:1: remark:     LDS Size [bytes/block]: 80016 [-Rpass-analysis=kernel-resource-usage]",
        "k.h:9:1: remark: Function Name: _Z3barv [-Rpass-analysis=kernel-resource-usage]",
        "k.h:9:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
    ])
    rep = B.parse_resource_remarks(text)
    assert rep == {"_Z3fooi": {"vgprs": 64, "agprs": 0, "scratch_bytes": 20, "occupancy": 8, "lds_bytes": 80016},
                   "_Z3barv": {"scratch_bytes": 0}}


def test_report_covers_hot_kernels():
    rep = _report()
    for name, prefix in HOT.items():
        k = _find(rep, prefix)
        assert {"vgprs", "scratch_bytes", "occupancy", "lds_bytes"} <= set(k), name


def test_no_scratch_spills():
    rep = _report()
    for name, k in rep.items():
        allowed = next((v for p, v in ALLOWED_SCRATCH.items() if name.startswith(p)), 0)
        assert k.get("scratch_bytes", 0) <= allowed, (name, k)


def test_sort_tiles_fit_their_occupancy():
    rep = _report()
    s = _find(rep, HOT["s_sort"])
    # S-run buckets: two 1024-thread workgroups per CU (8 waves per SIMD)
    assert s["occupancy"] >= 8 and s["lds_bytes"] <= 160 * 1024 // 2, s
    for name in ("r_sort", "r_retry"):
        r = _find(rep, HOT[name])
        assert r["occupancy"] >= 4 and r["lds_bytes"] <= 160 * 1024, r
