"""GPU parity on the workloads of the paper's other experiments: the
negatively correlated 80:20 skew with every splitter form (Section 5.6),
role reversal over multiplicities 1, 4, 8, 16 (Section 5.4) and location
skew of S (Section 5.5).  Every result against the CPU oracle (or the
foreign-key closed form, which the oracle pins tests fix)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1207_0145_amd as mpsm
import workloads

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to("cuda")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _oracle_sliced(R, S, nslices=16):
    smp = np.sort(R[np.random.default_rng(0).integers(0, len(R), 1 << 14), 0])
    bounds = np.unique(smp[(np.arange(1, nslices) * len(smp)) // nslices])
    return oracle.join_sliced(R, S, bounds, threads=16)


FORMS = {
    "sampled": dict(),
    "learned": dict(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED),
    "cost": dict(splitter=mpsm.SPLIT_COST),
}


@pytest.mark.parametrize("shift", [4, 0])
def test_negcorr_every_splitter_form_matches_oracle(shift):
    """|R| = 2^(24-shift), |S| = 4 |R| with negatively correlated 80:20
    skew: sampled, learned and cost-balanced splitters all equal the
    oracle."""
    w = workloads.negcorr(1 << (24 - shift), 1 << (26 - shift), seed=0x1207014500000701)
    want = _oracle_sliced(w.R, w.S)
    R, S = _dev(w.R), _dev(w.S)
    for name, kw in FORMS.items():
        _say(f"negcorr |R|=2^{24 - shift} form {name}")
        got = mpsm.join(R, S, mpsm.config(**kw))
        assert (got["count"], got["checksum"]) == (want.count, want.checksum), name


@pytest.mark.parametrize("m", [1, 4, 8, 16])
def test_role_reversal_multiplicities(m):
    """|S| = m |R| foreign keys, joined with R private (as given) and with S
    private (swapped): the same result in the caller's orientation, equal
    to the foreign-key closed form."""
    w = workloads.fk_uniform(1 << 17, m << 17, seed=0x1207014500000800 + m, spread=True)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    R, S = _dev(w.R), _dev(w.S)
    for role in (mpsm.ROLE_AS_GIVEN, mpsm.ROLE_SWAP, mpsm.ROLE_AUTO):
        _say(f"roles m={m} role={role}")
        got = mpsm.join(R, S, mpsm.config(role=role), with_stats=True)
        assert (got["count"], got["checksum"]) == (fk.count, fk.checksum), role
        assert got["stats"]["swapped"] == (1 if role == mpsm.ROLE_SWAP else 0)


@pytest.mark.parametrize("clusters", [0, 4, 1024])
def test_location_skew(clusters):
    """S ordered small to large in clusters (0: one cluster per S run, the
    extreme case where each partition's partners sit in one run): equal to
    the foreign-key closed form."""
    base = workloads.fk_uniform(1 << 20, 1 << 22, seed=0x1207014500000901, spread=True)
    lay = mpsm.layout(len(base.R), len(base.S))
    k = clusters or lay["runs"]
    w = workloads.location_skew(base, k, seed=3)
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    _say(f"location skew: {k} clusters over {lay['runs']} runs")
    got = mpsm.join(_dev(w.R), _dev(w.S), with_stats=True)
    assert (got["count"], got["checksum"]) == (fk.count, fk.checksum)
