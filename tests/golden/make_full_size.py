"""Writes full_size.json: the expected join results of the two large named
workloads at full size, computed on the CPU by the oracle alone.

  skewed     |R| = 2^26 clustered keys, |S| = 2^28 Zipf(1.0) foreign keys:
             the foreign-key closed form (every S tuple with its partner).
  lognormal  |R| = 2^28 log-normal keys with duplicates, |S| = 2^30:
             the oracle's sort-merge join, summed over key-range slices
             (the slices partition the key space; one thread per slice).

Each entry also stores a fingerprint of the generated inputs (SHA-256 of
every 4097th row of R and every 4099th row of S), so that a test can tell a
generator that behaves differently on another host from a wrong join.

Run from the repository root:  python tests/golden/make_full_size.py
(about 3 minutes and 45 GB of host memory on 8 cores)."""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402


def fingerprint(w) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w.R[::4097]).tobytes())
    h.update(np.ascontiguousarray(w.S[::4099]).tobytes())
    return h.hexdigest()


def slice_bounds(R, n):
    rng = np.random.default_rng(0)
    smp = np.sort(R[rng.integers(0, len(R), 1 << 16), 0])
    return np.unique(smp[(np.arange(1, n) * len(smp)) // n])


def main():
    out = {"source": "written by tests/golden/make_full_size.py (oracle only)"}
    t = time.time()
    w = workloads.make("skewed")
    fk = oracle.fk_closed_form(w.R, w.S, w.partner)
    out["skewed"] = {"nR": len(w.R), "nS": len(w.S), "count": fk.count, "checksum_hex": f"{fk.checksum:016x}",
                     "method": "foreign-key closed form", "inputs_sha256": fingerprint(w)}
    print("skewed", out["skewed"], f"{time.time() - t:.0f} s", flush=True)
    del w
    t = time.time()
    w = workloads.make("lognormal")
    r = oracle.join_sliced(w.R, w.S, slice_bounds(w.R, 32), threads=os.cpu_count() or 1)
    assert r.count == w.expected_count
    out["lognormal"] = {"nR": len(w.R), "nS": len(w.S), "count": r.count, "checksum_hex": f"{r.checksum:016x}",
                        "method": "sort-merge join over 32 key-range slices",
                        "inputs_sha256": fingerprint(w)}
    print("lognormal", out["lognormal"], f"{time.time() - t:.0f} s", flush=True)
    with open(os.path.join(HERE, "full_size.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
