"""Compile the HIP library libmpsm.so for gfx950 (in-tree)."""
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libmpsm.so")
# per-kernel register, scratch and LDS use reported by the compiler for the
# library last built (read by the tests that keep hot kernels spill-free)
RESOURCES = os.path.join(HERE, "libmpsm.resources.json")
SOURCES = [os.path.join(HERE, "csrc", "mpsm.hip")]
HEADERS = ["common.h", "block_sort.h", "join_slices.h", "search_window.h", "kernels.h", "learned.h", "batch.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
    "-Rpass-analysis=kernel-resource-usage",
]

_FIELDS = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch_bytes",
           "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "lds_bytes"}


def parse_resource_remarks(text: str) -> dict:
    """Per-kernel figures from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split("[-Rpass-analysis", 1)[0].strip()
        if body.startswith("Function Name:"):
            cur = body.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur is not None and ":" in body:
            k, v = body.rsplit(":", 1)
            if k.strip() in _FIELDS:
                out[cur][_FIELDS[k.strip()]] = int(v.strip())
    return out


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = SO + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the resource remarks and their source excerpts are data, not diagnostics
    errs = "\n".join(l for l in (r.stderr or "").splitlines()
                     if ("error" in l or "warning" in l) and "packed-fp32-ops" not in l
                     and "remark:" not in l)
    if r.returncode != 0:
        full = "\n".join(l for l in (r.stderr or "").splitlines() if "remark:" not in l)
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{full}")
    if verbose and errs.strip():
        print(errs, file=sys.stderr)
    os.replace(tmp, SO)
    with open(RESOURCES + ".tmp", "w") as f:
        json.dump(parse_resource_remarks(r.stderr or ""), f, indent=1, sort_keys=True)
    os.replace(RESOURCES + ".tmp", RESOURCES)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
