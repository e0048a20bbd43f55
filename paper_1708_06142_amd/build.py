"""Build libocttree.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libocttree.so")
BUILD = os.path.join(HERE, "_build")

# Files whose floating-point decisions must be reproducible bit for bit
# (node moments, MAC accept/open) are compiled without FMA contraction.
SOURCES = {
    "topology.cpp": [],
    "cache.cpp": [],
    "api.hip": [],
    "k_build.hip": ["-ffp-contract=off"],
    "k_list.hip": ["-ffp-contract=off"],
    "k_eval.hip": [],
    "k_ewald.hip": [],
    "k_columns.hip": [],
    # matrix products in ordinary vector registers (the activations read them
    # next; accumulation registers would cost a copy per value)
    "k_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def hipcc():
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def _compile(name, flags):
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), "-c"] + COMMON + flags + ["-x", "hip", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        res = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    objs = [o for o, _ in res]
    for _, w in res:
        if w and verbose:
            print(w, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
