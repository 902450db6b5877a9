"""Build libwcl.so (hipcc, gfx950) in-tree next to this file."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwcl.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions stay off (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit contraction: every fused multiply-add is written in the source
    "-ffp-contract=off",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link the library."""
    import concurrent.futures
    import tempfile

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory() as tmp:
        jobs = []
        for src in sources():
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            flags = [f for f in HIPCC_FLAGS if f != "-shared"]
            jobs.append(([hipcc, *flags, *inc, "-c", src, "-o", obj], obj))
        if verbose:
            for cmd, _ in jobs:
                print(" ".join(cmd), flush=True)
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
            for res in ex.map(lambda j: subprocess.run(j[0], capture_output=True, text=True), jobs):
                if res.returncode != 0:
                    raise RuntimeError("hipcc failed:\n" + res.stderr)
        out_tmp = LIB + ".tmp"
        link = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", out_tmp, *[o for _, o in jobs]]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
