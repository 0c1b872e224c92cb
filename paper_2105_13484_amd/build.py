"""Build the HIP library ``libssprkse.so`` in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libssprkse.so")
SOURCES = ["sse_mesh.cpp", "sse_kernels.hip", "sse_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from emitting packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source into ``libssprkse.so`` (always rebuilds).  The
    sources compile in parallel to objects in a temporary folder, then link."""
    import tempfile
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="ssprkse_build_") as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src + ".o")
            cmd = [cc, *[f for f in HIPCC_FLAGS if f != "-shared"], "-c", "-o", obj, os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
            objs.append(obj)
        errors = []
        for src, proc in procs:
            out, err = proc.communicate()
            if proc.returncode != 0:
                errors.append(f"{src}: hipcc failed ({proc.returncode}):\n{out}\n{err}")
        if errors:
            raise RuntimeError("\n".join(errors))
        tmp = LIB + ".tmp"
        cmd = [cc, *HIPCC_FLAGS, "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc link failed ({res.returncode}):\n{res.stdout}\n{res.stderr}")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
