"""Build libcct.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

Usage: python -m paper_2607_00981_amd.build   (or build() from Python)
"""

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libcct.so")

SOURCES = ["gemm.hip", "tensor_ops.hip", "q_ops.hip", "q_abc.hip", "contract.cpp", "cct_api.cpp", "slab.cpp", "quad.cpp"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    "-Wno-unused-value",
    # packed-FP32 VALU instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def build(verbose=False, jobs=4):
    """Compile every source (always) and link libcct.so atomically."""
    tmpdir = tempfile.mkdtemp(prefix="cct_build_")
    objs = []
    procs = []
    try:
        for src in SOURCES:
            obj = os.path.join(tmpdir, src.replace(".", "_") + ".o")
            cmd = [hipcc()] + FLAGS + ["-I", INCLUDE, "-I", CSRC]
            if src.endswith(".cpp"):
                cmd += ["-x", "hip"]
            cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
            objs.append(obj)
            procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            if len([p for p in procs if p[2].poll() is None]) >= jobs:
                procs[0][2].wait()
        for src, cmd, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip())
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{text}")
            if verbose and text:
                print(text)
        tmp_lib = LIB + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib] + objs
        r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
