"""Build libroaring_gpu.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libroaring_gpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["rg_api.cpp", "rg_build_host.cpp", "rg_match.hip", "rg_bitset.hip", "rg_generic.hip",
           "rg_variants.hip", "rg_assemble.hip", "rg_pool.hip", "rg_kway.hip", "rg_serve.cpp", "rg_mlp.hip", "rg_dispatch.cpp",
           "rg_access.hip", "rg_access_api.cpp", "rg_mutable.hip", "rg_mutable_api.cpp", "rg_small.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(jobs: int = 8) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(objdir, s + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if s.endswith(".cpp") else []
        procs.append(subprocess.Popen([HIPCC, *FLAGS, *lang, "-c", src, "-o", obj]))
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


def _wait(procs):
    bad = [p for p in procs if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(bad[0].returncode, bad[0].args)


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
