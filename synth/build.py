"""Build the synthetic-input generators: libsynth.so (host, gcc) and
libsynth_gpu.so (device twin for the dense-bitset workload, hipcc gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    subprocess.run(cmd, check=True)


def build_cpu():
    _run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", os.path.join(HERE, "libsynth.so"),
          os.path.join(HERE, "synth.c"), "-lm"])


def build_gpu():
    _run([HIPCC, *HIP_FLAGS, "-o", os.path.join(HERE, "libsynth_gpu.so"), os.path.join(HERE, "synth_gpu.hip")])


def build():
    build_cpu()
    build_gpu()


if __name__ == "__main__":
    build()
