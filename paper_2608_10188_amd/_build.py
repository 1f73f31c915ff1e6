"""Build the HIP library (gfx950) in-tree: paper_2608_10188_amd/libaceapex.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libaceapex.so")
SOURCES = ["csrc/decoder.hip", "csrc/range.hip", "csrc/encoder.cpp", "csrc/ax_common.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build_library():
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-o", LIB + ".tmp", "-l:libxxhash.so.0"]
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build_library()
