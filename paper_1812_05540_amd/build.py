"""Build libps.so (HIP for gfx950 + host C++) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libps.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PS_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
          "-I" + os.path.join(HERE, "..", "include")]
# HIP device code is built without packed-FP32 instructions: some of their forms have
# produced wrong results, without an error, on MI355X.
HIP_FLAGS = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-munsafe-fp-atomics"]
SOURCES = [
    # (file, extra flags); host setup is evaluated without FMA contraction so that
    # its floating-point sums are reproducible in a fixed order
    ("host_setup.cpp", ["-x", "c++", "-ffp-contract=off"]),
    ("device.hip", HIP_FLAGS),
    ("galerkin.hip", HIP_FLAGS),
    ("api.cpp", HIP_FLAGS),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n  %s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    cmds = []
    for name, flags in SOURCES:
        obj = os.path.join(OBJ, name + ".o")
        objs.append(obj)
        cmds.append([HIPCC] + COMMON + flags + ["-c", os.path.join(SRC, name), "-o", obj])
    with ThreadPoolExecutor(max_workers=4) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = OUT + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
