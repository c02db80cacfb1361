"""Build libshellhom.so (HIP kernels + host runtime + C ABI) for gfx950 in-tree.

    python -m paper_2511_04025_amd.build

Compiles every translation unit under csrc/ with hipcc and links one shared
library next to this file.  Packed FP32 instructions are disabled
(-target-feature -packed-fp32-ops); the host pass warns that it does not know
that feature, which is harmless.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libshellhom.so")
ARCH = os.environ.get("SHH_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required)")


FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(HERE, "..", "include"),
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build(verbose=True, out=None, defines=()):
    """Compile and link; `out` and `defines` (-D macros) build a variant
    elsewhere for A/B timing, the default is the in-tree library."""
    lib = out or LIB
    obj_dir = OBJ if out is None else os.path.join(os.path.dirname(os.path.abspath(out)), "_obj_" +
                                                    os.path.basename(out))
    os.makedirs(obj_dir, exist_ok=True)
    srcs = sources()
    extra = [f"-D{d}" for d in defines]

    def comp(src):
        o = os.path.join(obj_dir, os.path.basename(src) + ".o")
        cmd = [hipcc()] + FLAGS + extra + ["-c", src, "-o", o]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return o

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    LIB_OUT = lib
    tmp = LIB_OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_OUT)
    if verbose:
        print(f"built {LIB_OUT}")
    return LIB_OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
