"""Build step: compile the HIP sources into libspin1.so for gfx950 with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("kernels_xstream.hip", "kernels_sstream.hip", "kernels.hip", "kernels_smodes.hip",
                     "kernels_step.hip", "kernels_aux.hip", "api.hip")]
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspin1.so")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-fvisibility=hidden",
    "-Wall", "-Werror",
    # packed FP32 instructions stay off: some of their forms have given wrong
    # results on this hardware without any error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = os.path.join(rocm, "bin", "hipcc")
    return exe if os.path.exists(exe) else "hipcc"


def _compile(src, verbose):
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    return obj, subprocess.run(cmd, capture_output=True, text=True)


def _errors(res):
    # hipcc's host pass warns that it does not know the packed-fp32 feature: drop that line
    return "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())


def build(verbose=False):
    """Compile libspin1.so in place (always recompiles): every translation unit
    in parallel, then one link."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    for (obj, res), src in zip(results, SOURCES):
        if res.returncode != 0:
            raise RuntimeError("hipcc failed on %s (%d):\n%s" % (os.path.basename(src), res.returncode, _errors(res)))
        if verbose and _errors(res):
            print(_errors(res), file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [obj for obj, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed (%d):\n%s" % (res.returncode, _errors(res)))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
