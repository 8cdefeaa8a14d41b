"""Build libheatbem.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2102_09811_amd._build        # or __graft_entry__.build()
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libheatbem.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include")]
# MFMA accumulators stay in ordinary VGPRs (gfx950 allows it), which avoids copies to and from
# the accumulation registers around every chain of matrix instructions.
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-amdgpu-mfma-vgpr-form=1"]


def _compile(src, obj):
    cmd = [HIPCC] + COMMON + (DEVICE if src.endswith(".hip") else []) + ["-c", src, "-o", obj]
    subprocess.check_call(cmd)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    if verbose:
        print("[build] hipcc", " ".join(os.path.basename(s) for s in srcs), flush=True)
    # one hipcc per source, several at a time
    from concurrent.futures import ThreadPoolExecutor
    jobs = max(1, min(len(srcs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_compile, s, o) for s, o in zip(srcs, objs)]:
            f.result()
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, OUT)
    if verbose:
        print("[build] wrote", OUT, flush=True)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
