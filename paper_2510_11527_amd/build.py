"""Build the HIP library libaf4.so (gfx950) in-tree with hipcc.

    python -m paper_2510_11527_amd.build

Every translation unit is compiled in parallel into _build/, then linked.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libaf4.so")
SOURCES = ["af_runtime.cpp", "aux_kernels.hip", "stage_d1.hip", "stage_d2.hip", "stage_d3.hip"]
ARCH = os.environ.get("AF4_OFFLOAD_ARCH", "gfx950")


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-variable",
            "-Wno-unused-but-set-variable",
            # packed FP32 instructions stay off (v_pk_* forms are avoided on this target)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # the backend's iterative ILP scheduler: the stage kernels wait on
            # latency at an occupancy their LDS fixes, and this schedule keeps
            # each kernel's occupancy while shortening its critical path
            # (1-2% per stage on the 2D, 3D and 1D kernels; the greedy max-ILP
            # strategy raises the 1D kernel's registers past five waves)
            "-mllvm", "-amdgpu-sched-strategy=iterative-ilp",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src, incremental=False):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) >= max(
            os.path.getmtime(os.path.join(CSRC, src)), _deps_header_mtime(src)):
        return src, obj, 0, ""
    cmd = [hipcc()] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return src, obj, r.returncode, out


def _deps_header_mtime(src):
    """Latest modification time of the headers (every translation unit is
    taken to include all of them)."""
    files = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".hpp"))]
    files.append(os.path.join(ROOT, "include", "af.h"))
    return max(os.path.getmtime(f) for f in files)


def build(verbose=True, incremental=False):
    """Compile every translation unit and link libaf4.so.  incremental=True
    skips units whose object is newer than the unit and every header."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        results = list(ex.map(lambda f: _compile(f, incremental), SOURCES))
    failed = [r for r in results if r[2] != 0]
    for src, _, rc, out in results:
        if out and (verbose or rc):
            print("[%s]\n%s" % (src, out), file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(r[0] for r in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [r[1] for r in results]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(incremental="--incremental" in sys.argv))
