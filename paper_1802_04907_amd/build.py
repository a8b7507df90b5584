"""Build libqiht.so (HIP for gfx950) in-tree.

Usage: python -m paper_1802_04907_amd.build   (or build() from Python)
       python -m paper_1802_04907_amd.build --host-sanitizers   (ASan/UBSan
       build of the host code into _build/host_san/, for the CPU tests)

Every HIP source is compiled for gfx950 with packed FP32 instructions
disabled; the quantizer is compiled without floating-point contraction so
its FP64 rounding positions are the plain IEEE results.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqiht.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("QIHT_OFFLOAD_ARCH", "gfx950")

COMMON = ["-I" + os.path.join(os.path.dirname(HERE), "include"), "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]
PER_FILE = {"quantize.hip": ["-ffp-contract=off"]}
SOURCES = ["api.hip", "quantize.hip", "gather.hip", "pass.hip", "select.hip", "refit.hip", "gemm.hip", "solve_host.hip", "fourier.hip", "complex.hip"]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _compile(src):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + \
        PER_FILE.get(src, [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


# Host-sanitizer build: every source with its host code compiled under
# AddressSanitizer and UndefinedBehaviorSanitizer (the device code as
# usual), linked against the shared sanitizer runtime.  Loaded instead of
# libqiht.so through QIHT_LIB_PATH, with that runtime preloaded.
SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()
SAN_DIR = os.path.join(BUILD, "host_san")
SAN_LIB = os.path.join(SAN_DIR, "libqiht_san.so")


def sanitizer_runtime():
    """Path of the shared ASan runtime of ROCm's clang (None if absent)."""
    import glob
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "llvm", "lib", "clang")
    hits = sorted(glob.glob(os.path.join(root, "*", "lib", "*", "libclang_rt.asan-x86_64.so")))
    if not hits:
        hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/*/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _compile_san(src):
    obj = os.path.join(SAN_DIR, src.replace(".hip", ".o"))
    flags = [f if f != "-O3" else "-O1" for f in COMMON]
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj, "-g"] + flags + PER_FILE.get(src, []) + \
        SANITIZE + ["-Xarch_host", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build_host_sanitized(verbose=False):
    os.makedirs(SAN_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile_san, SOURCES))
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC", "-shared-libsan"] + SANITIZE
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    if "--host-sanitizers" in sys.argv[1:]:
        build_host_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
