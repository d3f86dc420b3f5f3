"""Build libomniseg.so for gfx950 in-tree.

Every HIP source is compiled with hipcc for gfx950 only; the shared library
is linked against the HIP runtime that torch loads (torch/lib), so device
pointers and hipStream_t handles from torch are valid inside the library.
Usage: python -m paper_2305_14566_amd.build  (or build() from Python).
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libomniseg.so")
SOURCES = ["k_prep.hip", "k_tissue.hip", "k_map.hip", "k_conv.hip", "k_head.hip", "k_stitch.hip", "k_pack.hip", "k_bwd.hip", "api.cpp", "api_train.cpp", "api_map.cpp", "api_noalloc.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-mcode-object-version=5",
    # packed FP32 forms stay off: hipcc -O3 would otherwise emit them from float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _torch_lib():
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("torch is required for its HIP runtime")
    return os.path.join(list(spec.submodule_search_locations)[0], "lib")


def _compile(src, hipcc):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc, *HIPCC_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    """Compile every source and link libomniseg.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc), SOURCES))
    tlib = _torch_lib()
    tmp = LIB + ".tmp"
    cmd = ["g++", "-shared", "-o", tmp, *objs, f"-L{tlib}", "-l:libamdhip64.so",
           f"-Wl,-rpath,{tlib}", "-Wl,--no-undefined", "-Wl,-z,defs"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host sanitizers for the C-ABI sources: every api*.cpp file is compiled with
# AddressSanitizer and UndefinedBehaviorSanitizer on its host code only (device
# code is built as usual) and linked with the normally built kernel objects.
# The result needs the clang ASan runtime preloaded (sanitizer_runtime()).
SANITIZED_LIB = os.path.join(BUILD, "sanitized", "libomniseg_sanitized.so")
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-shared-libasan"]


def sanitizer_runtime():
    """Path of clang's shared ASan runtime (with the UBSan handlers)."""
    r = subprocess.run([os.path.join(os.path.dirname(_hipcc()), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(p) or not os.path.exists(p):
        import glob
        cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        if not cands:
            raise RuntimeError("clang ASan runtime not found")
        p = cands[-1]
    return os.path.realpath(p)


def build_sanitized(verbose=False):
    """Build the library with host ASan + UBSan on the C-ABI sources."""
    sdir = os.path.dirname(SANITIZED_LIB)
    os.makedirs(sdir, exist_ok=True)
    hipcc = _hipcc()
    kernels = [s for s in SOURCES if s.endswith(".hip")]
    hosts = [s for s in SOURCES if not s.endswith(".hip")]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        kobjs = list(ex.map(lambda s: _compile(s, hipcc), kernels))

        def comp_san(src):
            obj = os.path.join(sdir, os.path.basename(src) + ".o")
            cmd = [hipcc, *HIPCC_FLAGS, *HOST_SANITIZE, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
            return obj

        hobjs = list(ex.map(comp_san, hosts))
    tlib = _torch_lib()
    tmp = SANITIZED_LIB + ".tmp"
    cmd = ["g++", "-shared", "-o", tmp, *kobjs, *hobjs, f"-L{tlib}", "-l:libamdhip64.so", f"-Wl,-rpath,{tlib}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SANITIZED_LIB)
    if verbose:
        print("built", SANITIZED_LIB)
    return SANITIZED_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
