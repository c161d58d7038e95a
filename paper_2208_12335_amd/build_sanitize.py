"""Host-sanitized build of the library for CPU-side checks: the host code of every source (set-up,
validation, batching, the density-matrix driver) compiled with AddressSanitizer and
UndefinedBehaviorSanitizer, the device code unchanged.  Output: ``libaimsgrid_san.so`` next to
the regular library.  It is loaded with the sanitizer runtime preloaded, e.g.

    LD_PRELOAD=$(python -m paper_2208_12335_amd.build_sanitize --runtime) \\
        AIMS_LIB=paper_2208_12335_amd/libaimsgrid_san.so python -m pytest tests/test_abi_cpu.py
"""
import glob
import os
import sys

from .build import ARCH, CSRC, HERE, ROOT, SOURCES, _hipcc, _run

LIB_SAN = os.path.join(HERE, "libaimsgrid_san.so")
# every -fsanitize option applies to the host compilation only (-Xarch_host before each)
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str:
    """Path of the AddressSanitizer runtime of the ROCm clang (to preload into Python)."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("AddressSanitizer runtime not found under /opt/rocm/llvm")
    return hits[-1]


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-mfma-vgpr-form",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SAN_HOST]
    bdir = os.path.join(HERE, "_build_san")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".", "_") + ".o")
        _run([hipcc, *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB_SAN + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_HOST, "-shared-libasan", "-o", tmp,
          *objs, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocsolver", "-lrocblas",
          "-lrocprofiler-sdk-roctx", "-lpthread"], verbose)
    os.replace(tmp, LIB_SAN)
    return LIB_SAN


if __name__ == "__main__":
    if "--runtime" in sys.argv:
        print(runtime())
    else:
        print(build(verbose="-v" in sys.argv))
