"""Build libfespmv.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfespmv.so")
SOURCES = ["api.cpp", "layout.cpp", "solver.cpp", "server.cpp", "kernels.hip",
           "engine.hip", "batch.hip", "persist.hip", "csr.hip", "asm.cpp",
           "asm.hip", "build.hip", "noalloc.hip", "wgsolve.hip"]
ARCH = os.environ.get("FESPMV_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (the compiler would otherwise form
    # them from scalar float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Host code built with AddressSanitizer and UndefinedBehaviorSanitizer
# (device code unchanged): a checking build of the library's host paths
# (validation, layout builder, assembly planner), loaded by a Python process
# started with the sanitizer runtime preloaded (FESPMV_LIB names it).
LIB_SAN = os.path.join(HERE, "libfespmv_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def sanitizer_runtime():
    """Path of clang's shared AddressSanitizer runtime (to preload)."""
    import glob
    root = os.environ.get("ROCM_PATH", "/opt/rocm")
    hits = sorted(glob.glob(os.path.join(
        root, "lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")))
    return hits[-1] if hits else None


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + \
        [os.path.join(HERE, "..", "include", "fespmv.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def needs_build_sanitized():
    if not os.path.exists(LIB_SAN):
        return True
    t = os.path.getmtime(LIB_SAN)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + \
        [os.path.join(HERE, "..", "include", "fespmv.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build_sanitized(verbose=False):
    """libfespmv_san.so: the library with ASan + UBSan host code."""
    return build(verbose, lib=LIB_SAN, extra=SAN_FLAGS, opt="-O1")


def build(verbose=False, lib=LIB, extra=(), opt="-O3"):
    objs = []
    procs = []
    tag = ".san" if extra else ""
    flags = [f if f != "-O3" else opt for f in FLAGS] + list(extra)
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src) + tag + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = ["hipcc", *flags, *lang, "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
        objs.append(obj)
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines()
                         if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError("hipcc failed: %s\n%s" % (" ".join(cmd), text))
        if verbose and text.strip():
            print(text, file=sys.stderr)
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "--offload-arch=" + ARCH, "-shared",
                           "-fPIC", *extra, *objs, "-o", tmp])
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
