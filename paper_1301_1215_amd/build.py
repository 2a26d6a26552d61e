"""Build libnlinv.so for gfx950 with hipcc (in-tree, no JIT cache).

Each grid size is one translation unit (csrc/inst.hip with -DNLINV_SIZE=n),
compiled in parallel; the host library csrc/nlinv_lib.hip links them.
Usage: python -m paper_1301_1215_amd.build [-j JOBS]
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libnlinv.so")

SIZES = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
ARCH = os.environ.get("NLINV_OFFLOAD_ARCH", "gfx950")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (v_pk_* forms are avoided on purpose)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def _deps(src):
    """Sources an object depends on: the .hip file, the headers it includes
    from csrc/ (transitively) and include/nlinv.h."""
    import re
    seen, todo = set(), [src]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(f):
            continue
        seen.add(f)
        for inc in re.findall(r'#include\s+"([^"]+)"', open(f).read()):
            for d in (CSRC, INCLUDE):
                if os.path.exists(os.path.join(d, inc)):
                    todo.append(os.path.join(d, inc))
    return seen


def _stale(obj, src):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(src))


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every object and link the library; with `incremental`, only
    objects older than one of their sources."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    objs = []
    cmds = []
    inst = os.path.join(CSRC, "inst.hip")
    for n in SIZES:
        o = os.path.join(BUILD, f"inst_{n}.o")
        objs.append(o)
        if not incremental or _stale(o, inst):
            cmds.append([HIPCC, *FLAGS, f"-DNLINV_SIZE={n}", "-c", inst, "-o", o])
    lib_src = os.path.join(CSRC, "nlinv_lib.hip")
    lib_o = os.path.join(BUILD, "nlinv_lib.o")
    objs.append(lib_o)
    if not incremental or _stale(lib_o, lib_src):
        cmds.append([HIPCC, *FLAGS, "-c", lib_src, "-o", lib_o])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


SAN_LIB = os.path.join(PKG, "libnlinv_san.so")
# host code only: each sanitizer flag applies to the host compilation (the
# GPU code objects are the same as the library's)
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """The ASan runtime of the host compiler (to preload into a process that
    loads the sanitised library)."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    hits = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")) +
                  glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found")
    return hits[-1]


def build_sanitized(jobs: int | None = None) -> str:
    """libnlinv_san.so: the host library compiled with AddressSanitizer and
    UndefinedBehaviorSanitizer (the pass-kernel objects of build() reused)."""
    build(jobs, incremental=True)
    lib_o = os.path.join(BUILD, "nlinv_lib_san.o")
    _run([HIPCC, *FLAGS, *SAN_FLAGS, "-c", os.path.join(CSRC, "nlinv_lib.hip"), "-o", lib_o])
    objs = [os.path.join(BUILD, f"inst_{n}.o") for n in SIZES] + [lib_o]
    tmp = SAN_LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", tmp, *objs])
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("-i", "--incremental", action="store_true", help="rebuild only stale objects")
    ap.add_argument("--sanitize", action="store_true",
                    help="also build libnlinv_san.so (host code under ASan and UBSan)")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose, a.incremental))
    if a.sanitize:
        print(build_sanitized(a.jobs))


if __name__ == "__main__":
    sys.exit(main())
