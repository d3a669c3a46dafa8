"""Build the gfx950 shared library libgritdbscan.so in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgritdbscan.so")
SOURCES = ["partition.hip", "neighbors.hip", "walk.hip", "core.hip", "merge.hip", "border.hip", "learned.hip",
           "api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off: the compiler must not emit them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-result",
]


def _host_sanitizer_flags(sanitize: str) -> list[str]:
    """Instrument the host half of every source (the gfx950 code is never
    instrumented): each flag is scoped to the host compilation."""
    flags = []
    for f in (f"-fsanitize={sanitize}", "-fno-sanitize=vptr", "-g", "-fno-omit-frame-pointer"):
        flags += ["-Xarch_host", f]
    return flags


def _sanitizer_runtime(sanitize: str) -> str:
    """clang's shared runtime for `sanitize` (UndefinedBehaviorSanitizer's
    standalone one), which the library then lists as a dependency."""
    if sanitize != "undefined":
        raise ValueError("only the host UndefinedBehaviorSanitizer build is supported "
                         "(the others need their runtime preloaded ahead of the interpreter)")
    found = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "llvm", "lib", "clang", "*",
                                          "lib", "linux", "libclang_rt.ubsan_standalone-x86_64.so")))
    if not found:
        raise RuntimeError("libclang_rt.ubsan_standalone-x86_64.so not found beside hipcc")
    return found[-1]


def _compile(src: str, build_dir: str = BUILD, extra: tuple = ()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{out}")
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def build(jobs: int = 6, sanitize: str | None = None) -> str:
    """Compile every kernel source for gfx950 and link the shared library.

    sanitize="undefined" builds a checking variant apart from the product
    library (libgritdbscan_undefined.so, objects in _build_undefined/): the
    host code carries UndefinedBehaviorSanitizer checks that report and
    continue, and the library depends on clang's shared runtime, so it loads
    into an uninstrumented interpreter (select it with GRITDBSCAN_LIBRARY)."""
    build_dir, lib, extra, link_extra = BUILD, LIB, (), []
    if sanitize:
        rt = _sanitizer_runtime(sanitize)
        build_dir = os.path.join(HERE, f"_build_{sanitize}")
        lib = os.path.join(HERE, f"libgritdbscan_{sanitize}.so")
        extra = tuple(_host_sanitizer_flags(sanitize))
        link_extra = [rt, "-Wl,-rpath," + os.path.dirname(rt)]
    os.makedirs(build_dir, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, extra), SOURCES))
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, *link_extra]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(sanitize=sys.argv[1] if len(sys.argv) > 1 else None))
