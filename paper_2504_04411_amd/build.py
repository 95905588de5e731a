"""Builds libhk.so (all HIP sources of csrc/, gfx950) in-tree with hipcc.

Each source is compiled to its own object in parallel (every kernel is launched from the file that
defines it, so no device-side linking is needed), then the objects are linked into the library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhk.so")
OBJ = os.path.join(ROOT, "_build")
ARCH = os.environ.get("HK_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off",                       # float32 ops exactly as written (no fused a*b+c)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _stale(obj: str, src: str) -> bool:
    """An object is stale when it is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [src, os.path.join(ROOT, "include", "hk.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return any(os.path.getmtime(d) > os.path.getmtime(obj) for d in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source (with `incremental`, only those whose object is stale) and links."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = []
    for src in sources():
        obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
        jobs.append(([hipcc] + FLAGS + inc + ["-c", src, "-o", obj], obj, src))
    todo = [cmd for cmd, obj, src in jobs if not incremental or _stale(obj, src)]
    if verbose:
        for cmd in todo:
            print(" ".join(cmd), flush=True)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(subprocess.check_call, cmd) for cmd in todo]:
            f.result()
    link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + [o for _, o, _ in jobs] + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    print(LIB)
    sys.exit(0)
