"""Build the gfx950 library ``liblbmgrow.so`` in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbmgrow.so")
SOURCES = ["lbm_inst_f64.hip", "lbm_inst_f32.hip", "lbm_inst_f16.hip", "lbm_inst_bf16.hip",
           "lbm_common.hip", "lbm_api.cpp"]

# -ffp-contract=off: every product and sum is rounded on its own (the float64
# path reproduces a sequential float64 evaluation bit for bit).
# -packed-fp32-ops off: no packed fp32 arithmetic is generated.
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def source_files() -> list:
    """Every file the library is compiled from: the C ABI header and the
    sources and headers under csrc/, in a fixed order."""
    files = [os.path.join(ROOT, "include", "lbmgrow.h")]
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            files.append(os.path.join(CSRC, f))
    return files


def source_hash(exclude=()) -> str:
    """First 16 hex digits of the SHA-256 of the library's sources; the
    library built from them reports it in lbm_version()."""
    h = hashlib.sha256()
    for f in source_files():
        if os.path.basename(f) in exclude:
            continue
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit (in parallel) and link liblbmgrow.so.
    incremental: keep the objects compiled from exactly the current sources
    (each object records the source hash taken before it was compiled, so a
    source edited during a build cannot leave a stale object behind)."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    flags = [f for f in HIPFLAGS if f != "-shared"]
    tree = source_hash()
    # what the kernel units are compiled from (they do not include the C ABI
    # unit, which carries the hash of everything and is always rebuilt)
    kernels = source_hash(exclude=("lbm_api.cpp",))

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        stamp = obj + ".src"
        extra = [f'-DLBM_SOURCE_HASH="{tree}"'] if src == "lbm_api.cpp" else []
        if incremental and not extra and os.path.exists(obj) and os.path.exists(stamp):
            with open(stamp) as fh:
                if fh.read().strip() == kernels:
                    return obj
        if os.path.exists(stamp):
            os.remove(stamp)
        cmd = [hipcc(), *flags, *extra, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{err}")
        if err.strip() and verbose:
            print(err, flush=True)
        with open(stamp, "w") as fh:
            fh.write(kernels)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    if source_hash() != tree:
        raise RuntimeError("a source changed while the library was being built: build again")
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="-i" in sys.argv)
