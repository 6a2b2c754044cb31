"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the C ABI unit is compiled with both sanitizers (host side only),
linked with the kernel objects of the in-tree build and a C driver
(tests/host/abi_sanitize.c) that sweeps parameter validation, layout and
workspace sizes, argument checks and an empty batch's life cycle.  Any
sanitizer report fails the run (UBSan does not recover; ASan checks leaks at
exit)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2303_02210_amd")
OBJ = os.path.join(PKG, "_build")
KERNEL_UNITS = ["lbm_inst_f64", "lbm_inst_f32", "lbm_inst_f16", "lbm_inst_bf16", "lbm_common"]
LLVM = "/opt/rocm/llvm/bin"


def _kernel_objects():
    from paper_2303_02210_amd import build
    want = build.source_hash(exclude=("lbm_api.cpp",))
    objs = []
    for u in KERNEL_UNITS:
        o = os.path.join(OBJ, u + ".o")
        try:
            with open(o + ".src") as fh:
                if fh.read().strip() != want:
                    return None
        except OSError:
            return None
        objs.append(o)
    return objs


def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not (os.path.exists(hipcc) and os.path.exists(os.path.join(LLVM, "clang"))):
        pytest.skip("ROCm toolchain not available")
    objs = _kernel_objects()
    if objs is None:
        pytest.skip("kernel objects not built from this tree (python paper_2303_02210_amd/build.py -i)")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    api = str(tmp_path / "lbm_api_san.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "abi_sanitize")
    # host side only: every sanitizer flag of the hipcc line goes to the host pass
    host_san = []
    for f in san:
        host_san += ["-Xarch_host", f]
    steps = [
        [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
         "-fno-omit-frame-pointer", *host_san, *inc, '-DLBM_SOURCE_HASH="sanitize"',
         "-c", os.path.join(PKG, "csrc", "lbm_api.cpp"), "-o", api],
        [os.path.join(LLVM, "clang"), "-O1", "-g", "-fno-omit-frame-pointer", *san, *inc,
         "-c", os.path.join(ROOT, "tests", "host", "abi_sanitize.c"), "-o", drv],
        [os.path.join(LLVM, "clang++"), *san, "-o", exe, drv, api, *objs,
         "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, (cmd[0], r.stderr[-3000:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "abi_sanitize ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
