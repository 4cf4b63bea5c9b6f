"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

The host runtime (csrc/capi.hip: validation, layouts, footprints, graph and
checkpoint bookkeeping) is compiled for the host only with both sanitizers and
linked with the objects of the other sources from the regular build (device code
is not instrumented); a plain C program (tests/abi_host_driver.c) then drives every
path that returns before touching a device.  Any out-of-bounds access, use
after free, signed overflow, misaligned or null dereference ends the run.
"""
import glob
import importlib.util
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_04069_amd", "csrc")
LLVM = "/opt/rocm/llvm"
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = os.path.join(LLVM, "bin", "clang")
CLANGXX = os.path.join(LLVM, "bin", "clang++")


def _build_module():
    # build.py by path: importing the package would load the regular library
    spec = importlib.util.spec_from_file_location("pm_build", os.path.join(ROOT, "paper_1607_04069_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed:\n{r.stdout}\n{r.stderr}"
    return r


def test_host_paths_are_clean_under_sanitizers(tmp_path):
    rt = glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG) and rt):
        pytest.skip("no ROCm clang with sanitizer runtimes")
    B = _build_module()
    os.makedirs(B.OUT_DIR, exist_ok=True)
    kernels = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        if os.path.basename(src) == "capi.hip":
            continue
        obj = os.path.join(B.OUT_DIR, os.path.basename(src) + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src):
            obj = B._compile(src)
        kernels.append(obj)
    host_obj = str(tmp_path / "capi_san.o")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-host-only",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, "capi.hip"), "-o", host_obj])
    lib = str(tmp_path / "libpicmcc_san.so")
    _run([CLANGXX, "-shared", "-fsanitize=address,undefined", "-shared-libasan", host_obj, *kernels,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", lib])
    exe = str(tmp_path / "abi_host_driver")
    _run([CLANG, "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-shared-libasan",
          "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_host_driver.c"),
          "-L", str(tmp_path), "-lpicmcc_san", f"-Wl,-rpath,{tmp_path}", "-lm", "-o", exe])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["LD_LIBRARY_PATH"] = os.pathsep.join([os.path.dirname(rt[0]), env.get("LD_LIBRARY_PATH", "")])
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
