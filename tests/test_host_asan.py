"""The library's host logic under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

The host C++ files (plan creation and validation, workspace layout, reduced
padding, the batched plan's instance table and radix schedules, the plan
log) are compiled host-only with the sanitizers and linked, together with the
regular kernel objects of the in-tree build, into the driver
tests/host_asan/abi_host_checks.cpp.  The driver runs thousands of seeded
random plan and batch-plan creations and the refusals of the C ABI; none of
these paths makes a device call, so no GPU is needed."""

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1112_3010_amd")
CSRC = os.path.join(PKG, "csrc")
DRIVER = os.path.join(ROOT, "tests", "host_asan", "abi_host_checks.cpp")
HOST_SOURCES = ["plan.cpp", "batch.cpp", "log.cpp"]


def _tool(path, name):
    for cand in (path, shutil.which(name)):
        if cand and os.path.exists(cand):
            return cand
    return None


def _kernel_objects():
    """Objects of the regular build for every .hip source (device code plus
    their launchers); built here if the in-tree build has not run."""
    from paper_1112_3010_amd import build as b
    hips = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs = [os.path.join(b.BUILD, f + ".o") for f in hips]
    if not all(os.path.exists(o) for o in objs):
        b.build()
    return objs


def test_host_code_under_sanitizers(tmp_path):
    hipcc = _tool("/opt/rocm/bin/hipcc", "hipcc")
    clang = _tool("/opt/rocm/llvm/bin/clang++", "amdclang++")
    if not hipcc or not clang:
        pytest.skip("ROCm compilers not found")
    kobjs = _kernel_objects()
    # host-only compilation; each sanitizer flag applies to the host pass
    flags = ["--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    srcs = [os.path.join(CSRC, f) for f in HOST_SOURCES] + [DRIVER]
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]

    def compile_one(src, obj):
        return subprocess.run([hipcc, *flags, "-c", src, "-o", obj], capture_output=True, text=True)

    with cf.ThreadPoolExecutor(4) as ex:
        for src, res in zip(srcs, ex.map(compile_one, srcs, objs)):
            assert res.returncode == 0, f"{os.path.basename(src)}:\n{res.stderr[-3000:]}"
    exe = str(tmp_path / "abi_host_checks")
    link = [clang, "-fsanitize=address,undefined", *objs, *kobjs, "-L/opt/rocm/lib", "-lamdhip64",
            "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    res = subprocess.run(link, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env.pop("DT_LOG", None)
    res = subprocess.run([exe, "3000", "300"], capture_output=True, text=True, env=env, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "all host checks passed" in res.stdout
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
    print(res.stdout)
    # the plan log's formatting paths, on fewer plans
    env["DT_LOG"] = "1"
    res = subprocess.run([exe, "300", "30"], capture_output=True, text=True, env=env, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "[dt] plan " in res.stderr and "[dt] batch plan " in res.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
