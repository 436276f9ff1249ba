"""Host-code sanitizer runs (CPU only).

* The FP64 oracle is rebuilt with AddressSanitizer and UndefinedBehaviour-
  Sanitizer and every oracle pin runs against the instrumented copy.
* The HIP library's host code that validates arguments and plans workspaces
  (bp_api.cpp, and bp_core.hip, which holds the level plans) is rebuilt with
  the same sanitizers on its host side only (device code is untouched) and the
  ABI tests run against it.

Each run is a child pytest process with the sanitizer runtime preloaded; a
report aborts the child, so the run fails on any finding.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SOURCES = ["bp_oracle.c", "bp_oracle_adjoint.c", "bp_oracle_remap.c", "bp_oracle_features.c"]
ORACLE_PINS = ["test_oracle_dt.py", "test_oracle_bp.py", "test_oracle_misc.py", "test_oracle_store16.py",
               "test_oracle_adjoint.py", "test_oracle_triangulate.py", "test_oracle_undistort.py",
               "test_oracle_features.py", "test_oracle_icp.py"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def _child(env_extra, tests, libname):
    """Runs pytest on `tests` in a child with the given environment, then
    checks that the instrumented library `libname` was the one loaded."""
    code = ("import os, sys, pytest\n"
            f"rc = pytest.main(['-q', '-s', '-p', 'no:cacheprovider'] + {tests!r})\n"
            f"assert {libname!r} in open('/proc/self/maps').read(), 'instrumented library not loaded'\n"
            "sys.exit(int(rc))\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", **env_extra)
    r = subprocess.run([sys.executable, "-c", code], cwd=os.path.join(ROOT, "tests"), env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.isabs(ubsan)):
        pytest.skip("gcc sanitizer runtimes not found")
    lib = str(tmp_path / "liboracle_san.so")
    srcs = [os.path.join(ROOT, "oracle", s) for s in ORACLE_SOURCES]
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", lib] + srcs + ["-lm"], check=True)
    out = _child({"LD_PRELOAD": f"{asan}:{ubsan}", "BP_TEST_ORACLE_LIB": lib}, ORACLE_PINS, "liboracle_san.so")
    assert " passed" in out


def test_abi_host_code_under_asan_ubsan(tmp_path):
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt or not os.path.exists(HIPCC):
        pytest.skip("clang sanitizer runtime or hipcc not found")
    from paper_1902_09733_amd import build as hip_build
    csrc = hip_build.CSRC
    instrumented = ["bp_api.cpp", "bp_core.hip"]
    objs = {os.path.basename(s): os.path.join(hip_build.OBJ, os.path.basename(s) + ".o") for s in hip_build.sources()}
    if not all(os.path.exists(o) for n, o in objs.items() if n not in instrumented):
        hip_build.build()
    flags = [f for f in hip_build.FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_HOST
    san_objs = []
    for name in instrumented:
        o = str(tmp_path / (name + ".o"))
        lang = ["-x", "hip"] if name.endswith(".cpp") else []
        subprocess.run([HIPCC] + flags + lang + ["-c", os.path.join(csrc, name), "-o", o], check=True,
                       capture_output=True)
        san_objs.append(o)
    lib = str(tmp_path / "libbpstereo_san.so")
    others = [o for n, o in objs.items() if n not in instrumented]
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib] + san_objs + others, check=True,
                   capture_output=True)
    out = _child({"LD_PRELOAD": rt[0], "BP_TEST_LIBRARY": lib}, ["test_abi.py"], "libbpstereo_san.so")
    assert " passed" in out
