"""Sanitizer builds on the CPU: the FP64 oracle built with AddressSanitizer
and UndefinedBehaviorSanitizer runs its pins, and the library's host code
(argument checks, context creation without a device, the tune store and its
JSON reader) built the same way runs tests/sanitize/abi_host.c.  Any
sanitizer report fails the build's run (errors are not recoverable)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# sanitizers on the host side of every hipcc line (there is no GPU code here)
HOST_SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all".split()


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None or _gcc_runtime("libasan.so") is None,
                    reason="gcc with libasan needed")
def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
          os.path.join(ROOT, "oracle", "dgal_oracle.c"),
          os.path.join(ROOT, "oracle", "simple_oracle.c"), "-o", lib, "-lm"])
    env = dict(os.environ, LD_PRELOAD=_gcc_runtime("libasan.so"), DGAL_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
              os.path.join(ROOT, "tests", "test_oracle_pins.py"),
              os.path.join(ROOT, "tests", "test_oracle_simple.py")], env=env, cwd=ROOT,
             timeout=900)
    assert " passed" in r.stdout and "ERROR" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc needed")
def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2011_11134_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include")]
    objs = []
    for src, lang in ((os.path.join(csrc, "api.hip"), []),
                      (os.path.join(csrc, "tune_cache.cpp"), []),
                      (os.path.join(ROOT, "tests", "sanitize", "device_stubs.cpp"), []),
                      (os.path.join(ROOT, "tests", "sanitize", "abi_host.c"), ["-x", "c"])):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        std = [] if lang else ["-std=c++17"]
        _run([HIPCC, "--offload-host-only", "-O1", "-g", "-fno-omit-frame-pointer", *std,
              *HOST_SAN, *inc, *lang, "-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "abi_host")
    _run([HIPCC, *HOST_SAN, *objs, "-o", exe])
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", HIP_VISIBLE_DEVICES="",
               ROCR_VISIBLE_DEVICES="")
    r = _run([exe, str(scratch)], env=env, timeout=600)
    assert "abi_host ok" in r.stdout
