"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host sources of the library (argument validation in api.cpp and the
multithreaded octree builder in octree_build.cpp, section 4.1's scene-volume
octree) are compiled with g++ and -fsanitize=address,undefined and linked
with the regular device objects into a second copy of the library.  The C-ABI
tests then run against that copy in a child process with the ASan runtime
preloaded (the interpreter itself is not instrumented), and any sanitizer
report fails the test.  GPU code is not instrumented (the device sanitizer is
not used here)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2205_07058_amd")
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
OUT = os.path.join(OBJ, "host_sanitized")
HOST_SOURCES = ("api.cpp", "octree_build.cpp")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def _build_sanitized():
    from paper_2205_07058_amd import build as b
    device_objs = [os.path.join(OBJ, s + ".o") for s in b.SOURCES if not s.endswith(".cpp")]
    if not all(os.path.exists(o) for o in device_objs):
        b.build()
    os.makedirs(OUT, exist_ok=True)
    flags = ["-O1", "-g", "-fPIC", "-std=c++17", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC]
    host_objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(OUT, src + ".o")
        _run(["g++"] + flags + ["-c", os.path.join(CSRC, src), "-o", obj])
        host_objs.append(obj)
    lib = os.path.join(OUT, "libsvlf_host_sanitized.so")
    _run(["g++", "-shared", "-fsanitize=address,undefined", "-o", lib] + host_objs + device_objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
          "-lpthread"])
    return lib


def test_abi_and_host_octree_under_asan_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("g++ ASan runtime not available")
    lib = _build_sanitized()
    nm = _run(["nm", "-D", lib]).stdout
    assert "__asan_report" in nm and "__ubsan_handle" in nm, "sanitizers not linked"
    env = dict(os.environ)
    # the ASan runtime must come first; anything already preloaded stays
    preload = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env.update(SVLF_LIBRARY=lib, LD_PRELOAD=preload,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0 and " passed" in out, out[-6000:]
