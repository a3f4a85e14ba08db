"""CPU hygiene of the host code, no GPU:

* a plain C program (tests/c/abi_harness.c) includes include/beamform.h and
  calls the host-only entry points (default configuration, the Eq. (1) bin
  table, status strings, the serving loop's scheduler dry run) -- against the
  built libbeamform.so, and again with the library's host C++ (bf_host.cpp,
  bf_stream.cpp, linked with stand-ins for the device launchers) built with
  AddressSanitizer and UndefinedBehaviorSanitizer;
* the oracle (oracle/oracle.c) built with AddressSanitizer and
  UndefinedBehaviorSanitizer runs its whole pin suite.
Every run must end with status 0 and no sanitizer report."""
import ctypes
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
CSRC = os.path.join(ROOT, "paper_1702_04728_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "c", "abi_harness.c")
STUBS = os.path.join(ROOT, "tests", "c", "device_stubs.cpp")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
REPORT_MARKERS = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:",
                  "SUMMARY: UndefinedBehaviorSanitizer")
# host-side sanitizers on a hipcc line: each -fsanitize= right after -Xarch_host
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _run(cmd, env=None, timeout=600):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, env=env,
                       timeout=timeout)
    out = p.stdout.decode(errors="replace")
    return p.returncode, out


def _clean(out):
    return not any(m in out for m in REPORT_MARKERS)


def test_c_harness_against_library(tmp_path):
    import paper_1702_04728_amd as bf
    if not os.path.exists(bf.LIB_PATH):
        pytest.skip("libbeamform.so is not built")
    exe = str(tmp_path / "abi_harness")
    rc, out = _run(["gcc", "-std=c11", "-O1", "-Wall", "-Werror", "-I", INC, HARNESS, "-o", exe,
                    bf.LIB_PATH, "-Wl,-rpath," + os.path.dirname(bf.LIB_PATH), "-lm"])
    assert rc == 0, out
    rc, out = _run([exe])
    print(out)
    assert rc == 0 and out.strip().endswith("abi harness ok"), out
    # the ctypes binding mirrors the C structs byte for byte
    sizes = next(l for l in out.splitlines() if l.startswith("sizes ")).split()[1:]
    c_sizes = dict(zip(sizes[0::2], (int(v) for v in sizes[1::2])))
    assert c_sizes == {"config": ctypes.sizeof(bf.beamform.BfConfig),
                       "stream_event": ctypes.sizeof(bf.beamform.BfStreamEvent),
                       "stream_desc": ctypes.sizeof(bf.beamform.BfStreamDesc),
                       "stream_stats": ctypes.sizeof(bf.beamform.BfStreamStats)}, c_sizes


def test_host_code_under_asan_ubsan(tmp_path):
    objs = []
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-I", INC] + SAN
    for src in (os.path.join(CSRC, "bf_host.cpp"), os.path.join(CSRC, "bf_stream.cpp"), STUBS):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        rc, out = _run([HIPCC] + flags + ["-c", src, "-o", obj])
        assert rc == 0, out
        objs.append(obj)
    hobj = str(tmp_path / "harness.o")
    rc, out = _run([HIPCC, "-x", "c", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-I", INC]
                   + SAN + ["-c", HARNESS, "-o", hobj])
    assert rc == 0, out
    exe = str(tmp_path / "abi_harness_san")
    rc, out = _run([HIPCC] + SAN + [hobj] + objs + ["-o", exe, "-lm"])
    assert rc == 0, out
    rc, nm = _run(["nm", exe])
    assert "__asan_init" in nm and "__ubsan_handle" in nm, "sanitizers not linked in"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    rc, out = _run([exe], env=env)
    print(out)
    assert rc == 0 and _clean(out) and out.strip().endswith("abi harness ok"), out


def _gcc_runtime(name):
    rc, out = _run(["gcc", "-print-file-name=" + name])
    path = out.strip()
    return path if rc == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = oracle.build_variant(open(os.path.join(ROOT, "oracle", "oracle.c")).read(),
                               str(tmp_path / "liboracle_san.so"),
                               ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                "-fno-sanitize-recover=undefined"])
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan + ":" + ubsan,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    rc, out = _run([sys.executable, "-c", "import sys; sys.path.insert(0, %r); import oracle; "
                    "print(oracle._load()._name)" % ROOT], env=env)
    assert rc == 0 and out.strip().endswith(lib), out   # the pins below use the sanitizer build
    rc, out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                    os.path.join(ROOT, "tests", "test_oracle_pins.py")], env=env, timeout=900)
    print(out[-3000:])
    assert rc == 0 and _clean(out), out[-3000:]
