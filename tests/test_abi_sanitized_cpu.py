"""The C-ABI tests run against a build of the library whose host code is compiled with
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged).  Argument checks, error
paths, tuning knobs and the symbol table go through the sanitized host code; any report of the
sanitizers ends the child process with an error.  CPU only: no GPU call succeeds here."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1904_11201_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "asan")
LIB = os.path.join(OUT, "libjoin_asan.so")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-shared-libasan", "-Xarch_host", "-fno-omit-frame-pointer"]


def _asan_runtime():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return rt[-1] if rt else None


def _build():
    from paper_1904_11201_amd import build as B
    srcs = B.sources()
    deps = srcs + glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(f) for f in deps):
        return
    os.makedirs(OUT, exist_ok=True)
    flags = [f for f in B.CFLAGS if f != "-O3"] + ["-O1", "-g"] + SAN
    procs = [subprocess.Popen(["hipcc", *flags, "-c", s, "-o", os.path.join(OUT, os.path.basename(s) + ".o")],
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for s in srcs]
    for p in procs:
        out = p.communicate()[0]
        assert p.returncode == 0, out.decode()[-2000:]
    objs = [os.path.join(OUT, os.path.basename(s) + ".o") for s in srcs]
    subprocess.check_call(["hipcc", f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *objs,
                           "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host",
                           "-shared-libasan", "-o", LIB])


CHECK = r'''
import paper_1904_11201_amd._native as n
maps = open("/proc/self/maps").read()
assert "libclang_rt.asan" in maps and "libjoin_asan.so" in maps, "sanitized library not mapped"
print("mapped", n.LIB_PATH)
'''


def test_abi_under_address_and_undefined_behavior_sanitizers():
    rt = _asan_runtime()
    if rt is None or subprocess.run(["which", "hipcc"], capture_output=True).returncode != 0:
        pytest.skip("hipcc or the AddressSanitizer runtime is not installed")
    _build()
    env = dict(os.environ, JOIN_LIBRARY=LIB, LD_PRELOAD=rt, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", CHECK], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0 and "mapped" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
