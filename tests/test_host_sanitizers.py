"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two sanitized builds are made in a temporary directory:
- the oracle (gmpea_oracle.c) with gcc's ASan + UBSan;
- the library's host sources (gmpea_abi.cpp, lattice.cpp) with clang's ASan +
  UBSan on the host pass only, linked with the kernel objects of the in-tree
  build (device code is not instrumented).
The oracle's pins and the ABI's CPU tests then run against those builds in a
child process that preloads the sanitizer runtime, and any report fails the
test. A planted heap overflow and a planted signed overflow, built the same
way, show that each runtime reports what it should.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2509_19821_amd import build as libbuild  # noqa: E402

HOST_SOURCES = ("gmpea_abi.cpp", "lattice.cpp")
KERNEL_OBJECTS = ("gmpea_kernels.o", "gmpea_kernels_wide.o")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
GCC_SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"]
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _gcc_runtime():
    return ":".join(subprocess.run(["gcc", "-print-file-name=" + n], check=True, capture_output=True,
                                   text=True).stdout.strip() for n in ("libasan.so", "libubsan.so"))


def _clang_runtime():
    llvm = os.path.join(os.path.dirname(os.path.dirname(libbuild.hipcc())), "llvm")
    out = subprocess.run([os.path.join(llvm, "bin", "clang"), "-print-resource-dir"], check=True,
                         capture_output=True, text=True).stdout.strip()
    for sub in ("lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so", "lib/linux/libclang_rt.asan-x86_64.so"):
        p = os.path.join(out, sub)
        if os.path.exists(p):
            return p
    pytest.skip("clang's shared ASan runtime is not installed")


def _env(preload, **extra):
    env = dict(os.environ)
    env.update(LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4",
               PYTHONPATH=ROOT)
    env.update(extra)
    return env


def _run(cmd, env, timeout=600):
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return p.returncode, p.stdout + p.stderr


@pytest.fixture(scope="module")
def san(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    d = tmp_path_factory.mktemp("sanitized")
    orc = str(d / "libgmpea_oracle_san.so")
    subprocess.run(["gcc"] + GCC_SAN + ["-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", orc,
                                         os.path.join(ROOT, "oracle", "gmpea_oracle.c"), "-lm"], check=True)
    objs = [os.path.join(libbuild.OUT_DIR, o) for o in KERNEL_OBJECTS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("the in-tree library is not built (its kernel objects are missing)")
    libdir = d / "lib"
    libdir.mkdir()
    flags = [f for f in libbuild.flags() if f != "-O3"] + ["-O1"] + SAN_HOST
    for src in HOST_SOURCES:
        obj = str(d / (os.path.splitext(src)[0] + ".o"))
        subprocess.run([libbuild.hipcc()] + flags + ["-x", "hip", "-c", os.path.join(libbuild.CSRC, src),
                                                    "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    lib = str(libdir / "libgmpea.so")
    subprocess.run([libbuild.hipcc(), "--offload-arch=" + libbuild.ARCH, "-shared", "-fPIC", "-o", lib] + objs
                   + libbuild.LIBS + SAN_HOST[:4], check=True, capture_output=True)
    shutil.copy(os.path.join(libbuild.OUT_DIR, "build_info.json"), str(libdir))
    return {"dir": d, "oracle": orc, "lib": lib, "gcc_rt": _gcc_runtime(), "clang_rt": _clang_runtime()}


def _clean(rc, out):
    assert rc == 0, out[-4000:]
    for r in REPORTS:
        assert r not in out, out[-4000:]


def test_oracle_pins_under_sanitizers(san):
    """The oracle's structure, operator, RNG, generation, selection and
    many-objective pins, and the robustness classifier's curve cases."""
    tests = ["tests/test_oracle_structures.py", "tests/test_oracle_operators.py", "tests/test_oracle_rng.py",
             "tests/test_oracle_generation.py", "tests/test_oracle_selection.py", "tests/test_oracle_many.py",
             "tests/test_oracle_robustness.py", "-k", "not robustness or curve"]
    rc, out = _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                   + tests, _env(san["gcc_rt"], GMPEA_ORACLE_LIBRARY=san["oracle"]))
    _clean(rc, out)
    assert " passed" in out


def test_library_host_code_under_sanitizers(san):
    """Argument validation, dead handles, the host lattice and layered
    reference sets against brute force, and the prototypes, on the sanitized
    host code."""
    rc, out = _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                    "tests/test_abi.py", "tests/test_bindings.py"],
                   _env(san["clang_rt"], GMPEA_LIBRARY=san["lib"]))
    _clean(rc, out)
    assert " passed" in out


PLANTED = textwrap.dedent("""
    #include <stdlib.h>
    int heap_past_end(int n) { int *a = (int *)malloc(n * sizeof(int)); a[n] = 1; int v = a[0]; free(a); return v; }
    int signed_overflow(int x) { return x + 2147483647; }
""")


@pytest.mark.parametrize("runtime", ["gcc", "clang"])
@pytest.mark.parametrize("fn,report", [("heap_past_end", "heap-buffer-overflow"),
                                       ("signed_overflow", "runtime error:")])
def test_sanitizers_report_planted_errors(san, runtime, fn, report):
    src = san["dir"] / "planted.c"
    src.write_text(PLANTED)
    so = str(san["dir"] / ("planted_%s.so" % runtime))
    if runtime == "gcc":
        subprocess.run(["gcc"] + GCC_SAN + ["-fPIC", "-shared", "-o", so, str(src)], check=True)
        rt = san["gcc_rt"]
    else:
        subprocess.run([libbuild.hipcc(), "-O1", "-fPIC", "-shared", "-x", "c", "-o", so, str(src)] + SAN_HOST[:6],
                       check=True, capture_output=True)
        rt = san["clang_rt"]
    code = "import ctypes; L = ctypes.CDLL(%r); print(getattr(L, %r)(4))" % (so, fn)
    rc, out = _run([sys.executable, "-c", code], _env(rt), timeout=120)
    assert rc != 0 and report in out, out[-2000:]
