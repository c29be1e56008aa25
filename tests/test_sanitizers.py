"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle (plain C) driven through every function on small inputs, and the
host side of libpir.so (hipcc, sanitizers on the host code only: each
-fsanitize flag goes to the host compiler through -Xarch_host) driven
through the argument checks and error paths of its C ABI.  Neither run
touches a GPU; a sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.slow


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", exe, os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(HERE, "oracle_driver.c")])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="4"), timeout=300)
    assert "oracle driver ok" in r.stdout


HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_host_abi_under_asan_ubsan(tmp_path):
    from paper_2604_04696_amd import build as hb
    objs = []
    for src in hb.sources():
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize=vptr", "-Xarch_host", "-fno-omit-frame-pointer",
             f"-I{os.path.join(ROOT, 'include')}"]
    procs = [subprocess.Popen([HIPCC, *flags, "-c", src, "-o", obj], stdout=subprocess.PIPE,
                              stderr=subprocess.PIPE, text=True)
             for src, obj in zip(hb.sources(), objs)]
    for p in procs:
        out, err = p.communicate(timeout=900)
        assert p.returncode == 0, err[-3000:]
    lib = str(tmp_path / "libpir_asan.so")
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-fsanitize=address,undefined", "-o", lib, *objs])
    exe = str(tmp_path / "abi_driver")
    _run(["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          f"-I{os.path.join(ROOT, 'include')}", "-o", exe, os.path.join(HERE, "abi_driver.c"), lib,
          f"-Wl,-rpath,{tmp_path}"])
    r = _run([exe], env=ENV, timeout=300)
    assert "abi driver ok" in r.stdout
