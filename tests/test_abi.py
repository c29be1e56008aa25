"""C-ABI checks that need no GPU: every function the public headers declare
is exported by libpir.so and bound by the Python layer, and argument
validation fails with PIR_EINVAL (and a message) before any device work."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

import paper_2604_04696_amd as pir
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("pir.h", "pir_synth.h", "pir_peak.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(pir_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def exported_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", pir.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pir.LIB_PATH):
        pytest.fail("libpir.so is not built (run __graft_entry__.build())")
    return pir.lib()


def test_every_declared_function_is_exported(L):
    decl = declared_functions()
    assert decl, "no declarations parsed"
    missing = decl - exported_symbols()
    assert not missing, f"declared but not exported: {sorted(missing)}"


def test_binding_covers_exactly_the_headers(L):
    assert set(pir.SIGNATURES) == declared_functions()
    for name in pir.SIGNATURES:
        assert hasattr(L, name)


def _create(params, layouts=pir.PIR_LAYOUT_VALU):
    h = ctypes.c_void_p()
    st = pir.lib().pir_db_create(ctypes.byref(params), layouts, ctypes.byref(h))
    return st, pir.pir_last_error()


@pytest.mark.parametrize("n,primes,d0,d1,frag", [
    (1000, [1073707009], 16, 16, "power of two"),
    (4, [1073707009], 16, 16, "power of two"),
    (32768, [1073707009], 16, 16, "power of two"),
    (1024, [1073707009 - 2048], 16, 16, "not prime"),          # 1 mod 2048 but composite
    (1024, [1073707011], 16, 16, "not 1 mod"),
    (1024, [], 16, 16, "nprimes"),
    (1024, [1073707009] * 5, 16, 16, "nprimes"),
    (1024, [1073707009], 0, 16, "d0"),
    (1024, [1073707009], 16, 0, "d1"),
    (1024, [1073707009], 16, 70000, "d1"),
])
def test_create_rejects_bad_params(L, n, primes, d0, d1, frag):
    p = pir.pir_params()
    p.n, p.nprimes, p.d0, p.d1 = n, len(primes), d0, d1
    for i, q in enumerate(primes[:4]):
        p.q[i] = q
    st, msg = _create(p)
    assert st == pir.PIR_EINVAL, msg
    assert frag in msg


def test_wide_prime_passes_validation_on_both_layouts():
    # a 32-bit prime (products up to 2^64) is taken by both layouts: creation
    # gets past parameter checks (to the device lookup, which fails without a GPU)
    p = pir.pir_params()
    p.n, p.nprimes, p.d0, p.d1 = 4096, 1, 16, 16
    p.q[0] = 4294828033
    for layouts in (pir.PIR_LAYOUT_MFMA, pir.PIR_LAYOUT_VALU | pir.PIR_LAYOUT_MFMA):
        h = ctypes.c_void_p()
        st = pir.lib().pir_db_create(ctypes.byref(p), layouts, ctypes.byref(h))
        assert st in (pir.PIR_OK, pir.PIR_EDEVICE), pir.pir_last_error()
        if st == pir.PIR_OK:
            pir.lib().pir_db_free(h)


def test_composite_fixture_is_composite():
    # the composite used above really is composite and 1 mod 2048
    x = 1073707009 - 2048
    assert x % 2048 == 1 and any(x % d == 0 for d in range(2, 40000))


def test_create_rejects_bad_layouts(L):
    p = pir.make_params(1024, [1073707009], 16, 16)
    assert _create(p, 0)[0] == pir.PIR_EINVAL
    assert _create(p, 4)[0] == pir.PIR_EINVAL


def test_null_arguments(L):
    assert L.pir_rowsel(None, None, 1, None, 0, None) == pir.PIR_EINVAL
    assert "NULL" in pir.pir_last_error()
    assert L.pir_db_load_ntt(None, None, 0, 1, 0, None) == pir.PIR_EINVAL
    assert L.pir_db_create(None, 1, None) == pir.PIR_EINVAL
    L.pir_db_free(None)   # no-op
    tiles = (ctypes.c_uint32 * 3)()
    assert L.pir_rowsel_grouped_tiles(None, 0, None) == pir.PIR_EINVAL
    assert L.pir_rowsel_grouped_tiles(None, 1, tiles) == pir.PIR_EINVAL
    assert "NULL" in pir.pir_last_error()


def test_rowsel_coeff_rejects_null_db(L):
    assert L.pir_rowsel_coeff(None, None, 1, None, 0, None) == pir.PIR_EINVAL
    assert "db is NULL" in pir.pir_last_error()


def test_kernel_timing_without_a_device(L):
    assert L.pir_kernel_time_read(None, None) == pir.PIR_EINVAL
    assert L.pir_kernel_timing(0) == pir.PIR_OK
    n, ms = ctypes.c_uint32(7), ctypes.c_double(1.0)
    assert L.pir_kernel_time_read(ctypes.byref(n), ctypes.byref(ms)) == pir.PIR_OK
    assert (n.value, ms.value) == (0, 0.0)


def test_ntt_helper_rejects_bad_modulus(L):
    assert L.pir_ntt_forward(None, None, 1, 1024, 1073707011, None) == pir.PIR_EINVAL
    assert L.pir_ntt_inverse(None, None, 1, 1000, 1073707009, None) == pir.PIR_EINVAL
    # count 0 with valid parameters is a no-op
    assert L.pir_ntt_forward(None, None, 0, 1024, 1073707009, None) == pir.PIR_OK


def test_synth_rejects_bad_shapes(L):
    qa = (ctypes.c_uint32 * 1)(1073707009)
    assert L.pir_synth_query(None, 0, 0, 1, 4, 0, 8, qa, None) == pir.PIR_EINVAL
    assert L.pir_synth_query(None, 0, 0, 0, 4, 1, 8, qa, None) == pir.PIR_OK   # empty
    assert L.pir_synth_db_coeffs(None, 0, 0, 1, 4, 1, 8, None) == pir.PIR_EINVAL


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pir, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pir, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        pir.lib()


@pytest.mark.parametrize("n,primes,log2z,ell,status,frag", [
    (4096, synth.PRIMES_Q108, 22, 4, "PIR_EINVAL", "must exceed Q"),
    (4096, synth.PRIMES_Q108, 30, 4, "PIR_EINVAL", "below every prime"),
    (4096, synth.PRIMES_Q108, 22, 9, "PIR_EINVAL", "ell must be"),
    (4096, synth.PRIMES_Q108, 0, 5, "PIR_EINVAL", "log2z must be"),
    (16384, (1073643521, 1073479681), 22, 3, "PIR_EUNSUPPORTED", "at most 16384"),
    (4096, synth.PRIMES_Q108, 22, 5, "PIR_EINVAL", "must not be NULL"),
])
def test_coltor_stage_validation(n, primes, log2z, ell, status, frag):
    # all checks run on the host before any device work
    ring = pir.make_params(n, primes, 1, 1)
    st = pir.lib().pir_coltor_stage(ctypes.byref(ring), None, 1, 2, None, log2z, ell, None, None)
    assert st == getattr(pir, status), pir.pir_last_error()
    assert frag in pir.pir_last_error()
    # B = 0 is a no-op once the parameters are valid
    if status == "PIR_EINVAL" and frag == "must not be NULL":
        assert pir.lib().pir_coltor_stage(ctypes.byref(ring), None, 0, 2, None, log2z, ell, None, None) == pir.PIR_OK


def test_library_load_brings_torch_first():
    # libpir.so must bind to torch's HIP runtime: loading the library imports
    # torch before it (a fresh process, nothing imported beforehand)
    code = ("import sys, paper_2604_04696_amd as p\n"
            "assert 'torch' not in sys.modules\n"
            "p.lib()\n"
            "assert 'torch' in sys.modules\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]


def test_peak_argument_checks(L):
    d = ctypes.c_double()
    assert L.pir_peak_mfma_i8(1, 0, None, ctypes.byref(d), None) == pir.PIR_EINVAL
    assert L.pir_peak_mfma_i8(0, 0, ctypes.byref(d), ctypes.byref(d), None) == pir.PIR_EINVAL
    assert "iters" in pir.pir_last_error()
    assert L.pir_peak_valu_mad64(1 << 25, ctypes.byref(d), ctypes.byref(d), None) == pir.PIR_EINVAL
    assert L.pir_peak_hbm_read(None, 16, ctypes.byref(d), None) == pir.PIR_EINVAL
    assert L.pir_peak_hbm_read(ctypes.c_void_p(4096), 10, ctypes.byref(d), None) == pir.PIR_EINVAL
    assert "multiple of 16" in pir.pir_last_error()

