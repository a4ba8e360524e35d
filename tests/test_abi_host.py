"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-only helpers (admission, root choice) agree with
the oracle's independent number theory.  No kernel is launched here."""
import ctypes
import os
import re

import pytest

import oracle
import paper_2410_05934_amd as ntt
from paper_2410_05934_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(ntt_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ntt.lib()
    names = _declared_functions()
    assert "ntt_plan_create" in names and "ntt_forward" in names
    for name in names:
        assert hasattr(lib, name), name


def test_library_has_no_unresolved_internal_symbols():
    """Every internal (nttk) symbol the library uses is defined in it: a function
    declared in one translation unit and defined inline in another would only
    fail when first called."""
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    out = subprocess.run(["nm", "-D", "--undefined-only", ntt.library_path()],
                         capture_output=True, text=True, check=True).stdout
    assert "nttk" not in out, out


def test_version_and_empty_error():
    lib = ntt.lib()
    assert b"gfx950" in lib.ntt_version()


@pytest.mark.parametrize("N,q,wb,want", [
    (1024, 536881153, 32, 0),
    (3, 97, 64, 1),                   # N not a power of two
    (1 << 17, 786433, 64, 1),         # N too large
    (1, 97, 64, 1),                   # N too small
    (1024, 536881153, 16, 1),         # bad word width
    (1024, 4294967291, 32, 3),        # prime, but 2048 does not divide q-1
    (1024, 536881155, 32, 2),         # composite
    (16, (1 << 32) + 97, 32, 4),      # too wide for 32-bit words
    (16, (1 << 62) + 1, 64, 4),       # too wide for 64-bit words
    (1024, 4294957057, 32, 0),
    (1 << 16, 1125899903827969, 64, 0),
])
def test_check_modulus_codes(N, q, wb, want):
    assert ntt.check_modulus(N, q, wb) == want


def test_error_message_is_set():
    lib = ntt.lib()
    assert lib.ntt_check_modulus(3, 97, 64) == 1
    assert b"power of two" in lib.ntt_last_error()
    assert lib.ntt_check_modulus(1024, 536881153, 32) == 0
    assert lib.ntt_last_error() == b""


def test_find_root_matches_oracle_choice():
    primes = (synth.c2_primes(8) + synth.primes_below(1 << 32, 1 << 11, 4)
              + synth.primes_below(1 << 62, 1 << 17, 4) + [17, 97, 257, 7681, 12289, 998244353])
    for q in primes:
        N = 2
        while (q - 1) % (2 * N) == 0 and N <= (1 << 16):
            assert ntt.find_root(N, q) == oracle.psi(N, q), (N, q)
            N *= 2


def test_null_pointer_arguments_are_rejected():
    lib = ntt.lib()
    assert lib.ntt_plan_create(None, 1024, None, 1, 32, 0) == 1
    assert lib.ntt_forward(None, None, 1, None) == 1
    assert lib.ntt_inverse(None, None, 1, None) == 1
    assert lib.ntt_polymul(None, None, None, None, 1, None) == 1
    assert lib.ntt_pointwise_mul(None, None, None, None, 1, None) == 1
    assert lib.ntt_mac(None, None, None, None, 1, 1, 1, None) == 1
    assert lib.ntt_plan_destroy(None) == 1
    out = ctypes.c_uint64()
    assert lib.ntt_find_root(1024, 97, ctypes.byref(out)) == 3


def test_plan_create_rejects_bad_moduli_before_touching_the_device():
    h = ctypes.c_void_p()
    lib = ntt.lib()
    arr = (ctypes.c_uint64 * 2)(536881153, 536881155)
    assert lib.ntt_plan_create(ctypes.byref(h), 1024, arr, 2, 32, 0) == 2
    assert h.value is None
    arr1 = (ctypes.c_uint64 * 1)(536881153)
    assert lib.ntt_plan_create(ctypes.byref(h), 1024, arr1, 0, 32, 0) == 1
    assert lib.ntt_plan_create(ctypes.byref(h), 1024, arr1, 1, 32, ntt.flag_split(7)) == 1
    src = (ctypes.c_uint64 * 1)(536881153)
    assert lib.ntt_bconv_create(ctypes.byref(h), 1024, src, 1, src, 1, 64, 8) == 1
    assert b"flags" in lib.ntt_last_error()
    assert lib.ntt_bconv_create(ctypes.byref(h), 1024, src, 1, src, 1, 64, 3) == 1
    assert b"exclusive" in lib.ntt_last_error()
    assert lib.ntt_bconv_create(ctypes.byref(h), 1024, src, 0, src, 1, 64, 0) == 1
    both = ntt.FLAG_ROW_RADIX8 | ntt.FLAG_ROW_RADIX4
    assert lib.ntt_plan_create(ctypes.byref(h), 1024, arr1, 1, 32, both) == 1
    assert b"exclusive" in lib.ntt_last_error()


def test_basis_ext_create_rejects_bad_arguments_before_touching_the_device():
    """ModUp / ModDown basis: sizes, a modulus in both sets, a composite or a too
    wide modulus are rejected with their codes and no handle."""
    h = ctypes.c_void_p()
    lib = ntt.lib()
    q = (ctypes.c_uint64 * 2)(536881153, 1073707009)
    p_shared = (ctypes.c_uint64 * 1)(536881153)
    p_comp = (ctypes.c_uint64 * 1)(536881155)
    p_wide = (ctypes.c_uint64 * 1)(1 << 62)
    p_ok = (ctypes.c_uint64 * 2)(1073698817, 1073698817)
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 2, p_shared, 1, 64, 0) == 1
    assert b"distinct" in lib.ntt_last_error()
    assert h.value is None
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 0, p_comp, 1, 64, 0) == 1
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 2, p_comp, 65, 64, 0) == 1
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1000, q, 2, p_ok, 1, 64, 0) == 1
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 2, p_comp, 1, 64, 0) == 2
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 2, p_wide, 1, 64, 0) == 4
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 2, p_ok, 1, 64, 3) == 1
    assert b"exclusive" in lib.ntt_last_error()
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 2, p_ok, 2, 64, 0) == 1
    assert b"distinct" in lib.ntt_last_error()
    assert lib.ntt_basis_ext_create(ctypes.byref(h), 1024, q, 2, p_ok, 1, 48, 0) == 1
    assert h.value is None
    assert lib.ntt_mod_up(None, None, None, 1, None) == 1
    assert lib.ntt_mod_down(None, None, None, 1, None) == 1
    assert lib.ntt_basis_ext_destroy(None) == 1


def test_tuning_table_round_trips_on_the_host(tmp_path):
    """The tuning table loads, merges and saves every kind it records (split,
    ragged row length, row radices, column workgroup size) without a device, and
    a file without entries is refused."""
    import json
    entries = [{"kind": 0, "log_n": 16, "cls": 1, "bucket": 7, "value": 4, "us": 107.5},
               {"kind": 1, "log_n": 16, "cls": 0, "bucket": 0, "value": 12, "us": 900.0},
               {"kind": 2, "log_n": 16, "cls": 1, "bucket": 7, "value": 3, "us": 0.0},
               {"kind": 3, "log_n": 16, "cls": 1, "bucket": 7, "value": 4, "us": 0.0},
               {"kind": 4, "log_n": 16, "cls": 1, "bucket": 7, "value": 4, "us": 0.0},
               {"kind": 5, "log_n": 16, "cls": 1, "bucket": 7, "value": 128, "us": 107.1}]
    src = tmp_path / "in.json"
    src.write_text(json.dumps({"version": 1, "entries": entries}))
    out = tmp_path / "out.json"
    try:
        ntt.tune_clear()
        ntt.tune_load(str(src))
        ntt.tune_save(str(out))
        got = json.load(open(out))
        assert got["arch"] == "gfx950"
        key = lambda e: (e["kind"], e["log_n"], e["cls"], e["bucket"])
        assert sorted((key(e), e["value"]) for e in got["entries"]) == \
            sorted((key(e), e["value"]) for e in entries)
        bad = tmp_path / "bad.json"
        bad.write_text(json.dumps({"version": 1}))
        with pytest.raises(ntt.NTTError) as ei:
            ntt.tune_load(str(bad))
        assert ei.value.name == "NTT_EINVAL"
    finally:
        ntt.tune_clear()
