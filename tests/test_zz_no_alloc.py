"""GPU: the polymul entry point that allocates nothing (ntt_polymul_noalloc)
against ntt_polymul, word for word, through the C ABI: two calls in a row, the
second smaller, on shapes that need the two-pass workspace and on single-pass
shapes; sizes beyond the fixed scratch and validating plans are refused."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2410_05934_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2410_05934_amd as ntt  # noqa: E402
from paper_2410_05934_amd.tensors import to_device, to_host  # noqa: E402

SCRATCH_BYTES = 64 << 20


def _garbage(shape, wb):
    dt = torch.int64 if wb == 64 else torch.int32
    return torch.full(tuple(shape), -1, dtype=dt, device="cuda")


def _both(plan, a, b, wb):
    """(words of ntt_polymul_noalloc, words of ntt_polymul), both through the C ABI."""
    lib = ntt.lib()
    da, db = to_device(a, wb), to_device(b, wb)
    out_na, out_ref = _garbage(a.shape, wb), _garbage(a.shape, wb)
    batch = a.shape[0]
    assert lib.ntt_polymul_noalloc(plan._h, out_na.data_ptr(), da.data_ptr(), db.data_ptr(),
                                   batch, None) == 0, lib.ntt_last_error()
    assert lib.ntt_polymul(plan._h, out_ref.data_ptr(), da.data_ptr(), db.data_ptr(),
                           batch, None) == 0, lib.ntt_last_error()
    torch.cuda.synchronize()
    return to_host(out_na, wb), to_host(out_ref, wb)


def test_two_calls_two_pass_then_smaller():
    """CKKS shape at the scratch's size (2 x 36 limbs x 2^16 words of 64 bits,
    37.7 MB of workspace), then a smaller two-pass product on another plan."""
    moduli = synth.c2_primes(36)
    plan = ntt.Plan(1 << 16, moduli, 64)
    a = synth.uniform_poly(601, moduli, 2, 1 << 16)
    b = synth.uniform_poly(602, moduli, 2, 1 << 16)
    got, ref = _both(plan, a, b, 64)
    assert np.array_equal(got, ref)
    sl = np.s_[:, :2, :]
    assert np.array_equal(got[sl].astype(np.uint64), oracle.polymul(a[sl], b[sl], moduli[:2]))
    small = synth.c2_primes(5)
    plan2 = ntt.Plan(1 << 13, small, 64)
    a2 = synth.uniform_poly(603, small, 1, 1 << 13)
    b2 = synth.uniform_poly(604, small, 1, 1 << 13)
    got2, ref2 = _both(plan2, a2, b2, 64)
    assert np.array_equal(got2, ref2)
    assert np.array_equal(got2.astype(np.uint64), oracle.polymul(a2, b2, small))


@pytest.mark.parametrize("n1", [1, 2, 5])
def test_two_calls_every_split_u32(n1):
    """32-bit words, forced two-pass splits (the workspace holds b's column pass),
    batch 6 then batch 2."""
    q = synth.primes_below(1 << 32, 1 << 17, 1)
    plan = ntt.Plan(1 << 12, q, 32, ntt.flag_split(n1))
    for seed, batch in ((611, 6), (612, 2)):
        a = synth.uniform_poly(seed, q, batch, 1 << 12)
        b = synth.uniform_poly(seed + 50, q, batch, 1 << 12)
        got, ref = _both(plan, a, b, 32)
        assert np.array_equal(got, ref)
        assert np.array_equal(got.astype(np.uint64), oracle.polymul(a, b, q))


def test_single_pass_takes_any_batch():
    """N = 2^10 products run on-chip and need no workspace: 4096 pairs, then 3."""
    q = [synth.c3_prime()]
    plan = ntt.Plan(1 << 10, q, 32)
    for seed, batch in ((621, 4096), (622, 3)):
        a = synth.uniform_poly(seed, q, batch, 1 << 10)
        b = synth.uniform_poly(seed + 50, q, batch, 1 << 10)
        got, ref = _both(plan, a, b, 32)
        assert np.array_equal(got, ref)
    assert np.array_equal(got.astype(np.uint64), oracle.polymul(a, b, q))


def test_refuses_beyond_scratch_and_validating_plans():
    lib = ntt.lib()
    moduli = synth.c2_primes(36)
    plan = ntt.Plan(1 << 16, moduli, 64)
    batch = SCRATCH_BYTES // (36 * (1 << 16) * 8) + 1  # 3 pairs: 56.6 MB fits, 4 do not
    assert batch == 4
    buf = torch.zeros((batch, 36, 1 << 16), dtype=torch.int64, device="cuda")
    out = torch.empty_like(buf)
    assert lib.ntt_polymul_noalloc(plan._h, out.data_ptr(), buf.data_ptr(), buf.data_ptr(),
                                   batch, None) == 1
    assert b"scratch" in lib.ntt_last_error()
    vplan = ntt.Plan(1 << 12, synth.primes_below(1 << 32, 1 << 17, 1), 32, ntt.FLAG_VALIDATE)
    x = torch.zeros((1, 1, 1 << 12), dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    assert lib.ntt_polymul_noalloc(vplan._h, y.data_ptr(), x.data_ptr(), x.data_ptr(), 1, None) == 1
    assert b"VALIDATE" in lib.ntt_last_error()
    assert lib.ntt_polymul_noalloc(plan._h, out.data_ptr(), out.data_ptr(), buf.data_ptr(), 1, None) == 1
    torch.cuda.synchronize()
