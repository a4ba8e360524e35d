"""GPU parity: forward transforms of two operands with their elementwise product
from one row pass (Eq. (1): the transform and the pointwise product), against the
oracle and the separate calls."""
import numpy as np
import pytest

import oracle
from paper_2410_05934_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2410_05934_amd as ntt  # noqa: E402
from paper_2410_05934_amd.tensors import empty_device, to_device, to_host  # noqa: E402

CLASSES = {
    "u32": (32, synth.primes_below(1 << 32, 1 << 17, 2)),
    "f64": (64, synth.c2_primes(3)),
    "i64": (64, synth.primes_below(1 << 61, 1 << 17, 2)),
    "mixed64": (64, [synth.c2_primes(1)[0], synth.primes_below(1 << 61, 1 << 17, 1)[0]]),
}


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn", [1, 3, 4, 10, 12, 13, 14, 16])
def test_forward_mul_matches_oracle(cls, logn):
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    batch = 3 if logn <= 13 else 2
    a = synth.uniform_poly(140 + logn, moduli, batch, N)
    b = synth.uniform_poly(141 + logn, moduli, batch, N)
    plan = ntt.Plan(N, moduli, word_bits)
    da, db = to_device(a, word_bits), to_device(b, word_bits)
    out = empty_device(a.shape, word_bits)
    plan.forward_mul(out, da, db)
    torch.cuda.synchronize()
    fa, fb = oracle.forward(a, moduli), oracle.forward(b, moduli)
    assert np.array_equal(to_host(da, word_bits).astype(np.uint64), fa)
    assert np.array_equal(to_host(db, word_bits).astype(np.uint64), fb)
    assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.pointwise_mul(fa, fb, moduli))


@pytest.mark.parametrize("n1", [0, 2, 4, 5])
def test_forward_mul_every_split_equals_separate_calls(n1):
    """Forced splits (row parts 2^16 / 2^14 take the separate-call path) on the
    CKKS-shaped prime set, 2 pairs x 4 limbs x 2^12 .. 2^16."""
    mods = synth.c2_primes(4)
    N = 1 << 16 if n1 else 1 << 12
    a = synth.uniform_poly(150 + n1, mods, 2, N)
    b = synth.uniform_poly(151 + n1, mods, 2, N)
    plan = ntt.Plan(N, mods, 64, flags=ntt.flag_split(n1))
    da, db = to_device(a, 64), to_device(b, 64)
    out = empty_device(a.shape, 64)
    plan.forward_mul(out, da, db)
    ea, eb = to_device(a, 64), to_device(b, 64)
    ref = empty_device(a.shape, 64)
    plan.forward(ea)
    plan.forward(eb)
    plan.pointwise_mul(ref, ea, eb)
    torch.cuda.synchronize()
    assert torch.equal(da, ea) and torch.equal(db, eb) and torch.equal(out, ref)


def test_forward_mul_rejects_aliases():
    q = synth.c3_prime()
    plan = ntt.Plan(1 << 10, [q], 32)
    a = to_device(synth.uniform_poly(160, [q], 2, 1 << 10), 32)
    b = to_device(synth.uniform_poly(161, [q], 2, 1 << 10), 32)
    for out, x, y in ((a, a, b), (b, a, b), (empty_device(a.shape, 32), a, a)):
        with pytest.raises(ntt.NTTError) as ei:
            plan.forward_mul(out, x, y)
        assert ei.value.name == "NTT_EINVAL"
