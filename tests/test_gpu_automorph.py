"""GPU parity: the automorphism sigma_k of Z_q[x]/(x^N+1) (a(x) -> a(x^k), Sec. III
and Sec. IV-B) through the C ABI against the oracle, word for word, in the
coefficient domain and in the forward transform's slot order."""
import random

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

Q32 = synth.primes_below(1 << 32, 1 << 17, 2)
Q50 = synth.c2_primes(3)
Q60 = synth.primes_below(1 << 61, 1 << 17, 2)
CLASSES = {
    "u32": (32, Q32),
    "f64": (64, Q50),
    "i64": (64, Q60),
    "mixed64": (64, [Q50[0], Q60[0], synth.primes_below(1 << 30, 1 << 17, 1)[0]]),
}


def _ks(N, seed):
    """k = 1, conjugation, small k (scattered by the library in the coefficient
    domain) and their inverses mod 2N (gathered), and a random odd k."""
    rng = random.Random(seed)
    two_n = 2 * N
    ks = {1, two_n - 1, 3 % two_n, 5 % two_n, pow(3, -1, two_n), pow(5, -1, two_n),
          rng.randrange(N) * 2 + 1}
    return sorted(k for k in ks if k % 2 == 1)


def _apply(plan, x, word_bits, k, transformed):
    d = to_device(x, word_bits)
    out = empty_device(x.shape, word_bits)
    plan.automorph(out, d, k, transformed=transformed)
    torch.cuda.synchronize()
    return to_host(out, word_bits).astype(np.uint64)


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn", [1, 2, 5, 10, 12, 16])
def test_automorph_matches_oracle(cls, logn):
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    batch = 3 if logn <= 12 else 2
    a = synth.uniform_poly(40 + logn, moduli, batch, N)
    fa = oracle.forward(a, moduli)
    plan = ntt.Plan(N, moduli, word_bits)
    for k in _ks(N, logn):
        assert np.array_equal(_apply(plan, a, word_bits, k, False),
                              oracle.automorph(a, moduli, k)), k
        assert np.array_equal(_apply(plan, fa, word_bits, k, True),
                              oracle.automorph_transformed(fa, moduli, k)), k


def test_automorph_full_ckks_shape():
    """4 x 36 x 2^16 words (the CKKS-shaped configuration), k = 5 and k = 2N - 1."""
    mods = synth.c2_primes(36)
    N = 1 << 16
    a = synth.uniform_poly(41, mods, 4, N)
    plan = ntt.Plan(N, mods, 64)
    fa = oracle.forward(a, mods)
    for k in (5, pow(5, -1, 2 * N), 2 * N - 1):
        assert np.array_equal(_apply(plan, a, 64, k, False), oracle.automorph(a, mods, k))
        assert np.array_equal(_apply(plan, fa, 64, k, True), oracle.automorph_transformed(fa, mods, k))


def test_automorph_commutes_with_the_library_transform():
    """forward(sigma_k(a)) == sigma_k applied to forward(a) in slot order, all on the GPU."""
    mods = synth.c2_primes(2)
    N = 1 << 13
    a = synth.uniform_poly(42, mods, 3, N)
    plan = ntt.Plan(N, mods, 64)
    da = to_device(a, 64)
    s1 = empty_device(a.shape, 64)
    plan.automorph(s1, da, 25)
    plan.forward(s1)
    plan.forward(da)
    s2 = empty_device(a.shape, 64)
    plan.automorph(s2, da, 25, transformed=True)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2)


def test_automorph_rejects_bad_arguments_before_any_launch():
    N = 1 << 10
    q = synth.c3_prime()
    plan = ntt.Plan(N, [q], 32)
    a = to_device(synth.uniform_poly(43, [q], 2, N), 32)
    out = empty_device(a.shape, 32)
    for k in (0, 2, 2 * N, 2 * N + 1):
        with pytest.raises(ntt.NTTError) as ei:
            plan.automorph(out, a, k)
        assert ei.value.name == "NTT_EINVAL"
    with pytest.raises(ntt.NTTError) as ei:
        plan.automorph(a, a, 5)
    assert ei.value.name == "NTT_EINVAL"
    a3 = to_device(synth.uniform_poly(44, [q], 3, N), 32)
    with pytest.raises(ntt.NTTError) as ei:  # overlapping by one polynomial
        plan.automorph(a3[1:], a3[:2], 5)
    assert ei.value.name == "NTT_EINVAL"
    plan.automorph(a3[2:], a3[:1], 5)  # adjacent, not overlapping
    torch.cuda.synchronize()
    lib = ntt.lib()
    assert lib.ntt_automorph(plan.handle, out.data_ptr(), a.data_ptr(), 2, 5, 2, None) == 1
    assert b"flags" in lib.ntt_last_error()
