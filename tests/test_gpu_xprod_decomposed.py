"""GPU parity: the external product with the gadget decomposition fused in
(Sec. II-B, Sec. IV-A: Decompose, NTT, MAC against an RGSW key, INTT) through the
C ABI against the oracle, word for word."""
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
    "f64": (64, synth.c2_primes(2)),
    "i64": (64, synth.primes_below(1 << 61, 1 << 17, 2)),
}


def _log_base(moduli, levels):
    """Smallest base exponent with q <= 2^(levels * log_base - 1) for every q."""
    bits = max(int(q).bit_length() for q in moduli)
    return -(-(bits + 1) // levels)


def _run(plan, ct, key, levels, log_base, word_bits):
    num_ct, cols = ct.shape[0], key.shape[1]
    L, N = ct.shape[2], ct.shape[3]
    dct, dkey = to_device(ct, word_bits), to_device(key, word_bits)
    out = empty_device((num_ct, cols, L, N), word_bits)
    plan.external_product_decomposed(out, dct, dkey, levels, log_base)
    torch.cuda.synchronize()
    return to_host(out, word_bits).astype(np.uint64)


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn", [4, 10, 12, 13])
@pytest.mark.parametrize("num_ct,comps,levels,cols", [(5, 2, 3, 2), (3, 1, 2, 1), (2, 3, 2, 3),
                                                      (3, 1, 2, 3)])
def test_decomposed_external_product_matches_oracle(cls, logn, num_ct, comps, levels, cols):
    """Fused shapes (N <= 2^12, cols <= rows) and the workspace path (N = 2^13, or
    more columns than rows) give the oracle's words."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    lb = _log_base(moduli, levels)
    ct = synth.uniform_poly(60 + logn, moduli, num_ct * comps, N).reshape(num_ct, comps, len(moduli), N)
    key = synth.uniform_poly(61 + logn, moduli, comps * levels * cols, N).reshape(
        comps * levels, cols, len(moduli), N)
    plan = ntt.Plan(N, moduli, word_bits)
    got = _run(plan, ct, key, levels, lb, word_bits)
    want = oracle.external_product_decomposed(ct, key, moduli, levels, lb, cols)
    assert np.array_equal(got, want)


def test_decomposed_external_product_tfhe_shape():
    """342 ciphertexts of (k+1) = 2 components at N = 2^10 over the ~32-bit prime,
    3 levels of base 2^11 (the TFHE-shaped configuration with the digits computed
    on the GPU), against the oracle and against ntt_external_product on the
    oracle's digits."""
    q = synth.c3_prime()
    N, num_ct, comps, levels, lb, cols = 1 << 10, 342, 2, 3, 11, 2
    ct = synth.uniform_poly(62, [q], num_ct * comps, N).reshape(num_ct, comps, 1, N)
    key = synth.uniform_poly(63, [q], comps * levels * cols, N).reshape(comps * levels, cols, 1, N)
    plan = ntt.Plan(N, [q], 32)
    got = _run(plan, ct, key, levels, lb, 32)
    assert np.array_equal(got, oracle.external_product_decomposed(ct, key, [q], levels, lb, cols))
    ops = oracle.decompose(ct, [q], levels, lb).reshape(num_ct * comps * levels, 1, N)
    out = empty_device((num_ct * cols, 1, N), 32)
    plan.external_product(out, to_device(ops, 32), to_device(key.reshape(-1, 1, N), 32),
                          comps * levels, cols)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out, 32).astype(np.uint64).reshape(got.shape), got)


def test_decomposed_external_product_rejects_bad_arguments():
    q = synth.c3_prime()
    N = 1 << 10
    plan = ntt.Plan(N, [q], 32)
    ct = to_device(synth.uniform_poly(64, [q], 4, N), 32).reshape(2, 2, 1, N)
    key = to_device(synth.uniform_poly(65, [q], 12, N), 32).reshape(6, 2, 1, N)
    out = empty_device((2, 2, 1, N), 32)
    for levels, lb in [(3, 10), (1, 32), (3, 0), (2, 33), (3, 22)]:
        # 3 x 10 - 1 = 29 bits < 32; one level of 32 bits covers only 2^31; base 0 or
        # > 32; 3 x 22 = 66 digit bits > 64
        with pytest.raises(ntt.NTTError) as ei:
            plan.external_product_decomposed(out, ct, key[: 2 * levels] if levels < 3 else key,
                                             levels, lb)
        assert ei.value.name == "NTT_EINVAL", (levels, lb)
    lib = ntt.lib()
    assert lib.ntt_external_product_decomposed(plan.handle, ct.data_ptr(), ct.data_ptr(),
                                               key.data_ptr(), 2, 2, 3, 11, 2, None) == 1
