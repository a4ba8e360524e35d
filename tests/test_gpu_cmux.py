"""GPU parity: one batched CMux step of blind rotation (Sec. II-B, Sec. IV-A),
acc + ExtProd(key, X^rot acc - acc), through the C ABI against the oracle."""
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
    "u32": (32, synth.primes_below(1 << 32, 1 << 17, 1)),
    "f64": (64, synth.c2_primes(2)),
    "i64": (64, synth.primes_below(1 << 61, 1 << 17, 1)),
}


def _log_base(moduli, levels):
    bits = max(int(q).bit_length() for q in moduli)
    return -(-(bits + 1) // levels)


def _cmux(plan, acc, rot, key, levels, lb, word_bits):
    dacc, dkey = to_device(acc, word_bits), to_device(key, word_bits)
    drot = torch.tensor(np.array(rot, dtype=np.int64).astype(np.uint32).view(np.int32), device="cuda")
    out = empty_device(acc.shape, word_bits)
    plan.cmux(out, dacc, drot, dkey, levels, lb)
    torch.cuda.synchronize()
    return to_host(out, word_bits).astype(np.uint64)


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn", [4, 10, 12, 13])
@pytest.mark.parametrize("comps,levels", [(2, 3), (1, 2)])
def test_cmux_matches_oracle(cls, logn, comps, levels):
    """Single-launch shapes (N <= 2^12) and the workspace path (N = 2^13)."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    L = len(moduli)
    lb = _log_base(moduli, levels)
    num_ct = 5
    acc = synth.uniform_poly(110 + logn, moduli, num_ct * comps, N).reshape(num_ct, comps, L, N)
    key = synth.uniform_poly(111 + logn, moduli, comps * levels * comps, N).reshape(
        comps * levels, comps, L, N)
    rot = [0, N - 1, N, 2 * N - 1, 3 * N + 5]  # the last is taken mod 2N
    plan = ntt.Plan(N, moduli, word_bits)
    got = _cmux(plan, acc, rot, key, levels, lb, word_bits)
    assert np.array_equal(got, oracle.cmux(acc, key, moduli, rot, levels, lb))


@pytest.mark.parametrize("bit", [0, 1])
def test_cmux_with_a_noise_free_key_selects_on_the_gpu(bit):
    """The gadget encryption of a bit without noise: the GPU CMux returns exactly
    X^(rot b) acc, 342 TFHE-shaped ciphertexts at N = 2^10."""
    q = synth.c3_prime()
    N, comps, levels, lb, num_ct = 1 << 10, 2, 3, 11, 342
    key = np.zeros((comps * levels, comps, 1, N), dtype=np.uint64)
    for c in range(comps):
        for j in range(levels):
            poly = np.zeros(N, dtype=np.uint64)
            poly[0] = (bit << (lb * j)) % q
            key[c * levels + j, c, 0] = oracle.forward(poly, [q])
    acc = synth.uniform_poly(120 + bit, [q], num_ct * comps, N).reshape(num_ct, comps, 1, N)
    rot = [(37 * g + 11) % (2 * N) for g in range(num_ct)]
    plan = ntt.Plan(N, [q], 32)
    got = _cmux(plan, acc, rot, key, levels, lb, 32)
    want = oracle.monomial_mul(acc[:8], [q], rot[:8]) if bit else acc[:8]
    assert np.array_equal(got[:8], want)
    assert np.array_equal(got, oracle.cmux(acc, key, [q], rot, levels, lb))


def test_cmux_rejects_bad_arguments():
    q = synth.c3_prime()
    N = 1 << 10
    plan = ntt.Plan(N, [q], 32)
    acc = to_device(synth.uniform_poly(130, [q], 4, N), 32).reshape(2, 2, 1, N)
    key = to_device(synth.uniform_poly(131, [q], 12, N), 32).reshape(6, 2, 1, N)
    rot = torch.zeros(2, dtype=torch.int32, device="cuda")
    lib = ntt.lib()
    out = empty_device((2, 2, 1, N), 32)
    # aliasing, digits too short for q, null rotation array
    assert lib.ntt_cmux(plan.handle, acc.data_ptr(), acc.data_ptr(), rot.data_ptr(), key.data_ptr(),
                        2, 2, 3, 11, None) == 1
    assert lib.ntt_cmux(plan.handle, out.data_ptr(), acc.data_ptr(), rot.data_ptr(), key.data_ptr(),
                        2, 2, 3, 10, None) == 1
    assert lib.ntt_cmux(plan.handle, out.data_ptr(), acc.data_ptr(), None, key.data_ptr(),
                        2, 2, 3, 11, None) == 1
