"""GPU parity: ModUp and ModDown of CKKS key switching (Sec. III: BConv with
ModMul and ModAdd around it) through the C ABI against the oracle, word for word."""
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


def _bases(word_bits, L, K, wide=False):
    """L moduli of Q and K of P: 32-bit words take primes below 2^32; 64-bit words
    below 2^50 (the fp64 forms), or P near 2^61 with wide=True (64-bit Shoup)."""
    if word_bits == 32:
        pool = synth.primes_below(1 << 32, 1 << 17, L + K)
        return pool[:L], pool[L:]
    if wide:
        return synth.primes_below(1 << 50, 1 << 17, L), synth.primes_below(1 << 61, 1 << 17, K)
    pool = synth.primes_below(1 << 50, 1 << 17, L + K)
    return pool[:L], pool[L:]


def _up(ext, x, wb):
    out = empty_device((x.shape[0], ext.L + ext.K, x.shape[-1]), wb)
    ext.mod_up(out, to_device(x, wb))
    torch.cuda.synchronize()
    return to_host(out, wb).astype(np.uint64)


def _down(ext, x, wb):
    out = empty_device((x.shape[0], ext.L, x.shape[-1]), wb)
    ext.mod_down(out, to_device(x, wb))
    torch.cuda.synchronize()
    return to_host(out, wb).astype(np.uint64)


CASES = [(1, 1, False), (3, 5, False), (9, 17, False), (20, 3, False), (36, 36, False),
         (4, 3, True), (17, 16, True)]


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("L,K,wide", CASES)
@pytest.mark.parametrize("mfma", [None, False, True, "streaming"])
@pytest.mark.parametrize("logn", [1, 6, 11])
def test_mod_up_and_down_match_oracle(word_bits, L, K, wide, mfma, logn):
    if word_bits == 32 and wide:
        pytest.skip("wide P is a 64-bit case")
    if mfma and (wide or logn < 5):
        pytest.skip("the matrix-core form needs fp64-sized moduli and N >= 32")
    N = 1 << logn
    q, p = _bases(word_bits, L, K, wide)
    if mfma == "streaming":
        ext = ntt.BasisExtension(N, q, p, word_bits, mfma=True, stationary=False)
    else:
        ext = ntt.BasisExtension(N, q, p, word_bits, mfma=mfma)
    x = synth.uniform_poly(300 + L + K + logn, q, 3, N)
    assert np.array_equal(_up(ext, x, word_bits), oracle.mod_up(x, q, p))
    xw = synth.uniform_poly(400 + L + K + logn, q + p, 3, N)
    assert np.array_equal(_down(ext, xw, word_bits), oracle.mod_down(xw, q, p))


def test_mod_down_of_mod_up_times_p():
    """ModDown(P * ModUp-shaped input) through both calls: X = P Y over Q u P is
    exactly Y after ModDown (no fast-conversion error on multiples of P), and
    ModUp keeps the Q limbs word for word."""
    q, p = _bases(64, 12, 8)
    N = 1 << 12
    ext = ntt.BasisExtension(N, q, p, 64)
    y = synth.uniform_poly(77, q, 2, N)
    up = _up(ext, y, 64)
    assert np.array_equal(up[:, :12], y)
    P = 1
    for pk in p:
        P *= pk
    # P * Y over Q u P: residues P*y_i mod q_i on Q, 0 on P.
    xw = np.zeros((2, 20, N), dtype=np.uint64)
    for i, qi in enumerate(q):
        xw[:, i] = np.array([(P % qi) * int(v) % qi for v in y[:, i].ravel()],
                            dtype=np.uint64).reshape(2, N)
    assert np.array_equal(_down(ext, xw, 64), y)


def test_ckks_shape_36_plus_36_sampled():
    """Q = the 36 primes of the CKKS-shaped configuration, P = the next 36 primes
    = 1 mod 2^17 below them, N = 2^16, 4 polynomials; the map is per coefficient,
    so the oracle checks the first and last 2048 coefficients of each."""
    pool = synth.c2_primes(72)
    q, p = pool[:36], pool[36:]
    N = 1 << 16
    ext = ntt.BasisExtension(N, q, p, 64)
    x = synth.uniform_poly(501, q, 4, N)
    up = _up(ext, x, 64)
    for sl in (slice(0, 2048), slice(N - 2048, N)):
        assert np.array_equal(up[:, :, sl], oracle.mod_up(x[:, :, sl], q, p))
    xw = synth.uniform_poly(502, q + p, 4, N)
    down = _down(ext, xw, 64)
    for sl in (slice(0, 2048), slice(N - 2048, N)):
        assert np.array_equal(down[:, :, sl], oracle.mod_down(xw[:, :, sl], q, p))


def test_edge_residues():
    """Residues 0 and q - 1 on every limb, matrix-core and vector forms."""
    q, p = _bases(64, 16, 16)
    N = 64
    xw = synth.uniform_poly(503, q + p, 3, N)
    xw[0] = 0
    for i, m in enumerate(q + p):
        xw[1, i] = m - 1
    x = xw[:, :16].copy()
    for mfma in (False, True):
        ext = ntt.BasisExtension(N, q, p, 64, mfma=mfma)
        assert np.array_equal(_up(ext, x, 64), oracle.mod_up(x, q, p))
        assert np.array_equal(_down(ext, xw, 64), oracle.mod_down(xw, q, p))


def test_rejects_overlap_and_bad_sizes():
    q, p = _bases(64, 3, 2)
    N = 1024
    ext = ntt.BasisExtension(N, q, p, 64)
    wide = to_device(synth.uniform_poly(504, q + p, 2, N), 64)
    narrow_alias = wide.view(-1)[: 2 * 3 * N].view(2, 3, N)
    with pytest.raises(ntt.NTTError) as ei:
        ext.mod_down(narrow_alias, wide)
    assert ei.value.name == "NTT_EINVAL"
    with pytest.raises(ntt.NTTError) as ei:
        ext.mod_up(wide, narrow_alias)
    assert ei.value.name == "NTT_EINVAL"
    with pytest.raises(ntt.NTTError) as ei:
        ntt.BasisExtension(N, q, [q[0]], 64)
    assert ei.value.name == "NTT_EINVAL"
