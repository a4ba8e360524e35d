"""GPU parity: RNS basis conversion (BConv, Sec. III) through the C ABI against
the oracle, word for word."""
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


def _bases(word_bits, L, M):
    if word_bits == 32:
        pool = synth.primes_below(1 << 32, 1 << 17, L + M)
    else:
        pool = synth.primes_below(1 << 50, 1 << 17, L) + synth.primes_below(1 << 61, 1 << 17, M)
    return pool[:L], pool[L:L + M]


def _run(conv, x, M, word_bits):
    out = empty_device((x.shape[0], M, x.shape[-1]), word_bits)
    conv(out, to_device(x, word_bits))
    torch.cuda.synchronize()
    return to_host(out, word_bits).astype(np.uint64)


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("L,M", [(1, 1), (3, 5), (8, 8), (9, 17), (20, 3), (64, 9)])
@pytest.mark.parametrize("logn", [1, 10])
def test_bconv_matches_oracle(word_bits, L, M, logn):
    N = 1 << logn
    src, dst = _bases(word_bits, L, M)
    x = synth.uniform_poly(80 + L + logn, src, 3, N)
    conv = ntt.BasisConversion(N, src, dst, word_bits)
    assert np.array_equal(_run(conv, x, M, word_bits), oracle.bconv(x, src, dst))


def test_bconv_ckks_shape_36_to_36():
    """36 limbs of the CKKS-shaped configuration to 36 other 50-bit primes at 2^16,
    two polynomials."""
    pool = synth.primes_below(1 << 50, 1 << 17, 72)
    src, dst = pool[:36], pool[36:]
    N = 1 << 16
    x = synth.uniform_poly(85, src, 2, N)
    conv = ntt.BasisConversion(N, src, dst, 64)
    got = _run(conv, x, 36, 64)
    want = oracle.bconv(x[:, :, :4096], src, dst)  # the map is per coefficient
    assert np.array_equal(got[:, :, :4096], want)
    tail = oracle.bconv(x[:, :, -4096:], src, dst)
    assert np.array_equal(got[:, :, -4096:], tail)


def test_bconv_rejects_bad_arguments():
    src, dst = _bases(64, 3, 2)
    for bad_src in ([], list(range(3, 3 + 65)), [src[0], src[0]], [src[0], 15]):
        with pytest.raises(ntt.NTTError):
            ntt.BasisConversion(1024, bad_src, dst, 64)
    with pytest.raises(ntt.NTTError) as ei:
        ntt.BasisConversion(1024, src, [1 << 62], 64)
    assert ei.value.name == "NTT_ERANGE"
    with pytest.raises(ntt.NTTError) as ei:
        ntt.BasisConversion(1000, src, dst, 64)
    assert ei.value.name == "NTT_EINVAL"
    conv = ntt.BasisConversion(1024, src, dst, 64)
    buf = to_device(synth.uniform_poly(86, src, 2, 1024), 64)
    alias = buf.view(-1)[: 2 * 2 * 1024].view(2, 2, 1024)  # the first words of buf
    with pytest.raises(ntt.NTTError) as ei:
        conv(alias, buf)
    assert ei.value.name == "NTT_EINVAL"


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("L,M", [(1, 1), (2, 4), (9, 17), (36, 36), (64, 5)])
def test_bconv_matrix_core_form_equals_vector_form(word_bits, L, M):
    """With every modulus below 2^50 and N >= 32 the conversion runs on the int8
    matrix cores; it gives the vector form's words and the oracle's."""
    if word_bits == 32:
        pool = synth.primes_below(1 << 32, 1 << 17, L + M)
    else:
        pool = synth.primes_below(1 << 50, 1 << 17, L + M)
    src, dst = pool[:L], pool[L:]
    N = 1 << 12
    x = synth.uniform_poly(90 + L, src, 3, N)
    mf = _run(ntt.BasisConversion(N, src, dst, word_bits, mfma=True), x, M, word_bits)
    vec = _run(ntt.BasisConversion(N, src, dst, word_bits, mfma=False), x, M, word_bits)
    assert np.array_equal(mf, vec)
    assert np.array_equal(mf[:, :, :512], oracle.bconv(x[:, :, :512], src, dst))


def test_bconv_matrix_core_form_at_n_32_and_edge_values():
    """N = 32 (one tile per polynomial) and residues at 0 and q - 1."""
    pool = synth.primes_below(1 << 50, 1 << 17, 11)
    src, dst = pool[:5], pool[5:]
    N = 32
    x = synth.uniform_poly(95, src, 4, N)
    x[0] = 0
    for i, q in enumerate(src):
        x[1, i] = q - 1
    got = _run(ntt.BasisConversion(N, src, dst, 64, mfma=True), x, 6, 64)
    assert np.array_equal(got, oracle.bconv(x, src, dst))


@pytest.mark.parametrize("L,M,logn,batch", [(1, 1, 5, 3), (3, 4, 6, 2), (9, 17, 12, 3), (36, 36, 10, 5),
                                            (37, 48, 7, 2), (64, 47, 8, 2), (64, 49, 7, 1), (33, 12, 9, 3),
                                            (2, 16, 16, 1)])
def test_bconv_weights_stationary_form_equals_streaming_form(L, M, logn, batch):
    """The matrix-core form that keeps constant operands in registers (up to 48
    targets: one wave per 4 targets beside four digit-forming waves, workgroups
    walking 32-coefficient tiles) gives the words of the form that reloads them
    per tile, and the oracle's."""
    pool = synth.primes_below(1 << 50, 1 << 17, L + M)
    src, dst = pool[:L], pool[L:]
    N = 1 << logn
    x = synth.uniform_poly(97 + L + M, src, batch, N)
    x[0, :, :2] = 0
    for i, q in enumerate(src):
        x[-1, i, -2:] = q - 1
    ws = _run(ntt.BasisConversion(N, src, dst, 64, mfma=True), x, M, 64)
    st = _run(ntt.BasisConversion(N, src, dst, 64, mfma=True, stationary=False), x, M, 64)
    assert np.array_equal(ws, st)
    k = min(N, 256)
    assert np.array_equal(ws[:, :, :k], oracle.bconv(x[:, :, :k], src, dst))
    assert np.array_equal(ws[:, :, -k:], oracle.bconv(x[:, :, -k:], src, dst))
