"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Sizes span several tiles and ragged tails (batch * limbs not a multiple of the
workgroup's chunk count); full-size cases use the configurations' own shapes.
Chameleon (arXiv 2410.05934), Sec. II-D / Eq. (1).
"""
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

# Moduli for each arithmetic class, all = 1 mod 2^17 so every N <= 2^16 is admissible.
Q32 = synth.primes_below(1 << 32, 1 << 17, 2)              # fp64 class, 32-bit words
Q50 = synth.c2_primes(3)                                   # fp64 class, 64-bit words
Q60 = synth.primes_below(1 << 61, 1 << 17, 2)              # integer Shoup class
Q30 = synth.primes_below(1 << 30, 1 << 17, 2)              # small q in 64-bit words

CLASSES = {
    "u32": (32, Q32),
    "f64": (64, Q50),
    "i64": (64, Q60),
    "small64": (64, Q30),
    "mixed64": (64, [Q50[0], Q60[0], Q30[0]]),
}


def _data(seed, moduli, batch, N, word_bits):
    return synth.uniform_poly(seed, moduli, batch, N, np.uint64)


def _run_fwd(plan, host, word_bits):
    d = to_device(host, word_bits)
    plan.forward(d)
    torch.cuda.synchronize()
    return to_host(d, word_bits).astype(np.uint64)


def _run_inv(plan, host, word_bits):
    d = to_device(host, word_bits)
    plan.inverse(d)
    torch.cuda.synchronize()
    return to_host(d, word_bits).astype(np.uint64)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_c1_single_forward_inverse(seed):
    """N=2^10, one 30-bit prime chosen from the seed, one u32 polynomial."""
    N = 1 << 10
    q = synth.c1_prime(seed, N)
    a = _data(seed, [q], 1, N, 32)
    plan = ntt.Plan(N, [q], 32)
    f = _run_fwd(plan, a, 32)
    assert np.array_equal(f, oracle.forward(a, [q]))
    assert np.array_equal(_run_inv(plan, f, 32), a)
    assert np.array_equal(_run_inv(plan, a, 32), oracle.inverse(a, [q]))
    assert plan.root(0) == oracle.psi(N, q)


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn", list(range(1, 17)))
def test_all_sizes_forward_inverse(cls, logn):
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    batch = 3 if logn >= 12 else 5
    a = _data(100 + logn, moduli, batch, N, word_bits)
    plan = ntt.Plan(N, moduli, word_bits)
    assert np.array_equal(_run_fwd(plan, a, word_bits), oracle.forward(a, moduli))
    assert np.array_equal(_run_inv(plan, a, word_bits), oracle.inverse(a, moduli))


def _valid_splits(logn):
    out = []
    for n1 in range(0, logn + 1):
        if n1 == 0 and 4 <= logn <= 14:
            out.append(n1)
        elif n1 == logn and logn <= 5 and n1 != 0:
            out.append(n1)
        elif 1 <= n1 <= 5 and 4 <= logn - n1 <= 14:
            out.append(n1)
    return out


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
@pytest.mark.parametrize("logn", [5, 10, 13, 14, 15, 16])
def test_every_split_is_bit_identical(cls, logn):
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    a = _data(7 + logn, moduli, 2, N, word_bits)
    want_f = oracle.forward(a, moduli)
    want_i = oracle.inverse(a, moduli)
    for n1 in _valid_splits(logn):
        plan = ntt.Plan(N, moduli, word_bits, flags=ntt.flag_split(n1))
        assert plan.split == n1
        assert np.array_equal(_run_fwd(plan, a, word_bits), want_f), n1
        assert np.array_equal(_run_inv(plan, a, word_bits), want_i), n1


@pytest.mark.parametrize("logn", [4, 12, 16])
def test_force_int64_matches_fp64_class(logn):
    N = 1 << logn
    a = _data(5, Q50, 2, N, 64)
    p1 = ntt.Plan(N, Q50, 64)
    p2 = ntt.Plan(N, Q50, 64, flags=ntt.FLAG_FORCE_INT64)
    assert p1.limb_class(0) == 1 and p2.limb_class(0) == 2
    assert np.array_equal(_run_fwd(p1, a, 64), _run_fwd(p2, a, 64))
    assert np.array_equal(_run_inv(p1, a, 64), _run_inv(p2, a, 64))


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
@pytest.mark.parametrize("logn", [12, 16])
def test_edge_values(cls, logn):
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    rows = []
    for q in moduli:
        rows.append(np.stack([np.zeros(N, np.uint64), np.full(N, q - 1, np.uint64),
                              np.where(np.arange(N) % 2 == 0, q - 1, 0).astype(np.uint64)]))
    a = np.ascontiguousarray(np.stack(rows, axis=1))  # [3][L][N]
    plan = ntt.Plan(N, moduli, word_bits)
    f = _run_fwd(plan, a, word_bits)
    assert np.array_equal(f, oracle.forward(a, moduli))
    assert np.array_equal(_run_inv(plan, f, word_bits), a)


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn", [1, 3, 4, 10, 12, 13, 16])
def test_pointwise_and_polymul(cls, logn):
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    batch = 3
    a = _data(31, moduli, batch, N, word_bits)
    b = _data(32, moduli, batch, N, word_bits)
    plan = ntt.Plan(N, moduli, word_bits)
    da, db = to_device(a, word_bits), to_device(b, word_bits)
    out = empty_device(a.shape, word_bits)
    plan.pointwise_mul(out, da, db)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.pointwise_mul(a, b, moduli))
    plan.polymul(out, da, db)
    torch.cuda.synchronize()
    got = to_host(out, word_bits).astype(np.uint64)
    assert np.array_equal(got, oracle.polymul(a, b, moduli))
    # inputs untouched
    assert np.array_equal(to_host(da, word_bits).astype(np.uint64), a)
    assert np.array_equal(to_host(db, word_bits).astype(np.uint64), b)


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
@pytest.mark.parametrize("logn", [14, 15, 16])
def test_polymul_every_split(cls, logn):
    """Every admissible split, including those whose transform rows are 2^14
    words (single pass at 2^14, n1 = 1 at 2^15, n1 = 2 at 2^16): polymul and
    forward-and-multiply then take 2^13-word rows, with the same words."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    a = _data(41, moduli, 1, N, word_bits)
    b = _data(42, moduli, 1, N, word_bits)
    want = oracle.polymul(a, b, moduli)
    fa, fb = oracle.forward(a, moduli), oracle.forward(b, moduli)
    want_pw = oracle.pointwise_mul(fa, fb, moduli)
    da, db = to_device(a, word_bits), to_device(b, word_bits)
    for n1 in _valid_splits(logn):
        plan = ntt.Plan(N, moduli, word_bits, flags=ntt.flag_split(n1))
        out = empty_device(a.shape, word_bits)
        plan.polymul(out, da, db)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out, word_bits).astype(np.uint64), want), n1
        xa, xb = to_device(a, word_bits), to_device(b, word_bits)
        plan.forward_mul(out, xa, xb)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out, word_bits).astype(np.uint64), want_pw), n1
        assert np.array_equal(to_host(xa, word_bits).astype(np.uint64), fa), n1
        assert np.array_equal(to_host(xb, word_bits).astype(np.uint64), fb), n1


def test_c2_full_size():
    """4 polynomials x 36 limbs x 2^16 over the 36 largest primes = 1 mod 2^17 below 2^50."""
    N, L = 1 << 16, 36
    moduli = synth.c2_primes(L)
    a = synth.uniform_poly(0, moduli, 4, N)
    plan = ntt.Plan(N, moduli, 64)
    d = to_device(a, 64)
    plan.forward(d)
    torch.cuda.synchronize()
    f = to_host(d, 64)
    want_f = oracle.forward(a, moduli)
    assert np.array_equal(f, want_f)
    # pointwise on the two ciphertext pairs (0,1), (2,3)
    out = empty_device((2, L, N), 64)
    plan.pointwise_mul(out, d[0::2].contiguous(), d[1::2].contiguous())
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out, 64), oracle.pointwise_mul(want_f[0::2], want_f[1::2], moduli))
    plan.inverse(d)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(d, 64), a)
    # polymul on the pairs, checked on sampled coefficients against the definition
    da = to_device(np.ascontiguousarray(a[0::2]), 64)
    db = to_device(np.ascontiguousarray(a[1::2]), 64)
    plan.polymul(out, da, db)
    torch.cuda.synchronize()
    got = to_host(out, 64)
    want = oracle.polymul(a[0::2], a[1::2], moduli)
    assert np.array_equal(got, want)
    rng = np.random.default_rng(0)
    for _ in range(3):
        p, l, k = int(rng.integers(2)), int(rng.integers(L)), int(rng.integers(N))
        assert int(got[p, l, k]) == oracle.negacyclic_at(a[2 * p, l], a[2 * p + 1, l], moduli[l], k)


def test_c3_tfhe_batch_mac():
    """2048 x 2^10 u32 operands: forward, MAC against a 6x2 key table, inverse (684)."""
    N, P, rows, cols = 1 << 10, 2048, 6, 2
    q = synth.c3_prime()
    a = synth.uniform_poly(3, [q], P, N)
    key = synth.uniform_poly(4, [q], rows * cols, N).reshape(rows, cols, 1, N)
    plan = ntt.Plan(N, [q], 32)
    d = to_device(a, 32)
    plan.forward(d)
    k = to_device(key, 32)
    G = (P + rows - 1) // rows
    out = empty_device((G, cols, 1, N), 32)
    plan.mac(out, d, k, rows, cols)
    torch.cuda.synchronize()
    fa = oracle.forward(a, [q])
    assert np.array_equal(to_host(d, 32).astype(np.uint64), fa)
    want_mac = oracle.mac(fa, key, [q], rows, cols)
    assert np.array_equal(to_host(out, 32).astype(np.uint64), want_mac)
    o2 = out.view(G * cols, 1, N)
    plan.inverse(o2)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(o2, 32).astype(np.uint64),
                          oracle.inverse(want_mac.reshape(G * cols, 1, N), [q]))


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
@pytest.mark.parametrize("logn,groups,rows,cols,tail", [(10, 342, 6, 2, 2), (10, 5, 6, 2, 0),
                                                        (4, 3, 3, 3, 1), (12, 7, 4, 1, 3)])
def test_pointwise_mac_groups_and_tail(cls, logn, groups, rows, cols, tail):
    """ntt_pointwise_mac: groups of `rows` operands with a partial last group of
    batch_tail (0 = full); the TFHE shape is 342 groups with a tail of 2."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    P = (groups - 1) * rows + (tail or rows)
    fa = _data(91, moduli, P, N, word_bits)
    key = _data(92, moduli, rows * cols, N, word_bits)
    plan = ntt.Plan(N, moduli, word_bits)
    acc = empty_device((groups * cols, len(moduli), N), word_bits)
    plan.pointwise_mac(acc, to_device(fa, word_bits), to_device(key, word_bits), rows, cols, groups, tail)
    torch.cuda.synchronize()
    want = oracle.mac(fa, key.reshape(rows, cols, len(moduli), N), moduli, rows, cols)
    assert np.array_equal(to_host(acc, word_bits).astype(np.uint64).reshape(want.shape), want)


def test_pointwise_mac_rejects_bad_group_shapes():
    plan = ntt.Plan(16, Q50[:1], 64)
    a = empty_device((6, 1, 16), 64)
    lib = ntt.lib()
    EINVAL = 1
    assert lib.ntt_pointwise_mac(plan._h, a.data_ptr(), a.data_ptr(), a.data_ptr(), 3, 1, 0, 0, None) == EINVAL
    assert lib.ntt_pointwise_mac(plan._h, a.data_ptr(), a.data_ptr(), a.data_ptr(), 3, 1, 2, 4, None) == EINVAL
    assert lib.ntt_pointwise_mac(plan._h, a.data_ptr(), a.data_ptr(), a.data_ptr(), 0, 1, 2, 0, None) == EINVAL


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
def test_validate_flag_reports_out_of_range_words(cls):
    """NTT_FLAG_VALIDATE: canonical inputs give the oracle's words; a word equal
    to q (or all ones) makes the call return NTT_ERANGE before anything runs,
    leaving the data untouched, for transforms, polymul, pointwise and MAC."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << 12
    a = _data(95, moduli, 3, N, word_bits)
    b = _data(96, moduli, 3, N, word_bits)
    plan = ntt.Plan(N, moduli, word_bits, flags=ntt.FLAG_VALIDATE)
    assert np.array_equal(_run_fwd(plan, a, word_bits), oracle.forward(a, moduli))
    out = empty_device(a.shape, word_bits)
    plan.polymul(out, to_device(a, word_bits), to_device(b, word_bits))
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.polymul(a, b, moduli))
    bad = a.copy()
    bad[2, len(moduli) - 1, 1234] = moduli[-1]
    bad[2, len(moduli) - 1, 3000] = (1 << word_bits) - 1
    d = to_device(bad, word_bits)
    for call in (lambda: plan.forward(d), lambda: plan.inverse(d),
                 lambda: plan.polymul(out, to_device(b, word_bits), d),
                 lambda: plan.pointwise_mul(out, to_device(b, word_bits), d)):
        with pytest.raises(ntt.NTTError) as e:
            call()
        assert e.value.name == "NTT_ERANGE"
        assert "word 1234 of polynomial 2" in str(e.value)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(d, word_bits).astype(np.uint64), bad)
    key = to_device(_data(97, moduli, 2, N, word_bits), word_bits)
    acc = empty_device((2, len(moduli), N), word_bits)
    with pytest.raises(ntt.NTTError) as e:
        plan.mac(acc, d, key, 2, 1)
    assert e.value.name == "NTT_ERANGE"


def test_repeat_runs_are_identical():
    N = 1 << 16
    a = _data(9, Q50, 2, N, 64)
    plan = ntt.Plan(N, Q50, 64)
    r1 = _run_fwd(plan, a, 64)
    r2 = _run_fwd(plan, a, 64)
    assert np.array_equal(r1, r2)


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
@pytest.mark.parametrize("logn", [10, 12, 13, 15, 16])
def test_radix8_rows_are_bit_identical(cls, logn):
    """Row passes with 8 values per thread (radix-8 rounds) give the same words."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    a = _data(77 + logn, moduli, 3, N, word_bits)
    b = _data(78 + logn, moduli, 3, N, word_bits)
    plan = ntt.Plan(N, moduli, word_bits, flags=ntt.FLAG_ROW_RADIX8)
    assert np.array_equal(_run_fwd(plan, a, word_bits), oracle.forward(a, moduli))
    assert np.array_equal(_run_inv(plan, a, word_bits), oracle.inverse(a, moduli))
    da, db = to_device(a, word_bits), to_device(b, word_bits)
    out = empty_device(a.shape, word_bits)
    plan.polymul(out, da, db)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.polymul(a, b, moduli))


@pytest.mark.parametrize("cls", ["u32", "f64", "i64", "mixed64"])
@pytest.mark.parametrize("logn", [8, 10, 12, 13, 16])
def test_radix4_rows_are_bit_identical(cls, logn):
    """Row passes with 4 values per thread (radix-4 rounds), forced for every split
    whose row part is 2^8 .. 2^12 words, give the oracle's words in both directions;
    polymul under the same flag keeps its own rows and stays exact."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    a = _data(300 + logn, moduli, 3, N, word_bits)
    b = _data(301 + logn, moduli, 3, N, word_bits)
    want_f = oracle.forward(a, moduli)
    want_i = oracle.inverse(a, moduli)
    splits = [n1 for n1 in _valid_splits(logn) if 8 <= logn - n1 <= 12]
    assert splits
    for n1 in splits:
        plan = ntt.Plan(N, moduli, word_bits, flags=ntt.flag_split(n1) | ntt.FLAG_ROW_RADIX4)
        assert np.array_equal(_run_fwd(plan, a, word_bits), want_f), n1
        assert np.array_equal(_run_inv(plan, a, word_bits), want_i), n1
    da, db = to_device(a, word_bits), to_device(b, word_bits)
    out = empty_device(a.shape, word_bits)
    ntt.Plan(N, moduli, word_bits, flags=ntt.FLAG_ROW_RADIX4).polymul(out, da, db)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.polymul(a, b, moduli))


Q56 = synth.latency_prime()


@pytest.mark.parametrize("logn", [10, 12, 13, 14, 15, 16])
def test_single_polynomial_56_bit_prime_uses_radix4_rows(logn):
    """One polynomial over one 56-bit prime (the paper's single-transform setting):
    the default plan runs radix-4 rows (few row chunks) and matches the oracle."""
    N = 1 << logn
    a = _data(500 + logn, [Q56], 1, N, 64)
    b = _data(501 + logn, [Q56], 1, N, 64)
    plan = ntt.Plan(N, [Q56], 64)
    assert plan.limb_class(0) == 2  # the 64-bit integer class
    ntt.stats_reset()
    ntt.stats_enable(True)
    try:
        f = _run_fwd(plan, a, 64)
        i = _run_inv(plan, a, 64)
        names = set(ntt.stats_collect())
    finally:
        ntt.stats_enable(False)
        ntt.stats_reset()
    assert np.array_equal(f, oracle.forward(a, [Q56]))
    assert np.array_equal(i, oracle.inverse(a, [Q56]))
    n2 = logn - plan.split_for(1)
    if 8 <= n2 <= 12:
        assert any(k.startswith("row4_fwd_i64") for k in names), names
        assert any(k.startswith("row4_inv_i64") for k in names), names
    da, db = to_device(a, 64), to_device(b, 64)
    out = empty_device(a.shape, 64)
    plan.polymul(out, da, db)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out, 64).astype(np.uint64), oracle.polymul(a, b, [Q56]))


@pytest.mark.parametrize("cls", ["u32", "i64"])
@pytest.mark.parametrize("logn", [10, 12, 16])
def test_tuning_table_radix4_rows_are_bit_identical(cls, logn, tmp_path):
    """A tuning table that picks 4 values per row-pass thread for forward and
    inverse rows (and, invalidly, for polymul rows, which keep radix-8/16) gives
    the oracle's words at a batch far above the radix-4 default."""
    import json
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    entries = [{"kind": k, "log_n": logn, "cls": c, "bucket": bk, "value": 2}
               for k in (2, 3, 4) for c in range(3) for bk in range(25)]
    path = tmp_path / "rb4.json"
    path.write_text(json.dumps({"entries": entries}))
    ntt.tune_clear()
    ntt.tune_load(str(path))
    try:
        batch = 150
        a = _data(93 + logn, moduli, batch, N, word_bits)
        b = _data(94 + logn, moduli, batch, N, word_bits)
        plan = ntt.Plan(N, moduli, word_bits)
        assert np.array_equal(_run_fwd(plan, a, word_bits), oracle.forward(a, moduli))
        assert np.array_equal(_run_inv(plan, a, word_bits), oracle.inverse(a, moduli))
        da, db = to_device(a, word_bits), to_device(b, word_bits)
        out = empty_device(a.shape, word_bits)
        plan.polymul(out, da, db)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.polymul(a, b, moduli))
    finally:
        ntt.tune_clear()


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
@pytest.mark.parametrize("logn", [10, 13, 16])
def test_tuning_table_radix16_rows_are_bit_identical(cls, logn, tmp_path):
    """A tuning table that picks 16 values per row-pass thread for every direction
    (forward, inverse and polymul rows) gives the same words as the oracle."""
    import json
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    entries = [{"kind": k, "log_n": logn, "cls": c, "bucket": b, "value": 4}
               for k in (2, 3, 4) for c in range(3) for b in range(25)]
    path = tmp_path / "rb16.json"
    path.write_text(json.dumps({"entries": entries}))
    ntt.tune_clear()
    ntt.tune_load(str(path))
    try:
        a = _data(91 + logn, moduli, 3, N, word_bits)
        b = _data(92 + logn, moduli, 3, N, word_bits)
        plan = ntt.Plan(N, moduli, word_bits)
        assert np.array_equal(_run_fwd(plan, a, word_bits), oracle.forward(a, moduli))
        assert np.array_equal(_run_inv(plan, a, word_bits), oracle.inverse(a, moduli))
        da, db = to_device(a, word_bits), to_device(b, word_bits)
        out = empty_device(a.shape, word_bits)
        plan.polymul(out, da, db)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.polymul(a, b, moduli))
    finally:
        ntt.tune_clear()


@pytest.mark.parametrize("cls", ["u32", "f64", "i64", "mixed64"])
@pytest.mark.parametrize("logn", [5, 9, 12, 16])
@pytest.mark.parametrize("block", [64, 128])
def test_tuning_table_column_workgroup_sizes_are_bit_identical(cls, logn, block, tmp_path):
    """A tuning table that picks 64 or 128 columns per column-pass workgroup gives
    the oracle's words at every split, forward, inverse and polymul, with column
    counts that leave the last workgroup partly empty (3 polynomials)."""
    import json
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    entries = [{"kind": 5, "log_n": logn, "cls": c, "bucket": b, "value": block}
               for c in range(3) for b in range(25)]
    path = tmp_path / "cb.json"
    path.write_text(json.dumps({"entries": entries}))
    ntt.tune_clear()
    ntt.tune_load(str(path))
    try:
        a = _data(95 + logn, moduli, 3, N, word_bits)
        b = _data(96 + logn, moduli, 3, N, word_bits)
        want_f = oracle.forward(a, moduli)
        want_i = oracle.inverse(a, moduli)
        for n1 in _valid_splits(logn):
            if n1 == 0:
                continue
            plan = ntt.Plan(N, moduli, word_bits, flags=ntt.flag_split(n1))
            assert np.array_equal(_run_fwd(plan, a, word_bits), want_f), n1
            assert np.array_equal(_run_inv(plan, a, word_bits), want_i), n1
        plan = ntt.Plan(N, moduli, word_bits)
        da, db = to_device(a, word_bits), to_device(b, word_bits)
        out = empty_device(a.shape, word_bits)
        plan.polymul(out, da, db)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out, word_bits).astype(np.uint64), oracle.polymul(a, b, moduli))
    finally:
        ntt.tune_clear()


@pytest.mark.parametrize("cls", ["u32", "f64", "i64", "mixed64"])
@pytest.mark.parametrize("logn", [13, 14, 15, 16])
@pytest.mark.parametrize("batch", [1, 3])
def test_single_launch_two_pass_is_bit_identical(cls, logn, batch):
    """Both passes in one persistent launch (per-transform counters) give the
    oracle's words, forward and inverse, radix-16 and radix-8 rows."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    a = _data(300 + logn + batch, moduli, batch, N, word_bits)
    want_f = oracle.forward(a, moduli)
    want_i = oracle.inverse(a, moduli)
    for extra in (0, ntt.FLAG_ROW_RADIX8):
        plan = ntt.Plan(N, moduli, word_bits, flags=ntt.FLAG_FUSED | extra)
        assert np.array_equal(_run_fwd(plan, a, word_bits), want_f), extra
        assert np.array_equal(_run_inv(plan, a, word_bits), want_i), extra


def test_single_launch_full_c2_shape_matches_two_launches():
    """4 x 36 x 2^16 (the CKKS-shaped workload): the single-launch form gives the
    same words as the two-launch form for forward and inverse, and the oracle's
    words on sampled limb-rows."""
    mods = synth.c2_primes(36)
    N = 1 << 16
    a = synth.uniform_poly(5, mods, 4, N)
    two = ntt.Plan(N, mods, 64)
    one = ntt.Plan(N, mods, 64, flags=ntt.FLAG_FUSED)
    d1, d2 = to_device(a, 64), to_device(a, 64)
    two.forward(d1)
    one.forward(d2)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2)
    f = to_host(d2, 64)
    for (b, l) in [(0, 0), (1, 17), (3, 35), (2, 8)]:
        assert np.array_equal(f[b:b + 1, l:l + 1], oracle.forward(a[b:b + 1, l:l + 1], [mods[l]]))
    two.inverse(d1)
    one.inverse(d2)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2)
    assert np.array_equal(to_host(d2, 64), a)


def test_single_launch_wait_expiry_is_reported():
    """A wait of the single-launch form that gives up is reported as
    NTT_ETIMEOUT.  The condition is forced from the host: every wait's target is
    made unreachable and the poll bound is 4, so each wait gives up quickly and
    every workgroup still finishes its pieces and exits.  Afterwards the
    default restores bit-exact results."""
    mods = Q50[:2]
    N = 1 << 14
    a = _data(83, mods, 2, N, 64)
    plan = ntt.Plan(N, mods, 64, flags=ntt.FLAG_FUSED)
    d = to_device(a, 64)
    ntt.debug_wait_limit(4, True)
    try:
        with pytest.raises(ntt.NTTError) as e:
            plan.forward(d)
        assert e.value.name == "NTT_ETIMEOUT"
        with pytest.raises(ntt.NTTError) as e:
            plan.inverse(d)
        assert e.value.name == "NTT_ETIMEOUT"
    finally:
        ntt.debug_wait_limit(0, False)
    torch.cuda.synchronize()
    d = to_device(a, 64)
    plan.forward(d)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(d, 64).astype(np.uint64), oracle.forward(a, mods))


@pytest.mark.parametrize("cls", ["u32", "f64", "i64"])
def test_pointwise_with_operands_not_16_byte_aligned(cls):
    """Operands one word past a 16-byte boundary take the one-word-per-thread path
    and give the same words."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << 10
    a = _data(41, moduli, 2, N, word_bits)
    b = _data(42, moduli, 2, N, word_bits)
    n = a.size
    fa = torch.zeros(n + 1, dtype=torch.int64 if word_bits == 64 else torch.int32, device="cuda")
    fb, fo = torch.zeros_like(fa), torch.zeros_like(fa)
    da, db, do = fa[1:].view(a.shape), fb[1:].view(a.shape), fo[1:].view(a.shape)
    da.copy_(to_device(a, word_bits))
    db.copy_(to_device(b, word_bits))
    plan = ntt.Plan(N, moduli, word_bits)
    plan.pointwise_mul(do, da, db)
    torch.cuda.synchronize()
    assert do.data_ptr() % 16 != 0
    assert np.array_equal(to_host(do, word_bits).astype(np.uint64), oracle.pointwise_mul(a, b, moduli))
    assert int(fo[0].item()) == 0


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn,P,rows,cols", [(1, 5, 2, 3), (3, 7, 3, 2), (10, 13, 6, 2), (12, 4, 4, 1)])
def test_mac_matches_oracle(cls, logn, P, rows, cols):
    """Grouped MAC for every class, with a partial last group where P % rows != 0."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    a = _data(51 + logn, moduli, P, N, word_bits)
    key = _data(52 + logn, moduli, rows * cols, N, word_bits).reshape(rows, cols, len(moduli), N)
    G = (P + rows - 1) // rows
    plan = ntt.Plan(N, moduli, word_bits)
    da = to_device(a, word_bits)
    dk = to_device(key.reshape(rows * cols, len(moduli), N), word_bits)
    out = empty_device((G * cols, len(moduli), N), word_bits)
    plan.mac(out, da, dk, rows, cols)
    torch.cuda.synchronize()
    want = oracle.mac(a, key, moduli, rows, cols).reshape(G * cols, len(moduli), N)
    assert np.array_equal(to_host(out, word_bits).astype(np.uint64), want)


@pytest.mark.parametrize("cls", list(CLASSES))
@pytest.mark.parametrize("logn,P,rows,cols", [
    (10, 2048, 6, 2),   # the TFHE-shaped batch: 342 groups, the last one partial
    (4, 7, 3, 2), (6, 5, 5, 5), (8, 9, 4, 1), (12, 5, 4, 3),   # one launch
    (12, 3, 8, 2),      # 8 slots of 2^12: more than 1024 threads -> three steps
    (10, 4, 2, 3),      # cols > rows -> three steps
    (13, 3, 2, 2), (2, 5, 2, 2)])  # N outside 2^4..2^12 -> three steps
def test_external_product_matches_forward_mac_inverse(cls, logn, P, rows, cols):
    """INTT(sum_r NTT(a_r) (.) key[r][c]) against the oracle's forward, MAC and
    inverse; the operands are left unchanged."""
    word_bits, moduli = CLASSES[cls]
    N = 1 << logn
    if cls == "u32" and logn == 10 and P == 2048:
        moduli = moduli[:1]
    a = _data(61 + logn + P, moduli, P, N, word_bits)
    key = _data(62 + logn, moduli, rows * cols, N, word_bits).reshape(rows, cols, len(moduli), N)
    G = (P + rows - 1) // rows
    plan = ntt.Plan(N, moduli, word_bits)
    da = to_device(a, word_bits)
    dk = to_device(key.reshape(rows * cols, len(moduli), N), word_bits)
    out = empty_device((G * cols, len(moduli), N), word_bits)
    plan.external_product(out, da, dk, rows, cols)
    torch.cuda.synchronize()
    fa = oracle.forward(a, moduli)
    acc = oracle.mac(fa, key, moduli, rows, cols).reshape(G * cols, len(moduli), N)
    want = oracle.inverse(acc, moduli)
    assert np.array_equal(to_host(out, word_bits).astype(np.uint64), want)
    assert np.array_equal(to_host(da, word_bits).astype(np.uint64), a)


def test_bad_sizes_and_arguments_are_rejected_before_any_launch():
    """batch 0, batch * L * N >= 2^32 words, null data, aliasing and empty MAC
    shapes return NTT_EINVAL (1) from the C ABI; nothing is launched."""
    N = 1 << 16
    plan = ntt.Plan(N, Q50[:1], 64)
    a = empty_device((1, 1, N), 64)
    b = empty_device((1, 1, N), 64)
    lib = ntt.lib()
    h = plan._h
    EINVAL = 1
    assert lib.ntt_forward(h, a.data_ptr(), 0, None) == EINVAL
    assert lib.ntt_forward(h, a.data_ptr(), 1 << 16, None) == EINVAL     # exactly 2^32 words
    assert lib.ntt_inverse(h, None, 1, None) == EINVAL
    assert lib.ntt_pointwise_mul(h, a.data_ptr(), a.data_ptr(), None, 1, None) == EINVAL
    assert lib.ntt_polymul(h, a.data_ptr(), a.data_ptr(), b.data_ptr(), 1, None) == EINVAL
    assert lib.ntt_mac(h, a.data_ptr(), b.data_ptr(), b.data_ptr(), 0, 1, 1, None) == EINVAL
    assert lib.ntt_external_product(h, a.data_ptr(), a.data_ptr(), b.data_ptr(), 1, 1, 1, None) == EINVAL
    assert lib.ntt_external_product(h, a.data_ptr(), b.data_ptr(), b.data_ptr(), 1, 0, 1, None) == EINVAL
    torch.cuda.synchronize()


def test_a_thousand_limbs():
    """A plan over 1000 distinct primes (N = 16, 40-bit primes, 64-bit words):
    per-limb tables and class lists far beyond the configurations' 36 limbs."""
    N = 16
    mods = synth.primes_below(1 << 40, 2 * N, 1000)
    a = _data(71, mods, 2, N, 64)
    plan = ntt.Plan(N, mods, 64)
    f = _run_fwd(plan, a, 64)
    assert np.array_equal(f, oracle.forward(a, mods))
    assert np.array_equal(_run_inv(plan, f, 64), a)
