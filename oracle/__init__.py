"""CPU oracle for the negacyclic NTT (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's ``cpu_baseline`` leg
may import this package.  The product library never imports, links or calls
it, and it imports nothing from the product library.

The arithmetic lives in ``ntt_oracle.c`` (plain radix-2 loops and the plain
definitions, unsigned __int128 products and ``%``); this module only compiles
it with gcc on first use and marshals numpy arrays.  ``py_ref`` holds a second,
pure-Python big-integer version of the definitions for tiny sizes.

Paper: Chameleon (arXiv 2410.05934), Sec. II-D and Eq. (1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntt_oracle.c")
_LIB = os.path.join(_HERE, "libntt_oracle.so")
_lock = threading.Lock()
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False) -> str:
    """Compile ntt_oracle.c into libntt_oracle.so with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
            sig = {
                "orc_powmod": (u64, [u64, u64, u64]),
                "orc_is_prime": (i32, [u64]),
                "orc_smallest_qnr": (u64, [u64]),
                "orc_psi": (u64, [u32, u64]),
                "orc_invmod": (u64, [u64, u64]),
                "orc_bitrev": (u32, [u32, i32]),
                "orc_forward": (i32, [_u64p, u32, u64]),
                "orc_inverse": (i32, [_u64p, u32, u64]),
                "orc_forward_at": (u64, [_u64p, u32, u64, u32]),
                "orc_inverse_at": (u64, [_u64p, u32, u64, u32]),
                "orc_negacyclic_at": (u64, [_u64p, _u64p, u32, u64, u32]),
                "orc_schoolbook": (None, [_u64p, _u64p, _u64p, u32, u64]),
                "orc_pointwise_mul": (None, [_u64p, _u64p, _u64p, u64, u64]),
                "orc_mac": (None, [_u64p, ctypes.POINTER(_u64p), ctypes.POINTER(_u64p), u32, u64, u64]),
                "orc_polymul": (i32, [_u64p, _u64p, _u64p, u32, u64]),
                "orc_automorph": (None, [_u64p, _u64p, u32, u64, u64]),
                "orc_bconv": (None, [_u64p, _u64p, u32, _u64p, u32, _u64p, u32]),
                "orc_sub_scale": (None, [_u64p, _u64p, _u64p, u32, ctypes.c_uint64, ctypes.c_uint64]),
                "orc_forward_batch": (i32, [_u64p, u64, u32, u32, _u64p, i32]),
                "orc_inverse_batch": (i32, [_u64p, u64, u32, u32, _u64p, i32]),
                "orc_num_cores": (i32, []),
            }
            for name, (res, args) in sig.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a).astype(np.uint64, copy=False))


# -- number theory -----------------------------------------------------------

def is_prime(n: int) -> bool:
    return bool(_load().orc_is_prime(int(n)))


def powmod(a: int, e: int, q: int) -> int:
    return int(_load().orc_powmod(int(a), int(e), int(q)))


def smallest_qnr(q: int) -> int:
    return int(_load().orc_smallest_qnr(int(q)))


def psi(N: int, q: int) -> int:
    """The oracle's primitive 2N-th root (0 if q is not admissible)."""
    return int(_load().orc_psi(int(N), int(q)))


def bitrev(x: int, bits: int) -> int:
    return int(_load().orc_bitrev(int(x), int(bits)))


def num_cores() -> int:
    return int(_load().orc_num_cores())


# -- transforms --------------------------------------------------------------

def _check_rows(a: np.ndarray, moduli) -> tuple[np.ndarray, np.ndarray, int, int, int]:
    a = _u64(a).copy()
    mod = _u64(np.atleast_1d(moduli))
    N = a.shape[-1]
    L = mod.shape[0]
    if a.ndim == 1:
        a = a.reshape(1, 1, N)
    if a.shape[-2] != L and not (a.ndim == 2 and L == 1):
        raise ValueError("limb axis does not match the number of moduli")
    batch = a.size // (L * N)
    return a, mod, batch, L, N


def forward(a, moduli, nthreads: int = 0) -> np.ndarray:
    """Forward negacyclic NTT (CT, natural in, bit-reversed out) of
    data[..., L, N] with moduli[L]; returns a new uint64 array."""
    shape = np.shape(a)
    x, mod, batch, L, N = _check_rows(a, moduli)
    rc = _load().orc_forward_batch(_p(x), batch, L, N, _p(mod), int(nthreads))
    if rc != 0:
        raise ValueError("oracle forward: inadmissible (N, q)")
    return x.reshape(shape)


def inverse(a, moduli, nthreads: int = 0) -> np.ndarray:
    """Inverse negacyclic NTT (GS, bit-reversed in, natural out, times N^-1)."""
    shape = np.shape(a)
    x, mod, batch, L, N = _check_rows(a, moduli)
    rc = _load().orc_inverse_batch(_p(x), batch, L, N, _p(mod), int(nthreads))
    if rc != 0:
        raise ValueError("oracle inverse: inadmissible (N, q)")
    return x.reshape(shape)


def forward_at(a, q: int, j: int) -> int:
    """One output of the forward transform from its definition, O(N)."""
    x = _u64(a)
    return int(_load().orc_forward_at(_p(x), x.shape[-1], int(q), int(j)))


def inverse_at(ahat, q: int, i: int) -> int:
    x = _u64(ahat)
    return int(_load().orc_inverse_at(_p(x), x.shape[-1], int(q), int(i)))


def negacyclic_at(a, b, q: int, k: int) -> int:
    """One coefficient of a*b mod (x^N+1, q) from its definition, O(N)."""
    x, y = _u64(a), _u64(b)
    return int(_load().orc_negacyclic_at(_p(x), _p(y), x.shape[-1], int(q), int(k)))


def schoolbook(a, b, q: int) -> np.ndarray:
    x, y = _u64(a), _u64(b)
    c = np.empty_like(x)
    _load().orc_schoolbook(_p(c), _p(x), _p(y), x.shape[-1], int(q))
    return c


def pointwise_mul(a, b, moduli) -> np.ndarray:
    """c = a (.) b mod q_l for data[..., L, N]."""
    x, y = _u64(a), _u64(b)
    mod = _u64(np.atleast_1d(moduli))
    N, L = x.shape[-1], mod.shape[0]
    xr = x.reshape(-1, L, N)
    yr = y.reshape(-1, L, N)
    c = np.empty_like(xr)
    lib = _load()
    for p in range(xr.shape[0]):
        for l in range(L):
            xa = np.ascontiguousarray(xr[p, l])
            ya = np.ascontiguousarray(yr[p, l])
            ca = np.empty(N, dtype=np.uint64)
            lib.orc_pointwise_mul(_p(ca), _p(xa), _p(ya), N, int(mod[l]))
            c[p, l] = ca
    return c.reshape(x.shape)


def mac(a, key, moduli, rows: int, cols: int) -> np.ndarray:
    """Grouped multiply-accumulate.

    a[P][L][N] are P transformed operands; operand p belongs to group
    g = p // rows at row r = p % rows; key[rows][cols][L][N].
    out[g][c] = sum over the rows r present in group g of a[g*rows + r] (.) key[r][c].
    The last group may be partial (fewer than `rows` operands).
    """
    x, k = _u64(a), _u64(key)
    mod = _u64(np.atleast_1d(moduli))
    P, L, N = x.shape
    G = (P + rows - 1) // rows
    out = np.empty((G, cols, L, N), dtype=np.uint64)
    lib = _load()
    for g in range(G):
        present = [r for r in range(rows) if g * rows + r < P]
        for c in range(cols):
            for l in range(L):
                xs = [np.ascontiguousarray(x[g * rows + r, l]) for r in present]
                ks = [np.ascontiguousarray(k[r, c, l]) for r in present]
                xp = (_u64p * len(xs))(*[_p(v) for v in xs])
                kp = (_u64p * len(ks))(*[_p(v) for v in ks])
                o = np.empty(N, dtype=np.uint64)
                lib.orc_mac(_p(o), xp, kp, len(xs), N, int(mod[l]))
                out[g, c, l] = o
    return out


def polymul(a, b, moduli, nthreads: int = 0) -> np.ndarray:
    """Negacyclic product through Eq. (1) on data[..., L, N]."""
    fa = forward(a, moduli, nthreads)
    fb = forward(b, moduli, nthreads)
    return inverse(pointwise_mul(fa, fb, moduli), moduli, nthreads)


# -- automorphisms (Sec. III, Sec. IV-B) --------------------------------------

def automorph(a, moduli, k: int) -> np.ndarray:
    """sigma_k on data[..., L, N] in the coefficient domain: b(x) = a(x^k) in
    Z_q[x]/(x^N+1) per limb, k odd (the plain substitution, term by term)."""
    x = _u64(a)
    mod = _u64(np.atleast_1d(moduli))
    N, L = x.shape[-1], mod.shape[0]
    xr = x.reshape(-1, L, N)
    out = np.empty_like(xr)
    lib = _load()
    for p in range(xr.shape[0]):
        for l in range(L):
            src = np.ascontiguousarray(xr[p, l])
            dst = np.empty(N, dtype=np.uint64)
            lib.orc_automorph(_p(dst), _p(src), N, int(mod[l]), int(k))
            out[p, l] = dst
    return out.reshape(x.shape)


def automorph_transformed(ahat, moduli, k: int) -> np.ndarray:
    """sigma_k on transformed data (the forward transform's output order): the
    transform of sigma_k applied to the polynomial whose transform is ahat."""
    return forward(automorph(inverse(ahat, moduli), moduli, k), moduli)


# -- gadget decomposition and the external product (Sec. II-B, Sec. IV-A) --------

def decompose(ct, moduli, levels: int, log_base: int) -> np.ndarray:
    """Signed base-B digits (B = 2^log_base) of every coefficient, the Decompose
    step of the external product.  Digit j of a is taken from the remainder r_j
    (r_0 = a): d_j = r_j mod B, moved to [-B/2, B/2) by subtracting B when it is
    B/2 or more, and r_(j+1) = (r_j - d_j) / B; the top digit is the remainder
    itself, d_(levels-1) = r_(levels-1).  Then a = sum_j d_j B^j exactly.

    ct[num_ct][comps][L][N] (words in [0, q)) -> operands[num_ct][comps*levels][L][N];
    operand c*levels + j holds d_j mod q_l of component c.
    """
    x = _u64(ct)
    num_ct, comps, L, N = x.shape
    mod = [int(q) for q in np.atleast_1d(moduli)]
    B = 1 << log_base
    out = np.empty((num_ct, comps * levels, L, N), dtype=np.uint64)
    for l in range(L):
        q = mod[l]
        r = x[:, :, l, :].astype(np.int64)
        for j in range(levels):
            if j < levels - 1:
                d = r % B
                d = np.where(d >= B // 2, d - B, d)
                r = (r - d) // B
            else:
                d = r
            out[:, j::levels, l, :] = np.where(d < 0, d + q, d).astype(np.uint64)
    return out


def external_product_decomposed(ct, key, moduli, levels: int, log_base: int, cols: int) -> np.ndarray:
    """out[g][c] = INTT( sum_r NTT(decompose(ct[g])[r]) (.) key[r][c] ): the external
    product of each ciphertext g with a key of comps*levels rows (transform domain)."""
    ops = decompose(ct, moduli, levels, log_base)
    num_ct, rows, L, N = ops.shape
    f = forward(ops.reshape(num_ct * rows, L, N), moduli)
    return inverse(mac(f, key, moduli, rows, cols), moduli)


# -- RNS basis conversion (Sec. III) -----------------------------------------------

def bconv(x, src_moduli, dst_moduli) -> np.ndarray:
    """Fast basis conversion of x[..., L, N] (residues mod src_moduli) to
    y[..., M, N] (mod dst_moduli): y_j = sum_i [x_i (Q/q_i)^-1]_(q_i) (Q/q_i) mod p_j,
    i.e. X + alpha Q mod p_j with 0 <= alpha < L."""
    a = _u64(x)
    src = _u64(np.atleast_1d(src_moduli))
    dst = _u64(np.atleast_1d(dst_moduli))
    L, M, N = src.shape[0], dst.shape[0], a.shape[-1]
    rows = a.reshape(-1, L, N)
    out = np.empty((rows.shape[0], M, N), dtype=np.uint64)
    lib = _load()
    for b in range(rows.shape[0]):
        xb = np.ascontiguousarray(rows[b])
        yb = np.empty((M, N), dtype=np.uint64)
        lib.orc_bconv(_p(yb), _p(xb), N, _p(src), L, _p(dst), M)
        out[b] = yb
    return out.reshape(a.shape[:-2] + (M, N))


def mod_up(x, q_moduli, p_moduli) -> np.ndarray:
    """ModUp (Sec. III: BConv among the CKKS key-switching operators): the
    polynomial x[..., L, N] over Q = prod q_i, extended to the basis Q u P:
    out[..., :L, :] = x and out[..., L:, :] = BConv_{Q->P}(x), i.e. X + alpha Q
    mod p_j with one 0 <= alpha < L per coefficient (not corrected)."""
    a = _u64(x)
    return np.concatenate([a, bconv(a, q_moduli, p_moduli)], axis=-2)


def mod_down(x, q_moduli, p_moduli) -> np.ndarray:
    """ModDown (Sec. III): x[..., L + K, N] over Q u P (the L limbs of Q first,
    then the K limbs of P) to out[..., L, N] over Q:
        out_i = (x_i - BConv_{P->Q}(x_P)_i) * P^-1 mod q_i,    P = prod p_k.
    For X = P Y + e (0 <= e < P) this is Y - alpha mod Q with one
    0 <= alpha < K per coefficient (the fast conversion's error, not corrected)."""
    a = _u64(x)
    qm = [int(q) for q in np.atleast_1d(q_moduli)]
    pm = [int(p) for p in np.atleast_1d(p_moduli)]
    L, K, N = len(qm), len(pm), a.shape[-1]
    assert a.shape[-2] == L + K
    rows = a.reshape(-1, L + K, N)
    conv = bconv(rows[:, L:, :], pm, qm)
    P = 1
    for pk in pm:
        P *= pk
    out = np.empty((rows.shape[0], L, N), dtype=np.uint64)
    lib = _load()
    for i, q in enumerate(qm):
        s = pow(P % q, -1, q)
        for b in range(rows.shape[0]):
            xi = np.ascontiguousarray(rows[b, i])
            ci = np.ascontiguousarray(conv[b, i])
            yi = np.empty(N, dtype=np.uint64)
            lib.orc_sub_scale(_p(yi), _p(xi), _p(ci), N, q, s)
            out[b, i] = yi
    return out.reshape(a.shape[:-2] + (L, N))


# -- one batched CMux step of blind rotation (Sec. II-B, Sec. IV-A) -------------------

def monomial_mul(a, moduli, rot) -> np.ndarray:
    """X^rot[g] * a[g] in Z_q[x]/(x^N+1) for a[num][comps][L][N] (rot[g] taken mod 2N):
    the term a_i x^i becomes a_i x^(i + r), negated each time the exponent passes N."""
    x = _u64(a)
    mod = [int(q) for q in np.atleast_1d(moduli)]
    num, comps, L, N = x.shape
    out = np.empty_like(x)
    for g in range(num):
        r = int(rot[g]) % (2 * N)
        for l in range(L):
            q = mod[l]
            for c in range(comps):
                row = [int(v) for v in x[g, c, l]]
                res = [0] * N
                for i, v in enumerate(row):
                    e = (i + r) % (2 * N)
                    if e < N:
                        res[e] = (res[e] + v) % q
                    else:
                        res[e - N] = (res[e - N] - v) % q
                out[g, c, l] = np.array(res, dtype=np.uint64)
    return out


def cmux(acc, key, moduli, rot, levels: int, log_base: int) -> np.ndarray:
    """out[g] = acc[g] + ExtProd(key, X^rot[g] acc[g] - acc[g]): the external product
    of the gadget digits of the rotated difference with the RGSW key
    key[comps*levels][comps][L][N] (transform domain), added back to acc."""
    x = _u64(acc)
    mod = np.atleast_1d(moduli).astype(np.uint64)
    rotated = monomial_mul(x, moduli, rot)
    diff = (rotated + (mod[None, None, :, None] - x)) % mod[None, None, :, None]
    prod = external_product_decomposed(diff, key, moduli, levels, log_base, x.shape[1])
    return (prod + x) % mod[None, None, :, None]
