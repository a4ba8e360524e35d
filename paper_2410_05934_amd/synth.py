"""Seeded synthetic inputs shaped like the paper's NTT workloads.

This module holds no transform arithmetic.  It draws coefficients and picks
NTT-friendly primes; the GPU library and the CPU oracle both receive what it
returns, so both sides see identical inputs.

Generator: SplitMix64 in counter form.  The k-th output (k = 1, 2, ...) of the
stream with seed s is mix(s + k * 0x9E3779B97F4A7C15 mod 2^64), where
mix(z) = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
z *= 0x94D049BB133111EB; z ^= z >> 31 (all mod 2^64).
Uniform values in [0, q) come by rejection: a draw r is accepted when
r < floor(2^64 / q) * q and then gives r mod q; a rejected position takes the
next unused draw after the block (positions in increasing order).

The paper draws random polynomials for given N and a 56-bit q (Sec. VI-B);
it names no dataset, so these synthetic inputs stand in for its workloads.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start+1 .. start+count of the stream with the given seed."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA)


def derive_seed(*parts: int) -> int:
    """Fold integers into one 64-bit seed (SplitMix64 mixing of a running sum)."""
    s = 0x243F6A8885A308D3
    for p in parts:
        s = int(splitmix64((s ^ (int(p) & 0xFFFFFFFFFFFFFFFF)), 0, 1)[0])
    return s


def uniform_below(seed: int, q: int, count: int) -> np.ndarray:
    """count values uniform in [0, q), q >= 2 (rejection, see module doc)."""
    q = int(q)
    limit = ((1 << 64) // q) * q
    r = splitmix64(seed, 0, count)
    if limit < (1 << 64):
        bad = np.nonzero(r >= np.uint64(limit))[0]
        nxt = count
        for pos in bad:
            while True:
                v = int(splitmix64(seed, nxt, 1)[0])
                nxt += 1
                if v < limit:
                    r[pos] = np.uint64(v)
                    break
    return r % np.uint64(q)


def uniform_poly(seed: int, moduli, batch: int, N: int, dtype=np.uint64) -> np.ndarray:
    """Array [batch][L][N]: row (p, l) uniform in [0, moduli[l]), its own stream."""
    moduli = [int(m) for m in np.atleast_1d(moduli)]
    L = len(moduli)
    out = np.empty((batch, L, N), dtype=dtype)
    for p in range(batch):
        for l, q in enumerate(moduli):
            out[p, l] = uniform_below(derive_seed(seed, p, l), q, N).astype(dtype)
    return out


# -- NTT-friendly primes (inputs; each consumer validates them itself) -------

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for b in _MR_BASES:
        x = pow(b, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes_below(bound: int, step: int, count: int) -> list[int]:
    """The `count` largest primes q < bound with q = 1 mod step."""
    out = []
    k = (bound - 2) // step
    while len(out) < count and k > 0:
        q = k * step + 1
        if q < bound and is_prime(q):
            out.append(q)
        k -= 1
    return out


def c1_prime(seed: int, N: int = 1 << 10) -> int:
    """30-bit prime q = k*2N + 1, scanning k upward from ceil(2^29/2N) + (seed mod 2^12)."""
    two_n = 2 * N
    k = -(-(1 << 29) // two_n) + (seed % (1 << 12))
    while True:
        q = k * two_n + 1
        if is_prime(q):
            return q
        k += 1


def c2_primes(L: int = 36) -> list[int]:
    """The L largest primes q = 1 mod 2^17 below 2^50."""
    return primes_below(1 << 50, 1 << 17, L)


def c3_prime() -> int:
    """The largest prime q = 1 mod 2^11 below 2^32."""
    return primes_below(1 << 32, 1 << 11, 1)[0]


def latency_prime() -> int:
    """The largest prime q = 1 mod 2^17 below 2^56: one 56-bit modulus, the width the
    paper's single-transform measurements use (Sec. VI-A), admissible for every N <= 2^16."""
    return primes_below(1 << 56, 1 << 17, 1)[0]


def c4_pool(seed: int, size: int = 64) -> list[int]:
    """`size` distinct primes q = 1 mod 2^17, widths uniform in 30..60 bits."""
    pool: list[int] = []
    i = 0
    while len(pool) < size:
        r = splitmix64(derive_seed(seed, 0xC4, i), 0, 2)
        i += 1
        bits = 30 + int(r[0] % np.uint64(31))
        lo, hi = 1 << (bits - 1), 1 << bits
        step = 1 << 17
        k = (lo + int(r[1] % np.uint64(hi - lo))) // step
        while True:
            q = k * step + 1
            if q >= hi:
                k = lo // step + 1
                continue
            if q >= lo and is_prime(q) and q not in pool:
                pool.append(q)
                break
            k += 1
    return pool


@dataclass
class RaggedInstance:
    N: int
    moduli: list[int] = field(default_factory=list)


def c4_instances(seed: int, count: int = 256, pool_size: int = 64,
                 log_n_range=(10, 16), limb_range=(1, 40)) -> list[RaggedInstance]:
    """Ragged mix: N = 2^(10+U{0..6}), L = U{1..40} distinct primes from the pool."""
    pool = c4_pool(seed, pool_size)
    out = []
    for j in range(count):
        r = splitmix64(derive_seed(seed, 0xC40, j), 0, 2)
        logn = log_n_range[0] + int(r[0] % np.uint64(log_n_range[1] - log_n_range[0] + 1))
        L = limb_range[0] + int(r[1] % np.uint64(limb_range[1] - limb_range[0] + 1))
        perm = np.argsort(splitmix64(derive_seed(seed, 0xC41, j), 0, len(pool)), kind="stable")
        out.append(RaggedInstance(1 << logn, [pool[int(i)] for i in perm[:L]]))
    return out


@dataclass
class Request:
    arrival_s: float
    N: int
    moduli: list[int]
    pairs: int  # number of polymul pairs (batch)
    word_bits: int
    seed: int


def c5_requests(seed: int, count: int, rate_per_s: float) -> list[Request]:
    """Poisson arrivals; 70%: 1..64 polymul pairs at N=2^10, 32-bit prime (u32);
    30%: one pair at N=2^16 with L = U{8..36} limbs of the ~50-bit primes (u64)."""
    small_q = c3_prime()
    big = c2_primes(36)
    out = []
    t = 0.0
    for i in range(count):
        r = splitmix64(derive_seed(seed, 0xC5, i), 0, 4)
        u = (int(r[0] >> np.uint64(11)) + 0.5) / float(1 << 53)
        t += -np.log(u) / rate_per_s
        if int(r[1] % np.uint64(10)) < 7:
            pairs = 1 + int(r[2] % np.uint64(64))
            out.append(Request(t, 1 << 10, [small_q], pairs, 32, derive_seed(seed, 0xC50, i)))
        else:
            L = 8 + int(r[2] % np.uint64(29))
            out.append(Request(t, 1 << 16, big[:L], 1, 64, derive_seed(seed, 0xC50, i)))
    return out
