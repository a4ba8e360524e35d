"""Pure-Python big-integer definitions for tiny sizes (TEST INFRASTRUCTURE ONLY).

A second, independent statement of the same definitions the C oracle
implements, in arbitrary-precision Python integers, used only to cross-check
the C oracle for N <= 64.  Paper: Chameleon (arXiv 2410.05934), Sec. II-D.
"""
from __future__ import annotations


def is_prime_trial(n: int) -> bool:
    """Trial division: slow but beyond doubt, for small n."""
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def smallest_qnr_bruteforce(q: int) -> int:
    """Smallest g >= 2 that is not a square mod q, by listing all squares."""
    squares = {(x * x) % q for x in range(q)}
    for g in range(2, q):
        if g not in squares:
            return g
    raise ValueError("no non-residue")


def brv(x: int, bits: int) -> int:
    return int(format(x, f"0{bits}b")[::-1], 2) if bits else 0


def ntt_definition(a: list[int], q: int, psi: int) -> list[int]:
    """out[j] = a(psi^(2*brv(j)+1)) mod q, each term summed explicitly."""
    N = len(a)
    bits = N.bit_length() - 1
    out = []
    for j in range(N):
        e = 2 * brv(j, bits) + 1
        out.append(sum(a[i] * pow(psi, e * i, q) for i in range(N)) % q)
    return out


def intt_definition(ahat: list[int], q: int, psi: int) -> list[int]:
    N = len(ahat)
    bits = N.bit_length() - 1
    psi_inv = pow(psi, q - 2, q)
    n_inv = pow(N, q - 2, q)
    out = []
    for i in range(N):
        s = sum(ahat[j] * pow(psi_inv, (2 * brv(j, bits) + 1) * i, q) for j in range(N))
        out.append(s * n_inv % q)
    return out


def negacyclic_schoolbook(a: list[int], b: list[int], q: int) -> list[int]:
    """Product in Z_q[x]/(x^N+1): multiply as polynomials, then x^N -> -1."""
    N = len(a)
    full = [0] * (2 * N)
    for i in range(N):
        for j in range(N):
            full[i + j] += a[i] * b[j]
    return [(full[k] - full[k + N]) % q for k in range(N)]
