"""Pure-Python copy of the oracle's definitions for tiny N (test infrastructure only).

Written independently of ``oracle.c`` so that the two cross-check each other:
Python's arbitrary-precision integers and the built-in three-argument ``pow``
replace the C code's 128-bit products.  Follows arXiv 2109.14704, section II-B
(psi-twisted NTT, psi^2 = omega) and section II-A (product in Z_q[x]/(x^N+1)).
"""


def bitrev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def is_prime_trial(n):
    """Trial division; only for the small moduli of the tiny tests."""
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def order(x, q):
    k, y = 1, x % q
    while y != 1:
        y = y * x % q
        k += 1
    return k


def smallest_psi(q, n):
    """Smallest element of multiplicative order exactly 2n, by exhaustive search."""
    for x in range(2, q):
        if pow(x, 2 * n, q) == 1 and order(x, q) == 2 * n:
            return x
    raise ValueError("no primitive 2N-th root")


def ntt_fwd(a, q, psi):
    n = len(a)
    bits = n.bit_length() - 1
    return [sum(a[i] * pow(psi, i * (2 * bitrev(k, bits) + 1), q) for i in range(n)) % q for k in range(n)]


def ntt_inv(A, q, psi):
    n = len(A)
    bits = n.bit_length() - 1
    psi_inv = pow(psi, -1, q)
    n_inv = pow(n, -1, q)
    return [n_inv * sum(A[k] * pow(psi_inv, i * (2 * bitrev(k, bits) + 1), q) for k in range(n)) % q
            for i in range(n)]


def negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                out[i + j] += a[i] * b[j]
            else:
                out[i + j - n] -= a[i] * b[j]
    return [v % q for v in out]
