"""Pins of the CPU oracle to things other than itself (CPU only).

The paper (arXiv 2109.14704) prints no worked example, so the pins are
mathematical: hand-worked tiny cases (tests/golden/hand_examples.json), the
O(N^2) definitions of section II-B against the radix-2 algorithms, an
independent pure-Python copy, closed forms, the convolution theorem against
the schoolbook product of section II-A, round trips, twiddle-order
invariants, and number-theory facts for the prime search.
"""
import json
import os
import random

import numpy as np
import pytest

import oracle
from oracle import tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_poly(rng, n, q):
    return np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)


# ---------------------------------------------------------------- primes ---
def test_is_prime_known_values():
    primes = [2, 3, 5, 17, 257, 65537, 2147483647, 1000000007, (1 << 61) - 1, 18446744073709551557]
    composites = [1, 4, 561, 41041, 825265, 3215031751, 2152302898747, 3474749660383, 341550071728321,
                  3825123056546413051, (1 << 64) - 1, 4294967297, 18446744073709551615]
    for p in primes:
        assert oracle.is_prime(p), p
    for c in composites:
        assert not oracle.is_prime(c), c


def test_is_prime_matches_trial_division():
    for n in range(0, 20000):
        assert oracle.is_prime(n) == tiny.is_prime_trial(n), n


def test_gen_primes_small_matches_trial_division():
    for bits, M in [(12, 8), (14, 32), (16, 64)]:
        want = []
        q = ((1 << bits) - 1) // M * M + 1
        if q >= (1 << bits):
            q -= M
        while len(want) < 3:
            if tiny.is_prime_trial(q):
                want.append(q)
            q -= M
        assert oracle.gen_primes(bits, M, 3) == want


def test_moduli_fixture_is_consistent():
    with open(os.path.join(GOLDEN, "moduli.json")) as f:
        chains = json.load(f)
    for name, ch in chains.items():
        mods = ch["moduli"]
        assert len(set(mods)) == len(mods)
        for q, b in zip(mods, ch["bits"]):
            assert oracle.is_prime(q) and (q - 1) % ch["M"] == 0 and q < (1 << b) and q >= (1 << (b - 1))
            assert q < (1 << 60)


# ------------------------------------------------------------------ psi ----
@pytest.mark.parametrize("q,log_n", [(5, 1), (17, 2), (17, 3), (97, 4), (193, 5), (257, 7), (7681, 8),
                                     (12289, 10)])
def test_psi_is_smallest_primitive_root(q, log_n):
    assert oracle.psi(q, log_n) == tiny.smallest_psi(q, 1 << log_n)


def test_hand_examples():
    with open(os.path.join(GOLDEN, "hand_examples.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        q, ln = c["q"], c["log_n"]
        assert oracle.psi(q, ln) == c["psi"]
        f, i = oracle.psi_tables(q, ln)
        assert list(f) == c["psi_rev"] and list(i) == c["inv_psi_rev"]
        assert oracle.invmod(1 << ln, q) == c["n_inv"]
        for a, A in c["fwd"]:
            assert list(oracle.dft_fwd(a, q, ln)) == A
            assert list(oracle.ntt_fwd_r2(a, q, ln)) == A
            assert list(oracle.dft_inv(A, q, ln)) == a
            assert list(oracle.ntt_inv_r2(A, q, ln)) == a
            assert tiny.ntt_fwd(a, q, c["psi"]) == A


def test_exhaustive_n2_q5():
    for a0 in range(5):
        for a1 in range(5):
            a = [a0, a1]
            A = oracle.ntt_fwd_r2(a, 5, 1)
            assert list(A) == tiny.ntt_fwd(a, 5, 2) == list(oracle.dft_fwd(a, 5, 1))
            assert list(oracle.ntt_inv_r2(A, 5, 1)) == a


def test_exhaustive_n4_q17():
    # all 17^4 inputs: radix-2 forward vs the O(N^2) definition, and round trip
    import itertools
    q, ln = 17, 2
    f, i = oracle.psi_tables(q, ln)
    for a in itertools.product(range(17), repeat=4):
        A = oracle.ntt_fwd_r2(list(a), q, ln)
        assert tuple(oracle.ntt_inv_r2(A, q, ln)) == a
        if sum(a) % 7 == 0:
            assert np.array_equal(A, oracle.dft_fwd(list(a), q, ln))


# -------------------------------------------- definitions vs algorithms ----
SMALL_PRIMES = [(7681, 8), (12289, 10), (40961, 12)]


def _chain_primes(n):
    return oracle.gen_primes(60, 1 << 18, n) + oracle.gen_primes(50, 1 << 18, n)


@pytest.mark.parametrize("log_n", [1, 2, 3, 4, 5, 6])
def test_pure_python_copy_agrees(log_n):
    rng = random.Random(log_n)
    for q in [p for p, m in SMALL_PRIMES if m > log_n] + _chain_primes(1):
        ps = oracle.psi(q, log_n)
        a = [rng.randrange(q) for _ in range(1 << log_n)]
        assert list(oracle.dft_fwd(a, q, log_n)) == tiny.ntt_fwd(a, q, ps)
        assert list(oracle.dft_inv(a, q, log_n)) == tiny.ntt_inv(a, q, ps)
        b = [rng.randrange(q) for _ in range(1 << log_n)]
        assert list(oracle.negacyclic_schoolbook(a, b, q)) == tiny.negacyclic(a, b, q)


@pytest.mark.parametrize("log_n", [3, 5, 7, 8, 10])
def test_radix2_matches_definition(log_n):
    rng = random.Random(100 + log_n)
    for q in _chain_primes(2):
        a = rand_poly(rng, 1 << log_n, q)
        A = oracle.dft_fwd(a, q, log_n)
        assert np.array_equal(oracle.ntt_fwd_r2(a, q, log_n), A)
        assert np.array_equal(oracle.ntt_inv_r2(A, q, log_n), a)
        assert np.array_equal(oracle.dft_inv(A, q, log_n), a)
        for k in [0, 1, (1 << log_n) - 1, rng.randrange(1 << log_n)]:
            assert oracle.ntt_fwd_point(a, q, log_n, k) == int(A[k])
            assert oracle.ntt_inv_point(A, q, log_n, k) == int(a[k])


# --------------------------------------------------------- closed forms ----
@pytest.mark.parametrize("log_n", [4, 9, 12])
def test_monomial_closed_form(log_n):
    q = _chain_primes(1)[0]
    n = 1 << log_n
    ps = oracle.psi(q, log_n)
    for m in [0, 1, 3, n - 1]:
        a = np.zeros(n, dtype=np.uint64)
        a[m] = 1
        A = oracle.ntt_fwd_r2(a, q, log_n)
        want = [pow(ps, m * (2 * tiny.bitrev(k, log_n) + 1), q) for k in range(n)]
        assert [int(v) for v in A] == want


def test_constant_and_linearity():
    rng = random.Random(7)
    log_n = 10
    n = 1 << log_n
    for q in _chain_primes(2):
        c = rng.randrange(q)
        a = np.zeros(n, dtype=np.uint64)
        a[0] = c
        assert np.all(oracle.ntt_fwd_r2(a, q, log_n) == c)
        x, y = rand_poly(rng, n, q), rand_poly(rng, n, q)
        al, be = rng.randrange(q), rng.randrange(q)
        comb = np.array([(al * int(u) + be * int(v)) % q for u, v in zip(x, y)], dtype=np.uint64)
        X, Y = oracle.ntt_fwd_r2(x, q, log_n), oracle.ntt_fwd_r2(y, q, log_n)
        want = [(al * int(u) + be * int(v)) % q for u, v in zip(X, Y)]
        assert [int(v) for v in oracle.ntt_fwd_r2(comb, q, log_n)] == want


def test_negacyclic_shift_and_wraparound():
    rng = random.Random(8)
    log_n = 8
    n = 1 << log_n
    q = _chain_primes(1)[0]
    a = rand_poly(rng, n, q)
    xpoly = np.zeros(n, dtype=np.uint64)
    xpoly[1] = 1
    prod = oracle.batch_polymul(xpoly.reshape(1, 1, n), a.reshape(1, 1, n), [q])[0, 0]
    want = [(q - int(a[-1])) % q] + [int(v) for v in a[:-1]]
    assert [int(v) for v in prod] == want
    for i in [1, 5, n - 1]:
        u = np.zeros(n, dtype=np.uint64); u[i] = 1
        v = np.zeros(n, dtype=np.uint64); v[n - i] = 1
        p = oracle.batch_polymul(u.reshape(1, 1, n), v.reshape(1, 1, n), [q])[0, 0]
        assert int(p[0]) == q - 1 and not p[1:].any()


# ------------------------------------------------ convolution theorem ----
@pytest.mark.parametrize("log_n", [2, 6, 9, 11])
def test_convolution_theorem(log_n):
    rng = random.Random(200 + log_n)
    n = 1 << log_n
    mods = _chain_primes(2)
    a = np.stack([rand_poly(rng, n, q) for q in mods]).reshape(1, len(mods), n)
    b = np.stack([rand_poly(rng, n, q) for q in mods]).reshape(1, len(mods), n)
    prod = oracle.batch_polymul(a, b, mods)
    for l, q in enumerate(mods):
        assert np.array_equal(prod[0, l], oracle.negacyclic_schoolbook(a[0, l], b[0, l], q))
        for k in [0, n - 1, rng.randrange(n)]:
            assert oracle.negacyclic_point(a[0, l], b[0, l], q, k) == int(prod[0, l, k])


def test_polymul_plain4096_against_schoolbook():
    import workloads
    w = workloads.plain4096()
    q = w["moduli"][0]
    prod = oracle.batch_polymul(w["a"], w["b"], [q])
    assert np.array_equal(prod[0, 0], oracle.negacyclic_schoolbook(w["a"][0, 0], w["b"][0, 0], q))


def test_tensor_definition():
    rng = random.Random(9)
    log_n = 6
    n = 1 << log_n
    mods = _chain_primes(2)
    c = np.stack([np.stack([rand_poly(rng, n, q) for q in mods]) for _ in range(2)]).reshape(1, 2, 4, n)
    d = np.stack([np.stack([rand_poly(rng, n, q) for q in mods]) for _ in range(2)]).reshape(1, 2, 4, n)
    out = oracle.batch_ct_tensor_coeff(c, d, mods)
    for l, q in enumerate(mods):
        c0, c1, d0, d1 = c[0, 0, l], c[0, 1, l], d[0, 0, l], d[0, 1, l]
        s = oracle.negacyclic_schoolbook
        assert np.array_equal(out[0, 0, l], s(c0, d0, q))
        mid = [(int(u) + int(v)) % q for u, v in zip(s(c0, d1, q), s(c1, d0, q))]
        assert [int(v) for v in out[0, 1, l]] == mid
        assert np.array_equal(out[0, 2, l], s(c1, d1, q))
    # NTT-domain tensor element by element with Python integers
    C = oracle.batch_ntt(c, mods, +1)
    D = oracle.batch_ntt(d, mods, +1)
    T = oracle.batch_tensor(C, D, mods)
    for l, q in enumerate(mods):
        for k in range(0, n, 7):
            c0, c1, d0, d1 = (int(C[0, 0, l, k]), int(C[0, 1, l, k]), int(D[0, 0, l, k]), int(D[0, 1, l, k]))
            assert int(T[0, 0, l, k]) == c0 * d0 % q
            assert int(T[0, 1, l, k]) == (c0 * d1 + c1 * d0) % q
            assert int(T[0, 2, l, k]) == c1 * d1 % q


# ------------------------------------------------------------ round trip --
@pytest.mark.parametrize("shape,log_n", [((3, 2), 6), ((2, 3), 12), ((1, 2), 15)])
def test_round_trip_batched(shape, log_n):
    rng = np.random.default_rng(log_n)
    mods = _chain_primes(2)[: shape[1]]
    x = np.stack([rng.integers(0, q, size=(shape[0], 1 << log_n), dtype=np.uint64) for q in mods], axis=1)
    X = oracle.batch_ntt(x, mods, +1)
    assert np.array_equal(oracle.batch_ntt(X, mods, -1), x)


# ------------------------------------------------- twiddle-order invariants --
@pytest.mark.parametrize("log_n", [5, 12, 17])
def test_twiddle_invariants(log_n):
    n = 1 << log_n
    for q in _chain_primes(1):
        ps = oracle.psi(q, log_n)
        f, i = oracle.psi_tables(q, log_n)
        f = [int(v) for v in f]
        i = [int(v) for v in i]
        assert f[0] == 1 and pow(f[1], 2, q) == q - 1 and pow(ps, n, q) == q - 1
        for k in range(1, min(n // 2, 4096)):
            assert pow(f[2 * k], 2, q) == f[k]
            assert f[2 * k + 1] == f[2 * k] * f[1] % q
        for k in range(0, n, max(1, n // 512)):
            assert f[k] * i[k] % q == 1


# ---------------------------------------------------------------- rescale --
# RS of section II-A: c' = round(c q_{l-1} / q_l) mod q_{l-1}.  Pinned against
# the definition itself: CRT reconstruction of each coefficient as a Python
# integer and exact rational rounding (fractions), independent of the RNS
# formula the oracle uses.
def _crt(residues, moduli):
    Q = 1
    for q in moduli:
        Q *= q
    x = 0
    for r, q in zip(residues, moduli):
        Mi = Q // q
        x += int(r) * Mi * pow(Mi, -1, q)
    return x % Q, Q


def _round_div(x, d):
    from fractions import Fraction
    return round(Fraction(x, d))   # d odd: no exact halves, so the tie rule never applies


@pytest.mark.parametrize("limbs", [2, 3, 5])
def test_rescale_is_rounded_division(limbs):
    import workloads
    mods = workloads.moduli("ct_tensor")[:limbs]
    rng = random.Random(70 + limbs)
    n = 16
    x = np.array([[[rng.randrange(q) for _ in range(n)] for q in mods] for _ in range(3)], dtype=np.uint64)
    got = oracle.batch_rescale(x, mods)
    assert got.shape == (3, limbs - 1, n)
    for b in range(3):
        for k in range(n):
            X, _ = _crt([x[b, l, k] for l in range(limbs)], mods)
            want = _round_div(X, mods[-1])
            for i in range(limbs - 1):
                assert int(got[b, i, k]) == want % mods[i], (b, k, i)


def test_rescale_rounding_boundaries():
    """x = k qL + h rounds down, k qL + h + 1 rounds up (h = (qL - 1) / 2),
    exact multiples divide exactly, and the largest residue wraps to 0."""
    import workloads
    mods = workloads.moduli("ct_tensor")[:3]
    qL = mods[-1]
    h = (qL - 1) // 2
    Q = mods[0] * mods[1] * qL
    cases = []
    for k in [0, 1, 12345, mods[0] * mods[1] - 1]:
        cases += [(k * qL, k), (k * qL + h, k), (k * qL + h + 1, k + 1)]
    cases = [(x, want) for x, want in cases if x < Q]
    cases.append((Q - 1, mods[0] * mods[1]))           # rounds up to Q / qL = 0 mod q_i
    x = np.array([[[X % q for X, _ in cases] for q in mods]], dtype=np.uint64)
    got = oracle.batch_rescale(x, mods)
    for k, (X, want) in enumerate(cases):
        for i in range(2):
            assert int(got[0, i, k]) == want % mods[i], (X, i)


def test_rescale_ntt_domain_is_linear_and_scales_by_the_dropped_prime():
    """In the NTT domain the rescale commutes with the transforms; for inputs
    that are exact multiples of qL (x = qL y) it returns NTT(y)."""
    import workloads
    mods = workloads.moduli("ct_tensor")[:3]
    qL = mods[-1]
    rng = np.random.default_rng(5)
    n = 64
    y = np.stack([rng.integers(0, mods[i], size=(2, n), dtype=np.uint64) for i in range(2)], axis=1)
    # x = qL * y in every limb (residue 0 in the dropped limb)
    x = np.zeros((2, 3, n), dtype=np.uint64)
    for i in range(2):
        x[:, i] = [[(int(v) * qL) % mods[i] for v in row] for row in y[:, i]]
    X = oracle.batch_ntt(x, mods, +1)
    got = oracle.batch_rescale_ntt(X, mods)
    assert np.array_equal(got, oracle.batch_ntt(y, mods[:2], +1))


# ----------------------------------------------------------------- matMul --
def test_ct_matmul_matches_schoolbook_products():
    """C += A*B over ciphertexts in the NTT domain (section IV-E) equals, after
    the inverse transform, the coefficient-domain sum of negacyclic schoolbook
    tensor products: the convolution theorem, not the oracle's own formula."""
    import workloads
    mods = workloads.moduli("uneven")[:2]
    n, m, nn, k = 32, 2, 3, 2
    rng = np.random.default_rng(11)
    def coeff(shape):
        out = np.empty(shape + (2, n), dtype=np.uint64)
        for l, q in enumerate(mods):
            out[..., l, :] = rng.integers(0, q, size=shape + (n,), dtype=np.uint64)
        return out
    a, b, c = coeff((m, k, 2)), coeff((k, nn, 2)), coeff((m, nn, 3))
    ntt = lambda x: oracle.batch_ntt(x.reshape(-1, 2, n), mods, +1).reshape(x.shape)
    got = oracle.ct_matmul(ntt(a), ntt(b), ntt(c), mods)
    got = oracle.batch_ntt(got.reshape(-1, 2, n), mods, -1).reshape(got.shape)
    for i in range(m):
        for j in range(nn):
            for li, q in enumerate(mods):
                want = [c[i, j, s, li].astype(object) for s in range(3)]
                for l in range(k):
                    x0, x1 = a[i, l, 0, li], a[i, l, 1, li]
                    y0, y1 = b[l, j, 0, li], b[l, j, 1, li]
                    p = lambda u, v: oracle.negacyclic_schoolbook(u, v, q).astype(object)
                    want[0] = (want[0] + p(x0, y0)) % q
                    want[1] = (want[1] + p(x0, y1) + p(x1, y0)) % q
                    want[2] = (want[2] + p(x1, y1)) % q
                for s in range(3):
                    assert np.array_equal(got[i, j, s, li].astype(object), want[s]), (i, j, s, li)


# ------------------------------------------------------------------ relin --
def test_relin_matches_big_integer_key_switch():
    """Relin of section II-A, c' = (c0, c1) + round(P^-1 c2 evk) mod q, pinned
    against a big-integer formulation: digits of c2 as integers, key
    polynomials reconstructed by CRT over q_0 .. q_{l-1}, P, exact negacyclic
    products over the integers, exact rounding of the sum divided by P."""
    import workloads
    mods = workloads.moduli("uneven")[:3]        # q0, q1 and the special prime P
    l, n = 2, 8
    P = mods[-1]
    QP = mods[0] * mods[1] * P
    rng = np.random.default_rng(21)
    c = np.stack([np.stack([rng.integers(0, mods[i], size=n, dtype=np.uint64) for i in range(l)])
                  for _ in range(3)])[None]                                   # [1][3][l][n], NTT domain
    ksk = np.stack([np.stack([np.stack([rng.integers(0, mods[t], size=n, dtype=np.uint64) for t in range(l + 1)])
                              for _ in range(2)]) for _ in range(l)])        # [l][2][l+1][n]
    got = oracle.batch_ntt(oracle.relin(c, ksk, mods)[0], mods[:l], -1)       # [2][l][n], coefficients
    cc = oracle.batch_ntt(c[0], mods[:l], -1)                                # [3][l][n]
    kc = oracle.batch_ntt(ksk.reshape(l * 2, l + 1, n), mods, -1).reshape(l, 2, l + 1, n)

    def crt(res):
        x = 0
        for r, q in zip(res, mods):
            Mi = QP // q
            x += int(r) * Mi * pow(Mi, -1, q)
        return x % QP

    def negacyclic(a, b):
        out = [0] * n
        for i in range(n):
            for j in range(n):
                if i + j < n:
                    out[i + j] += a[i] * b[j]
                else:
                    out[i + j - n] -= a[i] * b[j]
        return out

    for s in range(2):
        S = [0] * n
        for j in range(l):
            digit = [int(v) for v in cc[2, j]]                               # [c2]_{q_j} as integers
            key = [crt(kc[j, s, :, k]) for k in range(n)]
            S = [x + y for x, y in zip(S, negacyclic(digit, key))]
        for k in range(n):
            X = S[k] % QP
            r = (X + (P - 1) // 2) // P
            for i in range(l):
                assert int(got[s, i, k]) == (int(cc[s, i, k]) + r) % mods[i], (s, i, k)
