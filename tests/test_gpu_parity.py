"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

All integer work, so the bar is bit-exactness everywhere.  Small cases are
compared element by element; full workload sizes are compared on sampled
outputs the oracle evaluates one by one (O(N) each) plus properties that
hold at any size (round trip).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

CHAIN = workloads.moduli("uneven")          # q = 1 mod 2^18: valid for every N <= 2^17


def dev(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(device)


def host(t):
    return t.cpu().numpy().view(np.uint64)


def rand_limbs(rng, shape, mods):
    out = np.empty(shape, dtype=np.uint64)
    for l, q in enumerate(mods):
        out[..., l, :] = rng.integers(0, q, size=shape[:-2] + (shape[-1],), dtype=np.uint64)
    return out


@pytest.mark.parametrize("log_n", list(range(6, 18)))
def test_fwd_inv_every_size(gpu, log_n):
    import paper_2109_14704_amd as H
    print("case fwd/inv log_n=%d" % log_n, flush=True)
    rng = np.random.default_rng(log_n)
    limbs = 3 if log_n <= 14 else 2
    batch = 3 if log_n <= 15 else 2
    mods = CHAIN[:limbs]
    x = rand_limbs(rng, (batch, limbs, 1 << log_n), mods)
    # edge values: zeros, q-1 everywhere, a monomial
    x[0, 0, :] = 0
    x[-1, -1, :] = mods[-1] - 1
    t = H.Tables(log_n, mods)
    d = dev(x, gpu)
    H.ntt_fwd(t, d)
    want = oracle.batch_ntt(x, mods, +1)
    assert np.array_equal(host(d), want)
    H.ntt_inv(t, d)
    assert np.array_equal(host(d), x)
    # inverse alone on arbitrary canonical NTT-domain input
    d2 = dev(want, gpu)
    H.ntt_inv(t, d2)
    assert np.array_equal(host(d2), x)


@pytest.mark.parametrize("log_n", [6, 12, 14, 15, 17])
def test_dyadic_and_polymul(gpu, log_n):
    import paper_2109_14704_amd as H
    print("case dyadic/polymul log_n=%d" % log_n, flush=True)
    rng = np.random.default_rng(100 + log_n)
    mods = CHAIN[:2]
    a = rand_limbs(rng, (2, 2, 1 << log_n), mods)
    b = rand_limbs(rng, (2, 2, 1 << log_n), mods)
    t = H.Tables(log_n, mods)
    out = H.dyadic_mul(t, dev(a, gpu), dev(b, gpu))
    assert np.array_equal(host(out), oracle.batch_dyadic(a, b, mods))
    p = H.polymul(t, dev(a, gpu), dev(b, gpu))
    assert np.array_equal(host(p), oracle.batch_polymul(a, b, mods))


@pytest.mark.parametrize("log_n", [6, 13, 16])
@pytest.mark.parametrize("in_ntt,out_ntt", [(False, False), (True, False), (False, True), (True, True)])
def test_ct_tensor_flags(gpu, log_n, in_ntt, out_ntt):
    import paper_2109_14704_amd as H
    print("case ct_tensor log_n=%d in_ntt=%s out_ntt=%s" % (log_n, in_ntt, out_ntt), flush=True)
    rng = np.random.default_rng(200 + log_n)
    mods = CHAIN[:3]
    c = rand_limbs(rng, (2, 2, 3, 1 << log_n), mods)
    d = rand_limbs(rng, (2, 2, 3, 1 << log_n), mods)
    C = oracle.batch_ntt(c, mods, +1)
    D = oracle.batch_ntt(d, mods, +1)
    T = oracle.batch_tensor(C, D, mods)
    want = T if out_ntt else oracle.batch_ntt(T, mods, -1)
    t = H.Tables(log_n, mods)
    cin, din = (C, D) if in_ntt else (c, d)
    cd, dd = dev(cin, gpu), dev(din, gpu)
    out = H.ct_tensor(t, cd, dd, in_ntt=in_ntt, out_ntt=out_ntt)
    assert np.array_equal(host(out), want)
    assert np.array_equal(host(cd), cin) and np.array_equal(host(dd), din)   # inputs untouched


@pytest.mark.parametrize("log_n", [13, 14, 15, 16, 17])
@pytest.mark.parametrize("batch,limbs", [(1, 1), (3, 2), (13, 5)])
def test_fused_product_shapes(gpu, log_n, batch, limbs):
    """Fused polymul and tensor for every size of the two-pass split and unit
    counts from 1 to 65, compared element by element."""
    import paper_2109_14704_amd as H
    print("case fused products log_n=%d batch=%d limbs=%d" % (log_n, batch, limbs), flush=True)
    rng = np.random.default_rng(300 + 7 * log_n + batch * limbs)
    mods = CHAIN[:limbs]
    t = H.Tables(log_n, mods)
    a = rand_limbs(rng, (batch, limbs, 1 << log_n), mods)
    b = rand_limbs(rng, (batch, limbs, 1 << log_n), mods)
    got = H.polymul(t, dev(a, gpu), dev(b, gpu))
    assert np.array_equal(host(got), oracle.batch_polymul(a, b, mods))
    if log_n <= 16:
        c = rand_limbs(rng, (batch, 2, limbs, 1 << log_n), mods)
        d = rand_limbs(rng, (batch, 2, limbs, 1 << log_n), mods)
        want = oracle.batch_ntt(oracle.batch_tensor(oracle.batch_ntt(c, mods, +1), oracle.batch_ntt(d, mods, +1), mods),
                                mods, -1)
        assert np.array_equal(host(H.ct_tensor(t, dev(c, gpu), dev(d, gpu))), want)


@pytest.mark.parametrize("log_n,variant", [(6, 1), (12, 1), (15, 1), (17, 1), (15, 5), (15, 2), (15, 3), (15, 4), (15, 0),
                                           (15, 6), (15, 7), (15, 8)])
def test_design_ladder_variants(gpu, log_n, variant):
    """Every kernel design of the ladder (naive radix-2, staged radix-2, the
    wave-shuffle SIMD variants with 1, 2 and 4 register slots, staged
    radix-4/8/16) gives the forward transform word for word."""
    import paper_2109_14704_amd as H
    print("case ladder variant=%d log_n=%d" % (variant, log_n), flush=True)
    rng = np.random.default_rng(400 + 10 * log_n + variant)
    mods = CHAIN[:3]
    x = rand_limbs(rng, (2, 3, 1 << log_n), mods)
    t = H.Tables(log_n, mods)
    got = H.ntt_fwd_variant(t, dev(x, gpu), variant)
    assert np.array_equal(host(got), oracle.batch_ntt(x, mods, +1))


def test_design_ladder_rejects(gpu):
    import paper_2109_14704_amd as H
    mods = CHAIN[:1]
    x = dev(rand_limbs(np.random.default_rng(1), (1, 1, 1 << 14), mods), gpu)
    t = H.Tables(14, mods)
    for variant in (H.VARIANT_STAGED_R8, H.VARIANT_STAGED_R2, H.VARIANT_SIMD1, H.VARIANT_SIMD4, 9, -1):
        with pytest.raises(H.HenttError):
            H.ntt_fwd_variant(t, x, variant)


@pytest.mark.parametrize("log_n", [6, 12, 14, 15, 16, 17])
@pytest.mark.parametrize("limbs", [2, 4])
def test_rescale(gpu, log_n, limbs):
    """Rescale (RS, section II-A) in both domains, element by element."""
    import paper_2109_14704_amd as H
    print("case rescale log_n=%d limbs=%d" % (log_n, limbs), flush=True)
    mods = CHAIN[:limbs]
    rng = np.random.default_rng(500 + 3 * log_n + limbs)
    t = H.Tables(log_n, mods)
    x = rand_limbs(rng, (3, limbs, 1 << log_n), mods)
    got = H.rescale(t, dev(x, gpu))
    assert np.array_equal(host(got), oracle.batch_rescale(x, mods))
    X = oracle.batch_ntt(x, mods, +1)
    Xd = dev(X, gpu)
    got = H.rescale(t, Xd, ntt=True)
    assert np.array_equal(host(got), oracle.batch_rescale_ntt(X, mods))
    assert np.array_equal(host(Xd), X)                       # input untouched


def test_rescale_level_views_and_errors(gpu):
    """A level view rescales by its own last prime; bad calls are refused."""
    import paper_2109_14704_amd as H
    mods = workloads.moduli("ct_tensor")[:5]
    t = H.Tables(15, mods)
    v = t.view(3)
    rng = np.random.default_rng(9)
    x = rand_limbs(rng, (2, 3, 1 << 15), mods[:3])
    got = H.rescale(v, dev(x, gpu), ntt=True)
    assert np.array_equal(host(got), oracle.batch_rescale_ntt(x, mods[:3]))
    one = t.view(1)
    with pytest.raises(H.HenttError):
        H.rescale(one, dev(x[:, :1], gpu))
    xd = dev(x, gpu)
    alias = xd.view(-1)[: 2 * 2 * (1 << 15)].view(2, 2, 1 << 15)
    with pytest.raises(H.HenttError):                        # out overlapping c (refused by the library)
        H.rescale(v, xd, out=alias)
    import ctypes
    rc = H.lib().hentt_rescale(v.handle, ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(dev(x, gpu).data_ptr()),
                               2, H.HENTT_IN_NTT, None)
    assert rc != 0                                           # only both-or-neither NTT flags


@pytest.mark.parametrize("m,n,k,log_n", [(2, 3, 2, 13), (5, 4, 1, 12), (10, 9, 8, 6), (3, 2, 3, 13), (4, 3, 2, 8)])
def test_ct_matmul(gpu, m, n, k, log_n):
    """Encrypted element-wise polynomial matrix product, element by element."""
    import paper_2109_14704_amd as H
    print("case matmul %dx%dx%d log_n=%d" % (m, n, k, log_n), flush=True)
    mods = workloads.moduli("ct_tensor")[:4]
    rng = np.random.default_rng(600 + m * n * k + log_n)
    A = rand_limbs(rng, (m, k, 2, 4, 1 << log_n), mods)
    B = rand_limbs(rng, (k, n, 2, 4, 1 << log_n), mods)
    C = rand_limbs(rng, (m, n, 3, 4, 1 << log_n), mods)
    t = H.Tables(log_n, mods)
    Cd = dev(C, gpu)
    H.ct_matmul(t, dev(A, gpu), dev(B, gpu), Cd)
    assert np.array_equal(host(Cd), oracle.ct_matmul(A, B, C, mods))


def test_ct_matmul_paper_shape_sampled(gpu):
    """100 x 100 x 1 at N = 8192, 4 limbs (the paper's first matMul shape):
    sampled output elements against the oracle."""
    import paper_2109_14704_amd as H
    mods = workloads.moduli("ct_tensor")[:4]
    rng = np.random.default_rng(601)
    A = rand_limbs(rng, (100, 1, 2, 4, 8192), mods)
    B = rand_limbs(rng, (1, 100, 2, 4, 8192), mods)
    t = H.Tables(13, mods)
    import torch
    Cd = torch.zeros((100, 100, 3, 4, 8192), dtype=torch.int64, device=gpu)
    H.ct_matmul(t, dev(A, gpu), dev(B, gpu), Cd)
    for i, j in [(0, 0), (99, 99), (17, 42), (63, 5)]:
        want = oracle.ct_matmul(A[i:i + 1], B[:, j:j + 1], np.zeros((1, 1, 3, 4, 8192), np.uint64), mods)
        assert np.array_equal(host(Cd[i:i + 1, j:j + 1]), want), (i, j)


@pytest.mark.parametrize("log_n,l", [(6, 2), (12, 3), (13, 2), (14, 3), (15, 2), (16, 2), (17, 2), (12, 1)])
def test_relin(gpu, log_n, l):
    """Relinearization (digit key switch, division by the special prime with
    rounding), element by element against the oracle."""
    import paper_2109_14704_amd as H
    print("case relin log_n=%d l=%d" % (log_n, l), flush=True)
    mods = CHAIN[:l + 1]                     # the last one plays the special prime P
    rng = np.random.default_rng(700 + 7 * log_n + l)
    c = rand_limbs(rng, (2, 3, l, 1 << log_n), mods[:l])
    ksk = rand_limbs(rng, (l, 2, l + 1, 1 << log_n), mods)
    t = H.Tables(log_n, mods)
    cd = dev(c, gpu)
    got = H.relin(t, cd, dev(ksk, gpu))
    assert np.array_equal(host(got), oracle.relin(c, ksk, mods))
    assert np.array_equal(host(cd), c)


def test_rescale_bench_shape_sampled(gpu):
    """Rescale at the benchmarked shape (64 polynomials of N = 2^16, 24 -> 23
    limbs, NTT domain, one call over the whole batch as the benchmark makes
    it): sampled batch entries, every limb and coefficient, against the oracle."""
    import paper_2109_14704_amd as H
    print("case rescale 64 x 24 x 2^16", flush=True)
    mods = workloads.moduli("ct_tensor")
    rng = np.random.default_rng(801)
    x = rand_limbs(rng, (64, 24, 1 << 16), mods)
    t = H.Tables(16, mods)
    got = host(H.rescale(t, dev(x, gpu), ntt=True))
    for b in (0, 37, 63):
        assert np.array_equal(got[b:b + 1], oracle.batch_rescale_ntt(x[b:b + 1], mods)), b


def test_relin_bench_shape_sampled(gpu):
    """Relinearization at the routine benchmark's shape (32 ciphertexts of
    N = 2^15 at 8 primes plus P, one call over the batch): sampled batch
    entries, every limb and coefficient, against the oracle."""
    import paper_2109_14704_amd as H
    print("case relin 32 x 8 x 2^15", flush=True)
    mods = workloads.moduli("ct_tensor")[:9]
    rng = np.random.default_rng(802)
    c = rand_limbs(rng, (32, 3, 8, 1 << 15), mods[:8])
    ksk = rand_limbs(rng, (8, 2, 9, 1 << 15), mods)
    t = H.Tables(15, mods)
    got = host(H.relin(t, dev(c, gpu), dev(ksk, gpu)))
    for b in (0, 19, 31):
        assert np.array_equal(got[b:b + 1], oracle.relin(c[b:b + 1], ksk, mods)), b


TOP = [q for q in CHAIN if q.bit_length() == 60]  # the largest primes (q < 2^60): tightest lazy ranges


def extremes(rng, shape, mods):
    """Half the words at q - 1, the rest uniform: the largest operands the
    products and their lazy ranges must take."""
    x = rand_limbs(rng, shape, mods)
    for l, q in enumerate(mods):
        sl = x[..., l, :]
        sl[..., ::2] = q - 1
    return x


@pytest.mark.parametrize("log_n", [12, 15, 16])
def test_products_at_largest_primes_and_operands(gpu, log_n):
    """Fused and NTT-domain products (Montgomery ahead of the inverse
    transform, Barrett otherwise) with 60-bit primes and operands at q - 1."""
    import paper_2109_14704_amd as H
    print("case extremes products log_n=%d" % log_n, flush=True)
    mods = TOP[:2]
    rng = np.random.default_rng(900 + log_n)
    t = H.Tables(log_n, mods)
    a, b = extremes(rng, (2, 2, 1 << log_n), mods), extremes(rng, (2, 2, 1 << log_n), mods)
    assert np.array_equal(host(H.polymul(t, dev(a, gpu), dev(b, gpu))), oracle.batch_polymul(a, b, mods))
    c, d = extremes(rng, (2, 2, 2, 1 << log_n), mods), extremes(rng, (2, 2, 2, 1 << log_n), mods)
    want_ntt = oracle.batch_tensor(c, d, mods)                  # NTT-domain in and out: plain products
    assert np.array_equal(host(H.ct_tensor(t, dev(c, gpu), dev(d, gpu), in_ntt=True, out_ntt=True)), want_ntt)
    want = oracle.batch_ntt(want_ntt, mods, -1)                 # NTT-domain in, coefficient out: Montgomery
    assert np.array_equal(host(H.ct_tensor(t, dev(c, gpu), dev(d, gpu), in_ntt=True)), want)


def test_relin_and_matmul_at_largest_primes_and_operands(gpu):
    """Key switch (Montgomery accumulation) and matMul (both accumulation
    forms) with 60-bit primes and operands at q - 1."""
    import paper_2109_14704_amd as H
    mods = TOP[:3]
    rng = np.random.default_rng(903)
    t = H.Tables(13, mods)
    c = extremes(rng, (2, 3, 2, 1 << 13), mods[:2])
    ksk = extremes(rng, (2, 2, 3, 1 << 13), mods)
    assert np.array_equal(host(H.relin(t, dev(c, gpu), dev(ksk, gpu))), oracle.relin(c, ksk, mods))
    m2 = TOP[:2]
    t2 = H.Tables(12, m2)
    for k in (1, 4):
        A = extremes(rng, (2, k, 2, 2, 1 << 12), m2)
        B = extremes(rng, (k, 3, 2, 2, 1 << 12), m2)
        C = extremes(rng, (2, 3, 3, 2, 1 << 12), m2)
        Cd = dev(C, gpu)
        H.ct_matmul(t2, dev(A, gpu), dev(B, gpu), Cd)
        assert np.array_equal(host(Cd), oracle.ct_matmul(A, B, C, m2)), k


def test_plain4096_workload(gpu):
    """Workload 1 at full size: 8 polys fwd + inv, one polymul vs schoolbook."""
    import paper_2109_14704_amd as H
    w = workloads.plain4096()
    q = w["moduli"]
    t = H.Tables(12, q)
    x = dev(w["x"], gpu)
    H.ntt_fwd(t, x)
    assert np.array_equal(host(x), oracle.batch_ntt(w["x"], q, +1))
    H.ntt_inv(t, x)
    assert np.array_equal(host(x), w["x"])
    p = H.polymul(t, dev(w["a"], gpu), dev(w["b"], gpu))
    assert np.array_equal(host(p)[0, 0], oracle.negacyclic_schoolbook(w["a"][0, 0], w["b"][0, 0], q[0]))


def _sample_points(rng, n, k):
    return sorted(set([0, n - 1] + [int(v) for v in rng.integers(0, n, size=k)]))


def test_ckks_level_workload_sampled(gpu):
    """Workload 2 at full size [128][16][2^15]: fwd, dyadic, inv; sampled outputs."""
    import paper_2109_14704_amd as H
    w = workloads.ckks_level()
    mods, ln = w["moduli"], w["log_n"]
    n = 1 << ln
    t = H.Tables(ln, mods)
    A, B = dev(w["a"], gpu), dev(w["b"], gpu)
    H.ntt_fwd(t, A)
    H.ntt_fwd(t, B)
    fa = host(A)
    rng = np.random.default_rng(5)
    for (bi, l) in [(0, 0), (127, 15), (64, 7), (3, 11)]:
        ps = oracle.psi(mods[l], ln)
        for k in _sample_points(rng, n, 6):
            assert int(fa[bi, l, k]) == oracle.ntt_fwd_point(w["a"][bi, l], mods[l], ln, k, ps)
    H.dyadic_mul(t, A, B, out=A)
    H.ntt_inv(t, A)
    prod = host(A)
    for (bi, l) in [(0, 0), (127, 15), (31, 4)]:
        for k in _sample_points(rng, n, 4):
            assert int(prod[bi, l, k]) == oracle.negacyclic_point(w["a"][bi, l], w["b"][bi, l], mods[l], k)
    # fused polymul gives the same words
    P = H.polymul(t, dev(w["a"], gpu), dev(w["b"], gpu))
    assert np.array_equal(host(P), prod)


def test_ct_tensor_workload_sampled(gpu):
    """Workload 3 at full size: [32][2][24][2^16] pairs -> [32][3][24][2^16]; sampled outputs."""
    import paper_2109_14704_amd as H
    w = workloads.ct_tensor()
    mods, ln = w["moduli"], w["log_n"]
    n = 1 << ln
    t = H.Tables(ln, mods)
    out = host(H.ct_tensor(t, dev(w["c"], gpu), dev(w["d"], gpu)))
    rng = np.random.default_rng(6)
    c, d = w["c"], w["d"]
    for (bi, l) in [(0, 0), (31, 23), (17, 9)]:
        q = mods[l]
        for k in _sample_points(rng, n, 3):
            c0d0 = oracle.negacyclic_point(c[bi, 0, l], d[bi, 0, l], q, k)
            c0d1 = oracle.negacyclic_point(c[bi, 0, l], d[bi, 1, l], q, k)
            c1d0 = oracle.negacyclic_point(c[bi, 1, l], d[bi, 0, l], q, k)
            c1d1 = oracle.negacyclic_point(c[bi, 1, l], d[bi, 1, l], q, k)
            assert int(out[bi, 0, l, k]) == c0d0
            assert int(out[bi, 1, l, k]) == (c0d1 + c1d0) % q
            assert int(out[bi, 2, l, k]) == c1d1


def test_uneven_batch_matches_oracle(gpu):
    """Workload 4 shape mix (reduced count): one ntt_batch call vs the oracle per job."""
    import paper_2109_14704_amd as H
    mods = workloads.moduli("uneven")
    jobs = workloads.uneven_jobs(njobs=24)
    tables = {ln: H.Tables(ln, mods) for ln in range(12, 18)}
    xs, devs = [], []
    for j, (ln, L) in enumerate(jobs):
        x = workloads.uneven_operand(j, ln, L, mods)
        xs.append(x)
        devs.append(dev(x, gpu))
    H.ntt_batch([(d_, tables[ln], L) for d_, (ln, L) in zip(devs, jobs)], +1)
    for j, (ln, L) in enumerate(jobs):
        got = host(devs[j])
        if (1 << ln) * L <= (1 << 17) * 4:
            assert np.array_equal(got, oracle.batch_ntt(xs[j], mods[:L], +1)), j
        else:
            rng = np.random.default_rng(j)
            for l in [0, L - 1]:
                for k in _sample_points(rng, 1 << ln, 2):
                    assert int(got[0, l, k]) == oracle.ntt_fwd_point(xs[j][0, l], mods[l], ln, k)
    H.ntt_batch([(d_, tables[ln], L) for d_, (ln, L) in zip(devs, jobs)], -1)
    for j in range(len(jobs)):
        assert np.array_equal(host(devs[j]), xs[j]), j


def test_views_and_levels(gpu):
    """A view on the first l moduli transforms exactly like tables built for them."""
    import paper_2109_14704_amd as H
    mods = workloads.moduli("serving")
    t = H.Tables(14, mods)
    v = t.view(5)
    rng = np.random.default_rng(9)
    x = rand_limbs(rng, (2, 5, 1 << 14), mods[:5])
    d = dev(x, gpu)
    H.ntt_fwd(v, d)
    assert np.array_equal(host(d), oracle.batch_ntt(x, mods[:5], +1))
    del t
    H.ntt_inv(v, d)
    assert np.array_equal(host(d), x)


@pytest.mark.parametrize("log_n,pairs,limbs", [(12, 16, 8), (16, 8, 6)])
def test_repeat_determinism(gpu, log_n, pairs, limbs):
    """Identical launches give identical words (every kernel shape, many workgroups)."""
    import torch
    import paper_2109_14704_amd as H
    print("case determinism log_n=%d pairs=%d limbs=%d" % (log_n, pairs, limbs), flush=True)
    mods = workloads.moduli("ct_tensor")[:limbs]
    rng = np.random.default_rng(77)
    c = rand_limbs(rng, (pairs, 2, limbs, 1 << log_n), mods)
    d = rand_limbs(rng, (pairs, 2, limbs, 1 << log_n), mods)
    t = H.Tables(log_n, mods)
    cd, dd = dev(c, gpu), dev(d, gpu)
    outs = {k: [] for k in ["coeff", "ntt", "poly", "fwd", "dyad"]}
    for _ in range(3):
        outs["coeff"].append(H.ct_tensor(t, cd, dd))
        outs["ntt"].append(H.ct_tensor(t, cd, dd, in_ntt=True, out_ntt=True))
        outs["poly"].append(H.polymul(t, cd[:, 0], dd[:, 1].contiguous()) if False else
                            H.polymul(t, cd[:, 0].contiguous(), dd[:, 1].contiguous()))
        x = cd.clone()
        outs["fwd"].append(H.ntt_fwd(t, x.view(-1, limbs, 1 << log_n)))
        outs["dyad"].append(H.dyadic_mul(t, cd, dd))
    torch.cuda.synchronize()
    for k, v in outs.items():
        assert torch.equal(v[0], v[1]) and torch.equal(v[0], v[2]), k
    # spot-check against the oracle
    got = host(outs["coeff"][0])
    q = mods[-1]
    for k in [0, 5, (1 << log_n) - 1]:
        want = (oracle.negacyclic_point(c[-1, 0, -1], d[-1, 1, -1], q, k)
                + oracle.negacyclic_point(c[-1, 1, -1], d[-1, 0, -1], q, k)) % q
        assert int(got[-1, 1, -1, k]) == want
    nt = host(outs["ntt"][0])
    assert np.array_equal(nt, oracle.batch_tensor(c, d, mods))


def _uneven_setup(gpu, njobs, seed_jobs=None):
    import paper_2109_14704_amd as H
    mods = workloads.moduli("uneven")
    jobs = seed_jobs or workloads.uneven_jobs(njobs=njobs)
    tables = {ln: H.Tables(ln, mods) for ln in sorted(set(ln for ln, _ in jobs))}
    xs = [workloads.uneven_operand(j, ln, L, mods) for j, (ln, L) in enumerate(jobs)]
    return H, mods, jobs, tables, xs


def _check_uneven(xs, got, jobs, mods, direction):
    for j, (ln, L) in enumerate(jobs):
        g = host(got[j])
        if (1 << ln) * L <= (1 << 16) * 3:
            assert np.array_equal(g, oracle.batch_ntt(xs[j], mods[:L], direction)), j
        else:
            rng = np.random.default_rng(j)
            for l in sorted({0, L - 1}):
                for k in _sample_points(rng, 1 << ln, 2):
                    f = oracle.ntt_fwd_point if direction > 0 else oracle.ntt_inv_point
                    assert int(g[0, l, k]) == f(xs[j][0, l], mods[l], ln, k), (j, l, k)


def test_batch_plan_all_sizes(gpu):
    """Persistent launch over every N in 2^12..2^17 (plus N < 2^12 fallbacks), both directions."""
    import torch
    print("case batch plan all sizes", flush=True)
    jobs = [(12, 3), (13, 2), (14, 1), (15, 2), (16, 1), (17, 2), (11, 2), (12, 1), (17, 1)]
    H, mods, jobs, tables, xs = _uneven_setup(gpu, 0, jobs)
    for direction in (+1, -1):
        devs = [dev(x, gpu) for x in xs]
        plan = H.BatchPlan([(d_, tables[ln], L) for d_, (ln, L) in zip(devs, jobs)], direction)
        # the default grid: every workgroup resident at once (four 256-lane workgroups per CU on gfx950)
        assert plan.info()["grid"] == 4 * torch.cuda.get_device_properties(0).multi_processor_count
        plan.run()
        plan.status()
        _check_uneven(xs, devs, jobs, mods, direction)
        plan.close()
        torch.cuda.synchronize()


def test_batch_graph_replays_match_eager(gpu):
    """hipGraph replays of the persistent launch equal eager runs, every replay."""
    import torch
    print("case batch graph replays", flush=True)
    H, mods, jobs, tables, xs = _uneven_setup(gpu, 40)
    devs = [dev(x, gpu) for x in xs]
    plan = H.BatchPlan([(d_, tables[ln], L) for d_, (ln, L) in zip(devs, jobs)], +1)
    plan.run()
    plan.status()
    eager = [d_.clone() for d_ in devs]
    _check_uneven(xs, eager, jobs, mods, +1)
    plan.capture()
    for rep in range(3):
        for d_, x in zip(devs, xs):
            d_.copy_(dev(x, gpu))
        torch.cuda.synchronize()
        plan.replay()
        plan.status()
        torch.cuda.synchronize()
        for a, b in zip(devs, eager):
            assert torch.equal(a, b), rep
    plan.close()


@pytest.mark.parametrize("grid,look,group", [(1, 200, 8), (7, 200, 8), (256, 200, 8), (2048, 200, 8), (1024, 0, 8),
                                             (1024, 50, 1), (512, 1000, 4096), (1024, 200, 3)])
def test_batch_grid_sizes(gpu, grid, look, group):
    """Any persistent grid size and pass-2 lookahead gives the same words
    (load balance and waits only)."""
    import torch
    print("case batch grid %d lookahead %d group %d" % (grid, look, group), flush=True)
    H, mods, jobs, tables, xs = _uneven_setup(gpu, 12)
    devs = [dev(x, gpu) for x in xs]
    plan = H.BatchPlan([(d_, tables[ln], L) for d_, (ln, L) in zip(devs, jobs)], +1)
    plan.set_grid(grid)
    plan.set_schedule(look, group)
    plan.run()
    plan.status()
    _check_uneven(xs, devs, jobs, mods, +1)
    plan.close()
