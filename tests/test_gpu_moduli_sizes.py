"""GPU parity across modulus sizes.  The canonical reduction of forward
outputs (and the reduction ahead of the Montgomery products) takes a quotient
estimate for moduli above 2^33 and a chain of conditional subtractions below;
this chain holds NTT primes of 20 to 60 bits, both bit lengths at the switch
(33 and 34) included, and 55 and 56 bits, the largest sizes at which the fused
products skip that reduction (the tensor up to 55, the polymul up to 56 bits),
so every kernel family that reduces forward outputs --
the two-pass and whole-block transforms, the persistent batch, the fused
products, rescale -- is compared with the oracle on both sides of it, with
operands at q - 1 as well as uniform ones (and the grouped tensor, whose jobs
take different paths within one launch)."""
import numpy as np
import pytest

import oracle

BITS = [20, 30, 33, 34, 35, 45, 55, 56, 60]


def _chain():
    out = []
    for b in BITS:
        out += oracle.gen_primes(b, 1 << 18, 1, exclude=out)   # q = 1 mod 2^18: every N <= 2^17
    return out


MODS = _chain()


def dev(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(device)


def host(t):
    return t.cpu().numpy().view(np.uint64)


def operands(rng, shape, mods):
    """Uniform words, with every third word of each limb at q - 1."""
    out = np.empty(shape, dtype=np.uint64)
    for l, q in enumerate(mods):
        sl = rng.integers(0, q, size=shape[:-2] + (shape[-1],), dtype=np.uint64)
        sl[..., ::3] = q - 1
        out[..., l, :] = sl
    return out


def test_chain_spans_the_switch():
    """The chain itself (CPU): prime, NTT-friendly for N <= 2^17, one prime per size."""
    assert [q.bit_length() for q in MODS] == BITS
    assert all(oracle.is_prime(q) and q % (1 << 18) == 1 for q in MODS)


@pytest.mark.gpu
@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16, 17])
def test_fwd_inv_all_sizes_of_q(gpu, log_n):
    import paper_2109_14704_amd as H
    print("case moduli sizes fwd/inv log_n=%d" % log_n, flush=True)
    rng = np.random.default_rng(7000 + log_n)
    t = H.Tables(log_n, MODS)
    x = operands(rng, (2, len(MODS), 1 << log_n), MODS)
    d = dev(x, gpu)
    H.ntt_fwd(t, d)
    assert np.array_equal(host(d), oracle.batch_ntt(x, MODS, +1))
    H.ntt_inv(t, d)
    assert np.array_equal(host(d), x)


@pytest.mark.gpu
@pytest.mark.parametrize("log_n", [12, 14, 15, 16])
def test_products_all_sizes_of_q(gpu, log_n):
    """Fused polymul (Montgomery path), NTT-domain output of the tensor (the
    exact forward reduction inside the fused kernel) and the full tensor."""
    import paper_2109_14704_amd as H
    print("case moduli sizes products log_n=%d" % log_n, flush=True)
    rng = np.random.default_rng(7100 + log_n)
    t = H.Tables(log_n, MODS)
    L = len(MODS)
    a = operands(rng, (1, L, 1 << log_n), MODS)
    b = operands(rng, (1, L, 1 << log_n), MODS)
    assert np.array_equal(host(H.polymul(t, dev(a, gpu), dev(b, gpu))), oracle.batch_polymul(a, b, MODS))
    c = operands(rng, (1, 2, L, 1 << log_n), MODS)
    e = operands(rng, (1, 2, L, 1 << log_n), MODS)
    T = oracle.batch_tensor(oracle.batch_ntt(c, MODS, +1), oracle.batch_ntt(e, MODS, +1), MODS)
    assert np.array_equal(host(H.ct_tensor(t, dev(c, gpu), dev(e, gpu), out_ntt=True)), T)
    assert np.array_equal(host(H.ct_tensor(t, dev(c, gpu), dev(e, gpu))), oracle.batch_ntt(T, MODS, -1))


@pytest.mark.gpu
def test_uneven_batch_all_sizes_of_q(gpu):
    """The persistent batch kernel: one job per N = 2^12 .. 2^17 over the chain."""
    import paper_2109_14704_amd as H
    print("case moduli sizes uneven batch", flush=True)
    rng = np.random.default_rng(7200)
    tables = {ln: H.Tables(ln, MODS) for ln in range(12, 18)}
    xs = [operands(rng, (1, len(MODS), 1 << ln), MODS) for ln in range(12, 18)]
    devs = [dev(x, gpu) for x in xs]
    jobs = [(d, tables[ln], len(MODS)) for d, ln in zip(devs, range(12, 18))]
    H.ntt_batch(jobs, +1)
    H.ntt_batch_status(jobs, +1)                 # raises if a tile gave up waiting
    for x, d in zip(xs, devs):
        assert np.array_equal(host(d), oracle.batch_ntt(x, MODS, +1))
    H.ntt_batch(jobs, -1)
    for x, d in zip(xs, devs):
        assert np.array_equal(host(d), x)


@pytest.mark.gpu
@pytest.mark.parametrize("log_n", [12, 15, 16])
def test_rescale_all_sizes_of_q(gpu, log_n):
    import paper_2109_14704_amd as H
    print("case moduli sizes rescale log_n=%d" % log_n, flush=True)
    rng = np.random.default_rng(7300 + log_n)
    t = H.Tables(log_n, MODS)
    x = operands(rng, (2, len(MODS), 1 << log_n), MODS)
    assert np.array_equal(host(H.rescale(t, dev(x, gpu))), oracle.batch_rescale(x, MODS))
    X = oracle.batch_ntt(x, MODS, +1)
    assert np.array_equal(host(H.rescale(t, dev(X, gpu), ntt=True)), oracle.batch_rescale_ntt(X, MODS))


@pytest.mark.gpu
def test_grouped_tensor_all_sizes_of_q(gpu):
    """The grouped tensor with jobs whose limbs take different reduction paths
    in one launch (levels 2..9 of the chain at three ring dimensions)."""
    import torch
    import paper_2109_14704_amd as H
    print("case moduli sizes grouped tensor", flush=True)
    rng = np.random.default_rng(7400)
    tabs = {ln: H.Tables(ln, MODS) for ln in (13, 14, 15)}
    spec = [(13, 9), (14, 3), (15, 6), (14, 9), (13, 2), (15, 9)]
    args, want = [], []
    for ln, lvl in spec:
        mods = MODS[:lvl]
        c = operands(rng, (1, 2, lvl, 1 << ln), mods)
        d = operands(rng, (1, 2, lvl, 1 << ln), mods)
        out = torch.full((1, 3, lvl, 1 << ln), -1, dtype=torch.int64, device=gpu)
        args.append((tabs[ln].view(lvl), dev(c, gpu), dev(d, gpu), out))
        want.append(oracle.batch_ct_tensor_coeff(c, d, mods))
    H.ct_tensor_grouped(args)
    torch.cuda.synchronize()
    for (ln, lvl), (_, _, _, out), w in zip(spec, args, want):
        assert np.array_equal(host(out), w), (ln, lvl)
