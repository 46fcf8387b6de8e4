"""GPU parity of the grouped ciphertext tensor (hentt_ct_tensor_grouped):
jobs of mixed ring dimension, level and batch, more jobs of one N than one
launch sequence takes, every domain form; each job's output is compared word
for word with the CPU oracle and with the single-job product."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

CHAIN = workloads.moduli("serving")      # q = 1 mod 2^17: valid for every N here


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


def _jobs(rng, spec):
    """spec: (log_n, level, batch) per job -> host operands."""
    return [(ln, lvl, rand_limbs(rng, (b, 2, lvl, 1 << ln), CHAIN[:lvl]), rand_limbs(rng, (b, 2, lvl, 1 << ln),
                                                                                     CHAIN[:lvl]))
            for ln, lvl, b in spec]


def _run(gpu, jobs, in_ntt=False, out_ntt=False):
    import torch
    import paper_2109_14704_amd as H
    tabs = {}
    args, outs = [], []
    for ln, lvl, c, d in jobs:
        if ln not in tabs:
            tabs[ln] = H.Tables(ln, CHAIN[:8])
        t = tabs[ln].view(lvl)
        cd, dd = dev(c, gpu), dev(d, gpu)
        out = torch.full((c.shape[0], 3, lvl, 1 << ln), -1, dtype=torch.int64, device=gpu)
        args.append((t, cd, dd, out))
        outs.append(out)
    H.ct_tensor_grouped(args, in_ntt=in_ntt, out_ntt=out_ntt)
    torch.cuda.synchronize()
    return args, outs


def test_grouped_mixed_levels_and_sizes(gpu):
    """30 jobs at N = 2^14 (two launch sequences), jobs at 2^12, 2^13, 2^15 and
    2^16, levels 1..8, batch 1..3: oracle and single-job results."""
    import paper_2109_14704_amd as H
    print("case grouped ct_tensor mixed", flush=True)
    rng = np.random.default_rng(9100)
    spec = [(14, int(rng.integers(1, 9)), int(rng.integers(1, 3))) for _ in range(30)]
    spec += [(12, 3, 2), (13, 8, 1), (15, 5, 1), (16, 2, 3), (13, 1, 1), (15, 8, 2)]
    order = rng.permutation(len(spec))
    spec = [spec[i] for i in order]
    jobs = _jobs(rng, spec)
    args, outs = _run(gpu, jobs)
    for (ln, lvl, c, d), (t, cd, dd, _), out in zip(jobs, args, outs):
        want = oracle.batch_ct_tensor_coeff(c, d, CHAIN[:lvl])
        got = host(out)
        assert np.array_equal(got, want), (ln, lvl, c.shape[0])
        assert np.array_equal(host(H.ct_tensor(t, cd, dd)), got)
        assert np.array_equal(host(cd), c) and np.array_equal(host(dd), d)    # inputs untouched


@pytest.mark.parametrize("in_ntt,out_ntt", [(True, False), (False, True), (True, True)])
def test_grouped_domain_forms(gpu, in_ntt, out_ntt):
    print("case grouped ct_tensor in_ntt=%s out_ntt=%s" % (in_ntt, out_ntt), flush=True)
    rng = np.random.default_rng(9200 + 2 * in_ntt + out_ntt)
    spec = [(12, 2, 1), (13, 3, 2), (14, 1, 1), (15, 4, 1), (15, 2, 2), (16, 3, 1)]
    raw = _jobs(rng, spec)
    jobs = []
    for ln, lvl, c, d in raw:
        if in_ntt:
            c, d = oracle.batch_ntt(c, CHAIN[:lvl], +1), oracle.batch_ntt(d, CHAIN[:lvl], +1)
        jobs.append((ln, lvl, c, d))
    _, outs = _run(gpu, jobs, in_ntt=in_ntt, out_ntt=out_ntt)
    for (ln, lvl, c, d), (_, _, c0, d0), out in zip(jobs, raw, outs):
        mods = CHAIN[:lvl]
        T = oracle.batch_tensor(oracle.batch_ntt(c0, mods, +1), oracle.batch_ntt(d0, mods, +1), mods)
        want = T if out_ntt else oracle.batch_ntt(T, mods, -1)
        assert np.array_equal(host(out), want), (ln, lvl)


def test_grouped_empty_and_errors(gpu):
    import torch
    import paper_2109_14704_amd as H
    print("case grouped ct_tensor errors", flush=True)
    H.ct_tensor_grouped([])                             # nothing to do
    t = H.Tables(13, CHAIN[:2])
    P = 2 << 13                                          # words of one polynomial at 2 limbs
    rng = np.random.default_rng(9300)
    buf = dev(rand_limbs(rng, (6, 2, 1 << 13), CHAIN[:2]), gpu).view(-1)
    c = buf[: 4 * P].view(2, 2, 2, 1 << 13)              # job A's c: polynomials 0..3 of buf
    d = dev(rand_limbs(rng, (2, 2, 2, 1 << 13), CHAIN[:2]), gpu)
    out = torch.zeros((2, 3, 2, 1 << 13), dtype=torch.int64, device=gpu)
    out_b = buf[2 * P: 5 * P].view(1, 3, 2, 1 << 13)     # job B's out: polynomials 2..4 of buf
    keep_buf, keep_out = buf.clone(), out.clone()
    # job B's output over job A's input (job B's own inputs are clear of it)
    with pytest.raises(H.HenttError):
        H.ct_tensor_grouped([(t, c, d, out), (t, c[:1], d[:1], out_b)])
    # two outputs over each other
    with pytest.raises(H.HenttError):
        H.ct_tensor_grouped([(t, c[:1], d[:1], out[:1]), (t, c[1:], d[1:], out[:1])])
    torch.cuda.synchronize()
    assert torch.equal(buf, keep_buf) and torch.equal(out, keep_out)   # rejected before any launch
