"""GPU tests of the C ABI's contracts beyond the arithmetic: the canonical-input
check, refusals of forbidden overlaps, the batch-plan cache's lifetime rules
(references on tables, eviction on destroy), plans with live graphs, and
status after graph replays.  All calls go through the C ABI."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

CHAIN = workloads.moduli("uneven")


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


@pytest.mark.parametrize("log_n", [6, 12, 16])
def test_check_canonical(gpu, log_n):
    import torch
    import paper_2109_14704_amd as H
    print("case check_canonical log_n=%d" % log_n, flush=True)
    mods = CHAIN[:3]
    t = H.Tables(log_n, mods)
    rng = np.random.default_rng(11 + log_n)
    x = rand_limbs(rng, (2, 3, 1 << log_n), mods)
    x[1, 2, -1] = mods[2] - 1                 # largest canonical value
    d = dev(x, gpu)
    H.check_canonical(t, d)                   # all canonical: no error
    n = 1 << log_n
    bad = [(1, 2, n - 1, mods[2]), (0, 1, 5 % n, (1 << 64) - 1), (1, 0, 0, mods[0] + 7)]
    for b, l, i, v in bad:
        x[b, l, i] = v
    d = dev(x, gpu)
    with pytest.raises(H.NonCanonicalError) as ei:
        H.check_canonical(t, d)
    flat = sorted((b * 3 + l) * n + i for b, l, i, _ in bad)
    assert "%d words" % len(bad) in str(ei.value)
    assert ("flat index %d" % flat[0]) in str(ei.value)
    # raw C ABI: counts and first index
    L = H.lib()
    cnt, first = ctypes.c_uint64(), ctypes.c_uint64()
    rc = L.hentt_check_canonical(t.handle, ctypes.c_void_p(d.data_ptr()), 2, ctypes.byref(cnt), ctypes.byref(first),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -7 and cnt.value == len(bad) and first.value == flat[0]


def test_overlap_refusals(gpu):
    import torch
    import paper_2109_14704_amd as H
    print("case overlap refusals", flush=True)
    mods = CHAIN[:2]
    log_n = 13
    n = 1 << log_n
    t = H.Tables(log_n, mods)
    rng = np.random.default_rng(5)
    a = rand_limbs(rng, (2, 2, n), mods)
    b = rand_limbs(rng, (2, 2, n), mods)
    big = dev(np.concatenate([a, b, a]), gpu)          # [6][2][n] arena
    A, B = big[0:2], big[2:4]
    # polymul: the output may not touch an input
    with pytest.raises(H.HenttError):
        H.polymul(t, A, B, out=big[1:3])
    with pytest.raises(H.HenttError):
        H.polymul(t, A, B, out=A)
    # dyadic_mul: exact aliasing allowed, partial overlap refused
    want = oracle.batch_dyadic(a, b, mods)
    A2 = A.clone()
    H.dyadic_mul(t, A2, B, out=A2)
    assert np.array_equal(host(A2), want)
    with pytest.raises(H.HenttError):
        H.dyadic_mul(t, A, B, out=big[1:3])
    # ct_tensor: out [1][3][2][n] may not overlap c or d
    c = big[0:2].view(1, 2, 2, n)
    d_ = big[2:4].view(1, 2, 2, n)
    arena = torch.zeros((5, 2, n), dtype=torch.int64, device=gpu)
    arena[0:2].copy_(big[0:2])
    c2 = arena[0:2].view(1, 2, 2, n)
    with pytest.raises(H.HenttError):
        H.ct_tensor(t, c2, d_, out=arena[1:4].view(1, 3, 2, n))
    out = H.ct_tensor(t, c, d_)
    assert out.shape == (1, 3, 2, n)
    torch.cuda.synchronize()


def test_plan_cache_survives_table_destroy_and_reuse(gpu):
    """hentt_ntt_batch caches plans; destroying a table handle evicts the plans
    of its storage, and new job lists at possibly reused addresses transform
    correctly."""
    import gc
    import torch
    import paper_2109_14704_amd as H
    print("case plan cache lifetime", flush=True)
    rng = np.random.default_rng(21)
    for rnd, (ln, L) in enumerate([(13, 2), (14, 3), (13, 2), (12, 4)]):
        t = H.Tables(ln, CHAIN[:4])
        v = t.view(L)
        x = rand_limbs(rng, (1, L, 1 << ln), CHAIN[:L])
        d = dev(x, gpu)
        H.ntt_batch([(d, v, L)], +1)
        H.ntt_batch_status([(d, t, L)], +1)            # same storage, data, shape: the same cached plan
        assert np.array_equal(host(d), oracle.batch_ntt(x, CHAIN[:L], +1)), rnd
        H.ntt_batch([(d, v, L)], -1)
        H.ntt_batch_status([(d, v, L)], -1)
        assert np.array_equal(host(d), x), rnd
        torch.cuda.synchronize()
        v.close()                                      # evicts the cached plans of this storage
        with pytest.raises(H.HenttError):
            H.ntt_batch_status([(d, t, L)], +1)
        H.ntt_batch([(d, t, L)], +1)                   # a fresh plan on the surviving handle
        assert np.array_equal(host(d), oracle.batch_ntt(x, CHAIN[:L], +1)), rnd
        torch.cuda.synchronize()
        t.close()
        del d
        gc.collect()


def test_plan_with_live_graph_refuses_regrid(gpu):
    import torch
    import paper_2109_14704_amd as H
    print("case live graph refusals", flush=True)
    t = H.Tables(15, CHAIN[:2])
    rng = np.random.default_rng(8)
    x = rand_limbs(rng, (1, 2, 1 << 15), CHAIN[:2])
    d = dev(x, gpu)
    plan = H.BatchPlan([(d, t, 2)], +1)
    plan.capture()
    L = H.lib()
    assert L.hentt_batch_plan_set_grid(plan._h, 64) == -6          # HENTT_EBUSY: a graph holds the old shape
    assert L.hentt_batch_plan_destroy(plan._h) == -6
    plan.replay()
    plan.status()                                                   # waits for the replay
    assert np.array_equal(host(d), oracle.batch_ntt(x, CHAIN[:2], +1))
    plan.set_grid(64)                                               # drops the graph first
    d.copy_(dev(x, gpu))
    plan.run()
    plan.status()
    assert np.array_equal(host(d), oracle.batch_ntt(x, CHAIN[:2], +1))
    plan.close()
    torch.cuda.synchronize()


def test_pool_trim_releases_idle_workspace(gpu):
    import torch
    import paper_2109_14704_amd as H
    print("case pool trim", flush=True)
    t = H.Tables(15, CHAIN[:2])
    rng = np.random.default_rng(4)
    a = dev(rand_limbs(rng, (2, 2, 1 << 15), CHAIN[:2]), gpu)
    b = dev(rand_limbs(rng, (2, 2, 1 << 15), CHAIN[:2]), gpu)
    p1 = H.polymul(t, a, b)
    assert H.pool_bytes() >= 2 * a.numel() * 8        # the forward column pass's workspace
    torch.cuda.synchronize()
    H.pool_trim()
    assert H.pool_bytes() == 0
    p2 = H.polymul(t, a, b)                            # allocates again
    assert torch.equal(p1, p2)
    torch.cuda.synchronize()


def test_pool_soft_cap_from_environment(gpu):
    """HENTT_POOL_MAX_BYTES (read once per process, so in a child process):
    two polymuls on two streams leave two 8 MiB workspaces in the pool
    without a cap, and one with a 12 MiB cap (the idle buffer is trimmed
    before the second allocation)."""
    import os
    import subprocess
    import sys
    print("case pool soft cap", flush=True)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "import torch, workloads, paper_2109_14704_amd as H\n"
        "t = H.Tables(15, workloads.moduli('ckks_level')[:4])\n"
        "A = torch.zeros((4, 4, 1 << 15), dtype=torch.int64, device='cuda:0')\n"
        "s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()\n"
        "H.polymul(t, A, A, stream=s1); torch.cuda.synchronize(); b1 = H.pool_bytes()\n"
        "H.polymul(t, A, A, stream=s2); torch.cuda.synchronize(); b2 = H.pool_bytes()\n"
        "print(b1, b2)\n" % (root, os.path.join(root, "tests")))
    ws = 2 * 4 * 4 * (1 << 15) * 8          # two inputs after the forward column pass
    got = {}
    for cap in (None, ws * 3 // 2):
        env = dict(os.environ)
        env.pop("HENTT_POOL_MAX_BYTES", None)
        if cap:
            env["HENTT_POOL_MAX_BYTES"] = str(cap)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        got[cap] = [int(v) for v in r.stdout.split()[-2:]]
    assert got[None] == [ws, 2 * ws], got
    assert got[ws * 3 // 2] == [ws, ws], got
