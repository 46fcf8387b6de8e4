"""GPU test of hentt_ct_tensor_noalloc, the ciphertext tensor product that
allocates nothing (its column-pass workspace is a static device array):
through the C ABI, its outputs equal hentt_ct_tensor's word for word on two
calls in a row (the second smaller, so stale scratch contents from the first
would show), in every domain combination; sizes beyond the array are
refused before anything is enqueued, and the library's pool does not grow."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _rand(rng, shape, mods):
    out = np.empty(shape, dtype=np.uint64)
    for l, q in enumerate(mods):
        out[..., l, :] = rng.integers(0, q, size=shape[:-2] + (shape[-1],), dtype=np.uint64)
    return out


def _call(L, fn, t, c, d, out, batch, flags, st):
    VP = ctypes.c_void_p
    return getattr(L, fn)(t.handle, VP(c.data_ptr()), VP(d.data_ptr()), VP(out.data_ptr()), batch, flags, st)


@pytest.mark.parametrize("log_n,limbs,batches", [(16, 24, (1, 1)), (15, 16, (4, 2)), (13, 5, (9, 3)), (12, 3, (5, 2))])
def test_ct_tensor_noalloc_matches_ct_tensor(gpu, log_n, limbs, batches):
    import torch
    import paper_2109_14704_amd as H
    print("case ct_tensor_noalloc log_n=%d limbs=%d batches=%s" % (log_n, limbs, batches), flush=True)
    L = H.lib()
    L.hentt_ct_tensor_noalloc.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
    L.hentt_ct_tensor_noalloc.restype = ctypes.c_int
    mods = workloads.moduli("serving")[:limbs]
    t = H.Tables(log_n, mods)
    n = 1 << log_n
    rng = np.random.default_rng(1000 + log_n)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for flags in (0, 1, 2, 3):
        for batch in batches:                      # second call smaller than (or as large as) the first
            c = torch.from_numpy(_rand(rng, (batch, 2, limbs, n), mods).view(np.int64)).cuda()
            d = torch.from_numpy(_rand(rng, (batch, 2, limbs, n), mods).view(np.int64)).cuda()
            want = torch.empty((batch, 3, limbs, n), dtype=torch.int64, device="cuda")
            got = torch.full_like(want, -1)
            assert _call(L, "hentt_ct_tensor", t, c, d, want, batch, flags, st) == 0
            pool_before = H.pool_bytes()
            assert _call(L, "hentt_ct_tensor_noalloc", t, c, d, got, batch, flags, st) == 0
            assert H.pool_bytes() == pool_before
            torch.cuda.synchronize()
            assert torch.equal(got, want), (flags, batch)


def test_ct_tensor_noalloc_refuses_oversize(gpu):
    import torch
    import paper_2109_14704_amd as H
    print("case ct_tensor_noalloc oversize", flush=True)
    L = H.lib()
    L.hentt_ct_tensor_noalloc.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
    mods = workloads.moduli("serving")
    t = H.Tables(16, mods)
    c = torch.zeros((2, 2, 24, 1 << 16), dtype=torch.int64, device="cuda")
    d = torch.zeros_like(c)
    out = torch.full((2, 3, 24, 1 << 16), 7, dtype=torch.int64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert _call(L, "hentt_ct_tensor_noalloc", t, c, d, out, 2, 0, st) == -8      # 4*2*24*2^16 > 2^23 words
    torch.cuda.synchronize()
    assert int(out.min()) == 7 and int(out.max()) == 7                            # nothing was enqueued
    # NTT-domain inputs need no workspace: any size is accepted
    assert _call(L, "hentt_ct_tensor_noalloc", t, c, d, out, 2, 3, st) == 0
    torch.cuda.synchronize()
    assert int(out.abs().max()) == 0
