"""GPU tests of the autotuner's search space (section III-B's tuning
constants: stage split and words per lane): every compiled kernel instance
of every tunable operation gives the oracle's result word for word, and the
autotuner's choice is gated by an oracle check of the default instance."""
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


@pytest.mark.parametrize("op", ["fwd", "inv", "polymul", "tensor"])
@pytest.mark.parametrize("log_n", [13, 14, 15, 16, 17])
def test_every_instance_matches_oracle(gpu, op, log_n):
    import paper_2109_14704_amd as H
    print("case tuned instances op=%s log_n=%d" % (op, log_n), flush=True)
    batch, limbs = 2, 3
    mods = CHAIN[:limbs]
    t = H.Tables(log_n, mods)
    rng = np.random.default_rng(7000 + 10 * log_n + H.TUNE_OPS[op])
    n = 1 << log_n
    cls = H.shape_class(batch * limbs)
    if op in ("fwd", "inv"):
        x = rand_limbs(rng, (batch, limbs, n), mods)
        want = oracle.batch_ntt(x, mods, +1 if op == "fwd" else -1)
    elif op == "polymul":
        a, b = rand_limbs(rng, (batch, limbs, n), mods), rand_limbs(rng, (batch, limbs, n), mods)
        want = oracle.batch_polymul(a, b, mods)
    else:
        c, d = rand_limbs(rng, (batch, 2, limbs, n), mods), rand_limbs(rng, (batch, 2, limbs, n), mods)
        want = oracle.batch_ct_tensor_coeff(c, d, mods)
    count = H.tune_count(op, log_n)
    assert count >= 2
    try:
        for i in range(count):
            H.tune_select(op, log_n, cls, i)
            assert H.tune_get(op, log_n, cls) == i
            if op == "fwd":
                got = H.ntt_fwd(t, dev(x, gpu))
            elif op == "inv":
                got = H.ntt_inv(t, dev(x, gpu))
            elif op == "polymul":
                got = H.polymul(t, dev(a, gpu), dev(b, gpu))
            else:
                got = H.ct_tensor(t, dev(c, gpu), dev(d, gpu))
            assert np.array_equal(host(got), want), (op, log_n, i, H.tune_describe(op, log_n, i))
    finally:
        H.tune_select(op, log_n, cls, 0)


def test_autotuner_gates_on_the_oracle(gpu, tmp_path, monkeypatch):
    """kernel_config times only instances equal to the oracle-checked default,
    caches its choice, and a default that fails the check raises."""
    import json
    import torch
    import paper_2109_14704_amd as H
    from paper_2109_14704_amd import autotune
    print("case autotune kernel config", flush=True)
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("HENTT_TUNE_CACHE", str(cache))
    log_n, batch, limbs = 15, 8, 4
    mods = CHAIN[:limbs]
    t = H.Tables(log_n, mods)
    rng = np.random.default_rng(4242)
    a, b = rand_limbs(rng, (batch, limbs, 1 << log_n), mods), rand_limbs(rng, (batch, limbs, 1 << log_n), mods)
    want = oracle.batch_polymul(a, b, mods)
    A, B = dev(a, gpu), dev(b, gpu)
    out = torch.empty_like(A)
    cls = H.shape_class(batch * limbs)
    try:
        desc = autotune.kernel_config("polymul", t, lambda: H.polymul(t, A, B, out=out), [out], batch * limbs,
                                      check=lambda outs: np.array_equal(host(outs[0]), want))
        choice = H.tune_get("polymul", log_n, cls)
        assert desc == H.tune_describe("polymul", log_n, choice)
        H.polymul(t, A, B, out=out)
        assert np.array_equal(host(out), want)
        ent = [v for k, v in json.loads(cache.read_text()).items() if k.startswith("kernel/")]
        assert len(ent) == 1 and ent[0]["choice"] == choice and len(ent[0]["ms"]) == H.tune_count("polymul", log_n)
        with pytest.raises(autotune.ParityError):
            autotune.kernel_config("polymul", t, lambda: H.polymul(t, A, B, out=out), [out], batch * limbs,
                                   check=lambda outs: False, force=True)
    finally:
        H.tune_select("polymul", log_n, cls, 0)
