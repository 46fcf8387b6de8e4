"""GPU test of the serving path: requests of mixed N and level served with
continuous batching give, word for word, the result of the same request run
alone, and agree with the oracle on sampled coefficients."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def test_served_results_match_alone_and_oracle(gpu):
    import torch
    import paper_2109_14704_amd as H
    from paper_2109_14704_amd import serve
    print("case serving mix", flush=True)
    chain = workloads.moduli("serving")
    budget = serve.footprint(16, 12) * 6
    be = serve.HipBackend(chain, streams=2, verify=True, budget_bytes=budget)
    trace = workloads.serving_trace(36, rate_per_s=3000.0, seed_stream=7)
    reqs, host_ops = [], {}
    for i, (t, ln, lvl) in enumerate(trace):
        lvl = 4 + lvl % 9                      # keep the test small: levels 4..12
        c, d = workloads.serving_operands(i, ln, lvl, chain)
        host_ops[i] = (c, d)
        reqs.append(serve.Request(i, t, ln, lvl, torch.from_numpy(c.view(np.int64)).cuda(),
                                  torch.from_numpy(d.view(np.int64)).cuda()))
    sched = serve.Scheduler(be, budget_bytes=budget, streams=2)
    sched.run_trace(reqs)
    torch.cuda.synchronize()
    assert all(r.state == "done" for r in reqs), [(r.rid, r.state, r.error) for r in reqs if r.state != "done"]
    assert sched.steps >= 2 and sched.reserved == 0
    # outputs + library workspace within their shares (7/11) of the budget; the operands are the client's
    assert 0 < be.peak_held <= budget * (serve.OUTPUT_POLYS + serve.WORKSPACE_POLYS) // 11, (be.peak_held, budget)
    for r in reqs:
        alone = H.ct_tensor(be.view(r.log_n, r.level), r.c, r.d)
        assert torch.equal(alone, r.result), r.rid
    rng = np.random.default_rng(3)
    for r in reqs[:4]:
        c, d = host_ops[r.rid]
        got = r.result.cpu().numpy().view(np.uint64)
        l = int(rng.integers(0, r.level))
        q = chain[l]
        k = int(rng.integers(0, 1 << r.log_n))
        want = (oracle.negacyclic_point(c[0, 0, l], d[0, 1, l], q, k)
                + oracle.negacyclic_point(c[0, 1, l], d[0, 0, l], q, k)) % q
        assert int(got[0, 1, l, k]) == want


@pytest.mark.parametrize("log_n", [14, 15])
@pytest.mark.parametrize("level", [13, 19, 24])
def test_ct_tensor_high_levels(gpu, log_n, level):
    """The serving product at levels 13..24 of the serving chain (level views
    of one 24-prime table), element by element against the oracle."""
    import paper_2109_14704_amd as H
    print("case ct_tensor level=%d log_n=%d" % (level, log_n), flush=True)
    chain = workloads.moduli("serving")
    t = H.Tables(log_n, chain)
    v = t.view(level)
    c, d = workloads.serving_operands(900 + level, log_n, level, chain)
    import torch
    got = H.ct_tensor(v, torch.from_numpy(c.view(np.int64)).cuda(), torch.from_numpy(d.view(np.int64)).cuda())
    mods = chain[:level]
    want = oracle.batch_ct_tensor_coeff(c, d, mods)
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)


def test_served_mix_all_levels(gpu):
    """The serving workload's full level range (4..24) and sizes (2^14..2^16):
    every served result equals the same request run alone."""
    import torch
    import paper_2109_14704_amd as H
    from paper_2109_14704_amd import serve
    print("case serving mix, all levels", flush=True)
    chain = workloads.moduli("serving")
    budget = serve.footprint(16, 24) * 8
    be = serve.HipBackend(chain, streams=2, verify=True, budget_bytes=budget)
    trace = workloads.serving_trace(48, rate_per_s=5000.0, seed_stream=9)
    reqs = []
    for i, (t, ln, lvl) in enumerate(trace):
        c, d = workloads.serving_operands(2000 + i, ln, lvl, chain)
        reqs.append(serve.Request(i, t, ln, lvl, torch.from_numpy(c.view(np.int64)).cuda(),
                                  torch.from_numpy(d.view(np.int64)).cuda()))
    assert max(r.level for r in reqs) >= 20 and min(r.level for r in reqs) <= 8
    sched = serve.Scheduler(be, budget_bytes=budget, streams=2)
    sched.run_trace(reqs)
    torch.cuda.synchronize()
    assert all(r.state == "done" for r in reqs), [(r.rid, r.state, r.error) for r in reqs if r.state != "done"]
    assert 0 < be.peak_held <= budget * (serve.OUTPUT_POLYS + serve.WORKSPACE_POLYS) // 11, (be.peak_held, budget)
    for r in reqs:
        alone = H.ct_tensor(be.view(r.log_n, r.level), r.c, r.d)
        assert torch.equal(alone, r.result), r.rid
