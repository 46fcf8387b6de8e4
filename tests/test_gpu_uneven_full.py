"""GPU parity of the uneven-batch workload at its full size: all 512 jobs
(N from 2^12 to 2^17, 1 to 32 limbs, about 3.6e8 coefficients), forward
and inverse, compared word for word with the CPU oracle:

  * through hentt_ntt_batch (the cached-plan path), with its status read;
  * through an explicit plan at the autotuned grid, captured into a hipGraph
    and replayed, with the plan status read after every replay;
  * the autotuner's default grid is checked against the oracle before any
    candidate is timed (parity gate).

The persistent kernel orders pass-2 tiles after their pass-1 tiles through
per-unit counters in the L2 of the XCD that runs both passes; this is the
configuration with the most pass-2 waits and workgroups per queue.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def dev(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(device)


@pytest.fixture(scope="module")
def full_uneven():
    mods = workloads.moduli("uneven")
    jobs = workloads.uneven_jobs()
    print("case uneven 512 jobs: drawing inputs", flush=True)
    xs = [workloads.uneven_operand(j, ln, L, mods) for j, (ln, L) in enumerate(jobs)]
    print("case uneven 512 jobs: oracle forward", flush=True)
    fw = [oracle.batch_ntt(x, mods[:L], +1) for x, (ln, L) in zip(xs, jobs)]
    return mods, jobs, xs, fw


def _equal_all(devs, want):
    import torch
    for j, (d_, w) in enumerate(zip(devs, want)):
        if not torch.equal(d_, dev(w, d_.device)):
            return j
    return None


@pytest.mark.timeout(900)
def test_uneven_512_jobs_ntt_batch(gpu, full_uneven):
    import torch
    import paper_2109_14704_amd as H
    mods, jobs, xs, fw = full_uneven
    assert len(jobs) == 512
    tables = {ln: H.Tables(ln, mods) for ln in sorted(set(ln for ln, _ in jobs))}
    devs = [dev(x, gpu) for x in xs]
    spec = [(d_, tables[ln], L) for d_, (ln, L) in zip(devs, jobs)]
    print("case uneven 512 jobs: ntt_batch forward", flush=True)
    H.ntt_batch(spec, +1)
    H.ntt_batch_status(spec, +1)
    assert _equal_all(devs, fw) is None
    print("case uneven 512 jobs: ntt_batch inverse", flush=True)
    H.ntt_batch(spec, -1)
    H.ntt_batch_status(spec, -1)
    assert _equal_all(devs, xs) is None
    # the cached plans run again on the same job list
    H.ntt_batch(spec, +1)
    H.ntt_batch(spec, -1)
    H.ntt_batch_status(spec, -1)
    assert _equal_all(devs, xs) is None
    torch.cuda.synchronize()


@pytest.mark.timeout(900)
def test_uneven_512_jobs_tuned_graph_replay(gpu, full_uneven, tmp_path, monkeypatch):
    import torch
    import paper_2109_14704_amd as H
    from paper_2109_14704_amd import autotune
    monkeypatch.setenv("HENTT_TUNE_CACHE", str(tmp_path / "tune.json"))   # tune afresh, gated by the oracle
    mods, jobs, xs, fw = full_uneven
    tables = {ln: H.Tables(ln, mods) for ln in sorted(set(ln for ln, _ in jobs))}
    devs = [dev(x, gpu) for x in xs]
    spec = [(d_, tables[ln], L) for d_, (ln, L) in zip(devs, jobs)]
    plan_f, plan_i = H.BatchPlan(spec, +1), H.BatchPlan(spec, -1)
    print("case uneven 512 jobs: autotuning the persistent grid", flush=True)
    grid, look, group = autotune.persistent_grid(plan_f, devs, check=lambda outs: _equal_all(outs, fw) is None)
    assert grid > 0 and plan_f.info()["grid"] == grid
    assert _equal_all(devs, xs) is None          # the tuner restored the inputs
    # the inverse tunes on its own (its own cache entry), gated by the round trip
    print("case uneven 512 jobs: autotuning the inverse plan", flush=True)
    for d_, w in zip(devs, fw):
        d_.copy_(dev(w, d_.device))
    grid_i, look_i, group_i = autotune.persistent_grid(plan_i, devs, check=lambda outs: _equal_all(outs, xs) is None)
    assert grid_i > 0 and plan_i.info()["grid"] == grid_i
    assert _equal_all(devs, fw) is None
    for d_, w in zip(devs, xs):
        d_.copy_(dev(w, d_.device))
    plan_f.capture()
    plan_i.capture()
    for rep in range(2):
        print("case uneven 512 jobs: graph replay %d at (%d, %d%%, %d) forward, (%d, %d%%, %d) inverse"
              % (rep, grid, look, group, grid_i, look_i, group_i), flush=True)
        plan_f.replay()
        plan_f.status()
        assert _equal_all(devs, fw) is None, rep
        plan_i.replay()
        plan_i.status()
        assert _equal_all(devs, xs) is None, rep
    plan_f.close()
    plan_i.close()
    torch.cuda.synchronize()
