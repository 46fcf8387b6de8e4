"""Benchmark of the batched negacyclic NTT path on one MI355X.

Default workload (CKKS-level batch): N = 2^15, 16 RNS primes of 50-60 bits,
64 ciphertexts x 2 polynomials = 128 polynomials per operand; one step is the
whole path -- forward NTT of A and B, dyadic product, inverse NTT -- run as
the library's fused polymul.  Inputs are resident in HBM before timing.

Prints ONE JSON line: Gcoeff/s (B*L*N coefficients per transform, three
transforms per step), the roofline of the dominant kernel (HIP-event timed on
the launching stream), the per-polynomial-launch comparator, and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NTT Gcoeff/s & % HBM/int-mul roofline, batched vs per-poly; p50/p99 ct-mul"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed steps; the clocks settle after about 20 steps of the default workload")
    ap.add_argument("--workload", default="ckks_level",
                    choices=["ckks_level", "ct_tensor", "plain4096", "uneven", "serving", "ladder", "rescale",
                             "matmul", "routines"])
    ap.add_argument("--requests", type=int, default=2200, help="serving: requests per trace (first 200 warm up)")
    ap.add_argument("--grid", type=int, default=0, help="persistent workgroups for the uneven batch (0 = tuned/default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-per-poly", action="store_true", help="skip the per-polynomial comparator")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work for the oracle sample")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def to_dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda:0")


def _tuned_grid(plan, grid_arg, data=None):
    if grid_arg:
        return grid_arg
    from paper_2109_14704_amd import autotune
    return autotune.persistent_grid(plan, data=data)


def setup(name, torch, H, grid_arg=0):
    """Device-resident operands and the step function for a workload."""
    import workloads
    if name == "ckks_level":
        w = workloads.ckks_level()
        t = H.Tables(w["log_n"], w["moduli"])
        A, B = to_dev(w["a"], torch), to_dev(w["b"], torch)
        out = torch.empty_like(A)
        polys, L, n = A.shape[0], A.shape[1], A.shape[2]

        def step():
            H.polymul(t, A, B, out=out)

        def per_poly_step():
            for i in range(polys):
                H.polymul(t, A[i:i + 1], B[i:i + 1], out=out[i:i + 1])

        info = {"workload": "ckks_level", "N": n, "limbs": L, "polys_per_operand": polys,
                "ops": "fwd(A), fwd(B), dyadic, inv (fused polymul)"}
        return dict(step=step, per_poly=per_poly_step, coeffs=3 * polys * L * n, t=t, info=info, w=w,
                    cpu=lambda k: cpu_ckks(w, k), cpu1=lambda k: cpu_ckks_1core(w, k))
    if name == "ct_tensor":
        w = workloads.ct_tensor()
        t = H.Tables(w["log_n"], w["moduli"])
        C, D = to_dev(w["c"], torch), to_dev(w["d"], torch)
        pairs, L, n = C.shape[0], C.shape[2], C.shape[3]
        out = torch.empty((pairs, 3, L, n), dtype=torch.int64, device="cuda:0")

        def step():
            H.ct_tensor(t, C, D, out=out)

        def per_poly_step():
            for i in range(pairs):
                H.ct_tensor(t, C[i:i + 1], D[i:i + 1], out=out[i:i + 1])

        info = {"workload": "ct_tensor", "N": n, "limbs": L, "ct_pairs": pairs,
                "ops": "fwd of c0,c1,d0,d1; tensor (c0d0, c0d1+c1d0, c1d1); inv of 3 outputs"}
        return dict(step=step, per_poly=per_poly_step, coeffs=7 * pairs * L * n, t=t, info=info, w=w,
                    cpu=lambda k: cpu_tensor(w, k), ctmul=pairs)
    if name == "uneven":
        mods = workloads.moduli("uneven")
        jobs = workloads.uneven_jobs()
        tables = {ln: H.Tables(ln, mods) for ln in sorted(set(ln for ln, _ in jobs))}
        xs = [to_dev(workloads.uneven_operand(j, ln, L, mods), torch) for j, (ln, L) in enumerate(jobs)]
        plan_f = H.BatchPlan([(x, tables[ln], L) for x, (ln, L) in zip(xs, jobs)], +1)
        plan_i = H.BatchPlan([(x, tables[ln], L) for x, (ln, L) in zip(xs, jobs)], -1)
        grid = _tuned_grid(plan_f, grid_arg, data=xs)
        plan_f.set_grid(grid)
        plan_i.set_grid(grid)
        plan_f.capture()
        plan_i.capture()
        coeffs = sum(L << ln for ln, L in jobs)

        def step():
            plan_f.replay()
            plan_i.replay()

        views = {(ln, L): tables[ln].view(L) for ln, L in set(jobs)}

        def per_poly_step():              # one launch sequence per polynomial
            for x, (ln, L) in zip(xs, jobs):
                H.ntt_fwd(views[(ln, L)], x)
            for x, (ln, L) in zip(xs, jobs):
                H.ntt_inv(views[(ln, L)], x)

        info = {"workload": "uneven", "jobs": len(jobs), "N_range": [1 << 12, 1 << 17], "limbs_range": [1, 32],
                "coefficients": coeffs, "ops": "fwd then inv, each one persistent launch, hipGraph replay",
                "persistent_grid": grid}
        def prof_step():                 # same launches outside the graph, so each is event-timed
            plan_f.run()
            plan_i.run()

        return dict(step=step, per_poly=per_poly_step, coeffs=2 * coeffs, t=tables, info=info, w={"x": xs},
                    cpu=lambda k: cpu_uneven(jobs, mods, k), plans=(plan_f, plan_i), prof_step=prof_step)
    if name == "rescale":
        # RS after Mul at the top of the ct_tensor chain: 32 ciphertexts (64
        # polynomials) of N = 2^16 at 24 limbs, NTT domain -> 23 limbs
        mods = workloads.moduli("ct_tensor")
        polys, L, logn = 64, len(mods), 16
        n = 1 << logn
        t = H.Tables(logn, mods)
        gen = torch.Generator(device="cuda:0")
        gen.manual_seed(2109_14704 + 7)
        C = torch.empty((polys, L, n), dtype=torch.int64, device="cuda:0")
        for l, q in enumerate(mods):
            C[:, l].copy_(torch.randint(0, q, (polys, n), generator=gen, device="cuda:0", dtype=torch.int64))
        out = torch.empty((polys, L - 1, n), dtype=torch.int64, device="cuda:0")
        tmp = torch.empty_like(C)
        lower = t.view(L - 1)

        def step():
            H.rescale(t, C, out=out, ntt=True)

        def unfused_step():           # inverse of every limb, coefficient rescale, forward of the rest
            tmp.copy_(C)
            H.ntt_inv(t, tmp)
            H.rescale(t, tmp, out=out)
            H.ntt_fwd(lower, out)

        info = {"workload": "rescale", "N": n, "limbs": L, "polys": polys,
                "ops": "RS in the NTT domain: inverse of the last limb, fused forward + subtract + scale per limb"}
        return dict(step=step, per_poly=unfused_step, coeffs=polys * (L - 1) * n, t=t, info=info,
                    w={"x": [None] * polys}, cpu=lambda k: cpu_rescale(mods, logn, k))
    w = workloads.plain4096()
    t = H.Tables(12, w["moduli"])
    X = to_dev(w["x"], torch)

    def step():
        H.ntt_fwd(t, X)
        H.ntt_inv(t, X)

    def per_poly_step():
        for i in range(X.shape[0]):
            H.ntt_fwd(t, X[i:i + 1])
            H.ntt_inv(t, X[i:i + 1])

    info = {"workload": "plain4096", "N": 4096, "limbs": 1, "polys": 8, "ops": "fwd, inv"}
    return dict(step=step, per_poly=per_poly_step, coeffs=2 * 8 * 4096, t=t, info=info, w=w,
                cpu=lambda k: cpu_plain(w, k))


# ---------------------------------------------------------------- CPU oracle
def cpu_ckks(w, k):
    import oracle
    a, b = w["a"][:k], w["b"][:k]
    t0 = time.perf_counter()
    oracle.batch_polymul(a, b, w["moduli"])
    dt = time.perf_counter() - t0
    return dt, 3 * a.size


def cpu_ckks_1core(w, k):
    """The CKKS-level oracle on one host thread."""
    import oracle
    a, b = w["a"][:k], w["b"][:k]
    t0 = time.perf_counter()
    oracle.batch_polymul(a, b, w["moduli"], threads=1)
    dt = time.perf_counter() - t0
    return dt, 3 * a.size


def cpu_tensor(w, k):
    import oracle
    c, d = w["c"][:k], w["d"][:k]
    t0 = time.perf_counter()
    oracle.batch_ct_tensor_coeff(c, d, w["moduli"])
    dt = time.perf_counter() - t0
    return dt, 7 * c[:, 0].size


def cpu_uneven(jobs, mods, k):
    import oracle
    import workloads
    t0 = time.perf_counter()
    coeffs = 0
    for j, (ln, L) in enumerate(jobs[:k]):
        x = workloads.uneven_operand(j, ln, L, mods)
        X = oracle.batch_ntt(x, mods[:L], +1)
        oracle.batch_ntt(X, mods[:L], -1)
        coeffs += 2 * x.size
    return time.perf_counter() - t0, coeffs


def cpu_rescale(mods, logn, k):
    import oracle
    import workloads
    x = workloads.uniform(7, 0, (k, len(mods), 1 << logn), mods)
    t0 = time.perf_counter()
    oracle.batch_rescale_ntt(x, mods)
    return time.perf_counter() - t0, k * (len(mods) - 1) << logn


def cpu_plain(w, k):
    import oracle
    x = w["x"]
    t0 = time.perf_counter()
    for _ in range(k):
        X = oracle.batch_ntt(x, w["moduli"], +1)
        oracle.batch_ntt(X, w["moduli"], -1)
    dt = time.perf_counter() - t0
    return dt, 2 * x.size * k


def cpu_baseline(s, target_s, one_core=False):
    import oracle
    k, limit = 1, len(s["w"].get("a", s["w"].get("c", s["w"].get("x"))))
    if s["info"]["workload"] == "uneven":
        k = 4
    cpu = s["cpu1"] if one_core else s["cpu"]
    dt, coeffs = cpu(k)
    while dt < target_s / 2 and k < limit:      # grow the sample to about the target time
        k = min(limit, max(k + 1, int(k * target_s / max(dt, 1e-3))))
        dt, coeffs = cpu(k)
    reps = 1
    if dt < target_s / 2:                       # the whole workload is short: repeat it
        reps = max(1, int(round(target_s / max(dt, 1e-3))))
        dt, coeffs = 0.0, 0
        for _ in range(reps):
            d1, c1 = cpu(k)
            dt, coeffs = dt + d1, coeffs + c1
    return {"value": coeffs / dt / 1e9, "unit": "Gcoeff/s", "cores": 1 if one_core else oracle.max_threads(), "kind": "oracle",
            "sample": "%d batch entr%s of the same workload%s (radix-2 oracle, %s), %.1f s"
                      % (k, "y" if k == 1 else "ies", ", %d times" % reps if reps > 1 else "",
                         "one thread" if one_core else "OpenMP over (batch, limb)", dt)}


# ---------------------------------------------------------------- roofline
# Algorithmic ALU work in VALU lane-operations (gfx950 has no 64-bit
# multiplier; v_mad_u64_u32 / v_mul_hi_u32 / v_mul_lo_u32 issue at full rate, so
# every VALU op costs one issue slot):
VALU_BFLY = 21     # Harvey/Shoup butterfly: 9 32-bit multiplies + 12 adds, compares, selects
VALU_PROD = 19     # Montgomery product a b R^-1 mod q: 128-bit product, low product by -q^-1, high product by q
VALU_TENSOR = 68   # c0d0, c1d1 (2 x 19) + c0d1 + c1d0 with one Montgomery reduction (30)
VALU_RS_EPI = 17   # rescale epilogue: Shoup product by qL^-1 (9 + adds) and a reduction from [0, 4q)
VALU_MAC = 83      # one matMul product term, k >= 3: the tensor's Montgomery products (68), three lazy additions (5 each)
VALU_MAC_B = 121   # one matMul product term, k <= 2: the tensor's three outputs accumulated with Barrett mad_mod
VALU_KS_MAC = 24   # key switch, per digit word and key component: Montgomery product (19), lazy addition (5)
VALU_KS_FIN = 20   # key switch, per output word: Shoup product by R mod q (12), reduction from [0, 4q) (8)
VALU_KS_FIN_C = 38 # the same plus P c_s: a second Shoup product, an addition, a reduction from [0, 8q)


def kernel_work(name, info):
    """Algorithmic HBM bytes and VALU operations of ONE launch of `name` in
    the benchmarked step: per-unit figures times the units one launch handles.
    Bytes: every coefficient word a launch must read once and write once
    (8 B each).  ALU: VALU_BFLY per butterfly, N/2 butterflies per stage per
    polynomial limb, plus the products."""
    import paper_2109_14704_amd as H
    n, L = info["N"], info["limbs"]
    logn = n.bit_length() - 1
    t_cols, p_cols = H.stage_split(logn)                   # stages in the column passes (library plan)
    if info["workload"] == "rescale":
        # column pass: reads the last limb's words once per polynomial (its
        # other reads, one per output limb, hit the caches) and writes one
        # scratch word per output coefficient; the block pass reads it and c_i
        # and writes the result; the epilogue is about one Shoup product and a
        # reduction
        units = info["polys"] * (L - 1)
        base = name.split("<")[0]
        if base == "k_rs_cols":
            return 8.0 * (units + info["polys"]) * n, VALU_BFLY * units * (n // 2) * t_cols
        if base == "k_rs_blocks":
            return 24.0 * units * n, VALU_BFLY * units * (n // 2) * (logn - t_cols) + VALU_RS_EPI * units * n
        return None, None
    if info["workload"] == "ckks_level":
        p = info["polys_per_operand"]
        n_in, n_out, prod_mul = 2 * p, p, VALU_PROD * p * L * n
    elif info["workload"] == "ct_tensor":
        c = info["ct_pairs"]
        n_in, n_out, prod_mul = 4 * c, 3 * c, VALU_TENSOR * c * L * n
    else:
        n_in = n_out = info["polys"]
        prod_mul = 0
    bfly = lambda polys, stages: VALU_BFLY * polys * L * (n // 2) * stages
    base = name.split("<")[0]
    ec = p_cols if info["workload"] in ("ckks_level", "ct_tensor") else t_cols
    if base == "k_cols_fwd":
        return 16.0 * n_in * L * n, bfly(n_in, ec)
    if base == "k_cols_inv":
        return 16.0 * n_out * L * n, bfly(n_out, ec)
    if base.startswith("k_prod"):
        stages = logn - ec
        return 8.0 * (n_in + n_out) * L * n, bfly(n_in + n_out, stages) + prod_mul
    if base in ("k_fwd_whole", "k_inv_whole"):
        return 16.0 * n_in * L * n, bfly(n_in, logn)
    if base in ("k_fwd_blocks", "k_inv_blocks"):
        return 16.0 * n_in * L * n, bfly(n_in, logn - t_cols)
    return None, None


def batch_work(info, jobs):
    """One persistent launch over the uneven batch: each (polynomial, limb) of
    N = 2^12 is read and written once, larger N twice (two passes); butterflies
    (N/2) log2 N per (polynomial, limb)."""
    nbytes = sum(L * (1 << ln) * (16 if ln == 12 else 32) for ln, L in jobs)
    muls = sum(VALU_BFLY * L * (1 << (ln - 1)) * ln for ln, L in jobs)
    return float(nbytes), float(muls)


def ks_work(batch, l, logn, ec):
    """ONE launch of the key-switch block kernel (k_ks_blocks): per (batch
    entry, target prime t <= l, digit j < l) the last logn - ec forward stages
    of a digit and two Montgomery multiply-adds per word; per output word the
    finishing products.  Bytes: the column-pass words read once, the key read
    once (shared by the batch), c0 and c1 read once, the accumulators written."""
    n = 1 << logn
    L1 = l + 1
    ops = batch * L1 * l * (VALU_BFLY * (n // 2) * (logn - ec) + 2 * VALU_KS_MAC * n)
    ops += batch * 2 * n * (l * VALU_KS_FIN_C + VALU_KS_FIN)
    nbytes = 8.0 * n * (batch * l * L1 + l * 2 * L1 + batch * 2 * l + batch * 2 * L1)
    return nbytes, float(ops)


def alu_or_hbm(nbytes, ops, per_launch_s):
    """Roofline object of one launch against the binding roof."""
    from paper_2109_14704_amd import roofline as R
    if nbytes / (R.HBM_PEAK_GBS * 1e9) >= ops / (R.VALU_PEAK_TOPS * 1e12):
        ach = nbytes / per_launch_s / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": R.HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / R.HBM_PEAK_GBS, 4)}
    ach = ops / per_launch_s / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": round(R.VALU_PEAK_TOPS, 2), "unit": "T VALU-op/s",
            "frac": round(ach / R.VALU_PEAK_TOPS, 4)}


def roofline(prof, info, steps):
    from paper_2109_14704_amd import roofline as R
    # dominant kernel by total time
    name, (ms, cnt) = max(prof.items(), key=lambda kv: kv[1][0])
    per_launch_s = ms / 1e3 / cnt
    if name.startswith("k_batch"):
        import workloads
        nbytes, muls = batch_work(info, workloads.uneven_jobs())
    else:
        nbytes, muls = kernel_work(name, info)
    if nbytes is None:
        return None, name, per_launch_s
    t_hbm = nbytes / (R.HBM_PEAK_GBS * 1e9)
    t_alu = muls / (R.VALU_PEAK_TOPS * 1e12)
    if t_hbm >= t_alu:
        ach = nbytes / per_launch_s / 1e9
        rl = {"bound": "hbm", "achieved": round(ach, 1), "peak": R.HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(ach / R.HBM_PEAK_GBS, 4)}
    else:
        ach = muls / per_launch_s / 1e12
        rl = {"bound": "alu", "achieved": round(ach, 3), "peak": round(R.VALU_PEAK_TOPS, 2),
              "unit": "T VALU-op/s", "frac": round(ach / R.VALU_PEAK_TOPS, 4)}
    rl.update({"kernel": name, "launch_ms": round(per_launch_s * 1e3, 4), "traffic": R.stored_traffic(name)})
    return rl, name, per_launch_s


def bench_ladder(args):
    """The kernel-design ladder of the paper's NTT evaluation on its own shape:
    forward transforms of [1024][8][2^15] (8 primes of 55 bits) by the naive
    radix-2 design, staged designs with radix-2/4/8/16 LDS rounds, and the
    library's kernels.  Each design's time, speedup over naive, and VALU
    roofline fraction (21 ops per butterfly)."""
    import torch
    import workloads
    import paper_2109_14704_amd as H
    polys, L, logn = 1024, 8, 15
    n = 1 << logn
    mods = workloads.moduli("ct_tensor")[:L]
    t = H.Tables(logn, mods)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(2109_14704 + 6)
    x = torch.empty((polys, L, n), dtype=torch.int64, device="cuda:0")
    for l, q in enumerate(mods):                  # uniform [0, q) per limb, on the device
        x[:, l].copy_(torch.randint(0, q, (polys, n), generator=gen, device="cuda:0", dtype=torch.int64))
    coeffs = polys * L * n
    ops = 21.0 * polys * L * (n // 2) * logn
    from paper_2109_14704_amd import roofline as R
    designs = [(H.VARIANT_NAIVE, "naive radix-2, one global-memory launch per stage"),
               (H.VARIANT_STAGED_R2, "4 naive global stages + LDS blocks of 2048, radix-2 rounds"),
               (H.VARIANT_STAGED_R4, "column pass + LDS blocks of 4096, radix-4 rounds"),
               (H.VARIANT_STAGED_R8, "column pass + LDS blocks of 4096, radix-8 rounds (the paper's best)"),
               (H.VARIANT_STAGED_R16, "column pass + LDS blocks of 4096, radix-16 rounds"),
               (H.VARIANT_LIBRARY, "library: 5-stage radix-32 column pass + radix-16 LDS blocks of 1024")]
    rows = []
    for v, desc in designs:
        for _ in range(max(2, args.warmup // 4)):
            H.ntt_fwd_variant(t, x, v)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k = max(3, args.steps // 3)
        a.record()
        for _ in range(k):
            H.ntt_fwd_variant(t, x, v)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / k
        rows.append({"variant": v, "design": desc, "ms": round(ms, 4), "gcoeff_s": round(coeffs / ms / 1e6, 3),
                     "alu_frac": round(ops / (ms / 1e3) / (R.VALU_PEAK_TOPS * 1e12), 4)})
    base = rows[0]["ms"]
    for r in rows:
        r["x_naive"] = round(base / r["ms"], 2)
    lib_row = rows[-1]
    H.prof_enable(True)
    for _ in range(3):
        H.ntt_fwd(t, x)
    torch.cuda.synchronize()
    prof = H.prof_read()
    H.prof_enable(False)
    info = {"workload": "ladder", "N": n, "limbs": L, "polys": polys, "ops": "fwd (the paper's NTT shape)"}
    rl, _, _ = roofline(prof, info, 3)
    result = {"metric": METRIC, "value": lib_row["gcoeff_s"], "unit": "Gcoeff/s", "n_gpus": 1,
              "steps": max(3, args.steps // 3), "warmup": max(2, args.warmup // 4), "ms_per_step": lib_row["ms"],
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
              "data": "synthetic", "config": info, "roofline": rl,
              "kernels_ms": {kk: round(vv[0] / vv[1], 4) for kk, vv in sorted(prof.items())}, "ladder": rows}
    print(json.dumps(result), flush=True)


def bench_matmul(args):
    """The paper's encrypted element-wise polynomial matMul shapes (section
    IV-E): C += A*B with ciphertext elements of N = 8192 over 4 limbs, NTT
    domain, 100x100x1 and 10x9x8 (m x n x k).  Value: element ciphertext
    products per second on 100x100x1.  Roofline against the compulsory bytes
    (A and B once, C read and written) and VALU_MAC ops per product term
    (VALU_MAC_B for k <= 2, which the kernel accumulates with Barrett)."""
    import torch
    import workloads
    import paper_2109_14704_amd as H
    from paper_2109_14704_amd import roofline as R
    mods = workloads.moduli("ct_tensor")[:4]
    L, logn = len(mods), 13
    n_ = 1 << logn
    t = H.Tables(logn, mods)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(2109_14704 + 8)

    def operand(shape):
        x = torch.empty(shape + (L, n_), dtype=torch.int64, device="cuda:0")
        for l, q in enumerate(mods):
            x[..., l, :].copy_(torch.randint(0, q, shape + (n_,), generator=gen, device="cuda:0", dtype=torch.int64))
        return x

    rows = []
    for (m, n, k) in [(100, 100, 1), (10, 9, 8)]:
        A, B, C = operand((m, k, 2)), operand((k, n, 2)), operand((m, n, 3))
        for _ in range(max(2, args.warmup // 4)):
            H.ct_matmul(t, A, B, C)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(3, args.steps // 3)
        a.record()
        for _ in range(reps):
            H.ct_matmul(t, A, B, C)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        nbytes = 8.0 * L * n_ * (2 * m * k + 2 * k * n + 6 * m * n)
        ops = float(VALU_MAC if k >= 3 else VALU_MAC_B) * m * n * k * L * n_
        t_hbm, t_alu = nbytes / (R.HBM_PEAK_GBS * 1e9), ops / (R.VALU_PEAK_TOPS * 1e12)
        if t_hbm >= t_alu:
            rl = {"bound": "hbm", "achieved": round(nbytes / ms / 1e6, 1), "peak": R.HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(nbytes / ms / 1e6 / R.HBM_PEAK_GBS, 4)}
        else:
            rl = {"bound": "alu", "achieved": round(ops / ms / 1e9, 3), "peak": round(R.VALU_PEAK_TOPS, 2),
                  "unit": "T VALU-op/s", "frac": round(ops / ms / 1e9 / R.VALU_PEAK_TOPS, 4)}
        rl.update({"kernel": "k_ct_matmul<13>", "launch_ms": round(ms, 4), "traffic": R.stored_traffic("k_ct_matmul<13>")})
        rows.append({"shape": "%dx%dx%d" % (m, n, k), "ms": round(ms, 4),
                     "element_products_per_s": round(m * n * k / ms * 1e3, 1), "roofline": rl})
        del A, B, C
    first = rows[0]
    info = {"workload": "matmul", "N": n_, "limbs": L, "shapes": [r["shape"] for r in rows],
            "ops": "C += A*B, ciphertext elements, NTT domain, mad_mod accumulation"}
    result = {"metric": METRIC, "value": first["element_products_per_s"], "unit": "ct element products/s",
              "n_gpus": 1, "steps": max(3, args.steps // 3), "warmup": max(2, args.warmup // 4),
              "ms_per_step": first["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "u64", "data": "synthetic", "config": info, "roofline": first["roofline"], "shapes": rows}
    print(json.dumps(result), flush=True)


def bench_routines(args):
    """The paper's HE routine benchmark (section IV-C) on its parameters,
    N = 2^15 and 8 primes (plus a special prime for the key switch), NTT
    domain, synthetic ciphertexts and key: MulLin = Mul (tensor) + Relin;
    MulLinRS = MulLin + rescale.  One ciphertext pair (the paper's unbatched
    routines) and a batch of 32.  Value: MulLinRS per second at batch 32."""
    import torch
    import workloads
    import paper_2109_14704_amd as H
    chain = workloads.moduli("ct_tensor")
    l, logn = 8, 15
    n_ = 1 << logn
    t8, t9 = H.Tables(logn, chain[:l]), H.Tables(logn, chain[:l + 1])
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(2109_14704 + 9)

    def operand(shape, mods):
        x = torch.empty(shape + (len(mods), n_), dtype=torch.int64, device="cuda:0")
        for i, q in enumerate(mods):
            x[..., i, :].copy_(torch.randint(0, q, shape + (n_,), generator=gen, device="cuda:0", dtype=torch.int64))
        return x

    ksk = operand((l, 2), chain[:l + 1])
    rows = []
    for batch in (1, 32):
        c, d = operand((batch, 2), chain[:l]), operand((batch, 2), chain[:l])
        prod = torch.empty((batch, 3, l, n_), dtype=torch.int64, device="cuda:0")
        lin = torch.empty((batch, 2, l, n_), dtype=torch.int64, device="cuda:0")
        rs = torch.empty((batch * 2, l - 1, n_), dtype=torch.int64, device="cuda:0")

        def mullin():
            H.ct_tensor(t8, c, d, out=prod, in_ntt=True, out_ntt=True)
            H.relin(t9, prod, ksk, out=lin)

        def mullinrs():
            mullin()
            H.rescale(t8, lin.view(batch * 2, l, n_), out=rs, ntt=True)

        for name, fn in (("MulLin", mullin), ("MulLinRS", mullinrs)):
            for _ in range(max(3, args.warmup // 2)):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = max(5, args.steps)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            rows.append({"routine": name, "batch": batch, "us": round(ms * 1e3, 1),
                         "per_s": round(batch / ms * 1e3, 1)})
    H.prof_enable(True)
    for _ in range(3):
        mullinrs()
    torch.cuda.synchronize()
    prof = H.prof_read()
    H.prof_enable(False)
    value = [r for r in rows if r["routine"] == "MulLinRS" and r["batch"] == 32][0]
    info = {"workload": "routines", "N": n_, "limbs": l, "special_primes": 1, "batches": [1, 32],
            "ops": "MulLin = tensor + relin; MulLinRS = MulLin + rescale (NTT domain)"}
    from paper_2109_14704_amd import roofline as R
    kname = "k_ks_blocks<%d>" % logn
    rl = None
    if kname in prof:               # the profiled launches ran at batch 32
        per_launch_s = prof[kname][0] / 1e3 / prof[kname][1]
        nbytes, ops = ks_work(32, l, logn, 5 if logn >= 15 else logn - 12)   # the key switch's column stages
        rl = alu_or_hbm(nbytes, ops, per_launch_s)
        rl.update({"kernel": kname, "launch_ms": round(per_launch_s * 1e3, 4), "traffic": R.stored_traffic(kname)})
    result = {"metric": METRIC, "value": value["per_s"], "unit": "MulLinRS/s", "n_gpus": 1,
              "steps": max(5, args.steps), "warmup": max(3, args.warmup // 2), "ms_per_step": value["us"] / 1e3,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
              "data": "synthetic", "config": info, "roofline": rl,
              "kernels_ms": {k: round(v[0] / v[1], 4) for k, v in sorted(prof.items())}, "routines": rows}
    print(json.dumps(result), flush=True)


def bench_serving(args):
    """Poisson ct-mul serving: saturation throughput, then p50/p99 latency of the
    continuous-batching server and of per-request launches on the same traces
    at 0.5, 0.8 and 0.95 of the server's saturation rate."""
    import torch
    import workloads
    from paper_2109_14704_amd import serve
    chain = workloads.moduli("serving")
    be = serve.HipBackend(chain, streams=2)
    gen = torch.Generator(device="cuda:0")
    ops = {}

    def operands(ln, lvl, k):
        key = (ln, lvl, k)
        if key not in ops:          # seeded, uniform per limb, device-resident
            gen.manual_seed(2109_14704 + 4 * 1000003 + ln * 1009 + lvl * 31 + k)
            c = torch.empty((1, 2, lvl, 1 << ln), dtype=torch.int64, device="cuda:0")
            d = torch.empty_like(c)
            for l in range(lvl):
                c[:, :, l].random_(0, chain[l], generator=gen)
                d[:, :, l].random_(0, chain[l], generator=gen)
            ops[key] = (c, d)
        return ops[key]

    def requests(trace):
        return [serve.Request(i, t, ln, lvl, *operands(ln, lvl, i % 2)) for i, (t, ln, lvl) in enumerate(trace)]

    budget = 24 << 30
    warm = 200
    n = args.requests
    # saturation: every request offered at t = 0
    sat_trace = [(0.0, ln, lvl) for _, ln, lvl in workloads.serving_trace(n, 1.0, seed_stream=2)]
    reqs = requests(sat_trace)
    sched = serve.Scheduler(be, budget, streams=2)
    sched.run_trace(reqs[:warm])
    torch.cuda.synchronize()
    reqs = requests(sat_trace)
    sched = serve.Scheduler(be, budget, streams=2)
    el = sched.run_trace(reqs)
    sat = n / el
    print("bench: serving saturation %.0f ct-mul/s (%d steps)" % (sat, sched.steps), file=sys.stderr, flush=True)
    rows = []
    for f in (0.5, 0.8, 0.95):
        trace = workloads.serving_trace(n, f * sat, seed_stream=1)
        rs = requests(trace)
        sched = serve.Scheduler(be, budget, streams=2)
        el = sched.run_trace(rs)
        srv = serve.latency_stats(rs[warm:])
        srv["throughput"] = round(len(rs) / el, 1)
        rb = requests(trace)
        elb = serve.serve_per_request(rb, be)
        base = serve.latency_stats(rb[warm:])
        base["throughput"] = round(len(rb) / elb, 1)
        rows.append({"load": f, "rate_per_s": round(f * sat, 1), "server": srv, "per_request": base})
        print("bench: load %.2f server p50 %.3f p99 %.3f ms; per-request p50 %.3f p99 %.3f ms" % (
            f, srv.get("p50_ms", -1), srv.get("p99_ms", -1), base.get("p50_ms", -1), base.get("p99_ms", -1)),
            file=sys.stderr, flush=True)
    result = {"metric": METRIC, "value": round(sat, 1), "unit": "ct-mul/s", "n_gpus": 1, "steps": n,
              "warmup": warm, "ms_per_step": round(1e3 / sat, 4), "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "u64", "data": "synthetic",
              "config": {"workload": "serving", "N": [1 << 14, 1 << 15, 1 << 16], "levels": [4, 24],
                         "hbm_budget_bytes": budget, "streams": 2, "requests": n},
              "latency": rows}
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.workload == "routines":
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        return bench_routines(args)
    if args.workload == "matmul":
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        return bench_matmul(args)
    if args.workload == "ladder":
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        return bench_ladder(args)
    if args.workload == "serving":
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        return bench_serving(args)
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported (the path shards by batch "
              "with no exchange, see the design notes)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2109_14704_amd as H
    H.lib()
    print("bench: setting up workload %s" % args.workload, file=sys.stderr, flush=True)
    s = setup(args.workload, torch, H, args.grid)
    step = s["step"]
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1) / args.steps
    value = s["coeffs"] / (ms / 1e3) / 1e9
    print("bench: %.3f ms/step (%.1f Gcoeff/s), wall %.3f s" % (ms, value, wall), file=sys.stderr, flush=True)

    # per-kernel durations (HIP events on the launching stream), separate pass
    H.prof_enable(True)
    prof_steps = max(3, min(args.steps, 10))
    for _ in range(prof_steps):
        s.get("prof_step", step)()
    torch.cuda.synchronize()
    prof = H.prof_read()
    H.prof_enable(False)
    rl, kname, kdur = roofline(prof, s["info"], prof_steps)

    result = {"metric": METRIC, "value": round(value, 3), "unit": "Gcoeff/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "u64", "data": "synthetic", "config": s["info"], "roofline": rl,
              "kernels_ms": {k: round(v[0] / v[1], 4) for k, v in sorted(prof.items())}}
    if "ctmul" in s:
        result["ct_mul_per_s"] = round(s["ctmul"] / (ms / 1e3), 1)
    if not args.no_per_poly:
        s["per_poly"]()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        a.record()
        for _ in range(reps):
            s["per_poly"]()
        b.record()
        torch.cuda.synchronize()
        pms = a.elapsed_time(b) / reps
        if s["info"]["workload"] == "rescale":      # the comparator is the unfused sequence
            result["unfused"] = {"ms_per_step": round(pms, 4), "value": round(s["coeffs"] / (pms / 1e3) / 1e9, 3),
                                 "unit": "Gcoeff/s", "fused_speedup": round(pms / ms, 3),
                                 "ops": "inverse of every limb, coefficient rescale, forward of the rest"}
        else:
            result["per_poly"] = {"ms_per_step": round(pms, 4), "value": round(s["coeffs"] / (pms / 1e3) / 1e9, 3),
                                  "unit": "Gcoeff/s", "batched_speedup": round(pms / ms, 3)}
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
        if "cpu1" in s:                          # the same oracle on one host thread, a shorter sample
            result["cpu_baseline_1core"] = cpu_baseline(s, args.cpu_seconds / 3, one_core=True)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
