"""Seeded synthetic inputs for the five workloads (shared by the tests, the
benchmark and the oracle-side checks).  Holds no modular arithmetic: only
random draws, shapes and the stored modulus chains.

Recipe: numpy PCG64 seeded from SeedSequence([2109_14704 + workload_index, stream]);
coefficients of limb l are drawn uniformly from [0, q_l) as uint64.  The paper
evaluates only on random ciphertexts of these shapes (section IV), so nothing
else stands in for a dataset.
"""
import json
import os

import numpy as np

SEED_BASE = 2109_14704
_HERE = os.path.dirname(os.path.abspath(__file__))
MODULI_JSON = os.path.join(_HERE, "..", "tests", "golden", "moduli.json")

# name -> (index, log_n or None, description)
WORKLOADS = {
    "plain4096": (0, 12, "single negacyclic NTT, N=4096, one 50-bit prime, 8 polys + one polymul"),
    "ckks_level": (1, 15, "N=2^15, 16 primes 50-60 bit, 64 ciphertexts x 2 polys: fwd, dyadic, inv"),
    "ct_tensor": (2, 16, "N=2^16, 24 x 55-bit primes, 32 ciphertext pairs: fused ct tensor product"),
    "uneven": (3, None, "512 polys, N in 2^12..2^17, limbs U[1,32], one persistent launch"),
    "serving": (4, None, "Poisson ct-mul requests, N in 2^14..2^16, levels 4..24"),
}


def rng(index, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + index, stream])))


def moduli(name):
    with open(MODULI_JSON) as f:
        return [int(v) for v in json.load(f)[name]["moduli"]]


def uniform(index, stream, shape, mods):
    """uint64 array of `shape` (..., limbs, N) with limb l uniform in [0, mods[l])."""
    shape = tuple(shape)
    limbs = shape[-2]
    g = rng(index, stream)
    out = np.empty(shape, dtype=np.uint64)
    for l in range(limbs):
        out[..., l, :] = g.integers(0, mods[l], size=shape[:-2] + (shape[-1],), dtype=np.uint64)
    return out


def plain4096():
    m = moduli("plain4096")
    return {"moduli": m, "log_n": 12,
            "x": uniform(0, 1, (8, 1, 4096), m),
            "a": uniform(0, 2, (1, 1, 4096), m),
            "b": uniform(0, 3, (1, 1, 4096), m)}


def ckks_level(batch=128):
    m = moduli("ckks_level")
    return {"moduli": m, "log_n": 15,
            "a": uniform(1, 1, (batch, 16, 1 << 15), m),
            "b": uniform(1, 2, (batch, 16, 1 << 15), m)}


def ct_tensor(pairs=32, limbs=24, log_n=16):
    m = moduli("ct_tensor")[:limbs]
    return {"moduli": m, "log_n": log_n,
            "c": uniform(2, 1, (pairs, 2, limbs, 1 << log_n), m),
            "d": uniform(2, 2, (pairs, 2, limbs, 1 << log_n), m)}


def uneven_jobs(njobs=512, min_log=12, max_log=17, max_limbs=32):
    """(log_n, limbs) per job, drawn uniformly; job j uses the first limbs_j primes."""
    g = rng(3, 1)
    log_n = g.integers(min_log, max_log + 1, size=njobs)
    limbs = g.integers(1, max_limbs + 1, size=njobs)
    return [(int(a), int(b)) for a, b in zip(log_n, limbs)]


def uneven_operand(job_index, log_n, limbs, mods):
    return uniform(3, 100 + job_index, (1, limbs, 1 << log_n), mods[:limbs])


def serving_trace(nreq, rate_per_s, seed_stream=1):
    """Poisson arrivals: (arrival_time_s, log_n, level) per request."""
    g = rng(4, seed_stream)
    gaps = g.exponential(1.0 / rate_per_s, size=nreq)
    log_n = g.integers(14, 17, size=nreq)
    level = g.integers(4, 25, size=nreq)
    t = np.cumsum(gaps)
    return [(float(a), int(b), int(c)) for a, b, c in zip(t, log_n, level)]


def serving_operands(req_index, log_n, level, mods):
    c = uniform(4, 1000 + 2 * req_index, (1, 2, level, 1 << log_n), mods[:level])
    d = uniform(4, 1001 + 2 * req_index, (1, 2, level, 1 << log_n), mods[:level])
    return c, d
