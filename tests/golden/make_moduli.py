"""Writes tests/golden/moduli.json: the RNS modulus chains of the five workloads.

Calls only the CPU oracle (its Miller-Rabin prime search).  Each chain holds
NTT-friendly primes q = 1 (mod M), the largest ones below 2^bits, as the
workloads state:
  plain4096  : one 50-bit prime, M = 2N = 8192                    (N = 4096)
  ckks_level : 16 primes, bit sizes drawn uniformly from 50..60,  M = 2^16
  ct_tensor  : the 24 largest 55-bit primes,                      M = 2^17
  uneven     : 32 primes, bit sizes drawn uniformly from 50..60,  M = 2^18
  serving    : the ct_tensor chain (level l uses its first l primes)
Bit sizes are drawn from the workload's seeded stream 0 (workloads.rng).
Run:  python tests/golden/make_moduli.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.abspath(os.path.join(HERE, "..", "..")))

import oracle  # noqa: E402
import workloads  # noqa: E402


def chain(bits_list, M):
    out = []
    for b in bits_list:
        out += oracle.gen_primes(int(b), M, 1, exclude=out)
    return out


def main():
    r1 = workloads.rng(1, 0).integers(50, 61, size=16)
    r3 = workloads.rng(3, 0).integers(50, 61, size=32)
    chains = {
        "plain4096": {"M": 8192, "bits": [50], "moduli": chain([50], 8192)},
        "ckks_level": {"M": 1 << 16, "bits": [int(b) for b in r1], "moduli": chain(r1, 1 << 16)},
        "ct_tensor": {"M": 1 << 17, "bits": [55] * 24, "moduli": oracle.gen_primes(55, 1 << 17, 24)},
        "uneven": {"M": 1 << 18, "bits": [int(b) for b in r3], "moduli": chain(r3, 1 << 18)},
    }
    chains["serving"] = dict(chains["ct_tensor"])
    with open(os.path.join(HERE, "moduli.json"), "w") as f:
        json.dump(chains, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
