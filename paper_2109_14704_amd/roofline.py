"""Roofline accounting for the NTT path.

Two parts:
  * the paper's own density arithmetic (section IV-B, Table I): int64 ALU
    operations per work-item per round, divided by global-memory bytes, for
    the naive radix-2 NTT and the staged radix-8 shared-local-memory NTT;
  * the MI355X figures our benchmark divides by: algorithmic HBM bytes and
    VALU instruction counts per launch of a kernel.
"""
import hashlib
import json
import math
import os

# Table I: 64-bit integer ALU operations per work-item per round (other + butterfly).
TABLE_I = {2: 48, 4: 157, 8: 456, 16: 1156}

# MI355X published peaks (unit counts x clock).
HBM_PEAK_GBS = 8000.0                 # HBM3E, GB/s
CUS, SIMDS_PER_CU, LANES, CLOCK_GHZ = 256, 4, 16, 2.4
# VALU lane-operations per second: every SIMD retires 16 lanes of one VALU
# instruction per clock; gfx950 issues v_mad_u64_u32 and v_mul_hi_u32 at that
# full rate (measured), so integer multiplies need no separate roof.
VALU_PEAK_TOPS = CUS * SIMDS_PER_CU * LANES * CLOCK_GHZ / 1000.0   # 39.32 T lane-ops/s


def paper_density(kind, n):
    """Operational density (int64 ops per byte) as section IV-B computes it."""
    logn = int(math.log2(n))
    if kind == "naive":
        ops = TABLE_I[2] * (n // 2) * logn
        accesses = 2 * n * logn
    elif kind == "radix8_slm":
        ops = TABLE_I[8] * (n // 8) * math.log(n, 8)
        accesses = 2 * 2 * n          # load+store, two global rounds
    else:
        raise ValueError(kind)
    return ops / (accesses * 8)


def transform_bytes(coeffs, passes):
    """Algorithmic HBM bytes of `passes` read+write sweeps over `coeffs` words."""
    return 16.0 * coeffs * passes


def butterflies(n, polys):
    return polys * (n // 2) * int(math.log2(n))


_TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                             "traffic.json")


def source_digest():
    """Hash of the kernel sources; stored traffic figures are void once it changes."""
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch measured with rocprofv3 counters for `kernel`, or None
    if not measured or measured on different kernel sources."""
    try:
        with open(_TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_digest") != source_digest():
        return None
    return d.get("kernels", {}).get(kernel)
