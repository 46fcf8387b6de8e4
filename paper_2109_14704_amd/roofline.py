"""Roofline accounting for the NTT path.

Three parts:
  * the paper's own density arithmetic (section IV-B, Table I): int64 ALU
    operations per work-item per round, divided by global-memory bytes, for
    the naive radix-2 NTT and the staged radix-8 shared-local-memory NTT;
  * algorithmic work per kernel launch and per benchmark step, in the units
    the roofline divides by: compulsory HBM bytes (every word a launch must
    read once and write once, 8 B each) and 32-bit integer multiplies (a
    Shoup product, hence a butterfly, counts 10; a full modular product of
    two variables 11; v_mad_u64_u32 counts as one multiply);
  * the same work in VALU lane-operations of this implementation's
    instruction stream (a separate figure: multiplies are only part of it).

Peaks: MI355X's published HBM3E bandwidth, and a VALU issue peak derived
from unit counts and clock (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32 T
lane-operations/s), which is also the multiply peak: gfx950 issues
v_mad_u64_u32, v_mul_hi_u32 and v_mul_lo_u32 at that rate (the measured
rates of microbench.py are reported beside it).
"""
import hashlib
import json
import math
import os

# Table I: 64-bit integer ALU operations per work-item per round (other + butterfly).
TABLE_I = {2: 48, 4: 157, 8: 456, 16: 1156}

# MI355X peaks.
HBM_PEAK_GBS = 8000.0                 # HBM3E, GB/s (published)
CUS, SIMDS_PER_CU, LANES, CLOCK_GHZ = 256, 4, 16, 2.4
VALU_PEAK_TOPS = CUS * SIMDS_PER_CU * LANES * CLOCK_GHZ / 1000.0   # 39.32 T lane-ops/s
MUL_PEAK_TOPS = VALU_PEAK_TOPS        # one 32-bit multiply per lane per clock

# Algorithmic 32-bit multiplies per unit of work.
MUL_BFLY = 10       # Shoup butterfly: quotient estimate (3), W Y mod 2^64 (3), Q q mod 2^64 (3), ~1 more
MUL_SHOUP = 10      # a Shoup product by a constant (the butterfly's multiply)
MUL_PROD = 11       # a b mod q for two variables: 128-bit product (4) + Montgomery/Barrett reduction (7)
MUL_TENSOR = 37     # c0 d0, c1 d1 (11 each) + c0 d1 + c1 d0 summed before one reduction (4 + 4 + 7)
MUL_KS_MAC = 22     # key switch, per digit word: products with both key components
MUL_RS_PRO = 7      # rescale prologue: floor-estimate of s / q_i (4) and its product by q_i (3)

# VALU lane-operations of this implementation per unit (counted in its AMD asm).
VALU_BFLY = 21      # 9 multiplies + 64-bit adds, one compare, two selects
VALU_PROD = 19      # Montgomery product a b R^-1 mod q
VALU_TENSOR = 68    # c0d0, c1d1 (2 x 19) + c0d1 + c1d0 with one Montgomery reduction (30)
VALU_RS_EPI = 17    # rescale epilogue: Shoup product by qL^-1 and a reduction from [0, 4q)
VALU_MAC = 83       # one matMul product term, k >= 3: the tensor's Montgomery products (68), three lazy additions
VALU_MAC_B = 121    # one matMul product term, k <= 2: the tensor's three outputs accumulated with Barrett mad_mod
VALU_KS_MAC = 24    # key switch, per digit word and key component: Montgomery product (19), lazy addition (5)
VALU_KS_FIN = 20    # key switch, per output word: Shoup product by R mod q (12), reduction from [0, 4q) (8)
VALU_KS_FIN_C = 38  # the same plus P c_s: a second Shoup product, an addition, a reduction from [0, 8q)


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


def butterflies(n, polys, stages=None):
    """Butterflies of `stages` stages (all log2 n by default) over `polys` polynomials."""
    return polys * (n // 2) * (int(math.log2(n)) if stages is None else stages)


class Work:
    """Algorithmic work: compulsory HBM bytes, 32-bit multiplies, VALU lane-ops."""

    def __init__(self, nbytes=0.0, muls=0.0, valu=0.0):
        self.nbytes, self.muls, self.valu = float(nbytes), float(muls), float(valu)

    def __add__(self, o):
        return Work(self.nbytes + o.nbytes, self.muls + o.muls, self.valu + o.valu)

    def as_dict(self):
        return {"bytes": self.nbytes, "multiplies": self.muls, "valu_ops": self.valu}


def transform_work(n, polys, stages=None):
    """Butterfly arithmetic of `stages` stages of `polys` (polynomial, limb) transforms (no bytes)."""
    b = butterflies(n, polys, stages)
    return Work(0, MUL_BFLY * b, VALU_BFLY * b)


def roof(work, seconds, measured=None):
    """Roofline object of one launch (or one step) doing `work` in `seconds`:
    the binding roof is the one whose peak gives the longer time for the
    work.  With `measured` (microbench.measure_all()), the measured stream
    bandwidth and multiply rate are reported beside the published peaks."""
    t_hbm = work.nbytes / (HBM_PEAK_GBS * 1e9)
    t_mul = work.muls / (MUL_PEAK_TOPS * 1e12)
    if t_hbm >= t_mul:
        ach = work.nbytes / seconds / 1e9
        r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4)}
        if measured:
            r["peak_measured"] = measured["hbm_copy_gbs"]
            r["frac_measured"] = round(ach / measured["hbm_copy_gbs"], 4)
    else:
        ach = work.muls / seconds / 1e12
        r = {"bound": "alu", "achieved": round(ach, 3), "peak": round(MUL_PEAK_TOPS, 2),
             "unit": "T int32-mul/s", "frac": round(ach / MUL_PEAK_TOPS, 4)}
        if measured:
            r["peak_measured"] = measured["mul_mix_tops"]
            r["frac_measured"] = round(ach / measured["mul_mix_tops"], 4)
    if work.valu:
        va = work.valu / seconds / 1e12
        r["valu"] = {"achieved": round(va, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "T VALU-op/s",
                     "frac": round(va / VALU_PEAK_TOPS, 4)}
    return r


def step_roof(work, step_seconds, measured):
    """T_bound / T_measured for a whole step: T_bound = max(compulsory bytes /
    measured stream bandwidth, multiplies / measured multiply rate)."""
    t_bw = work.nbytes / (measured["hbm_copy_gbs"] * 1e9)
    t_mul = work.muls / (measured["mul_mix_tops"] * 1e12)
    t_valu = work.valu / (VALU_PEAK_TOPS * 1e12)
    t_bound = max(t_bw, t_mul)
    return {"bound": "hbm" if t_bw >= t_mul else "alu", "t_bound_ms": round(t_bound * 1e3, 4),
            "t_measured_ms": round(step_seconds * 1e3, 4), "frac": round(t_bound / step_seconds, 4),
            "t_hbm_ms": round(t_bw * 1e3, 4), "t_mul_ms": round(t_mul * 1e3, 4),
            "valu_frac": round(t_valu / step_seconds, 4), **work.as_dict()}


_TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                             "traffic.json")


def source_digest():
    """Hash of the kernel sources; stored traffic figures are void once it changes."""
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sorted(os.listdir(csrc)):
        if f == "microbench.hip":
            continue
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
