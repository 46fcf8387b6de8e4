"""Measured rates behind the benchmark's roofline: HBM stream bandwidth and the
VALU issue rate of the 32-bit integer multiplies the modular arithmetic is
built from (csrc/microbench.hip, built into libhentt_mb.so).

All rates come from HIP events on torch's current stream around launches of
known work:
  * hbm_copy: each byte of a 4 GiB buffer read once and written once (the
    best of streaming and ordinary accesses over a few grid sizes);
  * hbm_read: each byte read once;
  * mad64 / mulhi / mullo / add: lane-operations per second of
    v_mad_u64_u32, v_mul_hi_u32, v_mul_lo_u32, v_add_u32;
  * add64 / cmp64 / add3 / mov: the same for the other instructions the
    butterflies issue (v_lshl_add_u64, v_cmp_lt_u64, v_add3_u32, v_mov_b32);
  * mul_mix: the rate of the Shoup butterfly's own multiply mix (3
    v_mad_u64_u32, 2 v_mul_hi_u32, 4 v_mul_lo_u32 per butterfly), i.e. nine
    multiplies in the time the three measured rates give them;
  * bfly: Shoup forward butterflies per second, the library's own lazy
    butterfly on registers with no memory traffic.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhentt_mb.so")
_lib = None

MB_MAD64, MB_MULHI, MB_MULLO, MB_ADD, MB_BFLY, MB_ADD64, MB_CMP64, MB_ADD3, MB_MOV = range(9)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhentt_mb.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        VP, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.mb_copy.argtypes = [VP, VP, U64, U32, ctypes.c_int, VP]
        L.mb_read.argtypes = [VP, U64, VP, U32, VP]
        L.mb_issue.argtypes = [ctypes.c_int, VP, U32, U32, U32, U64, U64, U64, VP]
        for f in (L.mb_copy, L.mb_read, L.mb_issue):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _timed(fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def _cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


def hbm_copy_gbs(nbytes=4 << 30, reps=5, detail=None):
    """Best copy rate (bytes read + written per second) over streaming and
    ordinary accesses and a few grid sizes; `detail` (a dict) receives every
    configuration's rate."""
    src = torch.arange(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    L = lib()
    best = 0.0
    for nt in (1, 0):
        for per_cu in (4, 8, 16):
            grid = _cus() * per_cu

            def run():
                assert L.mb_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes, grid, nt,
                                 _stream()) == 0

            gbs = 2 * nbytes / _timed(run, reps) / 1e9
            if detail is not None:
                detail["copy_%s_%dpercu" % ("nt" if nt else "plain", per_cu)] = round(gbs, 1)
            best = max(best, gbs)
    assert torch.equal(src, dst)
    return best


def hbm_read_gbs(nbytes=4 << 30, reps=5):
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    grid = _cus() * 8
    out = torch.empty(grid * 256, dtype=torch.int64, device="cuda")
    L = lib()

    def run():
        assert L.mb_read(ctypes.c_void_p(src.data_ptr()), nbytes, ctypes.c_void_p(out.data_ptr()), grid, _stream()) == 0

    s = _timed(run, reps)
    return nbytes / s / 1e9


def issue_rate(kind, iters=None, reps=3):
    """Lane-operations (or butterflies, for MB_BFLY) per second."""
    grid = _cus() * 8
    out = torch.empty(grid * 256, dtype=torch.int64, device="cuda")
    iters = iters or (4000 if kind == MB_BFLY else 60000)
    L = lib()
    q = (1 << 55) - (1 << 22) + 1        # odd 55-bit modulus: the butterfly's timing does not depend on primality
    w = 12345678901234 % q
    ws = (w << 64) // q

    def run():
        assert L.mb_issue(kind, ctypes.c_void_p(out.data_ptr()), iters, grid, 0x9E3779B9, w, ws, q, _stream()) == 0

    s = _timed(run, reps)
    return grid * 256 * 8 * iters / s


def measure_all(detail=None):
    r = {
        "hbm_copy_gbs": hbm_copy_gbs(detail=detail),
        "hbm_read_gbs": hbm_read_gbs(),
        "mad64_tops": issue_rate(MB_MAD64) / 1e12,
        "mulhi_tops": issue_rate(MB_MULHI) / 1e12,
        "mullo_tops": issue_rate(MB_MULLO) / 1e12,
        "add_tops": issue_rate(MB_ADD) / 1e12,
        "add64_tops": issue_rate(MB_ADD64) / 1e12,
        "cmp64_tops": issue_rate(MB_CMP64) / 1e12,
        "add3_tops": issue_rate(MB_ADD3) / 1e12,
        "mov_tops": issue_rate(MB_MOV) / 1e12,
        "bfly_gbfly_s": issue_rate(MB_BFLY) / 1e9,
    }
    # the butterfly's nine multiplies at the measured rates of their kinds
    t9 = 3 / r["mad64_tops"] + 2 / r["mulhi_tops"] + 4 / r["mullo_tops"]
    r["mul_mix_tops"] = 9 / t9
    return {k: round(v, 3) for k, v in r.items()}


if __name__ == "__main__":
    import json
    print(json.dumps(measure_all()))
