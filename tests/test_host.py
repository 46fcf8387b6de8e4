"""CPU-only checks of the library's host side and of its arithmetic.

- the C-ABI library loads and exports every symbol include/hentt.h declares;
- argument and modulus validation returns the documented status codes
  (these paths return before any device work);
- the library's psi agrees with the oracle's for every modulus chain;
- the device modular arithmetic, built for the host, keeps Algorithm 1's
  contracts and matches exact 128-bit arithmetic.
"""
import ctypes
import os
import re
import subprocess

import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hentt.h")


def _lib():
    import paper_2109_14704_amd as H
    return H, H.lib()


def test_exports_every_declared_symbol():
    H, L = _lib()
    names = set(re.findall(r"\b(hentt_[a-z_0-9]+)\s*\(", open(HEADER).read()))
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(L, n), n


def test_psi_agrees_with_oracle():
    H, _ = _lib()
    for name in ["plain4096", "ckks_level", "ct_tensor", "uneven"]:
        for q in workloads.moduli(name):
            for ln in range(6, 18):
                if (q - 1) % (2 << ln) == 0:
                    assert H.psi(q, ln) == oracle.psi(q, ln), (name, q, ln)


def test_status_codes():
    H, L = _lib()
    U64 = ctypes.c_uint64
    out = ctypes.c_void_p()
    good = workloads.moduli("uneven")[0]

    def create(log_n, mods):
        arr = (U64 * max(1, len(mods)))(*mods)
        return L.hentt_tables_create(log_n, len(mods), arr, None, ctypes.byref(out))

    assert create(5, [good]) == -1          # log_n below range
    assert create(18, [good]) == -1         # log_n above range
    assert create(12, []) == -1             # zero limbs
    assert create(12, [good + 2]) == -2     # not 1 mod 2N / not prime
    assert create(12, [(1 << 60) + 1]) == -2   # 1 mod 2N but >= 2^60
    composite = 8193 * 16385                    # 1 mod 8192, composite
    assert (composite - 1) % 8192 == 0 and create(12, [composite]) == -2
    assert create(12, [97]) == -2           # below 2^7 / not 1 mod 8192
    assert L.hentt_tables_create(12, 1, None, None, ctypes.byref(out)) == -1
    assert L.hentt_ntt_fwd(None, None, 1, None) == -1
    assert L.hentt_ntt_inv(None, None, 1, None) == -1
    assert L.hentt_dyadic_mul(None, None, None, None, 1, None) == -1
    assert L.hentt_polymul(None, None, None, None, 1, None) == -1
    assert L.hentt_ct_tensor(None, None, None, None, 1, 0, None) == -1
    assert L.hentt_ct_tensor_grouped(None, 0, 0, None) == 0            # no jobs: nothing to do
    assert L.hentt_ct_tensor_grouped(None, 1, 0, None) == -1
    jobs = (H._CtJob * 2)()                                             # zeroed: NULL pointers
    assert L.hentt_ct_tensor_grouped(jobs, 2, 0, None) == -1
    assert L.hentt_ct_tensor_grouped(jobs, 2, 4, None) == -1            # unknown flag
    assert L.hentt_ntt_batch(None, 0, 1, None) == -1
    assert L.hentt_tables_destroy(None) == -1
    assert L.hentt_check_canonical(None, None, 1, None, None, None) == -1
    assert L.hentt_ntt_batch_status(None, 0, 1) == -1
    assert L.hentt_batch_plan_set_grid(None, 1) == -1
    assert L.hentt_batch_plan_destroy(None) == -1
    assert L.hentt_graph_launch(None, None) == -1
    assert L.hentt_pool_bytes(None) == -1
    n = ctypes.c_uint64(1)
    assert L.hentt_pool_bytes(ctypes.byref(n)) == 0 and n.value == 0     # nothing allocated on the CPU
    assert L.hentt_rescale(None, None, None, 1, 0, None) == -1
    assert L.hentt_relin(None, None, None, None, 1, None) == -1
    assert L.hentt_ct_matmul(None, None, None, None, 1, 1, 1, None) == -1
    assert L.hentt_status_str(-2).decode().startswith("bad modulus")
    assert "graphs" in L.hentt_status_str(-6).decode()
    assert "[0, q)" in L.hentt_status_str(-7).decode()
    with pytest.raises(H.HenttError):
        H.psi(good + 2, 12)


def test_device_arithmetic_on_host(tmp_path):
    exe = str(tmp_path / "host_modarith")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(ROOT, "tests", "host_modarith.cpp")])
    r = subprocess.run([exe, "300000"], stdout=subprocess.PIPE, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout


def test_roofline_accounting_reproduces_table_one():
    from paper_2109_14704_amd import roofline
    # section IV-B: naive radix-2 density 1.5, staged radix-8 SLM density 8.9 at N = 32K
    assert roofline.paper_density("naive", 1 << 15) == pytest.approx(1.5)
    assert roofline.paper_density("radix8_slm", 1 << 15) == pytest.approx(8.906, abs=1e-3)


def test_tuning_abi_host_only():
    """The autotuner's instance lists and selections (host-only calls)."""
    H, L = _lib()
    assert H.tune_count("fwd", 12) == 1 and H.tune_count("fwd", 15) >= 3 and H.tune_count("tensor", 16) >= 2
    # instance 0 of every op is the library's default stage split
    for ln in range(6, 18):
        tc, pc = H.stage_split(ln)
        assert H.tune_describe("fwd", ln, 0, cols=True)[1] == tc
        assert H.tune_describe("polymul", ln, 0, cols=True)[1] == pc
    assert [H.shape_class(u) for u in (1, 63, 64, 1023, 1024, 10 ** 6)] == [0, 0, 1, 1, 2, 2]
    H.tune_select("inv", 16, 1, 2)
    assert H.tune_get("inv", 16, 1) == 2 and H.tune_get("inv", 16, 0) == 0 and H.tune_get("fwd", 16, 1) == 0
    H.tune_select("inv", 16, 1, 0)
    U32 = ctypes.c_uint32
    c = U32()
    assert L.hentt_tune_count(4, 15, ctypes.byref(c)) == -1            # unknown op
    assert L.hentt_tune_count(0, 18, ctypes.byref(c)) == -1            # log_n out of range
    assert L.hentt_tune_select(0, 15, 3, 0) == -1                      # no such class
    assert L.hentt_tune_select(0, 15, 0, H.tune_count("fwd", 15)) == -1
    assert L.hentt_tune_describe(0, 15, 0, None, 0, None) == -1


def test_roctx_ranges_and_tune_mode_host_only(tmp_path):
    """HENTT_ROCTX=1 opens the roctx library and brackets entry points (an
    invalid call still returns its status); HENTT_TUNE accepts its modes only."""
    import subprocess
    import sys
    code = ("import ctypes, sys; sys.path.insert(0, %r); import paper_2109_14704_amd as H; "
            "L = H.lib(); print(L.hentt_ntt_fwd(None, None, 1, None), L.hentt_ct_tensor_grouped(None, 1, 0, None))" % ROOT)
    env = dict(os.environ, HENTT_ROCTX="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["-1", "-1"]
    from paper_2109_14704_amd import autotune
    os.environ["HENTT_TUNE"] = "bogus"
    try:
        with pytest.raises(ValueError):
            autotune.tune_mode()
        for m in ("cached", "force", "off"):
            os.environ["HENTT_TUNE"] = m
            assert autotune.tune_mode() == m
    finally:
        del os.environ["HENTT_TUNE"]
