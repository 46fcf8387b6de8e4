"""CPU oracle for the negacyclic NTT path -- test infrastructure only.

Plain, slow, obviously correct reference implementation of what the GPU
library computes (arXiv 2109.14704, section II-A and section II-B).  It shares
no code with the GPU library.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.

The arithmetic lives in ``oracle.c`` (exact ``unsigned __int128`` products and
``%``), compiled with gcc into ``liboracle.so``; ``tiny.py`` holds a pure-Python
copy of the definitions for N <= 64 that cross-checks the C code.

Parity pins (tests/test_oracle.py): hand-derived N=2 and N=4 examples, the
O(N^2) definitions against the radix-2 algorithms, the pure-Python copy,
closed forms for monomials, the convolution theorem against the schoolbook
product, round trips, and twiddle-order invariants.  No function here is
parity-unpinned.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

U64 = ctypes.c_uint64
U32 = ctypes.c_uint32
P64 = ctypes.POINTER(ctypes.c_uint64)


def build(force=False):
    """Compile liboracle.so with gcc (OpenMP over (batch, limb))."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        sig = {
            "or_mulmod": (U64, [U64, U64, U64]),
            "or_addmod": (U64, [U64, U64, U64]),
            "or_submod": (U64, [U64, U64, U64]),
            "or_powmod": (U64, [U64, U64, U64]),
            "or_invmod": (U64, [U64, U64]),
            "or_is_prime": (ctypes.c_int, [U64]),
            "or_gen_primes": (ctypes.c_int, [U32, U64, U32, P64, U32]),
            "or_bitrev": (U32, [U32, U32]),
            "or_psi": (U64, [U64, U32]),
            "or_psi_tables": (None, [U64, U32, U64, P64, P64]),
            "or_dft_fwd": (None, [P64, P64, U32, U64, U64]),
            "or_dft_inv": (None, [P64, P64, U32, U64, U64]),
            "or_ntt_fwd_point": (U64, [P64, U32, U64, U64, U32]),
            "or_ntt_inv_point": (U64, [P64, U32, U64, U64, U32]),
            "or_negacyclic_schoolbook": (None, [P64, P64, P64, U32, U64]),
            "or_negacyclic_point": (U64, [P64, P64, U32, U64, U32]),
            "or_ntt_fwd_r2": (None, [P64, U32, U64, P64]),
            "or_ntt_inv_r2": (None, [P64, U32, U64, P64]),
            "or_max_threads": (ctypes.c_int, []),
            "or_batch_ntt": (ctypes.c_int, [P64, U32, U32, U32, P64, ctypes.c_int, ctypes.c_int]),
            "or_batch_dyadic": (None, [P64, P64, P64, U32, U32, U32, P64]),
            "or_batch_tensor": (None, [P64, P64, P64, U32, U32, U32, P64]),
            "or_batch_rescale": (None, [P64, P64, U32, U32, U32, P64]),
            "or_ct_matmul": (None, [P64, P64, P64, U32, U32, U32, U32, U32, P64]),
            "or_relin": (ctypes.c_int, [P64, P64, P64, U32, U32, U32, P64, ctypes.c_int]),
            "or_batch_polymul": (ctypes.c_int, [P64, P64, P64, U32, U32, U32, P64, ctypes.c_int]),
            "or_batch_ct_tensor_coeff": (ctypes.c_int, [P64, P64, P64, U32, U32, U32, P64, ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(P64)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


# ---- scalar helpers -----------------------------------------------------------------
def mulmod(a, b, q): return int(lib().or_mulmod(a, b, q))
def powmod(a, e, q): return int(lib().or_powmod(a, e, q))
def invmod(a, q): return int(lib().or_invmod(a, q))
def is_prime(n): return bool(lib().or_is_prime(n))
def bitrev(x, bits): return int(lib().or_bitrev(x, bits))
def psi(q, log_n): return int(lib().or_psi(q, log_n))


def gen_primes(bits, M, count, exclude=()):
    """Largest primes < 2^bits that are 1 mod M, skipping ``exclude``."""
    buf = np.zeros(len(exclude) + count, dtype=np.uint64)
    buf[: len(exclude)] = list(exclude)
    got = lib().or_gen_primes(bits, M, count, _p(buf), len(exclude))
    return [int(v) for v in buf[len(exclude): len(exclude) + got]]


def psi_tables(q, log_n):
    n = 1 << log_n
    f = np.zeros(n, dtype=np.uint64)
    i = np.zeros(n, dtype=np.uint64)
    lib().or_psi_tables(q, log_n, psi(q, log_n), _p(f), _p(i))
    return f, i


# ---- single-polynomial transforms ---------------------------------------------------
def dft_fwd(a, q, log_n):
    a = _u64(a); out = np.zeros_like(a)
    lib().or_dft_fwd(_p(a), _p(out), log_n, q, psi(q, log_n))
    return out


def dft_inv(A, q, log_n):
    A = _u64(A); out = np.zeros_like(A)
    lib().or_dft_inv(_p(A), _p(out), log_n, q, psi(q, log_n))
    return out


def ntt_fwd_r2(a, q, log_n):
    a = _u64(a).copy(); f, _ = psi_tables(q, log_n)
    lib().or_ntt_fwd_r2(_p(a), log_n, q, _p(f))
    return a


def ntt_inv_r2(A, q, log_n):
    A = _u64(A).copy(); _, i = psi_tables(q, log_n)
    lib().or_ntt_inv_r2(_p(A), log_n, q, _p(i))
    return A


def ntt_fwd_point(a, q, log_n, k, psi_val=None):
    a = _u64(a)
    return int(lib().or_ntt_fwd_point(_p(a), log_n, q, psi_val or psi(q, log_n), k))


def ntt_inv_point(A, q, log_n, i, psi_val=None):
    A = _u64(A)
    return int(lib().or_ntt_inv_point(_p(A), log_n, q, psi_val or psi(q, log_n), i))


def negacyclic_schoolbook(a, b, q):
    a = _u64(a); b = _u64(b); out = np.zeros_like(a)
    lib().or_negacyclic_schoolbook(_p(a), _p(b), _p(out), a.size, q)
    return out


def negacyclic_point(a, b, q, k):
    a = _u64(a); b = _u64(b)
    return int(lib().or_negacyclic_point(_p(a), _p(b), a.size, q, k))


# ---- batched forms over [batch][limbs][N] --------------------------------------------
def _moduli(moduli):
    return np.ascontiguousarray(np.asarray(moduli, dtype=np.uint64))


def batch_ntt(x, moduli, direction, threads=0):
    """Transform x[..., limbs, N] (copy); direction +1 forward, -1 inverse."""
    x = _u64(x).copy(); m = _moduli(moduli)
    limbs, n = x.shape[-2], x.shape[-1]
    log_n = n.bit_length() - 1
    batch = x.size // (limbs * n)
    rc = lib().or_batch_ntt(_p(x), batch, limbs, log_n, _p(m), int(direction), int(threads))
    if rc:
        raise ValueError("oracle: no primitive 2N-th root for some modulus")
    return x


def batch_dyadic(a, b, moduli):
    a = _u64(a); b = _u64(b); out = np.zeros_like(a); m = _moduli(moduli)
    limbs, n = a.shape[-2], a.shape[-1]
    lib().or_batch_dyadic(_p(a), _p(b), _p(out), a.size // (limbs * n), limbs, n, _p(m))
    return out


def batch_tensor(c, d, moduli):
    """c, d [batch][2][limbs][N] in the NTT domain -> [batch][3][limbs][N]."""
    c = _u64(c); d = _u64(d); m = _moduli(moduli)
    batch, two, limbs, n = c.shape
    out = np.zeros((batch, 3, limbs, n), dtype=np.uint64)
    lib().or_batch_tensor(_p(c), _p(d), _p(out), batch, limbs, n, _p(m))
    return out


def batch_polymul(a, b, moduli, threads=0):
    a = _u64(a); b = _u64(b); out = np.zeros_like(a); m = _moduli(moduli)
    limbs, n = a.shape[-2], a.shape[-1]
    rc = lib().or_batch_polymul(_p(a), _p(b), _p(out), a.size // (limbs * n), limbs, n.bit_length() - 1,
                                _p(m), int(threads))
    if rc:
        raise ValueError("oracle: bad modulus")
    return out


def batch_ct_tensor_coeff(c, d, moduli, threads=0):
    c = _u64(c); d = _u64(d); m = _moduli(moduli)
    batch, two, limbs, n = c.shape
    out = np.zeros((batch, 3, limbs, n), dtype=np.uint64)
    rc = lib().or_batch_ct_tensor_coeff(_p(c), _p(d), _p(out), batch, limbs, n.bit_length() - 1, _p(m),
                                        int(threads))
    if rc:
        raise ValueError("oracle: bad modulus")
    return out


def batch_rescale(x, moduli):
    """Rescale of section II-A (drop the last prime with rounding), coefficient
    domain: x [batch][limbs][N] over moduli[:limbs] -> [batch][limbs - 1][N]."""
    x = _u64(x); m = _moduli(moduli)
    batch, limbs, n = x.shape
    if limbs < 2:
        raise ValueError("oracle: rescale needs at least two limbs")
    out = np.zeros((batch, limbs - 1, n), dtype=np.uint64)
    lib().or_batch_rescale(_p(x), _p(out), batch, limbs, n, _p(m[:limbs]))
    return out


def batch_rescale_ntt(c, moduli):
    """Rescale of NTT-domain ciphertext limbs: the coefficient-domain rescale
    between an inverse and a forward transform."""
    c = _u64(c)
    limbs = c.shape[1]
    x = batch_ntt(c, moduli[:limbs], -1)
    return batch_ntt(batch_rescale(x, moduli[:limbs]), moduli[:limbs - 1], +1)


def ct_matmul(A, B, C, moduli):
    """C + A * B for ciphertext matrices in the NTT domain (section IV-E):
    A [m][k][2][limbs][N], B [k][n][2][limbs][N], C [m][n][3][limbs][N]."""
    A = _u64(A); B = _u64(B); out = _u64(C).copy(); m_ = _moduli(moduli)
    m, k, _, limbs, n_ = A.shape
    n = B.shape[1]
    if B.shape != (k, n, 2, limbs, n_) or out.shape != (m, n, 3, limbs, n_):
        raise ValueError("oracle: matmul shapes")
    lib().or_ct_matmul(_p(A), _p(B), _p(out), m, n, k, limbs, n_, _p(m_[:limbs]))
    return out


def relin(c, ksk, moduli, threads=0):
    """Relinearization of section II-A with the RNS digit decomposition, NTT
    domain: c [batch][3][l][N], ksk [l][2][l + 1][N] over moduli[:l + 1] (the
    last one the special prime P) -> [batch][2][l][N]."""
    c = _u64(c); ksk = _u64(ksk); m = _moduli(moduli)
    batch, three, l, n = c.shape
    if three != 3 or ksk.shape != (l, 2, l + 1, n) or len(m) < l + 1:
        raise ValueError("oracle: relin shapes")
    out = np.zeros((batch, 2, l, n), dtype=np.uint64)
    rc = lib().or_relin(_p(c), _p(ksk), _p(out), batch, l, n.bit_length() - 1, _p(m[:l + 1]), int(threads))
    if rc:
        raise ValueError("oracle: bad modulus")
    return out


def max_threads():
    return int(lib().or_max_threads())
