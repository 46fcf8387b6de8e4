"""hentt: batched negacyclic NTT over RNS limbs on AMD MI355X (gfx950).

Python binding of libhentt.so (C ABI in include/hentt.h).  Argument
marshalling only: shapes, dtypes and device pointers are checked here and
every step of the computation runs in the library's HIP kernels.  PyTorch
supplies device memory (int64 or uint64 tensors used as raw 64-bit words)
and streams.  If the library is not built, every call raises HenttError.
"""
import ctypes
import os

import torch

__all__ = ["HenttError", "Tables", "ntt_fwd", "ntt_inv", "dyadic_mul", "polymul", "ct_tensor", "ntt_batch",
           "psi", "lib", "LIB_PATH", "prof_enable", "prof_read", "BatchPlan", "stage_split", "ntt_fwd_variant",
           "rescale", "ct_matmul", "relin", "check_canonical", "ntt_batch_status", "pool_bytes", "pool_trim",
           "NonCanonicalError", "ct_tensor_grouped", "tune_count", "tune_describe", "shape_class", "tune_select", "tune_get", "TUNE_OPS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HENTT_LIB") or os.path.join(_HERE, "libhentt.so")  # HENTT_LIB: alternative build

HENTT_IN_NTT = 1
HENTT_OUT_NTT = 2
_VP = ctypes.c_void_p
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64


class HenttError(RuntimeError):
    pass


class NonCanonicalError(HenttError):
    """Raised by check_canonical: input words outside [0, q)."""


class _Job(ctypes.Structure):
    _fields_ = [("data", _VP), ("t", _VP), ("limbs", _U32), ("batch", _U32)]


class _CtJob(ctypes.Structure):
    _fields_ = [("c", _VP), ("d", _VP), ("out", _VP), ("t", _VP), ("batch", _U32), ("reserved", _U32)]


_lib = None


def lib():
    """Load libhentt.so (built by __graft_entry__.build()); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HenttError("libhentt.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        sigs = {
            "hentt_tables_create": [_U32, _U32, ctypes.POINTER(_U64), _VP, ctypes.POINTER(_VP)],
            "hentt_tables_destroy": [_VP],
            "hentt_tables_view": [_VP, _U32, ctypes.POINTER(_VP)],
            "hentt_tables_info": [_VP, ctypes.POINTER(_U32), ctypes.POINTER(_U32)],
            "hentt_tables_device_ptrs": [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP)],
            "hentt_psi": [_U64, _U32, ctypes.POINTER(_U64)],
            "hentt_ntt_fwd": [_VP, _VP, _U32, _VP],
            "hentt_ntt_fwd_variant": [_VP, _VP, _U32, ctypes.c_int, _VP],
            "hentt_rescale": [_VP, _VP, _VP, _U32, _U32, _VP],
            "hentt_ct_matmul": [_VP, _VP, _VP, _VP, _U32, _U32, _U32, _VP],
            "hentt_relin": [_VP, _VP, _VP, _VP, _U32, _VP],
            "hentt_ntt_inv": [_VP, _VP, _U32, _VP],
            "hentt_dyadic_mul": [_VP, _VP, _VP, _VP, _U32, _VP],
            "hentt_polymul": [_VP, _VP, _VP, _VP, _U32, _VP],
            "hentt_ct_tensor": [_VP, _VP, _VP, _VP, _U32, _U32, _VP],
            "hentt_ct_tensor_grouped": [ctypes.POINTER(_CtJob), _U32, _U32, _VP],
            "hentt_ntt_batch": [ctypes.POINTER(_Job), _U32, ctypes.c_int, _VP],
            "hentt_ntt_batch_status": [ctypes.POINTER(_Job), _U32, ctypes.c_int],
            "hentt_check_canonical": [_VP, _VP, _U32, ctypes.POINTER(_U64), ctypes.POINTER(_U64), _VP],
            "hentt_pool_bytes": [ctypes.POINTER(_U64)],
            "hentt_pool_trim": [],
            "hentt_last_hip_error": [],
            "hentt_batch_plan_create": [ctypes.POINTER(_Job), _U32, ctypes.c_int, ctypes.POINTER(_VP)],
            "hentt_batch_plan_set_grid": [_VP, _U32],
            "hentt_batch_plan_set_schedule": [_VP, _U32, _U32],
            "hentt_batch_plan_info": [_VP, ctypes.POINTER(_U32), ctypes.POINTER(_U32), ctypes.POINTER(_U32)],
            "hentt_batch_plan_run": [_VP, _VP],
            "hentt_batch_plan_status": [_VP],
            "hentt_batch_plan_destroy": [_VP],
            "hentt_batch_graph_create": [_VP, ctypes.POINTER(_VP)],
            "hentt_graph_launch": [_VP, _VP],
            "hentt_graph_destroy": [_VP],
            "hentt_stage_split": [_U32, ctypes.POINTER(_U32), ctypes.POINTER(_U32)],
            "hentt_tune_count": [ctypes.c_int, _U32, ctypes.POINTER(_U32)],
            "hentt_tune_describe": [ctypes.c_int, _U32, _U32, ctypes.c_char_p, _U32, ctypes.POINTER(_U32)],
            "hentt_tune_class": [_U64, ctypes.POINTER(_U32)],
            "hentt_tune_select": [ctypes.c_int, _U32, _U32, _U32],
            "hentt_tune_get": [ctypes.c_int, _U32, _U32, ctypes.POINTER(_U32)],
            "hentt_prof_enable": [ctypes.c_int],
            "hentt_prof_count": [],
            "hentt_prof_get": [_U32, ctypes.c_char_p, _U32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_U32)],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.hentt_status_str.argtypes = [ctypes.c_int]
        L.hentt_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        L = lib()
        msg = L.hentt_status_str(rc).decode()
        if rc == -4:
            msg += " (hipError %d)" % L.hentt_last_hip_error()
        raise HenttError("%s failed: %s [%d]" % (what, msg, rc))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return _VP(stream.cuda_stream)
    return _VP(int(stream))


def _words(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HenttError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype not in (torch.int64, torch.uint64):
        raise HenttError("%s must be int64 or uint64 (64-bit words), got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise HenttError("%s must be contiguous" % name)
    return _VP(t.data_ptr())


def prof_enable(on=True):
    """Start (clearing old records) or stop per-kernel event timing."""
    _check(lib().hentt_prof_enable(1 if on else 0), "hentt_prof_enable")


def prof_read():
    """Wait for the timed launches; {kernel name: (total_ms, launches)}."""
    L = lib()
    n = L.hentt_prof_count()
    if n < 0:
        _check(n, "hentt_prof_count")
    out = {}
    buf = ctypes.create_string_buffer(128)
    for i in range(n):
        ms, cnt = ctypes.c_double(), _U32()
        _check(L.hentt_prof_get(i, buf, 128, ctypes.byref(ms), ctypes.byref(cnt)), "hentt_prof_get")
        out[buf.value.decode()] = (ms.value, cnt.value)
    return out


def stage_split(log_n):
    """(column stages of a plain transform, column stages of a fused product); 0 = whole."""
    a, b = _U32(), _U32()
    _check(lib().hentt_stage_split(log_n, ctypes.byref(a), ctypes.byref(b)), "hentt_stage_split")
    return a.value, b.value


# Operations with tunable kernel instances (hentt_tune_*).
TUNE_OPS = {"fwd": 0, "inv": 1, "polymul": 2, "tensor": 3}


def _op(op):
    return TUNE_OPS[op] if isinstance(op, str) else int(op)


def tune_count(op, log_n):
    """Number of compiled kernel instances of op ("fwd", "inv", "polymul", "tensor") at N = 2^log_n."""
    n = _U32()
    _check(lib().hentt_tune_count(_op(op), log_n, ctypes.byref(n)), "hentt_tune_count")
    return n.value


def tune_describe(op, log_n, choice, cols=False):
    """Text of instance `choice`; with cols=True, (text, column-pass stages)."""
    buf = ctypes.create_string_buffer(128)
    c = _U32()
    _check(lib().hentt_tune_describe(_op(op), log_n, choice, buf, 128, ctypes.byref(c)), "hentt_tune_describe")
    return (buf.value.decode(), c.value) if cols else buf.value.decode()


def shape_class(units):
    """The library's shape class of a call over `units` (batch x limbs) units."""
    c = _U32()
    _check(lib().hentt_tune_class(int(units), ctypes.byref(c)), "hentt_tune_class")
    return c.value


def tune_select(op, log_n, cls, choice):
    """Use instance `choice` for op at N = 2^log_n and shape class `cls` from now on."""
    _check(lib().hentt_tune_select(_op(op), log_n, cls, choice), "hentt_tune_select")


def tune_get(op, log_n, cls):
    c = _U32()
    _check(lib().hentt_tune_get(_op(op), log_n, cls, ctypes.byref(c)), "hentt_tune_get")
    return c.value


def psi(q, log_n):
    """The library's psi: smallest primitive 2N-th root of unity mod q."""
    out = _U64()
    _check(lib().hentt_psi(q, log_n, ctypes.byref(out)), "hentt_psi")
    return out.value


class Tables:
    """Device twiddle tables for a modulus chain at N = 2^log_n."""

    def __init__(self, log_n, moduli, stream=None, _handle=None):
        self._h = None
        if _handle is not None:
            self._h = _handle
        else:
            arr = (_U64 * len(moduli))(*[int(m) for m in moduli])
            h = _VP()
            _check(lib().hentt_tables_create(log_n, len(moduli), arr, _stream(stream), ctypes.byref(h)),
                   "hentt_tables_create")
            self._h = h
        ln, lm = _U32(), _U32()
        _check(lib().hentt_tables_info(self._h, ctypes.byref(ln), ctypes.byref(lm)), "hentt_tables_info")
        self.log_n, self.limbs = ln.value, lm.value
        self.n = 1 << self.log_n

    def view(self, limbs):
        h = _VP()
        _check(lib().hentt_tables_view(self._h, limbs, ctypes.byref(h)), "hentt_tables_view")
        return Tables(None, None, _handle=h)

    def device_ptrs(self):
        f, i, m = _VP(), _VP(), _VP()
        _check(lib().hentt_tables_device_ptrs(self._h, ctypes.byref(f), ctypes.byref(i), ctypes.byref(m)),
               "hentt_tables_device_ptrs")
        return f.value, i.value, m.value

    def close(self):
        if self._h is not None and _lib is not None:
            lib().hentt_tables_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def _batch_of(tables, x, per_item=1, name="x"):
    if x.dim() < 2 or x.shape[-1] != tables.n or x.shape[-2] != tables.limbs:
        raise HenttError("%s must have shape [..., limbs=%d, N=%d], got %s" % (name, tables.limbs, tables.n,
                                                                               tuple(x.shape)))
    b = x.numel() // (tables.limbs * tables.n * per_item)
    if b * per_item * tables.limbs * tables.n != x.numel() or b == 0:
        raise HenttError("%s: size is not a whole number of items" % name)
    return b


def check_canonical(tables, x, stream=None):
    """Debug check that every word of x[..., limbs, N] is below its limb's
    modulus.  Synchronises the stream.  Returns None, or raises
    NonCanonicalError naming the count and the first offending flat index."""
    bad, first = _U64(), _U64()
    rc = lib().hentt_check_canonical(tables.handle, _words(x, "x"), _batch_of(tables, x), ctypes.byref(bad),
                                     ctypes.byref(first), _stream(stream))
    if rc == -7:
        raise NonCanonicalError("%d words outside [0, q); first at flat index %d" % (bad.value, first.value))
    _check(rc, "hentt_check_canonical")


def pool_bytes():
    """Device bytes held by the library's workspace pool."""
    n = _U64()
    _check(lib().hentt_pool_bytes(ctypes.byref(n)), "hentt_pool_bytes")
    return n.value


def pool_trim():
    """Free the pool's idle workspace buffers (after their streams finish)."""
    _check(lib().hentt_pool_trim(), "hentt_pool_trim")


def ntt_fwd(tables, x, stream=None):
    """In-place forward negacyclic NTT of x[..., limbs, N] (bit-reversed output)."""
    _check(lib().hentt_ntt_fwd(tables.handle, _words(x, "x"), _batch_of(tables, x), _stream(stream)),
           "hentt_ntt_fwd")
    return x


def rescale(tables, c, out=None, ntt=False, stream=None):
    """Rescale (RS of section II-A): c [batch, limbs, N] at the tables' level
    (limbs >= 2) -> [batch, limbs - 1, N] = round(c / q_last) per remaining
    limb.  ntt: NTT-domain input and output (else coefficient domain)."""
    if c.dim() != 3:
        raise HenttError("c must have shape [batch, limbs, N]")
    batch = _batch_of(tables, c, name="c")
    if out is None:
        out = torch.empty((batch, tables.limbs - 1, tables.n), dtype=c.dtype, device=c.device)
    elif tuple(out.shape) != (batch, tables.limbs - 1, tables.n):
        raise HenttError("out must have shape [%d, %d, %d]" % (batch, tables.limbs - 1, tables.n))
    flags = (HENTT_IN_NTT | HENTT_OUT_NTT) if ntt else 0
    _check(lib().hentt_rescale(tables.handle, _words(c, "c"), _words(out, "out"), batch, flags, _stream(stream)),
           "hentt_rescale")
    return out


def ct_matmul(tables, A, B, C, stream=None):
    """C += A * B for ciphertext matrices in the NTT domain (section IV-E):
    A [m, k, 2, limbs, N], B [k, n, 2, limbs, N], C [m, n, 3, limbs, N]; C in place."""
    L, n_ = tables.limbs, tables.n
    if A.dim() != 5 or B.dim() != 5 or C.dim() != 5:
        raise HenttError("A, B, C must be 5-dimensional ciphertext matrices")
    m, k = A.shape[0], A.shape[1]
    n = B.shape[1]
    if (tuple(A.shape) != (m, k, 2, L, n_) or tuple(B.shape) != (k, n, 2, L, n_)
            or tuple(C.shape) != (m, n, 3, L, n_)):
        raise HenttError("shapes: A [m,k,2,%d,%d], B [k,n,2,%d,%d], C [m,n,3,%d,%d]" % (L, n_, L, n_, L, n_))
    _check(lib().hentt_ct_matmul(tables.handle, _words(A, "A"), _words(B, "B"), _words(C, "C"), m, n, k,
                                 _stream(stream)), "hentt_ct_matmul")
    return C


def relin(tables, c, ksk, out=None, stream=None):
    """Relinearization (section II-A) with the RNS digit key switch, NTT domain.
    tables: l + 1 limbs, the ciphertext's primes then the special prime P;
    c [batch, 3, l, N]; ksk [l, 2, l + 1, N] -> out [batch, 2, l, N]."""
    l, n_ = tables.limbs - 1, tables.n
    if c.dim() != 4 or c.shape[1:] != (3, l, n_):
        raise HenttError("c must have shape [batch, 3, %d, %d]" % (l, n_))
    if tuple(ksk.shape) != (l, 2, l + 1, n_):
        raise HenttError("ksk must have shape [%d, 2, %d, %d]" % (l, l + 1, n_))
    batch = c.shape[0]
    if out is None:
        out = torch.empty((batch, 2, l, n_), dtype=c.dtype, device=c.device)
    elif tuple(out.shape) != (batch, 2, l, n_):
        raise HenttError("out must have shape [%d, 2, %d, %d]" % (batch, l, n_))
    _check(lib().hentt_relin(tables.handle, _words(c, "c"), _words(ksk, "ksk"), _words(out, "out"), batch,
                             _stream(stream)), "hentt_relin")
    return out


# Kernel designs of hentt_ntt_fwd_variant (the ladder of section III-B).
VARIANT_LIBRARY, VARIANT_NAIVE, VARIANT_STAGED_R4, VARIANT_STAGED_R8, VARIANT_STAGED_R16, VARIANT_STAGED_R2 = \
    0, 1, 2, 3, 4, 5
VARIANT_SIMD1, VARIANT_SIMD2, VARIANT_SIMD4 = 6, 7, 8     # wave-shuffle stages, 1, 2 or 4 register slots per lane


def ntt_fwd_variant(tables, x, variant, stream=None):
    """Forward NTT of x[..., limbs, N] in place by one of the reference kernel
    designs (VARIANT_*); same result as ntt_fwd."""
    _check(lib().hentt_ntt_fwd_variant(tables.handle, _words(x, "x"), _batch_of(tables, x), int(variant),
                                       _stream(stream)), "hentt_ntt_fwd_variant")
    return x


def ntt_inv(tables, x, stream=None):
    """In-place inverse negacyclic NTT of x[..., limbs, N]."""
    _check(lib().hentt_ntt_inv(tables.handle, _words(x, "x"), _batch_of(tables, x), _stream(stream)),
           "hentt_ntt_inv")
    return x


def dyadic_mul(tables, a, b, out=None, stream=None):
    if a.shape != b.shape:
        raise HenttError("a and b must have the same shape")
    if out is None:
        out = torch.empty_like(a)
    _check(lib().hentt_dyadic_mul(tables.handle, _words(a, "a"), _words(b, "b"), _words(out, "out"),
                                  _batch_of(tables, a, name="a"), _stream(stream)), "hentt_dyadic_mul")
    return out


def polymul(tables, a, b, out=None, stream=None):
    """Negacyclic products of coefficient-domain a, b [..., limbs, N]."""
    if a.shape != b.shape:
        raise HenttError("a and b must have the same shape")
    if out is None:
        out = torch.empty_like(a)
    _check(lib().hentt_polymul(tables.handle, _words(a, "a"), _words(b, "b"), _words(out, "out"),
                               _batch_of(tables, a, name="a"), _stream(stream)), "hentt_polymul")
    return out


def ct_tensor(tables, c, d, out=None, in_ntt=False, out_ntt=False, stream=None):
    """Ciphertext tensor: c, d [batch, 2, limbs, N] -> [batch, 3, limbs, N]."""
    if c.shape != d.shape or c.dim() != 4 or c.shape[1] != 2:
        raise HenttError("c and d must both have shape [batch, 2, limbs, N]")
    batch = _batch_of(tables, c, per_item=2, name="c")
    if out is None:
        out = torch.empty((batch, 3, tables.limbs, tables.n), dtype=c.dtype, device=c.device)
    elif tuple(out.shape) != (batch, 3, tables.limbs, tables.n):
        raise HenttError("out must have shape [batch, 3, limbs, N]")
    flags = (HENTT_IN_NTT if in_ntt else 0) | (HENTT_OUT_NTT if out_ntt else 0)
    _check(lib().hentt_ct_tensor(tables.handle, _words(c, "c"), _words(d, "d"), _words(out, "out"), batch, flags,
                                 _stream(stream)), "hentt_ct_tensor")
    return out


def ct_tensor_grouped(jobs, in_ntt=False, out_ntt=False, stream=None):
    """Many ciphertext tensors in a few launches (hentt_ct_tensor_grouped).
    jobs: (tables, c, d, out) with c, d [batch, 2, limbs, N] and out
    [batch, 3, limbs, N] at the tables' (or level view's) limbs and N; the
    outputs are written in place."""
    arr = (_CtJob * len(jobs))()
    for i, (t, c, d, out) in enumerate(jobs):
        if c.shape != d.shape or c.dim() != 4 or c.shape[1] != 2:
            raise HenttError("job %d: c and d must both have shape [batch, 2, limbs, N]" % i)
        batch = _batch_of(t, c, per_item=2, name="c")
        if tuple(out.shape) != (batch, 3, t.limbs, t.n):
            raise HenttError("job %d: out must have shape [batch, 3, limbs, N]" % i)
        arr[i].c = _words(c, "c")
        arr[i].d = _words(d, "d")
        arr[i].out = _words(out, "out")
        arr[i].t = t.handle
        arr[i].batch = batch
    flags = (HENTT_IN_NTT if in_ntt else 0) | (HENTT_OUT_NTT if out_ntt else 0)
    _check(lib().hentt_ct_tensor_grouped(arr, len(jobs), flags, _stream(stream)), "hentt_ct_tensor_grouped")


def _job_array(jobs):
    arr = (_Job * len(jobs))()
    keep = []
    for i, (x, t, limbs) in enumerate(jobs):
        if x.shape[-1] != t.n or x.shape[-2] != limbs:
            raise HenttError("job %d: x must have shape [batch, limbs=%d, N=%d]" % (i, limbs, t.n))
        arr[i].data = _words(x, "job data")
        arr[i].t = t.handle
        arr[i].limbs = limbs
        arr[i].batch = x.numel() // (limbs * t.n)
        keep.append(x)
    return arr


class BatchPlan:
    """A persistent-launch plan for an uneven batch (see hentt_batch_plan_*)."""

    def __init__(self, jobs, direction):
        self._keep = [(x, t) for x, t, _ in jobs]      # the plan holds raw pointers into these
        arr = _job_array(jobs)
        h = _VP()
        _check(lib().hentt_batch_plan_create(arr, len(jobs), int(direction), ctypes.byref(h)), "plan_create")
        self._h = h
        self.direction = +1 if int(direction) > 0 else -1
        self._graph = None

    def info(self):
        u, t, g = _U32(), _U32(), _U32()
        _check(lib().hentt_batch_plan_info(self._h, ctypes.byref(u), ctypes.byref(t), ctypes.byref(g)), "plan_info")
        return {"units": u.value, "tiles": t.value, "grid": g.value}

    def set_grid(self, workgroups):
        self.drop_graph()              # a captured graph holds the old launch shape
        _check(lib().hentt_batch_plan_set_grid(self._h, int(workgroups)), "plan_set_grid")

    def set_schedule(self, lookahead_pct=200, group_units=8):
        """Tile order: pass-2 lookahead in percent of the workgroups serving a
        queue, and the units of one twiddle table ordered block-major together."""
        self.drop_graph()
        _check(lib().hentt_batch_plan_set_schedule(self._h, int(lookahead_pct), int(group_units)), "plan_set_schedule")

    def run(self, stream=None):
        _check(lib().hentt_batch_plan_run(self._h, _stream(stream)), "plan_run")

    def status(self):
        rc = lib().hentt_batch_plan_status(self._h)
        _check(rc, "plan_status")

    def capture(self):
        """Capture the launch sequence into a hipGraph (replayed by replay())."""
        self.drop_graph()
        g = _VP()
        _check(lib().hentt_batch_graph_create(self._h, ctypes.byref(g)), "graph_create")
        self._graph = g

    def replay(self, stream=None):
        if self._graph is None:
            self.capture()
        _check(lib().hentt_graph_launch(self._graph, _stream(stream)), "graph_launch")

    def drop_graph(self):
        if self._graph is not None and _lib is not None:
            lib().hentt_graph_destroy(self._graph)
        self._graph = None

    def close(self):
        self.drop_graph()
        if getattr(self, "_h", None) is not None and _lib is not None:
            lib().hentt_batch_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ntt_batch(jobs, direction, stream=None):
    """Transform an uneven batch in one launch.  jobs: list of (x, tables, limbs)
    with x [batch, limbs, N] for that tables' N; direction +1 or -1."""
    arr = _job_array(jobs)
    _check(lib().hentt_ntt_batch(arr, len(jobs), int(direction), _stream(stream)), "hentt_ntt_batch")


def ntt_batch_status(jobs, direction):
    """Wait for the last ntt_batch call with this job list and direction and
    raise if one of its tiles gave up waiting (results incomplete)."""
    arr = _job_array(jobs)
    _check(lib().hentt_ntt_batch_status(arr, len(jobs), int(direction)), "hentt_ntt_batch_status")
