"""Python binding of the MI355X strided-swap stencil library (libspider.so).

Argument marshalling only: every step of the stencil path runs in the HIP
library; PyTorch supplies device memory and streams.  The library must have
been built (``python -m paper_2506_22035_amd.build``); using any function
without it raises ``SpiderError`` -- there is no fallback.

The C ABI is declared and documented in ``include/spider.h``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspider.so")

DTYPES = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
ENGINES = {"auto": 0, "sparse": 1, "dense": 2, "direct": 3}
_ENGINE_NAMES = {v: k for k, v in ENGINES.items()}
_DTYPE_NAMES = {v: k for k, v in DTYPES.items()}
STATUS = {0: "OK", 1: "INVALID", 2: "UNSUPPORTED", 3: "OOM", 4: "HIP", 5: "NOT_READY", 6: "BUSY", 7: "CLOSED"}


class SpiderError(RuntimeError):
    """A library call returned a status other than OK."""

    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [("carry", ctypes.c_int), ("engine", ctypes.c_int), ("split", ctypes.c_int),
                ("tile_h", ctypes.c_int), ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("time_block", ctypes.c_int), ("operand", ctypes.c_int), ("band_height", ctypes.c_int),
                ("row_swap", ctypes.c_int)]


_lib = None


def lib():
    """The loaded C library (raises SpiderError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SpiderError(-1, "libspider.so is not built (run python -m paper_2506_22035_amd.build)")
        # The library must run on the same HIP runtime as torch, whose stream handles and
        # device pointers it is given.  torch ships its own copy of libamdhip64.so.7;
        # importing torch first loads it, and the library then binds to it by its soname
        # (loaded the other way round, the process would hold two runtimes and the
        # second to initialise would find no GPU).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, I, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
        sig = {
            "spider_opts_default": [P],
            "spider_plan": [P, I, P, I, P, P],
            "spider_apply": [P, P, P, I, P],
            "spider_apply_noalloc": [P, P, P, I, P],
            "spider_plan_destroy": [P],
            "spider_plan_info": [P, P, P, P, P, P, P, P, P],
            "spider_plan_work": [P, I, P, P],
            "spider_measure_matrix_rate": [I, I, I, P, P, P, P],
            "spider_apply_batch": [I, P, P, P, P, P],
            "spider_server_create": [ctypes.c_size_t, I, I, P],
            "spider_submit": [P, P, P, P, I, P],
            "spider_poll": [P, U64, P, P],
            "spider_server_stats": [P, P, P, P, P],
            "spider_server_destroy": [P],
            "spider_gather_positions": [P],
            "spider_swap_columns": [I, I, P],
            "spider_compress_24": [P, I, I, P, P],
            "spider_pack_row": [P, I, I, I, P, P, P],
            "spider_pair_gather_positions": [P],
            "spider_pack_pair": [P, I, I, I, I, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.spider_last_error.restype = ctypes.c_char_p
        L.spider_last_error.argtypes = []
        L.spider_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise SpiderError(status, lib().spider_last_error().decode())


def version():
    return lib().spider_version().decode()


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def measure_matrix_rate(sparse=True, waves_per_simd=2, iterations=20000, stream=None):
    """Sustained fp16 matrix-instruction rate of the current device (spider.h):
    dict with dense-equivalent TFLOP/s, the shader clock held meanwhile (GHz) and
    clock cycles per instruction per SIMD."""
    t, g, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().spider_measure_matrix_rate(1 if sparse else 0, int(waves_per_simd), int(iterations), stream,
                                            ctypes.byref(t), ctypes.byref(g), ctypes.byref(c)))
    return {"TFLOPs": t.value, "clock_GHz": g.value, "cycles_per_instruction": c.value}


# ------------------------------------------------------------------ planner introspection (host only)

def gather_positions():
    """Window column feeding each of the 32 K slots of a band (see spider.h)."""
    out = np.zeros(32, dtype=np.int32)
    _check(lib().spider_gather_positions(_ptr(out)))
    return out


def swap_columns(L, granularity=1):
    """The strided column swap on an L x 2L band: perm[j] = source column of column j."""
    out = np.zeros(2 * L, dtype=np.int32)
    _check(lib().spider_swap_columns(int(L), int(granularity), _ptr(out)))
    return out


def compress_24(m):
    """2:4 compression: (values rows x cols/2, 2-bit positions rows x cols/2)."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    rows, cols = m.shape
    vals = np.zeros((rows, cols // 2))
    meta = np.zeros((rows, cols // 2), dtype=np.uint8)
    _check(lib().spider_compress_24(_ptr(m), rows, cols, _ptr(vals), _ptr(meta)))
    return vals, meta


def pack_row(row, radius, operand="f16", split=2):
    """Packed smfmac operands of one kernel row: (A bits (64, 8), index (64,), dense A bits (64, 16))."""
    row = np.ascontiguousarray(row, dtype=np.float64)
    a = np.zeros((64, 8), dtype=np.uint16)
    idx = np.zeros(64, dtype=np.uint16)
    dense = np.zeros((64, 16), dtype=np.uint16)
    _check(lib().spider_pack_row(_ptr(row), int(radius), DTYPES[operand], int(split), _ptr(a), _ptr(idx),
                                 _ptr(dense)))
    return a, idx, dense


def pair_gather_positions():
    """Window column of each of the 16 K slots of a line in the paired-line band (see spider.h)."""
    out = np.zeros(16, dtype=np.int32)
    _check(lib().spider_pair_gather_positions(_ptr(out)))
    return out


def pack_pair(w, radius, k, operand="f16", split=2):
    """Packed operands of instruction k of the paired-line band: (A bits (64, 8), index (64,), dense (64, 16))."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    a = np.zeros((64, 8), dtype=np.uint16)
    idx = np.zeros(64, dtype=np.uint16)
    dense = np.zeros((64, 16), dtype=np.uint16)
    _check(lib().spider_pack_pair(_ptr(w), int(radius), DTYPES[operand], int(split), int(k), _ptr(a), _ptr(idx),
                                  _ptr(dense)))
    return a, idx, dense


# ------------------------------------------------------------------ plans

def _torch():
    import torch
    return torch


def torch_dtype(carry):
    t = _torch()
    return {"f64": t.float64, "f32": t.float32, "f16": t.float16, "bf16": t.bfloat16}[carry]


def _stream_handle(stream):
    if stream is None:
        return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A stencil plan: coefficients (2r+1,)*ndim (w[dz][dy][dx] multiplies x[p + offset]),
    grid shape, carry dtype and engine.  `operand` ("f16"/"bf16") selects the 16-bit
    operand type of the matrix engines for an "f32" carry.  Owns device memory until `close()`."""

    def __init__(self, coeffs, shape, carry="f16", engine="auto", split=2, tile_h=0, use_graph=True, autotune=False,
                 time_block=0, operand=None, band_height=0, row_swap="implicit"):
        w = np.ascontiguousarray(coeffs, dtype=np.float64)
        ndim = len(shape)
        if w.ndim != ndim or len(set(w.shape)) != 1 or w.shape[0] % 2 != 1:
            raise ValueError("coeffs must have shape (2r+1,)*ndim")
        self.radius = (w.shape[0] - 1) // 2
        self.shape = tuple(int(s) for s in shape)
        self.carry = carry
        opts = _Opts()
        _check(lib().spider_opts_default(ctypes.byref(opts)))
        opts.carry = DTYPES[carry]
        opts.engine = ENGINES[engine]
        opts.split = int(split)
        opts.tile_h = int(tile_h)
        opts.use_graph = 1 if use_graph else 0
        opts.autotune = 1 if autotune else 0
        opts.time_block = int(time_block)
        opts.operand = DTYPES[operand] if operand else 0
        opts.band_height = int(band_height)
        opts.row_swap = {"implicit": 0, "explicit": 1}[row_swap]
        shp = (ctypes.c_int64 * ndim)(*self.shape)
        h = ctypes.c_void_p()
        _check(lib().spider_plan(_ptr(w), ndim, shp, self.radius, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise SpiderError(1, "plan is closed")
        return self._h

    def info(self):
        e, c, t, n, tb, t2, bh = (ctypes.c_int() for _ in range(7))
        sb = ctypes.c_size_t()
        _check(lib().spider_plan_info(self.handle, ctypes.byref(e), ctypes.byref(c), ctypes.byref(t),
                                      ctypes.byref(n), ctypes.byref(sb), ctypes.byref(tb), ctypes.byref(t2),
                                      ctypes.byref(bh)))
        return dict(engine=_ENGINE_NAMES[e.value], carry=_DTYPE_NAMES[c.value], tile_h=t.value,
                    nrows_nonzero=n.value, scratch_bytes=sb.value, time_block=tb.value, tile_h2=t2.value,
                    band_height=bh.value)

    def work(self, steps):
        """(launches, matrix instructions) that apply(..., steps) issues; the count is
        None where the library keeps none (see spider_plan_work)."""
        n, m = ctypes.c_uint64(), ctypes.c_uint64()
        st = lib().spider_plan_work(self.handle, int(steps), ctypes.byref(n), ctypes.byref(m))
        if st == 2:
            return n.value, None
        _check(st)
        return n.value, m.value

    def check_tensor(self, t):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise SpiderError(1, "grids must be CUDA (HIP) tensors")
        if tuple(t.shape) != self.shape or not t.is_contiguous() or t.dtype != torch_dtype(self.carry):
            raise SpiderError(1, "grid must be contiguous %s of shape %s" % (self.carry, self.shape))

    def apply(self, x_in, x_out, steps, stream=None):
        """x_out = S^steps(x_in) on `stream` (default: torch's current stream); asynchronous."""
        self.check_tensor(x_in)
        self.check_tensor(x_out)
        _check(lib().spider_apply(self.handle, ctypes.c_void_p(x_in.data_ptr()), ctypes.c_void_p(x_out.data_ptr()),
                                  int(steps), _stream_handle(stream)))

    def apply_noalloc(self, x_in, x_out, steps, stream=None):
        """As apply, through the library's fixed device scratch array: allocates no device
        memory (grids up to SPIDER_NOALLOC_SCRATCH_BYTES; calls on one GPU must not overlap)."""
        self.check_tensor(x_in)
        self.check_tensor(x_out)
        _check(lib().spider_apply_noalloc(self.handle, ctypes.c_void_p(x_in.data_ptr()),
                                          ctypes.c_void_p(x_out.data_ptr()), int(steps), _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().spider_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_batch(plans, ins, outs, steps, stream=None):
    """Advance several grids together, one batched launch per time step."""
    n = len(plans)
    for p, a, b in zip(plans, ins, outs):
        p.check_tensor(a)
        p.check_tensor(b)
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    hi = (ctypes.c_void_p * n)(*[a.data_ptr() for a in ins])
    ho = (ctypes.c_void_p * n)(*[b.data_ptr() for b in outs])
    hs = (ctypes.c_int * n)(*[int(s) for s in steps])
    _check(lib().spider_apply_batch(n, hp, hi, ho, hs, _stream_handle(stream)))


class Server:
    """Continuous-batching request loop (see spider_server_create in spider.h)."""

    def __init__(self, hbm_budget_bytes, max_slots=64, max_queue=4096):
        h = ctypes.c_void_p()
        _check(lib().spider_server_create(ctypes.c_size_t(int(hbm_budget_bytes)), int(max_slots), int(max_queue),
                                          ctypes.byref(h)))
        self._h = h
        # the plan and both grids of every ticket in flight: the server reads them
        # until the ticket is done, so they must not be freed before that
        self._inflight = {}
        self._finished = {}   # ticket -> status, once the library has reported it done

    def submit(self, plan, x_in, x_out, steps):
        plan.check_tensor(x_in)
        plan.check_tensor(x_out)
        t = ctypes.c_uint64()
        _check(lib().spider_submit(self._h, plan.handle, ctypes.c_void_p(x_in.data_ptr()),
                                   ctypes.c_void_p(x_out.data_ptr()), int(steps), ctypes.byref(t)))
        self._inflight[t.value] = (plan, x_in, x_out)
        return t.value

    def try_submit(self, plan, x_in, x_out, steps):
        """Like submit, but returns None instead of raising when the queue is full."""
        try:
            return self.submit(plan, x_in, x_out, steps)
        except SpiderError as e:
            if e.status == 6:
                return None
            raise

    def poll(self, ticket):
        """(done, status) of a ticket.  Once done, the ticket's plan and grids are released
        by the server object (the caller's own references are untouched)."""
        if ticket in self._finished:
            return True, self._finished[ticket]
        d, r = ctypes.c_int(), ctypes.c_int()
        _check(lib().spider_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(d), ctypes.byref(r)))
        if d.value:
            self._finished[ticket] = r.value
            self._inflight.pop(ticket, None)
        return bool(d.value), r.value

    def stats(self):
        p50, p99, up = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_uint64()
        _check(lib().spider_server_stats(self._h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(n),
                                         ctypes.byref(up)))
        return dict(p50_us=p50.value, p99_us=p99.value, completed=n.value, stencil_updates=up.value)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(lib().spider_server_destroy(self._h))
            self._h = None
            self._inflight.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
