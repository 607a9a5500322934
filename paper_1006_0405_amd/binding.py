"""Python binding of libssa.so (include/ssa.h): argument marshalling only.

Every step of the multiplication runs in the library's HIP kernels; this module
passes device pointers of torch tensors (PyTorch serves as the device-memory and
stream provider) and sizes through ctypes, and converts status codes.  If the
library has not been built the import of the functions below raises: there is
no other implementation to fall back to.
"""
import ctypes
import os

import numpy as np
import torch  # loaded first: libssa.so then binds to the HIP runtime torch brought in

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssa.so")

SSA_OK = 0
SSA_ENCLOSURE_TOO_WIDE = 1
SSA_INVALID_ARGUMENT = 2
SSA_OUT_OF_MEMORY = 3
SSA_DEVICE_ERROR = 4
SSA_INTERNAL_ERROR = 5
STATUS_NAMES = {0: "OK", 1: "ENCLOSURE_TOO_WIDE", 2: "INVALID_ARGUMENT", 3: "OUT_OF_MEMORY",
                4: "DEVICE_ERROR", 5: "INTERNAL_ERROR"}

SSA_FP64 = 0
SSA_FP32_FALLBACK = 1
PRECISIONS = {"fp64": SSA_FP64, "fp32_fallback": SSA_FP32_FALLBACK}
SSA_ARITH_RECT, SSA_ARITH_DISC, SSA_ARITH_NAIVE, SSA_ARITH_NAIVE32 = 0, 1, 2, 3
# "naive", "naive32": the non-rigorous point-arithmetic baselines in double and
# single precision (products not certified)
ARITHMETICS = {"rect": SSA_ARITH_RECT, "disc": SSA_ARITH_DISC, "naive": SSA_ARITH_NAIVE,
               "naive32": SSA_ARITH_NAIVE32}
SSA_CERTIFY_ONE_INTEGER = 0
SSA_CERTIFY_HALF_INTEGER = 1

# Every entry point declared in include/ssa.h.
EXPORTS = ("ssa_fft_size", "ssa_plan_create", "ssa_plan_destroy", "ssa_mul", "ssa_get_stats",
           "ssa_batch_create", "ssa_batch_run", "ssa_batch_stats", "ssa_batch_destroy",
           "ssa_mul_batch", "ssa_debug_enclosures", "ssa_twiddle_table", "ssa_probe_directed",
           "ssa_batch_run_timed", "ssa_batch_kernel_times", "ssa_plan_get_config",
           "ssa_plan_set_config", "ssa_plan_autotune", "ssa_plan_set_fp32_policy",
           "ssa_fft_forward", "ssa_plan_force_too_wide", "ssa_plan_corrupt_bound",
           "ssa_probe_certify", "ssa_mul_noalloc", "ssa_mul_long")
KERNEL_KINDS = ("small", "col_fwd", "row", "col_inv", "carry", "status")


class SsaError(RuntimeError):
    pass


class PlanOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("digit_bits", ctypes.c_int),
                ("certify_mode", ctypes.c_int), ("separate_transforms", ctypes.c_int),
                ("refine_digits", ctypes.c_int), ("arithmetic", ctypes.c_int),
                ("refine_disc", ctypes.c_int), ("fp64_digit_bits", ctypes.c_int),
                ("exact_fallback", ctypes.c_int)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("log_n1", ctypes.c_int), ("cols", ctypes.c_int), ("rows", ctypes.c_int),
                ("persistent", ctypes.c_int), ("inv_cols", ctypes.c_int)]

    def as_dict(self):
        return {"log_n1": self.log_n1, "cols": self.cols, "rows": self.rows,
                "persistent": self.persistent, "inv_cols": self.inv_cols}


class Stats(ctypes.Structure):
    _fields_ = [("max_radius", ctypes.c_double), ("half_int", ctypes.c_uint64),
                ("too_wide", ctypes.c_uint32), ("internal", ctypes.c_uint32),
                ("carry_err", ctypes.c_uint32), ("log_n", ctypes.c_uint32),
                ("status", ctypes.c_int), ("fallback", ctypes.c_int),
                ("fp32_attempt", ctypes.c_int), ("refined", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t


def lib():
    """Load libssa.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SsaError("libssa.so is not built (%s); run __graft_entry__.build() or "
                           "python paper_1006_0405_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.ssa_fft_size.restype = _sz
        L.ssa_fft_size.argtypes = [_sz, _sz, ctypes.c_int]
        L.ssa_plan_create.restype = ctypes.c_int
        L.ssa_plan_create.argtypes = [ctypes.POINTER(_vp), _sz, _sz, ctypes.POINTER(PlanOpts), _vp]
        L.ssa_plan_destroy.restype = None
        L.ssa_plan_destroy.argtypes = [_vp]
        L.ssa_mul.restype = ctypes.c_int
        L.ssa_mul.argtypes = [_vp, _vp, _sz, _vp, _sz, _vp, ctypes.POINTER(ctypes.c_int)]
        L.ssa_mul_noalloc.restype = ctypes.c_int
        L.ssa_mul_noalloc.argtypes = [_vp, _sz, _vp, _sz, _vp, _vp, _vp]
        L.ssa_mul_long.restype = ctypes.c_int
        L.ssa_mul_long.argtypes = [_vp, _vp, _sz, _vp, _sz, _vp, ctypes.POINTER(ctypes.c_int)]
        L.ssa_get_stats.restype = ctypes.c_int
        L.ssa_get_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
        L.ssa_batch_create.restype = ctypes.c_int
        L.ssa_batch_create.argtypes = [_vp, _sz, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
        L.ssa_batch_run.restype = ctypes.c_int
        L.ssa_batch_run.argtypes = [_vp, _vp]
        L.ssa_batch_stats.restype = ctypes.c_int
        L.ssa_batch_stats.argtypes = [_vp, _vp]
        L.ssa_batch_destroy.restype = None
        L.ssa_batch_destroy.argtypes = [_vp]
        L.ssa_batch_run_timed.restype = ctypes.c_int
        L.ssa_batch_run_timed.argtypes = [_vp, _vp]
        L.ssa_batch_kernel_times.restype = ctypes.c_int
        L.ssa_batch_kernel_times.argtypes = [_vp, _vp, _vp]
        L.ssa_mul_batch.restype = ctypes.c_int
        L.ssa_mul_batch.argtypes = [_vp, _sz, _vp, _vp, _vp, _vp, _vp, _vp]
        L.ssa_debug_enclosures.restype = ctypes.c_int
        L.ssa_debug_enclosures.argtypes = [_vp, _vp, _sz, _vp, _sz, _vp, _vp,
                                           ctypes.POINTER(ctypes.c_int)]
        L.ssa_twiddle_table.restype = ctypes.c_int
        L.ssa_twiddle_table.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int)]
        L.ssa_plan_get_config.restype = ctypes.c_int
        L.ssa_plan_get_config.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(LaunchConfig)]
        L.ssa_plan_set_config.restype = ctypes.c_int
        L.ssa_plan_set_config.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(LaunchConfig)]
        L.ssa_plan_autotune.restype = ctypes.c_int
        L.ssa_plan_autotune.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(LaunchConfig),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int)]
        L.ssa_plan_set_fp32_policy.restype = ctypes.c_int
        L.ssa_plan_set_fp32_policy.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
        L.ssa_plan_force_too_wide.restype = ctypes.c_int
        L.ssa_plan_force_too_wide.argtypes = [_vp, ctypes.c_int]
        L.ssa_fft_forward.restype = ctypes.c_int
        L.ssa_fft_forward.argtypes = [_vp, ctypes.c_int, _sz, _vp, _vp, ctypes.POINTER(ctypes.c_int),
                                      _vp]
        L.ssa_plan_corrupt_bound.restype = ctypes.c_int
        L.ssa_plan_corrupt_bound.argtypes = [_vp, ctypes.c_longlong]
        L.ssa_probe_certify.restype = ctypes.c_int
        L.ssa_probe_certify.argtypes = [_vp, _sz, _sz, ctypes.c_int, _vp, _vp,
                                        ctypes.POINTER(Stats), _vp]
        L.ssa_probe_directed.restype = ctypes.c_int
        L.ssa_probe_directed.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != SSA_OK:
        raise SsaError("%s failed: %s" % (what, STATUS_NAMES.get(rc, rc)))


def _dev_u8(x, device):
    if isinstance(x, torch.Tensor):
        t = x
    else:
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.uint8)))
    t = t.to(device=device, dtype=torch.uint8).contiguous()
    if t.device.type != "cuda":
        raise SsaError("operands must live on the GPU")
    return t


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def fft_size(na, nb, digit_bits=8):
    return int(lib().ssa_fft_size(na, nb, digit_bits))


class Plan:
    """A plan for products with at most max_na x max_nb bytes."""

    def __init__(self, max_na, max_nb, digit_bits=8, certify_mode=SSA_CERTIFY_ONE_INTEGER,
                 separate_transforms=False, precision="fp64", stream=None, device=None,
                 refine_digits=False, arithmetic="rect", refine_disc=False, fp64_digit_bits=0,
                 exact_fallback=False):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.digit_bits = digit_bits
        self.separate_transforms = bool(separate_transforms)
        if precision not in PRECISIONS:
            raise SsaError("precision %r is not available (one of %s)" % (precision, sorted(PRECISIONS)))
        self.precision = precision
        if arithmetic not in ARITHMETICS:
            raise SsaError("arithmetic %r is not available (one of %s)" % (arithmetic, sorted(ARITHMETICS)))
        self.arithmetic = arithmetic
        opts = PlanOpts(PRECISIONS[precision], digit_bits, certify_mode,
                        int(bool(separate_transforms)), int(bool(refine_digits)),
                        ARITHMETICS[arithmetic], int(bool(refine_disc)), int(fp64_digit_bits),
                        int(bool(exact_fallback)))
        h = _vp()
        with torch.cuda.device(self.device):
            _check(lib().ssa_plan_create(ctypes.byref(h), max_na, max_nb, ctypes.byref(opts),
                                         _vp(self.stream.cuda_stream)), "ssa_plan_create")
        self.handle = h
        self.max_na, self.max_nb = max_na, max_nb
        self.refine_digits = bool(refine_digits)
        self.fp64_digit_bits = int(fp64_digit_bits)

    def close(self):
        if self.handle:
            lib().ssa_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mul(self, a, b, out=None):
        """Product of two byte vectors (tensors or arrays).  Returns (status, out)
        with out a uint8 device tensor of len(a) + len(b) bytes."""
        a = _dev_u8(a, self.device)
        b = _dev_u8(b, self.device)
        if out is None:
            out = torch.empty(a.numel() + b.numel(), dtype=torch.uint8, device=self.device)
        st = ctypes.c_int(-1)
        _check(lib().ssa_mul(self.handle, a.data_ptr(), a.numel(), b.data_ptr(), b.numel(),
                             out.data_ptr(), ctypes.byref(st)), "ssa_mul")
        return st.value, out

    def mul_long(self, a, b, out=None):
        """Long multiplication (ssa_mul_long): (status, out) like mul."""
        a = _dev_u8(a, self.device)
        b = _dev_u8(b, self.device)
        if out is None:
            out = torch.empty(a.numel() + b.numel(), dtype=torch.uint8, device=self.device)
        st = ctypes.c_int(-1)
        _check(lib().ssa_mul_long(self.handle, a.data_ptr(), a.numel(), b.data_ptr(), b.numel(),
                                  out.data_ptr(), ctypes.byref(st)), "ssa_mul_long")
        return st.value, out

    def stats(self):
        s = Stats()
        _check(lib().ssa_get_stats(self.handle, ctypes.byref(s)), "ssa_get_stats")
        return s.as_dict()

    def set_fp32_policy(self, max_coeffs, force_fail=False):
        """FP32 first attempt for products with at most max_coeffs coefficients
        (L = digits(a) + digits(b) - 1, 0: never) whose transform fits one
        workgroup; force_fail makes every attempt fail (tests the FP64 re-run)."""
        _check(lib().ssa_plan_set_fp32_policy(self.handle, int(max_coeffs), int(bool(force_fail))),
               "ssa_plan_set_fp32_policy")

    def force_too_wide(self, on=True):
        """Test hook: certification refuses every coefficient while on."""
        _check(lib().ssa_plan_force_too_wide(self.handle, int(bool(on))), "ssa_plan_force_too_wide")

    def corrupt_bound(self, index):
        """Test hook: certification lowers the upper bound of coefficient
        `index` by 1 (-1 turns it off)."""
        _check(lib().ssa_plan_corrupt_bound(self.handle, int(index)), "ssa_plan_corrupt_bound")

    def debug_enclosures(self, a, b):
        """(status, out, enclosures N x 4 float64 {re_lo, re_hi, im_lo, im_hi})."""
        a = _dev_u8(a, self.device)
        b = _dev_u8(b, self.device)
        N = fft_size(a.numel(), b.numel(), self.digit_bits)
        enc = torch.empty((N, 4), dtype=torch.float64, device=self.device)
        out = torch.empty(a.numel() + b.numel(), dtype=torch.uint8, device=self.device)
        st = ctypes.c_int(-1)
        _check(lib().ssa_debug_enclosures(self.handle, a.data_ptr(), a.numel(), b.data_ptr(),
                                          b.numel(), out.data_ptr(), enc.data_ptr(),
                                          ctypes.byref(st)), "ssa_debug_enclosures")
        return st.value, out, enc

    def get_config(self, log_n):
        c = LaunchConfig()
        _check(lib().ssa_plan_get_config(self.handle, log_n, ctypes.byref(c)), "ssa_plan_get_config")
        return c.as_dict()

    def set_config(self, log_n, log_n1, cols, rows, persistent=0, inv_cols=0):
        """inv_cols: columns per inverse column-pass workgroup (0: as cols)."""
        c = LaunchConfig(log_n1, cols, rows, int(persistent), int(inv_cols))
        _check(lib().ssa_plan_set_config(self.handle, log_n, ctypes.byref(c)), "ssa_plan_set_config")

    def autotune(self, log_n, count=16, cache=None):
        """Pick the fastest launch shape for transforms of length 2^log_n.  With
        `cache` (a JSON file path) a shape measured before on the same GPU
        architecture and plan options is reused instead of measured again."""
        key = None
        if cache:
            import json
            props = torch.cuda.get_device_properties(self.device)
            key = "%s/log_n=%d/digit_bits=%d/separate=%d/arithmetic=%s/precision=%s/fp64_digit_bits=%d" % (
                getattr(props, "gcnArchName", props.name), log_n, self.digit_bits,
                int(self.separate_transforms), self.arithmetic, self.precision,
                self.fp64_digit_bits)
            try:
                table = json.load(open(cache))
            except (OSError, ValueError):
                table = {}
            if key in table:
                c = table[key]
                self.set_config(log_n, c["log_n1"], c["cols"], c["rows"], c.get("persistent", 0),
                                c.get("inv_cols", 0))
                return dict(c, cached=True)
        best = LaunchConfig()
        ms = ctypes.c_double(0)
        tried = ctypes.c_int(0)
        _check(lib().ssa_plan_autotune(self.handle, log_n, count, ctypes.byref(best),
                                       ctypes.byref(ms), ctypes.byref(tried)), "ssa_plan_autotune")
        res = dict(best.as_dict(), ms_per_batch=ms.value, batch=count, tried=tried.value,
                   cached=False)
        if cache:
            import json
            try:
                table = json.load(open(cache))
            except (OSError, ValueError):
                table = {}
            table[key] = res
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return res

    def fft_forward(self, x, log_n, y=None, timed=False):
        """Forward interval DFT of x (count x N x 4 float64 device tensor, {re_lo,
        re_hi, im_lo, im_hi}).  Returns (y in four-step order, log_n1, pass times
        in ms or None)."""
        if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 3 or x.shape[1:] != (1 << log_n, 4):
            raise SsaError("x must be a (count, 2^log_n, 4) float64 device tensor")
        x = x.contiguous()
        if y is None:
            y = torch.empty_like(x)
        l1 = ctypes.c_int(0)
        ms = (ctypes.c_double * 2)() if timed else None
        _check(lib().ssa_fft_forward(self.handle, log_n, x.shape[0], x.data_ptr(), y.data_ptr(),
                                     ctypes.byref(l1), ctypes.cast(ms, _vp) if timed else None),
               "ssa_fft_forward")
        return y, l1.value, (tuple(ms) if timed else None)

    def twiddles(self):
        """(table Ntab x 2 float64 device tensor, error bound e, log2 Ntab)."""
        n = fft_size(self.max_na, self.max_nb, self.digit_bits)
        if self.refine_digits:  # the plan also holds the base-16 transform (at most 2^22)
            n = max(n, min(fft_size(self.max_na, self.max_nb, 4), 1 << 22))
        tab = torch.empty((n, 2), dtype=torch.float64, device=self.device)
        e = ctypes.c_double(0)
        lg = ctypes.c_int(0)
        _check(lib().ssa_twiddle_table(self.handle, tab.data_ptr(), ctypes.byref(e),
                                       ctypes.byref(lg)), "ssa_twiddle_table")
        return tab[: 1 << lg.value], e.value, lg.value


class Batch:
    """Many products in one captured launch.  A, B: lists of uint8 device
    tensors; outputs are allocated here (len(a) + len(b) bytes each)."""

    def __init__(self, plan, A, B):
        self.plan = plan
        self.A = [_dev_u8(a, plan.device) for a in A]
        self.B = [_dev_u8(b, plan.device) for b in B]
        n = len(self.A)
        if n != len(self.B) or n == 0:
            raise SsaError("A and B must be non-empty and of equal length")
        self.OUT = [torch.empty(a.numel() + b.numel(), dtype=torch.uint8, device=plan.device)
                    for a, b in zip(self.A, self.B)]
        self.status = torch.full((n,), -1, dtype=torch.int32, device=plan.device)
        pa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.A])
        pb = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.B])
        po = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.OUT])
        na = (ctypes.c_size_t * n)(*[t.numel() for t in self.A])
        nb = (ctypes.c_size_t * n)(*[t.numel() for t in self.B])
        h = _vp()
        _check(lib().ssa_batch_create(plan.handle, n, ctypes.cast(pa, _vp), ctypes.cast(na, _vp),
                                      ctypes.cast(pb, _vp), ctypes.cast(nb, _vp),
                                      ctypes.cast(po, _vp), ctypes.byref(h)), "ssa_batch_create")
        self.handle = h
        self.count = n

    def run(self):
        _check(lib().ssa_batch_run(self.handle, self.status.data_ptr()), "ssa_batch_run")
        return self.status

    def run_timed(self):
        """Run without the graph, with HIP events around every kernel."""
        _check(lib().ssa_batch_run_timed(self.handle, self.status.data_ptr()), "ssa_batch_run_timed")
        return self.status

    def kernel_times(self):
        """{kind: (total ms, launches)} of the timed runs since the last call."""
        ms = (ctypes.c_double * 6)()
        n = (ctypes.c_int * 6)()
        _check(lib().ssa_batch_kernel_times(self.handle, ctypes.cast(ms, _vp), ctypes.cast(n, _vp)),
               "ssa_batch_kernel_times")
        return {KERNEL_KINDS[k]: (ms[k], n[k]) for k in range(6)}

    def stats(self):
        arr = (Stats * self.count)()
        _check(lib().ssa_batch_stats(self.handle, ctypes.cast(arr, _vp)), "ssa_batch_stats")
        return [s.as_dict() for s in arr]

    def close(self):
        if self.handle:
            lib().ssa_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_directed(op, a, b, c, stream=None):
    """Device directed-rounding primitives (see include/ssa.h) on float64 tensors."""
    a, b, c = (torch.as_tensor(x, dtype=torch.float64).cuda().contiguous() for x in (a, b, c))
    out = torch.empty_like(a)
    _check(lib().ssa_probe_directed(op, a.data_ptr(), b.data_ptr(), c.data_ptr(), out.data_ptr(),
                                    a.numel(), _vp(_stream_handle(stream))), "ssa_probe_directed")
    return out


def probe_certify(enc, L, mode=SSA_CERTIFY_ONE_INTEGER, stream=None):
    """The device certification step on enclosures enc (n x 4 float64,
    {re_lo, re_hi, im_lo, im_hi}) of which the first L are coefficients.
    Returns (stats dict, int64 coefficients[L], per-entry outcome int32[n])."""
    e = torch.as_tensor(enc, dtype=torch.float64).reshape(-1, 4).cuda().contiguous()
    n = e.shape[0]
    c = torch.zeros(max(L, 1), dtype=torch.int64, device=e.device)
    cls = torch.full((n,), -1, dtype=torch.int32, device=e.device)
    st = Stats()
    _check(lib().ssa_probe_certify(e.data_ptr(), n, L, mode, c.data_ptr(), cls.data_ptr(),
                                   ctypes.byref(st), _vp(_stream_handle(stream))),
           "ssa_probe_certify")
    return st.as_dict(), c[:L].cpu().numpy(), cls.cpu().numpy()


def mul_noalloc(a, b, out, status, stream=None):
    """ssa_mul_noalloc: the product of a and b (uint8 device tensors) into out
    (len(a) + len(b) bytes) with its status into status (an int32 device tensor
    of at least one element), stream-ordered, without any allocation by the
    library.  Nothing is synchronised."""
    for t in (a, b, out):
        if t.dtype != torch.uint8 or t.device.type != "cuda" or not t.is_contiguous():
            raise SsaError("operands and output must be contiguous uint8 device tensors")
    if out.numel() != a.numel() + b.numel():
        raise SsaError("out must hold len(a) + len(b) bytes")
    if status.dtype != torch.int32 or status.device.type != "cuda" or status.numel() < 1:
        raise SsaError("status must be an int32 device tensor")
    _check(lib().ssa_mul_noalloc(a.data_ptr(), a.numel(), b.data_ptr(), b.numel(), out.data_ptr(),
                                 status.data_ptr(), _vp(_stream_handle(stream))), "ssa_mul_noalloc")


def mul(a, b, digit_bits=8, certify_mode=SSA_CERTIFY_ONE_INTEGER):
    """One-off product of two byte arrays; returns (status, numpy uint8 product)."""
    a = np.asarray(a, dtype=np.uint8)
    b = np.asarray(b, dtype=np.uint8)
    p = Plan(len(a), len(b), digit_bits=digit_bits, certify_mode=certify_mode)
    try:
        st, out = p.mul(a, b)
        return st, out.cpu().numpy()
    finally:
        p.close()
