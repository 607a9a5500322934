"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE).

Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
module.  The GPU library never imports, links or calls it, and this module
imports nothing from the GPU library.

Every function restates the paper's method on the CPU in IEEE double (or
single) interval arithmetic with fesetround(); see oracle.cpp for the
section-by-section correspondence with the paper.
"""
import contextlib
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

ST_OK, ST_TOO_WIDE, ST_INVALID, ST_INTERNAL = 0, 1, 2, 5

_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_sz = ctypes.c_size_t


def lib():
    """Load liboracle.so, building it first only if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIBPATH)
        for name in ("oracle_mul_f64", "oracle_mul_f32"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [_u8p, _sz, _u8p, _sz, ctypes.c_int, ctypes.c_int, _u8p, _dp, _i64p]
        for name in ("oracle_mul_naive_f64", "oracle_mul_naive_f32"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [_u8p, _sz, _u8p, _sz, ctypes.c_int, _u8p]
        L.oracle_fft_size.restype = _sz
        L.oracle_fft_size.argtypes = [_sz, _sz, ctypes.c_int]
        L.oracle_conv_enclosure_f64.restype = _sz
        L.oracle_conv_enclosure_f64.argtypes = [_u8p, _sz, _u8p, _sz, ctypes.c_int, _dp]
        L.oracle_dft_f64.restype = None
        L.oracle_dft_f64.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.oracle_twiddles_f64.restype = None
        L.oracle_twiddles_f64.argtypes = [ctypes.c_int, _dp]
        L.oracle_roots_f64.restype = None
        L.oracle_roots_f64.argtypes = [ctypes.c_int, _dp]
        L.oracle_iop_f64.restype = ctypes.c_int
        L.oracle_iop_f64.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_iop_f32.restype = ctypes.c_int
        L.oracle_iop_f32.argtypes = [ctypes.c_int, _fp, _fp, _fp]
        L.oracle_cmul_f64.restype = None
        L.oracle_cmul_f64.argtypes = [_dp, _dp, _dp]
        L.oracle_certify_f64.restype = ctypes.c_int
        L.oracle_certify_f64.argtypes = [_dp, _sz, _sz, ctypes.c_int, _i64p, _dp, _i64p]
        L.oracle_carry.restype = None
        L.oracle_carry.argtypes = [_i64p, _sz, ctypes.c_int, _u8p, _sz]
        L.oracle_set_mutation.restype = None
        L.oracle_set_mutation.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _u8(x):
    a = np.ascontiguousarray(np.frombuffer(bytes(x), dtype=np.uint8) if isinstance(x, (bytes, bytearray)) else np.asarray(x, dtype=np.uint8))
    return a


def _ptr(a, t):
    return a.ctypes.data_as(t)


def fft_size(na, nb, digit_bits=8):
    return int(lib().oracle_fft_size(na, nb, digit_bits))


def mul(a, b, digit_bits=8, certify_mode=0, precision="f64"):
    """Rigorous interval SSA product.

    Returns (status, product bytes as np.uint8[na+nb], max real radius,
    half-integer straddle count).  On failure the product is all zeros.
    """
    a, b = _u8(a), _u8(b)
    out = np.zeros(len(a) + len(b), dtype=np.uint8)
    r = ctypes.c_double(0)
    h = ctypes.c_int64(0)
    f = lib().oracle_mul_f64 if precision == "f64" else lib().oracle_mul_f32
    st = f(_ptr(a, _u8p), len(a), _ptr(b, _u8p), len(b), digit_bits, certify_mode,
           _ptr(out, _u8p), ctypes.byref(r), ctypes.byref(h))
    return st, out, r.value, h.value


def mul_naive(a, b, digit_bits=8, precision="f64"):
    """Non-rigorous round-to-nearest SSA (no certification)."""
    a, b = _u8(a), _u8(b)
    out = np.zeros(len(a) + len(b), dtype=np.uint8)
    f = lib().oracle_mul_naive_f64 if precision == "f64" else lib().oracle_mul_naive_f32
    st = f(_ptr(a, _u8p), len(a), _ptr(b, _u8p), len(b), digit_bits, _ptr(out, _u8p))
    return st, out


def conv_enclosure(a, b, digit_bits=8):
    """Enclosures (N x 4: re_lo, re_hi, im_lo, im_hi) of all N outputs."""
    a, b = _u8(a), _u8(b)
    N = fft_size(len(a), len(b), digit_bits)
    out = np.zeros((N, 4), dtype=np.float64)
    lib().oracle_conv_enclosure_f64(_ptr(a, _u8p), len(a), _ptr(b, _u8p), len(b), digit_bits,
                                    _ptr(out, _dp))
    return out


def dft(k, x4, inverse=False):
    x4 = np.ascontiguousarray(x4, dtype=np.float64).reshape(1 << k, 4)
    out = np.zeros_like(x4)
    lib().oracle_dft_f64(k, int(inverse), _ptr(x4, _dp), _ptr(out, _dp))
    return out


def twiddles(k):
    n = max((1 << k) // 2, 1)
    out = np.zeros((n, 4), dtype=np.float64)
    lib().oracle_twiddles_f64(k, _ptr(out, _dp))
    return out


def roots(k):
    out = np.zeros((k + 1, 4), dtype=np.float64)
    lib().oracle_roots_f64(k, _ptr(out, _dp))
    return out


OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4}


def iop(op, a, b=None, precision="f64"):
    """One real interval operation; returns (lo, hi) or None if undefined."""
    dt, pt, f = ((np.float64, _dp, lib().oracle_iop_f64) if precision == "f64"
                 else (np.float32, _fp, lib().oracle_iop_f32))
    A = np.asarray(a, dtype=dt)
    B = np.asarray(b if b is not None else (0, 0), dtype=dt)
    R = np.zeros(2, dtype=dt)
    rc = f(OPS[op], _ptr(A, pt), _ptr(B, pt), _ptr(R, pt))
    return None if rc != 0 else (R[0], R[1])


def cmul(a4, b4):
    A = np.asarray(a4, dtype=np.float64)
    B = np.asarray(b4, dtype=np.float64)
    R = np.zeros(4, dtype=np.float64)
    lib().oracle_cmul_f64(_ptr(A, _dp), _ptr(B, _dp), _ptr(R, _dp))
    return R


def certify(enc4, L, mode=0):
    """Returns (status, int64 coefficients[L], max radius, half-int count)."""
    E = np.ascontiguousarray(enc4, dtype=np.float64).reshape(-1, 4)
    c = np.zeros(max(L, 1), dtype=np.int64)
    r = ctypes.c_double(0)
    h = ctypes.c_int64(0)
    st = lib().oracle_certify_f64(_ptr(E, _dp), E.shape[0], L, mode, _ptr(c, _i64p),
                                  ctypes.byref(r), ctypes.byref(h))
    return st, c[:L], r.value, h.value


def carry(c, digit_bits, nout):
    C = np.ascontiguousarray(c, dtype=np.int64)
    out = np.zeros(nout, dtype=np.uint8)
    lib().oracle_carry(_ptr(C, _i64p), len(C), digit_bits, _ptr(out, _u8p), nout)
    return out


@contextlib.contextmanager
def mutation(m):
    """Plant mistake number m in the oracle for the duration of the block."""
    lib().oracle_set_mutation(m)
    try:
        yield
    finally:
        lib().oracle_set_mutation(0)
