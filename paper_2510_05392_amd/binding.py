"""Thin ctypes binding of the megpu C ABI (include/megpu.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libmegpu.so.  Device buffers come from torch tensors (their
data_ptr()); the library never sees torch types.  If the library is missing
the import of this module still succeeds but every call raises, so nothing
can silently fall back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libmegpu.so')

ME_OK = 0
ME_EINVAL = -1
ME_ENOMEM = -2
ME_EHIP = -3
ME_ESTATE = -4
ME_CS_FP64 = 0
ME_CS_FP16X2 = 1
ME_CS_BF16X2 = 2

EXPORTS = ['me_params_default', 'me_init', 'me_compute', 'me_filter_helicities',
           'me_good_helicities', 'me_info', 'me_colour_matrix', 'me_helicity_sums',
           'me_jamps', 'me_set_colorsum_mode', 'me_finalize', 'me_last_error']


class MeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'megpu error {code}: {msg}')
        self.code = code


class me_params(ctypes.Structure):
    _fields_ = [('mt', ctypes.c_double), ('colorsum_mode', ctypes.c_int),
                ('all_helicities', ctypes.c_int)]


_lib = None


def load(path=LIB_PATH):
    """Load libmegpu.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f'{path} is missing: build it with python -m paper_2510_05392_amd.build')
    lib = ctypes.CDLL(path)
    vp, i64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)
    lib.me_params_default.argtypes = [ctypes.POINTER(me_params)]
    lib.me_init.argtypes = [ctypes.c_char_p, ctypes.POINTER(me_params), ctypes.POINTER(vp)]
    lib.me_compute.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp]
    lib.me_filter_helicities.argtypes = [vp, vp, i64, ctypes.c_double, vp]
    lib.me_good_helicities.argtypes = [vp, i32p, ctypes.c_int32, i32p]
    lib.me_info.argtypes = [vp, i32p, i32p, i32p, i32p]
    lib.me_colour_matrix.argtypes = [vp, i32p, ctypes.c_int32, i32p]
    lib.me_helicity_sums.argtypes = [vp, vp, i64, ctypes.c_double, i32p, ctypes.c_int32, vp, vp]
    lib.me_jamps.argtypes = [vp, vp, i64, ctypes.c_double, i32p, ctypes.c_int32, vp, vp]
    lib.me_set_colorsum_mode.argtypes = [vp, ctypes.c_int]
    lib.me_finalize.argtypes = [vp]
    lib.me_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-1]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != ME_OK:
        raise MeError(rc, load().me_last_error().decode())
    return rc


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else (t if isinstance(t, int) else t.data_ptr()))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)


class MatrixElement:
    """One handle of the C ABI for one process."""

    def __init__(self, process: str, mt: float = 173.0, all_helicities: bool = False,
                 colorsum_mode: int = ME_CS_FP64):
        lib = load()
        p = me_params()
        _check(lib.me_params_default(ctypes.byref(p)))
        p.mt = mt
        p.all_helicities = int(all_helicities)
        p.colorsum_mode = int(colorsum_mode)
        h = ctypes.c_void_p()
        _check(lib.me_init(process.encode(), ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.process = process
        a, b, c, d = (ctypes.c_int32() for _ in range(4))
        _check(lib.me_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        self.npar, self.ncolor, self.nhel, self.ndiag = a.value, b.value, c.value, d.value

    # the binding names mirror the C entry points
    def me_compute(self, momenta, nevt, alpha_s, out, stream=None):
        _check(load().me_compute(self._h, _ptr(momenta), nevt, alpha_s, _ptr(out), _stream(stream)))

    def me_filter_helicities(self, momenta, nevt, alpha_s, stream=None):
        _check(load().me_filter_helicities(self._h, _ptr(momenta), nevt, alpha_s, _stream(stream)))

    def me_good_helicities(self):
        n = ctypes.c_int32()
        _check(load().me_good_helicities(self._h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int32 * max(1, n.value))()
        _check(load().me_good_helicities(self._h, buf, n.value, ctypes.byref(n)))
        return list(buf[:n.value])

    def me_colour_matrix(self):
        buf = (ctypes.c_int32 * (self.ncolor * self.ncolor))()
        den = ctypes.c_int32()
        _check(load().me_colour_matrix(self._h, buf, len(buf), ctypes.byref(den)))
        return [list(buf[i * self.ncolor:(i + 1) * self.ncolor]) for i in range(self.ncolor)], den.value

    def me_helicity_sums(self, momenta, nevt, alpha_s, hels, out, stream=None):
        arr = (ctypes.c_int32 * len(hels))(*hels)
        _check(load().me_helicity_sums(self._h, _ptr(momenta), nevt, alpha_s, arr, len(hels),
                                       _ptr(out), _stream(stream)))

    def me_jamps(self, momenta, nevt, alpha_s, hels, out, stream=None):
        arr = (ctypes.c_int32 * len(hels))(*hels)
        _check(load().me_jamps(self._h, _ptr(momenta), nevt, alpha_s, arr, len(hels),
                               _ptr(out), _stream(stream)))

    def me_set_colorsum_mode(self, mode):
        _check(load().me_set_colorsum_mode(self._h, int(mode)))

    def me_finalize(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(load().me_finalize(h))

    def __del__(self):
        try:
            self.me_finalize()
        except Exception:
            pass

    # convenience wrappers on torch tensors -------------------------------
    def compute(self, momenta, alpha_s=0.118, out=None, stream=None):
        """|M|^2 for a device tensor momenta[nevt][npar][4] (float64, contiguous)."""
        import torch
        if momenta.dtype != torch.float64 or not momenta.is_cuda or not momenta.is_contiguous():
            raise ValueError('momenta must be a contiguous float64 device tensor')
        nevt = momenta.shape[0]
        if momenta.shape[1:] != (self.npar, 4):
            raise ValueError(f'momenta must have shape [nevt, {self.npar}, 4]')
        if out is None:
            out = torch.empty(nevt, dtype=torch.float64, device=momenta.device)
        if stream is None:
            stream = torch.cuda.current_stream(momenta.device)
        self.me_compute(momenta, nevt, alpha_s, out, stream)
        return out
