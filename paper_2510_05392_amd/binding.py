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
ME_EXEC_LANE = 0
ME_EXEC_TEAM = 1
ME_EXEC_SPLIT = 2
ME_EXEC_BG = 3
# per-kernel timing classes (me_kernel_times)
ME_KT_DIAGRAM, ME_KT_FLOWS, ME_KT_COLOUR, ME_KT_REDUCE = 0, 1, 2, 3
ME_KT_KINDS = 4

EXPORTS = ['me_params_default', 'me_init', 'me_compute', 'me_compute_host', 'me_compute_noalloc',
           'me_filter_helicities',
           'me_good_helicities', 'me_info', 'me_colour_matrix', 'me_helicity_sums',
           'me_jamps', 'me_set_colorsum_mode', 'me_set_launch', 'me_autotune', 'me_compute_batch',
           'me_compute_alphas', 'me_select', 'me_set_executor', 'me_set_kernel_timing',
           'me_kernel_times', 'me_finalize', 'me_channel_weights', 'me_num_channels', 'me_set_split', 'me_set_bg',
           'me_sur_init', 'me_sur_finalize', 'me_sur_num_params', 'me_sur_get_params',
           'me_sur_set_params', 'me_sur_get_grads', 'me_sur_set_normalisation', 'me_sur_features',
           'me_sur_predict', 'me_sur_grads', 'me_sur_adam', 'me_sur_train_step',
           'me_unweight_stage1', 'me_gather_momenta', 'me_unweight_stage2',
           'me_sur_fit_normalisation', 'me_sur_activations', 'me_sur_targets', 'me_sur_gather_rows', 'me_sur_log_error',
           'me_unweight_maxima', 'me_unweight_quantile', 'me_unweight_onestage', 'me_unweight_summary',
           'me_last_error']


class MeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'megpu error {code}: {msg}')
        self.code = code


class me_params(ctypes.Structure):
    _fields_ = [('mt', ctypes.c_double), ('wt', ctypes.c_double), ('colorsum_mode', ctypes.c_int),
                ('all_helicities', ctypes.c_int), ('use_graph', ctypes.c_int), ('check', ctypes.c_int),
                ('autotune', ctypes.c_int)]


class me_sur_params(ctypes.Structure):
    _fields_ = [('nfeat', ctypes.c_int), ('width', ctypes.c_int), ('depth', ctypes.c_int),
                ('seed', ctypes.c_uint64)]


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
    lib.me_compute_noalloc.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp]
    lib.me_compute_host.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_double)]
    lib.me_filter_helicities.argtypes = [vp, vp, i64, ctypes.c_double, vp]
    lib.me_good_helicities.argtypes = [vp, i32p, ctypes.c_int32, i32p]
    lib.me_info.argtypes = [vp, i32p, i32p, i32p, i32p]
    lib.me_colour_matrix.argtypes = [vp, i32p, ctypes.c_int32, i32p]
    lib.me_helicity_sums.argtypes = [vp, vp, i64, ctypes.c_double, i32p, ctypes.c_int32, vp, vp]
    lib.me_jamps.argtypes = [vp, vp, i64, ctypes.c_double, i32p, ctypes.c_int32, vp, vp]
    lib.me_set_colorsum_mode.argtypes = [vp, ctypes.c_int]
    lib.me_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.me_autotune.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp, i32p]
    lib.me_compute_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(i64), ctypes.c_double, ctypes.POINTER(vp), vp]
    lib.me_compute_alphas.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.me_set_executor.argtypes = [vp, ctypes.c_int]
    lib.me_set_split.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.me_set_bg.argtypes = [vp, ctypes.c_int]
    lib.me_select.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp, vp, vp, vp, vp]
    lib.me_finalize.argtypes = [vp]
    lib.me_channel_weights.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp, vp, vp]
    lib.me_num_channels.argtypes = [vp, i32p]
    fp, dbl = ctypes.POINTER(ctypes.c_float), ctypes.c_double
    lib.me_sur_init.argtypes = [ctypes.POINTER(me_sur_params), ctypes.POINTER(vp)]
    lib.me_sur_finalize.argtypes = [vp]
    lib.me_sur_num_params.argtypes = [vp, ctypes.POINTER(i64)]
    lib.me_sur_get_params.argtypes = [vp, fp, i64]
    lib.me_sur_set_params.argtypes = [vp, fp, i64]
    lib.me_sur_get_grads.argtypes = [vp, fp, i64]
    lib.me_sur_set_normalisation.argtypes = [vp, fp, fp]
    lib.me_sur_features.argtypes = [vp, vp, i64, ctypes.c_int, vp, vp, vp]
    lib.me_sur_predict.argtypes = [vp, vp, i64, vp, vp]
    lib.me_sur_grads.argtypes = [vp, vp, vp, i64, vp, vp]
    lib.me_sur_adam.argtypes = [vp, ctypes.c_float, vp]
    lib.me_sur_train_step.argtypes = [vp, vp, vp, i64, ctypes.c_float, vp, vp]
    lib.me_unweight_stage1.argtypes = [vp, vp, vp, i64, dbl, dbl, dbl, vp, vp, ctypes.POINTER(i64), vp]
    lib.me_gather_momenta.argtypes = [vp, vp, i64, ctypes.c_int, vp, vp]
    lib.me_unweight_stage2.argtypes = [vp, vp, i64, vp, vp, vp, dbl, dbl, vp, vp]
    dblp, i64p = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)
    lib.me_sur_fit_normalisation.argtypes = [vp, vp, i64, vp, dblp, dblp, vp]
    lib.me_sur_targets.argtypes = [vp, i64, dbl, dbl, vp, vp]
    lib.me_sur_activations.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64, fp]
    lib.me_sur_gather_rows.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp, vp, vp]
    lib.me_sur_log_error.argtypes = [vp, vp, i64, dbl, dbl, dblp, dblp, vp]
    lib.me_unweight_maxima.argtypes = [vp, vp, vp, i64, dbl, dbl, dbl, dblp, dblp, vp]
    lib.me_unweight_quantile.argtypes = [vp, vp, i64, dbl, dblp, vp]
    lib.me_unweight_onestage.argtypes = [vp, vp, vp, i64, dbl, vp, vp]
    lib.me_unweight_summary.argtypes = [vp, i64, i64p, i64p, dblp, dblp, vp]
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


def me_compute_batch(handles, momenta, nevts, alpha_s, outs, stream=None):
    """One launch over several processes: handles[i] (MatrixElement) on momenta[i] -> outs[i]."""
    n = len(handles)
    vp = ctypes.c_void_p
    hs = (vp * n)(*[h._h.value for h in handles])
    ms = (vp * n)(*[_ptr(m).value for m in momenta])
    ns = (ctypes.c_int64 * n)(*nevts)
    os_ = (vp * n)(*[_ptr(o).value for o in outs])
    _check(load().me_compute_batch(n, hs, ms, ns, alpha_s, os_, _stream(stream)))


class MatrixElement:
    """One handle of the C ABI for one process."""

    def __init__(self, process: str, mt: float = 173.0, all_helicities: bool = False,
                 colorsum_mode: int = ME_CS_FP64, use_graph: bool = False, check=None, wt: float = 0.0,
                 autotune: bool = False):
        lib = load()
        p = me_params()
        _check(lib.me_params_default(ctypes.byref(p)))
        p.mt = mt
        p.wt = wt
        p.all_helicities = int(all_helicities)
        p.colorsum_mode = int(colorsum_mode)
        p.use_graph = int(use_graph)
        if check is not None:
            p.check = int(bool(check))
        p.autotune = int(bool(autotune))
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

    def me_compute_host(self, momenta, alpha_s):
        """Host-pointer variant: momenta is a C-contiguous float64 numpy array [nevt][npar][4]."""
        import numpy as np
        mom = np.ascontiguousarray(momenta, dtype=np.float64)
        out = np.zeros(mom.shape[0], dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().me_compute_host(self._h, mom.ctypes.data_as(dp), mom.shape[0], alpha_s,
                                      out.ctypes.data_as(dp)))
        return out

    def me_compute_noalloc(self, momenta, nevt, alpha_s, out, stream=None):
        _check(load().me_compute_noalloc(self._h, _ptr(momenta), nevt, alpha_s, _ptr(out), _stream(stream)))

    def me_compute_alphas(self, momenta, nevt, alpha_s, out, stream=None):
        _check(load().me_compute_alphas(self._h, _ptr(momenta), nevt, _ptr(alpha_s), _ptr(out),
                                        _stream(stream)))

    def me_select(self, momenta, nevt, alpha_s, r_hel, r_col, out, sel_hel, sel_col, stream=None):
        _check(load().me_select(self._h, _ptr(momenta), nevt, alpha_s, _ptr(r_hel), _ptr(r_col), _ptr(out),
                                _ptr(sel_hel), _ptr(sel_col), _stream(stream)))

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

    def me_channel_weights(self, momenta, nevt, alpha_s, chan, num, den, stream=None):
        _check(load().me_channel_weights(self._h, _ptr(momenta), nevt, alpha_s, _ptr(chan), _ptr(num), _ptr(den),
                                         _stream(stream)))

    def me_num_channels(self):
        n = ctypes.c_int32()
        _check(load().me_num_channels(self._h, ctypes.byref(n)))
        return n.value

    def me_set_launch(self, persistent, waves_per_simd=1, hel_per_item=0, target_waves=4096):
        _check(load().me_set_launch(self._h, persistent, waves_per_simd, hel_per_item, target_waves))

    TUNE_FIELDS = ('persistent', 'waves_per_simd', 'hel_per_item', 'target_waves', 'executor', 'split_wpe',
                   'split_fchunk', 'split_rounds', 'colour_grid', 'bg_variant')

    def me_autotune(self, momenta, nevt, alpha_s, out, stream=None):
        best = (ctypes.c_int32 * len(self.TUNE_FIELDS))()
        _check(load().me_autotune(self._h, _ptr(momenta), nevt, alpha_s, _ptr(out), _stream(stream), best))
        return dict(zip(self.TUNE_FIELDS, list(best)))

    def me_set_bg(self, variant=0):
        _check(load().me_set_bg(self._h, variant))

    def me_set_split(self, wpe=0, fchunk=0, rounds=0, colour_grid=0):
        _check(load().me_set_split(self._h, wpe, fchunk, rounds, colour_grid))

    def me_set_executor(self, executor):
        _check(load().me_set_executor(self._h, int(executor)))

    def me_set_kernel_timing(self, on):
        _check(load().me_set_kernel_timing(self._h, int(bool(on))))

    def me_kernel_times(self):
        """(total ms, launches) per kernel class since timing was switched on or last read."""
        ms = (ctypes.c_double * ME_KT_KINDS)()
        n = (ctypes.c_int64 * ME_KT_KINDS)()
        _check(load().me_kernel_times(self._h, ms, n))
        return list(ms), list(n)

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


class Surrogate:
    """A handle of the surrogate C ABI (MLP on pair invariants, BF16 on the matrix cores)."""

    def __init__(self, nfeat, width=256, depth=4, seed=1):
        lib = load()
        p = me_sur_params(nfeat, width, depth, seed)
        h = ctypes.c_void_p()
        _check(lib.me_sur_init(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.nfeat, self.width, self.depth = nfeat, width, depth
        self.kpad = ((nfeat + 15) // 16) * 16
        n = ctypes.c_int64()
        _check(lib.me_sur_num_params(h, ctypes.byref(n)))
        self.nparams = n.value

    def _host(self, arr):
        import numpy as np
        arr = np.ascontiguousarray(arr, dtype=np.float32)
        return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def me_sur_get_params(self):
        import numpy as np
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(load().me_sur_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size))
        return out

    def me_sur_set_params(self, flat):
        arr, ptr = self._host(flat)
        _check(load().me_sur_set_params(self._h, ptr, arr.size))

    def me_sur_get_grads(self):
        import numpy as np
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(load().me_sur_get_grads(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size))
        return out

    def me_sur_set_normalisation(self, mean, inv_std):
        m, pm = self._host(mean)
        s, ps = self._host(inv_std)
        _check(load().me_sur_set_normalisation(self._h, pm, ps))

    def me_sur_fit_normalisation(self, raw, n, me2, stream=None):
        """Sets the feature normalisation from raw[n][nfeat]; returns (ymean, ystd) of log|M|^2."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(load().me_sur_fit_normalisation(self._h, _ptr(raw), n, _ptr(me2), ctypes.byref(a), ctypes.byref(b),
                                               _stream(stream)))
        return a.value, b.value

    def me_sur_activations(self, layer, kind, rows):
        """Input (kind 0) or pre-activation output (kind 1) of linear layer `layer` in the last forward pass."""
        import numpy as np
        n = (self.nfeat if layer == 0 else self.width) if kind == 0 else (1 if layer == self.depth else self.width)
        out = np.zeros((rows, n), dtype=np.float32)
        _check(load().me_sur_activations(self._h, layer, kind, rows,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def me_sur_features(self, momenta, nevt, npar, feat, raw=None, stream=None):
        _check(load().me_sur_features(self._h, _ptr(momenta), nevt, npar, _ptr(feat), _ptr(raw),
                                      _stream(stream)))

    def me_sur_predict(self, feat, n, y, stream=None):
        _check(load().me_sur_predict(self._h, _ptr(feat), n, _ptr(y), _stream(stream)))

    def me_sur_grads(self, feat, target, nb, loss=None, stream=None):
        _check(load().me_sur_grads(self._h, _ptr(feat), _ptr(target), nb, _ptr(loss), _stream(stream)))

    def me_sur_adam(self, lr, stream=None):
        _check(load().me_sur_adam(self._h, lr, _stream(stream)))

    def me_sur_train_step(self, feat, target, nb, lr, loss=None, stream=None):
        _check(load().me_sur_train_step(self._h, _ptr(feat), _ptr(target), nb, lr, _ptr(loss),
                                        _stream(stream)))

    def me_sur_finalize(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(load().me_sur_finalize(h))

    def __del__(self):
        try:
            self.me_sur_finalize()
        except Exception:
            pass


def me_unweight_stage1(y, wps, r1, n, ymean, ystd, what_max, what, idx, stream=None):
    """Returns the number of stage-1 events (their indices are in idx[:n_keep])."""
    nk = ctypes.c_int64()
    _check(load().me_unweight_stage1(_ptr(y), _ptr(wps), _ptr(r1), n, ymean, ystd, what_max, _ptr(what),
                                     _ptr(idx), ctypes.byref(nk), _stream(stream)))
    return nk.value


def me_gather_momenta(momenta, idx, m, npar, out, stream=None):
    _check(load().me_gather_momenta(_ptr(momenta), _ptr(idx), m, npar, _ptr(out), _stream(stream)))


def me_unweight_stage2(me_exact, idx, m, wps, what, r2, what_max, x_max, resid, stream=None):
    _check(load().me_unweight_stage2(_ptr(me_exact), _ptr(idx), m, _ptr(wps), _ptr(what), _ptr(r2),
                                     what_max, x_max, _ptr(resid), _stream(stream)))


def me_sur_targets(me2, n, ymean, ystd, target, stream=None):
    _check(load().me_sur_targets(_ptr(me2), n, ymean, ystd, _ptr(target), _stream(stream)))


def me_sur_gather_rows(feat, target, perm, n, kpad, feat_out, target_out, stream=None):
    _check(load().me_sur_gather_rows(_ptr(feat), _ptr(target), _ptr(perm), n, kpad, _ptr(feat_out),
                                     _ptr(target_out), _stream(stream)))


def me_sur_log_error(y, me2, n, ymean, ystd, stream=None):
    """(RMS, largest absolute) error of the surrogate's log|M|^2."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(load().me_sur_log_error(_ptr(y), _ptr(me2), n, ymean, ystd, ctypes.byref(a), ctypes.byref(b),
                                   _stream(stream)))
    return a.value, b.value


def me_unweight_maxima(y, wps, me2, n, ymean, ystd, q, stream=None):
    """(what_max, x_max): q-quantiles of the surrogate weight and of the exact/surrogate ratio."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(load().me_unweight_maxima(_ptr(y), _ptr(wps), _ptr(me2), n, ymean, ystd, q, ctypes.byref(a),
                                     ctypes.byref(b), _stream(stream)))
    return a.value, b.value


def me_unweight_quantile(me2, wps, n, q, stream=None):
    a = ctypes.c_double()
    _check(load().me_unweight_quantile(_ptr(me2), _ptr(wps), n, q, ctypes.byref(a), _stream(stream)))
    return a.value


def me_unweight_onestage(me2, wps, r, n, w_max, resid, stream=None):
    _check(load().me_unweight_onestage(_ptr(me2), _ptr(wps), _ptr(r), n, w_max, _ptr(resid), _stream(stream)))


def me_unweight_summary(resid, m, stream=None):
    """(accepted, overweights, sum of weights, sum of squared weights)."""
    a, o = ctypes.c_int64(), ctypes.c_int64()
    s1, s2 = ctypes.c_double(), ctypes.c_double()
    _check(load().me_unweight_summary(_ptr(resid), m, ctypes.byref(a), ctypes.byref(o), ctypes.byref(s1),
                                      ctypes.byref(s2), _stream(stream)))
    return a.value, o.value, s1.value, s2.value
