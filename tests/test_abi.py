"""The C-ABI library loads and exports every entry point include/megpu.h declares.

No compute call is made here (no GPU on this machine); the binding's names
must mirror the header's.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'megpu.h')


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r'^\s*(?:int|const char\s*\*)\s+(me_\w+)\s*\(', text, re.M)))


@pytest.fixture(scope='module')
def libpath():
    from paper_2510_05392_amd import binding, build
    if os.path.exists(binding.LIB_PATH):
        return binding.LIB_PATH
    # not built yet: build a one-process library just for the symbol check
    out = os.path.join(ROOT, '_build', 'abi_check', 'libmegpu.so')
    return build.build(['gg_ttx'], lib=out, verbose=False)


def test_header_declares_the_abi():
    names = declared()
    for n in ('me_init', 'me_compute', 'me_good_helicities', 'me_finalize', 'me_last_error'):
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_header():
    from paper_2510_05392_amd import binding
    assert sorted(binding.EXPORTS) == declared()


def test_host_only_entry_points(libpath):
    from paper_2510_05392_amd import binding
    lib = ctypes.CDLL(libpath)
    lib.me_params_default.argtypes = [ctypes.POINTER(binding.me_params)]
    p = binding.me_params()
    assert lib.me_params_default(ctypes.byref(p)) == 0
    assert p.mt == 173.0 and p.colorsum_mode == 0 and p.all_helicities == 0
    assert lib.me_params_default(None) == binding.ME_EINVAL
    lib.me_last_error.restype = ctypes.c_char_p
    assert b'null' in lib.me_last_error()
    # argument validation happens before any device call
    lib.me_init.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.me_init(None, None, None) == binding.ME_EINVAL
    h = ctypes.c_void_p()
    assert lib.me_init(b'gg_ttxq', None, ctypes.byref(h)) == binding.ME_EINVAL
    assert b'unknown process' in lib.me_last_error()
    lib.me_finalize.argtypes = [ctypes.c_void_p]
    assert lib.me_finalize(None) == 0
    lib.me_compute.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_void_p, ctypes.c_void_p]
    assert lib.me_compute(None, None, 1, 0.118, None, None) == binding.ME_EINVAL
    bogus = ctypes.c_void_p(0x1000)
    assert lib.me_compute(bogus, None, 1, 0.118, None, None) == binding.ME_ESTATE


def test_host_validation_of_batch_select_and_executor(libpath):
    # these entry points check their arguments on the host before any device call
    from paper_2510_05392_amd import binding
    lib = ctypes.CDLL(libpath)
    lib.me_last_error.restype = ctypes.c_char_p
    vp = ctypes.c_void_p
    lib.me_compute_batch.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_double, vp, vp]
    assert lib.me_compute_batch(0, None, None, None, 0.118, None, None) == binding.ME_EINVAL
    assert lib.me_compute_batch(9, None, None, None, 0.118, None, None) == binding.ME_EINVAL
    assert lib.me_compute_batch(1, None, None, None, 0.118, None, None) == binding.ME_EINVAL
    hs = (vp * 1)(0x1000)
    ms = (vp * 1)(None)
    ns = (ctypes.c_int64 * 1)(8)
    os_ = (vp * 1)(None)
    assert lib.me_compute_batch(1, hs, ms, ns, 0.118, os_, None) == binding.ME_ESTATE
    assert lib.me_compute_batch(1, hs, ms, ns, -1.0, os_, None) == binding.ME_EINVAL
    lib.me_select.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, vp, vp, vp, vp, vp, vp]
    assert lib.me_select(None, None, 4, 0.118, None, None, None, None, None, None) == binding.ME_EINVAL
    lib.me_compute_alphas.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
    assert lib.me_compute_alphas(vp(0x1000), None, 4, None, None, None) == binding.ME_ESTATE
    lib.me_set_executor.argtypes = [vp, ctypes.c_int]
    assert lib.me_set_executor(None, 1) == binding.ME_EINVAL
    assert lib.me_set_executor(vp(0x1000), 1) == binding.ME_ESTATE
    lib.me_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    assert lib.me_set_launch(None, 1, 1, 1, 1) == binding.ME_EINVAL


def test_params_width_check_and_host_call_validation(libpath, monkeypatch):
    # me_params carries the top width (only 0 is implemented) and the input-check
    # switch, whose default follows ME_CHECK; all of this is host-side
    from paper_2510_05392_amd import binding
    lib = ctypes.CDLL(libpath)
    lib.me_last_error.restype = ctypes.c_char_p
    lib.me_params_default.argtypes = [ctypes.POINTER(binding.me_params)]
    p = binding.me_params()
    monkeypatch.delenv('ME_CHECK', raising=False)
    assert lib.me_params_default(ctypes.byref(p)) == 0
    assert p.wt == 0.0 and p.check == 0 and p.use_graph == 0
    monkeypatch.setenv('ME_CHECK', '1')
    assert lib.me_params_default(ctypes.byref(p)) == 0
    assert p.check == 1
    monkeypatch.setenv('ME_CHECK', '0')
    assert lib.me_params_default(ctypes.byref(p)) == 0
    assert p.check == 0
    # a non-zero width is refused before any device call
    p.wt = 1.4915
    h = ctypes.c_void_p()
    lib.me_init.argtypes = [ctypes.c_char_p, ctypes.POINTER(binding.me_params), ctypes.POINTER(ctypes.c_void_p)]
    assert lib.me_init(b'gg_ttx', ctypes.byref(p), ctypes.byref(h)) == binding.ME_EINVAL
    assert b'width' in lib.me_last_error()
    assert h.value is None
    # host-pointer variant: argument checks precede any device work
    dp = ctypes.POINTER(ctypes.c_double)
    lib.me_compute_host.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64, ctypes.c_double, dp]
    assert lib.me_compute_host(None, None, 1, 0.118, None) == binding.ME_EINVAL
    assert lib.me_compute_host(ctypes.c_void_p(0x1000), None, 1, 0.118, None) == binding.ME_ESTATE
