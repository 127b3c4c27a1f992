"""Compile the host (CPU) build of a generated process for the tests."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, 'paper_2510_05392_amd', 'csrc')
OUT = os.path.join(ROOT, '_build', 'cpu_harness')


def build(name, opt='-O1', sums_parts=None, remat=None):
    """sums_parts: number of group-sum parts of the split executor; remat: momentum
    sums recomputed at each use in them (defaults: the generator's choice)."""
    from paper_2510_05392_amd.gen import codegen
    os.makedirs(OUT, exist_ok=True)
    src, _, _ = codegen.generate(name, sums_parts=sums_parts, remat=remat)
    tag = name + (f'_p{sums_parts}' if sums_parts else '') + ('' if remat is None else f'_r{int(remat)}')
    hdr = os.path.join(OUT, f'{tag}.inc')
    if not os.path.exists(hdr) or open(hdr).read() != src:
        with open(hdr, 'w') as f:
            f.write(src)
    lib = os.path.join(OUT, f'harness_{tag}.so')
    deps = [hdr, os.path.join(CSRC, 'me_device.h'), os.path.join(CSRC, 'me_team.h'),
            os.path.join(HERE, 'harness.cpp')]
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(d) for d in deps):
        cmd = ['g++', opt, '-std=c++17', '-shared', '-fPIC', '-I', os.path.join(HERE),
               '-I', CSRC, f'-DPROCESS_HEADER="{hdr}"', f'-DPROCNAME={name}',
               os.path.join(HERE, 'harness.cpp'), '-o', lib + '.tmp']
        subprocess.run(cmd, check=True)
        os.replace(lib + '.tmp', lib)
    return Harness(lib)


class Harness:
    def __init__(self, path):
        self.lib = ctypes.CDLL(path)
        self.lib.harness_ncol.restype = ctypes.c_int
        self.ncol = self.lib.harness_ncol()

    def eval(self, mom, g, mt, hels, want_jamps=False):
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        nevt = mom.shape[0]
        hels = np.ascontiguousarray(hels, dtype=np.int32)
        meh = np.zeros((len(hels), nevt))
        jam = np.zeros((len(hels), nevt, self.ncol, 2)) if want_jamps else None
        dp = ctypes.POINTER(ctypes.c_double)
        self.lib.harness_eval(mom.ctypes.data_as(dp), ctypes.c_int(nevt), ctypes.c_double(g),
                              ctypes.c_double(mt), hels.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              ctypes.c_int(len(hels)), meh.ctypes.data_as(dp),
                              jam.ctypes.data_as(dp) if want_jamps else None)
        if want_jamps:
            return meh, jam[..., 0] + 1j * jam[..., 1]
        return meh

    def team_eval(self, mom, g, mt, hels):
        """Per-helicity colour sums from the serial emulation of the team executor."""
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        nevt = mom.shape[0]
        hels = np.ascontiguousarray(hels, dtype=np.int32)
        meh = np.zeros((len(hels), nevt))
        dp = ctypes.POINTER(ctypes.c_double)
        self.lib.harness_team_eval(mom.ctypes.data_as(dp), ctypes.c_int(nevt), ctypes.c_double(g),
                                   ctypes.c_double(mt), hels.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   ctypes.c_int(len(hels)), meh.ctypes.data_as(dp))
        return meh

    def split_eval(self, mom, g, mt, hels, chunk=16):
        """Per-helicity colour sums from the split evaluation (group sums, then flows
        formed from chunks of `chunk` group sums: 8, 16 or 32)."""
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        nevt = mom.shape[0]
        hels = np.ascontiguousarray(hels, dtype=np.int32)
        meh = np.zeros((len(hels), nevt))
        dp = ctypes.POINTER(ctypes.c_double)
        self.lib.harness_split_eval(mom.ctypes.data_as(dp), ctypes.c_int(nevt), ctypes.c_double(g),
                                    ctypes.c_double(mt), hels.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                    ctypes.c_int(len(hels)), meh.ctypes.data_as(dp), ctypes.c_int(chunk))
        return meh


def build_sde(name, opt='-O1'):
    """Host build of the generated single-diagram-enhancement function of a process."""
    from paper_2510_05392_amd.gen import codegen
    os.makedirs(OUT, exist_ok=True)
    src, _ = codegen.generate_sde(name)
    hdr = os.path.join(OUT, f'{name}_sde.inc')
    if not os.path.exists(hdr) or open(hdr).read() != src:
        with open(hdr, 'w') as f:
            f.write(src)
    lib = os.path.join(OUT, f'sde_harness_{name}.so')
    deps = [hdr, os.path.join(CSRC, 'me_device.h'), os.path.join(HERE, 'sde_harness.cpp')]
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(d) for d in deps):
        cmd = ['g++', opt, '-std=c++17', '-shared', '-fPIC', '-I', os.path.join(HERE),
               '-I', CSRC, f'-DSDE_HEADER="{hdr}"', f'-DSDENAME={name}_sde',
               os.path.join(HERE, 'sde_harness.cpp'), '-o', lib + '.tmp']
        subprocess.run(cmd, check=True)
        os.replace(lib + '.tmp', lib)
    return SdeHarness(lib)


class SdeHarness:
    def __init__(self, path):
        self.lib = ctypes.CDLL(path)
        self.lib.harness_nchan.restype = ctypes.c_int
        self.nchan = self.lib.harness_nchan()

    def eval(self, mom, g, mt, hels, chan):
        """(num, den) per helicity and event: [nh][nevt] each."""
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        nevt = mom.shape[0]
        hels = np.ascontiguousarray(hels, dtype=np.int32)
        chan = np.ascontiguousarray(chan, dtype=np.int32)
        num = np.zeros((len(hels), nevt))
        den = np.zeros((len(hels), nevt))
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        self.lib.harness_sde_eval(mom.ctypes.data_as(dp), ctypes.c_int(nevt), ctypes.c_double(g),
                                  ctypes.c_double(mt), hels.ctypes.data_as(ip), ctypes.c_int(len(hels)),
                                  chan.ctypes.data_as(ip), num.ctypes.data_as(dp), den.ctypes.data_as(dp))
        return num, den


def build_count(name, opt='-O1'):
    """Host build of a process's generated code with the operation-counting scalar."""
    from paper_2510_05392_amd.gen import codegen
    os.makedirs(OUT, exist_ok=True)
    src, _, _ = codegen.generate(name)
    hdr = os.path.join(OUT, f'{name}.inc')
    if not os.path.exists(hdr) or open(hdr).read() != src:
        with open(hdr, 'w') as f:
            f.write(src)
    lib = os.path.join(OUT, f'count_harness_{name}.so')
    deps = [hdr, os.path.join(CSRC, 'me_device.h'), os.path.join(CSRC, 'me_team.h'),
            os.path.join(HERE, 'count_harness.cpp')]
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(d) for d in deps):
        cmd = ['g++', opt, '-std=c++17', '-shared', '-fPIC', '-I', os.path.join(HERE),
               '-I', CSRC, f'-DPROCESS_HEADER="{hdr}"', f'-DPROCNAME={name}',
               os.path.join(HERE, 'count_harness.cpp'), '-o', lib + '.tmp']
        subprocess.run(cmd, check=True)
        os.replace(lib + '.tmp', lib)
    return CountHarness(lib)


class CountHarness:
    def __init__(self, path):
        self.lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        for f in ('count_amplitudes', 'count_group_sums'):
            getattr(self.lib, f).restype = ctypes.c_longlong
            getattr(self.lib, f).argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        self.lib.count_colour_sum.restype = ctypes.c_longlong
        self.lib.count_routine.restype = ctypes.c_longlong
        self.lib.count_routine.argtypes = [ctypes.c_int]

    def _mom(self, mom):
        m = np.ascontiguousarray(mom, dtype=np.float64)
        return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def amplitudes(self, mom, hel, g=1.2, mt=173.0):
        m, ptr = self._mom(mom)
        return self.lib.count_amplitudes(ptr, hel, g, mt)

    def group_sums(self, mom, hel, g=1.2, mt=173.0):
        m, ptr = self._mom(mom)
        return self.lib.count_group_sums(ptr, hel, g, mt)

    def colour_sum(self):
        return self.lib.count_colour_sum()

    def routine(self, which):
        return self.lib.count_routine(which)


def build_bg(opt='-O2'):
    """Host build of the Berends-Giele executor's device functions (all gluon counts)."""
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, 'bg_harness.so')
    deps = [os.path.join(CSRC, h) for h in ('me_device.h', 'me_bg.h', 'me_bgh.h', 'me_bg_desc.h', 'me_bg_tables.h')]
    deps.append(os.path.join(HERE, 'bg_harness.cpp'))
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(d) for d in deps):
        cmd = ['g++', opt, '-std=c++17', '-shared', '-fPIC', '-I', os.path.join(HERE), '-I', CSRC,
               os.path.join(HERE, 'bg_harness.cpp'), '-o', lib + '.tmp']
        subprocess.run(cmd, check=True)
        os.replace(lib + '.tmp', lib)
    return BgHarness(lib)


class BgHarness:
    def __init__(self, path):
        self.lib = ctypes.CDLL(path)

    def jamps(self, n, mom, g, mt, hels):
        """Dual amplitudes [nh][nevt][n!] (complex) of n-gluon events."""
        import math
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        nevt = mom.shape[0]
        hels = np.ascontiguousarray(hels, dtype=np.int32)
        out = np.zeros((len(hels), nevt, math.factorial(n), 2))
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        rc = self.lib.harness_bg_eval(ctypes.c_int(n), mom.ctypes.data_as(dp), ctypes.c_int(nevt), ctypes.c_double(g),
                                      ctypes.c_double(mt), hels.ctypes.data_as(ip), ctypes.c_int(len(hels)),
                                      out.ctypes.data_as(dp))
        assert rc == 0
        return out[..., 0] + 1j * out[..., 1]

    def jamps_recycled(self, n, mom, g, mt, hels):
        """The same dual amplitudes from the helicity-recycling kernel's work (n = 4, 5)."""
        import math
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        nevt = mom.shape[0]
        hels = np.ascontiguousarray(hels, dtype=np.int32)
        out = np.zeros((len(hels), nevt, math.factorial(n), 2))
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        rc = self.lib.harness_bgh_eval(ctypes.c_int(n), mom.ctypes.data_as(dp), ctypes.c_int(nevt),
                                       ctypes.c_double(g), ctypes.c_double(mt), hels.ctypes.data_as(ip),
                                       ctypes.c_int(len(hels)), out.ctypes.data_as(dp))
        assert rc == 0
        return out[..., 0] + 1j * out[..., 1]


def build_count_bg(opt='-O1'):
    """Host build of the Berends-Giele device functions with the operation-counting scalar."""
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, 'count_bg_harness.so')
    deps = [os.path.join(CSRC, h) for h in ('me_device.h', 'me_bg.h', 'me_bgh.h', 'me_bg_desc.h', 'me_bg_tables.h')]
    deps.append(os.path.join(HERE, 'count_bg_harness.cpp'))
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(d) for d in deps):
        cmd = ['g++', opt, '-std=c++17', '-shared', '-fPIC', '-I', os.path.join(HERE), '-I', CSRC,
               os.path.join(HERE, 'count_bg_harness.cpp'), '-o', lib + '.tmp']
        subprocess.run(cmd, check=True)
        os.replace(lib + '.tmp', lib)
    lib = ctypes.CDLL(lib)

    def count(n, mom, hel=None):
        """hel given: one row of the row kernels; hel None: one event of the
        helicity-recycling kernel (every helicity good)."""
        m = np.ascontiguousarray(mom, dtype=np.float64)
        out = (ctypes.c_longlong * 4)()
        ptr = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if hel is None:
            assert lib.count_bgh_event(n, ptr, out) == 0
        else:
            assert lib.count_bg_row(n, ptr, hel, out) == 0
        return list(out)
    return count
