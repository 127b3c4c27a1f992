"""Build the HIP library libmegpu.so for gfx950 (MI355X).

Steps: run the process generator for every process, write one HIP translation
unit per process (so that the large generated units compile in parallel),
compile them and the runtime with hipcc, link the shared library in-tree.

    python -m paper_2510_05392_amd.build [--procs gg_ttx,gg_ttxg] [-j N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
GEN = os.path.join(CSRC, 'generated')
OBJ = os.path.join(ROOT, '_build', 'obj')
INCLUDE = os.path.join(ROOT, 'include')
LIB = os.path.join(HERE, 'libmegpu.so')

PROCESSES = ['gg_ttx', 'gg_ttxg', 'gg_ttxgg', 'gg_ttxggg', 'gg_ttxgggg']
# headers the generated process units include
PROC_HEADERS = ['me_device.h', 'me_kernels.h', 'me_process.h', 'colour_mfma.h', 'me_team.h']
SDE_HEADERS = ['me_sde.h', 'me_sde_desc.h']
BG_HEADERS = ['me_device.h', 'me_bg.h', 'me_bgh.h', 'me_bg_desc.h', 'colour_mfma.h', 'me_colour_big.h']


def bg_unit(name, n):
    """Source of the Berends-Giele unit of a process: the recursion kernel for n gluons
    and the FP64 colour form of its n! flows (the full matrix held in LDS up to 128
    flows, the block-triangular form streamed through LDS beyond)."""
    import math
    ncol = math.factorial(n)
    if ncol <= 128:
        # the full matrix fits in LDS: the split executor's colour kernel
        colour = ('  constexpr int RPB = 4 * 8 * COLOUR_F64_TILES;\n'
                  '  const int64_t tiles = (nrow + RPB - 1) / RPB;\n'
                  f'  hipLaunchKernelGGL(colour_f64_kernel<{ncol}>, dim3((unsigned)std::min<int64_t>(tiles, '
                  'COLOUR_F64_GRID)), dim3(256), 0, s, jt, nrow, cf64, out);\n')
    else:
        colour = ('  const int64_t tiles = (nrow + 32 * BIG_NT - 1) / (32 * BIG_NT);\n'
                  f'  hipLaunchKernelGGL(colour_f64_tri_kernel<{ncol}>, dim3((unsigned)std::min<int64_t>(tiles, '
                  'BIG_GRID)), dim3(256), 0, s, jt, nrow, cf64, out);\n')
    tri = 0 if ncol <= 128 else 1
    return (f'// Berends-Giele executor of process {name} (generated).\n'
            '#include <algorithm>\n#include "me_bgh.h"\n#include "colour_mfma.h"\n#include "me_colour_big.h"\n'
            'namespace me {\n'
            f'static hipError_t colour64_{name}(const double* jt, int64_t nrow, const double* cf64, double* out, '
            'hipStream_t s) {\n' + colour + '  return hipGetLastError();\n}\n'
            f'const BgDesc* bg_{name}() {{\n  static const BgDesc d = {{"{name}", {n}, {ncol}, &launch_bg<{n}>, '
            f'&colour64_{name}, {tri}, {int(n in (4, 5))}, &bgh_fused_per_cu<{n}>, &bgh_fused_slot_doubles<{n}>, '
            f'&bgh_block_events<{n}>}};\n'
            '  return &d;\n}\n}\n')
ARCH = 'gfx950'
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
FLAGS = ['-std=c++17', '-O3', '-fPIC', f'--offload-arch={ARCH}',
         # the compiler may not form packed FP32 (v_pk_*_f32) instructions: they
         # are kept out of every kernel as a correctness precaution
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
         '-I', INCLUDE, '-I', CSRC, '-I', GEN]



def _write_if_changed(path, text):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path, 'w') as f:
        f.write(text)


def generate_sources(procs, build_dir):
    sys.path.insert(0, ROOT)
    from paper_2510_05392_amd.gen import codegen
    os.makedirs(GEN, exist_ok=True)
    os.makedirs(build_dir, exist_ok=True)
    units = []
    for name in procs:
        src, _, _ = codegen.generate(name)
        inc = os.path.join(GEN, f'{name}.inc')
        _write_if_changed(inc, src)
        lane = codegen.PROCESS_NPAR[name] <= codegen.LANE_MAX_NPAR
        if lane:
            unit = (f'// Kernels and descriptor of process {name} (generated).\n'
                    f'#include "{name}.inc"\n#include "me_kernels.h"\n'
                    f'namespace me {{\nhipError_t split_{name}(const SplitArgs& a);\n'
                    f'const ProcessDesc* process_{name}() {{ return describe<me::{name}>(&split_{name}); }}\n}}\n')
            # the split executor's kernels compile in parallel in a unit of their own
            split = (f'// Split-executor kernels of process {name} (generated).\n'
                     f'#include "{name}.inc"\n#include "me_kernels.h"\n'
                     f'namespace me {{\nhipError_t split_{name}(const SplitArgs& a) '
                     f'{{ return launch_split<me::{name}>(a); }}\n}}\n')
            spath = os.path.join(GEN, f'split_{name}.hip')
            _write_if_changed(spath, split)
            units.append((spath, os.path.join(OBJ, f'split_{name}.o'),
                          [inc] + [os.path.join(CSRC, h) for h in PROC_HEADERS]))
            # single-diagram-enhancement channel sums: generated code of their own,
            # in a unit of their own
            sde_src, _ = codegen.generate_sde(name)
            sinc = os.path.join(GEN, f'{name}_sde.inc')
            _write_if_changed(sinc, sde_src)
            sde = (f'// Single-diagram-enhancement kernel of process {name} (generated).\n'
                   f'#include "{name}_sde.inc"\n#include "me_sde.h"\n'
                   f'namespace me {{\nconst SdeDesc* sde_{name}() {{ return describe_sde<me::{name}_sde>(); }}\n}}\n')
            sdepath = os.path.join(GEN, f'sde_{name}.hip')
            _write_if_changed(sdepath, sde)
            units.append((sdepath, os.path.join(OBJ, f'sde_{name}.o'),
                          [sinc] + [os.path.join(CSRC, h) for h in PROC_HEADERS + SDE_HEADERS]))
        else:
            unit = (f'// Kernels and descriptor of process {name} (generated).\n'
                    f'#include "{name}.inc"\n#include "me_kernels.h"\n'
                    f'namespace me {{\nconst ProcessDesc* process_{name}() '
                    f'{{ return describe<me::{name}>(nullptr); }}\n}}\n')
        bgpath = os.path.join(GEN, f'bg_{name}.hip')
        _write_if_changed(bgpath, bg_unit(name, codegen.PROCESS_NPAR[name] - 2))
        units.append((bgpath, os.path.join(OBJ, f'bg_{name}.o'), [os.path.join(CSRC, h) for h in BG_HEADERS]))
        path = os.path.join(GEN, f'proc_{name}.hip')
        _write_if_changed(path, unit)
        units.append((path, os.path.join(OBJ, f'proc_{name}.o'),
                      [inc] + [os.path.join(CSRC, h) for h in PROC_HEADERS]))
    reg = ['// Processes compiled into this library (generated).']
    reg += [f'const ProcessDesc* process_{n}();' for n in procs]
    reg.append('static const ProcessDesc* (*const kProcesses[])() = {'
               + ', '.join(f'process_{n}' for n in procs) + '};')
    reg.append(f'static const int kNumProcesses = {len(procs)};')
    reg.append('// one persistent kernel over all of them (multi-process batches)')
    reg.append('hipError_t launch_batch_all(const BatchArgs& a, int waves, hipStream_t stream);')
    # the batch kernel covers the leading processes that have one-lane code
    lane = []
    for n in procs:
        if codegen.PROCESS_NPAR[n] > codegen.LANE_MAX_NPAR:
            break
        lane.append(n)
    reg.append(f'static const int kNumBatchProcesses = {len(lane)};')
    # single-diagram-enhancement kernels, aligned with kProcesses (none without one-lane code)
    reg += [f'const SdeDesc* sde_{n}();' for n in lane]
    reg.append('static const SdeDesc* (*const kSde[])() = {'
               + ', '.join(f'sde_{n}' if n in lane else 'nullptr' for n in procs) + '};')
    # Berends-Giele executors, aligned with kProcesses
    reg += [f'const BgDesc* bg_{n}();' for n in procs]
    reg.append('static const BgDesc* (*const kBg[])() = {' + ', '.join(f'bg_{n}' for n in procs) + '};')
    batch = ['// Multi-process batch kernel over the processes of this library (generated).']
    batch += [f'#include "{n}.inc"' for n in lane]
    batch += ['#include "me_kernels.h"', 'namespace me {',
              'hipError_t launch_batch_all(const BatchArgs& a, int waves, hipStream_t stream) {',
              '  return launch_batch<' + ', '.join(f'me::{n}' for n in lane) + '>(a, waves, stream);',
              '}', '}']
    batchfile = os.path.join(build_dir, 'batch.hip')
    _write_if_changed(batchfile, '\n'.join(batch) + '\n')
    regfile = os.path.join(build_dir, 'registry.inc')
    _write_if_changed(regfile, '\n'.join(reg) + '\n')
    units.insert(0, (batchfile, os.path.join(build_dir, 'batch.o'),
                     [os.path.join(GEN, f'{n}.inc') for n in lane] + [os.path.join(CSRC, h) for h in PROC_HEADERS]))
    units.append((os.path.join(CSRC, 'me_api.hip'), os.path.join(build_dir, 'me_api.o'),
                  [regfile, os.path.join(INCLUDE, 'megpu.h'), os.path.join(CSRC, 'me_process.h'),
                   os.path.join(CSRC, 'me_error.h'), os.path.join(CSRC, 'me_sde_desc.h'),
                   os.path.join(CSRC, 'me_bg_desc.h'), os.path.join(CSRC, 'me_bg_tables.h')]))
    units.append((os.path.join(CSRC, 'surrogate.hip'), os.path.join(OBJ, 'surrogate.o'),
                  [os.path.join(INCLUDE, 'megpu.h'), os.path.join(CSRC, 'me_error.h')]))
    return units


def _compile(src, obj, extra_deps, build_dir, force=False, build_id=None):
    deps = [src] + list(extra_deps)
    flags = FLAGS + (['-I', build_dir] if src.endswith('me_api.hip') or src.startswith(build_dir) else [])
    if build_id and src.endswith('me_api.hip'):
        # the library's build identity (a hash of every source it is compiled from)
        # keys the autotuner's result cache
        flags = flags + [f'-DME_BUILD_ID="{build_id}"']
    # the object is reused only when the flags and the contents of every input are
    # those it was compiled from (contents, not modification times: a source edited
    # while its object was compiling must not pass for up to date)
    h = hashlib.sha1((' '.join(flags) + HIPCC).encode())
    for d in deps:
        with open(d, 'rb') as f:
            h.update(f.read())
    key = h.hexdigest()[:16]
    stamp = obj + '.flags'
    if not force and os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == key:
        return obj, False
    # the resource-usage remarks (registers, spills, occupancy) are kept next to the object
    cmd = [HIPCC, *flags, '-Rpass-analysis=kernel-resource-usage', '-c', src, '-o', obj + '.tmp']
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'hipcc failed for {src}:\n{r.stderr[-4000:]}')
    with open(obj + '.resources.txt', 'w') as f:
        f.write('\n'.join(l for l in r.stderr.splitlines() if 'remark' in l) + '\n')
    os.replace(obj + '.tmp', obj)
    with open(stamp, 'w') as f:
        f.write(key)
    return obj, True


def build(procs=None, jobs=None, verbose=True, lib=LIB, force=False):
    """Generate, compile and link.  Objects are reused when their inputs are
    unchanged, unless force is set (then every unit is compiled again)."""
    procs = list(procs or PROCESSES)
    tag = hashlib.sha1(','.join(procs).encode()).hexdigest()[:10]
    build_dir = os.path.join(ROOT, '_build', f'set_{tag}')
    os.makedirs(OBJ, exist_ok=True)
    units = generate_sources(procs, build_dir)
    # the largest units first: the batch kernel and the process with most diagrams
    units.sort(key=lambda u: (not u[0].endswith('batch.hip'), 'ggg' not in u[0], -len(os.path.basename(u[0]))))
    jobs = jobs or min(8, os.cpu_count() or 4)
    ident = hashlib.sha1()
    for src, _, deps in sorted(units):
        for d in [src] + sorted(deps):
            with open(d, 'rb') as f:
                ident.update(f.read())
    build_id = ident.hexdigest()[:16]
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, src, obj, deps, build_dir, force, build_id): src for src, obj, deps in units}
        for f in cf.as_completed(futs):
            obj, rebuilt = f.result()
            objs.append(obj)
            if verbose:
                print(('compiled ' if rebuilt else 'up to date ') + os.path.basename(futs[f]), flush=True)
    objs.sort()
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    cmd = [HIPCC, f'--offload-arch={ARCH}', '-shared', '-fPIC', *objs, '-o', lib + '.tmp']
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'link failed:\n{r.stderr[-4000:]}')
    os.replace(lib + '.tmp', lib)
    if verbose:
        print('linked', lib, flush=True)
    return lib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--procs', default=','.join(PROCESSES))
    ap.add_argument('-j', type=int, default=None)
    ap.add_argument('--force', action='store_true', help='compile every unit again')
    args = ap.parse_args()
    build(args.procs.split(','), args.j, force=args.force)


if __name__ == '__main__':
    main()
