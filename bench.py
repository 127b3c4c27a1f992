"""Throughput benchmark: ME evaluations per second on one MI355X.

Workload (default): g g -> t tbar g g g, 262144 flat RAMBO events at
sqrt(s) = 1500 GeV (seed 1003), m_t = 173 GeV, alpha_s = 0.118, FP64
diagrams and FP64 colour sum, all good helicities.  A step is one
me_compute call over the whole batch (momenta resident in HBM, output left
in HBM).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

FP64_VALU_PEAK_TFLOPS = 78.6      # MI355X: 256 CUs x 2.4 GHz x 128 FP64 flops/clk (FMA = 2)

# HBM bytes per launch of the FP64 diagram kernel (averaged over its launches in one call, like
# the kernel time), from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by the same counters on a
# plain 2 GiB copy (x2.0 and x1.0), keyed by the workload and the launch configuration that fixes
# the work items (persistent, helicities/item, executor; the persistent grid's size does not change
# what an item reads and writes); the numbers and the commands are in the named profile and hold
# only for the kernel they were taken on.
# key: (process, nevt, (persistent, hel_per_item, executor, split_wpe, split_rounds, bg_variant)) as me_autotune
# reports them.
TRAFFIC_KEY = ('persistent', 'hel_per_item', 'executor', 'split_wpe', 'split_rounds', 'bg_variant')
MEASURED_TRAFFIC = {
    # helicity-recycling kernel with the colour form and helicity sum fused, 16 launches per call
    ('gg_ttxggg', 262144, (0, 0, 3, 0, 0, 4)): (8.099e9, 'profiles/bgh_kernel_gg_ttxggg_262144.md'),
}

NPAR = {'gg_ttx': 4, 'gg_ttxg': 5, 'gg_ttxgg': 6, 'gg_ttxggg': 7, 'gg_ttxgggg': 8}
SEED = {'gg_ttx': 1001, 'gg_ttxg': 1004, 'gg_ttxgg': 1002, 'gg_ttxggg': 1003, 'gg_ttxgggg': 1005}


_ORACLE = {}


def _oracle_chunk(args):
    """One worker's share of the CPU baseline: the oracle on a chunk of events, one
    thread (numpy's BLAS pool limited to one thread in the worker)."""
    npar, mom, alpha_s = args
    from threadpoolctl import threadpool_limits
    from oracle import me as ome
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ome.matrix_element(_ORACLE[npar], mom, alpha_s)
        return mom.shape[0], time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                return line.split(':', 1)[1].strip()
    except OSError:
        pass
    return 'unknown'


def cpu_baseline(process, mom, alpha_s, budget_s):
    """The oracle on the host cores (rank 0, N=1): a one-core calibration on a few
    events, then one chunk per worker process (one per host core of this process's
    CPU share, at most 16), each sized to take about half the budget; the value is
    all the events over the wall time of the pooled run."""
    import multiprocessing as mp

    from oracle import me as ome
    npar = NPAR[process]
    if npar not in _ORACLE:
        _ORACLE[npar] = ome.process(npar)
    workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    n1 = {4: 256, 5: 64, 6: 16, 7: 4, 8: 1}[npar]
    done1, t1 = _oracle_chunk((npar, mom[:n1], alpha_s))
    rate1 = done1 / t1
    per = int(max(1, min(rate1 * 0.5 * budget_s, mom.shape[0] // workers)))
    chunks = [(npar, mom[n1 + w * per:n1 + (w + 1) * per], alpha_s) for w in range(workers)]
    chunks = [c for c in chunks if c[1].shape[0] > 0]
    w0 = time.perf_counter()
    with mp.get_context('fork').Pool(len(chunks)) as pool:
        res = pool.map(_oracle_chunk, chunks, chunksize=1)
    wall = time.perf_counter() - w0
    done = sum(r[0] for r in res)
    per_core = sorted(r[0] / r[1] for r in res)
    return {'value': done / wall, 'unit': 'ME evals/s', 'cores': len(chunks), 'kind': 'oracle',
            'single_core_value': per_core[len(per_core) // 2], 'cpu_model': _cpu_model(),
            'host_cpus': os.cpu_count(),
            'sample': f'events {n1}..{n1 + done - 1} of the same {process} workload ({per} per worker process, '
                      f'one thread each, all helicities, numpy FP64 oracle, {wall:.1f} s wall); single-core value: '
                      f'median worker rate in that run (sized from events 0..{n1 - 1}, {t1:.1f} s on one core)'}


HBM_PEAK_TBS = 8.0


def binding_resource(traffic, ms_per_launch, achieved_tflops):
    """Which roof the dominant kernel presses on: its measured HBM traffic per launch
    over its duration against HBM peak, next to its FP64 rate against the FP64 peak."""
    alu = achieved_tflops / FP64_VALU_PEAK_TFLOPS
    if not traffic:
        return {'fp64_frac': alu, 'hbm_frac': None, 'resource': 'unmeasured (no counter run for this kernel)'}
    tbs = traffic[0] / (ms_per_launch * 1e-3) / 1e12
    hbm = tbs / HBM_PEAK_TBS
    return {'fp64_frac': alu, 'hbm_TBps': tbs, 'hbm_frac': hbm,
            'resource': 'HBM (register-spill traffic)' if hbm > alu else 'FP64 vector ALU issue'}


def surrogate_leg(args, process, nevt, mom, dmom, binding, rambo, executor=None, bg_variant=0):
    """Mixed colour sum + surrogate two-stage unweighting of the same workload.

    The surrogate is trained on separate events labelled by the exact path;
    'value' is the effective rate: events resolved by two-stage unweighting per
    second of (features + network + stage-1 selection + exact |M|^2 of the
    stage-1 events + stage 2).  The one-stage reference needs the exact |M|^2 of
    every event.
    """
    import numpy as np
    import torch

    from paper_2510_05392_amd.surrogate import SurrogatePipeline
    npar = NPAR[process]
    print('# bench surrogate: training', file=sys.stderr, flush=True)
    try:
        exact_mode = binding.ME_CS_FP16X2
        pipe = SurrogatePipeline(process, width=256, depth=4, seed=11, alpha_s=args.alpha_s,
                                 colorsum_mode=exact_mode)
    except binding.MeError:
        # processes with only the team executor have the FP64 colour sum
        exact_mode = binding.ME_CS_FP64
        pipe = SurrogatePipeline(process, width=256, depth=4, seed=11, alpha_s=args.alpha_s,
                                 colorsum_mode=exact_mode)
    if executor is not None:
        # the exact path on the executor (and Berends-Giele kernel) the FP64 run was tuned to
        pipe.me.me_set_executor(executor)
        if executor == binding.ME_EXEC_BG:
            pipe.me.me_set_bg(bg_variant)
    train = torch.from_numpy(rambo.generate(npar, args.sur_train, 2001)).cuda()
    t0 = time.perf_counter()
    hist = pipe.fit(train, epochs=args.sur_epochs, batch=4096, lr=2e-3, lr_final=1e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del train
    val = torch.from_numpy(rambo.generate(npar, min(32768, args.sur_cal), 2003)).cuda()
    rms, worst = pipe.log_error(val)
    calm, calw = rambo.generate(npar, args.sur_cal, 2005, return_weights=True)
    dcal, dcw = torch.from_numpy(calm).cuda(), torch.from_numpy(calw).cuda()
    what_max, x_max = pipe.calibrate(dcal, dcw, quantile=0.99)
    w_max = pipe.exact_weight_max(dcal, dcw, 0.99)
    _, wps = rambo.generate(npar, nevt, SEED[process], return_weights=True)
    dw = torch.from_numpy(wps).cuda()
    g = torch.Generator(device='cuda').manual_seed(7)
    r1 = torch.rand(nevt, dtype=torch.float64, device='cuda', generator=g)
    r2 = torch.rand(nevt, dtype=torch.float64, device='cuda', generator=g)
    print('# bench surrogate: unweighting', file=sys.stderr, flush=True)
    pipe.unweight(dmom, dw, r1, r2, what_max, x_max)            # warm-up
    two = pipe.unweight(dmom, dw, r1, r2, what_max, x_max)
    one = pipe.unweight_exact(dmom, dw, r2, w_max)
    return {'value': nevt / two['time_total'], 'unit': 'ME evals/s (effective)',
            'method': 'two-stage unweighting: BF16 MLP stage 1, '
                      + ('split-FP16' if exact_mode == binding.ME_CS_FP16X2 else 'FP64') + ' exact |M|^2 stage 2',
            'n_events': nevt, 'stage1_events': two['stage1'], 'exact_calls_saved': 1 - two['stage1'] / nevt,
            'accepted': two['accepted'], 'overweights': two['overweight'],
            'overweight_fraction': two['overweight'] / max(1, two['accepted']),
            'effective_sample_size': two['ess'],
            'ess_value': two['ess'] / two['time_total'],
            'one_stage_accepted': one['accepted'], 'one_stage_value': nevt / one['time_total'],
            'one_stage_effective_sample_size': one['ess'],
            'one_stage_ess_value': one['ess'] / one['time_total'],
            'unweighting_efficiency': two['accepted'] / nevt,
            'one_stage_efficiency': one['accepted'] / nevt,
            'rms_log_error': rms, 'max_log_error': worst, 'train_events': args.sur_train,
            'maxima': f'0.99 quantiles of a {args.sur_cal}-event calibration sample '
                      '(events above: residual weights > 1)',
            'train_epochs': args.sur_epochs, 'train_seconds': t_train, 'final_mse': hist[-1],
            'stated_err': 'exact path split FP16 <= 1e-5 relative per event; unweighted sample unbiased'}


def batch_leg(args, binding, rambo):
    """Uneven multi-process batch (8192 gg->ttg + 65536 gg->ttgg + 16384 gg->ttggg) in one
    persistent launch, against the three processes' own me_compute calls in sequence."""
    import torch
    names = ['gg_ttxg', 'gg_ttxgg', 'gg_ttxggg']
    sizes = [8192, 65536, 16384]
    moms = [torch.from_numpy(rambo.generate(NPAR[n], k, SEED[n])).cuda() for n, k in zip(names, sizes)]
    outs = [torch.empty(k, dtype=torch.float64, device='cuda') for k in sizes]
    hs = [binding.MatrixElement(n) for n in names]
    single = [binding.MatrixElement(n) for n in names]
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps

    t_batch = timed(lambda: binding.me_compute_batch(hs, moms, sizes, args.alpha_s, outs, stream))
    t_seq = timed(lambda: [m.me_compute(d, k, args.alpha_s, o, stream)
                           for m, d, k, o in zip(single, moms, sizes, outs)])
    n = sum(sizes)
    return {'segments': dict(zip(names, sizes)), 'ms_one_launch': t_batch, 'ms_three_launches': t_seq,
            'value': n / (t_batch * 1e-3), 'unit': 'ME evals/s (all segments)'}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=10)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--process', default='gg_ttxggg')
    ap.add_argument('--nevt', type=int, default=262144)
    ap.add_argument('--alpha-s', type=float, default=0.118)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--fp64-only', action='store_true', help='skip the mixed-precision run')
    ap.add_argument('--autotune', action=argparse.BooleanOptionalAction, default=True,
                    help='pick the FP64 launch configuration with the library autotuner first')
    ap.add_argument('--no-graph', action='store_true', help='do not replay me_compute from a hipGraph')
    ap.add_argument('--launch', default=None,
                    help='fixed FP64 launch "persistent,waves_per_simd,hel_per_item,target_waves,executor'
                         '[,bg_variant]" instead of autotuning (profiling runs)')
    ap.add_argument('--surrogate', action=argparse.BooleanOptionalAction, default=True,
                    help='also measure mixed precision + surrogate two-stage unweighting')
    ap.add_argument('--sur-train', type=int, default=131072)
    ap.add_argument('--sur-epochs', type=int, default=12)
    ap.add_argument('--sur-cal', type=int, default=65536, help='calibration events for the maxima')
    ap.add_argument('--cpu-budget', type=float, default=20.0)
    ap.add_argument('--batch', action='store_true',
                    help='also time the uneven multi-process batch in one persistent launch')
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py runs on one GPU only (got --gpus {args.gpus}): events are independent, '
              'so more GPUs would each run this same kernel on their own share of events.',
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_05392_amd import binding, flops, rambo

    process, nevt = args.process, args.nevt
    mom = rambo.generate(NPAR[process], nevt, SEED[process])
    dev = torch.device('cuda:0')
    dmom = torch.from_numpy(mom).to(dev)
    stream = torch.cuda.current_stream(dev)

    def run(mode, executor=None):
        """Time me_compute over the batch in one colour-sum mode (on the given executor,
        else the tuned or default one)."""
        out = torch.empty(nevt, dtype=torch.float64, device=dev)
        m = binding.MatrixElement(process, colorsum_mode=mode, use_graph=not args.no_graph)
        tuned = None
        if args.launch and mode == binding.ME_CS_FP64:
            p_, w_, h_, t_, x_, *v_ = (int(v) for v in args.launch.split(','))
            v_ = v_[0] if v_ else 0
            m.me_set_launch(p_, w_, h_, t_)
            m.me_set_executor(x_)
            if x_ == binding.ME_EXEC_BG:
                m.me_set_bg(v_)
            tuned = {'persistent': p_, 'waves_per_simd': w_, 'hel_per_item': h_, 'target_waves': t_,
                     'executor': x_, 'split_wpe': 0, 'split_fchunk': 0, 'split_rounds': 0, 'colour_grid': 0,
                     'bg_variant': v_}
        elif args.autotune:
            nt = min(nevt, 65536)
            print(f'# bench autotune on {nt} events (mode {mode})', file=sys.stderr, flush=True)
            tuned = m.me_autotune(dmom[:nt], nt, args.alpha_s, out[:nt], stream)
        elif executor is not None:
            m.me_set_executor(executor)
        print(f'# bench {process} nevt={nevt} mode={mode}: warmup {args.warmup}', file=sys.stderr,
              flush=True)
        for _ in range(max(1, args.warmup)):
            m.me_compute(dmom, nevt, args.alpha_s, out, stream)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        # the timed region: eager calls with every kernel bracketed by events on the
        # stream it runs on (per-kernel durations for the roofline); the same steps
        # replayed from the captured graph are timed after it
        timing = mode == binding.ME_CS_FP64
        if timing:
            m.me_set_kernel_timing(True)
        print(f'# bench timing {args.steps} steps', file=sys.stderr, flush=True)
        start.record(stream)
        for _ in range(args.steps):
            m.me_compute(dmom, nevt, args.alpha_s, out, stream)
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / args.steps
        ktimes = None
        if timing:
            ktimes = m.me_kernel_times()
            m.me_set_kernel_timing(False)
        res = out.cpu().numpy()
        if not np.all(np.isfinite(res)):
            print('non-finite matrix elements', file=sys.stderr)
            sys.exit(1)
        graph_ms = None
        if timing and not args.no_graph:
            m.me_compute(dmom, nevt, args.alpha_s, out, stream)   # graph (captured in the warmup) warm
            torch.cuda.synchronize()
            start.record(stream)
            for _ in range(args.steps):
                m.me_compute(dmom, nevt, args.alpha_s, out, stream)
            stop.record(stream)
            torch.cuda.synchronize()
            graph_ms = start.elapsed_time(stop) / args.steps
            if not np.array_equal(out.cpu().numpy(), res):
                print('graph replay differs from eager evaluation', file=sys.stderr)
                sys.exit(1)
        return ms, res, len(m.me_good_helicities()), tuned, ktimes, graph_ms

    ms, res, nhel, tuned, ktimes, graph_ms = run(binding.ME_CS_FP64)
    value = nevt / (ms * 1e-3)
    mixed = None
    if not args.fp64_only:
        try:
            ms_m, res_m, _, tuned_m, _, _ = run(binding.ME_CS_FP16X2, (tuned or {}).get('executor'))
            rel = np.abs(res_m / res - 1)
            mixed = {'colorsum': 'split FP16 hi+lo on MFMA, FP32 accumulation, FP64 row dots',
                     'launch': tuned_m,
                     'value': nevt / (ms_m * 1e-3), 'unit': 'ME evals/s', 'ms_per_step': ms_m,
                     'max_rel_err_vs_fp64': float(rel.max()),
                     'rms_rel_err_vs_fp64': float(np.sqrt(np.mean(rel ** 2))), 'stated_bound': 1e-5}
        except binding.MeError as exc:
            mixed = {'skipped': str(exc)}

    traffic = None
    if tuned:
        key = (process, nevt, tuple(tuned[k] for k in TRAFFIC_KEY))
        traffic = MEASURED_TRAFFIC.get(key)
    executor = (tuned or {}).get('executor', 0)
    bg_variant = (tuned or {}).get('bg_variant', 0)
    bgk = {0: 'bg_kernel', 1: 'bg_kernel', 2: 'bg_kernel', 3: 'bgh_kernel'}.get(bg_variant, 'bgh_fused_kernel')
    kname = {1: f'team_kernel<{process}_team>', 2: f'sums_kernel<{process}>',
             3: f'{bgk}<{NPAR[process] - 2}>'}.get(executor, f'me_kernel<{process}>')
    ncol = {'gg_ttx': 2, 'gg_ttxg': 6, 'gg_ttxgg': 24, 'gg_ttxggg': 120, 'gg_ttxgggg': 720}[process]
    cname = (f'colour_f64_tri_kernel<{ncol}>' if ncol > 128 else f'colour_f64_kernel<{ncol}>') \
        if executor in (2, 3) else 'colour_mfma_kernel'
    # the dominant kernel is the diagram kernel; its algorithmic flops per (event, helicity)
    f_unit = flops.diagram_kernel(process, executor, bg_variant)
    tot_ms, launches = ktimes
    kms = tot_ms[binding.ME_KT_DIAGRAM]
    achieved = f_unit * nhel * nevt * args.steps / (kms * 1e-3) / 1e12
    kernels = {name: {'ms_total': tot_ms[k], 'launches': launches[k],
                      'ms_per_launch': tot_ms[k] / launches[k] if launches[k] else None}
               for k, name in ((binding.ME_KT_DIAGRAM, kname),
                               (binding.ME_KT_FLOWS, f'flows_kernel<{process}>'),
                               (binding.ME_KT_COLOUR, cname),
                               (binding.ME_KT_REDUCE, 'reduce_rows_kernel' if executor == 3 and bg_variant >= 3
                                else 'reduce_chunks_kernel')) if launches[k]}
    line = {
        'metric': 'ME evals/s', 'value': value, 'unit': 'ME evals/s', 'n_gpus': 1,
        'steps': args.steps, 'warmup': args.warmup, 'ms_per_step': ms,
        'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64',
        'data': 'synthetic (seeded flat RAMBO phase space)',
        'config': {'workload': f'{process} LO |M|^2, FP64 diagrams + FP64 colour sum', 'process': process,
                   'nevt': nevt, 'sqrt_s_GeV': 1500.0, 'mt_GeV': 173.0, 'alpha_s': args.alpha_s,
                   'good_helicities': nhel, 'parallelism': 'single GPU', 'launch': tuned,
                   'timed': 'eager calls, kernels bracketed by events',
                   'graph_replay_ms_per_step': graph_ms},
        'roofline': {'bound': 'alu', 'achieved': achieved, 'peak': FP64_VALU_PEAK_TFLOPS,
                     'unit': 'TFLOP/s', 'frac': achieved / FP64_VALU_PEAK_TFLOPS,
                     'traffic': traffic[0] if traffic else None,
                     'traffic_source': traffic[1] if traffic else None,
                     'kernel': kname, 'flops_per_event_helicity': f_unit,
                     'flops_source': 'operations of the generated code, counted (tests/test_generator.py)',
                     'kernel_ms_per_launch': kms / launches[binding.ME_KT_DIAGRAM],
                     'launches': launches[binding.ME_KT_DIAGRAM],
                     'binding_resource': binding_resource(traffic, kms / launches[binding.ME_KT_DIAGRAM],
                                                          achieved)},
        'kernels': kernels,
    }
    if mixed is not None:
        line['mixed'] = mixed
    if args.surrogate:
        line['surrogate'] = surrogate_leg(args, process, nevt, mom, dmom, binding, rambo,
                                          (tuned or {}).get('executor'), (tuned or {}).get('bg_variant', 0))
    if args.batch:
        print('# bench uneven batch', file=sys.stderr, flush=True)
        line['uneven_batch'] = batch_leg(args, binding, rambo)
    if not args.no_cpu_baseline:
        print('# bench cpu baseline (oracle)', file=sys.stderr, flush=True)
        line['cpu_baseline'] = cpu_baseline(process, mom, args.alpha_s, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == '__main__':
    main()
