"""Write the stored expected values used by the GPU parity tests.

Calls only the oracle (and the seeded input generator): no value here comes
from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py [ggttggg] [ggttgggg] [sde_ggttggg] [wide_c1] ...

(the wide_* sets run the oracle on every host core; wide_c2 takes about ten
minutes of eight cores, wide_c4a about half an hour)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import me  # noqa: E402
from paper_2510_05392_amd import rambo  # noqa: E402

AS = 0.118


def values(proc, mom):
    """Oracle |M|^2 in float64 and in extended precision (np.longdouble arithmetic,
    rounded to float64 for storage) to adjudicate ill-conditioned events."""
    return (me.matrix_element(proc, mom, AS),
            me.matrix_element(proc, mom.astype(np.longdouble), AS).astype(np.float64))


def ggttggg():
    proc = me.process(7)
    # g g -> t tbar g g g: three 64-event tiles and a ragged tail
    mom = rambo.generate(7, 197, 1003)
    m64, mext = values(proc, mom)
    np.savez_compressed(os.path.join(HERE, 'gg_ttxggg_seed1003_first197.npz'), momenta=mom,
                        me=m64, me_ext=mext)
    # the 262144-event benchmark workload, 64 events spread over the whole file
    full = rambo.generate(7, 262144, 1003)
    idx = np.unique(np.concatenate([np.linspace(0, 262143, 62).astype(int), [1, 262142]]))
    m64, mext = values(proc, full[idx])
    np.savez_compressed(os.path.join(HERE, 'gg_ttxggg_seed1003_n262144_sampled.npz'), index=idx,
                        momenta=full[idx], me=m64, me_ext=mext)


def ggttgggg():
    # g g -> t tbar g g g g, the 32768-event workload: 24 events spread over it
    proc = me.process(8)
    full = rambo.generate(8, 32768, 1005)
    idx = np.unique(np.concatenate([np.arange(3), np.linspace(3, 32767, 21).astype(int)]))
    m64, mext = values(proc, full[idx])
    np.savez_compressed(os.path.join(HERE, 'gg_ttxgggg_seed1005_n32768_sampled.npz'), index=idx,
                        momenta=full[idx], me=m64, me_ext=mext)


def sde_ggttggg():
    # single-diagram-enhancement channel sums of g g -> t tbar g g g: sum over all
    # 128 helicities of |A_c|^2 for each of the 945 channels, 16 events of seed 1003
    from oracle import sde
    proc = me.process(7)
    mom = rambo.generate(7, 16, 1003)
    a2 = sde.channel_amp2(proc, mom, AS)
    np.savez_compressed(os.path.join(HERE, 'gg_ttxggg_seed1003_sde16.npz'), momenta=mom, amp2=a2)


# --- the wide parity sets, computed on every host core (multiprocessing over event
# chunks; the oracle's arithmetic is unchanged)

_PROC = {}


def _chunk_values(args):
    npar, mom, ext = args
    if npar not in _PROC:
        _PROC[npar] = me.process(npar)
    if ext:
        return me.matrix_element(_PROC[npar], mom.astype(np.longdouble), AS).astype(np.float64)
    return me.matrix_element(_PROC[npar], mom, AS)


def pooled_values(npar, mom, ext=False, chunk=256, workers=None):
    import multiprocessing as mp
    workers = workers or len(os.sched_getaffinity(0))
    parts = [(npar, mom[i:i + chunk], ext) for i in range(0, len(mom), chunk)]
    with mp.get_context('fork').Pool(workers) as pool:
        return np.concatenate(pool.map(_chunk_values, parts, chunksize=1))


def _save(name, **arrays):
    np.savez_compressed(os.path.join(HERE, name), **arrays)
    print('wrote', name, flush=True)


def wide_c1():
    # g g -> t tbar g g, the whole 524288-event workload (seed 1002), FP64 oracle values
    mom = rambo.generate(6, 524288, 1002)
    _save('gg_ttxgg_seed1002_n524288.npz', me=pooled_values(6, mom, chunk=2048))


def wide_c2():
    # g g -> t tbar g g g, the first 16384 events of the 262144-event workload (seed
    # 1003), FP64 oracle values (the tests take extended-precision values of the few
    # events they need to adjudicate from the oracle at run time)
    mom = rambo.generate(7, 16384, 1003)
    _save('gg_ttxggg_seed1003_first16384.npz', me=pooled_values(7, mom))


def wide_c4a(n=1024):
    # g g -> t tbar g g g g, the first n events of the 32768-event workload (seed 1005);
    # 64-event chunks (about 15 minutes each on one core)
    mom = rambo.generate(8, n, 1005)
    _save(f'gg_ttxgggg_seed1005_first{n}.npz', me=pooled_values(8, mom, chunk=64))


def _rotate(mom, seed):
    # one random proper rotation of the three-momenta of each event: the
    # helicity-summed |M|^2 is unchanged, the FP64 rounding of its evaluation is not
    rng = np.random.default_rng(seed)
    out = np.array(mom, dtype=np.float64, copy=True)
    for e in range(len(out)):
        q, r = np.linalg.qr(rng.normal(size=(3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        out[e, :, 1:] = out[e, :, 1:] @ q.T
    return out


def wide_c4a_rot(n=1024, workers=None):
    # the FP64 conditioning of the oracle on the same events: its values on one random
    # rotation of each (two FP64 evaluations differ by about their rounding error; no
    # extended-precision values are stored for these events)
    mom = _rotate(rambo.generate(8, n, 1005), 4242)
    _save(f'gg_ttxgggg_seed1005_first{n}_rot.npz', me_rot=pooled_values(8, mom, chunk=16, workers=workers))


def wide_c4b():
    # the uneven batch: the first 1024 events of each segment
    out = {}
    for name, npar, seed in (('gg_ttxg', 5, 1004), ('gg_ttxgg', 6, 1006), ('gg_ttxggg', 7, 1007)):
        mom = rambo.generate(npar, 1024, seed)
        out[f'{name}_me'] = pooled_values(npar, mom, chunk=64)
        if npar == 7:
            out[f'{name}_me_ext'] = pooled_values(npar, mom, ext=True, chunk=32)
    _save('batch_first1024.npz', **out)


def c3_labels():
    # the surrogate's training labels: the first 4096 events of the 2097152-event
    # gg -> t tbar g g training sample (seed 2001), FP64 oracle values
    mom = rambo.generate(6, 4096, 2001)
    _save('gg_ttxgg_seed2001_first4096.npz', me=pooled_values(6, mom, chunk=256))


def _kappa_chunk(args):
    """Condition number of the colour sum of each event: with J = A + iB per helicity,
    kappa = sum_h (|A|^T |C| |A| + |B|^T |C| |B|) / sum_h (A^T C A + B^T C B)."""
    npar, mom = args
    if npar not in _PROC:
        _PROC[npar] = me.process(npar)
    proc = _PROC[npar]
    cf = np.asarray(proc.cf, dtype=np.float64)
    acf = np.abs(cf)
    num = np.zeros(mom.shape[0])
    den = np.zeros(mom.shape[0])
    for h in range(proc.nhel):
        j = me.jamps(proc, mom, h, AS)
        for part in (j.real, j.imag):
            num += np.einsum('ei,ij,ej->e', np.abs(part), acf, np.abs(part))
            den += np.einsum('ei,ij,ej->e', part, cf, part)
    return num / den


def kappa():
    # colour-sum condition numbers for the per-event mixed-precision bounds:
    # gg -> tt (first 512 events of seed 1001), gg -> ttgg (first 256 of seed 1002),
    # gg -> ttggg (the 64 sampled events of the 262144-event workload)
    import multiprocessing as mp
    workers = len(os.sched_getaffinity(0))
    out = {}
    full = rambo.generate(7, 262144, 1003)
    idx = np.load(os.path.join(HERE, 'gg_ttxggg_seed1003_n262144_sampled.npz'))['index']
    sets = {'gg_ttx': (4, rambo.generate(4, 512, 1001)), 'gg_ttxgg': (6, rambo.generate(6, 256, 1002)),
            'gg_ttxggg': (7, full[idx])}
    with mp.get_context('fork').Pool(workers) as pool:
        for name, (npar, mom) in sets.items():
            parts = [(npar, mom[i:i + 8]) for i in range(0, len(mom), 8)]
            out[name] = np.concatenate(pool.map(_kappa_chunk, parts, chunksize=1))
    _save('colour_kappa.npz', **out)


GENERATORS = {'kappa': kappa, 'ggttggg': ggttggg, 'ggttgggg': ggttgggg, 'sde_ggttggg': sde_ggttggg,
              'wide_c1': wide_c1, 'wide_c2': wide_c2, 'wide_c4a': wide_c4a, 'wide_c4a_rot': wide_c4a_rot,
              'wide_c4b': wide_c4b,
              'c3_labels': c3_labels}


def main(which):
    for name in which or tuple(GENERATORS):
        GENERATORS[name]()


if __name__ == '__main__':
    main(sys.argv[1:])
