"""Write the stored expected values used by the GPU parity tests.

Calls only the oracle (and the seeded input generator): no value here comes
from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py [ggttggg] [ggttgggg]
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


def main(which):
    for name in which or ('ggttggg', 'ggttgggg'):
        {'ggttggg': ggttggg, 'ggttgggg': ggttgggg}[name]()


if __name__ == '__main__':
    main(sys.argv[1:])
