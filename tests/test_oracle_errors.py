"""The oracle's own failure flags, forced through imported states (the same conditions
the library reports): a NaN population sets the NaN bit, a liquid cell next to gas
the invariant bit, and a step with either returns an error."""
import numpy as np

import oracle as O
from paper_1712_07028_amd import workloads as W

ERR_LG, ERR_NAN = 1, 2


def test_nan_population_sets_the_flag():
    o = O.Oracle(W.bubble_column_small(), n_threads=2)
    F = o.get(O.F)
    F[3, 20, 2, 2] = np.nan
    o.set(O.F, F)
    assert o.step(1) != 0 and o.error & ERR_NAN
    o.close()


def test_liquid_next_to_gas_sets_the_flag():
    o = O.Oracle(W.bubble_column_small(), n_threads=2)
    fl = o.get(O.FLAGS)
    z, y, x = np.argwhere(fl == O.IFC)[0]
    fl[z, y, x] = O.LIQ
    o.set(O.FLAGS, fl)
    assert o.step(1) != 0 and o.error & ERR_LG
    o.close()
