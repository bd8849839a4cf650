"""The oracle's own failure flags, forced through imported states (the same conditions
the library reports): a NaN population sets the NaN bit, a liquid cell next to gas
the invariant bit, a sphere that reaches a periodic face the particle bit, and a step
with any of them returns an error; sphere positions outside the supported region are
refused by the setter."""
import numpy as np
import pytest

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


ERR_ARG, ERR_PART = 16, 32


def _one_sphere(x, periodic=(1, 1, 1), n=(24, 24, 24), u=(0.0, 0.0, 0.0), R=3.0):
    p = W.Particles(x=np.array([x], dtype=np.float64), u=np.array([u], dtype=np.float64),
                    omega=np.zeros((1, 3)), R=np.array([R]), rho_p=np.array([1.5]))
    return W.Workload(name="one", n=n, trt=True, tau=0.6, g=(0.0, 0.0, 0.0), zs=-1.0, steps=0,
                      periodic=periodic, particles=p)


def test_unsupported_sphere_positions_are_rejected():
    """Coverage, pair search and lever arms do not wrap: a centre closer than R + 1
    to a periodic face (R + 2 on the far side), outside a walled box, or not finite
    is refused by the particle setter, as the library refuses it."""
    ok = _one_sphere((12.0, 12.0, 12.0))
    o = O.Oracle(ok, n_threads=2)
    for bad, per in [((3.5, 12.0, 12.0), (1, 1, 1)), ((12.0, 19.5, 12.0), (1, 1, 1)),
                     ((12.0, 12.0, 24.2), (0, 0, 0)), ((-0.7, 12.0, 12.0), (0, 0, 0)),
                     ((np.nan, 12.0, 12.0), (1, 1, 1)), ((12.0, np.inf, 12.0), (0, 0, 0))]:
        w = _one_sphere(bad, periodic=per)
        with pytest.raises(ValueError):
            O.Oracle(w, n_threads=2).close()
    # the limits themselves are allowed: R + 1 and n - R - 2 on periodic axes, the
    # faces at -1/2 and n - 1/2 on walled ones
    for x, per in [((4.0, 19.0, 12.0), (1, 1, 1)), ((-0.5, 12.0, 23.5), (0, 0, 0))]:
        O.Oracle(_one_sphere(x, periodic=per), n_threads=2).close()
    o.close()


def test_sphere_reaching_a_periodic_face_sets_the_flag():
    """A sphere driven toward a periodic face: once its centre is closer than R + 1
    the step reports it (and keeps running)."""
    w = _one_sphere((5.0, 12.0, 12.0), u=(-0.2, 0.0, 0.0)).replace(g=(-1e-3, 0.0, 0.0))
    o = O.Oracle(w, n_threads=2)
    rc = 0
    for _ in range(30):
        rc = o.step(1)
        if rc:
            break
    assert rc != 0 and o.error & ERR_PART
    assert not o.error & ~(ERR_PART | ERR_ARG)
    o.close()
