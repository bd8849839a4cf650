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
    """A centre outside a walled box (faces at -1/2 and n - 1/2) or not finite is
    refused by the particle setter, as the library refuses it; on periodic axes any
    finite centre is taken (into [0, n)), and the faces of a walled box themselves
    are allowed."""
    for bad, per in [((12.0, 12.0, 24.2), (0, 0, 0)), ((-0.7, 12.0, 12.0), (0, 0, 0)),
                     ((np.nan, 12.0, 12.0), (1, 1, 1)), ((12.0, np.inf, 12.0), (0, 0, 0))]:
        with pytest.raises(ValueError):
            O.Oracle(_one_sphere(bad, periodic=per), n_threads=2).close()
    for x, per in [((-0.5, 12.0, 23.5), (0, 0, 0)), ((0.5, 23.9, 12.0), (1, 1, 1))]:
        O.Oracle(_one_sphere(x, periodic=per), n_threads=2).close()
    o = O.Oracle(_one_sphere((-3.0, 27.5, 12.0), periodic=(1, 1, 0)), n_threads=2)
    np.testing.assert_allclose(o.particles_get(1)["x"][0], [21.0, 3.5, 12.0], rtol=0, atol=1e-12)
    o.close()


def test_sphere_with_a_nan_force_sets_the_flag():
    """A NaN population at a cell with links into a sphere makes its force, velocity
    and centre NaN: the step reports the particle flag beside the NaN flag (a sphere
    cannot leave a walled box otherwise: the face reverses its velocity)."""
    w = _one_sphere((12.0, 12.0, 12.0), periodic=(0, 1, 1))
    o = O.Oracle(w, n_threads=2)
    F = o.get(O.F)
    assert o.get(O.FLAGS)[12, 12, 16] == O.LIQ and o.get(O.FLAGS)[12, 12, 15] == O.SOL
    F[2, 12, 12, 16] = np.nan  # pulled by the particle link of the cell itself
    o.set(O.F, F)
    assert o.step(1) != 0 and o.error & ERR_PART
    o.close()
