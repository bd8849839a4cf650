"""Failure detection on the GPU: conditions forced from the host through imported
states or a configuration, reported by the next synchronising call with their own
error codes.  Every kernel still runs to its end: the errors are latched on the
device, never trapped.
  - a NaN population in a liquid cell: FSL_E_NUMERIC;
  - a liquid cell next to a gas cell (the interface layer broken): FSL_E_INVARIANT;
  - conversion lists of capacity 1 with many cells filling at once: FSL_E_CAPACITY.
The argument checks of the particle setter and of the differentiation window (no
moving faces) are checked here too: they need a context on the device.
"""
import numpy as np
import pytest

import oracle as O
import paper_1712_07028_amd as fsl
from paper_1712_07028_amd import workloads as W

from test_oracle_split import ball, hand_state, interface_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    fsl.load_library()


def test_nan_population_is_reported():
    w = W.bubble_column_small()
    s = fsl.Sim(w)
    F = s.get(fsl.FIELD_F)
    assert s.get(fsl.FIELD_FLAGS)[20, 2, 2] == fsl.LIQ  # far from the bubble and the surface
    F[3, 20, 2, 2] = np.nan
    s.set(fsl.FIELD_F, F)
    s.step(1)
    with pytest.raises(fsl.FslError, match="NaN"):
        s.sync()
    s.close()


def test_liquid_next_to_gas_is_reported():
    w = W.bubble_column_small()
    s = fsl.Sim(w)
    fl = s.get(fsl.FIELD_FLAGS)
    z, y, x = np.argwhere(fl == fsl.IFC)[0]
    fl[z, y, x] = fsl.LIQ  # an interface cell of the surface made liquid: it touches the gas
    s.set(fsl.FIELD_FLAGS, fl)
    s.step(1)
    with pytest.raises(fsl.FslError, match="gas neighbour"):
        s.sync()
    s.close()


def test_list_overflow_is_reported():
    n = (16, 16, 16)
    gas = ball(n, (8.0, 8.0, 8.0), 4.0)
    o, st = hand_state(n, gas, phi_ifc=1.001)  # every interface cell fills in the first step
    s = fsl.Sim(st["w"], list_capacity=1)
    for fo, fg in ((O.FLAGS, fsl.FIELD_FLAGS), (O.F, fsl.FIELD_F), (O.MASS, fsl.FIELD_MASS),
                   (O.PHI, fsl.FIELD_PHI), (O.BUBBLE_ID, fsl.FIELD_BUBBLE_ID), (O.PID, fsl.FIELD_PID)):
        s.set(fg, o.get(fo))
    s.bubbles_set([0.0, st["M"]], [0, 1], [0, 1])
    s.step(1)
    with pytest.raises(fsl.FslError, match="overflowed"):
        s.sync()
    o.close()
    s.close()


def _one_sphere(x, periodic=(1, 1, 1), n=(24, 24, 24), u=(0.0, 0.0, 0.0), g=(0.0, 0.0, 0.0)):
    p = W.Particles(x=np.array([x], dtype=np.float64), u=np.array([u], dtype=np.float64),
                    omega=np.zeros((1, 3)), R=np.array([3.0]), rho_p=np.array([1.5]))
    return W.Workload(name="one", n=n, trt=True, tau=0.6, g=g, zs=-1.0, steps=0, periodic=periodic,
                      particles=p)


def test_unsupported_sphere_positions_are_refused():
    """The particle setter refuses centres that are not finite or lie outside a walled
    box, and periodic axes not longer than 2R + 4; the faces of a walled box are
    allowed, and on periodic axes any centre, taken into [0, n), as by the oracle."""
    s = fsl.Sim(_one_sphere((12.0, 12.0, 12.0), periodic=(0, 0, 0)))
    for x in [(12.0, 12.0, 24.2), (-0.7, 12.0, 12.0), (12.0, np.inf, 12.0)]:
        with pytest.raises(fsl.FslError, match="particles_set"):
            s.particles_set(_one_sphere(x, periodic=(0, 0, 0)).particles)
    s.particles_set(_one_sphere((-0.5, 12.0, 23.5), periodic=(0, 0, 0)).particles)
    s.close()
    s = fsl.Sim(_one_sphere((12.0, 12.0, 12.0)))
    with pytest.raises(fsl.FslError, match="particles_set"):
        s.particles_set(_one_sphere((np.nan, 12.0, 12.0)).particles)
    big = _one_sphere((12.0, 12.0, 12.0)).particles
    big.R[:] = 10.0  # 2R + 4 = 24: the axis must be longer
    with pytest.raises(fsl.FslError, match="particles_set"):
        s.particles_set(big)
    s.particles_set(_one_sphere((-3.0, 27.5, 12.0)).particles)
    np.testing.assert_allclose(s.particles_get(1)["x"][0], [21.0, 3.5, 12.0], rtol=0, atol=1e-12)
    s.close()


def test_window_refuses_moving_faces():
    """The adjoint transposes resting bounce-back at the box faces only, so a window
    on a box whose faces move is refused (the oracle's window would include the
    moving-wall term and the two would disagree)."""
    w = W.Workload(name="walled", n=(20, 14, 12), trt=True, tau=0.6, g=(0.0, 0.0, -1e-5), zs=-1.0, steps=0,
                   periodic=(1, 0, 0), integrate=False)
    wall = [[[0.0] * 3, [0.0] * 3] for _ in range(3)]
    wall[1][1][0] = 0.01  # the face y = n - 1/2 moves along x
    s = fsl.Sim(w, window=(4, 2), wall_u=wall)
    with pytest.raises(fsl.FslError, match="moving box faces"):
        s.window_forward(4, 2)
    s.close()
    s = fsl.Sim(w, window=(4, 2))
    s.window_forward(4, 2)
    s.close()
