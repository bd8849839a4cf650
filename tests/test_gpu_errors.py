"""Failure detection on the GPU: conditions forced from the host through imported
states or a configuration, reported by the next synchronising call with their own
error codes.  Every kernel still runs to its end: the errors are latched on the
device, never trapped.
  - a NaN population in a liquid cell: FSL_E_NUMERIC;
  - a liquid cell next to a gas cell (the interface layer broken): FSL_E_INVARIANT;
  - conversion lists of capacity 1 with many cells filling at once: FSL_E_CAPACITY.
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
