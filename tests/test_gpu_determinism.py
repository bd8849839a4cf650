"""Repeatability on the GPU (race detection): two simulations from the same state.

Without gas and particles every cell's update is a function of its inputs only, so
the populations after 60 steps must agree to the last bit.  With a free surface and
spheres the only order-dependent sums are FP64 atomics (bubble volumes, excess mass,
forces); cell types, bubble ids and particle owners must still agree exactly and the
populations to rounding.
"""
import numpy as np
import pytest

import oracle as O
import paper_1712_07028_amd as fsl
from paper_1712_07028_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    fsl.load_library()


def run(w, steps, F=None):
    s = fsl.Sim(w)
    if F is not None:
        s.set(fsl.FIELD_F, F)
    s.step(steps)
    s.sync()
    out = {k: s.get(k) for k in (fsl.FIELD_FLAGS, fsl.FIELD_F, fsl.FIELD_BUBBLE_ID, fsl.FIELD_PID)}
    s.close()
    return out


def test_liquid_channel_is_bit_identical():
    w = W.Workload(name="chan", n=(70, 13, 11), trt=True, tau=0.6, g=(2e-5, 0, 0), zs=-1.0, steps=0,
                   periodic=(1, 0, 0))
    s = fsl.Sim(w)
    rng = np.random.Generator(np.random.PCG64(4))
    F = s.get(fsl.FIELD_F) * (1.0 + 0.01 * rng.standard_normal((19, 11, 13, 70)))
    s.close()
    a, b = run(w, 60, F), run(w, 60, F)
    np.testing.assert_array_equal(a[fsl.FIELD_F], b[fsl.FIELD_F])


@pytest.mark.parametrize("case", ["column", "bed"])
def test_free_surface_and_spheres_repeat(case):
    if case == "column":
        w, steps, tol = W.bubble_column_small(), 150, 1e-12
    else:
        bub = (20.0, 20.0, 10.0, 6.0, 1.0)
        p = W.particle_bed(12, 3.5, (40, 40, 40), 32.0, bub, seed=7, rho_p=2.5, vel_range=0.01)
        w = W.Workload(name="bed40", n=(40, 40, 40), trt=True, tau=0.55, g=(0, 0, -2e-5), zs=32.0, steps=0,
                       gas_spheres=[bub], particles=p)
        steps, tol = 60, 1e-9
    a, b = run(w, steps), run(w, steps)
    for k in (fsl.FIELD_FLAGS, fsl.FIELD_BUBBLE_ID, fsl.FIELD_PID):
        np.testing.assert_array_equal(a[k], b[k])
    act = (a[fsl.FIELD_FLAGS] == fsl.LIQ) | (a[fsl.FIELD_FLAGS] == fsl.IFC)
    fa, fb = a[fsl.FIELD_F][:, act], b[fsl.FIELD_F][:, act]
    assert np.abs(fa - fb).max() <= tol * np.abs(fa).max()


def test_checkpoint_resume():
    """A state dumped through the field, bubble and particle calls and restored into a
    fresh simulation continues like the original (bubble column without spheres: the
    particle update restarts its two-step force mean when a table is set)."""
    w = W.bubble_column_small()
    a = fsl.Sim(w)
    a.step(40)
    fields = {k: a.get(k) for k in (fsl.FIELD_FLAGS, fsl.FIELD_F, fsl.FIELD_MASS, fsl.FIELD_PHI,
                                    fsl.FIELD_BUBBLE_ID, fsl.FIELD_PID)}
    b0 = a.bubbles()
    M0, L0 = a.mass()  # the ledger is not part of the fields
    b = fsl.Sim(w)
    for k, v in fields.items():
        b.set(k, v)
    b.bubbles_set([x["M"] for x in b0], list(range(len(b0))), [x["alive"] for x in b0])
    assert abs(b.mass()[0] / (M0 - L0) - 1.0) < 1e-15
    a.step(40)
    b.step(40)
    fa, fb = a.get(fsl.FIELD_FLAGS), b.get(fsl.FIELD_FLAGS)
    np.testing.assert_array_equal(fa, fb)
    act = (fa == fsl.LIQ) | (fa == fsl.IFC)
    Fa, Fb = a.get(fsl.FIELD_F)[:, act], b.get(fsl.FIELD_F)[:, act]
    assert np.abs(Fa - Fb).max() <= 1e-12 * np.abs(Fa).max()
    a.close()
    b.close()
