"""fsl_init_static against fsl_init on the GPU: contexts whose working memory is the
library's device array step like contexts on a full workspace.

Two such contexts are alive at once, a particle bed with a bubble (40^3, coverage
events, particle pairs, conversions) and a smaller bubble column (32^3, splitting
pass, field staging): their calls alternate on the stream, so each call finds the
array as the other context's last call left it.  Cell types, bubble ids and
particle owners must agree exactly with the full-workspace runs, populations,
particle states and masses to the rounding of the FP64 atomic sums (the same bar
as two full-workspace runs of these cases).
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


def bed():
    bub = (20.0, 20.0, 10.0, 6.0, 1.0)
    p = W.particle_bed(12, 3.5, (40, 40, 40), 32.0, bub, seed=7, rho_p=2.5, vel_range=0.01)
    return W.Workload(name="bed40", n=(40, 40, 40), trt=True, tau=0.55, g=(0, 0, -2e-5), zs=32.0, steps=0,
                      gas_spheres=[bub], particles=p)


def compare(a, b, tol):
    for k in (fsl.FIELD_FLAGS, fsl.FIELD_BUBBLE_ID, fsl.FIELD_PID):
        np.testing.assert_array_equal(a.get(k), b.get(k))
    fl = a.get(fsl.FIELD_FLAGS)
    act = (fl == fsl.LIQ) | (fl == fsl.IFC)
    fa, fb = a.get(fsl.FIELD_F)[:, act], b.get(fsl.FIELD_F)[:, act]
    assert np.abs(fa - fb).max() <= tol * np.abs(fa).max()
    ma, mb = a.mass(), b.mass()
    assert abs(ma[0] - mb[0]) <= 1e-12 * abs(ma[0])
    if a.n_particles:
        pa, pb = a.particles_get(), b.particles_get()
        for k in ("x", "u"):
            assert np.abs(pa[k] - pb[k]).max() <= tol * max(1.0, np.abs(pa[k]).max()), k


def test_static_contexts_match_full_workspace():
    wa, wb = bed(), W.bubble_column_small()
    assert wb.cells < wa.cells  # the second context is the smaller input
    import torch

    ref_a, ref_b = fsl.Sim(wa), fsl.Sim(wb)
    shared = torch.cuda.Stream()  # calls on contexts that share the array must not overlap
    st_a = fsl.Sim(wa, static=True, stream=shared)
    st_b = fsl.Sim(wb, static=True, stream=shared)
    assert st_a.workspace.numel() < ref_a.workspace.numel()
    for _ in range(3):
        for ref, st in ((ref_a, st_a), (ref_b, st_b)):
            ref.step(10)
            st.step(10)
        st_a.sync()
        st_b.sync()
    compare(ref_a, st_a, 1e-9)
    compare(ref_b, st_b, 1e-12)
    # a bubble table import (splitting pass on the current fields) on the smaller one,
    # right after steps of the larger one
    b0 = ref_b.bubbles()
    args = ([x["M"] for x in b0], list(range(len(b0))), [x["alive"] for x in b0])
    st_a.step(5)
    ref_a.step(5)
    ref_b.bubbles_set(*args)
    st_b.bubbles_set(*args)
    for ref, st in ((ref_b, st_b), (ref_a, st_a)):
        ref.step(10)
        st.step(10)
    compare(ref_a, st_a, 1e-9)
    compare(ref_b, st_b, 1e-12)
    for s in (ref_a, ref_b, st_a, st_b):
        s.close()
