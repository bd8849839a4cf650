"""The storage forms: populations kept shifted (h = f - w) in binary16 (scaled by
2^10) or bfloat16, FP32 collision arithmetic, FP64 mass, volume and force sums.

Single steps from identical states: cell types bit-exact; every population within
k * u * max|h| of the FP64 oracle, u the unit roundoff of the storage format (2^-11
binary16, 2^-9 bfloat16) and k = 4: the stored inputs carry one rounding each,
the collision mixes them with weights summing to about one, and the output is
rounded once more.

1,000 steps of the 128^3 pool with one bubble (R = 12) and 1,400 spheres against
the oracle's stored results (tests/golden/precision_bed128.json): the total-mass
ledger of each run against its own initial value, and the bubble rise velocity and
mean particle drag against the oracle, to the bounds stated per form below.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle as O
import paper_1712_07028_amd as fsl
from paper_1712_07028_amd import workloads as W

from gpu_common import transfer

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
UNIT = {W.STORAGE_F16S: 2.0 ** -11, W.STORAGE_BF16S: 2.0 ** -9}
# bounds after 1,000 steps of the 128^3 bed: |M(T)/M(0) - 1|, rise velocity and mean
# drag relative to the oracle
BOUNDS = {
    W.STORAGE_F32: (1e-10, 0.01, 0.01),
    W.STORAGE_F16S: (1e-6, 0.01, 0.01),
    W.STORAGE_BF16S: (1e-5, 0.05, 0.05),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    fsl.load_library()


def bed(n=40, nsph=12, seed=7, storage=0):
    bub = (n / 2, n / 2, 10.0, 6.0, 1.0)
    p = W.particle_bed(nsph, 3.5, (n, n, n), 32.0, bub, seed=seed, rho_p=2.5, vel_range=0.01)
    return W.Workload(name=f"bed{n}", n=(n, n, n), trt=True, tau=0.55, g=(0, 0, -2e-5), zs=32.0,
                      steps=0, gas_spheres=[bub], particles=p, storage=storage)


@pytest.mark.parametrize("storage", [W.STORAGE_F16S, W.STORAGE_BF16S])
def test_single_step_storage_forms(storage):
    w = bed(storage=storage)
    say("single step, storage", storage)
    o = O.Oracle(w)
    o.step(20)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    fo = o.get(O.FLAGS)
    np.testing.assert_array_equal(fo, s.get(fsl.FIELD_FLAGS))
    act = (fo == O.LIQ) | (fo == O.IFC)
    wq = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    Fo, Fg = o.get(O.F), s.get(fsl.FIELD_F)
    hmax = np.abs(Fo - wq[:, None, None, None])[:, act].max()
    err = np.abs(Fg - Fo)[:, act].max()
    say(f"  max |f - f_oracle| = {err:.3e}, max|h| = {hmax:.3e}, ratio {err / hmax:.3e}")
    assert err <= 4 * UNIT[storage] * hmax
    # interface mass and fill level are FP64 in every form
    ifc = fo == O.IFC
    assert np.abs(o.get(O.MASS)[ifc] - s.get(fsl.FIELD_MASS)[ifc]).max() < 1e-4
    o.close()
    s.close()


def test_precision_bed128_vs_oracle():
    ref = json.load(open(os.path.join(HERE, "golden", "precision_bed128.json")))
    T = ref["steps"]
    for st in (W.STORAGE_F32, W.STORAGE_F16S, W.STORAGE_BF16S):
        w = W.bubble_bed_128(storage=st)
        n = w.particles.n
        say("128^3 bed, 1,400 spheres, storage", st)
        s = fsl.Sim(w)
        M0 = s.mass()[0]
        s.step(T - 10)
        b0 = s.bubbles()
        drag = []
        for _ in range(10):
            s.step(1)
            drag.append(s.particles_get(n)["F"][:, 2].mean())
        b1 = s.bubbles()
        M1 = s.mass()[0]
        s.close()
        rise = (b1[1]["centroid"][2] - b0[1]["centroid"][2]) / 10.0
        dm = abs(M1 / M0 - 1.0)
        er = abs(rise / ref["rise_velocity"] - 1.0)
        ed = abs(np.mean(drag) / ref["mean_drag_z"] - 1.0)
        say(f"  mass drift {dm:.3e} (vs oracle {abs(M1 / ref['mass'] - 1):.3e}), rise {rise:.6e} "
            f"(err {er:.3e}), drag {np.mean(drag):.6e} (err {ed:.3e})")
        bm, br, bd = BOUNDS[st]
        # the initial state is the oracle's up to the rounding of the stored rest
        # population (the moving ones are balanced by it exactly): per cell at most
        # u * |h_0| <= u * |g| z_s (hydrostatic pool, h_0 = (rho - 1)/3)
        bound0 = 1e-12 if st == W.STORAGE_F32 else UNIT[st] * abs(w.g[2]) * w.zs
        assert abs(M0 / ref["mass0"] - 1.0) < bound0
        assert dm < bm and er < br and ed < bd, (st, dm, er, ed)
