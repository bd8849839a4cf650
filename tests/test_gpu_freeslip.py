"""Free-slip faces and the pressure outlet on the GPU (set-up of the bubble regimes,
Sec. 3.2) against the FP64 oracle.

Single steps from identical states, with the plain parity bars: a pool with a bubble
cut by a free-slip face and spheres near the walls (free slip on x and y), and a
channel periodic in x with free-slip y faces over a moving no-slip floor (edges where
a free-slip and a moving no-slip face meet).  Then 150 steps with an open atmosphere:
the gas above the pool at exactly rho_g0 on both sides, the ledger mass within 1e-10
and the bubble volumes within 1e-6.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1712_07028_amd as fsl
from paper_1712_07028_amd import workloads as W

from gpu_common import compare_step, transfer

pytestmark = pytest.mark.gpu


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


def pool_with_walls(open_atmosphere=False):
    n = (22, 17, 20)
    bub = (1.5, 8.0, 6.0, 4.0, 1.0)  # cut by the x = -1/2 face
    p = W.particle_bed(6, 2.5, n, 14.0, bub, seed=31, rho_p=2.5, vel_range=0.01)
    return W.Workload(name="slip_pool", n=n, trt=True, tau=0.58, g=(0, 0, -3e-5), zs=14.3, steps=0,
                      gas_spheres=[bub], particles=p, freeslip=(1, 1, 0), open_atmosphere=open_atmosphere)


def slip_channel():
    n = (30, 11, 14)
    return W.Workload(name="slip_channel", n=n, trt=True, tau=0.7, g=(1e-5, 0, -1e-5), zs=10.6, steps=0,
                      periodic=(1, 0, 0), freeslip=(0, 1, 0), gas_spheres=[(15.0, 0.5, 4.0, 3.0, 1.0)])


@pytest.mark.parametrize("warm", [0, 15])
def test_single_step_free_slip_pool(warm):
    w = pool_with_walls()
    say("free-slip pool, warm", warm)
    o = O.Oracle(w)
    o.step(warm)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say("  ", compare_step(o, s, w))
    o.close()
    s.close()


def test_single_step_slip_over_moving_floor():
    w = slip_channel()
    wall = [[[0, 0, 0], [0, 0, 0]], [[0.3, 0.2, 0.1], [0.3, 0.2, 0.1]], [[0.01, 0.002, 0], [0, 0, 0]]]
    say("free-slip channel over a moving floor")
    o = O.Oracle(w, wall_u=wall)
    o.step(12)
    s = fsl.Sim(w, wall_u=wall)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say("  ", compare_step(o, s, w))
    o.close()
    s.close()


def test_open_atmosphere_multistep():
    w = pool_with_walls(open_atmosphere=True)
    o = O.Oracle(w, n_threads=8)
    s = fsl.Sim(w)
    M0o, M0g = o.mass()[0], s.mass()[0]
    o.step(150)
    s.step(150)
    bo, bg = o.bubbles(), s.bubbles()
    say(f"  atmosphere rho gpu {bg[0]['rho_g']!r} oracle {bo[0]['rho_g']!r}; V {bg[0]['V']:.6f} {bo[0]['V']:.6f}")
    assert bo[0]["rho_g"] == w.rho_g0 and bg[0]["rho_g"] == w.rho_g0
    assert len(bo) == len(bg)
    for x, y in zip(bo, bg):
        if x["alive"]:
            assert abs(y["V"] / x["V"] - 1.0) < 1e-6, (x, y)
    assert abs(s.mass()[0] / M0g - 1.0) < 1e-10 and abs(o.mass()[0] / M0o - 1.0) < 1e-10
    np.testing.assert_array_equal(s.get(fsl.FIELD_FLAGS), o.get(O.FLAGS))
    o.close()
    s.close()
