"""Bubble splitting on the GPU (bubble model, end of Sec. 2.2) against the oracle.

The library tests every gas cell that leaves the gas phase on its 3x3x3 block and
labels all gas cells only when a test fails; the oracle labels every step.  Hand-made
states (the oracle pins' constructions) are given to both sides before their bubble
tables are set, so each side splits on its own.  Checked: bubble ids of every cell
bit-exact, the bubble table (ids in use, alive flags, gas masses, volumes, densities)
to 1e-12 relative when a given state is split, and after steps to the plain parity
bars (1e-6 relative, fill levels differing by rounding) with the populations as in
the plain parity tests.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1712_07028_amd as fsl
from paper_1712_07028_amd import workloads as W

from gpu_common import compare_step
from test_oracle_split import ball, hand_state, interface_of

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


def twin(n, gas, particles=None, **kw):
    """The same hand state on both sides, bubble tables set (each side splits)."""
    o, st = hand_state(n, gas, particles=particles, **kw)
    w = st["w"]
    s = fsl.Sim(w, max_bubbles=kw.get("max_bubbles", 0))
    for fo, fg in ((O.FLAGS, fsl.FIELD_FLAGS), (O.F, fsl.FIELD_F), (O.MASS, fsl.FIELD_MASS),
                   (O.PHI, fsl.FIELD_PHI), (O.BUBBLE_ID, fsl.FIELD_BUBBLE_ID), (O.PID, fsl.FIELD_PID)):
        s.set(fg, o.get(fo))
    o.bubbles_set([0.0, st["M"]], [0, 1], [0, 1])
    s.bubbles_set([0.0, st["M"]], [0, 1], [0, 1])
    if particles is not None:
        o.particles_set(particles)
        s.particles_set(particles)
    return o, s, st


def compare_bubbles(o, s, rtol=1e-12):
    np.testing.assert_array_equal(s.get(fsl.FIELD_BUBBLE_ID), o.get(O.BUBBLE_ID))
    bo, bg = o.bubbles(), s.bubbles()
    assert len(bg) == len(bo), (len(bg), len(bo))
    for a, b in zip(bo, bg):
        assert a["alive"] == b["alive"], (a, b)
        if not a["alive"]:
            continue
        for k in ("M", "V", "rho_g"):
            assert abs(b[k] - a[k]) <= rtol * max(abs(a[k]), 1.0), (k, a, b)
    return len(bo)


def test_two_blobs_split_on_setting_the_table():
    n = (20, 14, 24)
    gas = ball(n, (9.3, 7.0, 6.0), 2.6) | ball(n, (10.0, 6.5, 16.0), 3.4)
    o, s, _ = twin(n, gas, rho_g=1.013)
    assert compare_bubbles(o, s) == 3
    o.close()
    s.close()


@pytest.mark.parametrize("contact,parts", [((1, 1, 0), 1), ((1, 1, 1), 2)])
def test_edges_connect_corners_do_not(contact, parts):
    n = (16, 16, 16)
    gas = np.zeros((16, 16, 16), bool)
    gas[4:7, 4:7, 4:7] = True
    lo = 7 - (1 - np.array(contact))
    gas[lo[2]:lo[2] + 3, lo[1]:lo[1] + 3, lo[0]:lo[0] + 3] = True
    o, s, _ = twin(n, gas)
    assert compare_bubbles(o, s) == parts + 1
    o.close()
    s.close()


def test_three_parts_and_shared_interface():
    n = (18, 12, 12)
    gas = np.zeros((12, 12, 18), bool)
    gas[4:8, 4:8, 12:16] = True
    gas[4:8, 4:8, 2:6] = True
    gas[4:8, 4:8, 7:11] = True
    o, s, _ = twin(n, gas, rho_g=0.97)
    assert compare_bubbles(o, s) == 4
    o.close()
    s.close()


def test_full_table_is_an_error():
    n = (16, 12, 12)
    gas = ball(n, (4.0, 6.0, 6.0), 2.2) | ball(n, (11.0, 6.0, 6.0), 2.2)
    o, st = hand_state(n, gas, max_bubbles=2)
    s = fsl.Sim(st["w"], max_bubbles=2)
    for fo, fg in ((O.FLAGS, fsl.FIELD_FLAGS), (O.PHI, fsl.FIELD_PHI), (O.BUBBLE_ID, fsl.FIELD_BUBBLE_ID)):
        s.set(fg, o.get(fo))
    with pytest.raises(fsl.FslError):
        s.bubbles_set([0.0, st["M"]], [0, 1], [0, 1])
    o.close()
    s.close()


def stepped(o, s, w, steps, label):
    split_at = None
    for t in range(steps):
        o.step(1)
        s.step(1)
        s.sync()
        # positions integrate forces that agree to 1e-7: the bar of the multi-step cases
        compare_step(o, s, w, x_tol=1e-7)
        if compare_bubbles(o, s, rtol=1e-6) > 2 and split_at is None:
            split_at = t
            say(f"  {label}: split in step {t}")
    return split_at


def test_neck_closed_by_conversions():
    n = (26, 16, 18)
    gas = ball(n, (6.0, 8.0, 9.0), 3.0) | ball(n, (19.0, 8.0, 9.0), 3.0)
    gas[9, 8, 8:19] = True
    z, y, x = np.nonzero(interface_of(gas))
    full = (x >= 11) & (x <= 14) & (abs(y - 8) <= 1) & (abs(z - 9) <= 1)
    o, s, st = twin(n, gas, phi_ifc=np.where(full, 1.001, 0.5))
    assert stepped(o, s, st["w"], 12, "conversions") is not None
    o.close()
    s.close()


def test_neck_cut_by_a_sphere():
    n = (26, 16, 20)
    gas = ball(n, (5.0, 8.0, 9.0), 3.0) | ball(n, (20.0, 8.0, 9.0), 3.0)
    gas[8:11, 7:10, 7:19] = True
    p = W.Particles(x=np.array([[13.0, 8.0, 5.0]]), u=np.array([[0.0, 0.0, 0.12]]),
                    omega=np.zeros((1, 3)), R=np.array([2.5]), rho_p=np.array([20.0]))
    o, s, st = twin(n, gas, phi_ifc=0.5, particles=p)
    assert stepped(o, s, st["w"], 30, "coverage") is not None
    o.close()
    s.close()


def copy_fields(o, s):
    for fo, fg in ((O.FLAGS, fsl.FIELD_FLAGS), (O.F, fsl.FIELD_F), (O.MASS, fsl.FIELD_MASS),
                   (O.PHI, fsl.FIELD_PHI), (O.BUBBLE_ID, fsl.FIELD_BUBBLE_ID), (O.PID, fsl.FIELD_PID)):
        s.set(fg, o.get(fo))


def test_split_takes_the_lowest_id_not_alive():
    n = (20, 14, 24)
    gas = ball(n, (9.3, 7.0, 6.0), 2.6) | ball(n, (10.0, 6.5, 16.0), 3.4)
    o, st = hand_state(n, gas, rho_g=1.02)
    s = fsl.Sim(st["w"])
    copy_fields(o, s)
    for x in (o, s):
        x.bubbles_set([0.0, st["M"], 0.0, 0.0], [0, 1, 2, 3], [0, 1, 0, 0])
    assert compare_bubbles(o, s) == 4
    o.close()
    s.close()


def test_merge_relabels_cells_to_the_root():
    n = (18, 12, 12)
    gas = np.zeros((12, 12, 18), bool)
    gas[4:8, 4:8, 2:6] = True
    gas[4:8, 4:8, 7:11] = True
    z, y, x = np.nonzero(interface_of(gas))
    o, st = hand_state(n, gas, phi_ifc=np.where(x == 6, 0.0, 0.5))
    ids = o.get(O.BUBBLE_ID)
    X = np.arange(18)[None, None, :]
    ids[(st["gas"] | st["ifc"]) & (X >= 7)] = 2
    o.set(O.BUBBLE_ID, ids)
    m1 = (st["gas"] & (X < 7)).sum() + (1.0 - st["phi"])[st["ifc"] & (X < 7)].sum()
    s = fsl.Sim(st["w"])
    copy_fields(o, s)
    for x in (o, s):
        x.bubbles_set([0.0, m1, st["V"] - m1], [0, 1, 2], [0, 1, 1])
    o.step(1)
    s.step(1)
    s.sync()
    compare_step(o, s, st["w"])
    assert compare_bubbles(o, s, rtol=1e-6) == 3
    assert set(np.unique(s.get(fsl.FIELD_BUBBLE_ID)[(s.get(fsl.FIELD_FLAGS) == fsl.GAS)])) == {1}
    o.close()
    s.close()
