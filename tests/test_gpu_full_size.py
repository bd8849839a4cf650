"""The hot path at the benchmark's full size: the 512 x 512 x 1024 bubble column with
10^5 spheres (R = 5), in the launch configuration the benchmark times.

The oracle cannot hold this box, so properties that hold at any size are checked:
the ledger mass is conserved (FP64 sums over 2 x 10^8 liquid cells), every bubble's
volume equals its gas cells plus the empty part of its interface cells (the bubble
model's definition, recounted on the host from the cell fields), and the run reports
no error (a liquid cell next to gas, a NaN, a list overflow).
"""
import numpy as np
import pytest

import paper_1712_07028_amd as fsl
from paper_1712_07028_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    fsl.load_library()


def test_column_full_size_properties():
    w = W.bubble_column_large()
    print(f"full-size column {w.n}, {w.particles.n} spheres", flush=True)
    s = fsl.Sim(w)
    M0 = s.mass()[0]
    s.step(30)
    s.sync()
    M1 = s.mass()[0]
    print("ledger mass drift", (M1 - M0) / M0, flush=True)
    assert abs(M1 - M0) / M0 < 1e-10
    flags = s.get(fsl.FIELD_FLAGS)
    bid = s.get(fsl.FIELD_BUBBLE_ID)
    phi = s.get(fsl.FIELD_PHI)
    bubbles = s.bubbles()
    s.close()
    gas, ifc = flags == fsl.GAS, flags == fsl.IFC
    assert ((flags == fsl.LIQ) | ifc).sum() > 2 * 10**8
    gid = bid[gas]
    iid, iphi = bid[ifc], phi[ifc]
    alive = [b for b in bubbles if b["alive"]]
    assert len(alive) >= 2  # the gas above the pool and the rising bubble
    for b in alive:
        V = float((gid == b["id"]).sum()) + float((1.0 - iphi[iid == b["id"]]).sum())
        print("bubble", b["id"], "V", b["V"], "recount", V, flush=True)
        assert abs(V - b["V"]) <= 1e-9 * V
    # every gas and interface cell belongs to a live bubble
    live = np.array([b["id"] for b in alive])
    assert np.isin(gid, live).all() and np.isin(iid, live).all()


def test_column_full_size_sampled_cells():
    """Sampled outputs at full size: 64 random liquid cells whose 3 x 3 x 3 block is
    liquid take the plain pull and collision; the oracle steps each block as a periodic
    3^3 window from the library's populations, and its centre must agree."""
    import oracle as O

    O.build(force=False)
    w = W.bubble_column_large()
    s = fsl.Sim(w)
    s.step(3)
    s.sync()
    flags = s.get(fsl.FIELD_FLAGS)
    nz, ny, nx = flags.shape
    rng = np.random.Generator(np.random.PCG64(5))
    picks = []
    for _ in range(100000):
        if len(picks) == 64:
            break
        z, y, x = (int(rng.integers(1, n - 1)) for n in (nz, ny, nx))
        if (flags[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2] == fsl.LIQ).all():
            picks.append((z, y, x))
    assert len(picks) == 64
    del flags
    F = s.get(fsl.FIELD_F)  # 19 x 2.7e8 FP64 values on the host (41 GB)
    wins = [F[:, z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].copy() for z, y, x in picks]
    del F
    s.step(1)
    s.sync()
    F = s.get(fsl.FIELD_F)
    got = [F[:, z, y, x].copy() for z, y, x in picks]
    del F
    s.close()
    ws = w.replace(name="window3", n=(3, 3, 3), zs=-1.0, periodic=(1, 1, 1), gas_spheres=[], particles=None)
    worst = 0.0
    for win, g in zip(wins, got):
        o = O.Oracle(ws)
        o.set(O.F, win)
        o.step(1)
        ref = o.get(O.F)[:, 1, 1, 1]
        o.close()
        worst = max(worst, float((np.abs(g - ref) / np.abs(ref)).max()))
    print("sampled cells: worst relative population error", worst, flush=True)
    assert worst < 1e-6
