"""Exactness of two shortcuts the library's kernels take and the oracle does not,
checked on the host builds of the same functions (libfsl_checks.so) against exact
definitions on seeded random inputs.

- Bubble splitting (bubble model, end of Sec. 2.2): a cell that leaves the gas is
  tested on its 3x3x3 block, and only a failed test asks for a labelling of all gas
  cells.  On 20,000 random connected gas sets with random sets of removed cells
  (scattered, and runs of neighbours), whenever every removed cell passes, the
  remaining gas must be one D3Q19-connected part by scipy.ndimage.label.
- Coverage (Sec. 2.3): for a sphere alone, only the nodes of each (x, y) column in
  the candidate ranges take the inside test.  On random sphere moves (small, large,
  none, centres on nodes, integer radii with nodes exactly on the surface, spheres
  cut by the box), every node whose inside test changes must lie in a range.
"""
import ctypes
import os

import numpy as np
import pytest
from scipy import ndimage

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1712_07028_amd", "libfsl_checks.so")

# D3Q19 neighbourhood: the 3x3x3 block without its 8 corners
D3Q19 = np.ones((3, 3, 3), bool)
for c in [(0, 0, 0), (0, 0, 2), (0, 2, 0), (0, 2, 2), (2, 0, 0), (2, 0, 2), (2, 2, 0), (2, 2, 2)]:
    D3Q19[c] = False
# bit (dx+1) + 3(dy+1) + 9(dz+1) of a block indexed [dz+1, dy+1, dx+1]
BIT = (1 << np.arange(27, dtype=np.int64)).reshape(3, 3, 3)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libfsl_checks.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    L.fsl_check_split_block.restype = ctypes.c_int
    L.fsl_check_split_block.argtypes = [ctypes.c_uint, ctypes.c_uint]
    L.fsl_check_cov_column.restype = None
    L.fsl_check_cov_column.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int, ctypes.c_int,
                                                               ctypes.POINTER(ctypes.c_int)]
    return L


def block_bits(a, z, y, x):
    """27-bit set of a boolean field's 3x3x3 block around (z, y, x); cells outside the
    box count as absent (non-periodic box)."""
    p = np.pad(a, 1)
    return int((p[z:z + 3, y:y + 3, x:x + 3] * BIT).sum())


def test_split_block_test_never_misses_a_split(lib):
    rng = np.random.Generator(np.random.PCG64(2024))
    n = 7
    passed = labelled = 0
    for trial in range(20000):
        lab, k = ndimage.label(rng.random((n, n, n)) < rng.uniform(0.3, 0.75), structure=D3Q19)
        if k == 0:
            continue
        big = np.bincount(lab.ravel())[1:].argmax() + 1
        gas = lab == big  # one connected bubble before the step
        cells = np.argwhere(gas)
        m = int(rng.integers(1, 7))
        removed = np.zeros_like(gas)
        if trial % 2 == 0:  # scattered cells
            for i in rng.choice(len(cells), size=min(m, len(cells)), replace=False):
                removed[tuple(cells[i])] = True
        else:  # a run of neighbouring cells
            c = cells[rng.integers(len(cells))]
            removed[tuple(c)] = True
            for _ in range(m - 1):
                nb = [c + d for d in np.argwhere(D3Q19) - 1
                      if ((c + d >= 0) & (c + d < n)).all() and gas[tuple(c + d)] and not removed[tuple(c + d)]]
                if not nb:
                    break
                c = nb[rng.integers(len(nb))]
                removed[tuple(c)] = True
        left = gas & ~removed
        ok = True
        for z, y, x in np.argwhere(removed):
            g = block_bits(left, z, y, x)
            r = block_bits(removed, z, y, x) & ~(1 << 13)
            if not lib.fsl_check_split_block(g, r):
                ok = False
                break
        if ok:
            passed += 1
            parts = ndimage.label(left, structure=D3Q19)[1]
            assert parts <= 1, (trial, np.argwhere(removed).tolist())
        else:
            labelled += 1
    # both outcomes occur often: the check is not vacuous
    assert passed > 3000 and labelled > 3000, (passed, labelled)


def test_split_block_special_cases(lib):
    # no gas neighbour left: nothing to disconnect
    assert lib.fsl_check_split_block(0, 0) == 1
    # two gas faces on opposite sides, joined only through the centre: must label
    left, right = BIT[1, 1, 0], BIT[1, 1, 2]
    assert lib.fsl_check_split_block(int(left | right), 0) == 0
    # the same two joined around the centre through edge cells of the block
    ring = left | right | BIT[1, 0, 0] | BIT[1, 0, 1] | BIT[1, 0, 2]
    assert lib.fsl_check_split_block(int(ring), 0) == 1
    # a removed neighbour that touches no remaining block gas: must label
    assert lib.fsl_check_split_block(int(left), int(BIT[1, 2, 2])) == 0


def moves(rng, count, n):
    """Seeded sphere moves (new centre, old centre, radius) of every kind the coverage
    update meets, some of them cut by the box."""
    out = []
    for i in range(count):
        kind = i % 6
        R = float(rng.integers(2, 9)) if kind in (2, 3) else rng.uniform(1.2, 12.0)
        xo = rng.uniform(-R / 2, n - 1 + R / 2, size=3) if kind == 5 else rng.uniform(R + 1, n - R - 2, size=3)
        if kind == 2:
            xo = np.round(xo)  # centre on a node: integer radii put nodes on the surface
        d = {0: rng.uniform(-0.49, 0.49, 3), 1: rng.uniform(-1e-9, 1e-9, 3), 2: rng.uniform(-0.49, 0.49, 3) * (rng.random(3) < 0.5),
             3: np.zeros(3), 4: rng.uniform(-3.0, 3.0, 3), 5: rng.uniform(-0.49, 0.49, 3)}[kind]
        out.append((xo + d, xo, R))
    return out


def test_coverage_column_ranges_hold_every_changed_node(lib):
    rng = np.random.Generator(np.random.PCG64(77))
    n = 40
    r = (ctypes.c_int * 4)()
    changed_total = 0
    for xn, xo, R in moves(rng, 3000, n):
        R2 = R * R
        lo = np.maximum(np.floor(np.minimum(xn, xo) - R), 0).astype(int)
        hi = np.minimum(np.ceil(np.maximum(xn, xo) + R), n - 1).astype(int)
        if (lo > hi).any():
            continue
        i = np.arange(lo[0], hi[0] + 1, dtype=np.float64)[None, :]
        j = np.arange(lo[1], hi[1] + 1, dtype=np.float64)[:, None]
        k = np.arange(n, dtype=np.float64)
        a0, a1, b0, b1 = i - xn[0], j - xn[1], i - xo[0], j - xo[1]
        sn, so = a0 * a0 + a1 * a1, b0 * b0 + b1 * b1  # (ny', nx') in the inside test's order
        a2, b2 = k - xn[2], k - xo[2]
        inn = sn[..., None] + a2 * a2 <= R2
        ino = so[..., None] + b2 * b2 <= R2
        chg = inn != ino
        changed_total += int(chg.sum())
        for jj, ii in np.argwhere(chg.any(axis=2) | (sn <= R2) | (so <= R2)):
            ks = np.flatnonzero(chg[jj, ii])
            if sn[jj, ii] > R2 and so[jj, ii] > R2:
                assert ks.size == 0
                continue
            lib.fsl_check_cov_column(sn[jj, ii], so[jj, ii], R2, xn[2], xo[2], int(lo[2]), int(hi[2]), r)
            inr = ((ks >= r[0]) & (ks <= r[1])) | ((ks >= r[2]) & (ks <= r[3]))
            assert inr.all(), (xn.tolist(), xo.tolist(), R, int(ii + lo[0]), int(jj + lo[1]), ks.tolist(), list(r))
    assert changed_total > 100000, changed_total
