"""The seeded inputs of the sheared suspension (Sec. 3.1): the paper's box and sphere
size, N = Phi V / V_P spheres at random non-overlapping positions, periodic along x
and y, and tau from the particle Reynolds number Re_P = gamma (2R)^2 / mu with
gamma = 2U / n_z.  Checked by brute force, with the distances written out here."""
import numpy as np
import pytest

from paper_1712_07028_amd import workloads as W


@pytest.mark.parametrize("phi,count", [(0.1, 111), (0.2, 222), (0.3, 333)])
def test_suspension_count_positions_and_gaps(phi, count):
    w, wall = W.sheared_suspension(phi)
    n, R = w.n, 8.0
    assert n == (114, 116, 180) and w.periodic == (1, 1, 0)
    x = w.particles.x
    assert x.shape == (count, 3) and np.all(w.particles.R == R) and np.all(w.particles.rho_p == 8.0)
    # the volume fraction the count gives is the nearest to phi
    vp = 4.0 / 3.0 * np.pi * R ** 3
    assert abs(count * vp / np.prod(n) - phi) <= 0.5 * vp / np.prod(n)
    # centres: x, y in [0, n), z with the whole sphere and a cell of margin inside the plates
    assert np.all((x[:, :2] >= 0) & (x[:, :2] < np.array(n[:2])))
    assert np.all(x[:, 2] - R >= 0.5 - 1e-12) and np.all(x[:, 2] + R <= n[2] - 1.5 + 1e-12)
    # every surface gap through the nearest periodic image at least 0.2
    gmin = np.inf
    for a in range(count):
        d = x[a + 1:] - x[a]
        for k in range(2):
            d[:, k] = np.where(d[:, k] > n[k] / 2, d[:, k] - n[k], np.where(d[:, k] < -n[k] / 2, d[:, k] + n[k], d[:, k]))
        if d.size:
            gmin = min(gmin, np.sqrt((d * d).sum(axis=1)).min() - 2 * R)
    assert gmin >= 0.2 - 1e-12
    # the plates move along x with -U and +U; Re_P = gamma (2R)^2 / mu = 0.1
    U = wall[2][1][0]
    assert wall[2][0][0] == -U and U == 0.01
    mu = (w.tau - 0.5) / 3.0
    assert abs((2 * U / n[2]) * (2 * R) ** 2 / mu - 0.1) < 1e-12


def test_suspension_is_seeded_and_batch_independent():
    a, _ = W.sheared_suspension(0.2)
    b, _ = W.sheared_suspension(0.2)
    np.testing.assert_array_equal(a.particles.x, b.particles.x)
    # candidates drawn in batches are tested in draw order: the same spheres as one by one
    p = W.periodic_rsa(25, 3.0, (30, 28, 24), seed=4)
    q = W.periodic_rsa(25, 3.0, (30, 28, 24), seed=4, batch=1)
    np.testing.assert_array_equal(p, q)


def test_eilers_closed_form():
    # Eq. Eilers at phi = 0 and at two values by hand
    assert W.eilers(0.0) == 1.0
    assert abs(W.eilers(0.3) - (1 + 1.25 * 0.3 / (1 - 0.3 / 0.63)) ** 2) < 1e-15
    assert abs(W.eilers(0.1) - 1.3192) < 1e-4
