"""Pins of the oracle's coverage bookkeeping (Sec. 2.3: nodes inside a particle are
obstacle nodes; what a covered or uncovered node does is a reading), on a closed
form: a fluid at rest at uniform density rho0 and a sphere set again at a shifted
position.

- The particle nodes afterwards are exactly the nodes inside the new sphere (the
  inside test written out here, in FP64 in the same order), owned by it.
- A node the sphere left is liquid and holds the equilibrium at the mean density of
  its liquid neighbours (rho0 here) and the sphere's rigid velocity at the node,
  u_P + omega x (x - x_P): the equilibrium written out here from its definition.
- The ledger takes rho0 for each covered node and pays rho0 for each uncovered one,
  and the total mass (fluid plus ledger) does not change.
A wrong density or velocity for uncovered nodes, a covered node not charged, or a
node left behind fails one of them.
"""
import numpy as np
import pytest

from paper_1712_07028_amd import workloads as W

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [1, -1, 0], [-1, 1, 0], [-1, -1, 0], [1, 0, 1], [1, 0, -1], [-1, 0, 1],
              [-1, 0, -1], [0, 1, 1], [0, 1, -1], [0, -1, 1], [0, -1, -1]], dtype=np.float64)
WQ = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def equilibrium(rho, u):
    cu = C @ u
    return WQ * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))


def inside(n, x, R):
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    d0, d1, d2 = i - x[0], j - x[1], k - x[2]
    return (d0 * d0 + d1 * d1) + d2 * d2 <= R * R


@pytest.mark.parametrize("shift", [(0.7, -0.3, 0.5), (-0.45, 0.0, -0.9)])
def test_cover_uncover_closed_form(orc, shift):
    n, R, rho0 = (20, 18, 16), 4.3, 1.03
    xa = np.array([9.2, 8.7, 7.6])
    xb = xa + np.array(shift)
    u, om = np.array([0.01, -0.02, 0.015]), np.array([0.003, -0.001, 0.002])
    pa = W.Particles(x=xa[None], u=u[None], omega=om[None], R=np.array([R]), rho_p=np.array([2.0]))
    w = W.Workload(name="cover", n=n, trt=True, tau=0.7, g=(0, 0, 0), zs=-1.0, steps=0, periodic=(0, 0, 0),
                   particles=pa, integrate=False)
    o = orc.Oracle(w)
    o.set(orc.F, np.broadcast_to(equilibrium(rho0, np.zeros(3))[:, None, None, None], (19,) + n[::-1]))
    ina, inb = inside(n, xa, R), inside(n, xb, R)
    np.testing.assert_array_equal(o.get(orc.FLAGS) == orc.SOL, ina)
    M0, L0 = o.mass()
    o.particles_set(W.Particles(x=xb[None], u=u[None], omega=om[None], R=np.array([R]), rho_p=np.array([2.0])))
    fl, pid, f = o.get(orc.FLAGS), o.get(orc.PID), o.get(orc.F)
    np.testing.assert_array_equal(fl == orc.SOL, inb)
    assert np.all(pid[inb] == 0)
    unc, cov = ina & ~inb, inb & ~ina
    assert unc.sum() > 10 and cov.sum() > 10
    assert np.all(fl[unc] == orc.LIQ)
    for k, j, i in np.argwhere(unc):
        ur = u + np.cross(om, np.array([i, j, k]) - xb)
        np.testing.assert_allclose(f[:, k, j, i], equilibrium(rho0, ur), rtol=0, atol=1e-15)
    M1, L1 = o.mass()
    assert abs((L1 - L0) - rho0 * (cov.sum() - unc.sum())) < 1e-12
    assert abs(M1 / M0 - 1) < 1e-14
    o.close()
