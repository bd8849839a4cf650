"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Single steps start from identical states (the oracle's state imported into the
library) and must give bit-exact cell types, populations within 1e-6 relative,
interface mass / fill level within 1e-6, and per particle and component the force
within 1e-5 of the particle's force and the torque within 1e-5 of the larger of
the particle's torque and its force at lever arm R + 1.  Multi-step runs must conserve the mass ledger to 1e-10 and
agree with the oracle on the bubble rise velocity and mean particle drag to 1 %.
"""
import math
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


def small_bed(n=40, nsph=12, seed=7, integrate=True, zs=32.0, periodic=(0, 0, 0), storage=0):
    bub = (n / 2, n / 2, 10.0, 6.0, 1.0)
    p = W.particle_bed(nsph, 3.5, (n, n, n), zs, bub, seed=seed, rho_p=2.5, vel_range=0.01)
    rng = np.random.Generator(np.random.PCG64(seed))
    p.omega = rng.uniform(-0.005, 0.005, size=p.x.shape)
    return W.Workload(name=f"bed{n}", n=(n, n, n), trt=True, tau=0.55, g=(0, 0, -2e-5), zs=zs,
                      steps=0, gas_spheres=[bub], particles=p, integrate=integrate, periodic=periodic,
                      storage=storage)


# ---------------------------------------------------------------------------------
def test_init_matches_oracle():
    for w in [W.bubble_column_small(), small_bed(), W.Workload(
            name="ragged", n=(37, 23, 19), trt=False, tau=0.7, g=(0, 0, -1e-5), zs=13.3, steps=0,
            gas_spheres=[(18.2, 11.7, 6.1, 4.3, 1.0), (9.0, 8.0, 5.0, 2.5, 1.1)])]:
        say("init", w.name)
        o, s = O.Oracle(w), fsl.Sim(w)
        np.testing.assert_array_equal(o.get(O.FLAGS), s.get(fsl.FIELD_FLAGS))
        np.testing.assert_array_equal(o.get(O.PHI), s.get(fsl.FIELD_PHI))
        fo = o.get(O.FLAGS)
        act = (fo == O.LIQ) | (fo == O.IFC)
        Fo, Fg = o.get(O.F), s.get(fsl.FIELD_F)
        assert (np.abs(Fg[:, act] - Fo[:, act]) / Fo[:, act]).max() < 1e-7
        ifc = fo == O.IFC
        np.testing.assert_allclose(s.get(fsl.FIELD_MASS)[ifc], o.get(O.MASS)[ifc], rtol=1e-7)
        bo, bg = o.bubbles(), s.bubbles()
        for x, y in zip(bo, bg):
            assert x["alive"] == y["alive"]
            if x["alive"]:
                assert abs(x["V0"] - y["V0"]) < 1e-9 and abs(x["M"] - y["M"]) < 1e-9 * x["M"]
        if w.particles is not None:
            np.testing.assert_array_equal(o.get(O.PID), s.get(fsl.FIELD_PID))
        Mo, Mg = o.mass()[0], s.mass()[0]
        assert abs(Mo - Mg) / Mo < 1e-8


@pytest.mark.parametrize("warm", [0, 25, 80])
def test_single_step_bubble_column(warm):
    w = W.bubble_column_small()
    say("single step, bubble column, after", warm)
    o = O.Oracle(w)
    o.step(warm)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))


@pytest.mark.parametrize("warm", [0, 30])
def test_single_step_particle_bed(warm):
    w = small_bed()
    say("single step, particle bed, after", warm)
    o = O.Oracle(w)
    o.step(warm)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))


def test_single_step_wide_offsets(monkeypatch):
    """The 64-bit form of the marching pass's bounce-back pulls, which boxes of 2^30
    cells and more take, forced on the particle bed: the same bars."""
    monkeypatch.setenv("FSL_WIDE_OFFSETS", "1")
    w = small_bed()
    say("single step, particle bed, 64-bit pull offsets")
    o = O.Oracle(w)
    o.step(30)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))


@pytest.mark.parametrize("integrate", [False, True])
def test_single_step_touching_spheres(integrate):
    """Three spheres with surface gaps below one cell: nodes of one sphere have links
    into another, so the particle-particle momentum exchange (equilibrium at the
    solid node) and lubrication are both active."""
    x = np.array([[10.2, 12.1, 11.4], [17.9, 12.6, 11.9], [14.1, 18.8, 11.2]])
    p = W.Particles(x=x, u=np.array([[0.01, 0, 0], [-0.01, 0.002, 0], [0, -0.005, 0.003]]),
                    omega=np.array([[0, 0, 0.004], [0.002, 0, 0], [0, 0, -0.003]]),
                    R=np.array([3.6, 3.8, 3.3]), rho_p=np.full(3, 2.5))
    w = W.Workload(name="touch", n=(28, 28, 24), trt=True, tau=0.6, g=(0, 0, -1e-5), zs=20.0,
                   steps=0, particles=p, integrate=integrate)
    say("single step, touching spheres, integrate", integrate)
    o = O.Oracle(w)
    o.step(6)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))


@pytest.mark.parametrize("speed", [0.3, 0.7])
def test_single_step_fast_sphere_coverage(speed):
    """A sphere that moves more than half a cell in one step takes every sphere
    through the claim path of the coverage update; a slower one leaves the isolated
    spheres on the path that derives cover and uncover events from the inside tests
    alone.  Both must give the oracle's cell types and owners."""
    x = np.array([[9.3, 10.2, 9.6], [19.4, 9.7, 10.3], [14.2, 19.1, 10.1]])
    p = W.Particles(x=x, u=np.array([[speed, 0.05, 0.0], [-0.02, 0.01, 0.0], [0.0, -0.03, 0.01]]),
                    omega=np.zeros((3, 3)), R=np.array([3.4, 3.1, 3.7]), rho_p=np.full(3, 2.5))
    w = W.Workload(name="fast", n=(28, 28, 22), trt=True, tau=0.7, g=(0, 0, -1e-5), zs=18.0,
                   steps=0, particles=p)
    say("single step, sphere speed", speed)
    o = O.Oracle(w)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    # at these speeds (Mach 0.5 to 1.2) the moving-wall term 6 w rho c.u brings
    # populations through zero, so they are compared against the largest population
    # instead of their own size; the cell types and owners, which are what this case
    # is about, must be identical
    np.testing.assert_array_equal(o.get(O.FLAGS), s.get(fsl.FIELD_FLAGS))
    np.testing.assert_array_equal(o.get(O.PID), s.get(fsl.FIELD_PID))
    fo = o.get(O.FLAGS)
    act = (fo == O.LIQ) | (fo == O.IFC)
    Fo, Fg = o.get(O.F)[:, act], s.get(fsl.FIELD_F)[:, act]
    err = np.abs(Fg - Fo).max() / np.abs(Fo).max()
    a, b = o.particles_get(3), s.particles_get(3)
    dx = np.abs(a["x"] - b["x"]).max()
    say(f"  populations {err:.2e} of the largest, positions {dx:.2e}")
    assert err < 1e-6 and dx < 1e-7


def test_single_step_periodic_window():
    w = W.adjoint_window(n=32, n_particles=6)
    say("single step, periodic window")
    o = O.Oracle(w)
    o.step(5)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))


def test_single_step_ragged_box():
    w = W.Workload(name="ragged", n=(37, 23, 19), trt=False, tau=0.7, g=(0, 0, -1e-5), zs=13.3,
                   steps=0, gas_spheres=[(18.2, 11.7, 6.1, 4.3, 1.0)], periodic=(1, 0, 0))
    say("single step, ragged")
    o = O.Oracle(w)
    o.step(15)
    s = fsl.Sim(w)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))


def test_poiseuille_gpu_closed_form():
    n, g, tau = 16, 1e-7, 0.6
    w = W.Workload(name="pois", n=(1, n, 1), trt=True, tau=tau, g=(g, 0, 0), zs=-1.0, steps=0,
                   periodic=(1, 0, 1), integrate=False)
    s = fsl.Sim(w)
    s.step(40000)
    F = s.get(fsl.FIELD_F)[:, 0, :, 0]
    C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [1, -1, 0], [-1, 1, 0], [-1, -1, 0], [1, 0, 1], [1, 0, -1], [-1, 0, 1],
                  [-1, 0, -1], [0, 1, 1], [0, 1, -1], [0, -1, 1], [0, -1, -1]], float)
    rho = F.sum(0)
    u = (C[:, 0] @ F) / rho - 0.5 * g
    nu = (tau - 0.5) / 3
    h = n / 2
    y = np.arange(n) - (n - 1) / 2
    ua = g / (2 * nu) * (h * h - y * y)
    assert np.abs(u - ua).max() / ua.max() < 1e-4


def test_couette_gpu_closed_form():
    """Faces at y = -1/2 and n - 1/2 moving with -U and +U along x (Eq. bbrule at the
    box walls): the steady profile is exactly linear, u_x = U (2 (y + 1/2)/n - 1)."""
    n, U = 12, 0.01
    w = W.Workload(name="couette", n=(1, n, 1), trt=True, tau=0.8, g=(0, 0, 0), zs=-1.0, steps=0,
                   periodic=(1, 0, 1), integrate=False)
    wall = [[[0, 0, 0], [0, 0, 0]], [[-U, 0, 0], [U, 0, 0]], [[0, 0, 0], [0, 0, 0]]]
    s = fsl.Sim(w, wall_u=wall)
    s.step(30000)
    F = s.get(fsl.FIELD_F)[:, 0, :, 0]
    C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [1, -1, 0], [-1, 1, 0], [-1, -1, 0], [1, 0, 1], [1, 0, -1], [-1, 0, 1],
                  [-1, 0, -1], [0, 1, 1], [0, 1, -1], [0, -1, 1], [0, -1, -1]], float)
    u = (C[:, 0] @ F) / F.sum(0)
    y = np.arange(n)
    ua = U * (2 * (y + 0.5) / n - 1)
    say("  couette max |u - u_exact| / U", np.abs(u - ua).max() / U)
    assert np.abs(u - ua).max() < 1e-5 * U


def test_single_step_moving_walls():
    """Every face of a closed box with a pool and a bubble moves with its own velocity:
    the wall links (edges and corners included, where the first axis beyond the box
    names the face) against the oracle."""
    w = W.Workload(name="walls", n=(20, 14, 18), trt=True, tau=0.7, g=(0, 0, -1e-5), zs=13.0, steps=0,
                   gas_spheres=[(10.0, 7.0, 6.0, 4.0, 1.0)])
    wall = [[[0.0, 0.004, -0.002], [0.0, -0.003, 0.001]], [[0.005, 0.0, 0.002], [-0.004, 0.0, 0.003]],
            [[0.003, -0.002, 0.0], [-0.001, 0.004, 0.0]]]
    o = O.Oracle(w, wall_u=wall)
    o.step(15)
    s = fsl.Sim(w, wall_u=wall)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))


# ---------------------------------------------------------------------------------
def rise_velocity(bubbles_t0, bubbles_t1, dt):
    return (bubbles_t1[1]["centroid"][2] - bubbles_t0[1]["centroid"][2]) / dt


def test_multistep_bubble_column():
    """200 steps of the 32^3 column: ledger mass within 1e-10 of its start value on
    both sides, bubble rise velocity (centroid over the last 10 steps) within 1 %."""
    w = W.bubble_column_small()
    say("multi-step bubble column")
    o, s = O.Oracle(w), fsl.Sim(w)
    Mo0, Mg0 = o.mass()[0], s.mass()[0]
    o.step(190)
    s.step(190)
    bo0, bg0 = o.bubbles(), s.bubbles()
    o.step(10)
    s.step(10)
    s.sync()
    Mo, Mg = o.mass()[0], s.mass()[0]
    vo, vg = rise_velocity(bo0, o.bubbles(), 10), rise_velocity(bg0, s.bubbles(), 10)
    say("mass drift oracle", (Mo - Mo0) / Mo0, "gpu", (Mg - Mg0) / Mg0, "rise", vo, vg)
    assert abs(Mo - Mo0) / Mo0 < 1e-10
    assert abs(Mg - Mg0) / Mg0 < 1e-10
    assert vo > 0 and abs(vg - vo) / abs(vo) < 0.01
    mism = (o.get(O.FLAGS) != s.get(fsl.FIELD_FLAGS)).sum()
    say("flag mismatches after 200 steps", mism)


def test_multistep_particle_bed():
    """300 steps of a 48^3 bed with a bubble and moving spheres: mass ledger within
    1e-10, rise velocity and mean drag (F_z averaged over particles and the last 10
    steps) within 1 % of the oracle."""
    w = small_bed(n=48, nsph=40, seed=3)
    w.particles.u[:] = 0.0
    w.particles.omega[:] = 0.0
    say("multi-step particle bed")
    o, s = O.Oracle(w), fsl.Sim(w)
    Mo0, Mg0 = o.mass()[0], s.mass()[0]
    o.step(290)
    s.step(290)
    bo0, bg0 = o.bubbles(), s.bubbles()
    dro, drg = [], []
    for _ in range(10):
        o.step(1)
        s.step(1)
        dro.append(o.particles_get(w.particles.n)["F"][:, 2].mean())
        drg.append(s.particles_get(w.particles.n)["F"][:, 2].mean())
    Mo, Mg = o.mass()[0], s.mass()[0]
    vo, vg = rise_velocity(bo0, o.bubbles(), 10), rise_velocity(bg0, s.bubbles(), 10)
    do, dg = np.mean(dro), np.mean(drg)
    say("mass drift", (Mo - Mo0) / Mo0, (Mg - Mg0) / Mg0, "rise", vo, vg, "drag", do, dg)
    assert abs(Mo - Mo0) / Mo0 < 1e-10
    assert abs(Mg - Mg0) / Mg0 < 1e-10
    assert abs(vg - vo) / abs(vo) < 0.01
    assert abs(dg - do) / abs(do) < 0.01
