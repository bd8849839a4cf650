"""The pieces of the sheared suspension (Sec. 3.1) on the GPU against the oracle:
spheres across periodic faces (coverage, links, lever arms, pair forces through the
nearest images), the force on the no-slip faces and the contact spring.

- single steps from the oracle's state with spheres straddling the periodic faces
  and moving plates: the single-step bars, the face forces included;
- 150 steps of spheres crossing the faces: positions and velocities against the
  oracle's after the same steps;
- Couette flow between plates: the plate force against mu 2U/n times the area;
- two overlapping spheres: the contact spring moves them apart as in the oracle.
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


def plates(U):
    return [[[0, 0, 0], [0, 0, 0]], [[0, 0, 0], [0, 0, 0]], [[-U, 0, 0], [U, 0, 0]]]


def straddling(integrate=True, contact=0.0):
    """periodic in x and y, plates in z; sphere 0 straddles the x and y faces, 2 the
    y face, 0 and 1 lie 0.31 apart across the x face, 3 sits inside"""
    n = (26, 22, 16)
    x = np.array([[1.3, 1.0, 6.4], [8.0 + 14.0, 1.2, 6.3], [11.6, 20.9, 9.7], [13.0, 11.0, 8.0]])
    p = W.Particles(x=x, u=np.array([[0.01, -0.004, 0.002], [-0.006, 0.008, 0.0], [0.0, 0.0, -0.003],
                                     [0.004, 0.003, 0.0]]),
                    omega=np.array([[0.002, 0.0, -0.003], [0.0, 0.004, 0.001], [-0.002, 0.0, 0.0], [0.0, 0.0, 0.002]]),
                    R=np.array([2.6, 2.4, 2.4, 3.0]), rho_p=np.array([2.0, 2.5, 3.0, 2.0]))
    return W.Workload(name="straddle", n=n, trt=True, tau=0.6, g=(0, 0, -1e-5), zs=-1.0, steps=0,
                      periodic=(1, 1, 0), particles=p, integrate=integrate, contact_k=contact)


@pytest.mark.parametrize("integrate", [False, True])
def test_single_step_spheres_across_periodic_faces(integrate):
    w = straddling(integrate)
    wall = plates(0.01)
    say("single step, spheres across periodic faces, integrate", integrate)
    o = O.Oracle(w, wall_u=wall)
    o.step(8)
    s = fsl.Sim(w, wall_u=wall)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))
    o.close()
    s.close()


def test_spheres_crossing_faces_multistep():
    """Spheres driven along x and y by a body force cross the periodic faces several
    times: positions and velocities against the oracle's after 150 steps (FP32
    populations against FP64: 1e-6 of the distance travelled, 1e-4 relative on the
    velocities), cell types within a few interface-free coverage flips."""
    n = (20, 18, 14)
    p = W.Particles(x=np.array([[17.5, 9.0, 6.5], [5.0, 16.8, 7.2]]), u=np.array([[0.08, 0.02, 0.0], [-0.05, 0.09, 0.0]]),
                    omega=np.zeros((2, 3)), R=np.array([3.0, 2.5]), rho_p=np.array([8.0, 8.0]))
    w = W.Workload(name="cross", n=n, trt=True, tau=0.7, g=(0, 0, 0), zs=-1.0, steps=0,
                   periodic=(1, 1, 0), particles=p, contact_k=0.05)
    o = O.Oracle(w, wall_u=plates(0.02))
    s = fsl.Sim(w, wall_u=plates(0.02))
    o.step(150)
    s.step(150)
    s.sync()
    a, b = o.particles_get(2), s.particles_get(2)
    say("  oracle x", a["x"].tolist(), "gpu x", b["x"].tolist())
    dx = b["x"] - a["x"]
    for k in range(2):
        dx[:, k] -= n[k] * np.round(dx[:, k] / n[k])
    travelled = 150 * np.abs(a["u"]).max()
    assert np.abs(dx).max() < 1e-6 * max(travelled, 1.0)
    assert np.abs(b["u"] - a["u"]).max() < 1e-4 * np.abs(a["u"]).max()
    mism = (o.get(O.FLAGS) != s.get(fsl.FIELD_FLAGS)).sum()
    assert mism <= 4, mism
    o.close()
    s.close()


def test_couette_plate_force_gpu():
    n, U, tau = (5, 4, 12), 0.01, 0.8
    w = W.Workload(name="couette", n=n, trt=True, tau=tau, g=(0, 0, 0), zs=-1.0, steps=0, periodic=(1, 1, 0),
                   integrate=False)
    s = fsl.Sim(w, wall_u=plates(U))
    s.step(20000)
    F = s.walls()
    s.close()
    mu, A = (tau - 0.5) / 3.0, n[0] * n[1]
    shear = mu * 2.0 * U / n[2] * A
    say("  plate forces", F[2].tolist(), "expected shear", shear)
    # FP32 populations: the shear within 1e-5, the pressure A/3 within 1e-6
    assert abs(F[2, 1, 0] / -shear - 1) < 1e-5 and abs(F[2, 0, 0] / shear - 1) < 1e-5
    assert abs(F[2, 1, 2] / (A / 3.0) - 1) < 1e-6 and abs(F[2, 0, 2] / (-A / 3.0) - 1) < 1e-6


def test_contact_spring_gpu():
    """Two spheres set 0.4 cells into each other in a fluid at rest: after 20 steps
    of the spring, lubrication and the fluid, velocities against the oracle's."""
    n = (24, 20, 20)
    p = W.Particles(x=np.array([[9.0, 10.0, 10.0], [14.6, 10.3, 10.0]]), u=np.zeros((2, 3)), omega=np.zeros((2, 3)),
                    R=np.array([3.0, 3.0]), rho_p=np.array([4.0, 4.0]))
    w = W.Workload(name="contact", n=n, trt=True, tau=0.8, g=(0, 0, 0), zs=-1.0, steps=0, periodic=(1, 1, 1),
                   particles=p, contact_k=0.05)
    o, s = O.Oracle(w), fsl.Sim(w)
    o.step(20)
    s.step(20)
    s.sync()
    a, b = o.particles_get(2), s.particles_get(2)
    say("  oracle u", a["u"].tolist(), "gpu u", b["u"].tolist())
    assert a["u"][1, 0] - a["u"][0, 0] > 1e-4  # pushed apart
    assert np.abs(b["u"] - a["u"]).max() < 1e-4 * np.abs(a["u"]).max()
    o.close()
    s.close()


def test_reduced_sheared_suspension_plate_force():
    """The sheared suspension on a reduced box (40 x 36 x 32, 26 spheres of R = 4 at
    Phi = 0.15, plates at +-0.01, Re_P = 0.5, contact on): the plate force of every
    step over 500 steps against the oracle's, and its mean over the last 250 steps
    (the quantity mu_s = F_x / (A gamma) is taken from) within 1e-4."""
    w, wall = W.sheared_suspension(0.15, re_p=0.5, n=(40, 36, 32), R=4.0, seed=3)
    assert w.particles.n == 26
    o, s = O.Oracle(w, wall_u=wall), fsl.Sim(w, wall_u=wall)
    fo, fg = [], []
    for t in range(500):
        o.step(1)
        s.step(1)
        Wo, Wg = o.walls(), s.walls()
        fo.append(0.5 * (Wo[2, 0, 0] - Wo[2, 1, 0]))
        fg.append(0.5 * (Wg[2, 0, 0] - Wg[2, 1, 0]))
    fo, fg = np.array(fo), np.array(fg)
    say("  plate force, oracle mean", fo[250:].mean(), "gpu mean", fg[250:].mean(),
        "max step difference", np.abs(fo - fg).max())
    assert np.abs(fo - fg).max() < 1e-4 * np.abs(fo).max()
    assert abs(fg[250:].mean() / fo[250:].mean() - 1) < 1e-4
    np.testing.assert_array_equal(o.get(O.FLAGS), s.get(fsl.FIELD_FLAGS))
    o.close()
    s.close()


def cut_by_plates(integrate=True, depth=0.6):
    """spheres reaching beyond both plates, one of them also across the periodic x face,
    one sliding towards the low plate"""
    n = (24, 20, 22)
    R = np.array([4.0, 3.5, 3.0])
    x = np.array([[1.2, 9.3, -0.5 + 4.0 - depth], [12.4, 10.2, 21.5 - 3.5 + depth], [12.0, 4.0, 3.4]])
    p = W.Particles(x=x, u=np.array([[0.004, -0.002, -0.003], [0.0, 0.003, 0.002], [0.002, 0.0, -0.02]]),
                    omega=np.array([[0.0, 0.002, 0.0], [0.001, 0.0, -0.002], [0.0, 0.0, 0.0]]),
                    R=R, rho_p=np.array([3.0, 3.0, 3.0]))
    return W.Workload(name="cut", n=n, trt=True, tau=0.7, g=(0, 0, 0), zs=-1.0, steps=0,
                      periodic=(1, 1, 0), particles=p, integrate=integrate, contact_k=0.05)


@pytest.mark.parametrize("integrate", [False, True])
def test_single_step_spheres_cut_by_moving_plates(integrate):
    """Links into sphere nodes from beyond the plates and the face lubrication and
    spring: one step from the oracle's state, the single-step bars (face forces
    included)."""
    w = cut_by_plates(integrate)
    wall = plates(0.01)
    say("single step, spheres cut by moving plates, integrate", integrate)
    o = O.Oracle(w, wall_u=wall)
    o.step(6)
    fo = o.get(O.FLAGS).reshape(w.n[2], w.n[1], w.n[0])
    assert (fo[0] == O.SOL).sum() > 0 and (fo[-1] == O.SOL).sum() > 0
    s = fsl.Sim(w, wall_u=wall)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))
    o.close()
    s.close()


def test_resting_spheres_cut_by_plates_gpu():
    """Fluid at rest, resting plates, resting spheres cut by the plates: no force or
    torque on the spheres and the pressure 1/3 over each plate's whole area."""
    w = cut_by_plates(False, depth=1.1)
    p = w.particles
    w = w.replace(particles=W.Particles(x=p.x, u=0 * p.u, omega=0 * p.omega, R=p.R, rho_p=p.rho_p))
    s = fsl.Sim(w)
    s.step(3)
    s.sync()
    q = s.particles_get(3)
    say("  F", q["F"].tolist(), "T", q["T"].tolist())
    np.testing.assert_allclose(q["F"], 0.0, atol=1e-12)
    # the lever arms are FP32 (x - x_P rounded to 2^-24 relative at |x - x_P| <= R + 2):
    # about a thousand links of 1/9 or 1/18 leave at most a few 1e-5 (missing face
    # links would leave about 1/3 per cut node at an arm of R)
    np.testing.assert_allclose(q["T"], 0.0, atol=1e-5)
    F = s.walls()
    A = w.n[0] * w.n[1]
    np.testing.assert_allclose(F[2, 0], [0, 0, -A / 3.0], rtol=0, atol=1e-9 * A)
    np.testing.assert_allclose(F[2, 1], [0, 0, A / 3.0], rtol=0, atol=1e-9 * A)
    s.close()


def test_spheres_at_moving_plates_multistep():
    """120 steps of spheres at the moving plates (one driven into the low plate): the
    positions and velocities against the oracle's."""
    w = cut_by_plates(True)
    wall = plates(0.02)
    o, s = O.Oracle(w, wall_u=wall), fsl.Sim(w, wall_u=wall)
    o.step(120)
    s.step(120)
    s.sync()
    a, b = o.particles_get(3), s.particles_get(3)
    say("  oracle x", a["x"].tolist(), "gpu x", b["x"].tolist())
    dx = b["x"] - a["x"]
    for k in range(2):
        dx[:, k] -= w.n[k] * np.round(dx[:, k] / w.n[k])
    assert np.abs(dx).max() < 1e-6
    assert np.abs(b["u"] - a["u"]).max() < 1e-4 * np.abs(a["u"]).max()
    assert a["x"][2, 2] - 3.0 > -0.5  # held off the low plate
    o.close()
    s.close()


def many_at_plates():
    """600 spheres (above the one-block integration's 512): a layer of 441 cut by the
    low plate on a 3-cell grid, 159 higher up, plates moving along x"""
    n = (64, 64, 20)
    g = np.arange(21) * 3.0 + 1.5
    gx, gy = np.meshgrid(g, g, indexing="ij")
    low = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 0.5)], axis=1)  # h = 1.0 < R
    rng = np.random.default_rng(4)
    high = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 10.0)], axis=1)[rng.permutation(gx.size)[:159]]
    x = np.concatenate([low, high])
    u = rng.uniform(-0.01, 0.01, size=x.shape)
    u[:441, 2] = -np.abs(u[:441, 2])  # the low layer moves into the plate
    p = W.Particles(x=x, u=u, omega=np.zeros_like(x), R=np.full(600, 1.2), rho_p=np.full(600, 3.0))
    return W.Workload(name="many_at_plates", n=n, trt=True, tau=0.7, g=(0, 0, -1e-5), zs=-1.0, steps=0,
                      periodic=(1, 1, 0), particles=p, contact_k=0.05)


def test_many_spheres_at_plates_single_step_and_multistep():
    """The per-substep launches (k_lub, k_substep with the face lubrication and spring)
    and the face links with 600 spheres: one step from the oracle's state within the
    single-step bars, then 30 steps from the start against the oracle's positions and
    velocities."""
    w = many_at_plates()
    wall = plates(0.01)
    o = O.Oracle(w, wall_u=wall)
    o.step(3)
    fo = o.get(O.FLAGS).reshape(w.n[2], w.n[1], w.n[0])
    assert (fo[0] == O.SOL).sum() >= 441
    s = fsl.Sim(w, wall_u=wall)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))
    o.close()
    s.close()
    o, s = O.Oracle(w, wall_u=wall), fsl.Sim(w, wall_u=wall)
    o.step(30)
    s.step(30)
    s.sync()
    a, b = o.particles_get(600), s.particles_get(600)
    dx = b["x"] - a["x"]
    for k in range(2):
        dx[:, k] -= w.n[k] * np.round(dx[:, k] / w.n[k])
    say("  max |dx|", np.abs(dx).max(), "max |du|", np.abs(b["u"] - a["u"]).max(), "of", np.abs(a["u"]).max())
    assert np.abs(dx).max() < 1e-6
    assert np.abs(b["u"] - a["u"]).max() < 1e-4 * np.abs(a["u"]).max()
    assert a["x"][:441, 2].min() > -0.5  # no centre reached the plate
    o.close()
    s.close()


def test_face_forces_off_changes_nothing_else():
    """A context made without the face forces: walls() fails, and after 20 steps at
    moving plates its cell types and particle owners equal those of a context that
    computes them, its populations and sphere states to rounding (the FP64 force sums
    take no fixed order, as between any two runs): the face forces are a diagnostic,
    never fed back."""
    w = cut_by_plates(True)
    wall = plates(0.01)
    a, b = fsl.Sim(w, wall_u=wall), fsl.Sim(w, wall_u=wall, face_forces=False)
    a.step(20)
    b.step(20)
    a.sync()
    b.sync()
    with pytest.raises(fsl.FslError, match="no_face_forces"):
        b.walls()
    assert np.abs(a.walls()).max() > 0
    for k in (fsl.FIELD_FLAGS, fsl.FIELD_PID):
        np.testing.assert_array_equal(a.get(k), b.get(k))
    fl = a.get(fsl.FIELD_FLAGS)
    act = (fl == fsl.LIQ) | (fl == fsl.IFC)
    fa, fb = a.get(fsl.FIELD_F)[:, act], b.get(fsl.FIELD_F)[:, act]
    assert np.abs(fa - fb).max() <= 1e-9 * np.abs(fa).max()
    pa, pb = a.particles_get(3), b.particles_get(3)
    assert np.abs(pa["x"] - pb["x"]).max() < 1e-9
    for k in ("u", "omega", "F", "T"):
        assert np.abs(pa[k] - pb[k]).max() <= 1e-6 * np.abs(pa[k]).max(), k
    a.close()
    b.close()


@pytest.mark.parametrize("slip", [False, True])
def test_spheres_cut_by_edges_and_corners(slip):
    """A walled box (no-slip, the low x face moving along y; or free-slip x and y faces
    with a no-slip floor): spheres cut by two or three faces at once, whose links
    from beyond an edge or a corner take the first no-slip face they cross (or rest
    when they cross free-slip faces only).  One step from the oracle's state within
    the single-step bars, face forces included."""
    n = (22, 20, 18)
    R = np.array([3.0, 2.5, 3.5, 2.0])
    x = np.array([[2.0, 1.9, 8.0],      # cut by the low x and low y faces
                  [19.6, 10.0, 1.6],    # high x and low z
                  [2.6, 17.0, 14.2],    # low x, high y, high z
                  [11.0, 9.0, 1.2]])    # the floor alone
    p = W.Particles(x=x, u=np.array([[0.003, -0.002, 0.0], [0.002, 0.001, -0.003], [0.0, 0.002, 0.001],
                                     [0.001, 0.0, -0.004]]),
                    omega=np.array([[0.0, 0.0, 0.003], [0.002, 0.0, 0.0], [0.0, -0.002, 0.0], [0.0, 0.0, 0.0]]),
                    R=R, rho_p=np.full(4, 3.0))
    w = W.Workload(name="corners", n=n, trt=True, tau=0.7, g=(0, 0, -1e-5), zs=-1.0, steps=0, periodic=(0, 0, 0),
                   particles=p, contact_k=0.05, freeslip=(1, 1, 0) if slip else (0, 0, 0))
    wall = [[[0.0] * 3, [0.0] * 3] for _ in range(3)]
    if not slip:
        wall[0][0][1] = 0.01  # the low x face moves along y
    o = O.Oracle(w, wall_u=wall)
    o.step(4)
    fo = o.get(O.FLAGS).reshape(n[2], n[1], n[0])
    assert (fo[:, :, 0] == O.SOL).any() and (fo[:, 0, :] == O.SOL).any() and (fo[0] == O.SOL).any()
    s = fsl.Sim(w, wall_u=wall)
    transfer(o, s, w)
    o.step(1)
    s.step(1)
    s.sync()
    say(compare_step(o, s, w))
    o.close()
    s.close()
