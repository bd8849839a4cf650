"""Pins of the oracle's frozen-window drag and its tangent-linear derivative.

The summed drag J = sum_t sum_P (-F_P(t) . u_P/|u_P|) of the window function is
checked against the forces that the oracle's ordinary step reports, and its
forward-mode derivatives in tau and g against central finite differences of
independent oracle runs (FP64), on small periodic and walled windows.
"""
import numpy as np
import pytest

import oracle as O
from paper_1712_07028_amd import workloads as W


def small_window(n=16, nsph=2, seed=11, trt=True, tau=0.6, g=(0.0, 0.0, -1e-5), periodic=(1, 1, 1),
                 omega=0.0):
    box = (n, n, n)
    p = W.particle_bed(nsph, 3.0, box, -1.0, None, seed=seed, vel_range=0.01)
    if omega:
        rng = np.random.Generator(np.random.PCG64(seed + 7))
        p.omega[:] = rng.uniform(-omega, omega, size=p.omega.shape)
    return W.Workload(name="win", n=box, trt=trt, tau=tau, g=g, zs=-1.0, steps=0,
                      periodic=periodic, integrate=False, particles=p)


def drag_by_steps(w, T, pre=0):
    """J from the forces reported by T ordinary oracle steps."""
    o = O.Oracle(w, n_threads=1)
    o.step(pre)
    n = w.particles.n
    u = w.particles.u
    uh = u / np.linalg.norm(u, axis=1)[:, None]
    J = 0.0
    for _ in range(T):
        o.step(1)
        F = o.particles_get(n)["F"]
        J += float(-(F * uh).sum())
    o.close()
    return J


def test_lambda_minus_derivative_through_J():
    # the tau derivative of J includes d lambda_- / d tau of the TRT constraint;
    # checked here against FD of J under SRT and TRT
    for trt in (False, True):
        w = small_window(n=12, nsph=1, trt=trt, tau=0.7)
        o = O.Oracle(w, n_threads=1)
        J, dJ = o.window_J(12)
        o.close()
        h = 1e-4
        Jp = drag_by_steps(w.replace(tau=w.tau + h), 12)
        Jm = drag_by_steps(w.replace(tau=w.tau - h), 12)
        fd = (Jp - Jm) / (2 * h)
        assert abs(dJ[0] - fd) <= 1e-6 * abs(fd), (trt, dJ[0], fd)


@pytest.mark.parametrize("periodic,omega", [((1, 1, 1), 0.0), ((1, 1, 0), 2e-3)])
def test_window_J_equals_step_forces(periodic, omega):
    w = small_window(periodic=periodic, omega=omega)
    T = 16
    o = O.Oracle(w, n_threads=1)
    o.step(3)
    f0 = o.get(O.F)
    J, _ = o.window_J(T)
    # the window leaves the state unchanged
    assert np.array_equal(o.get(O.F), f0)
    o.close()
    Js = drag_by_steps(w, T, pre=3)
    assert abs(J - Js) <= 1e-12 * max(abs(Js), 1e-300), (J, Js)


@pytest.mark.parametrize("periodic,omega", [((1, 1, 1), 0.0), ((1, 1, 0), 2e-3)])
def test_window_tangent_vs_central_differences(periodic, omega):
    w = small_window(periodic=periodic, omega=omega)
    T = 20
    o = O.Oracle(w, n_threads=1)
    J, dJ = o.window_J(T)
    o.close()
    assert abs(J - drag_by_steps(w, T)) <= 1e-12 * abs(J)
    h_tau = 1e-4
    fd_tau = (drag_by_steps(w.replace(tau=w.tau + h_tau), T) -
              drag_by_steps(w.replace(tau=w.tau - h_tau), T)) / (2 * h_tau)
    assert abs(dJ[0] - fd_tau) <= 1e-6 * abs(fd_tau), (dJ[0], fd_tau)
    h_g = 1e-3 * 1e-5
    for a in range(3):
        gp, gm = list(w.g), list(w.g)
        gp[a] += h_g
        gm[a] -= h_g
        fd = (drag_by_steps(w.replace(g=tuple(gp)), T) - drag_by_steps(w.replace(g=tuple(gm)), T)) / (2 * h_g)
        assert abs(dJ[1 + a] - fd) <= 1e-5 * max(abs(fd), 1e-3 * abs(dJ[1:]).max()), (a, dJ[1 + a], fd)


def test_window_rejects_free_surface_state():
    w = W.bubble_column_small()
    o = O.Oracle(w, n_threads=1)
    with pytest.raises(RuntimeError):
        o.window_J(2)
    o.close()
