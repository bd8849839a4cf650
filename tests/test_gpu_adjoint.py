"""Differentiation form on the GPU: summed sphere drag over a frozen-cell-type
window and its gradient with respect to tau and g from the library's adjoint
sweep, against the oracle's FP64 tangent-linear derivative (1e-4 relative) and
central finite differences of the oracle (1e-3 relative).

The window of 64^3 periodic fully liquid cells with 20 moving spheres (R = 4,
velocities uniform in [-0.01, 0.01]^3), TRT tau = 0.6, g = (0, 0, -1e-5), 200
steps with a checkpoint every 20, is the workload of the differentiation form; a
walled 160 x 16 x 16 box with rotating spheres and a ragged last segment covers
the interior-tile path and the wall links.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1712_07028_amd as fsl
from paper_1712_07028_amd import workloads as W

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


def oracle_drag(w, T):
    """J from the forces of T ordinary oracle steps."""
    o = O.Oracle(w)
    n = w.particles.n
    u = w.particles.u
    nu = np.linalg.norm(u, axis=1)
    uh = np.where(nu[:, None] > 0, u / np.where(nu > 0, nu, 1)[:, None], 0.0)
    J = 0.0
    for _ in range(T):
        o.step(1)
        J += float(-(o.particles_get(n)["F"] * uh).sum())
    o.close()
    return J


def gpu_window(w, T, k):
    s = fsl.Sim(w, window=(T, k))
    J = s.window_forward(T, k)
    dtau, dg = s.window_backward(1.0)
    s.close()
    return J, np.array([dtau, *dg])


def rel(a, b, scale=None):
    return abs(a - b) / (abs(b) if scale is None else scale)


def walled_box():
    n = (160, 16, 16)
    p = W.particle_bed(4, 3.0, n, -1.0, None, seed=21, vel_range=0.01)
    rng = np.random.Generator(np.random.PCG64(22))
    p.omega[:] = rng.uniform(-2e-3, 2e-3, size=p.omega.shape)
    return W.Workload(name="walled160", n=n, trt=True, tau=0.7, g=(2e-6, 0.0, -1e-5), zs=-1.0,
                      steps=0, periodic=(1, 0, 0), integrate=False, particles=p)


def test_window_gradient_vs_tangent_64():
    w = W.adjoint_window()
    T, k = 200, 20
    say("64^3 window: GPU forward + adjoint")
    J, g = gpu_window(w, T, k)
    say("64^3 window: oracle tangent-linear")
    o = O.Oracle(w)
    Jo, go = o.window_J(T)
    o.close()
    say(f"  J gpu {J:.10e} oracle {Jo:.10e} rel {rel(J, Jo):.2e}")
    scale = np.abs(go[1:]).max()
    for i, name in enumerate(("tau", "gx", "gy", "gz")):
        say(f"  dJ/d{name}: gpu {g[i]:.8e} oracle {go[i]:.8e} rel {rel(g[i], go[i]):.2e}")
    assert rel(J, Jo) < 1e-5
    assert rel(g[0], go[0]) < 1e-4
    # each g component against its own value, or the largest component when it is
    # small compared with the others
    for i in range(1, 4):
        assert abs(g[i] - go[i]) < 1e-4 * max(abs(go[i]), 1e-2 * scale), (i, g[i], go[i])


def test_window_gradient_vs_finite_differences_64():
    w = W.adjoint_window()
    T, k = 200, 20
    _, g = gpu_window(w, T, k)
    h_tau = 1e-4
    fd_tau = (oracle_drag(w.replace(tau=w.tau + h_tau), T) -
              oracle_drag(w.replace(tau=w.tau - h_tau), T)) / (2 * h_tau)
    say(f"  dJ/dtau gpu {g[0]:.8e} central FD {fd_tau:.8e} rel {rel(g[0], fd_tau):.2e}")
    assert rel(g[0], fd_tau) < 1e-3
    h_g = 1e-3 * 1e-5
    gz = list(w.g)
    gp, gm = list(gz), list(gz)
    gp[2] += h_g
    gm[2] -= h_g
    fd_gz = (oracle_drag(w.replace(g=tuple(gp)), T) - oracle_drag(w.replace(g=tuple(gm)), T)) / (2 * h_g)
    say(f"  dJ/dgz gpu {g[3]:.8e} central FD {fd_gz:.8e} rel {rel(g[3], fd_gz):.2e}")
    assert rel(g[3], fd_gz) < 1e-3


def test_window_walls_interior_tiles_ragged_segments():
    w = walled_box()
    T, k = 60, 7
    J, g = gpu_window(w, T, k)
    o = O.Oracle(w)
    Jo, go = o.window_J(T)
    o.close()
    say(f"  J gpu {J:.10e} oracle {Jo:.10e}; grad gpu {g} oracle {go}")
    assert rel(J, Jo) < 1e-5
    scale = np.abs(go).max()
    for i in range(4):
        assert abs(g[i] - go[i]) < 1e-4 * max(abs(go[i]), 1e-2 * scale), (i, g[i], go[i])


def test_drag_window_autograd():
    import torch

    w = W.adjoint_window(n=32, n_particles=4)
    T, k = 40, 10
    s = fsl.Sim(w, window=(T, k))
    tau = torch.tensor(w.tau, dtype=torch.float64, requires_grad=True)
    g = torch.tensor(w.g, dtype=torch.float64, requires_grad=True)
    J = fsl.drag_window(s, tau, g, T, k)
    J.backward()
    s.close()
    Jr, gr = gpu_window(w, T, k)
    assert abs(J.item() - Jr) <= 1e-12 * abs(Jr)
    assert abs(tau.grad.item() - gr[0]) <= 1e-9 * abs(gr[0])
    np.testing.assert_allclose(g.grad.numpy(), gr[1:], rtol=1e-9, atol=1e-9 * np.abs(gr[1:]).max())
    # a second evaluation at another tau: params_set takes effect and the gradient
    # follows (the state restarts from the initial one in a fresh simulation)
    s2 = fsl.Sim(w, window=(T, k))
    tau2 = torch.tensor(w.tau + 0.05, dtype=torch.float64, requires_grad=True)
    J2 = fsl.drag_window(s2, tau2, g.detach(), T, k)
    (dtau2,) = torch.autograd.grad(J2, tau2)
    s2.close()
    o = O.Oracle(w.replace(tau=w.tau + 0.05))
    Jo, go = o.window_J(T)
    o.close()
    assert rel(J2.item(), Jo) < 1e-5 and rel(dtau2.item(), go[0]) < 1e-4


def test_window_argument_errors():
    w = W.bubble_column_small()
    s = fsl.Sim(w, window=(10, 5))
    with pytest.raises(fsl.FslError):
        s.window_forward(10, 5)  # gas and interface cells
    with pytest.raises(fsl.FslError):
        s.window_backward(1.0)   # no completed forward
    s.close()
    w2 = W.adjoint_window(n=32, n_particles=2)
    s = fsl.Sim(w2, window=(10, 5))
    with pytest.raises(fsl.FslError):
        s.window_forward(12, 5)  # longer than reserved
    J = s.window_forward(10, 5)
    assert np.isfinite(J)
    s.params_set(w2.tau, w2.g)
    with pytest.raises(fsl.FslError):
        s.window_backward(1.0)   # parameters changed since the forward window
    s.close()
    s = fsl.Sim(w2)
    with pytest.raises(fsl.FslError):
        s.window_forward(2, 1)   # no window reserved
    s.close()
