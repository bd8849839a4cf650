"""MI355X-native free-surface lattice Boltzmann hot path for liquid-gas-solid flow.

Python binding of libfsl.so (C ABI declared in include/fsl.h): argument
marshalling only.  Every step of the method runs in the library's HIP kernels;
PyTorch provides the device workspace and the stream.  There is no CPU
fallback: without the built library or a HIP device the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsl.so")

FSL_OK, FSL_E_ARG, FSL_E_HIP, FSL_E_CAPACITY, FSL_E_NUMERIC, FSL_E_INVARIANT = 0, -1, -2, -3, -4, -5
FIELD_FLAGS, FIELD_MASS, FIELD_PHI, FIELD_F, FIELD_BUBBLE_ID, FIELD_PID, FIELD_KAPPA = range(7)
GAS, LIQ, IFC, SOL = 0, 1, 2, 3

EXPORTS = [
    "fsl_workspace_bytes", "fsl_init", "fsl_step", "fsl_particles_set", "fsl_particles_get",
    "fsl_bubbles_get", "fsl_bubbles_set", "fsl_fields_get", "fsl_fields_set", "fsl_mass_get",
    "fsl_sync", "fsl_error_string", "fsl_destroy", "fsl_profile_enable", "fsl_profile_get",
    "fsl_window_forward", "fsl_window_backward", "fsl_params_set", "fsl_init_static", "fsl_walls_get",
]


class FslConfig(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3), ("boundary", ctypes.c_int * 3), ("collision", ctypes.c_int),
        ("tau", ctypes.c_double), ("magic", ctypes.c_double), ("g", ctypes.c_double * 3),
        ("zs", ctypes.c_double), ("rho_g0", ctypes.c_double), ("n_gas_spheres", ctypes.c_int),
        ("gas_spheres", (ctypes.c_double * 5) * 16), ("max_particles", ctypes.c_int),
        ("n_sub", ctypes.c_int), ("integrate", ctypes.c_int), ("storage", ctypes.c_int),
        ("eps_c", ctypes.c_double), ("list_capacity", ctypes.c_int), ("max_bubbles", ctypes.c_int),
        ("window_steps", ctypes.c_int), ("window_every", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("wall_u", ((ctypes.c_double * 3) * 2) * 3),
        ("open_atmosphere", ctypes.c_int),
        ("contact_k", ctypes.c_double),
        ("no_face_forces", ctypes.c_int),
    ]


class FslBubble(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int), ("alive", ctypes.c_int), ("V", ctypes.c_double),
        ("M", ctypes.c_double), ("rho_g", ctypes.c_double), ("centroid", ctypes.c_double * 3),
        ("V0", ctypes.c_double), ("n_gas", ctypes.c_int64), ("n_iface", ctypes.c_int64),
    ]


class FslError(RuntimeError):
    pass


_lib = None


def load_library(path=LIB_PATH):
    """Load libfsl.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)

    if not os.path.exists(path):
        raise FslError(f"{path} is not built; run paper_1712_07028_amd.build.build()")
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.fsl_workspace_bytes.restype = ctypes.c_size_t
    L.fsl_workspace_bytes.argtypes = [ctypes.POINTER(FslConfig)]
    L.fsl_init.argtypes = [ctypes.POINTER(FslConfig), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.fsl_init_static.argtypes = [ctypes.POINTER(FslConfig), P, ctypes.POINTER(ctypes.c_size_t), P,
                                  ctypes.POINTER(P)]
    L.fsl_step.argtypes = [P, ctypes.c_int]
    L.fsl_particles_set.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp]
    L.fsl_particles_get.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp]
    L.fsl_bubbles_get.argtypes = [P, ctypes.POINTER(FslBubble), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.fsl_bubbles_set.argtypes = [P, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int)]
    L.fsl_fields_get.argtypes = [P, ctypes.c_int, P]
    L.fsl_fields_set.argtypes = [P, ctypes.c_int, P]
    L.fsl_mass_get.argtypes = [P, dp, dp]
    L.fsl_walls_get.argtypes = [P, dp]
    L.fsl_sync.argtypes = [P]
    L.fsl_error_string.restype = ctypes.c_char_p
    L.fsl_error_string.argtypes = [P]
    L.fsl_destroy.argtypes = [P]
    L.fsl_profile_enable.argtypes = [P, ctypes.c_int]
    L.fsl_profile_get.argtypes = [P, dp, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
    L.fsl_window_forward.argtypes = [P, ctypes.c_int, ctypes.c_int, dp]
    L.fsl_window_backward.argtypes = [P, ctypes.c_double, dp, dp]
    L.fsl_params_set.argtypes = [P, ctypes.c_double, dp]
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_config(w, max_particles=None, list_capacity=0, window=(0, 0), wall_u=None, max_bubbles=0,
                face_forces=True):
    """fsl_config from a workloads.Workload."""
    c = FslConfig()
    for a in range(3):
        c.n[a] = int(w.n[a])
        # 1 periodic, 2 free-slip, 0 no-slip
        c.boundary[a] = 1 if w.periodic[a] else (2 if getattr(w, "freeslip", (0, 0, 0))[a] else 0)
        c.g[a] = float(w.g[a])
    c.collision = 1 if w.trt else 0
    c.tau = float(w.tau)
    c.magic = float(w.magic)
    c.zs = float(w.zs)
    c.rho_g0 = float(w.rho_g0)
    c.n_gas_spheres = len(w.gas_spheres)
    for s, sp in enumerate(w.gas_spheres):
        for a in range(5):
            c.gas_spheres[s][a] = float(sp[a])
    npart = w.particles.n if w.particles is not None else 0
    c.max_particles = int(max_particles if max_particles is not None else max(npart, 1))
    c.n_sub = int(w.n_sub)
    c.integrate = int(bool(w.integrate))
    c.storage = int(w.storage)
    c.eps_c = float(w.eps_c)
    c.list_capacity = int(list_capacity)
    c.max_bubbles = int(max_bubbles)
    c.open_atmosphere = int(bool(getattr(w, "open_atmosphere", False)))
    c.contact_k = float(getattr(w, "contact_k", 0.0))
    c.no_face_forces = 0 if face_forces else 1
    c.window_steps, c.window_every = int(window[0]), int(window[1])
    c.sigma = float(getattr(w, "sigma", 0.0))
    if wall_u is not None:
        for a in range(3):
            for side in range(2):
                for d in range(3):
                    c.wall_u[a][side][d] = float(wall_u[a][side][d])
    return c


class Sim:
    """One simulation state on the current HIP device.

    The workspace is a torch uint8 tensor.  The library runs on ``stream`` (a
    torch.cuda.Stream), by default a stream of its own at default priority (steps
    replay from a HIP graph only off the null stream).  ``w`` is a
    workloads.Workload.  With ``static=True`` the context comes from
    fsl_init_static: the tensor holds the state only and the working memory is the
    library's own array on the device, shared by every such context on it (give them
    one stream).  ``face_forces=False`` leaves out the force on the no-slip faces
    (``walls()`` then fails)."""

    def __init__(self, w, device="cuda", max_particles=None, list_capacity=0, window=(0, 0),
                 set_particles=True, wall_u=None, max_bubbles=0, static=False, stream=None, face_forces=True):
        import torch

        self.L = load_library()
        if not torch.cuda.is_available():
            raise FslError("no HIP device")
        self.w = w
        self.N = w.cells
        self.cfg = make_config(w, max_particles, list_capacity, window, wall_u, max_bubbles, face_forces)
        self.ctx = ctypes.c_void_p()
        if static:
            dev = torch.device(device)
            if dev.index is None:
                dev = torch.device("cuda", torch.cuda.current_device())
            torch.cuda.set_device(dev)  # the library's array on the stream's device
            nb = ctypes.c_size_t(0)
            rc = self.L.fsl_init_static(ctypes.byref(self.cfg), None, ctypes.byref(nb), None, None)
            if rc:
                raise FslError(f"fsl_init_static failed ({rc}): {self.L.fsl_error_string(None).decode()}")
            self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.workspace.device)
            rc = self.L.fsl_init_static(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                                        ctypes.byref(nb), ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(self.ctx))
            if rc:
                raise FslError(f"fsl_init_static failed ({rc}): {self.L.fsl_error_string(None).decode()}")
        else:
            nbytes = self.L.fsl_workspace_bytes(ctypes.byref(self.cfg))
            if nbytes == 0:
                raise FslError("invalid configuration")
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.workspace.device)
            rc = self.L.fsl_init(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                                 ctypes.c_size_t(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(self.ctx))
            if rc:
                raise FslError(f"fsl_init failed ({rc})")
        self.n_particles = 0
        if set_particles and w.particles is not None and w.particles.n:
            self.particles_set(w.particles)

    def _check(self, rc, what):
        if rc:
            msg = self.L.fsl_error_string(self.ctx).decode()
            raise FslError(f"{what} failed ({rc}): {msg}")

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.L.fsl_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(self.L.fsl_step(self.ctx, int(n)), "fsl_step")

    def sync(self):
        self._check(self.L.fsl_sync(self.ctx), "fsl_sync")

    def particles_set(self, p):
        arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (p.x, p.u, p.omega, p.R, p.rho_p)]
        self._check(self.L.fsl_particles_set(self.ctx, int(p.n), *[_dp(v) for v in arr]),
                    "fsl_particles_set")
        self.n_particles = int(p.n)

    def particles_get(self, n=None):
        n = self.n_particles if n is None else n
        out = [np.zeros((n, 3)) for _ in range(5)]
        self._check(self.L.fsl_particles_get(self.ctx, int(n), *[_dp(v) for v in out]),
                    "fsl_particles_get")
        return dict(zip(("x", "u", "omega", "F", "T"), out))

    def bubbles(self):
        cap = max(64, int(self.cfg.max_bubbles))  # the table's capacity (0 = the default 64)
        buf = (FslBubble * cap)()
        n = ctypes.c_int(0)
        self._check(self.L.fsl_bubbles_get(self.ctx, buf, cap, ctypes.byref(n)), "fsl_bubbles_get")
        return [dict(id=b.id, alive=b.alive, V=b.V, M=b.M, rho_g=b.rho_g, centroid=tuple(b.centroid),
                     V0=b.V0, n_gas=b.n_gas, n_iface=b.n_iface) for b in buf[: n.value]]

    def bubbles_set(self, M, root, alive):
        M = np.ascontiguousarray(M, dtype=np.float64)
        r = np.ascontiguousarray(root, dtype=np.int32)
        a = np.ascontiguousarray(alive, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        self._check(self.L.fsl_bubbles_set(self.ctx, int(M.size), _dp(M), r.ctypes.data_as(ip),
                                           a.ctypes.data_as(ip)), "fsl_bubbles_set")

    def walls(self):
        """Force of the fluid on each no-slip face over the last step, (3, 2, 3):
        [axis][low/high side][component]."""
        F = np.zeros(18)
        self._check(self.L.fsl_walls_get(self.ctx, _dp(F)), "fsl_walls_get")
        return F.reshape(3, 2, 3)

    def mass(self):
        t, l = ctypes.c_double(0), ctypes.c_double(0)
        self._check(self.L.fsl_mass_get(self.ctx, ctypes.byref(t), ctypes.byref(l)), "fsl_mass_get")
        return t.value, l.value

    _dtypes = {FIELD_FLAGS: (np.uint8, 1), FIELD_MASS: (np.float64, 1), FIELD_PHI: (np.float64, 1),
               FIELD_F: (np.float64, 19), FIELD_BUBBLE_ID: (np.int32, 1), FIELD_PID: (np.int32, 1),
               FIELD_KAPPA: (np.float64, 1)}

    def get(self, which):
        dt, k = self._dtypes[which]
        out = np.zeros(k * self.N, dtype=dt)
        self._check(self.L.fsl_fields_get(self.ctx, which, out.ctypes.data_as(ctypes.c_void_p)),
                    "fsl_fields_get")
        nx, ny, nz = self.w.n
        return out.reshape((nz, ny, nx) if k == 1 else (k, nz, ny, nx))

    def set(self, which, arr):
        dt, k = self._dtypes[which]
        a = np.ascontiguousarray(arr, dtype=dt).reshape(-1)
        if a.size != k * self.N:
            raise ValueError("field size mismatch")
        self._check(self.L.fsl_fields_set(self.ctx, which, a.ctypes.data_as(ctypes.c_void_p)),
                    "fsl_fields_set")

    def profile(self, on=True):
        self._check(self.L.fsl_profile_enable(self.ctx, int(on)), "fsl_profile_enable")

    PHASES = ("stream_collide", "conversions", "bubbles", "particle_forces", "particle_substeps",
              "coverage", "curvature", "split")

    def profile_get(self):
        n = len(self.PHASES)
        ms = np.zeros(n)
        cnt = (ctypes.c_longlong * n)()
        rc = self.L.fsl_profile_get(self.ctx, _dp(ms), cnt, n)
        if rc < 0:
            self._check(rc, "fsl_profile_get")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(self.PHASES)}

    def window_forward(self, T, k):
        J = ctypes.c_double(0)
        self._check(self.L.fsl_window_forward(self.ctx, int(T), int(k), ctypes.byref(J)),
                    "fsl_window_forward")
        return J.value

    def window_backward(self, dJ=1.0):
        dtau = ctypes.c_double(0)
        dg = np.zeros(3)
        self._check(self.L.fsl_window_backward(self.ctx, float(dJ), ctypes.byref(dtau), _dp(dg)),
                    "fsl_window_backward")
        return dtau.value, dg

    def params_set(self, tau, g):
        gg = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(3))
        self._check(self.L.fsl_params_set(self.ctx, float(tau), _dp(gg)), "fsl_params_set")


def _drag_window_function():
    import torch

    class DragWindow(torch.autograd.Function):
        """J(tau, g): summed drag of a frozen-cell-type window run by the library
        (fsl_window_forward); the backward pass is the library's adjoint sweep
        (fsl_window_backward).  Runs T steps from the simulation's current state."""

        @staticmethod
        def forward(ctx, tau, g, sim, T, k):
            sim.params_set(float(tau), [float(v) for v in g.reshape(3)])
            J = sim.window_forward(T, k)
            ctx.sim = sim
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            dtau, dg = ctx.sim.window_backward(float(gJ))
            return (torch.tensor(dtau, dtype=torch.float64), torch.from_numpy(dg.copy()),
                    None, None, None)

    return DragWindow


_DRAG_WINDOW = None


def drag_window(sim, tau, g, T, k):
    """Differentiable summed sphere drag over T steps with checkpoints every k steps.

    tau: 0-d float64 tensor, g: float64 tensor of 3 entries; returns a 0-d float64
    tensor whose backward gives dJ/dtau and dJ/dg."""
    global _DRAG_WINDOW
    if _DRAG_WINDOW is None:
        _DRAG_WINDOW = _drag_window_function()
    return _DRAG_WINDOW.apply(tau, g, sim, int(T), int(k))
