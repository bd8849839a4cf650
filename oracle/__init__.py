"""ctypes loader of the plain FP64 CPU oracle (fsl_oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark; the product package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc_fsl.so")
SRC = os.path.join(HERE, "fsl_oracle.c")

FLAGS, MASS, PHI, F, BUBBLE_ID, PID, RHO, U = range(8)
GAS, LIQ, IFC, SOL = 0, 1, 2, 3


def build(force=True):
    """Compile the oracle with plain gcc: FP64, no FMA contraction, OpenMP loops."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-Wall", "-shared",
           "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


class OrcConfig(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("periodic", ctypes.c_int * 3),
        ("trt", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("magic", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("zs", ctypes.c_double),
        ("rho_g0", ctypes.c_double),
        ("n_gas_spheres", ctypes.c_int),
        ("gas_spheres", (ctypes.c_double * 5) * 16),
        ("eps_c", ctypes.c_double),
        ("integrate", ctypes.c_int),
        ("n_sub", ctypes.c_int),
        ("max_particles", ctypes.c_int),
        ("max_bubbles", ctypes.c_int),
        ("wall_u", ((ctypes.c_double * 3) * 2) * 3),
        ("n_threads", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("freeslip", ctypes.c_int * 3),
        ("open_atmosphere", ctypes.c_int),
        ("contact_k", ctypes.c_double),
    ]


class OrcBubble(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int), ("alive", ctypes.c_int), ("V", ctypes.c_double),
        ("M", ctypes.c_double), ("rho_g", ctypes.c_double), ("centroid", ctypes.c_double * 3),
        ("V0", ctypes.c_double), ("n_gas", ctypes.c_int64), ("n_iface", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_create.restype = P
        L.orc_create.argtypes = [ctypes.POINTER(OrcConfig)]
        L.orc_destroy.argtypes = [P]
        L.orc_step.argtypes = [P, ctypes.c_int]
        L.orc_particles_set.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp]
        L.orc_particles_get.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp]
        L.orc_bubbles_get.argtypes = [P, ctypes.POINTER(OrcBubble), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
        L.orc_mass_get.argtypes = [P, dp, dp]
        L.orc_field_get.argtypes = [P, ctypes.c_int, P]
        L.orc_field_set.argtypes = [P, ctypes.c_int, P]
        L.orc_bubbles_set.argtypes = [P, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]
        L.orc_error.restype = ctypes.c_uint32
        L.orc_error.argtypes = [P]
        L.orc_num_cells.argtypes = [P]
        L.orc_window_J.argtypes = [P, ctypes.c_int, dp, dp]
        L.orc_curvature.argtypes = [P, dp]
        L.orc_split.argtypes = [P]
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_lubrication.argtypes = [dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, dp]
        L.orc_contact.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_walls_get.argtypes = [P, dp]
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_face_force.argtypes = [ip, ip, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_lambda_minus.restype = ctypes.c_double
        L.orc_lambda_minus.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def equilibrium(rho, u):
    e = np.zeros(19)
    u = np.ascontiguousarray(u, dtype=np.float64)
    lib().orc_equilibrium(float(rho), _dp(u), _dp(e))
    return e


def lubrication(x1, x2, u1, u2, R1, R2, mu):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (x1, x2, u1, u2)]
    F = np.zeros(3)
    applied = lib().orc_lubrication(*[_dp(v) for v in a], float(R1), float(R2), float(mu), _dp(F))
    return F, bool(applied)


def contact(x1, x2, R1, R2, k):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (x1, x2)]
    F = np.zeros(3)
    applied = lib().orc_contact(*[_dp(v) for v in a], float(R1), float(R2), float(k), _dp(F))
    return F, bool(applied)


def face_force(n, noslip, x, u, R, mu, k):
    """Force of the no-slip faces on one sphere (lubrication limit and contact
    spring); returns (F, number of faces that acted)."""
    ni = np.ascontiguousarray(n, dtype=np.int32)
    ns = np.ascontiguousarray(noslip, dtype=np.int32)
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, u)]
    F = np.zeros(3)
    ip = ctypes.POINTER(ctypes.c_int)
    hits = lib().orc_face_force(ni.ctypes.data_as(ip), ns.ctypes.data_as(ip), *[_dp(v) for v in a],
                                float(R), float(mu), float(k), _dp(F))
    return F, int(hits)


def lambda_minus(tau, magic=3.0 / 16.0, trt=True):
    return lib().orc_lambda_minus(float(tau), float(magic), int(trt))


class Oracle:
    """One FP64 simulation state.  ``w`` is a workloads.Workload."""

    def __init__(self, w, wall_u=None, n_threads=0, max_particles=None, max_bubbles=64):
        cfg = OrcConfig()
        for a in range(3):
            cfg.n[a] = int(w.n[a])
            cfg.periodic[a] = int(w.periodic[a])
            cfg.g[a] = float(w.g[a])
        cfg.trt = int(bool(w.trt))
        cfg.tau = float(w.tau)
        cfg.magic = float(w.magic)
        cfg.zs = float(w.zs)
        cfg.rho_g0 = float(w.rho_g0)
        cfg.n_gas_spheres = len(w.gas_spheres)
        for s, sp in enumerate(w.gas_spheres):
            for a in range(5):
                cfg.gas_spheres[s][a] = float(sp[a])
        cfg.eps_c = float(w.eps_c)
        cfg.integrate = int(bool(w.integrate))
        cfg.n_sub = int(w.n_sub)
        npart = w.particles.n if w.particles is not None else 0
        cfg.max_particles = int(max_particles if max_particles is not None else max(npart, 1))
        cfg.max_bubbles = int(max_bubbles)
        if wall_u is not None:
            for a in range(3):
                for s in range(2):
                    for d in range(3):
                        cfg.wall_u[a][s][d] = float(wall_u[a][s][d])
        cfg.n_threads = int(n_threads)
        cfg.sigma = float(getattr(w, "sigma", 0.0))
        for a in range(3):
            cfg.freeslip[a] = int(getattr(w, "freeslip", (0, 0, 0))[a])
        cfg.open_atmosphere = int(bool(getattr(w, "open_atmosphere", False)))
        cfg.contact_k = float(getattr(w, "contact_k", 0.0))
        self.w = w
        self.N = w.cells
        self.L = lib()
        self.c = self.L.orc_create(ctypes.byref(cfg))
        if not self.c:
            raise MemoryError("oracle allocation failed")
        if npart:
            self.particles_set(w.particles)

    def close(self):
        if self.c:
            self.L.orc_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        return self.L.orc_step(self.c, int(n))

    @property
    def error(self):
        return int(self.L.orc_error(self.c))

    def particles_set(self, p):
        arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (p.x, p.u, p.omega, p.R, p.rho_p)]
        rc = self.L.orc_particles_set(self.c, int(p.n), *[_dp(v) for v in arr])
        if rc:
            raise ValueError("orc_particles_set failed")

    def walls(self):
        """Force of the fluid on each no-slip face over the last step, (3, 2, 3):
        [axis][low/high side][component]."""
        F = np.zeros(18)
        self.L.orc_walls_get(self.c, _dp(F))
        return F.reshape(3, 2, 3)

    def particles_get(self, n):
        out = [np.zeros((n, 3)) for _ in range(5)]
        self.L.orc_particles_get(self.c, int(n), *[_dp(v) for v in out])
        return dict(zip(("x", "u", "omega", "F", "T"), out))

    def bubbles(self):
        buf = (OrcBubble * 64)()
        n = ctypes.c_int(0)
        self.L.orc_bubbles_get(self.c, buf, 64, ctypes.byref(n))
        res = []
        for b in buf[: n.value]:
            res.append(dict(id=b.id, alive=b.alive, V=b.V, M=b.M, rho_g=b.rho_g,
                            centroid=tuple(b.centroid), V0=b.V0, n_gas=b.n_gas,
                            n_iface=b.n_iface))
        return res

    def mass(self):
        t, l = ctypes.c_double(0), ctypes.c_double(0)
        self.L.orc_mass_get(self.c, ctypes.byref(t), ctypes.byref(l))
        return t.value, l.value

    _dtypes = {FLAGS: (np.uint8, 1), MASS: (np.float64, 1), PHI: (np.float64, 1),
               F: (np.float64, 19), BUBBLE_ID: (np.int32, 1), PID: (np.int32, 1),
               RHO: (np.float64, 1), U: (np.float64, 3)}

    def get(self, which):
        dt, k = self._dtypes[which]
        out = np.zeros(k * self.N, dtype=dt)
        self.L.orc_field_get(self.c, which, out.ctypes.data_as(ctypes.c_void_p))
        nx, ny, nz = self.w.n
        shape = (nz, ny, nx) if k == 1 else (k, nz, ny, nx)
        return out.reshape(shape)

    def set(self, which, arr):
        dt, k = self._dtypes[which]
        a = np.ascontiguousarray(arr, dtype=dt).reshape(-1)
        assert a.size == k * self.N
        rc = self.L.orc_field_set(self.c, which, a.ctypes.data_as(ctypes.c_void_p))
        if rc:
            raise ValueError("orc_field_set failed")

    def curvature(self):
        k = np.zeros(self.N)
        if self.L.orc_curvature(self.c, _dp(k)):
            raise RuntimeError("orc_curvature failed")
        return k

    def bubbles_set(self, M, root, alive):
        M = np.ascontiguousarray(M, dtype=np.float64)
        r = np.ascontiguousarray(root, dtype=np.int32)
        a = np.ascontiguousarray(alive, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        if self.L.orc_bubbles_set(self.c, int(M.size), _dp(M), r.ctypes.data_as(ip), a.ctypes.data_as(ip)):
            raise ValueError("orc_bubbles_set failed")

    def split(self):
        """Bubble splitting of the current state: the number of new bubbles."""
        n = self.L.orc_split(self.c)
        if n < 0:
            raise RuntimeError("orc_split: bubble table full")
        return n

    def window_J(self, T, derivative=True):
        J = ctypes.c_double(0)
        dJ = np.zeros(4)
        rc = self.L.orc_window_J(self.c, int(T), ctypes.byref(J),
                                 _dp(dJ) if derivative else None)
        if rc:
            raise RuntimeError("orc_window_J failed")
        return J.value, dJ
