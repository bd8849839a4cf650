"""Seeded synthetic workloads of the free-surface liquid-gas-solid runs.

This module only generates inputs: box sizes, physical parameters and the
seeded random particle beds.  It holds none of the method's arithmetic and is
shared by the library tests, the oracle tests and the benchmark, so that both
implementations start from the same description.

The workloads follow the shapes of the paper's experiments: a liquid column
with a flat free surface, one spherical gas bubble near the bottom and a random
homogeneous bed of rigid spheres (Sec. 4.1 and 4.2: bubble in a particle bed,
bubble-induced particle mixing), plus a fully liquid periodic window with
moving spheres for the differentiation form.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

STORAGE_F32, STORAGE_F16S, STORAGE_BF16S = 0, 1, 2


@dataclass
class Particles:
    x: np.ndarray  # (n,3) float64 centres in node coordinates
    u: np.ndarray  # (n,3) velocities
    omega: np.ndarray  # (n,3) angular velocities
    R: np.ndarray  # (n,) radii
    rho_p: np.ndarray  # (n,) specific densities

    @property
    def n(self) -> int:
        return int(self.R.shape[0])


@dataclass
class Workload:
    name: str
    n: tuple
    trt: bool
    tau: float
    g: tuple
    zs: float
    steps: int
    periodic: tuple = (0, 0, 0)
    magic: float = 3.0 / 16.0
    rho_g0: float = 1.0
    gas_spheres: list = field(default_factory=list)  # (cx, cy, cz, r, rho_g)
    eps_c: float = 1e-6
    integrate: bool = True
    n_sub: int = 10
    storage: int = STORAGE_F32
    particles: Particles | None = None
    sigma: float = 0.0  # surface tension (0: no Laplace pressure jump)
    freeslip: tuple = (0, 0, 0)  # 1: the faces of a non-periodic axis are free-slip walls
    open_atmosphere: bool = False  # the gas above the pool held at rho_g0 (pressure outlet)
    contact_k: float = 0.0  # stiffness of the sphere contact spring (0: none)

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _draw_centres(rng, lo, hi, count):
    """count candidate centres, uniform per axis in [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((count, 3))


def rsa_spheres(n_target, R, box, zs, bubble=None, seed=0, gap=1.0, max_draws=None,
                batch=4096):
    """Random sequential addition of equal spheres.

    Candidate centres are uniform in [R+1, n-R-2] horizontally and in
    [R+1, top-R-2] vertically (top = zs, or the box height for a fully liquid box);
    a candidate is rejected when its surface gap to an accepted sphere is below
    ``gap`` or when it lies within R_b + R + 1 of the bubble centre.  Candidates
    are tested in draw order against every sphere accepted before them, so the
    result equals a one-by-one RSA with numpy.random.Generator(PCG64(seed)).
    """
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    top = zs if zs >= 0 else box[2]
    lo = [R + 1, R + 1, R + 1]
    hi = [box[0] - R - 2, box[1] - R - 2, top - R - 2]
    dmin = 2 * R + gap
    acc = np.empty((0, 3))
    draws = 0
    max_draws = max_draws or 2000 * n_target + 100000
    # the accepted set does not depend on the batch size (candidates are tested in
    # draw order); small targets use small batches to keep the pair lists short
    batch = min(batch, max(64, 8 * n_target))
    while acc.shape[0] < n_target and draws < max_draws:
        cand = _draw_centres(rng, lo, hi, batch)
        draws += batch
        ok = np.ones(batch, dtype=bool)
        if bubble is not None:
            bc, bR = np.asarray(bubble[:3], dtype=np.float64), float(bubble[3])
            ok &= np.linalg.norm(cand - bc, axis=1) >= bR + R + 1
        if acc.shape[0]:
            d, _ = cKDTree(acc).query(cand, k=1, distance_upper_bound=dmin)
            ok &= ~(d < dmin)
        idx = np.nonzero(ok)[0]
        if idx.size == 0:
            continue
        sub = cand[idx]
        pairs = cKDTree(sub).query_pairs(dmin, output_type="ndarray")
        conflicts = [[] for _ in range(idx.size)]
        for a, b in pairs:
            if np.linalg.norm(sub[a] - sub[b]) < dmin:
                lo_i, hi_i = (a, b) if a < b else (b, a)
                conflicts[hi_i].append(lo_i)
        keep = np.zeros(idx.size, dtype=bool)
        room = n_target - acc.shape[0]
        for i in range(idx.size):
            if room == 0:
                break
            if any(keep[j] for j in conflicts[i]):
                continue
            keep[i] = True
            room -= 1
        acc = np.vstack([acc, sub[keep]])
    return acc[:n_target]


def particle_bed(n, R, box, zs, bubble, seed, rho_p=2.5, vel_range=0.0):
    x = rsa_spheres(n, R, box, zs, bubble=bubble, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    u = (rng.uniform(-vel_range, vel_range, size=x.shape) if vel_range > 0
         else np.zeros_like(x))
    return Particles(x=x, u=u, omega=np.zeros_like(x), R=np.full(x.shape[0], float(R)),
                     rho_p=np.full(x.shape[0], float(rho_p)))


def bubble_column_small():
    """32^3 pool to z=24, bubble R=6 at (16,16,10), SRT tau=0.6, g=1e-5, no particles."""
    return Workload(name="pool32_bubble6_srt", n=(32, 32, 32), trt=False, tau=0.6,
                    g=(0.0, 0.0, -1e-5), zs=24.0, steps=200,
                    gas_spheres=[(16.0, 16.0, 10.0, 6.0, 1.0)])


def bubble_bed_128(n_particles=1400, storage=STORAGE_F32):
    """128^3 pool to z=110, bubble R=12 at (64,64,24), 1,400 spheres R=4 (rho 2.5)."""
    bub = (64.0, 64.0, 24.0, 12.0, 1.0)
    parts = particle_bed(n_particles, 4.0, (128, 128, 128), 110.0, bub, seed=2)
    return Workload(name="bed128_bubble12_1400spheres", n=(128, 128, 128), trt=True,
                    tau=0.55, g=(0.0, 0.0, -2e-5), zs=110.0, steps=1000,
                    gas_spheres=[bub], particles=parts, storage=storage)


def bubble_column_large(n_particles=100_000, nz=1024, zs=980.0):
    """512x512x1024 pool to z=980, bubble R=40 at (256,256,64), 1e5 spheres R=5."""
    bub = (256.0, 256.0, 64.0, 40.0, 1.0)
    parts = particle_bed(n_particles, 5.0, (512, 512, nz), zs, bub, seed=3)
    return Workload(name="column512x512x1024_bubble40_100k_spheres", n=(512, 512, nz),
                    trt=True, tau=0.55, g=(0.0, 0.0, -2e-5), zs=zs, steps=500,
                    gas_spheres=[bub], particles=parts)


def layers_of(w: Workload, z0: int, z1: int, spin_seed: int | None = None,
              vel_range: float = 0.01) -> Workload:
    """Layers z0 <= z < z1 of a walled column as a box of its own, with no-slip faces
    at the cut: the spheres that lie wholly inside with a cell to spare, the gas
    spheres that reach into the cut and the pool surface shifted down by z0 (a
    surface above the cut leaves it liquid throughout).  With spin_seed the kept
    spheres get seeded velocities and angular velocities in (-vel_range, vel_range)
    and (-vel_range/2, vel_range/2), so that moving-wall links and torques are
    exercised."""
    nz = z1 - z0
    p = w.particles
    if p is not None:
        z = p.x[:, 2] - z0
        keep = (z - p.R >= 1.0) & (z + p.R <= nz - 2.0)
        x = p.x[keep].copy()
        x[:, 2] -= z0
        u, om = p.u[keep].copy(), p.omega[keep].copy()
        if spin_seed is not None:
            rng = np.random.Generator(np.random.PCG64(spin_seed))
            u = rng.uniform(-vel_range, vel_range, size=x.shape)
            om = rng.uniform(-vel_range / 2, vel_range / 2, size=x.shape)
        p = Particles(x=x, u=u, omega=om, R=p.R[keep].copy(), rho_p=p.rho_p[keep].copy())
    gas = [(cx, cy, cz - z0, r, rho) for (cx, cy, cz, r, rho) in w.gas_spheres if cz - r < z1 and cz + r > z0]
    zs = w.zs - z0 if w.zs < z1 else -1.0  # a surface above the cut: liquid throughout
    return w.replace(name=f"{w.name}_z{z0}-{z1}", n=(w.n[0], w.n[1], nz), particles=p, zs=zs,
                     gas_spheres=gas)


def periodic_rsa(n_target, R, box, seed=0, gap=0.2, z_margin=1.0, max_draws=None, batch=2048):
    """Random sequential addition of equal spheres in a box periodic along x and y
    and walled along z: candidate centres uniform in [0, n) along x and y and in
    [R + z_margin - 1/2, nz - 1/2 - R - z_margin] along z, rejected when the surface
    gap to an accepted sphere, through the nearest periodic image, is below gap.
    Candidates are drawn in batches from numpy.random.Generator(PCG64(seed)) and
    tested in draw order, so the result equals a one-by-one addition."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.array(box[:2], dtype=np.float64)
    zlo, zhi = R + z_margin - 0.5, box[2] - 0.5 - R - z_margin
    dmin2 = (2 * R + gap) ** 2
    acc = np.empty((0, 3))
    max_draws = max_draws or 20000 * n_target + 100000
    draws = 0

    def sep2(a, b):
        d = a[:, None, :] - b[None, :, :]
        d[..., :2] -= L * np.round(d[..., :2] / L)
        return (d * d).sum(axis=2)

    while acc.shape[0] < n_target and draws < max_draws:
        u = rng.random((batch, 3))
        cand = np.column_stack([u[:, 0] * L[0], u[:, 1] * L[1], zlo + (zhi - zlo) * u[:, 2]])
        draws += batch
        ok = np.ones(batch, dtype=bool) if acc.shape[0] == 0 else (sep2(cand, acc) >= dmin2).all(axis=1)
        sub = cand[ok]
        if sub.shape[0] == 0:
            continue
        clash = sep2(sub, sub) < dmin2
        keep = []
        for k in range(sub.shape[0]):
            if len(keep) == n_target - acc.shape[0]:
                break
            if not any(clash[k, j] for j in keep):
                keep.append(k)
        acc = np.vstack([acc, sub[keep]])
    if acc.shape[0] < n_target:
        raise ValueError(f"placed only {acc.shape[0]} of {n_target} spheres")
    return acc


def sheared_suspension(phi, re_p=0.1, n=(114, 116, 180), R=8.0, rho_s=8.0, U=0.01, seed=11, contact_k=0.5):
    """The sheared suspension of Sec. 3.1 (validation of the particle suspension
    model): a box periodic along x and y between plates at z = -1/2 and nz - 1/2
    moving along x with -U and +U, flow and spheres initially at rest, no gravity,
    N = phi V / V_P spheres of radius R and specific density rho_s at random
    non-overlapping positions.  The particle Reynolds number Re_P = gamma (2R)^2 / mu,
    gamma = 2U / nz, fixes tau (mu = (tau - 1/2) / 3).  Returns the workload and
    the face velocities."""
    V = n[0] * n[1] * n[2]
    VP = 4.0 / 3.0 * np.pi * R ** 3
    N = int(round(phi * V / VP))
    gamma = 2.0 * U / n[2]
    mu = gamma * (2 * R) ** 2 / re_p
    tau = 0.5 + 3.0 * mu
    x = periodic_rsa(N, R, n, seed=seed) if N else np.zeros((0, 3))
    p = Particles(x=x, u=np.zeros_like(x), omega=np.zeros_like(x), R=np.full(N, float(R)),
                  rho_p=np.full(N, float(rho_s))) if N else None
    w = Workload(name=f"suspension{n[0]}x{n[1]}x{n[2]}_phi{phi:g}_re{re_p:g}", n=tuple(n), trt=True,
                 tau=float(tau), g=(0.0, 0.0, 0.0), zs=-1.0, steps=0, periodic=(1, 1, 0), particles=p,
                 contact_k=contact_k if N else 0.0)
    wall = [[[0.0] * 3, [0.0] * 3], [[0.0] * 3, [0.0] * 3], [[-U, 0.0, 0.0], [U, 0.0, 0.0]]]
    return w, wall


def eilers(phi, phi_max=0.63):
    """Eq. Eilers: relative viscosity of a suspension of spheres at volume fraction phi."""
    return (1.0 + 1.25 * phi / (1.0 - phi / phi_max)) ** 2


def adjoint_window(n=64, n_particles=20):
    """Fully liquid periodic n^3 window, 20 spheres R=4 moving with U(-0.01,0.01)^3."""
    parts = particle_bed(n_particles, 4.0, (n, n, n), -1.0, None, seed=5, vel_range=0.01)
    return Workload(name=f"window{n}_periodic_{n_particles}spheres", n=(n, n, n), trt=True,
                    tau=0.6, g=(0.0, 0.0, -1e-5), zs=-1.0, steps=200, periodic=(1, 1, 1),
                    integrate=False, particles=parts)


def slab_of(w: Workload, nz: int) -> Workload:
    """Same column cut to its lowest nz layers (keeps spheres whose box fits)."""
    p = w.particles
    if p is not None:
        keep = p.x[:, 2] + p.R + 2 < nz
        p = Particles(x=p.x[keep], u=p.u[keep], omega=p.omega[keep], R=p.R[keep],
                      rho_p=p.rho_p[keep])
    zs = w.zs if w.zs < nz else -1.0
    return w.replace(n=(w.n[0], w.n[1], nz), particles=p, zs=zs)


# Bubble regimes of Table tab:Annaland (Sec. 3.2): viscosity mu [Pa s], surface
# tension sigma [N/m] and gravity g [m/s^2] for a liquid of 1000 kg/m^3, on a grid of
# dx = 1e-3 m and dt = 1e-4 s; the Reynolds numbers the paper gives (Eq. Fan and its
# own simulations) are kept beside them for comparison.
BUBBLE_REGIMES = {
    "A_spherical": dict(mu=0.25, sigma=0.145, g=0.981, re_fan=1.66, re_paper=1.76),
    "B_ellipsoidal": dict(mu=0.42, sigma=0.145, g=9.81, re_fan=4.18, re_paper=4.43),
    "C_skirted": dict(mu=0.13211, sigma=0.014545, g=9.81, re_fan=18.56, re_paper=14.53),
    "D_dimpled": dict(mu=0.75, sigma=0.014545, g=9.81, re_fan=1.58, re_paper=1.46),
}


def bubble_regime(case: str, n=(40, 40, 100), R=6.0, zs=98.0) -> Workload:
    """A bubble of radius R at (n_x/2, n_y/2, 10) in a liquid column (the set-up of
    Fig. bubbleSetup): free-slip sides, no-slip floor, the gas above the liquid held
    at rho_g0 = 1 (pressure at the top).  Lattice units from dx = 1e-3 m, dt = 1e-4 s,
    rho = 1000 kg/m^3: nu = mu/rho dt/dx^2, g dt^2/dx, sigma dt^2/(rho dx^3).  The
    bubble starts at the liquid pressure at its centre plus the Laplace jump 2 sigma/R
    (density form: times 3)."""
    p = BUBBLE_REGIMES[case]
    dx, dt, rho = 1e-3, 1e-4, 1000.0
    nu = p["mu"] / rho * dt / dx ** 2
    g = p["g"] * dt ** 2 / dx
    sigma = p["sigma"] * dt ** 2 / (rho * dx ** 3)
    zc = 10.0
    rho_b = 1.0 + 3.0 * g * (zs - zc) + 6.0 * sigma / R
    return Workload(name=f"regime_{case}", n=tuple(n), trt=True, tau=3.0 * nu + 0.5, g=(0.0, 0.0, -g), zs=zs,
                    steps=0, gas_spheres=[((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, zc, R, rho_b)], sigma=sigma,
                    freeslip=(1, 1, 0), open_atmosphere=True)
