"""Seeded synthetic inputs for the two-component LB + ellipsoid workloads.

This module only draws numbers: initial density fields and particle
placements. It holds none of the method's arithmetic and imports neither the
HIP binding nor the CPU checker; both are fed from here.

Noise is U(-a, +a), independent per node and component, taken from the
(2 n + c)-th output of a SplitMix64 stream seeded by ``seed`` (Steele, Lea &
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
Particle centres, orientations and shapes use numpy's PCG64 with the same seed.

Workload recipes (the paper's own set-ups are random too: random initial
densities for the emulsions of Sec. 4, a flat two-lamella interface for the
single-particle adsorption of Sec. 4):

  interface   32x32x64, rho_A = 0.7 for z < 32 and 0.04 above, B mirrored,
              +-0.001 noise, one prolate ellipsoid (8, 4) on the interface,
              uniform random orientation, colour 0, density 1. seed 1.
  spinodal    128^3, both components 0.7 +- 0.01, no particles. seed 2.
  bijel       256^3, 50/50 (0.7/0.7) or 30/70 (0.42/0.98) +- 0.01, prolate
              (8, 4) ellipsoids at volume fraction 0.15 (4694), random
              non-overlapping centres, uniform orientations, colour 0,
              density 8. seed 3.
  mixed       512^3, 0.7 +- 0.01, aspect m ~ U[0.5, 2], Rperp = 4,
              Rpar = 4 m, colour ~ U[-0.3, 0.3], drawn until the analytic
              particle volume reaches 0.1 of the box, density 8. seed 4.
  ensemble    64 flat-interface systems of uneven sizes, one ellipsoid each
              (Rperp ~ U[3, 6], m log-uniform in [1/4, 4], tilt ~ U[0, 90 deg],
              azimuth ~ U[0, 360 deg), colour ~ U[-0.5, 0.5]). seed 5.
  adsorption  the single-ellipsoid adsorption of Sec. 4: 64^3, walls on the
              two z faces, two lamellae of 31 nodes (red below), g_br = 0.1,
              one ellipsoid R_p = 12, R_o = 6, colour 0 (contact angle 90 deg),
              its axis tilted 0.0057 deg from the interface normal, centred
              in x, y and below the interface. seed 6.
  contact     a sphere of radius R at a flat interface between walls, colour
              dr (the contact-angle calibration of Eq. (11)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """index-th output (0-based) of a SplitMix64 stream started at mix(seed)."""
    with np.errstate(over="ignore"):
        s0 = _mix64(np.array([np.uint64(seed % (1 << 64)) + _GAMMA], dtype=np.uint64))[0]
        st = s0 + (np.asarray(index, dtype=np.uint64) + np.uint64(1)) * _GAMMA
    return _mix64(st)


def uniform01(seed: int, index: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, index) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def node_noise(seed: int, N: int, comp: int, amp: float) -> np.ndarray:
    """U(-amp, +amp) per node for component comp (0 = A, 1 = B)."""
    idx = 2 * np.arange(N, dtype=np.uint64) + np.uint64(comp)
    return amp * (2.0 * uniform01(seed, idx) - 1.0)


def shoemake_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed unit quaternions (w, x, y, z) (Shoemake 1992)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                     b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)


def tilt_quaternion(theta: float, phi: float) -> np.ndarray:
    """Quaternion turning the body z axis to polar angle theta, azimuth phi."""
    h = 0.5 * theta
    return np.array([math.cos(h), -math.sin(h) * math.sin(phi), math.sin(h) * math.cos(phi), 0.0])


@dataclass
class System:
    """One periodic system: sizes, parameters, fields and particles."""
    name: str
    dims: tuple
    tau: float
    g_br: float
    rho_a: np.ndarray
    rho_b: np.ndarray
    radii: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    pos: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    quat: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    delta_rho: np.ndarray = field(default_factory=lambda: np.zeros(0))
    density: np.ndarray = field(default_factory=lambda: np.zeros(0))
    psi_kind: int = 1  # Psi = 1 - exp(-rho), the default effective mass
    seed: int = 0

    @property
    def N(self) -> int:
        return int(self.dims[0] * self.dims[1] * self.dims[2])

    @property
    def n_particles(self) -> int:
        return int(self.radii.shape[0])

    @property
    def max_radius(self) -> float:
        """Largest bounding radius max(R_par, R_perp) of the particles (0 if none)."""
        return float(self.radii.max()) if self.n_particles else 0.0


def _zcoord(dims) -> np.ndarray:
    nx, ny, nz = dims
    return np.repeat(np.arange(nz), nx * ny)


def layered_fields(dims, seed: int, hi: float = 0.7, lo: float = 0.04, amp: float = 0.001, z_split=None):
    """A below z_split, B above (mirrored), plus per-node noise."""
    nx, ny, nz = dims
    N = nx * ny * nz
    zs = nz // 2 if z_split is None else z_split
    z = _zcoord(dims)
    ra = np.where(z < zs, hi, lo) + node_noise(seed, N, 0, amp)
    rb = np.where(z < zs, lo, hi) + node_noise(seed, N, 1, amp)
    return ra, rb


def uniform_fields(dims, seed: int, mean_a: float, mean_b: float, amp: float):
    N = int(np.prod(dims))
    return mean_a + node_noise(seed, N, 0, amp), mean_b + node_noise(seed, N, 1, amp)


def _dilated_nodes(dims, center, quat, rpar, rperp, dil):
    """Flat indices of nodes within the ellipsoid grown by dil (placement only)."""
    nx, ny, nz = dims
    rb = max(rpar, rperp) + dil
    w, x, y, z = quat / np.linalg.norm(quat)
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    lo = np.ceil(np.asarray(center) - rb).astype(int)
    hi = np.floor(np.asarray(center) + rb).astype(int)
    gx, gy, gz = np.meshgrid(np.arange(lo[0], hi[0] + 1), np.arange(lo[1], hi[1] + 1),
                             np.arange(lo[2], hi[2] + 1), indexing="ij")
    d = np.stack([gx.ravel() - center[0], gy.ravel() - center[1], gz.ravel() - center[2]], axis=1)
    b = d @ R
    a_perp, a_par = rperp + dil, rpar + dil
    q = (b[:, 0] ** 2 + b[:, 1] ** 2) / a_perp ** 2 + b[:, 2] ** 2 / a_par ** 2
    m = q <= 1.0
    xs, ys, zs = gx.ravel()[m] % nx, gy.ravel()[m] % ny, gz.ravel()[m] % nz
    return xs + nx * (ys + ny * zs)


def place_particles(dims, rng, n_target: int, shape_fn, max_tries: int = 200000, volume_target=None):
    """Random sequential addition on the lattice: a candidate is kept when its
    shape grown by one node touches no node of an accepted particle, so
    particles start at least one lattice node apart. shape_fn(rng) returns
    (rpar, rperp, delta_rho). Stops at n_target particles, or when the summed
    analytic volume reaches volume_target (if given)."""
    nx, ny, nz = dims
    occ = np.zeros(nx * ny * nz, dtype=bool)
    radii, pos, quats, drho = [], [], [], []
    vol = 0.0
    tries = 0
    while tries < max_tries:
        if volume_target is None and len(radii) >= n_target:
            break
        if volume_target is not None and vol >= volume_target:
            break
        tries += 1
        rpar, rperp, dr = shape_fn(rng)
        c = rng.random(3) * np.array([nx, ny, nz])
        q = shoemake_quaternions(rng, 1)[0]
        idx = _dilated_nodes(dims, c, q, rpar, rperp, 1.0)
        if occ[idx].any():
            continue
        own = _dilated_nodes(dims, c, q, rpar, rperp, 0.0)
        occ[own] = True
        radii.append((rpar, rperp))
        pos.append(c)
        quats.append(q)
        drho.append(dr)
        vol += 4.0 / 3.0 * math.pi * rpar * rperp * rperp
    return (np.array(radii, dtype=np.float64).reshape(-1, 2), np.array(pos).reshape(-1, 3),
            np.array(quats).reshape(-1, 4), np.array(drho, dtype=np.float64))


def interface_system(dims=(32, 32, 64), seed: int = 1, rpar: float = 8.0, rperp: float = 4.0,
                     g_br: float = 0.08, tau: float = 1.0, delta_rho: float = 0.0) -> System:
    """Flat two-lamella interface with one ellipsoid centred on it."""
    nx, ny, nz = dims
    ra, rb = layered_fields(dims, seed)
    rng = np.random.default_rng(seed)
    q = shoemake_quaternions(rng, 1)
    pos = np.array([[nx / 2.0, ny / 2.0, nz / 2.0 - 0.5]])
    return System("interface", tuple(dims), tau, g_br, ra, rb, np.array([[rpar, rperp]]), pos, q,
                  np.array([delta_rho]), np.array([1.0]), seed=seed)


def spinodal_system(n: int = 128, seed: int = 2, g_br: float = 0.08, tau: float = 1.0, dims=None) -> System:
    dims = (n, n, n) if dims is None else tuple(dims)
    ra, rb = uniform_fields(dims, seed, 0.7, 0.7, 0.01)
    return System("spinodal", dims, tau, g_br, ra, rb, seed=seed)


def bijel_system(n: int = 256, seed: int = 3, ratio: str = "50/50", phi: float = 0.15, rpar: float = 8.0,
                 rperp: float = 4.0, g_br: float = 0.08, tau: float = 1.0, dims=None, density: float = 8.0) -> System:
    """Random 1:1 (or 30:70) mixture with prolate ellipsoids at volume
    fraction phi. Particle density 8: at density 1, lighter than the fluid
    (1.4), the gaps between neighbouring bodies develop fluid speeds near 0.9
    within 100 steps."""
    dims = (n, n, n) if dims is None else tuple(dims)
    ma, mb = (0.7, 0.7) if ratio == "50/50" else (0.42, 0.98)
    ra, rb = uniform_fields(dims, seed, ma, mb, 0.01)
    N = int(np.prod(dims))
    n_p = int(round(phi * N / (4.0 / 3.0 * math.pi * rpar * rperp * rperp)))
    rng = np.random.default_rng(seed)
    radii, pos, quat, dr = place_particles(dims, rng, n_p, lambda r: (rpar, rperp, 0.0))
    return System("bijel", dims, tau, g_br, ra, rb, radii, pos, quat, dr, np.full(len(dr), float(density)), seed=seed)


def mixed_system(n: int = 512, seed: int = 4, phi: float = 0.1, g_br: float = 0.08, tau: float = 1.0,
                 dims=None, density: float = 8.0) -> System:
    """Large mixed-precision domain: noise-initialised 50/50 mixture with
    ellipsoids of aspect ratio in [0.5, 2], R_perp = 4, colour in [-0.3, 0.3],
    volume fraction phi. Particle density 8 (the thinnest bodies, R_par = 2,
    run away under explicit momentum-exchange coupling when lighter than a
    few times the fluid density 1.4)."""
    dims = (n, n, n) if dims is None else tuple(dims)
    ra, rb = uniform_fields(dims, seed, 0.7, 0.7, 0.01)
    N = int(np.prod(dims))
    rng = np.random.default_rng(seed)

    def shape(r):
        m = r.uniform(0.5, 2.0)
        return 4.0 * m, 4.0, r.uniform(-0.3, 0.3)

    radii, pos, quat, dr = place_particles(dims, rng, 0, shape, volume_target=phi * N, max_tries=10 ** 7)
    return System("mixed", dims, tau, g_br, ra, rb, radii, pos, quat, dr, np.full(len(dr), float(density)), seed=seed)


def ensemble_systems(n_sys: int = 64, seed: int = 5, g_br: float = 0.08, tau: float = 1.0,
                     max_side: int = 96, density: float = 8.0) -> list:
    """Uneven flat-interface systems with one ellipsoid each. Particle density
    8: the thinnest bodies (R_par down to 0.75) run away under explicit
    momentum-exchange coupling at density 1 (lighter than the fluid)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_sys):
        rperp = rng.uniform(3.0, 6.0)
        m = math.exp(rng.uniform(math.log(0.25), math.log(4.0)))
        rpar = m * rperp
        theta = rng.uniform(0.0, 0.5 * math.pi)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        dr = rng.uniform(-0.5, 0.5)
        need = max(32, 8 * math.ceil((2.0 * max(rpar, rperp) + 8.0) / 8.0))
        need = min(need, max_side)
        sides = np.arange(need, max_side + 1, 8)
        nx = int(rng.choice(sides))
        ny = int(rng.choice(sides))
        nz = 2 * nx + 8 * int(rng.integers(0, 5))
        dims = (nx, ny, nz)
        ra, rb = layered_fields(dims, seed * 1000 + s)
        pos = np.array([[nx / 2.0, ny / 2.0, nz / 2.0 - 0.5]])
        q = tilt_quaternion(theta, phi)[None, :]
        out.append(System(f"ensemble{s}", dims, tau, g_br, ra, rb, np.array([[rpar, rperp]]), pos, q,
                          np.array([dr]), np.array([float(density)]), seed=seed * 1000 + s))
    return out


def wall_mask(dims) -> np.ndarray:
    """Static solid nodes on the two z faces (z = 0 and z = nz - 1)."""
    z = _zcoord(dims)
    return (z == 0) | (z == dims[2] - 1)


def adsorption_system(seed: int = 6, phi0_deg: float = 0.0057, z0: float = 16.5, rpar: float = 12.0,
                      rperp: float = 6.0, g_br: float = 0.1, hi: float = 1.4, lo: float = 0.05,
                      density: float = 1.0) -> System:
    """Sec. 4 single-particle adsorption: 64^3, walls at z = 0 and 63 (the
    paper's z = 1 and 64), fluid z = 1..62 in two lamellae of 31 nodes, red
    (A) below z = 32, g_br = 0.1; lamella densities near the coexisting pair
    at this g (hi / lo, +-0.001 noise); one ellipsoid R_p = 12, R_o = 6,
    colour 0, its axis tilted phi0 from the interface normal (about x), centre
    (32, 32, z0) in the red lamella below the interface at z = 31.5."""
    dims = (64, 64, 64)
    ra, rb = layered_fields(dims, seed, hi=hi, lo=lo, amp=0.001, z_split=32)
    th = math.radians(phi0_deg)
    q = np.array([[math.cos(0.5 * th), math.sin(0.5 * th), 0.0, 0.0]])
    return System("adsorption", dims, 1.0, g_br, ra, rb, np.array([[rpar, rperp]]), np.array([[32.0, 32.0, z0]]), q,
                  np.array([0.0]), np.array([float(density)]), seed=seed)


def contact_system(delta_rho: float, radius: float = 8.0, n: int = 48, seed: int = 7, g_br: float = 0.1,
                   hi: float = 1.4, lo: float = 0.05, density: float = 1.0) -> System:
    """A sphere of radius R with colour delta_rho at a flat interface between
    walls on the z faces (lamellae as in adsorption_system), its centre on the
    interface: the equilibrium height it settles at gives the contact angle."""
    dims = (n, n, n)
    zs = n // 2
    ra, rb = layered_fields(dims, seed, hi=hi, lo=lo, amp=0.001, z_split=zs)
    return System(f"contact{delta_rho:+.2f}", dims, 1.0, g_br, ra, rb, np.array([[radius, radius]]),
                  np.array([[n / 2 + 0.1, n / 2 - 0.2, zs - 0.5]]), np.array([[1.0, 0.0, 0.0, 0.0]]),
                  np.array([float(delta_rho)]), np.array([float(density)]), seed=seed)
