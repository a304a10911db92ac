"""Pins of the oracle's rotational coupling (Sec. 2, Eqs. (4)-(5) and the
kill / fill rule), no GPU.

Linear-momentum conservation holds for any lever arm and any surface velocity,
so it cannot pin the torque of Eq. (5), the W x r part of the bounce-back term
C of Eq. (4), or the centre about which kill / fill impulses act. Two pins do:

* an exact angular-momentum ledger (lever arms and impulse centres), and
* the textbook torque on a rotating sphere, 8 pi mu R^3 omega, with the
  hydrodynamic radius R calibrated from the drag on a fixed sphere in a
  periodic array (Hasimoto's correction), which fixes the magnitude of W x r.

Each pin is also run against a copy of the oracle built with one planted
mistake (ORC_PLANT in oracle/lb_oracle.c) and must reject it.
"""
import math

import numpy as np
import pytest


# ------------------------------------------------------------ angular momentum

def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _angular_ledger(o, c, O):
    """Total angular momentum about the fixed point O: the fluid's
    sum_n (x_n - O) x j_n over both components, the particle's orbital
    (X - O) x M V and spin L, and its pending kill / fill impulse
    H + (X - O) x J (applied at the next body update about the centre it then
    has, which is the current one). Also returns the sum of the magnitudes of
    the terms, the scale of the rounding."""
    nx, ny, nz = o.dims
    j = np.zeros((o.N, 3))
    for comp in (0, 1):
        j += o.get_pops(comp).T @ c
    idx = np.arange(o.N)
    x = np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], 1).astype(float) - O
    p, e = o.read_particles(), o.particle_extra(0)
    X, V = p["pos"][0] - O, p["vel"][0]
    total = np.cross(x, j).sum(0) + np.cross(X, e["M"] * V) + e["L"] + e["H"] + np.cross(X, e["J"])
    scale = (np.linalg.norm(x, axis=1) * np.linalg.norm(j, axis=1)).sum() + np.abs(e["L"]).sum() + \
        e["M"] * np.linalg.norm(V) * np.linalg.norm(X) + np.abs(e["H"]).sum() + np.linalg.norm(X) * np.abs(e["J"]).sum()
    return total, scale, np.abs(j).max(axis=1)


def _ledger_drift(oracle_mod, plant=0, L=44, steps=14):
    """A spinning, translating ellipsoid (g = 0) in an exactly uniform fluid at
    rest. The disturbance spreads one node per step, so for `steps` steps it
    stays clear of the periodic cut (where a wrapped lever arm would jump) and
    the total angular momentum about the box centre must stay constant to
    rounding: streaming moves f_i c_i along c_i (c_i x c_i = 0), BGK keeps each
    node's momentum, a bounce-back link hands (2 f* + C) c_i to the particle
    at the node's lever arm, kill / fill hand the node's momentum over at the
    moved centre. Returns the largest relative drift and bookkeeping."""
    dims = (L, L, L)
    N = L ** 3
    o = oracle_mod.Oracle(dims, 1.0, 0.0, plant=plant)
    o.init_fields(np.full(N, 0.5), np.full(N, 0.4))
    q = np.array([0.8, 0.3, -0.4, 0.2])
    q /= np.linalg.norm(q)
    ctr = np.array([L / 2 + 0.31, L / 2 - 0.27, L / 2 + 0.13])
    o.add_ellipsoids(np.array([[5.0, 3.0]]), ctr[None, :], q[None, :], np.zeros(1), np.array([1.0]))
    e = o.particle_extra(0)
    W = np.array([0.01, -0.015, 0.02])
    R = _rot(q)
    Lspin = R @ np.diag([e["Iperp"], e["Iperp"], e["Ipar"]]) @ R.T @ W
    o.set_particle_motion(0, V=[0.04, -0.03, 0.02], L=Lspin, W=W)
    c, _ = oracle_mod.lattice()
    O = np.array([L / 2, L / 2, L / 2])
    A0, _, _ = _angular_ledger(o, c, O)
    own0 = o.owner().copy()
    worst, events = 0.0, 0
    for _ in range(steps):
        o.step(1)
        led = o.ledger()
        events += (led["kill"] > 0) + (led["fill"] > 0)
        A, scale, jmax = _angular_ledger(o, c, O)
        worst = max(worst, float(np.abs(A - A0).max() / scale))
    idx = np.nonzero(jmax > 0)[0]
    xs = np.stack([idx % L, (idx // L) % L, idx // (L * L)], 1)
    extent = float(np.abs(xs - O).max())
    return worst, events, int((o.owner() != own0).sum()), extent


def test_angular_momentum_ledger(oracle_mod):
    """Exact angular-momentum balance of fluid, particle and pending impulses
    through moving bounce-back (Eq. (4)), the exchange torque (Eq. (5)) and
    kill / fill, with the particle crossing nodes."""
    worst, events, flips, extent = _ledger_drift(oracle_mod)
    assert extent < 22 - 1, extent  # the disturbance never reached the periodic cut
    assert events >= 5 and flips >= 5, (events, flips)
    assert worst <= 1e-13, worst


@pytest.mark.parametrize("plant", [1, 3])
def test_angular_momentum_ledger_rejects_planted_mistakes(oracle_mod, plant):
    """Planted: (1) the link torque arm taken from the centre after the coming
    body update; (3) kill / fill angular impulses taken about the centre
    before the update. Either breaks the ledger by many orders of magnitude."""
    oracle_mod.build(force=False, plant=plant)
    worst, _, _, _ = _ledger_drift(oracle_mod, plant=plant)
    assert worst > 1e-8, worst


# ------------------------------------------------------------ Stokes drag / torque

def _hasimoto_k(x):
    """Drag on a sphere in a simple-cubic periodic array, F = 6 pi mu a U / K,
    K = 1 - 2.837 x + 4.19 x^3 - 27.4 x^6, x = a / L (Hasimoto 1959, as tabulated
    for lattice Boltzmann calibration by Ladd 1994)."""
    return 1.0 - 2.837 * x + 4.19 * x ** 3 - 27.4 * x ** 6


TAU, L_BOX, R_IN = 1.25, 32, 4.0
NU = (TAU - 0.5) / 3.0  # kinematic viscosity of BGK


def _fixed_sphere(oracle_mod, plant, u0=None):
    N = L_BOX ** 3
    o = oracle_mod.Oracle((L_BOX,) * 3, TAU, 0.0, plant=plant)
    o.init_fields(np.full(N, 0.5), np.full(N, 0.5), None if u0 is None else np.tile(np.asarray(u0, float), (N, 1)))
    c = np.array([L_BOX / 2 + 0.23, L_BOX / 2 - 0.13, L_BOX / 2 + 0.11])
    # a density of 1e12 keeps the sphere in place and its spin constant
    o.add_ellipsoids(np.array([[R_IN, R_IN]]), c[None, :], np.array([[1.0, 0, 0, 0]]), np.zeros(1),
                     np.array([1e12]))
    return o


def _translational_radius(oracle_mod, plant=0, steps=1200):
    """Fixed sphere in a periodic box with a constant mean flow: the body force
    on the fluid is set every step to the drag on the sphere over the fluid
    mass, so the fluid momentum stays at its initial value and the flow
    relaxes to the steady Stokes flow through the array. Then
    R_h = F K(R_h / L) / (6 pi mu U), U the superficial fluid velocity (the
    physical velocity j/rho + a/2 averaged over the whole cell)."""
    o = _fixed_sphere(oracle_mod, plant, u0=(1e-3, 0.0, 0.0))
    N = L_BOX ** 3
    a = 0.0
    for _ in range(steps):
        o.step(1)
        F = o.particle_extra(0)["F_links"][0]
        s = o.stats()
        a = F / (s[0] + s[1])
        o.set_accel([a, 0.0, 0.0])
    ra, rb, u, own = o.read_fields()
    fl = own == -1
    U = (u[fl, 0].sum() + 0.5 * a * fl.sum()) / N
    mu = (ra + rb)[fl].mean() * NU
    Rh = R_IN
    for _ in range(60):
        Rh = F * _hasimoto_k(Rh / L_BOX) / (6 * math.pi * mu * U)
    return Rh


def _rotating_torque(oracle_mod, plant=0, steps=700, w=1e-3):
    """Steady torque on the same sphere spinning at w about z in fluid at rest,
    and the viscosity mu of that fluid."""
    o = _fixed_sphere(oracle_mod, plant)
    e = o.particle_extra(0)
    o.set_particle_motion(0, V=[0, 0, 0], L=[0, 0, e["Ipar"] * w], W=[0, 0, w])
    o.step(steps)
    ra, rb, _, own = o.read_fields()
    mu = (ra + rb)[own == -1].mean() * NU
    return o.particle_extra(0)["T_links"][2], mu, w


def _torque_ratio(oracle_mod, plant=0):
    Rh = _translational_radius(oracle_mod, plant)
    T, mu, w = _rotating_torque(oracle_mod, plant)
    return -T / (8 * math.pi * mu * Rh ** 3 * w), Rh


def test_rotating_sphere_torque_matches_stokes(oracle_mod):
    """Textbook Stokes results: the torque on a sphere rotating at w is
    -8 pi mu R^3 w, the drag of a sphere in a periodic array follows
    Hasimoto's law. With R_h taken from the drag, the torque agrees within 5 %
    (halfway bounce-back places the translational and rotational boundaries
    slightly differently; periodic images change the torque by O(volume
    fraction) = 0.8 %). The calibrated radius lies within half a spacing of
    the input radius."""
    ratio, Rh = _torque_ratio(oracle_mod)
    assert abs(Rh - R_IN) < 0.5, Rh
    assert abs(ratio - 1.0) < 0.05, (ratio, Rh)


def test_rotating_sphere_torque_rejects_doubled_spin_term(oracle_mod):
    """Planted (2): twice the W x r part of the surface velocity in C. The drag
    calibration is unchanged (W = 0 there) and the torque doubles."""
    oracle_mod.build(force=False, plant=2)
    ratio, _ = _torque_ratio(oracle_mod, plant=2)
    assert abs(ratio - 1.0) > 0.5, ratio


# ------------------------------------------------------------ demixing sign

def test_demixing_rejects_self_coupling(oracle_mod):
    """Planted (4): the Shan-Chen force of a component built from its own
    neighbour sum instead of the other's. Above the critical g the long wave
    then decays instead of growing (the threshold pin of the fluid tests)."""
    oracle_mod.build(force=False, plant=4)
    Lx, tau, kind = 32, 1.0, 1
    pp = (1 - math.exp(-0.7)) * math.exp(-0.7)
    g = 1.1 * (tau - 0.5) / (30.0 * pp * tau)

    def ratio(plant):
        x = np.tile(np.arange(Lx), 9)
        d = 1e-4 * np.sin(2 * np.pi * x / Lx)
        o = oracle_mod.Oracle((Lx, 3, 3), tau, g, kind, plant=plant)
        o.init_fields(0.7 + d, 0.7 - d)

        def amp():
            ra, rb, _, _ = o.read_fields()
            phi = (ra - rb).reshape(-1, Lx)
            return (phi * np.sin(2 * np.pi * np.arange(Lx) / Lx)).sum() / phi.shape[0]

        a0 = amp()
        o.step(800)
        return amp() / a0

    assert ratio(0) > 1.05
    assert ratio(4) < 0.95
