"""Pins of the oracle's particle-particle interactions (Sec. 2, Eqs. (6)-(9)),
no GPU: Hertz repulsion of equal spheres, its Berne-Pechukas extension to
ellipsoids and the lubrication correction, against closed forms, finite
differences of the pair energy and conservation laws."""
import math

import numpy as np
import pytest

K_H, DC = 100.0, 2.0 / 3.0


def _qaxis(axis):
    """Unit quaternion turning the body z axis onto `axis`."""
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    z = np.array([0.0, 0.0, 1.0])
    c = float(z @ a)
    if c < -1 + 1e-15:
        return np.array([0.0, 1.0, 0.0, 0.0])
    v = np.cross(z, a)
    q = np.array([1.0 + c, *v])
    return q / np.linalg.norm(q)


def _pair(oracle_mod, radii, X, q, dims=(64, 64, 64), V=None, tau=1.0):
    """Two particles in a quiescent fluid (only their pair terms are used)."""
    o = oracle_mod.Oracle(dims, tau, 0.0)
    N = int(np.prod(dims))
    o.init_fields(np.full(N, 0.7), np.full(N, 0.7))
    o.add_ellipsoids(np.asarray(radii, float), np.asarray(X, float), np.asarray(q, float), np.zeros(2),
                     np.full(2, 1.0))
    o.set_pairs(True, K_H, DC)
    if V is not None:
        for k in range(2):
            o.set_particle_motion(k, V=V[k])
    return o


def _contact(oracle_mod, radii, qi, qj, u, lo=0.5, hi=40.0):
    """Centre distance along u where the Hertz energy starts (bisection):
    sigma(o_i, o_j, u) of Eq. (7)."""
    c = np.array([32.0, 32.0, 32.0])
    o = _pair(oracle_mod, radii, [c, c + 1.0], [qi, qj])

    def energy(r):
        o.set_particle_pose(1, X=c - r * np.asarray(u, float))
        return o.pair_hertz(0, 1)[0]

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if energy(mid) > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_sigma_closed_forms(oracle_mod):
    """Eq. (7): chi = 0 (spheres) gives sigma = 2R; identical ellipsoids end
    to end (o_i = o_j = r) give 2 R_p, side by side (o_i = o_j normal to r)
    2 R_o, and the T configuration (o_i along r, o_j normal to it)
    sqrt(2 (R_p^2 + R_o^2)) (derived from Eq. (7) with chi of the pair)."""
    u = np.array([1.0, 0.0, 0.0])
    rp, ro = 8.0, 4.0
    assert abs(_contact(oracle_mod, [[5.0, 5.0]] * 2, _qaxis([0.3, 0.4, 0.5]), _qaxis([0.1, -1, 0.2]), u) - 10.0) < 1e-9
    assert abs(_contact(oracle_mod, [[rp, ro]] * 2, _qaxis(u), _qaxis(u), u) - 2 * rp) < 1e-9
    assert abs(_contact(oracle_mod, [[rp, ro]] * 2, _qaxis([0, 0, 1]), _qaxis([0, 0, 1]), u) - 2 * ro) < 1e-9
    assert abs(_contact(oracle_mod, [[rp, ro]] * 2, _qaxis(u), _qaxis([0, 1, 0]), u)
               - math.sqrt(2 * (rp * rp + ro * ro))) < 1e-9


def test_hertz_spheres_closed_form(oracle_mod):
    """Eq. (6): phi = K_H (2R - r)^{5/2}; the force on i is
    (5/2) K_H (2R - r)^{3/2} along X_i - X_j; no torque for spheres."""
    R, r = 5.0, 9.3
    u = np.array([0.6, -0.48, 0.64])
    c = np.array([30.0, 31.0, 29.0])
    o = _pair(oracle_mod, [[R, R]] * 2, [c + r * u, c], [_qaxis([0.2, 0.5, 0.7]), _qaxis([1, 0, 0])])
    e, F, Ti, Tj = o.pair_hertz(0, 1)
    assert abs(e - K_H * (2 * R - r) ** 2.5) < 1e-12 * e
    assert np.abs(F - 2.5 * K_H * (2 * R - r) ** 1.5 * u).max() < 1e-12 * np.abs(F).max()
    assert np.abs(Ti).max() < 1e-12 and np.abs(Tj).max() < 1e-12


@pytest.mark.parametrize("shape", [(8.0, 4.0), (3.0, 6.0)])
def test_force_and_torque_are_energy_gradients(oracle_mod, shape):
    """F_i = -d phi / d X_i and T_i = -d phi / d theta_i (rotating particle i
    by theta about each axis), by central differences of the oracle's own
    energy, at general orientations and an overlap; and the pair conserves
    angular momentum: T_i + T_j + (X_i - X_j) x F_i = 0."""
    rng = np.random.default_rng(3)
    qi, qj = rng.normal(size=4), rng.normal(size=4)
    qi /= np.linalg.norm(qi)
    qj /= np.linalg.norm(qj)
    c = np.array([32.0, 32.0, 32.0])
    rp, ro = shape
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    s0 = _contact(oracle_mod, [[rp, ro]] * 2, qi, qj, u)
    Xj = c - 0.93 * s0 * u
    o = _pair(oracle_mod, [[rp, ro]] * 2, [c, Xj], [qi, qj])
    o.set_particle_pose(1, X=Xj)
    e0, F, Ti, Tj = o.pair_hertz(0, 1)
    assert e0 > 0
    h = 1e-6
    for d in range(3):
        dx = np.zeros(3)
        dx[d] = h
        o.set_particle_pose(0, X=c + dx)
        ep = o.pair_hertz(0, 1)[0]
        o.set_particle_pose(0, X=c - dx)
        em = o.pair_hertz(0, 1)[0]
        assert abs(-(ep - em) / (2 * h) - F[d]) < 1e-6 * np.abs(F).max()
    o.set_particle_pose(0, X=c)
    for d in range(3):
        half = 0.5 * h
        rot = np.array([math.cos(half), *(math.sin(half) * np.eye(3)[d])])
        rotm = np.array([math.cos(half), *(-math.sin(half) * np.eye(3)[d])])

        def qmul(a, b):
            return np.array([a[0] * b[0] - a[1:] @ b[1:], *(a[0] * b[1:] + b[0] * a[1:] + np.cross(a[1:], b[1:]))])

        o.set_particle_pose(0, q=qmul(rot, qi))
        ep = o.pair_hertz(0, 1)[0]
        o.set_particle_pose(0, q=qmul(rotm, qi))
        em = o.pair_hertz(0, 1)[0]
        assert abs(-(ep - em) / (2 * h) - Ti[d]) < 1e-6 * max(np.abs(Ti).max(), 1e-3 * np.abs(F).max())
    o.set_particle_pose(0, q=qi)
    L = Ti + Tj + np.cross(c - Xj, F)
    assert np.abs(L).max() < 1e-11 * (np.abs(Ti).max() + np.abs(Tj).max() + s0 * np.abs(F).max())


def test_lubrication_closed_form_and_cutoff(oracle_mod):
    """Eq. (9) for spheres: (3 pi mu R^2 / 2) (1/h - 1/Delta_c) times the
    normal relative velocity, opposing it; zero at and beyond the cut-off
    Delta_c = 2/3 and for tangential relative motion."""
    R, tau = 4.0, 1.0
    mu = 1.4 * (tau - 0.5) / 3.0
    u = np.array([0.0, 0.0, 1.0])
    c = np.array([32.0, 32.0, 20.0])
    for h, want in ((0.3, 1.0), (DC, 0.0), (0.9, 0.0)):
        o = _pair(oracle_mod, [[R, R]] * 2, [c + (2 * R + h) * u, c], [_qaxis(u)] * 2,
                  V=[[0.0, 0.0, -0.01], [0.0, 0.0, 0.01]], tau=tau)
        F = o.pair_lub(0, 1)
        mag = 1.5 * math.pi * mu * R * R * 0.02 * (1 / h - 1 / DC)
        if want:
            assert np.abs(F - mag * u).max() < 1e-10 * mag  # pushes the approaching i back along +u
        elif h == DC:
            assert np.abs(F).max() < 1e-12  # continuous at the cut-off (up to the rounding of h)
        else:
            assert np.abs(F).max() == 0.0
    o = _pair(oracle_mod, [[R, R]] * 2, [c + (2 * R + 0.3) * u, c], [_qaxis(u)] * 2,
              V=[[0.01, 0.0, 0.0], [-0.01, 0.02, 0.0]])
    assert np.abs(o.pair_lub(0, 1)).max() < 1e-15


def test_colliding_pair_conserves_momentum_and_rebounds(oracle_mod):
    """Two heavy spheres driven towards each other through the fluid (g = 0):
    the pair forces are equal and opposite, so fluid + particle momentum stays
    constant through the collision (with kill / fill impulses); the Hertz
    repulsion stops the approach after a shallow overlap and reverses it."""
    dims = (48, 32, 32)
    N = int(np.prod(dims))
    o = oracle_mod.Oracle(dims, 1.0, 0.0)
    o.init_fields(np.full(N, 0.5), np.full(N, 0.5))
    o.add_ellipsoids(np.array([[4.0, 4.0], [4.0, 4.0]]), np.array([[14.6, 16.2, 15.9], [24.4, 16.0, 16.1]]),
                     np.tile([1.0, 0, 0, 0], (2, 1)), np.zeros(2), np.full(2, 5.0))
    o.set_pairs(True, K_H, DC)
    o.set_particle_motion(0, V=[0.06, 0, 0])
    o.set_particle_motion(1, V=[-0.06, 0, 0])
    M = [o.particle_extra(k)["M"] for k in range(2)]

    def total():
        s = o.stats()
        v = o.read_particles()["vel"]
        return s[2:5] + M[0] * v[0] + M[1] * v[1] + o.particle_extra(0)["J"] + o.particle_extra(1)["J"]

    P0 = total()
    dmin, rebound = np.inf, False
    for _ in range(50):
        o.step(1)
        p = o.read_particles()
        dmin = min(dmin, p["pos"][1, 0] - p["pos"][0, 0])
        rebound = rebound or (p["vel"][0, 0] < 0 < p["vel"][1, 0])
        assert np.abs(total() - P0).max() < 1e-12 * M[0] * 0.06
    assert 7.5 < dmin < 8.0, dmin  # touched (Hertz range 2R = 8), shallow overlap
    assert rebound
