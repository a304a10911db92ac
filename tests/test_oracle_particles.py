"""Pins of the CPU oracle's particle coupling (raster, shell fill, moving
bounce-back, rigid bodies, kill/fill) against exact arithmetic, closed forms
and conservation laws (no GPU)."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest


def _minimg_exact(d, L):
    h = Fr(L, 2)
    if d > h:
        return d - L
    if d < -h:
        return d + L
    return d


def _exact_owner(dims, parts):
    """Brute force over every node in exact rational arithmetic: the closed
    test (bx^2 + by^2)/Rperp^2 + bz^2/Rpar^2 <= 1 in the body frame, smallest
    particle index wins. parts: (Rpar, Rperp, centre, q) with Fractions and q a
    unit quaternion (w, x, y, z). Also returns |Q - 1| per node (closest)."""
    nx, ny, nz = dims
    own = np.full(nx * ny * nz, -1, dtype=np.int64)
    gap = np.full(nx * ny * nz, np.inf)
    for k, (rpar, rperp, c, q) in enumerate(parts):
        w, x, y, z = q
        R = [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
             [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
             [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]]
        for iz in range(nz):
            for iy in range(ny):
                for ix in range(nx):
                    d = [_minimg_exact(ix - c[0], nx), _minimg_exact(iy - c[1], ny), _minimg_exact(iz - c[2], nz)]
                    b = [sum(R[a][j] * d[a] for a in range(3)) for j in range(3)]
                    Q = (b[0] ** 2 + b[1] ** 2) / rperp ** 2 + b[2] ** 2 / rpar ** 2
                    n = ix + nx * (iy + ny * iz)
                    gap[n] = min(gap[n], abs(float(Q - 1)))
                    if Q <= 1 and own[n] < 0:
                        own[n] = k
    return own, gap


def _oracle_owner(oracle_mod, dims, parts):
    o = oracle_mod.Oracle(dims, 1.0, 0.0)
    N = int(np.prod(dims))
    o.init_fields(np.full(N, 0.5), np.full(N, 0.5))
    radii = np.array([[float(p[0]), float(p[1])] for p in parts])
    pos = np.array([[float(v) for v in p[2]] for p in parts])
    quat = np.array([[float(v) for v in p[3]] for p in parts])
    o.add_ellipsoids(radii, pos, quat, np.zeros(len(parts)))
    return o.owner()


def test_raster_exact_dyadic_with_ties(oracle_mod):
    """Closed inside test (ties Q = 1 count as inside) against exact rational
    brute force. Dyadic centres, radii with power-of-two squares and dyadic
    unit quaternions make the FP64 evaluation exact, so the match must be
    bitwise, including boundary nodes; two overlapping particles check the
    smallest-index rule and a centre near the faces checks the wrap."""
    h = Fr(1, 2)
    dims = (16, 16, 16)
    parts = [
        (Fr(4), Fr(4), (Fr(8), Fr(8), Fr(8)), (Fr(1), Fr(0), Fr(0), Fr(0))),
        (Fr(4), Fr(2), (Fr(10), Fr(33, 4), Fr(27, 4)), (h, h, h, h)),
        (Fr(2), Fr(4), (Fr(1, 2), Fr(61, 4), Fr(1)), (Fr(0), Fr(1), Fr(0), Fr(0))),
    ]
    want, gap = _exact_owner(dims, parts)
    assert (gap == 0).sum() > 0, "case must contain exact ties"
    got = _oracle_owner(oracle_mod, dims, parts)
    assert np.array_equal(got, want)


def test_raster_exact_rational_orientation(oracle_mod):
    """General rational orientation (1,2,2,4)/5 and (7,4,4,0)/9 with
    non-dyadic radii: equal to the exact owner map on every node not within
    1e-9 of the boundary."""
    dims = (16, 16, 16)
    parts = [
        (Fr(11, 2), Fr(11, 4), (Fr(37, 5), Fr(41, 6), Fr(15, 2)), (Fr(1, 5), Fr(2, 5), Fr(2, 5), Fr(4, 5))),
        (Fr(3, 1), Fr(27, 5), (Fr(3, 1), Fr(13, 1), Fr(29, 3)), (Fr(7, 9), Fr(4, 9), Fr(4, 9), Fr(0))),
    ]
    want, gap = _exact_owner(dims, parts)
    got = _oracle_owner(oracle_mod, dims, parts)
    ok = gap > 1e-9
    assert ok.sum() > 0.99 * ok.size
    assert np.array_equal(got[ok], want[ok])
    assert (want >= 0).sum() > 100


@pytest.mark.parametrize("rpar,rperp", [(20.0, 10.0), (9.0, 18.0)])
def test_raster_count_tends_to_volume(oracle_mod, rpar, rperp):
    """The number of covered nodes approaches (4/3) pi Rpar Rperp^2."""
    dims = (64, 64, 64)
    rng = np.random.default_rng(3)
    q = rng.normal(size=4)
    o = oracle_mod.Oracle(dims, 1.0, 0.0)
    N = 64 ** 3
    o.init_fields(np.full(N, 0.5), np.full(N, 0.5))
    o.add_ellipsoids(np.array([[rpar, rperp]]), np.array([[31.3, 30.7, 32.1]]), q[None, :], np.zeros(1))
    cnt = (o.owner() == 0).sum()
    vol = 4.0 / 3.0 * math.pi * rpar * rperp * rperp
    assert abs(cnt / vol - 1) < 0.01


def test_shell_fill_hand_example(oracle_mod):
    """Eq. (10) and the colour rule after it: a solid node with fluid
    neighbours takes the mean of the fluid neighbours only (nodes of any
    particle excluded), then +Delta rho on red (A) if positive, |Delta rho| on
    blue (B) if negative, nothing if zero."""
    dims = (9, 9, 9)
    N = 729
    rng = np.random.default_rng(5)
    ra = rng.uniform(0.2, 0.9, N)
    rb = rng.uniform(0.2, 0.9, N)
    o = oracle_mod.Oracle(dims, 1.0, 0.08)
    o.init_fields(ra, rb)
    # three one-node particles (sphere of radius 1/2 on a node); 0 and 1 touch
    nodes = [(4, 4, 4), (5, 4, 4), (1, 7, 2)]
    drho = [0.05, -0.03, 0.0]
    o.add_ellipsoids(np.full((3, 2), 0.5), np.array(nodes, float), np.tile([1.0, 0, 0, 0], (3, 1)),
                     np.array(drho))
    own = o.owner()
    assert sorted(np.nonzero(own >= 0)[0].tolist()) == sorted(x + 9 * (y + 9 * z) for x, y, z in nodes)
    o.stage("densities")
    o.stage("shell")
    sa, sb = o.rho_internal()
    c, _ = oracle_mod.lattice()
    for k, (x, y, z) in enumerate(nodes):
        nb = []
        for i in range(1, 19):
            m = (x + c[i, 0]) % 9 + 9 * (((y + c[i, 1]) % 9) + 9 * ((z + c[i, 2]) % 9))
            if own[m] < 0:
                nb.append(m)
        assert len(nb) == (17 if k < 2 else 18)
        ea, eb = ra[nb].mean(), rb[nb].mean()
        if drho[k] > 0:
            ea += drho[k]
        elif drho[k] < 0:
            eb += -drho[k]
        n = x + 9 * (y + 9 * z)
        assert abs(sa[n] - ea) < 1e-15 and abs(sb[n] - eb) < 1e-15


def _one_particle(oracle_mod, rpar, rperp, q, dens=1.0, dims=(24, 24, 24), pos=(12.0, 12.0, 12.0)):
    o = oracle_mod.Oracle(dims, 1.0, 0.0)
    N = int(np.prod(dims))
    o.init_fields(np.full(N, 0.5), np.full(N, 0.5))
    o.add_ellipsoids(np.array([[rpar, rperp]]), np.array([pos]), np.array([q], float), np.zeros(1),
                     np.array([dens]))
    return o


def test_mass_and_inertia_by_quadrature(oracle_mod):
    """Continuous ellipsoid of density rho_p: M and the principal moments agree
    with a midpoint quadrature of the defining integrals."""
    rpar, rperp, dens = 6.0, 2.5, 1.3
    o = _one_particle(oracle_mod, rpar, rperp, [1, 0, 0, 0], dens)
    e = o.particle_extra(0)
    n = 160
    ax = (np.arange(n) + 0.5) / n * 2 - 1
    X, Y, Z = np.meshgrid(ax * rperp, ax * rperp, ax * rpar, indexing="ij")
    ins = (X ** 2 + Y ** 2) / rperp ** 2 + Z ** 2 / rpar ** 2 <= 1
    dv = (2 * rperp / n) ** 2 * (2 * rpar / n)
    M = dens * ins.sum() * dv
    Ixx = dens * ((Y ** 2 + Z ** 2) * ins).sum() * dv
    Izz = dens * ((X ** 2 + Y ** 2) * ins).sum() * dv
    assert abs(e["M"] / M - 1) < 3e-3
    assert abs(e["Iperp"] / Ixx - 1) < 3e-3
    assert abs(e["Ipar"] / Izz - 1) < 3e-3


def _axis(q):
    w, x, y, z = q
    return np.array([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)])


def _rotate(v, axis, ang):
    a = axis / np.linalg.norm(axis)
    return v * math.cos(ang) + np.cross(a, v) * math.sin(ang) + a * np.dot(a, v) * (1 - math.cos(ang))


def test_free_rotation_rates(oracle_mod):
    """Torque-free spheroid: spinning about the symmetry axis leaves the axis
    fixed and turns the body by |L|/Ipar per step; L perpendicular to the axis
    turns the axis about L by |L|/Iperp per step (closed forms; unit |q|)."""
    rng = np.random.default_rng(9)
    q0 = rng.normal(size=4)
    q0 /= np.linalg.norm(q0)
    o = _one_particle(oracle_mod, 5.0, 3.0, q0)
    e = o.particle_extra(0)
    a0 = _axis(q0)
    w0 = 0.013
    o.set_particle_accum(0, [0, 0, 0], [0, 0, 0])
    o.set_particle_motion(0, V=[0, 0, 0], L=e["Ipar"] * w0 * a0)
    k = 40
    for _ in range(k):
        o.stage("bodies")
    q = o.read_particles()["quat"][0]
    assert abs(np.linalg.norm(q) - 1) < 1e-14
    assert np.abs(_axis(q) - a0).max() < 1e-13
    dq = np.array([q0[0] * q[0] + q0[1:] @ q[1:]])  # cos of half the angle between them
    assert abs(2 * math.acos(min(1.0, abs(dq[0]))) - k * w0) < 1e-11
    # perpendicular: axis precesses rigidly about L
    o2 = _one_particle(oracle_mod, 5.0, 3.0, q0)
    perp = np.cross(a0, [0.3, -0.5, 0.8])
    perp /= np.linalg.norm(perp)
    o2.set_particle_accum(0, [0, 0, 0], [0, 0, 0])
    o2.set_particle_motion(0, V=[0, 0, 0], L=e["Iperp"] * w0 * perp)
    for _ in range(k):
        o2.stage("bodies")
    q2 = o2.read_particles()["quat"][0]
    assert np.abs(_axis(q2) - _rotate(a0, perp, k * w0)).max() < 1e-12


def test_constant_force_and_torque(oracle_mod):
    """Symplectic Euler with dt = 1: constant F gives V_k = k F/M and
    X_k = X_0 + k(k+1)/2 F/M (wrapped into the box); constant torque on a
    sphere gives W_k = k T/I and a total turn of k(k+1)/2 |T|/I about T."""
    o = _one_particle(oracle_mod, 3.0, 3.0, [1, 0, 0, 0], dims=(16, 16, 16), pos=(15.5, 0.25, 8.0))
    e = o.particle_extra(0)
    F = np.array([0.3, -0.2, 0.05])
    T = np.array([0.0, 0.4, 0.3])
    o.set_particle_accum(0, F, T)
    k = 30
    for _ in range(k):
        o.stage("bodies")
    p = o.read_particles()
    assert np.allclose(p["vel"][0], k * F / e["M"], rtol=1e-13, atol=1e-16)
    X = (np.array([15.5, 0.25, 8.0]) + k * (k + 1) / 2 * F / e["M"]) % 16
    assert np.allclose(p["pos"][0], X, rtol=0, atol=1e-12)
    I = e["Iperp"]
    assert abs(e["Iperp"] - e["Ipar"]) < 1e-12 * I
    assert np.allclose(p["omega"][0], k * T / I, rtol=1e-13, atol=1e-16)
    ang = k * (k + 1) / 2 * np.linalg.norm(T) / I
    q = p["quat"][0]
    want = np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * T / np.linalg.norm(T)])
    assert np.abs(q - want).max() < 1e-12


def _moving_particle_system(oracle_mod, g=0.0, noise=0.0):
    dims = (20, 18, 22)
    N = int(np.prod(dims))
    rng = np.random.default_rng(21)
    o = oracle_mod.Oracle(dims, 1.0, g)
    ra = 0.5 + noise * rng.uniform(-1, 1, N)
    rb = 0.4 + noise * rng.uniform(-1, 1, N)
    o.init_fields(ra, rb)
    q = rng.normal(size=4)
    o.add_ellipsoids(np.array([[5.0, 3.0]]), np.array([[9.7, 8.9, 11.2]]), q[None, :], np.array([0.1]))
    e = o.particle_extra(0)
    o.set_particle_motion(0, V=[0.03, -0.02, 0.01], L=[0.3 * e["Iperp"] * 0.01, 0.0, e["Ipar"] * 0.01],
                          W=[0.003, 0.0, 0.01])
    return o


def test_momentum_conserved_with_moving_particle(oracle_mod):
    """g = 0: fluid momentum + M V + pending impulse J is invariant through
    moving bounce-back (Eq. (4)), the exchange force (Eq. (5)) and the
    kill / fill impulses, while the particle crosses lattice nodes."""
    o = _moving_particle_system(oracle_mod, g=0.0, noise=0.01)
    M = o.particle_extra(0)["M"]

    def total():
        s = o.stats()
        return s[2:5] + M * o.read_particles()["vel"][0] + o.particle_extra(0)["J"]

    P0 = total()
    own0 = o.owner().copy()
    changed = 0
    for _ in range(50):
        o.step(1)
        led = o.ledger()
        changed += led["kill"] > 0 or led["fill"] > 0
        assert np.abs(total() - P0).max() <= 1e-12 * M * 0.03
    assert changed > 5 and not np.array_equal(o.owner(), own0)


def test_mass_ledger_with_moving_particle(oracle_mod):
    """Each step the fluid mass changes by exactly the bounce-back sources C
    plus the filled mass minus the killed mass (bookkeeping identity)."""
    o = _moving_particle_system(oracle_mod, g=0.08, noise=0.01)
    for _ in range(40):
        m0 = o.stats()[:2].sum()
        o.step(1)
        m1 = o.stats()[:2].sum()
        led = o.ledger()
        assert abs((m1 - m0) - (led["link_C"] - led["kill"] + led["fill"])) < 1e-13 * m0
    assert abs(o.stats()[5]) > 0


def test_link_sources_cancel_on_uniform_fluid(oracle_mod):
    """For a rigid motion and uniform fluid density the bounce-back sources C
    of Eq. (4) sum to zero: along each lattice line the two boundary links
    point opposite ways and their midpoints differ by a multiple of c_i
    (derived)."""
    o = _moving_particle_system(oracle_mod, g=0.0, noise=0.0)
    o.step(1)
    assert abs(o.ledger()["link_C"]) < 1e-14


def test_rotating_and_translating_sphere_drag_fluid(oracle_mod):
    """Sign of the surface velocity V + W x r in Eq. (4): a sphere spinning
    about +z feels a torque against its spin and drags the adjacent fluid
    along its surface; a translating one feels drag against its motion."""
    dims = (24, 24, 24)
    N = 24 ** 3
    o = oracle_mod.Oracle(dims, 1.0, 0.0)
    o.init_fields(np.full(N, 0.5), np.full(N, 0.5))
    o.add_ellipsoids(np.array([[4.0, 4.0]]), np.array([[12.0, 12.0, 12.0]]), np.array([[1.0, 0, 0, 0]]),
                     np.zeros(1), np.array([50.0]))
    e = o.particle_extra(0)
    o.set_particle_motion(0, V=[0.01, 0, 0], L=[0, 0, e["Ipar"] * 0.01], W=[0, 0, 0.01])
    o.step(3)
    p = o.read_particles()
    assert p["torque"][0][2] < 0 and p["force"][0][0] < 0
    _, _, u, _ = o.read_fields()
    u = u.reshape(24, 24, 24, 3)  # [z][y][x]
    assert u[12, 12, 17, 1] > 0 and u[12, 12, 7, 1] < 0  # +x side moves +y, -x side moves -y
    assert u[12, 12, 17, 0] > 0 and u[12, 12, 7, 0] > 0  # fluid dragged along +x


@pytest.mark.parametrize("plant", [0, 5])
def test_fill_rule_hand_computed(oracle_mod, plant):
    """The fill rule, computed in the test from its statement: a node that a
    moving sphere uncovers gets f_i = f^eq_i(rho_bar^c, u_b) for each
    component, with rho_bar^c the mean of rho^c(t+1) over the node's 18
    neighbours that are fluid both before and after the step, and u_b =
    V + W x r the surface velocity of the particle that owned it, with the
    velocities and centre after the body update (r the minimum-image offset
    from that centre). f^eq and the lattice are pinned by the fluid tests.
    The copy of the oracle with planted mistake 5 (a fill that also averages
    the just-uncovered neighbours) must fail it."""
    dims = (16, 16, 16)
    nx, ny, nz = dims
    N = nx * ny * nz
    rng = np.random.default_rng(31)
    ra = 0.6 + 0.05 * rng.uniform(-1, 1, N)
    rb = 0.5 + 0.05 * rng.uniform(-1, 1, N)
    if plant:
        oracle_mod.build(force=False, plant=plant)
    o = oracle_mod.Oracle(dims, 1.0, 0.0, plant=plant)
    o.init_fields(ra, rb)
    R = 3.2
    o.add_ellipsoids(np.array([[R, R]]), np.array([[8.1, 7.9, 8.2]]), np.array([[1.0, 0.0, 0.0, 0.0]]),
                     np.zeros(1), np.array([1e6]))
    M = o.particle_extra(0)["M"]
    W0 = np.array([0.0, 0.02, 0.06])
    o.set_particle_motion(0, V=[0.45, -0.2, 0.1], L=0.4 * M * R * R * W0, W=W0)
    own0 = o.owner().copy()
    o.step(1)
    own1 = o.owner()
    filled = np.where((own0 == 0) & (own1 == -1))[0]
    assert len(filled) >= 5
    ra1, rb1, _, _ = o.read_fields()
    p = o.read_particles()
    X, V, W = p["pos"][0], p["vel"][0], p["omega"][0]
    c, w = oracle_mod.lattice()
    fa, fb = o.get_pops(0), o.get_pops(1)

    def feq(rho, u):
        cu = c @ u
        return w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))

    L = np.array(dims, float)
    worst = 0.0
    for n in filled:
        xyz = np.array([n % nx, (n // nx) % ny, n // (nx * ny)], float)
        nbrs = [int(((xyz[0] + ci[0]) % nx) + nx * (((xyz[1] + ci[1]) % ny) + ny * ((xyz[2] + ci[2]) % nz)))
                for ci in c[1:]]
        keep = [m for m in nbrs if own0[m] == -1 and own1[m] == -1]
        assert keep, n
        r = xyz - X
        r -= np.round(r / L) * L
        ub = V + np.cross(W, r)
        worst = max(worst, np.abs(fa[:, n] - feq(np.mean(ra1[keep]), ub)).max(),
                    np.abs(fb[:, n] - feq(np.mean(rb1[keep]), ub)).max())
    if plant == 0:
        assert worst <= 1e-14, worst
    else:
        assert worst > 1e-6, worst
