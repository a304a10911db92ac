"""A long ellipsoid spun up through lb_set_particle_motion (Sec. 2: rigid-body
state V, omega, L) against the CPU FP64 oracle given the same motion. The
body is heavy (density 60), so the fluid slows its spin over a few hundred
steps only. Its tips sweep about 0.13 node per step, so nodes change owner by
the rotation alone and kill / fill must cover the ellipsoid's box before and
after each turn; the bounce-back of Eq. (4) carries the W x r term at every
link."""
import numpy as np
import pytest

from paper_1109_3277_amd import workloads as W
from tests.parity_util import check, compare, log

pytestmark = pytest.mark.gpu


def _rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _spinning_rod(precision):
    import oracle
    from paper_1109_3277_amd.binding import Lattice

    dims = (36, 32, 34)
    ra, rb = W.uniform_fields(dims, 43, 0.7, 0.7, 0.01)
    rpar, rperp, dens = 9.0, 2.5, 60.0
    radii, pos = np.array([[rpar, rperp]]), np.array([[17.3, 15.6, 16.9]])
    quat = np.array([[0.8, 0.3, -0.4, 0.3]])
    quat /= np.linalg.norm(quat)
    # body inertia diag(I_perp, I_perp, I_par); L = R I R^T omega
    M = dens * 4.0 / 3.0 * np.pi * rpar * rperp ** 2
    I = np.diag([M * (rperp ** 2 + rpar ** 2) / 5.0] * 2 + [M * 2.0 * rperp ** 2 / 5.0])
    R = _rot(quat[0])
    omega = np.array([0.006, 0.012, -0.007])
    L = R @ I @ R.T @ omega
    vel = np.array([0.01, -0.006, 0.004])
    o = oracle.Oracle(dims, 1.0, 0.08, 1)
    o.init_fields(ra, rb)
    o.add_ellipsoids(radii, pos, quat, np.array([0.05]), np.array([dens]))
    o.set_particle_motion(0, V=vel, L=L, W=omega)
    g = Lattice(dims, 1.0, 0.08, 1, precision, max_particles=1, max_radius=rpar)
    g.init_fields(ra, rb)
    g.add_ellipsoids(radii, pos, quat, np.array([0.05]), np.array([dens]))
    g.set_particle_motion(0, vel=vel, omega=omega, angmom=L)
    return dims, radii, o, g


@pytest.mark.parametrize("precision,gate", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_spinning_rod_matches_oracle(precision, gate):
    dims, radii, o, g = _spinning_rod(precision)
    q0 = g.read_particles()["quat"][0].copy()
    own0 = g.read_fields()[3]
    log(f"case spinning rod {precision} dims={dims} R=(9, 2.5) |omega|=0.0151 steps=150")
    o.step(150)
    g.step(150)
    res = compare(o, g, dims, radii)
    log(f"  parity {res}")
    check(res, gate, vel_gate=1e-10 if gate < 1e-10 else gate)
    p = g.read_particles()
    turned = 2.0 * np.degrees(np.arccos(min(1.0, abs(float(np.dot(p["quat"][0], q0))))))
    flips = int((g.read_fields()[3] != own0).sum())
    log(f"  turned {turned:.1f} degrees, {flips} nodes changed owner")
    assert turned > 60.0 and flips > 150  # the oracle: 79 degrees, 214 nodes
    g.close()


def test_set_particle_motion_validates():
    from paper_1109_3277_amd.binding import LB_EINVAL, LBError

    dims, radii, o, g = _spinning_rod("fp64")
    before = g.read_particles()
    for bad in (dict(k=1, vel=np.zeros(3)), dict(k=-1, vel=np.zeros(3)), dict(k=0, omega=np.array([0.0, np.nan, 0.0]))):
        k = bad.pop("k")
        with pytest.raises(LBError) as e:
            g.set_particle_motion(k, **bad)
        assert e.value.code == LB_EINVAL
    after = g.read_particles()
    for key in ("vel", "omega"):
        assert np.array_equal(before[key], after[key])
    g.set_particle_motion(0, vel=np.array([0.0, 0.0, 0.02]))
    p = g.read_particles()
    assert np.array_equal(p["vel"][0], [0.0, 0.0, 0.02]) and np.array_equal(p["omega"], before["omega"])
    g.close()


def test_add_ellipsoids_rejects_bad_geometry():
    """lb_add_ellipsoids refuses, with LB_EGEOM and nothing placed, a radius
    that is not positive, a bounding radius of half the box or more, and one
    above the handle's max_radius; a zero quaternion is LB_EINVAL."""
    from paper_1109_3277_amd.binding import LB_EGEOM, LB_EINVAL, LBError, Lattice

    dims = (16, 16, 20)
    ra, rb = W.uniform_fields(dims, 5, 0.7, 0.7, 0.01)
    g = Lattice(dims, 1.0, 0.08, 1, "fp64", max_particles=4, max_radius=7.5)
    g.init_fields(ra, rb)
    pos, q = np.array([[8.0, 8.0, 10.0]]), np.array([[1.0, 0.0, 0.0, 0.0]])
    for radii, quat, code in (([[0.0, 2.0]], q, LB_EGEOM), ([[3.0, -1.0]], q, LB_EGEOM),
                              ([[8.0, 2.0]], q, LB_EGEOM), ([[2.0, 7.8]], q, LB_EGEOM),
                              ([[3.0, 2.0]], np.zeros((1, 4)), LB_EINVAL)):
        with pytest.raises(LBError) as e:
            g.add_ellipsoids(np.array(radii), pos, quat)
        assert e.value.code == code, (radii, e.value)
    assert g.num_particles() == 0
    g.add_ellipsoids(np.array([[3.0, 2.0]]), pos, q)
    assert g.num_particles() == 1
    g.step(2)
    g.close()
