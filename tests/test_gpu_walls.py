"""Static solid (wall) nodes on the GPU against the CPU FP64 oracle: links into
wall nodes take the moving bounce-back of Eq. (4) with the wall velocity, and
wall nodes next to fluid take the mean density of their fluid neighbours
(Eq. (10), colour 0). Channels with walls on the two z faces; the closed forms
of these flows (Couette, Poiseuille) pin the oracle in test_oracle_fluid."""
import numpy as np
import pytest

from paper_1109_3277_amd import workloads as W
from tests.parity_util import check, compare, log

pytestmark = pytest.mark.gpu


def _walls(dims):
    nx, ny, nz = dims
    z = np.repeat(np.arange(nz), nx * ny)
    return (z == 0) | (z == nz - 1)


def _pair(dims, tau, g, ra, rb, mask, wall_u=None, accel=None, precision="fp64", particles=None, max_radius=0.0):
    import oracle
    from paper_1109_3277_amd.binding import Lattice

    N = int(np.prod(dims))
    o = oracle.Oracle(dims, tau, g)
    o.set_walls(mask, None if wall_u is None else np.tile(np.asarray(wall_u, float), (N, 1)))
    o.init_fields(ra, rb)
    npart = 0 if particles is None else len(particles["pos"])
    gl = Lattice(dims, tau, g, 1, precision, max_particles=npart, max_radius=max_radius)
    gl.set_static_solid(mask, wall_u)
    gl.init_fields(ra, rb)
    for x in (o, gl):
        if accel is not None:
            x.set_body_accel(accel) if x is gl else x.set_accel(accel)
        if particles is not None:
            x.add_ellipsoids(particles["radii"], particles["pos"], particles["quat"], particles["drho"],
                             particles["density"])
    return o, gl


def _check(res, gate):
    check(res, gate, vel_gate=1e-10 if gate < 1e-10 else gate)


def test_poiseuille_resting_walls_fp64():
    """Body force between resting walls, two components, 300 steps."""
    dims = (8, 8, 16)
    N = int(np.prod(dims))
    log(f"case poiseuille dims={dims}")
    ra, rb = np.full(N, 0.6), np.full(N, 0.4)
    o, g = _pair(dims, 0.9, 0.08, ra, rb, _walls(dims), accel=[1e-6, 0.0, 0.0])
    o.step(300)
    g.step(300)
    _check(compare(o, g, dims), 1e-12)


def test_moving_walls_fp64():
    """Both walls moving along x and y (moving bounce-back, Eq. (4)) over a
    layered two-phase fluid, 300 steps."""
    dims = (8, 6, 14)
    ra, rb = W.layered_fields(dims, 31)
    log(f"case moving walls dims={dims}")
    o, g = _pair(dims, 1.0, 0.08, ra, rb, _walls(dims), wall_u=[0.01, -0.004, 0.0])
    o.step(300)
    g.step(300)
    _check(compare(o, g, dims), 1e-12)


def test_walls_with_particle_fp64():
    """A driven ellipsoid moving between resting walls (kill / fill, shell
    fill of particle and wall nodes side by side), 120 steps."""
    dims = (24, 20, 24)
    N = int(np.prod(dims))
    ra, rb = W.uniform_fields(dims, 41, 0.7, 0.7, 0.01)
    parts = {"radii": np.array([[6.0, 3.0]]), "pos": np.array([[11.3, 9.6, 8.2]]),
             "quat": np.array([[0.9, 0.2, 0.3, 0.1]]), "drho": np.array([0.1]), "density": np.array([1.0])}
    log(f"case walls + particle dims={dims}")
    o, g = _pair(dims, 1.0, 0.08, ra, rb, _walls(dims), accel=[2e-5, 1e-5, 0.0], particles=parts, max_radius=6.0)
    o.step(120)
    g.step(120)
    res = compare(o, g, dims, parts["radii"])
    _check(res, 1e-12)
    assert res["e_pos"] <= 1e-12 and res["e_vel"] <= 1e-10, res
    assert np.abs(g.read_particles()["pos"] - parts["pos"]).max() > 0


def test_moving_walls_fp32():
    dims = (16, 8, 12)
    ra, rb = W.layered_fields(dims, 37)
    log(f"case moving walls fp32 dims={dims}")
    o, g = _pair(dims, 1.0, 0.08, ra, rb, _walls(dims), wall_u=[0.02, 0.0, 0.0], precision="fp32")
    o.step(200)
    g.step(200)
    _check(compare(o, g, dims), 1e-5)


def test_static_solid_call_order():
    from paper_1109_3277_amd.binding import LB_ESTATE, LBError, Lattice

    dims = (8, 8, 8)
    g = Lattice(dims, 1.0, 0.08)
    g.init_fields(np.full(512, 0.5), np.full(512, 0.5))
    with pytest.raises(LBError) as e:
        g.set_static_solid(_walls(dims))
    assert e.value.code == LB_ESTATE
