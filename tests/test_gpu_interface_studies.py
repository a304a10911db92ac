"""A single particle at a flat fluid-fluid interface between walls (Sec. 4):
the adsorption of a prolate ellipsoid (Fig. 3: approach without turning,
then reorientation to phi = 90 degrees at the interface) and the contact
angle of coloured spheres against their colour (the linear calibration of
Eq. (11)). Both run on the HIP path; the first 100 steps of each box are
checked against the oracle at the FP64 gates."""
import numpy as np
import pytest

from paper_1109_3277_amd import workloads as W
from paper_1109_3277_amd.adsorption import (contact_angle_deg, equilibrium_height, fit_line, trajectory)
from tests.parity_util import check, compare, log

pytestmark = pytest.mark.gpu


def _walled(s, precision="fp64"):
    from paper_1109_3277_amd.binding import Lattice

    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, precision, max_particles=1, max_radius=s.max_radius)
    g.set_static_solid(W.wall_mask(s.dims))
    g.init_fields(s.rho_a, s.rho_b)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    return g


def _walled_oracle(s):
    import oracle

    o = oracle.Oracle(s.dims, s.tau, s.g_br, s.psi_kind)
    o.set_walls(W.wall_mask(s.dims))
    o.init_fields(s.rho_a, s.rho_b)
    o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    return o


@pytest.mark.parametrize("name,make", [
    ("adsorption", lambda: W.adsorption_system()),
    ("contact+0.08", lambda: W.contact_system(0.08)),
], ids=["adsorption", "contact+0.08"])
def test_interface_boxes_match_oracle_fp64(name, make):
    s = make()
    log(f"case {name} dims={s.dims} walls z=0,{s.dims[2] - 1} steps=100")
    o, g = _walled_oracle(s), _walled(s)
    o.step(100)
    g.step(100)
    res = compare(o, g, s.dims, s.radii)
    log(f"  parity {res}")
    check(res, 1e-12, vel_gate=1e-10)
    g.close()


def test_adsorption_trajectory():
    """64^3 between walls, R_p = 12, R_o = 6, Theta = 90 degrees, starting
    0.0057 degrees from the interface normal in the red lamella, its tip three
    nodes below the interface. The particle first moves to the interface
    without turning, then turns to lie in it (phi -> 90 degrees) with its
    centre at the interface, where it stays."""
    s = W.adsorption_system()
    g = _walled(s)
    tr = trajectory(g, 8000, 250)
    g.close()
    for t, z, phi in tr:
        log(f"  t {int(t):5d}  z {z:8.3f}  phi {phi:8.4f}")
    t, z, phi = tr[:, 0], tr[:, 1], tr[:, 2]
    approach = t <= 1500
    assert z[approach][-1] > z[0] + 2.0  # moved towards the interface
    assert phi[approach].max() < 0.1  # without turning
    assert phi[z < -10.0].max() < 1.0  # no turn before contact
    late = t >= 6000
    assert np.abs(z[late]).max() < 0.5 and phi[late].min() > 89.0  # adsorbed, lying in the interface
    turn = t[np.argmax(phi > 45.0)]
    log(f"  phi passes 45 degrees at t = {int(turn)}")
    assert 2000 <= turn <= 6500


def test_adsorption_from_a_large_tilt():
    """Started at phi = 45 degrees the particle also ends lying in the
    interface (the stable point of Fig. 3(b))."""
    s = W.adsorption_system(phi0_deg=45.0)
    g = _walled(s)
    tr = trajectory(g, 8000, 500)
    g.close()
    for t, z, phi in tr:
        log(f"  t {int(t):5d}  z {z:8.3f}  phi {phi:8.4f}")
    assert abs(tr[-1, 1]) < 0.5 and tr[-1, 2] > 89.0


def test_contact_angle_is_linear_in_colour():
    """Spheres (R = 8) of colour Delta rho at the interface of a 48^3 walled
    box: the equilibrium height gives Theta (cos Theta = -h / R, through the
    red phase). Theta(0) = 90 degrees by symmetry, Theta(-d) = 180 - Theta(d),
    Theta rises with Delta rho, and is linear in it, as the paper's fit
    Theta = 243.2 Delta rho + 90 (whose slope it calls parameter-dependent)."""
    colours = [-0.08, -0.04, 0.0, 0.04, 0.08]
    thetas = []
    for dr in colours:
        s = W.contact_system(dr)
        g = _walled(s)
        h, sd = equilibrium_height(g, 16000, 200, 8000)
        g.close()
        th = contact_angle_deg(h, s.radii[0, 0])
        log(f"  delta_rho {dr:+.2f}: h {h:8.4f} (std {sd:.4f}), Theta {th:7.2f} deg")
        thetas.append(th)
    th = np.array(thetas)
    a, b, res = fit_line(colours, th)
    log(f"  fit Theta = {a:.1f} deg * delta_rho + {b:.2f} deg, largest residual {res:.2f} deg (paper: 243.2, 90)")
    assert abs(th[2] - 90.0) < 0.5
    assert np.abs(th + th[::-1] - 180.0).max() < 1.0
    assert np.all(np.diff(th) > 0)
    assert abs(b - 90.0) < 0.5 and a > 0 and res < 2.0
