"""Host-side helpers of the interface and domain-growth studies (Sec. 4 and
Eq. (11)), checked against closed forms: the interface level of a density
profile, the tilt angle of a body axis, the contact angle of a sphere from its
height, the straight-line fit, and the volume fraction of placed ellipsoids."""
import math

import numpy as np

from paper_1109_3277_amd.adsorption import axis_angle_deg, contact_angle_deg, fit_line, interface_level
from paper_1109_3277_amd.coarsening import volume_fraction
from paper_1109_3277_amd.workloads import System, uniform_fields


def test_interface_level_of_a_linear_crossing():
    """rho_A - rho_B linear in z with its zero at z0 (between nodes) in every
    column: the level is z0 exactly (linear interpolation)."""
    dims = (8, 6, 20)
    nx, ny, nz = dims
    z0 = 11.37
    z = np.repeat(np.arange(nz, dtype=float), nx * ny)
    d = -0.05 * (z - z0)  # A-rich below, B-rich above
    ra = 0.7 + 0.5 * d
    rb = 0.7 - 0.5 * d
    assert abs(interface_level(ra, rb, dims) - z0) < 1e-12


def test_axis_angle_of_rotations_about_x():
    for deg in (0.0, 0.0057, 30.0, 45.0, 89.0, 90.0, 135.0, 180.0):
        h = math.radians(deg) / 2.0
        q = (math.cos(h), math.sin(h), 0.0, 0.0)
        want = deg if deg <= 90.0 else 180.0 - deg
        assert abs(axis_angle_deg(q) - want) < 1e-6, deg


def test_contact_angle_closed_forms():
    R = 8.0
    assert abs(contact_angle_deg(0.0, R) - 90.0) < 1e-12
    assert abs(contact_angle_deg(-R / 2, R) - 60.0) < 1e-12
    assert abs(contact_angle_deg(R / 2, R) - 120.0) < 1e-12
    assert abs(contact_angle_deg(2 * R, R) - 180.0) < 1e-12  # clamped: fully in the blue phase
    for h in (-3.1, 0.7, 5.2):  # Theta(h) + Theta(-h) = 180
        assert abs(contact_angle_deg(h, R) + contact_angle_deg(-h, R) - 180.0) < 1e-12


def test_fit_line_recovers_an_exact_line():
    x = np.array([1 / 0.08, 1 / 0.12, 1 / 0.16, 1 / 0.2, 1 / 0.24])
    a, b, res = fit_line(x, 2.2 * x + 11.08)
    assert abs(a - 2.2) < 1e-12 and abs(b - 11.08) < 1e-10 and res < 1e-10


def test_volume_fraction_of_placed_ellipsoids():
    dims = (64, 64, 64)
    ra, rb = uniform_fields(dims, 1, 0.7, 0.7, 0.0)
    radii = np.array([[8.0, 4.0], [2.0, 4.0], [6.0, 6.0]])
    s = System("vf", dims, 1.0, 0.08, ra, rb, radii, np.zeros((3, 3)), np.tile([1.0, 0, 0, 0], (3, 1)),
               np.zeros(3), np.ones(3))
    want = 4.0 / 3.0 * math.pi * (8 * 16 + 2 * 16 + 6 * 36) / 64 ** 3
    assert abs(volume_fraction(s) - want) < 1e-15
