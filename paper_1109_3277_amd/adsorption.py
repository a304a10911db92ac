"""Observables of a single particle at a fluid-fluid interface (Sec. 4):
the adsorption trajectory z(t), phi(t) of an ellipsoid, and the equilibrium
height of a coloured sphere, from which the contact angle follows (Sec. 2,
the calibration of Eq. (11)).

Every step runs in the HIP library; this module only reads the particle
state and the density field between steps.

z is the distance of the particle centre from the interface, positive on the
blue side (component B, above the red lamella in these boxes); the interface
level is where rho_A = rho_B, found by linear interpolation along z in the
columns of the box's x-y corner region (farthest from the particle) and
averaged. phi is the angle between the particle's symmetry axis and the
interface normal z, in [0, 90] degrees.

Contact angle: a sphere of radius R whose centre rests at height h above a
flat interface meets it at the angle Theta with cos(Theta) = -h / R, measured
through the red phase: a sphere sitting mostly in the blue phase (h > 0) has
Theta > 90 degrees. The colour Delta rho > 0 drives the sphere into the blue
phase in this method (the shell's extra red density repels the blue fluid,
and the particle feels the fluid only through Eq. (5)), so this convention
gives Theta rising with Delta rho, the sign of the paper's linear fit.
"""
from __future__ import annotations

import math

import numpy as np


def interface_level(rho_a, rho_b, dims, cols=None) -> float:
    """Mean z where rho_A - rho_B changes sign (first crossing from below) in
    the given (x, y) columns (default: a 4 x 4 patch at the box corner)."""
    nx, ny, nz = dims
    d = (np.asarray(rho_a) - np.asarray(rho_b)).reshape(nz, ny, nx)
    if cols is None:
        cols = [(x, y) for x in range(4) for y in range(4)]
    lv = []
    for x, y in cols:
        c = d[:, y, x]
        for z in range(1, nz - 2):
            if c[z] > 0 >= c[z + 1]:
                lv.append(z + c[z] / (c[z] - c[z + 1]))
                break
    return float(np.mean(lv)) if lv else float("nan")


def axis_angle_deg(q) -> float:
    """Angle between the body z axis of unit quaternion q (w, x, y, z) and the
    space z axis, folded into [0, 90] degrees."""
    w, x, y, _ = q
    oz = 1.0 - 2.0 * (x * x + y * y)
    return math.degrees(math.acos(min(1.0, abs(oz))))


def trajectory(lat, steps: int, every: int):
    """Advance lat (a Lattice with one particle) `steps` steps, recording
    (t, z, phi) every `every` steps and at t = 0."""
    out = []
    t = 0
    while True:
        ra, rb, _, _ = lat.read_fields()
        zi = interface_level(ra, rb, lat.dims)
        p = lat.read_particles()
        out.append((t, float(p["pos"][0, 2] - zi), axis_angle_deg(p["quat"][0])))
        if t >= steps:
            break
        n = min(every, steps - t)
        lat.step(n)
        t += n
    return np.array(out)


def sphere_height(lat) -> float:
    """Height of particle 0's centre above the interface (blue side positive)."""
    ra, rb, _, _ = lat.read_fields()
    return float(lat.read_particles()["pos"][0, 2] - interface_level(ra, rb, lat.dims))


def equilibrium_height(lat, steps: int, every: int, tail: int):
    """Advance `steps` steps and return the mean and the standard deviation of
    the sphere height over the last `tail` steps, sampled every `every`."""
    hs = []
    t = 0
    while t < steps:
        n = min(every, steps - t)
        lat.step(n)
        t += n
        if t > steps - tail:
            hs.append(sphere_height(lat))
    hs = np.array(hs)
    return float(hs.mean()), float(hs.std())


def contact_angle_deg(h: float, radius: float) -> float:
    """Theta of a sphere resting at height h (blue side positive) above the
    interface, measured through the red phase: cos(Theta) = -h / R."""
    return math.degrees(math.acos(max(-1.0, min(1.0, -h / radius))))


def fit_line(x, y):
    """Least-squares line y = a x + b: (a, b, largest |residual|)."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    A = np.stack([x, np.ones_like(x)], 1)
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(a), float(b), float(np.abs(A @ np.array([a, b]) - y).max())
