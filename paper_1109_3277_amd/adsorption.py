"""Observables of a single particle at a fluid-fluid interface (Sec. 4):
the adsorption trajectory z(t), phi(t) of an ellipsoid, and the equilibrium
height of a coloured sphere, from which the contact angle follows (Eq. (11)).

Every step runs in the HIP library; this module only reads the particle
state and the density field between steps.

z is the distance of the particle centre from the interface, positive on the
blue side; the interface level is where rho_A = rho_B, found by linear
interpolation along z in the columns of the box's x-y corner region (farthest
from the particle) and averaged. phi is the angle between the particle's
symmetry axis and the interface normal z, in [0, 90] degrees.
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
