"""Helpers that run one seeded system through the oracle and the HIP library
and measure their differences (used by the GPU parity tests and smoke())."""
from __future__ import annotations

import sys

import numpy as np


U_FLOOR = 1e-3


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_oracle(sysm, steps: int):
    import oracle

    o = oracle.Oracle(sysm.dims, sysm.tau, sysm.g_br, sysm.psi_kind)
    o.init_fields(sysm.rho_a, sysm.rho_b)
    if sysm.n_particles:
        o.add_ellipsoids(sysm.radii, sysm.pos, sysm.quat, sysm.delta_rho, sysm.density)
    o.step(steps)
    return o


def run_gpu(sysm, steps: int, precision: str = "fp64"):
    from paper_1109_3277_amd.binding import Lattice

    g = Lattice(sysm.dims, sysm.tau, sysm.g_br, sysm.psi_kind, precision, max_particles=sysm.n_particles,
                max_radius=sysm.max_radius)
    g.init_fields(sysm.rho_a, sysm.rho_b)
    if sysm.n_particles:
        g.add_ellipsoids(sysm.radii, sysm.pos, sysm.quat, sysm.delta_rho, sysm.density)
    g.step(steps)
    return g


def _minimg(d, L):
    return d - np.round(d / L) * L


def compare(o, g, dims):
    """Relative errors of the GPU state against the oracle's."""
    ra, rb, u, own = o.read_fields()
    ga, gb, gu, gown = g.read_fields()
    fl = own == -1
    out = {
        "e_rho": max(np.abs(ga - ra).max() / np.abs(ra).max(), np.abs(gb - rb).max() / np.abs(rb).max()),
        # u = sum_i f_i c_i / rho cancels populations of size w_i rho, so its
        # rounding floor is ~eps rho / |j|: velocity errors are measured against
        # max(|u|_max, U_FLOOR) lattice units (the raw L2 ratio is reported too)
        "e_u": float(np.abs(gu - u)[fl].max() / max(np.abs(u[fl]).max(), U_FLOOR)),
        "e_u_l2_raw": float(np.linalg.norm((gu - u)[fl]) / max(np.linalg.norm(u[fl]), 1e-300)),
        "u_max": float(np.abs(u[fl]).max()),
        "owner_equal": bool(np.array_equal(own, gown)),
        "owner_diff": int((own != gown).sum()),
    }
    so, sg = o.stats(), g.stats()
    out["e_mass"] = float(max(abs(sg[0] - so[0]) / so[0], abs(sg[1] - so[1]) / so[1]))
    out["n_fluid_equal"] = bool(so[6] == sg[6])
    if o.num_particles():
        po, pg = o.read_particles(), g.read_particles()
        L = np.array(dims, dtype=float)
        dX = _minimg(pg["pos"] - po["pos"], L)
        sgn = np.sign((pg["quat"] * po["quat"]).sum(1, keepdims=True))
        out["e_pos"] = float(np.abs(dX).max())
        out["e_quat"] = float(np.abs(pg["quat"] - sgn * po["quat"]).max())
        out["e_vel"] = float(np.abs(pg["vel"] - po["vel"]).max() / max(np.abs(po["vel"]).max(), 1e-300))
        out["e_omega"] = float(np.abs(pg["omega"] - po["omega"]).max() / max(np.abs(po["omega"]).max(), 1e-300))
        out["e_force"] = float(np.abs(pg["force"] - po["force"]).max() / max(np.abs(po["force"]).max(), 1e-300))
    return out
