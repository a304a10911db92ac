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


def compare(o, g, dims, radii=None):
    """Relative errors of the GPU state against the oracle's. radii (n x 2,
    R_par, R_perp) sets each particle's rim radius for its spin error."""
    ra, rb, u, own = o.read_fields()
    ga, gb, gu, gown = g.read_fields()
    fl = own == -1
    du = (gu - u)[fl]
    out = {
        "e_rho": max(np.abs(ga - ra).max() / np.abs(ra).max(), np.abs(gb - rb).max() / np.abs(rb).max()),
        # u = sum_i f_i c_i / rho cancels populations of size w_i rho, so its
        # rounding floor is ~eps rho / |j|: velocity errors are measured against
        # max(|u|_max, U_FLOOR) lattice units (L-inf), and against the L2 norm
        # of u floored at U_FLOOR per node (L2); the raw L2 ratio is reported
        "e_u": float(np.abs(du).max() / max(np.abs(u[fl]).max(), U_FLOOR)),
        "e_u_l2": float(np.linalg.norm(du) / max(np.linalg.norm(u[fl]), U_FLOOR * np.sqrt(max(fl.sum(), 1)))),
        "e_u_l2_raw": float(np.linalg.norm(du) / max(np.linalg.norm(u[fl]), 1e-300)),
        "u_max": float(np.abs(u[fl]).max()),
        "owner_equal": bool(np.array_equal(own, gown)),
        "owner_diff": int((own != gown).sum()),
    }
    so, sg = o.stats(), g.stats()
    out["e_mass"] = float(max(abs(sg[0] - so[0]) / so[0], abs(sg[1] - so[1]) / so[1]))
    out["n_fluid_equal"] = bool(so[6] == sg[6])
    # total fluid momentum against the momentum scale mass * max(|u|, U_FLOOR)
    # (it is a sum with cancellations, often near zero), and the mass removed
    # by particles (placement plus killed minus filled) against the fluid mass
    mass = so[0] + so[1]
    out["e_mom"] = float(np.abs(sg[2:5] - so[2:5]).max() / (mass * max(out["u_max"], U_FLOOR)))
    out["e_removed"] = float(abs(sg[5] - so[5]) / mass)
    if o.num_particles():
        po, pg = o.read_particles(), g.read_particles()
        L = np.array(dims, dtype=float)
        dX = _minimg(pg["pos"] - po["pos"], L)
        sgn = np.sign((pg["quat"] * po["quat"]).sum(1, keepdims=True))
        out["e_pos"] = float(np.abs(dX).max())
        out["e_quat"] = float(np.abs(pg["quat"] - sgn * po["quat"]).max())
        # particle velocities are velocities of the flow's boundary: measured
        # like the fluid velocity, against the flow's velocity scale
        # max(|u|_max, |V|_max, |omega R|_max, U_FLOOR), the spin by its rim
        # speed |omega| R (raw ratios reported)
        rim = np.ones((len(po["vel"]), 1)) if radii is None else np.asarray(radii, float).reshape(-1, 2).max(1)[:, None]
        dV, dW = np.abs(pg["vel"] - po["vel"]), np.abs(pg["omega"] - po["omega"]) * rim
        vscale = max(out["u_max"], np.abs(po["vel"]).max(), (np.abs(po["omega"]) * rim).max(), U_FLOOR)
        out["e_vel"] = float(dV.max() / vscale)
        out["e_omega"] = float(dW.max() / vscale)
        out["e_vel_raw"] = float(dV.max() / max(np.abs(po["vel"]).max(), 1e-300))
        out["e_omega_raw"] = float(np.abs(pg["omega"] - po["omega"]).max() / max(np.abs(po["omega"]).max(), 1e-300))
        out["e_force"] = float(np.abs(pg["force"] - po["force"]).max() / max(np.abs(po["force"]).max(), 1e-300))
    return out


def check(res, gate, vel_gate=None, particles=True):
    """Assert the parity gates: densities, velocity (floored L-inf and L2),
    total momentum and removed mass at `gate`; identical owner maps and fluid
    counts; particle centre (lattice units) and orientation at `gate`,
    particle V and spin (floored, see compare) at `vel_gate` (default
    `gate`)."""
    log(f"  parity {res}")
    vg = gate if vel_gate is None else vel_gate
    assert res["owner_equal"] and res["n_fluid_equal"], res
    for k in ("e_rho", "e_u", "e_u_l2", "e_mom", "e_removed"):
        assert res[k] <= gate, (k, res)
    if particles and "e_pos" in res:
        assert res["e_pos"] <= gate and res["e_quat"] <= gate, res
        assert res["e_vel"] <= vg and res["e_omega"] <= vg, res
