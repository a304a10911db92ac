"""Domain growth of a demixing two-component mixture with and without
particles (Sec. 4): the lateral domain size L(t) of Eq. (12) of a random 1:1
mixture at g_br = 0.08, and its arrest by prolate ellipsoids of neutral
wettability at a size that falls with the particle volume concentration C,
as L(C) = a / C + b.

Every step and every L(t) runs in the HIP library (lb_step, lb_domain_size);
this module only chooses the systems, reads L between steps and fits the
line. The particles are R_par = 8, R_perp = 4 (aspect ratio m = 2) with
uniform orientations, colour 0 (Theta = 90 degrees), density 8 and the
particle-particle terms of Eqs. (6)-(9) on.

    python -m paper_1109_3277_amd.coarsening --n 256 --steps 40000 --every 2000 \\
        --conc 0.08 0.12 0.16 0.20 0.24 --spinodal

prints L(t) of each system as it goes and the least-squares fit of
L = a / C + b to the final sizes.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

from . import workloads as W
from .adsorption import fit_line

PARTICLE_DENSITY = 8.0


def history(s, pairs: bool, steps: int, every: int, precision: str = "fp64", log=None, stop_on_unstable=False):
    """L(t) every `every` steps up to `steps`: rows (t, L_x, L_y, L_z, L).
    With stop_on_unstable, a run whose health check fails (lb_step's
    LB_EUNSTABLE) ends there and returns the rows before it."""
    from .binding import LB_EUNSTABLE, LBError, Lattice

    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, precision, max_particles=max(s.n_particles, 2),
                max_radius=max(s.max_radius, 1.0))
    try:
        g.init_fields(s.rho_a, s.rho_b)
        if s.n_particles:
            g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, np.full(s.n_particles, PARTICLE_DENSITY))
            g.set_pair_interactions(pairs)
        out = []
        for t in range(every, steps + 1, every):
            try:
                g.step(every)
            except LBError as e:
                if not (stop_on_unstable and e.code == LB_EUNSTABLE):
                    raise
                if log:
                    log(f"    unstable between t = {t - every} and {t}: {e}")
                break
            d = g.domain_size()
            out.append((t, d[0], d[1], d[2], d[3]))
            if log:
                log(f"    t {t:6d}  L {d[3]:8.3f}")
        return np.array(out)
    finally:
        g.close()


def volume_fraction(s) -> float:
    """Volume fraction of the system's ellipsoids (continuous volumes)."""
    r = np.asarray(s.radii, float).reshape(-1, 2)
    return float((4.0 / 3.0 * np.pi * r[:, 0] * r[:, 1] ** 2).sum() / np.prod(s.dims))


def arrested_sizes(n: int, concentrations, steps: int, every: int, precision: str = "fp64", seed: int = 22,
                   log=None):
    """Final L of a bijel for each requested concentration (the 1:1 mixture
    of the bijel workload with ellipsoids placed up to that volume fraction;
    at high fractions random sequential addition places fewer), keyed by the
    volume fraction actually placed, and the histories."""
    final, hist = {}, {}
    for C in concentrations:
        s = W.bijel_system(n=n, phi=C, seed=seed)
        Ca = volume_fraction(s)
        if log:
            log(f"  C = {C} requested, {Ca:.4f} placed ({s.n_particles} ellipsoids, {n}^3)")
        h = history(s, True, steps, every, precision, log, stop_on_unstable=True)
        if len(h):
            final[Ca], hist[Ca] = float(h[-1, 4]), h
    return final, hist


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--every", type=int, default=2000)
    ap.add_argument("--conc", type=float, nargs="+", default=[0.08, 0.12, 0.16, 0.20, 0.24])
    ap.add_argument("--spinodal", action="store_true", help="also the particle-free mixture")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--seed", type=int, default=22)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    if a.spinodal:
        log(f"  spinodal ({a.n}^3, no particles)")
        history(W.spinodal_system(n=a.n, seed=21), False, a.steps, a.every, a.precision, log, stop_on_unstable=True)
    final, hist = arrested_sizes(a.n, a.conc, a.steps, a.every, a.precision, a.seed, log)
    for C in sorted(final):
        log(f"  final L(C = {C:.4f}) = {final[C]:.3f} at t = {int(hist[C][-1, 0])}")
    if len(final) >= 2:
        Cs = sorted(final)
        fa, fb, res = fit_line([1.0 / C for C in Cs], [final[C] for C in Cs])
        log(f"  L = a / C + b: a = {fa:.3f}, b = {fb:.3f} (largest residual {res:.3f})")
    log(f"  {time.time() - t0:.0f} s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
