"""Short, self-contained GPU run for wrapping in a profiler.

    python paper_1109_3277_amd/profile_run.py --workload bijel --precision fp64 --steps 5

Builds the named synthetic workload, runs `--warmup` untimed and `--steps`
further time steps through the HIP library, then copies `--copy-mib` MiB with
the library's plain streaming kernel (k_copy16). The copy gives the
calibration point for hardware byte counters: its algorithmic traffic is
exactly that many bytes read and written.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="bijel", choices=["bijel", "spinodal", "interface"])
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args()
    import torch

    from paper_1109_3277_amd import workloads as W
    from paper_1109_3277_amd.binding import Lattice, probe_copy

    s = {"bijel": W.bijel_system, "spinodal": W.spinodal_system, "interface": W.interface_system}[a.workload]()
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, a.precision, max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    if s.n_particles:
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.step(a.warmup)
    g.step(a.steps)
    print(f"ran {a.workload} {a.precision}: {a.warmup} + {a.steps} steps, N = {s.N}", flush=True)
    if a.copy_mib:
        n = a.copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        probe_copy(dst, src)
        torch.cuda.synchronize()
        print(f"copied {a.copy_mib} MiB with k_copy16", flush=True)


if __name__ == "__main__":
    main()
