"""Short, self-contained GPU run for wrapping in a profiler.

    python paper_1109_3277_amd/profile_run.py --workload bijel --precision fp64 --steps 5

Builds the named synthetic workload, runs `--warmup` untimed and `--steps`
further time steps through the HIP library, then copies `--copy-mib` MiB with
the plain streaming kernel of liblbe_probe.so (k_probe_copy16). The copy gives
the calibration point for hardware byte counters: its algorithmic traffic is
exactly that many bytes read and written.
"""
from __future__ import annotations

import argparse
import ctypes as C
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="bijel", choices=["bijel", "spinodal", "interface", "mixed", "ensemble"])
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--domain-size", type=int, default=0, help="calls of the Eq. (12) domain-size pass afterwards")
    a = ap.parse_args()
    import torch

    from paper_1109_3277_amd import workloads as W
    from paper_1109_3277_amd.binding import Lattice

    if a.workload == "ensemble":
        # the 64-system interface ensemble as one batch (tuned, then stepped)
        from paper_1109_3277_amd.binding import Batch

        systems = W.ensemble_systems()
        g = Batch([{"dims": s.dims, "tau": s.tau, "g_br": s.g_br, "psi_kind": s.psi_kind,
                    "max_particles": s.n_particles, "max_radius": s.max_radius} for s in systems], a.precision)
        for k, s in enumerate(systems):
            g[k].init_fields(s.rho_a, s.rho_b)
            g[k].add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        print(f"tile {g.tune_report()['tile']}", flush=True)
        N = sum(s.N for s in systems)
    else:
        s = {"bijel": W.bijel_system, "spinodal": W.spinodal_system, "interface": W.interface_system,
             "mixed": W.mixed_system}[a.workload]()
        g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, a.precision, max_particles=s.n_particles,
                    max_radius=s.max_radius)
        g.init_fields(s.rho_a, s.rho_b)
        if s.n_particles:
            g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        N = s.N
    g.step(a.warmup)
    g.step(a.steps)
    print(f"ran {a.workload} {a.precision}: {a.warmup} + {a.steps} steps, N = {N}", flush=True)
    for _ in range(a.domain_size):
        print(f"domain size {g.domain_size()[:4].tolist()}", flush=True)
    if a.copy_mib:
        n = a.copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        probe = C.CDLL(os.path.join(ROOT, "paper_1109_3277_amd", "liblbe_probe.so"))
        probe.lbe_probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        rc = probe.lbe_probe_copy(dst.data_ptr(), src.data_ptr(), n, torch.cuda.current_stream().cuda_stream)
        assert rc == 0, rc
        torch.cuda.synchronize()
        print(f"copied {a.copy_mib} MiB with k_probe_copy16", flush=True)


if __name__ == "__main__":
    main()
