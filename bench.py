"""Benchmark: MLUPS of the full two-component D3Q19 Shan-Chen step with moving
ellipsoids on one MI355X, its HBM roofline fraction, the reduced-precision
forms on the same workload, and the CPU FP64 oracle timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload bijel]

Prints one JSON line. A step is one full time step of the method (densities,
shell fill, Shan-Chen force, BGK collision, streaming with moving bounce-back
and particle force/torque, rigid-body update, re-rasterisation with kill/fill)
over the whole box, inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "MLUPS (2-comp D3Q19+ellipsoids) FP64 vs mixed-prec; % HBM peak GB/s"
STORE = {"fp64": 8, "fp32": 4, "fp16_dev": 2, "bf16_dev": 2}
RHO = {"fp64": 8, "fp32": 4, "fp16_dev": 4, "bf16_dev": 4}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def fused_bytes_per_node(prec: str, solids: bool) -> int:
    """Algorithmic HBM bytes of one fused-kernel node update: the 2 x 19
    populations read and written once, the node's two densities read once, the
    owner code read once when solids exist."""
    s = STORE[prec]
    return 2 * 2 * 19 * s + 2 * RHO[prec] + (4 if solids else 0)


def step_bytes_per_node(prec: str) -> int:
    """Algorithmic bytes of one whole step: populations read and written once
    plus the two densities written and read once (640 B in FP64)."""
    return 2 * 2 * 19 * STORE[prec] + 2 * 2 * RHO[prec]


def make_workload(name: str):
    from paper_1109_3277_amd import workloads as W

    if name == "bijel":
        s = W.bijel_system()
        desc = (f"bijel: 256^3 periodic, two components 50/50 (0.7 +- 0.01 noise), g_br=0.08, tau=1, "
                f"{s.n_particles} prolate ellipsoids Rpar=8 Rperp=4 (volume fraction 0.15), colour 0")
    elif name == "spinodal":
        s = W.spinodal_system()
        desc = "spinodal: 128^3 periodic, two components 0.7 +- 0.01 noise, g_br=0.08, tau=1, no particles"
    elif name == "interface":
        s = W.interface_system()
        desc = "interface: 32x32x64 periodic flat interface, one prolate ellipsoid (8, 4), g_br=0.08, tau=1"
    else:
        raise SystemExit(f"unknown workload {name}")
    return s, desc


def run_gpu(s, prec, steps, warmup, profile=True):
    import torch

    from paper_1109_3277_amd.binding import Lattice

    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, prec, max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    if s.n_particles:
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.step(warmup)
    torch.cuda.synchronize()
    if profile:
        g.profile(True)
    t0 = time.perf_counter()
    g.step_async(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read() if profile else None
    g.profile(False)
    st = g.stats()
    g.step(0)  # health check of the timed steps
    sec = t1 - t0
    out = {"mlups": s.N * steps / sec / 1e6, "ms_per_step": 1e3 * sec / steps, "prof": prof, "stats": st}
    if profile:  # one host readout of rho_a, rho_b, u and the owner map (PCIe-inclusive figure)
        t2 = time.perf_counter()
        g.read_fields()
        out["readout_ms"] = 1e3 * (time.perf_counter() - t2)
    del g
    torch.cuda.empty_cache()
    return out


def roofline_of(s, prec, res, traffic):
    ms, launches = res["prof"]["fused"]
    avg_s = ms / launches / 1e3
    per_launch = fused_bytes_per_node(prec, s.n_particles > 0) * s.N
    achieved = per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_fused",
            "algorithmic_bytes_per_launch": per_launch, "avg_launch_ms": round(ms / launches, 5)}


def measured_traffic(workload: str, prec: str):
    """HBM bytes per fused launch from the committed rocprofv3 PMC summary, if
    it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"fused_{prec}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1109_3277_amd", "csrc", "lbe_fluid.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha256_16") != h:
        return None
    return rec.get("bytes_per_launch")


def run_batch(steps, warmup):
    """The 64-system interface ensemble (FP32 fluid, FP64 particles): batched
    (one launch per phase over all systems, two-step HIP graphs, tuned tile
    shape) against the same systems stepped one after another."""
    import torch

    from paper_1109_3277_amd import workloads as W
    from paper_1109_3277_amd.binding import Batch, Lattice

    systems = W.ensemble_systems()
    n_nodes = sum(s.N for s in systems)
    b = Batch([{"dims": s.dims, "tau": s.tau, "g_br": s.g_br, "psi_kind": s.psi_kind,
                "max_particles": s.n_particles, "max_radius": s.max_radius} for s in systems], "fp32")
    for k, s in enumerate(systems):
        b[k].init_fields(s.rho_a, s.rho_b)
        b[k].add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    bx = b.tune()
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step_async(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.step(0)
    b.close()
    del b
    torch.cuda.empty_cache()
    # one by one: every system on its own handle, all created first
    lone = []
    for s in systems:
        g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp32", max_particles=s.n_particles, max_radius=s.max_radius)
        g.init_fields(s.rho_a, s.rho_b)
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        g.step(warmup)
        lone.append(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in lone:
        g.step_async(steps)
    torch.cuda.synchronize()
    t_lone = time.perf_counter() - t0
    for g in lone:
        g.step(0)
    del lone
    torch.cuda.empty_cache()
    return {"systems": len(systems), "nodes": n_nodes, "steps": steps, "tile_width": bx,
            "mlups_batched": round(n_nodes * steps / t_batch / 1e6, 1),
            "mlups_one_by_one": round(n_nodes * steps / t_lone / 1e6, 1),
            "speedup": round(t_lone / t_batch, 3), "precision": "fp32 fluid, fp64 particles"}


def run_forms512(steps, warmup):
    """The 512^3 domain with 41,802 ellipsoids in each precision form (ms per
    step and MLUPS; errors against FP64 are checked by the test suite)."""
    from paper_1109_3277_amd import workloads as W

    s = W.mixed_system()
    out = {}
    for prec in ("fp64", "fp32", "fp16_dev", "bf16_dev"):
        log(f"timing 512^3 {prec}")
        r = run_gpu(s, prec, steps, warmup, profile=False)
        out[prec] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 3)}
    for prec in out:
        out[prec]["speedup_vs_fp64"] = round(out[prec]["mlups"] / out["fp64"]["mlups"], 3)
    return {"dims": list(s.dims), "n_particles": s.n_particles, "steps": steps, "forms": out}


def cpu_baseline(s, steps):
    import oracle

    o = oracle.Oracle(s.dims, s.tau, s.g_br, s.psi_kind)
    o.init_fields(s.rho_a, s.rho_b)
    if s.n_particles:
        o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    t0 = time.perf_counter()
    o.step(steps)
    sec = time.perf_counter() - t0
    return {"value": round(s.N * steps / sec / 1e6, 3), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"the same {s.dims[0]}x{s.dims[1]}x{s.dims[2]} system with its {s.n_particles} particles, "
                      f"{steps} full time steps (FP64 oracle, OpenMP over z-slabs)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bijel", choices=["bijel", "spinodal", "interface"])
    ap.add_argument("--precision", default="fp64", choices=list(STORE))
    ap.add_argument("--no-forms", action="store_true", help="skip the reduced-precision and pure-fluid runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: the whole periodic box lives on one MI355X and the library "
              f"has no multi-GPU path (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    t = time.perf_counter()
    s, desc = make_workload(args.workload)
    log(f"workload ready in {time.perf_counter() - t:.1f} s: {desc}")

    log(f"timing {args.precision}: warmup {args.warmup}, steps {args.steps}")
    main_res = run_gpu(s, args.precision, args.steps, args.warmup)
    log(f"  {main_res['mlups']:.1f} MLUPS, {main_res['ms_per_step']:.3f} ms/step, phases {main_res['prof']}")
    traffic = measured_traffic(args.workload, args.precision)
    roof = roofline_of(s, args.precision, main_res, traffic)

    forms = {}
    if not args.no_forms:
        for prec in ("fp64", "fp32", "fp16_dev", "bf16_dev"):
            if prec == args.precision:
                r = main_res
            else:
                log(f"timing form {prec}")
                r = run_gpu(s, prec, args.steps, args.warmup)
            forms[prec] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                           "speedup_vs_fp64": None,
                           "fused_roofline_frac": roofline_of(s, prec, r, None)["frac"],
                           "step_alg_gbs": round(r["mlups"] * 1e6 * step_bytes_per_node(prec) / 1e9, 1)}
        for prec in forms:
            forms[prec]["speedup_vs_fp64"] = round(forms[prec]["mlups"] / forms["fp64"]["mlups"], 3)
        if args.workload != "spinodal":
            sp, _ = make_workload("spinodal")
            for prec in ("fp64", "fp32"):
                log(f"timing pure fluid 128^3 {prec}")
                r = run_gpu(sp, prec, args.steps, args.warmup)
                forms[f"spinodal128_{prec}"] = {"mlups": round(r["mlups"], 1),
                                                "fused_roofline_frac": roofline_of(sp, prec, r, None)["frac"]}

    batch = forms512 = None
    if not args.no_forms:
        forms512 = run_forms512(50, 5)
        log(f"  512^3 forms {forms512}")
        log("timing the 64-system batch")
        batch = run_batch(args.steps, args.warmup)
        log(f"  batch {batch}")

    cpu = None
    if not args.no_cpu:
        log(f"timing the CPU oracle ({args.cpu_steps} steps)")
        cpu = cpu_baseline(s, args.cpu_steps)
        log(f"  oracle {cpu}")

    value = main_res["mlups"]
    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(main_res["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16_dev": "f16-storage/f32", "bf16_dev": "bf16-storage/f32"}[
            args.precision],
        "data": "synthetic",
        "config": {"workload": desc, "dims": list(s.dims), "n_nodes": s.N, "n_particles": s.n_particles,
                   "precision": args.precision, "parallelism": "1 GPU, whole box"},
        "roofline": roof,
        "step_hbm_frac_alg": round(value * 1e6 * step_bytes_per_node(args.precision) / 1e9 / HBM_PEAK_GBS, 4),
        "phases_ms_per_step": {k: round(v[0] / max(v[1], 1), 5) for k, v in main_res["prof"].items()},
        "host_readout_ms": round(main_res.get("readout_ms", 0.0), 1),
        "mlups_with_one_readout": round(s.N * args.steps / (1e-3 * (main_res["ms_per_step"] * args.steps +
                                                                     main_res.get("readout_ms", 0.0))) / 1e6, 1),
        "cpu_baseline": cpu,
        "forms": forms,
        "forms_512": forms512,
        "batch": batch,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
