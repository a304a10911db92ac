"""Benchmark: MLUPS of the full two-component D3Q19 Shan-Chen step with moving
ellipsoids on one MI355X, the HBM roofline fraction of its dominant kernel,
the reduced-precision forms on the same workload with their errors against
FP64, the smaller workloads, the batched ensemble, and the CPU FP64 oracle
timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mixed]

Prints one JSON line. A step is one full time step of the method (densities,
shell fill, Shan-Chen force, BGK collision, streaming with moving bounce-back
and particle force/torque, rigid-body update, re-rasterisation with kill/fill)
over the whole box, inputs resident in HBM. The headline workload is the
largest single-GPU one: 512^3 with 41,802 ellipsoids in FP64.
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
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16_dev": "f16-storage/f32", "bf16_dev": "bf16-storage/f32"}
PROFILE_STEPS = 20  # event-timed steps for the per-kernel roofline (after the timed region)


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

    if name == "mixed":
        s = W.mixed_system()
        desc = (f"mixed-precision domain: 512^3 periodic, two components 0.7 +- 0.01 noise, g_br=0.08, tau=1, "
                f"{s.n_particles} ellipsoids R_perp=4, aspect U[0.5,2], colour U[-0.3,0.3], volume fraction 0.1, "
                f"particle density 8")
    elif name == "bijel":
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


def _lattice(s, prec, density=None):
    from paper_1109_3277_amd.binding import Lattice

    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, prec, max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    if s.n_particles:
        dens = s.density if density is None else np.full(s.n_particles, float(density))
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, dens)
    return g


def domain_size_bytes_per_node(prec: str) -> int:
    """Algorithmic bytes of one lb_domain_size call per node: the order
    parameter pass reads 2 x 19 populations, the owner code and the bounce mask
    and writes phi (8 B); each of the three line passes reads phi once."""
    return 2 * 19 * STORE[prec] + 4 + 4 + 8 + 3 * 8


def run_domain_size(g, s, prec, calls=5):
    """Eq. (12) on the lattice's current state: `calls` timed lb_domain_size
    calls (each ends with its own synchronisation)."""
    g.domain_size()  # warm-up
    t0 = time.perf_counter()
    for _ in range(calls):
        out = g.domain_size()
    ms = 1e3 * (time.perf_counter() - t0) / calls
    per = domain_size_bytes_per_node(prec) * s.N
    return {"L": [round(float(v), 4) for v in out[:4]], "ms_per_call": round(ms, 3), "calls": calls,
            "algorithmic_bytes_per_call": per, "alg_gbs": round(per / (ms / 1e3) / 1e9, 1),
            "hbm_frac_alg": round(per / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def run_gpu(s, prec, steps, warmup, profile_steps=PROFILE_STEPS, keep_fields=False, analysis=False, pairs=False):
    """Warm-up, then `steps` timed steps with per-kernel profiling off, then
    `profile_steps` steps with HIP events around every launch (per-kernel
    average durations for the roofline); with `analysis`, the domain size of
    Eq. (12) timed on the final state; with `pairs`, the particle-particle
    terms of Eqs. (6)-(9) switched on."""
    import torch

    g = _lattice(s, prec)
    if pairs:
        g.set_pair_interactions(True)
    m0 = g.stats()[:2].copy()
    g.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step_async(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    g.step(0)  # health check of the timed steps
    out = {"mlups": s.N * steps / sec / 1e6, "ms_per_step": 1e3 * sec / steps}
    fields = None
    if keep_fields:  # densities and owner map after warm-up + timed steps
        ra, rb, _, own = g.read_fields()
        fields = (ra, rb, own)
        out["mass_change"] = ((g.stats()[:2] - m0) / m0).tolist()
    if profile_steps:
        g.profile(True)
        g.step_async(profile_steps)
        torch.cuda.synchronize()
        out["prof"] = g.profile_read()
        g.profile(False)
        g.step(0)
    if analysis:
        out["domain_size"] = run_domain_size(g, s, prec)
    g.close()
    del g
    torch.cuda.empty_cache()
    return out, fields


def roofline_of(s, prec, res, traffic):
    ms, launches = res["prof"]["fused"]
    avg_s = ms / launches / 1e3
    per_launch = fused_bytes_per_node(prec, s.n_particles > 0) * s.N
    achieved = per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_fused",
            "algorithmic_bytes_per_launch": per_launch, "avg_launch_ms": round(ms / launches, 5),
            "launches_timed": launches}


def measured_traffic(workload: str, prec: str, kind: str = "fused"):
    """HBM bytes per fused launch from the committed rocprofv3 PMC summary, if
    it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{prec}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1109_3277_amd", "csrc", "lbe_fluid.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha256_16") != h:
        return None
    return rec.get("bytes_per_launch")


def form_errors(ref, fields, s):
    """Densities of a form against FP64 after the same steps, on nodes fluid
    in both runs (RMS and max over max |rho|), owner codes that differ."""
    RA, RB, OWN = ref
    ra, rb, own = fields
    both = (own == -1) & (OWN == -1)
    sc = max(np.abs(RA).max(), np.abs(RB).max())
    d = np.concatenate([(ra - RA)[both], (rb - RB)[both]])
    return {"rho_rms": float(np.sqrt(np.mean(d * d)) / sc), "rho_max": float(np.abs(d).max() / sc),
            "owner_diff": int((own != OWN).sum())}


def heavy_form_errors(s, steps=100):
    """Each reduced form against FP64 after `steps` steps with the particles
    made heavy (density 1e6), so that no owner code differs between the runs:
    element-wise density and velocity errors on the device (densities over
    max |rho|, velocities over max(|u|, 1e-3))."""
    import torch

    def fields(prec):
        g = _lattice(s, prec, density=1e6)
        g.step(steps)
        N = s.N
        f = {"ra": torch.empty(N, dtype=torch.float64, device="cuda"),
             "rb": torch.empty(N, dtype=torch.float64, device="cuda"),
             "u": torch.empty(3 * N, dtype=torch.float64, device="cuda"),
             "own": torch.empty(N, dtype=torch.int32, device="cuda")}
        g.read_fields_dev(f["ra"], f["rb"], f["u"], f["own"])
        torch.cuda.synchronize()
        g.close()
        torch.cuda.empty_cache()
        return f

    ref = fields("fp64")
    out = {}
    for prec in ("fp32", "fp16_dev", "bf16_dev"):
        log(f"heavy-particle comparison {prec}")
        f = fields(prec)
        both = (ref["own"] == -1) & (f["own"] == -1)
        sc = torch.maximum(ref["ra"].abs().max(), ref["rb"].abs().max())
        e_rho = torch.maximum((f["ra"] - ref["ra"])[both].abs().max(), (f["rb"] - ref["rb"])[both].abs().max()) / sc
        b3 = both.repeat_interleave(3)
        umax = max(float(ref["u"][b3].abs().max()), 1e-3)
        out[prec] = {"heavy_steps": steps, "heavy_rho_linf": float(e_rho),
                     "heavy_u_linf": float((f["u"] - ref["u"])[b3].abs().max()) / umax,
                     "heavy_owner_diff": int((f["own"] != ref["own"]).sum())}
        del f
        torch.cuda.empty_cache()
    return out


def run_forms(s, workload, steps, warmup, main_prec, main_res, main_fields):
    forms = {}
    for prec in ("fp64", "fp32", "fp16_dev", "bf16_dev"):
        if prec == main_prec:
            r, fields = main_res, main_fields
        else:
            log(f"timing {workload} {prec}")
            r, fields = run_gpu(s, prec, steps, warmup, keep_fields=main_fields is not None)
        f = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
             "fused_roofline_frac": roofline_of(s, prec, r, None)["frac"],
             "fused_traffic_per_launch": measured_traffic(workload, prec),
             "step_alg_gbs": round(r["mlups"] * 1e6 * step_bytes_per_node(prec) / 1e9, 1)}
        if main_fields is not None and prec != "fp64" and main_prec == "fp64":
            f["vs_fp64_after_steps"] = warmup + steps
            f.update(form_errors(main_fields, fields, s))
            f["mass_drift_vs_fp64"] = [round(a - b, 9) for a, b in zip(r["mass_change"], main_res["mass_change"])]
        forms[prec] = f
        del fields
    for prec in forms:
        forms[prec]["speedup_vs_fp64"] = round(forms[prec]["mlups"] / forms["fp64"]["mlups"], 3)
    if main_prec == "fp64":
        for prec, e in heavy_form_errors(s).items():
            forms[prec].update(e)
    return forms


def run_batch(steps, warmup, lone_steps):
    """The 64-system interface ensemble (FP32 fluid, FP64 particles): `steps`
    steps of every system in one HIP-graph launch after tuning, against the
    same systems stepped one after another; fused-kernel roofline from the
    tuner's timing."""
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
    tune = b.tune_report()
    b.step(warmup)
    b.step(steps)  # records the graph of `steps` steps (untimed first launch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step_async(steps)  # one graph launch: `steps` steps of all 64 systems
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    g_steps, g_nodes = b.last_graph()
    b.step(0)
    b.close()
    del b
    torch.cuda.empty_cache()
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
        g.step_async(lone_steps)
    torch.cuda.synchronize()
    t_lone = time.perf_counter() - t0
    for g in lone:
        g.step(0)
        g.close()
    del lone
    torch.cuda.empty_cache()
    per = fused_bytes_per_node("fp32", True) * n_nodes
    fused_ms = tune["best_ms"]
    mlups_b = n_nodes * steps / t_batch / 1e6
    mlups_l = n_nodes * lone_steps / t_lone / 1e6
    assert g_steps == steps
    return {"systems": len(systems), "nodes": n_nodes, "steps": steps, "graph_launches": 1,
            "kernel_nodes_in_graph": g_nodes,
            "tile": tune["tile"], "tuner_candidates_ms": tune["candidates"], "tuner_cached": tune["cached"],
            "mlups_batched": round(mlups_b, 1), "mlups_one_by_one": round(mlups_l, 1),
            "one_by_one_steps": lone_steps, "speedup": round(mlups_b / mlups_l, 3),
            "precision": "fp32 fluid, fp64 particles",
            "roofline": {"bound": "hbm", "kernel": "k_fused_batch (all systems, one launch)",
                         "achieved": round(per / (fused_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(per / (fused_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic("ensemble", "fp32", "fused_batch"),
                         "algorithmic_bytes_per_launch": per, "avg_launch_ms": round(fused_ms, 5)}}


def host_info():
    model, mem = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return model, mem


def cpu_baseline(steps):
    """The CPU FP64 oracle on a bounded sample of the headline recipe: the
    512^3 recipe (same particle shapes, colours, density and volume fraction)
    on a 256^3 box, timed with all host threads and with one."""
    import oracle

    from paper_1109_3277_amd import workloads as W

    s = W.mixed_system(n=256)
    o = oracle.Oracle(s.dims, s.tau, s.g_br, s.psi_kind)
    o.init_fields(s.rho_a, s.rho_b)
    o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    o.step(steps)
    many = s.N * steps / (time.perf_counter() - t0) / 1e6
    oracle.set_threads(1)
    t0 = time.perf_counter()
    o.step(1)
    one = s.N / (time.perf_counter() - t0) / 1e6
    oracle.set_threads(threads)
    model, mem = host_info()
    return {"value": round(many, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "single_thread_mlups": round(one, 3), "cpu_model": model, "host_mem_gib": mem,
            "host_logical_cpus": os.cpu_count(),
            "sample": f"the 512^3 workload's recipe on a 256^3 box ({s.n_particles} ellipsoids, same shapes, colours, "
                      f"density and volume fraction), {steps} full time steps with {threads} threads and 1 step with "
                      f"1 thread (FP64 oracle, OpenMP over z-slabs)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="mixed", choices=["mixed", "bijel", "spinodal", "interface"])
    ap.add_argument("--precision", default="fp64", choices=list(STORE))
    ap.add_argument("--no-forms", action="store_true", help="skip the other precision forms and workloads")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--batch-steps", type=int, default=2000)
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

    keep = not args.no_forms
    log(f"timing {args.precision}: warmup {args.warmup}, steps {args.steps}, then {PROFILE_STEPS} event-timed steps")
    main_res, main_fields = run_gpu(s, args.precision, args.steps, args.warmup, keep_fields=keep, analysis=True)
    log(f"  {main_res['mlups']:.1f} MLUPS, {main_res['ms_per_step']:.3f} ms/step, phases {main_res['prof']}")
    traffic = measured_traffic(args.workload, args.precision)
    roof = roofline_of(s, args.precision, main_res, traffic)

    forms = other = pairs_on = None
    if not args.no_forms:
        forms = run_forms(s, args.workload, args.steps, args.warmup, args.precision, main_res, main_fields)
        log(f"  forms {forms}")
        del main_fields
        other = {}
        for wl, st in (("bijel", 200), ("spinodal", 200), ("interface", 500)):
            if wl == args.workload:
                continue
            w, wdesc = make_workload(wl)
            blk = {"workload": wdesc, "dims": list(w.dims), "n_particles": w.n_particles, "steps": st}
            for prec in {"bijel": ("fp64", "fp32", "fp16_dev"), "spinodal": ("fp64", "fp32"),
                         "interface": ("fp64",)}[wl]:
                log(f"timing {wl} {prec}")
                r, _ = run_gpu(w, prec, st, 10)
                blk[prec] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                             "fused_roofline_frac": roofline_of(w, prec, r, None)["frac"],
                             "traffic_per_fused_launch": measured_traffic(wl, prec),
                             "phases_ms_per_step": {k: round(v[0] / max(v[1], 1), 5) for k, v in r["prof"].items()}}
            other[wl] = blk
            log(f"  {wl} {blk}")
        # the same workload with the particle-particle terms on (the pair
        # kernels are timed with the link forces, in the "forces" phase)
        log(f"timing {args.workload} {args.precision} with the pair terms on")
        r, _ = run_gpu(s, args.precision, 100, args.warmup, pairs=True)
        pairs_on = {"steps": 100, "mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                    "phases_ms_per_step": {k: round(v[0] / max(v[1], 1), 5) for k, v in r["prof"].items()}}
        log(f"  pair terms on {pairs_on}")

    batch = None
    if not args.no_batch:
        log(f"timing the 64-system batch ({args.batch_steps} steps in one graph launch)")
        batch = run_batch(args.batch_steps, args.warmup, 200)
        log(f"  batch {batch}")

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle")
        cpu = cpu_baseline(args.cpu_steps)
        log(f"  oracle {cpu}")

    value = main_res["mlups"]
    if cpu is not None:  # the GPU's rate over the oracle's, per thread count
        cpu["gpu_over_oracle_all_threads"] = round(value / cpu["value"], 1)
        cpu["gpu_over_oracle_one_thread"] = round(value / cpu["single_thread_mlups"], 1)
    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(main_res["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": desc, "dims": list(s.dims), "n_nodes": s.N, "n_particles": s.n_particles,
                   "precision": args.precision, "parallelism": "1 GPU, whole box"},
        "roofline": roof,
        "step_hbm_frac_alg": round(value * 1e6 * step_bytes_per_node(args.precision) / 1e9 / HBM_PEAK_GBS, 4),
        "phases_ms_per_step": {k: round(v[0] / max(v[1], 1), 5) for k, v in main_res["prof"].items()},
        "domain_size": main_res["domain_size"],
        "cpu_baseline": cpu,
        "forms": forms,
        "other_workloads": other,
        "pair_terms_on": pairs_on,
        "batch": batch,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
