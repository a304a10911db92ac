"""Batched systems (many independent periodic systems, one launch per phase,
steps replayed as a HIP graph) against lone handles and the oracle."""
import numpy as np
import pytest

from paper_1109_3277_amd import workloads as W
from tests.parity_util import check, compare, log, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

FP64_GATE = 1e-12


def _small_ensemble(k):
    """The k smallest systems of the 64-system interface ensemble (uneven
    dims, one tilted ellipsoid each)."""
    ens = W.ensemble_systems()
    ens.sort(key=lambda s: s.N)
    return ens[:k]


def _batch(systems, precision):
    from paper_1109_3277_amd.binding import Batch

    b = Batch([{"dims": s.dims, "tau": s.tau, "g_br": s.g_br, "psi_kind": s.psi_kind,
                "max_particles": s.n_particles, "max_radius": s.max_radius} for s in systems], precision)
    for k, s in enumerate(systems):
        b[k].init_fields(s.rho_a, s.rho_b)
        if s.n_particles:
            b[k].add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    return b


def _same(a, b):
    """Bitwise equality of two handles' fields, owners and particles."""
    fa, fb = a.read_fields(), b.read_fields()
    for x, y in zip(fa, fb):
        if not np.array_equal(x, y):
            return False
    pa, pb = a.read_particles(), b.read_particles()
    return all(np.array_equal(pa[k], pb[k]) for k in pa)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16_dev"])
def test_batch_equals_lone_handles_bitwise(prec):
    """Each system of a batch ends bit for bit where a lone handle ends; the
    two-step graph is replayed several times with reads (eager work and
    synchronisation) between replays, and an odd count takes the direct path."""
    from paper_1109_3277_amd.binding import Lattice

    systems = _small_ensemble(6)
    log(f"case batch bitwise {prec}: dims {[s.dims for s in systems]}")
    b = _batch(systems, prec)
    lone = []
    for s in systems:
        g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, prec, max_particles=s.n_particles, max_radius=s.max_radius)
        g.init_fields(s.rho_a, s.rho_b)
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        lone.append(g)
    done = 0
    for n in (2, 4, 1, 6, 3):
        b.step(n)
        for g in lone:
            g.step(n)
        done += n
        for k in range(len(systems)):
            assert _same(b[k], lone[k]), f"system {k} differs after {done} steps"
    log(f"  {len(systems)} systems equal after {done} steps")


def test_batch_parity_vs_oracle_fp64():
    """Three systems of different sizes, 100 batched steps, against the oracle."""
    systems = _small_ensemble(3)
    b = _batch(systems, "fp64")
    b.step(100)
    for k, s in enumerate(systems):
        o = run_oracle(s, 100)
        res = compare(o, b[k], s.dims, s.radii)
        log(f"  system {k} {s.dims}")
        check(res, FP64_GATE, vel_gate=1e-10)


@pytest.mark.timeout(900)
def test_batch_fp32_vs_oracle_ensemble():
    """Eight systems of the ensemble, batched in its configured form (FP32
    fluid, FP64 particles), 100 steps, against the FP64 oracle at the FP32
    gates: the thinnest disk and the longest rod of the 64, and the six
    smallest of the rest."""
    ens = W.ensemble_systems()
    thin = min(range(len(ens)), key=lambda k: ens[k].radii[0, 0])
    rod = max(range(len(ens)), key=lambda k: ens[k].radii[0, 0])
    rest = sorted((k for k in range(len(ens)) if k not in (thin, rod)), key=lambda k: ens[k].N)[:6]
    pick = [thin, rod] + rest
    systems = [ens[k] for k in pick]
    log(f"case batch fp32 vs oracle: systems {pick}, R_par {[round(float(s.radii[0, 0]), 2) for s in systems]}, "
        f"dims {[s.dims for s in systems]}")
    b = _batch(systems, "fp32")
    b.step(100)
    for k, s in enumerate(systems):
        o = run_oracle(s, 100)
        res = compare(o, b[k], s.dims, s.radii)
        log(f"  system {pick[k]} {s.dims} R {s.radii[0].tolist()}")
        check(res, 1e-5)
        del o


def test_batch_walled_no_particles_keeps_rho_like_lone():
    """A walled system with Psi = 1 - exp(-rho), room for a particle but none
    placed: the batched density pass and wall shell fill must agree on
    whether the stored densities are live, as a lone handle's do (bit for
    bit)."""
    from paper_1109_3277_amd.binding import Batch, Lattice

    dims = (16, 12, 14)
    ra, rb = W.layered_fields(dims, 61)
    nx, ny, nz = dims
    z = np.repeat(np.arange(nz), nx * ny)
    mask = (z == 0) | (z == nz - 1)
    base = _small_ensemble(1)[0]
    plist = [{"dims": dims, "tau": 1.0, "g_br": 0.08, "psi_kind": 1, "max_particles": 1, "max_radius": 4.0},
             {"dims": base.dims, "tau": base.tau, "g_br": base.g_br, "psi_kind": base.psi_kind,
              "max_particles": base.n_particles, "max_radius": base.max_radius}]
    log(f"case batch walled, no particles, dims {dims}")
    b = Batch(plist, "fp64")
    g = Lattice(dims, 1.0, 0.08, 1, "fp64", max_particles=1, max_radius=4.0)
    for h in (b[0], g):
        h.set_static_solid(mask, [0.01, 0.0, 0.0])
        h.init_fields(ra, rb)
    b[1].init_fields(base.rho_a, base.rho_b)
    b[1].add_ellipsoids(base.radii, base.pos, base.quat, base.delta_rho, base.density)
    for n in (1, 4, 3):
        b.step(n)
        g.step(n)
        assert _same(b[0], g)
    o = run_oracle_walls(dims, ra, rb, mask, [0.01, 0.0, 0.0], 8)
    check(compare(o, g, dims), 1e-12, particles=False)


def run_oracle_walls(dims, ra, rb, mask, wall_u, steps):
    import oracle

    N = int(np.prod(dims))
    o = oracle.Oracle(dims, 1.0, 0.08, 1)
    o.set_walls(mask, np.tile(np.asarray(wall_u, float), (N, 1)))
    o.init_fields(ra, rb)
    o.step(steps)
    return o


def test_batch_tune_keeps_state_and_results():
    """The autotuner times both tile shapes without changing the state, and
    the tuned batch still matches lone handles."""
    from paper_1109_3277_amd.binding import Lattice

    systems = _small_ensemble(4)
    b = _batch(systems, "fp32")
    b.step(3)
    before = [b[k].read_fields() for k in range(len(systems))]
    bx = b.tune()
    assert bx in (16, 32, 64)
    for k in range(len(systems)):
        after = b[k].read_fields()
        assert all(np.array_equal(x, y) for x, y in zip(before[k], after))
    b.step(5)
    for k, s in enumerate(systems):
        g = run_gpu(s, 8, "fp32")
        assert _same(b[k], g), f"system {k} differs after tuning (tile width {bx})"


def test_batch_tuner_caches_and_one_graph_per_call():
    """The tuner times every tile candidate once per system shape and
    precision (a second batch of the same systems takes the cached choice),
    and a step call of n steps is one graph launch holding all n steps."""
    systems = _small_ensemble(3)
    a = _batch(systems, "fp32")
    r1 = a.tune_report()
    log(f"  tuner: {r1}")
    assert len(r1["candidates"]) == 3 and all(v > 0 for v in r1["candidates"].values())
    b = _batch(systems, "fp32")
    r2 = b.tune_report()
    assert r2["cached"] and r2["tile_width"] == r1["tile_width"] and r2["candidates"] == r1["candidates"]
    b.step(7)
    steps, nodes = b.last_graph()
    assert steps == 7 and nodes >= 7 * 8, (steps, nodes)


def test_batch_misuse_is_refused():
    from paper_1109_3277_amd.binding import LB_ESTATE, LBError, load_library

    systems = _small_ensemble(2)
    b = _batch(systems, "fp32")
    L = load_library()
    assert L.lb_step(b[0].handle, 1) == LB_ESTATE
    assert L.lb_step_async(b[1].handle, 1) == LB_ESTATE
    assert L.lb_read_fields(b._h, None, None, None, None) == LB_ESTATE
    assert L.lb_batch_size(b._h) == 2
    assert L.lb_batch_size(b[0].handle) < 0
    L.lb_destroy(b[0].handle)  # no-op: owned by the batch
    b.step(2)
    b[0].read_fields()


def test_full_ensemble_64_systems_equals_lone_handles():
    """The full 64-system ensemble (FP32 fluid, FP64 particles), 20 batched
    steps after tuning, against each system run alone."""
    systems = W.ensemble_systems()
    log(f"case ensemble 64: {sum(s.N for s in systems)} nodes")
    b = _batch(systems, "fp32")
    b.tune()
    b.step(20)
    for k, s in enumerate(systems):
        g = run_gpu(s, 20, "fp32")
        assert _same(b[k], g), f"system {k} {s.dims} differs"
        del g


def test_batch_mixed_kinds_equals_lone_handles():
    """A batch mixing a particle-free system, a Psi = rho system and a system
    with several moving particles of both colours matches lone handles bit for
    bit, stats included."""
    from paper_1109_3277_amd.binding import Lattice
    from paper_1109_3277_amd.workloads import System, layered_fields, uniform_fields

    a = W.spinodal_system(dims=(40, 24, 16), seed=21)
    ra, rb = layered_fields((32, 32, 48), 22)
    b = System("psi-rho", (32, 32, 48), 1.0, 0.08, ra, rb, np.array([[6.0, 3.0]]), np.array([[16.0, 16.0, 23.5]]),
               np.array([[0.9, 0.1, 0.3, 0.2]]), np.array([0.2]), np.array([2.0]), psi_kind=0)
    rc, rd = uniform_fields((48, 40, 32), 23, 0.7, 0.7, 0.01)
    c = System("several", (48, 40, 32), 1.0, 0.08, rc, rd, np.array([[5.0, 3.0], [4.0, 4.0], [3.0, 5.0]]),
               np.array([[10.0, 10.0, 10.0], [30.0, 25.0, 16.0], [12.0, 30.0, 24.0]]),
               np.array([[1.0, 0, 0, 0], [0.8, 0.2, -0.1, 0.5], [0.3, 0.9, 0.2, -0.1]]),
               np.array([0.3, -0.3, 0.0]), np.array([1.5, 1.5, 1.5]))
    systems = [a, b, c]
    bt = _batch(systems, "fp64")
    lone = [run_gpu(s, 0, "fp64") for s in systems]
    for n in (3, 2, 5):
        bt.step(n)
        for g in lone:
            g.step(n)
        for k in range(3):
            assert _same(bt[k], lone[k]), f"system {k} differs"
            assert np.array_equal(bt[k].stats(), lone[k].stats())


def test_batch_with_walled_systems_equals_lone_handles():
    """Systems with wall nodes (one moving-wall channel, one resting-wall
    channel with a particle) batched with a plain ensemble system: the batched
    wall shell and the wall-keeping owner clear match lone handles bit for
    bit."""
    from paper_1109_3277_amd.binding import Lattice

    base = _small_ensemble(1)[0]

    def walls(dims):
        nx, ny, nz = dims
        z = np.repeat(np.arange(nz), nx * ny)
        return (z == 0) | (z == nz - 1)

    d1, d2 = (16, 8, 14), (24, 20, 24)
    ra1, rb1 = W.layered_fields(d1, 51)
    ra2, rb2 = W.uniform_fields(d2, 52, 0.7, 0.7, 0.01)
    part = (np.array([[6.0, 3.0]]), np.array([[11.3, 9.6, 8.2]]), np.array([[0.9, 0.2, 0.3, 0.1]]),
            np.array([0.1]), np.array([1.0]))
    specs = [
        dict(dims=d1, ra=ra1, rb=rb1, wall_u=[0.01, 0.0, 0.0], parts=None, accel=None),
        dict(dims=d2, ra=ra2, rb=rb2, wall_u=None, parts=part, accel=[2e-5, 1e-5, 0.0]),
    ]
    log(f"case batch with walls: {[s['dims'] for s in specs]} + {base.dims}")
    from paper_1109_3277_amd.binding import Batch

    plist = [{"dims": s["dims"], "tau": 1.0, "g_br": 0.08, "psi_kind": 1,
              "max_particles": 0 if s["parts"] is None else 1, "max_radius": 6.0} for s in specs]
    plist.append({"dims": base.dims, "tau": base.tau, "g_br": base.g_br, "psi_kind": base.psi_kind,
                  "max_particles": base.n_particles, "max_radius": base.max_radius})
    b = Batch(plist, "fp64")
    lone = []
    for k, s in enumerate(specs):
        g = Lattice(s["dims"], 1.0, 0.08, 1, "fp64", max_particles=plist[k]["max_particles"], max_radius=6.0)
        for h in (b[k], g):
            h.set_static_solid(walls(s["dims"]), s["wall_u"])
            h.init_fields(s["ra"], s["rb"])
            if s["accel"] is not None:
                h.set_body_accel(s["accel"])
            if s["parts"] is not None:
                h.add_ellipsoids(*s["parts"])
        lone.append(g)
    b[2].init_fields(base.rho_a, base.rho_b)
    b[2].add_ellipsoids(base.radii, base.pos, base.quat, base.delta_rho, base.density)
    g = Lattice(base.dims, base.tau, base.g_br, base.psi_kind, "fp64", max_particles=base.n_particles,
                max_radius=base.max_radius)
    g.init_fields(base.rho_a, base.rho_b)
    g.add_ellipsoids(base.radii, base.pos, base.quat, base.delta_rho, base.density)
    lone.append(g)
    b.step(7)
    for g in lone:
        g.step(7)
    for k, g in enumerate(lone):
        assert _same(b[k], g), f"system {k} differs"
    assert np.abs(lone[1].read_particles()["pos"] - part[1]).max() > 0


def test_batch_systems_with_set_motion_and_domain_size_equal_lone_handles():
    """A particle set spinning and moving through lb_set_particle_motion on a
    system handle of a batch, and lb_domain_size called on the systems between
    steps: every system ends bit for bit where a lone handle given the same
    calls ends, and its domain size is bitwise the lone handle's."""
    from paper_1109_3277_amd.binding import Lattice

    systems = _small_ensemble(3)
    b = _batch(systems, "fp64")
    lone = []
    for s in systems:
        g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp64", max_particles=s.n_particles, max_radius=s.max_radius)
        g.init_fields(s.rho_a, s.rho_b)
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        lone.append(g)
    motion = dict(vel=np.array([0.004, -0.002, 0.003]), omega=np.array([0.002, 0.004, -0.003]),
                  angmom=np.array([5.0, 9.0, -7.0]))
    for h in [b[k] for k in range(len(systems))] + lone:
        h.set_particle_motion(0, **motion)
    b.step(20)
    for g in lone:
        g.step(20)
    for k, g in enumerate(lone):
        assert np.array_equal(b[k].domain_size(), g.domain_size()), k
    b.step(15)
    for g in lone:
        g.step(15)
    for k, g in enumerate(lone):
        assert _same(b[k], g), k
        log(f"  system {k} {systems[k].dims}: bitwise equal, L = {g.domain_size()[3]:.4f}")
        g.close()
    b.close()
