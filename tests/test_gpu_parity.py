"""GPU (HIP, through the C ABI) against the CPU FP64 oracle on the same seeded
inputs. Gates: FP64 <= 1e-12 relative after 100 steps (densities L-inf over
max |rho|; velocity L-inf over max(|u|_max, 1e-3) and raw L2; total momentum
and removed mass; see parity_util), owner map identical; FP32 <= 1e-5 on the
same quantities and on the particles; reduced storage <= 1e-3 with the mass
drift reported."""
import math

import numpy as np
import pytest

from paper_1109_3277_amd import workloads as W
from tests.parity_util import check, compare, log, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

FP64_GATE = 1e-12


def _check_fp64(res, particles=True):
    check(res, FP64_GATE, vel_gate=1e-10, particles=particles)
    assert res["e_mass"] <= FP64_GATE, res


FP32_GATE = 1e-5
RED_GATE = 1e-3


def _run(sysm, steps, precision="fp64"):
    log(f"case {sysm.name} dims={sysm.dims} np={sysm.n_particles} steps={steps} precision={precision}")
    o = run_oracle(sysm, steps)
    g = run_gpu(sysm, steps, precision)
    return o, g, compare(o, g, sysm.dims, sysm.radii)


def test_fluid_ragged_tiles_fp64():
    """Box sizes that leave partial tiles in x and y (several tiles, ragged tail)."""
    s = W.spinodal_system(dims=(40, 20, 12), seed=11)
    _, _, res = _run(s, 100)
    _check_fp64(res)


def test_tile_z_runs_ragged_fp64():
    """Planes of 2 x 129 tiles, ragged in x and y: enough tiles per plane that
    the fused kernel takes them in z-runs (x, then z, then y), with particles."""
    s = W.bijel_system(dims=(70, 516, 12), seed=21, phi=0.1, rpar=4.5, rperp=2.5)
    assert s.n_particles > 100
    _, _, res = _run(s, 30)
    _check_fp64(res)


def test_tile_z_runs_fp32():
    s = W.bijel_system(dims=(70, 516, 12), seed=22, phi=0.1, rpar=4.5, rperp=2.5)
    _, _, res = _run(s, 30, "fp32")
    check(res, FP32_GATE)


def test_zero_steps_and_minimum_box():
    s = W.spinodal_system(dims=(3, 3, 3), seed=12)
    o, g, res = _run(s, 0)
    assert res["e_rho"] <= 1e-15
    o.step(20)
    g.step(20)
    _check_fp64(compare(o, g, s.dims, s.radii))


def test_interface_full_size_fp64():
    """32x32x64 flat interface with one prolate ellipsoid, 100 steps (full size)."""
    s = W.interface_system()
    _, _, res = _run(s, 100)
    _check_fp64(res)


def test_interface_colour_and_psi_kind_fp64():
    """Non-zero particle colour (both signs) and Psi = 1 - exp(-rho)."""
    for dr, kind in ((0.2, 0), (-0.25, 1)):
        s = W.interface_system(dims=(24, 24, 40), rpar=5.0, rperp=3.0, delta_rho=dr, seed=13)
        s.psi_kind = kind
        _, _, res = _run(s, 60)
        _check_fp64(res)


def test_spinodal_full_size_fp64():
    """128^3 spinodal mixture, 100 steps (full size)."""
    s = W.spinodal_system()
    _, _, res = _run(s, 100)
    _check_fp64(res)


@pytest.mark.parametrize("prec,gate", [("fp64", 1e-13), ("fp32", FP32_GATE), ("fp16_dev", RED_GATE),
                                       ("bf16_dev", RED_GATE)])
def test_spinodal_mass_over_1000_steps(prec, gate):
    """The 128^3 spinodal for 1000 steps: without particles BGK and streaming
    conserve each component's mass exactly, so the relative change of the
    FP64 mass sums measures only the arithmetic of the form (the deviation
    forms store populations relative to w_i rho_ref and sum them in their
    own precision); the total momentum stays at its initial zero."""
    from paper_1109_3277_amd.binding import Lattice

    s = W.spinodal_system()
    log(f"case spinodal 128^3 {prec}: mass over 1000 steps")
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, prec)
    g.init_fields(s.rho_a, s.rho_b)
    m0 = g.stats()
    g.step(1000)
    m1 = g.stats()
    drift = np.abs((m1[:2] - m0[:2]) / m0[:2]).max()
    mom = np.abs(m1[2:5]).max() / (m1[0] + m1[1])
    log(f"  relative mass change {drift:.3e}, momentum / mass {mom:.3e}, domain size {g.domain_size()[3]:.2f}")
    assert drift <= gate and mom <= gate
    g.close()


def test_bijel_scaled_fp64():
    """64^3 with the bijel recipe (volume fraction 0.15 of (8,4) ellipsoids)."""
    s = W.bijel_system(dims=(64, 64, 64), seed=14)
    assert s.n_particles > 50
    _, _, res = _run(s, 100)
    _check_fp64(res)


def test_bijel_30_70_scaled_fp64():
    s = W.bijel_system(dims=(48, 40, 56), seed=15, ratio="30/70")
    _, _, res = _run(s, 60)
    _check_fp64(res)


def test_moving_particles_cross_nodes_fp64():
    """Particles given a push so they cross lattice nodes (kill / fill)."""
    s = W.bijel_system(dims=(40, 40, 40), seed=16, phi=0.1)
    rng = np.random.default_rng(16)
    u = 0.05 * rng.uniform(-1, 1, (s.N, 3))
    import oracle
    from paper_1109_3277_amd.binding import Lattice

    o = oracle.Oracle(s.dims, s.tau, s.g_br)
    o.init_fields(s.rho_a, s.rho_b, u)
    o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g = Lattice(s.dims, s.tau, s.g_br, max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b, u)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    own0 = o.owner().copy()
    o.step(100)
    g.step(100)
    res = compare(o, g, s.dims, s.radii)
    assert (o.owner() != own0).sum() > 0
    _check_fp64(res)


def test_large_particle_near_half_box_fp64():
    """Bounding radius just below half the shortest side (largest allowed)."""
    from paper_1109_3277_amd.workloads import System, layered_fields

    dims = (16, 18, 32)
    ra, rb = layered_fields(dims, 17)
    s = System("edge", dims, 1.0, 0.08, ra, rb, np.array([[7.95, 3.0]]), np.array([[8.0, 9.0, 15.5]]),
               np.array([[0.9, 0.1, 0.3, 0.2]]), np.array([0.1]), np.array([1.0]))
    _, _, res = _run(s, 50)
    _check_fp64(res)


def test_spinodal_fp32():
    s = W.spinodal_system(dims=(64, 48, 40), seed=18)
    _, _, res = _run(s, 100, "fp32")
    check(res, FP32_GATE)


def test_interface_fp32():
    s = W.interface_system()
    _, _, res = _run(s, 100, "fp32")
    check(res, FP32_GATE)


@pytest.mark.parametrize("prec", ["fp16_dev", "bf16_dev"])
def test_spinodal_reduced_storage(prec):
    s = W.spinodal_system(dims=(64, 48, 40), seed=19)
    o, g, res = _run(s, 100, prec)
    log(f"  {prec} {res}")
    assert res["e_rho"] <= RED_GATE, res


@pytest.mark.parametrize("prec", ["fp16_dev", "bf16_dev"])
def test_bijel_reduced_storage(prec):
    """48^3 with the bijel recipe in deviation storage. The particles move
    under forces from the rounded populations, so their positions differ from
    the oracle's by ~1e-5 nodes, and a node lying that close to a surface may
    be covered on one side only: densities are compared on the nodes fluid in
    both runs, owner maps up to a handful of such nodes."""
    s = W.bijel_system(dims=(48, 48, 48), seed=23)
    assert s.n_particles > 20
    o, g, res = _run(s, 60, prec)
    log(f"  {prec} {res}")
    ra, rb, _, own = o.read_fields()
    ga, gb, _, gown = g.read_fields()
    both = (own == -1) & (gown == -1)
    e_rho = max(np.abs(ga - ra)[both].max() / np.abs(ra).max(), np.abs(gb - rb)[both].max() / np.abs(rb).max())
    log(f"  e_rho on nodes fluid in both: {e_rho:.3e}")
    assert e_rho <= RED_GATE, res
    assert res["owner_diff"] <= 10, res
    assert res["e_pos"] <= 1e-4, res


def test_health_flag_reports_nan():
    from paper_1109_3277_amd.binding import LB_EUNSTABLE, LBError, Lattice

    s = W.spinodal_system(dims=(16, 16, 16), seed=20)
    ra = s.rho_a.copy()
    ra[100] = float("nan")
    g = Lattice(s.dims, 1.0, 0.08)
    g.init_fields(ra, s.rho_b)
    with pytest.raises(LBError) as e:
        g.step(1)
    assert e.value.code == LB_EUNSTABLE
    assert g.stats()[7] == 1.0


def test_checkpoint_roundtrip():
    from paper_1109_3277_amd.binding import Lattice

    s = W.interface_system(dims=(24, 24, 40), rpar=5.0, rperp=3.0, seed=21)

    def fresh():
        g = Lattice(s.dims, s.tau, s.g_br, max_particles=1, max_radius=s.max_radius)
        g.init_fields(s.rho_a, s.rho_b)
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        return g

    a = fresh()
    a.step(30)
    blob = a.save_state()
    a.step(20)
    b = fresh()
    b.load_state(blob)
    b.step(20)
    fa, fb = a.read_fields(), b.read_fields()
    # every reduction has a fixed order, so resuming reproduces the run bit for bit
    for k in range(4):
        assert np.array_equal(fa[k], fb[k])
    pa, pb = a.read_particles(), b.read_particles()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k


def test_checkpoint_save_leaves_run_unchanged():
    """Saving stores the populations in plain form (each value in its node's
    own slot, the values bounced into solid nodes copied out bit for bit); a
    run with a save in the middle matches one without, bit for bit."""
    from paper_1109_3277_amd.binding import Lattice

    s = W.bijel_system(dims=(32, 32, 32), seed=23, phi=0.12)
    log(f"case save-neutral dims={s.dims} np={s.n_particles}")

    def fresh():
        g = Lattice(s.dims, s.tau, s.g_br, max_particles=s.n_particles, max_radius=s.max_radius)
        g.init_fields(s.rho_a, s.rho_b)
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        return g

    a = fresh()
    a.step(25)
    a.save_state()
    a.step(25)
    b = fresh()
    b.step(50)
    fa, fb = a.read_fields(), b.read_fields()
    for k in range(4):
        assert np.array_equal(fa[k], fb[k])
    pa, pb = a.read_particles(), b.read_particles()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k


def test_particles_added_mid_run_fp64():
    """A second set of particles placed after 30 steps, into a lattice whose
    bounced populations sit in solid nodes, against the oracle doing the same."""
    import oracle
    from paper_1109_3277_amd.binding import Lattice

    s = W.bijel_system(dims=(40, 40, 40), seed=29, phi=0.1)
    h = s.n_particles // 2
    log(f"case mid-run placement dims={s.dims} np={h}+{s.n_particles - h}")
    o = oracle.Oracle(s.dims, s.tau, s.g_br)
    g = Lattice(s.dims, s.tau, s.g_br, max_particles=s.n_particles, max_radius=s.max_radius)
    for x in (o, g):
        x.init_fields(s.rho_a, s.rho_b)
        x.add_ellipsoids(s.radii[:h], s.pos[:h], s.quat[:h], s.delta_rho[:h], s.density[:h])
        x.step(30)
        x.add_ellipsoids(s.radii[h:], s.pos[h:], s.quat[h:], s.delta_rho[h:], s.density[h:])
        x.step(30)
    _check_fp64(compare(o, g, s.dims, s.radii))


def test_node_touching_three_particles_fp64():
    """A fluid node whose links end in three different particles (one more
    than the fused kernel keeps in registers), the particles carrying
    different colours."""
    import oracle
    from paper_1109_3277_amd.workloads import System, uniform_fields

    dims = (24, 24, 24)
    ra, rb = uniform_fields(dims, 22, 0.7, 0.7, 0.01)
    pos = np.array([[9.0, 12.0, 12.0], [15.0, 12.0, 12.0], [12.0, 15.0, 12.0]])
    s = System("three", dims, 1.0, 0.08, ra, rb, np.full((3, 2), 2.4), pos, np.tile([1.0, 0, 0, 0], (3, 1)),
               np.array([0.05, -0.05, 0.0]), np.full(3, 10.0))
    o0 = oracle.Oracle(dims, 1.0, 0.08)
    o0.init_fields(ra, rb)
    o0.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    own = o0.owner().reshape(24, 24, 24)
    assert own[12, 12, 12] == -1 and own[12, 12, 11] == 0 and own[12, 12, 13] == 1 and own[12, 13, 12] == 2
    _, _, res = _run(s, 20)
    _check_fp64(res)


def _five_particles():
    """Five small spheres around the node (12, 12, 12), which links to all
    five of them."""
    import oracle
    from paper_1109_3277_amd.workloads import System, uniform_fields

    dims = (24, 24, 24)
    ra, rb = uniform_fields(dims, 23, 0.7, 0.7, 0.01)
    pos = np.array([[9.0, 12.0, 12.0], [15.0, 12.0, 12.0], [12.0, 15.0, 12.0], [12.0, 9.0, 12.0],
                    [12.0, 12.0, 15.0]])
    s = System("five", dims, 1.0, 0.08, ra, rb, np.full((5, 2), 2.4), pos, np.tile([1.0, 0, 0, 0], (5, 1)),
               np.array([0.05, -0.05, 0.0, 0.03, -0.02]), np.full(5, 10.0))
    o0 = oracle.Oracle(dims, 1.0, 0.08)
    o0.init_fields(ra, rb)
    o0.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    own = o0.owner().reshape(24, 24, 24)
    assert own[12, 12, 12] == -1
    assert [own[12, 12, 11], own[12, 12, 13], own[12, 13, 12], own[12, 11, 12], own[13, 12, 12]] == [0, 1, 2, 3, 4]
    return s


def test_node_touching_five_particles_fp64():
    """Particles crowding so that one fluid node links to five of them: the
    third to fifth are handled link by link outside the two register slots
    and must still match the oracle."""
    _, _, res = _run(_five_particles(), 20)
    _check_fp64(res)


@pytest.mark.parametrize("prec", ["fp32", "fp16_dev", "bf16_dev"])
def test_node_touching_five_particles_reduced(prec):
    """The same crowded node in the float forms: FP32 takes the per-lane path
    for the third to fifth particles, the 2-byte forms the deferred one
    (pushed without C, completed after the pushes)."""
    _, _, res = _run(_five_particles(), 20, prec)
    log(f"  {prec} {res}")
    if prec == "fp32":
        check(res, FP32_GATE)
    else:
        assert res["e_rho"] <= RED_GATE and res["owner_equal"], res
        assert res["e_pos"] <= 1e-4 and res["e_quat"] <= 1e-4, res
        assert res["e_vel"] <= 1e-2 and res["e_omega"] <= 1e-2, res


@pytest.mark.parametrize("nx", [64, 128, 256, 512])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16_dev"])
@pytest.mark.parametrize("particles", [False, True])
def test_row_kernel_widths(nx, prec, particles):
    """Box widths whose x-rows fill whole blocks: without particles they run
    the aligned-store row kernel (wave-edge exchange, periodic seam), in FP64
    up to width 128; wider FP64 boxes and boxes with small particles crossing
    wave boundaries and the seam run the tile kernel."""
    from paper_1109_3277_amd.workloads import System, uniform_fields

    dims = (nx, 16, 12)
    ra, rb = uniform_fields(dims, 30 + nx, 0.7, 0.7, 0.01)
    rng = np.random.default_rng(nx)
    k = max(2, nx // 48)
    pos = np.stack([np.linspace(0.5, nx - 0.5, k, endpoint=False) + 1.3, rng.uniform(4, 12, k),
                    rng.uniform(3, 9, k)], 1)
    pos[-1, 0] = nx - 0.6  # straddles the periodic seam in x
    q = rng.normal(size=(k, 4))
    if particles:
        s = System(f"rows{nx}", dims, 1.0, 0.08, ra, rb, np.tile([3.5, 2.0], (k, 1)), pos, q,
                   rng.uniform(-0.1, 0.1, k), np.full(k, 2.0))
    else:
        s = System(f"rows{nx}", dims, 1.0, 0.08, ra, rb)
    o, g, res = _run(s, 40, prec)
    if prec == "fp64":
        _check_fp64(res)
    elif prec == "fp32":
        check(res, FP32_GATE)
    else:
        log(f"  {prec} {res}")
        assert res["e_rho"] <= RED_GATE and res["owner_equal"], res


@pytest.mark.timeout(900)
def test_bijel_full_size_fp64():
    """The full 256^3 bijel workload with its 4694 ellipsoids, 100 steps
    against the oracle (stepped in chunks with a progress line each); the
    particles move far enough for nodes to change owner."""
    import oracle
    from paper_1109_3277_amd.binding import Lattice

    s = W.bijel_system()
    log(f"case bijel 256^3 np={s.n_particles} steps=100 (oracle in chunks of 10)")
    o = oracle.Oracle(s.dims, s.tau, s.g_br, s.psi_kind)
    o.init_fields(s.rho_a, s.rho_b)
    o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    own0 = o.owner().copy()
    for k in range(10):
        o.step(10)
        log(f"  oracle step {10 * (k + 1)}")
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp64", max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.step(100)
    res = compare(o, g, s.dims, s.radii)
    flips = int((o.owner() != own0).sum())
    log(f"  owner changes over 100 steps: {flips}")
    assert flips > 0
    _check_fp64(res)
