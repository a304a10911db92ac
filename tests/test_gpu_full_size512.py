"""The 512^3 headline workload (41,802 ellipsoids, FP64) against the CPU FP64
oracle, at full size and in the launch configuration the benchmark times
(tile kernel in z-runs over 1024 tiles per plane, 1 GB population planes).
The oracle holds about 90 GB of host memory here and takes ~15 s per step on
16 threads, so the comparison covers 5 steps; the 256^3 bijel test covers
100 steps with owner changes."""
import numpy as np
import pytest

from tests.parity_util import check, compare, log

pytestmark = pytest.mark.gpu

STEPS = 5


@pytest.mark.timeout(900)
def test_mixed_512_fp64_against_oracle():
    import oracle
    from paper_1109_3277_amd import workloads as W
    from paper_1109_3277_amd.binding import Lattice

    s = W.mixed_system()
    log(f"case mixed 512^3 np={s.n_particles} steps={STEPS}: oracle (about 90 GB of host memory)")
    o = oracle.Oracle(s.dims, s.tau, s.g_br, s.psi_kind)
    o.init_fields(s.rho_a, s.rho_b)
    o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    for k in range(STEPS):
        o.step(1)
        log(f"  oracle step {k + 1}")
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp64", max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.step(STEPS)
    res = compare(o, g, s.dims, s.radii)
    log(f"  parity {res}")
    check(res, 1e-12, vel_gate=1e-10)
    assert res["e_mass"] <= 1e-12
    g.close()
    o.close()
