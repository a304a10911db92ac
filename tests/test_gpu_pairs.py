"""Particle-particle interactions (Sec. 2, Eqs. (6)-(9): Hertz repulsion with
the Berne-Pechukas extension to ellipsoids, and lubrication) on the GPU, with
its device cell list, against the oracle's all-pairs loop at the FP64
gates."""
import numpy as np
import pytest

from paper_1109_3277_amd.workloads import System, uniform_fields
from tests.parity_util import check, compare, log

pytestmark = pytest.mark.gpu


def _tilted(rng, n, amp):
    """Unit quaternions of small random tilts of the body z axis."""
    v = amp * rng.uniform(-1, 1, (n, 3))
    q = np.concatenate([np.ones((n, 1)), 0.5 * v], 1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _dense_contacts(seed=31):
    """64^3 box with 8 x 4 x 4 prolate ellipsoids (8, 4), axes near z: in x
    side by side 7.95 apart (Hertz range 2 R_o = 8) and in z end to end 15.95
    apart (range 2 R_p = 16), so neighbours overlap slightly or sit inside
    the lubrication range, including across both periodic seams; small random
    tilts make every pair general."""
    rng = np.random.default_rng(seed)
    dims = (64, 64, 64)
    ra, rb = uniform_fields(dims, seed, 0.7, 0.7, 0.01)
    pos = np.array([[4.0 + 7.95 * ix, 8.0 + 16.0 * iy, 8.0 + 15.95 * iz]
                    for iz in range(4) for iy in range(4) for ix in range(8)])
    pos += rng.uniform(-0.02, 0.02, pos.shape)
    n = len(pos)
    return System("dense-pairs", dims, 1.0, 0.08, ra, rb, np.tile([8.0, 4.0], (n, 1)), pos, _tilted(rng, n, 0.06),
                  rng.uniform(-0.1, 0.1, n), np.full(n, 10.0))


def _run(s, steps, u_amp=0.02, seed=7, precision="fp64"):
    import oracle
    from paper_1109_3277_amd.binding import Lattice

    u = u_amp * np.random.default_rng(seed).uniform(-1, 1, (s.N, 3))
    o = oracle.Oracle(s.dims, s.tau, s.g_br, s.psi_kind)
    o.init_fields(s.rho_a, s.rho_b, u)
    o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    o.set_pairs(True, 100.0, 2.0 / 3.0)
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, precision, max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b, u)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.set_pair_interactions(True, 100.0, 2.0 / 3.0)
    # pairs in Hertz contact at the start, by the oracle's own energy
    contacts = sum(o.pair_hertz(i, j)[0] > 0 for i in range(s.n_particles) for j in range(i + 1, s.n_particles))
    log(f"case {s.name} dims={s.dims} np={s.n_particles} steps={steps}: {contacts} pairs in Hertz contact")
    o.step(steps)
    g.step(steps)
    return o, g, contacts


def test_pairs_dense_contacts_fp64():
    s = _dense_contacts()
    o, g, contacts = _run(s, 60)
    assert contacts >= 50
    res = compare(o, g, s.dims, s.radii)
    check(res, 1e-12, vel_gate=1e-10)
    # the pair terms moved the particles: the force totals carry them
    assert np.abs(o.read_particles()["vel"]).max() > 1e-4


def test_pairs_dense_contacts_fp32():
    """The same dense contacts with FP32 fluid storage (particle state and
    the pair terms in FP64), at the FP32 gates."""
    s = _dense_contacts()
    o, g, contacts = _run(s, 60, precision="fp32")
    check(compare(o, g, s.dims, s.radii), 1e-5)


def test_pairs_small_box_few_cells_fp64():
    """A box two and three interaction ranges wide: the cell grid has fewer
    than three cells along x and y, where the 27-cell walk must not visit a
    cell twice."""
    rng = np.random.default_rng(41)
    dims = (24, 36, 48)
    ra, rb = uniform_fields(dims, 41, 0.7, 0.7, 0.01)
    pos = np.array([[6.0, 6.0, 6.0], [12.9, 6.3, 6.5], [18.5, 18.0, 24.0], [6.2, 29.7, 30.0], [12.0, 18.0, 41.0]])
    s = System("few-cells", dims, 1.0, 0.08, ra, rb, np.array([[5.5, 3.5]] * 5), pos, _tilted(rng, 5, 1.0),
               np.array([0.1, -0.1, 0.0, 0.2, -0.2]), np.full(5, 5.0))
    o, g, _ = _run(s, 80, u_amp=0.03)
    check(compare(o, g, s.dims, s.radii), 1e-12, vel_gate=1e-10)


def test_pairs_off_again_matches_no_pairs():
    """Turning the interactions off clears the pair terms: the run then
    matches a run that never had them (bit for bit)."""
    from paper_1109_3277_amd.binding import Lattice

    s = _dense_contacts(seed=33)

    def fresh():
        g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp64", max_particles=s.n_particles,
                    max_radius=s.max_radius)
        g.init_fields(s.rho_a, s.rho_b)
        g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
        return g

    a, b = fresh(), fresh()
    a.set_pair_interactions(True)
    a.set_pair_interactions(False)
    a.step(5)
    b.step(5)
    pa, pb = a.read_particles(), b.read_particles()
    assert all(np.array_equal(pa[k], pb[k]) for k in pa)
