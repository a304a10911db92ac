"""The lateral domain size L(t) of Eq. (12) (Sec. 4) computed on the GPU
(lb_domain_size), against the oracle on the same seeded systems and against
closed forms; FFT (power-of-two sides) and direct-DFT (other sides) paths,
particles and walls, the reduced-storage forms, and the full 512^3 size."""
import math

import numpy as np
import pytest

from oracle import domain_size as D
from paper_1109_3277_amd import workloads as W
from tests.parity_util import log, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

FP64_GATE = 1e-12


def _oracle_L(o, dims):
    ra, rb, _, own = o.read_fields()
    phi = D.order_parameter(ra, rb, own, dims)
    tot, m = D.spectrum_moments(phi)
    L = D.domain_size(phi)
    return np.array([*L, *(mi / tot for mi in m), tot])


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _modes_fields(dims, modes, base=0.7):
    """rho_A = base + phi/2, rho_B = base - phi/2 with phi a sum of
    separable cosines: modes = [(axis, m, amplitude, phase), ...]."""
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = (x, y, z)
    phi = np.zeros((nz, ny, nx))
    for ax, m, a, th in modes:
        phi += a * np.cos(2 * math.pi * m * X[ax] / dims[ax] + th)
    return (base + 0.5 * phi).ravel(), (base - 0.5 * phi).ravel()


def _modes_closed_form(dims, modes):
    """<k_i^2> of a sum of separable cosines (distinct (axis, m), 0 < m <
    n/2): sum over the modes along i of a^2 k^2 over the sum of all a^2."""
    tot = sum(a * a for _, _, a, _ in modes)
    k2 = [sum(a * a * (2 * math.pi * m / dims[ax]) ** 2 for ax, m, a, _ in modes if ax == i) / tot
          for i in range(3)]
    return k2


@pytest.mark.parametrize("dims", [(96, 40, 36), (64, 64, 64), (20, 128, 12)])
def test_separable_modes_closed_form(dims):
    """Cosines along each axis (no particles, no steps): <k_i^2> and L_i in
    closed form, through both the FFT and the DFT line paths."""
    from paper_1109_3277_amd.binding import Lattice

    modes = [(0, 3, 0.04, 0.4), (0, 5, 0.02, 1.3), (1, 2, 0.03, -0.7), (2, 1, 0.05, 0.2)]
    log(f"case separable modes dims={dims}")
    ra, rb = _modes_fields(dims, modes)
    g = Lattice(dims, 1.0, 0.08, 1, "fp64")
    g.init_fields(ra, rb)
    out = g.domain_size()
    k2 = _modes_closed_form(dims, modes)
    L = [2 * math.pi / math.sqrt(k) for k in k2]
    log(f"  L {out[:4].tolist()} closed form {L}")
    assert np.abs(out[4:7] - k2).max() <= FP64_GATE * max(k2)
    assert np.abs(out[:3] - L).max() <= FP64_GATE * max(L)
    g.close()


def _ellipsoid_interface(dims, seed):
    return W.interface_system(dims=dims, rpar=5.0, rperp=3.0, delta_rho=0.1, seed=seed)


CASES = [
    # name, system factory, steps: ragged DFT sides, FFT and DFT mixed, walls
    ("interface-40x20x12", lambda: _ellipsoid_interface((40, 20, 12), 3), 60),
    ("bijel-64x48x40", lambda: W.bijel_system(dims=(64, 48, 40), phi=0.12, seed=11), 100),
    ("spinodal-128x64x32", lambda: W.spinodal_system(dims=(128, 64, 32), seed=12), 150),
]


@pytest.mark.parametrize("name,make,steps", CASES, ids=[c[0] for c in CASES])
def test_domain_size_matches_oracle_fp64(name, make, steps):
    s = make()
    log(f"case {name} dims={s.dims} np={s.n_particles} steps={steps}")
    o = run_oracle(s, steps)
    g = run_gpu(s, steps)
    want = _oracle_L(o, s.dims)
    got = g.domain_size()
    log(f"  gpu {got.tolist()}\n  oracle {want.tolist()}")
    assert np.all(np.isfinite(want))
    assert _rel(got, want) <= FP64_GATE, _rel(got, want)
    # the call leaves the state as it was: the run goes on bit for bit
    g.step(3)
    h = run_gpu(s, steps + 3)
    assert all(np.array_equal(x, y) for x, y in zip(g.read_fields(), h.read_fields()))
    g.close()
    h.close()


def test_domain_size_walls_fp64():
    """The adsorption box: wall nodes (and the particle) count as phi = 0."""
    from paper_1109_3277_amd.binding import Lattice
    import oracle

    s = W.adsorption_system()
    steps = 100
    log(f"case adsorption walls dims={s.dims} steps={steps}")
    o = oracle.Oracle(s.dims, s.tau, s.g_br, s.psi_kind)
    o.set_walls(W.wall_mask(s.dims))
    o.init_fields(s.rho_a, s.rho_b)
    o.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    o.step(steps)
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp64", max_particles=1, max_radius=s.max_radius)
    g.set_static_solid(W.wall_mask(s.dims))
    g.init_fields(s.rho_a, s.rho_b)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.step(steps)
    want, got = _oracle_L(o, s.dims), g.domain_size()
    log(f"  gpu {got.tolist()}\n  oracle {want.tolist()}")
    assert _rel(got, want) <= FP64_GATE
    g.close()


@pytest.mark.parametrize("prec,gate", [("fp32", 1e-5), ("fp16_dev", 1e-3), ("bf16_dev", 1e-3)])
def test_domain_size_reduced_forms(prec, gate):
    s = W.bijel_system(dims=(64, 48, 40), phi=0.12, seed=11)
    steps = 60
    log(f"case bijel-64x48x40 {prec} steps={steps}")
    o = run_oracle(s, steps)
    g = run_gpu(s, steps, prec)
    want, got = _oracle_L(o, s.dims), g.domain_size()
    log(f"  gpu {got.tolist()}\n  oracle {want.tolist()} rel {_rel(got, want):.3e}")
    assert _rel(got[:4], want[:4]) <= gate
    g.close()


def test_domain_size_errors():
    import ctypes as C

    from paper_1109_3277_amd.binding import LB_EINVAL, LB_ESTATE, Batch, Lattice, LBError, load_library

    g = Lattice((8, 8, 2100), 1.0, 0.08, 1, "fp32")
    g.init_fields(np.full(8 * 8 * 2100, 0.7), np.full(8 * 8 * 2100, 0.7))
    with pytest.raises(LBError) as e:
        g.domain_size()
    assert e.value.code == LB_EINVAL
    g.close()
    b = Batch([{"dims": (8, 8, 8), "tau": 1.0, "g_br": 0.08}] * 2, "fp32")
    for k in range(2):
        b[k].init_fields(np.full(512, 0.7), np.full(512, 0.7))
    out = np.zeros(8)
    assert load_library().lb_domain_size(b._h, out.ctypes.data_as(C.POINTER(C.c_double))) == LB_ESTATE
    # a system of a batch works like a lone handle: uniform fields have no size
    assert np.isnan(b[0].domain_size()[:4]).all()
    b.close()


def test_domain_size_full_size_512():
    """512^3 (the benchmark's box): separable modes in closed form through the
    length-512 FFT; then the 41,802-ellipsoid workload after 20 steps, where
    two calls agree bit for bit and the field's sum of phi'^2 equals
    sum_k S(k) (Parseval)."""
    import torch

    from paper_1109_3277_amd.binding import Lattice

    dims = (512, 512, 512)
    modes = [(0, 7, 0.04, 0.4), (1, 3, 0.03, 1.0), (1, 40, 0.01, 0.1), (2, 2, 0.05, -0.3)]
    log("case separable modes 512^3")
    ra, rb = _modes_fields(dims, modes)
    g = Lattice(dims, 1.0, 0.08, 1, "fp64")
    g.init_fields(ra, rb)
    del ra, rb
    out = g.domain_size()
    k2 = _modes_closed_form(dims, modes)
    log(f"  <k^2> {out[4:7].tolist()} closed form {k2}")
    assert np.abs(out[4:7] - k2).max() <= FP64_GATE * max(k2)
    g.close()
    del g
    torch.cuda.empty_cache()

    s = W.mixed_system()
    log(f"case mixed 512^3 np={s.n_particles}: domain size after 20 steps")
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp64", max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.step(20)
    a, b = g.domain_size(), g.domain_size()
    assert np.array_equal(a, b)
    ra, rb, _, own = g.read_fields()
    phi = np.where(own == -1, ra - rb, 0.0)
    del ra, rb
    sq = float(((phi - phi.mean()) ** 2).sum())
    log(f"  L {a[:4].tolist()} sum S {a[7]} sum phi'^2 {sq}")
    assert abs(a[7] - sq) <= 1e-10 * sq
    assert np.all(np.isfinite(a)) and 2.0 < a[3] < 512.0
    g.close()
