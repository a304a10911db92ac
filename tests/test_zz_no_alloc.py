"""The allocation-free diagnostics entry point (lb_stats_noalloc), called
through the C ABI, against lb_stats / lb_stats_sys on the same states: two
calls in a row, the second on a smaller input (a batch of four systems, then
a lone handle), so that the second reuses the library's static scratch."""
import ctypes as C

import numpy as np
import pytest

from paper_1109_3277_amd import workloads as W
from tests.parity_util import log

pytestmark = pytest.mark.gpu


def _agree(dev, host, what):
    """FP64 gate of the diagnostics: masses relative to the mass, momentum
    relative to mass x 1e-3 (the velocity floor), removed mass relative to the
    mass; fluid count and health exactly."""
    mass = host[0] + host[1]
    assert abs(dev[0] - host[0]) <= 1e-12 * host[0] and abs(dev[1] - host[1]) <= 1e-12 * host[1], (what, dev, host)
    assert np.abs(dev[2:5] - host[2:5]).max() <= 1e-12 * mass * 1e-3, (what, dev, host)
    assert dev[5] == host[5] and dev[6] == host[6] and dev[7] == host[7], (what, dev, host)


def test_stats_noalloc_batch_then_lone():
    import torch

    from paper_1109_3277_amd.binding import Batch, Lattice, load_library

    L = load_library()
    ens = sorted(W.ensemble_systems(), key=lambda s: s.N)[:4]
    b = Batch([{"dims": s.dims, "tau": s.tau, "g_br": s.g_br, "psi_kind": s.psi_kind,
                "max_particles": s.n_particles, "max_radius": s.max_radius} for s in ens], "fp64")
    for k, s in enumerate(ens):
        b[k].init_fields(s.rho_a, s.rho_b)
        b[k].add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    b.step(9)
    out = torch.full((len(ens), 8), float("nan"), dtype=torch.float64, device="cuda")
    assert L.lb_stats_noalloc(b._h, C.c_void_p(out.data_ptr())) == 0
    torch.cuda.synchronize()
    dev = out.cpu().numpy()
    for k in range(len(ens)):
        host = b[k].stats()
        log(f"  batch system {k} {ens[k].dims}: noalloc {dev[k].tolist()} lb_stats {host.tolist()}")
        _agree(dev[k], host, f"system {k}")
    assert L.lb_stats_noalloc(b[0].handle, C.c_void_p(out.data_ptr())) < 0  # system handles are refused
    b.close()
    # second call: a smaller input, a lone handle in FP32
    s = W.interface_system(dims=(24, 24, 40), rpar=5.0, rperp=3.0, delta_rho=0.1, seed=8)
    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, "fp32", max_particles=1, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    g.step(13)
    out1 = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    assert L.lb_stats_noalloc(g.handle, C.c_void_p(out1.data_ptr())) == 0
    torch.cuda.synchronize()
    host = g.stats()
    dev1 = out1.cpu().numpy()
    log(f"  lone: noalloc {dev1.tolist()} lb_stats {host.tolist()}")
    _agree(dev1, host, "lone")
    g.close()


def test_stats_noalloc_refuses_a_changed_batch_until_stepped():
    """The call uploads nothing: a batch whose systems changed since its last
    step (here: fresh fields) is refused, and accepted after a step."""
    import torch

    from paper_1109_3277_amd.binding import LB_ESTATE, Batch, load_library

    L = load_library()
    ens = sorted(W.ensemble_systems(), key=lambda s: s.N)[:2]
    b = Batch([{"dims": s.dims, "tau": s.tau, "g_br": s.g_br, "psi_kind": s.psi_kind,
                "max_particles": s.n_particles, "max_radius": s.max_radius} for s in ens], "fp32")
    for k, s in enumerate(ens):
        b[k].init_fields(s.rho_a, s.rho_b)
    out = torch.zeros((len(ens), 8), dtype=torch.float64, device="cuda")
    assert L.lb_stats_noalloc(b._h, C.c_void_p(out.data_ptr())) == LB_ESTATE
    assert b"changed" in L.lb_last_error(b._h)
    b.step(2)
    assert L.lb_stats_noalloc(b._h, C.c_void_p(out.data_ptr())) == 0
    torch.cuda.synchronize()
    for k in range(len(ens)):
        host = b[k].stats()
        _agree(out[k].cpu().numpy(), host, f"system {k}")
    b.close()


def test_stats_noalloc_rejects_too_many_systems():
    import torch

    from paper_1109_3277_amd.binding import LB_EINVAL, Batch, load_library

    L = load_library()
    n = 257
    b = Batch([{"dims": (4, 4, 4), "tau": 1.0, "g_br": 0.08}] * n, "fp32")
    for k in range(n):
        b[k].init_fields(np.full(64, 0.7), np.full(64, 0.7))
    out = torch.zeros((n, 8), dtype=torch.float64, device="cuda")
    assert L.lb_stats_noalloc(b._h, C.c_void_p(out.data_ptr())) == LB_EINVAL
    assert b"exceeds" in L.lb_last_error(b._h)
    b.close()
