"""The 512^3 mixed-precision domain (41,802 ellipsoids): FP32 and the FP16 /
BF16 deviation-storage forms against the GPU FP64 run on the same seed (the
oracle would need ~90 GB of host memory at this size)."""
import numpy as np
import pytest

from tests.parity_util import log

pytestmark = pytest.mark.gpu

# relative RMS density error over nodes fluid in both runs, after 100 steps
RMS_GATE = {"fp32": 1e-5, "fp16_dev": 1e-3, "bf16_dev": 1e-3}


def _run(s, prec, steps):
    from paper_1109_3277_amd.binding import Lattice

    g = Lattice(s.dims, s.tau, s.g_br, s.psi_kind, prec, max_particles=s.n_particles, max_radius=s.max_radius)
    g.init_fields(s.rho_a, s.rho_b)
    g.add_ellipsoids(s.radii, s.pos, s.quat, s.delta_rho, s.density)
    m0 = g.stats()[:2].copy()
    g.step(steps)
    ra, rb, _, own = g.read_fields()
    dm = (g.stats()[:2] - m0) / m0
    pos = g.read_particles()["pos"]
    g.close()
    return ra, rb, own, dm, pos


def test_mixed_512_precision_forms_vs_fp64():
    import torch

    from paper_1109_3277_amd import workloads as W

    s = W.mixed_system()
    log(f"case mixed 512^3: {s.n_particles} ellipsoids, 100 steps per form")
    RA, RB, OWN, DM, POS = _run(s, "fp64", 100)
    torch.cuda.empty_cache()
    sc = max(np.abs(RA).max(), np.abs(RB).max())
    L = np.array(s.dims, float)
    for prec in ("fp32", "fp16_dev", "bf16_dev"):
        ra, rb, own, dm, pos = _run(s, prec, 100)
        torch.cuda.empty_cache()
        both = (own == -1) & (OWN == -1)
        d = np.concatenate([(ra - RA)[both], (rb - RB)[both]])
        e_rms = float(np.sqrt(np.mean(d * d)) / sc)
        e_max = float(np.abs(d).max() / sc)
        n_diff = int((own != OWN).sum())
        dX = pos - POS
        dX -= np.round(dX / L) * L
        res = {"e_rms": e_rms, "e_max": e_max, "owner_diff": n_diff, "mass_drift_vs_fp64": (dm - DM).tolist(),
               "fp64_mass_change": DM.tolist(), "max_dpos": float(np.abs(dX).max())}
        log(f"  {prec}: {res}")
        assert e_rms <= RMS_GATE[prec], res
        # kill / fill events at slightly different particle positions flip a
        # few owner codes; they stay a vanishing fraction of the box
        assert n_diff <= 1e-5 * own.size, res
        assert np.all(np.abs(dm - DM) <= 1e-4), res
