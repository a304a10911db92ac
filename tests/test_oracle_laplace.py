"""Laplace law for droplets of the oracle's two-component fluid (Sec. 2,
Eq. (3); the droplets and lamellae of Sec. 4), no GPU.

With the unweighted 18-neighbour sum of Eq. (3) (sum_i c_i c_i = 10 I), the
pair forces between A at x and B at x + c_i give a bulk pressure (virial of
the 18 bonds per node, sum_i |c_i|^2 = 30, over three dimensions)

    p = c_s^2 (rho^A + rho^B) + 10 g Psi^A Psi^B,

exact in a uniform bulk where the force vanishes (derived). A droplet of A in
B at rest then has p_in - p_out = 2 gamma / R. The series is self-similar (box
side 4 R), so the bulk state outside is the same for every radius and the
surface tension gamma stays fixed: Delta p * R must be constant and the
intercept of Delta p against 1/R must vanish, up to curvature corrections of
the finite interface width."""
import math

import numpy as np

G, TAU = 0.10, 1.0  # g_br of the paper's interface runs (Sec. 4), Psi = 1 - exp(-rho)


def _pressure(ra, rb):
    pa, pb = -np.expm1(-ra), -np.expm1(-rb)
    return (ra + rb) / 3.0 + 10.0 * G * pa * pb


def _droplet(oracle_mod, R0, steps):
    L = int(round(4 * R0))
    N = L ** 3
    idx = np.arange(N)
    c = L / 2 - 0.5
    r = np.sqrt((idx % L - c) ** 2 + ((idx // L) % L - c) ** 2 + (idx // (L * L) - c) ** 2)
    inside = 0.5 * (1 - np.tanh((r - R0) / 1.5))
    # start near the coexisting densities (A-rich 1.45 / 0.046, B-rich 0.065 / 1.33)
    ra = 0.065 + (1.45 - 0.065) * inside
    rb = 1.33 - (1.33 - 0.046) * inside
    o = oracle_mod.Oracle((L, L, L), TAU, G, 1)
    o.init_fields(ra, rb)
    o.step(steps)
    A, B, u, _ = o.read_fields()
    core, far = r < 1.5, r > 0.45 * L
    a_in, a_out = A[core].mean(), A[far].mean()
    # equimolar radius of the A-rich droplet
    R = (3.0 * ((A - a_out) / (a_in - a_out)).sum() / (4.0 * math.pi)) ** (1.0 / 3.0)
    dp = _pressure(A, B)[core].mean() - _pressure(A, B)[far].mean()
    return R, dp, float(np.abs(u).max())


def test_laplace_law_droplet_series(oracle_mod):
    res = [_droplet(oracle_mod, R0, 2000) for R0 in (6.0, 8.0, 10.0)]
    R = np.array([x[0] for x in res])
    dp = np.array([x[1] for x in res])
    assert np.all(dp > 0)
    dpR = dp * R
    spread = dpR.max() / dpR.min() - 1.0
    slope, icpt = np.linalg.lstsq(np.vstack([1.0 / R, np.ones_like(R)]).T, dp, rcond=None)[0]
    print(f"R {R}, dp {dp}, dp*R {dpR}, spread {spread:.3%}, intercept {icpt:.2e}")
    assert spread <= 0.05, (R, dpR)
    assert abs(icpt) <= 0.1 * dp.min(), (icpt, dp)
    assert all(abs(r - r0) < 0.5 for r, r0 in zip(R, (6.0, 8.0, 10.0))), R
