"""CPU FP64 oracle of the lateral domain size L(t) (arXiv:1109.3277, Sec. 4,
Eq. (12)).

TEST INFRASTRUCTURE ONLY: it checks the HIP library's domain-size pass. Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may use
it; the product package never imports it, and the two share no code.

What is computed, in the paper's order:
- the order parameter phi~ = rho_r - rho_b (red = component A, blue = B) on
  every node; nodes of particles and walls hold no fluid and take 0;
- its fluctuation phi' = phi~ - <phi~>, the mean over all N nodes;
- the 3-D discrete Fourier transform phi'_k (numpy's FFT, a library step);
- the structure function S(k) = |phi'_k|^2 / N. The paper prints |phi'_k|
  without the square; the square is the usual definition of a structure
  function and the one taken here;
- per axis i, <k_i^2> = sum_k k_i^2 S(k) / sum_k S(k) with k_i = 2 pi n_i /
  L_i and n_i in the symmetric range of the DFT (the Nyquist mode of an even
  length has k_i^2 = pi^2 either way);
- L_i = 2 pi / sqrt(<k_i^2>), and L = (L_x + L_y + L_z) / 3.

A component whose <k_i^2> is zero (phi' constant along axis i) gives an
infinite L_i; a field with no fluctuation at all gives NaN throughout.

Arrays use the library's node order: n = x + nx * (y + ny * z), reshaped here
to (nz, ny, nx).
"""
from __future__ import annotations

import math

import numpy as np

OWN_FLUID = -1  # owner code of a fluid node as read back by the test helpers


def order_parameter(rho_a, rho_b, owner, dims) -> np.ndarray:
    """phi~ = rho_A - rho_B on fluid nodes, 0 on particle and wall nodes,
    shaped (nz, ny, nx)."""
    nx, ny, nz = dims
    ra = np.asarray(rho_a, np.float64).reshape(nz, ny, nx)
    rb = np.asarray(rho_b, np.float64).reshape(nz, ny, nx)
    fluid = np.asarray(owner).reshape(nz, ny, nx) == OWN_FLUID
    return np.where(fluid, ra - rb, 0.0)


def spectrum_moments(phi: np.ndarray):
    """(sum_k S(k), [sum_k k_x^2 S(k), sum_k k_y^2 S(k), sum_k k_z^2 S(k)])
    of a (nz, ny, nx) field, by the 3-D FFT of its fluctuation."""
    phi = np.asarray(phi, np.float64)
    nz, ny, nx = phi.shape
    N = phi.size
    fluct = phi - phi.mean()
    S = np.abs(np.fft.fftn(fluct)) ** 2 / N
    kx = 2.0 * math.pi * np.fft.fftfreq(nx)  # = 2 pi n / nx, n in the symmetric range
    ky = 2.0 * math.pi * np.fft.fftfreq(ny)
    kz = 2.0 * math.pi * np.fft.fftfreq(nz)
    mx = float((S * (kx ** 2)[None, None, :]).sum())
    my = float((S * (ky ** 2)[None, :, None]).sum())
    mz = float((S * (kz ** 2)[:, None, None]).sum())
    return float(S.sum()), [mx, my, mz]


def domain_size(phi: np.ndarray) -> np.ndarray:
    """[L_x, L_y, L_z, L] of Eq. (12) for a (nz, ny, nx) order-parameter
    field."""
    total, m = spectrum_moments(phi)
    if not total > 0.0:
        return np.full(4, math.nan)
    Li = [2.0 * math.pi / math.sqrt(mi / total) if mi > 0.0 else math.inf for mi in m]
    return np.array([*Li, sum(Li) / 3.0])


def domain_size_of_fields(rho_a, rho_b, owner, dims) -> np.ndarray:
    """Eq. (12) from the macroscopic fields (as read back from a lattice)."""
    return domain_size(order_parameter(rho_a, rho_b, owner, dims))
