"""Pins of the domain-size oracle (Sec. 4, Eq. (12)), no GPU: closed forms
of single and mixed Fourier modes, a brute-force DFT on a tiny box, and the
invariances the definition implies. Each pin is chosen so that a plausible
mistake fails it: a missing 2 pi or a wrong frequency range (single modes), an
unsquared |phi_k| (two modes of unequal amplitude), a missing mean subtraction
(adding a constant), swapped axes (boxes with unequal sides)."""
import cmath
import math

import numpy as np
import pytest

from oracle import domain_size as D


def _grid(dims):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(float), y.astype(float), z.astype(float)


@pytest.mark.parametrize("axis,m", [(0, 1), (0, 3), (1, 2), (2, 5)])
def test_single_mode_gives_its_wavelength(axis, m):
    """phi = cos(2 pi m x_i / n_i + 0.3): all spectral weight at k_i = +-2 pi
    m / n_i, so L_i = n_i / m exactly; the other two axes see no variation
    (infinite L in exact arithmetic; the FFT's rounding leaves ~1e-30 of
    weight there)."""
    dims = (24, 20, 30)
    X = _grid(dims)
    phi = np.cos(2 * math.pi * m * X[axis] / dims[axis] + 0.3)
    L = D.domain_size(phi)
    assert abs(L[axis] - dims[axis] / m) <= 1e-12 * dims[axis]
    assert all(L[j] > 1e6 * max(dims) for j in range(3) if j != axis)


def test_product_mode_gives_each_wavelength():
    dims = (32, 16, 24)
    x, y, z = _grid(dims)
    phi = np.cos(2 * math.pi * 2 * x / 32) * np.sin(2 * math.pi * y / 16 + 0.7) * np.cos(2 * math.pi * 3 * z / 24)
    L = D.domain_size(phi)
    want = [16.0, 16.0, 8.0]
    assert np.abs(L[:3] - want).max() <= 1e-12 * 16
    assert abs(L[3] - sum(want) / 3) <= 1e-12 * 16


def test_two_modes_weight_by_squared_amplitude():
    """a cos(k1 x) + b cos(k2 x): <k_x^2> = (a^2 k1^2 + b^2 k2^2) / (a^2 + b^2)
    for the squared structure function (the unsquared one would weight by a
    and b)."""
    nx = 40
    x, _, _ = _grid((nx, 4, 4))
    a, b, m1, m2 = 1.0, 0.35, 2, 7
    phi = a * np.cos(2 * math.pi * m1 * x / nx) + b * np.cos(2 * math.pi * m2 * x / nx + 1.1)
    k1, k2 = 2 * math.pi * m1 / nx, 2 * math.pi * m2 / nx
    want = 2 * math.pi / math.sqrt((a * a * k1 * k1 + b * b * k2 * k2) / (a * a + b * b))
    assert abs(D.domain_size(phi)[0] - want) <= 1e-12 * want


def test_nyquist_mode_of_an_even_length():
    """phi = (-1)^x: the single mode at k = pi, L_x = 2."""
    x, _, _ = _grid((10, 3, 3))
    phi = np.where(x.astype(int) % 2 == 0, 1.0, -1.0)
    assert abs(D.domain_size(phi)[0] - 2.0) <= 1e-13


def test_brute_force_dft_on_a_tiny_box():
    """Eq. (12) evaluated with the DFT written out as triple sums over a
    5 x 4 x 3 box (odd and even lengths), against the FFT-based oracle."""
    rng = np.random.default_rng(12)
    nx, ny, nz = 5, 4, 3
    phi = rng.normal(size=(nz, ny, nx))
    N = nx * ny * nz
    mean = phi.sum() / N
    tot, mom = 0.0, [0.0, 0.0, 0.0]
    for qz in range(nz):
        for qy in range(ny):
            for qx in range(nx):
                acc = 0j
                for z in range(nz):
                    for y in range(ny):
                        for x in range(nx):
                            acc += (phi[z, y, x] - mean) * cmath.exp(
                                -2j * math.pi * (qx * x / nx + qy * y / ny + qz * z / nz))
                S = abs(acc) ** 2 / N
                # wave numbers in the symmetric range (-n/2, n/2]
                k = [2 * math.pi * (q if q <= n // 2 else q - n) / n for q, n in ((qx, nx), (qy, ny), (qz, nz))]
                tot += S
                for d in range(3):
                    mom[d] += k[d] ** 2 * S
    want = [2 * math.pi / math.sqrt(m / tot) for m in mom]
    got = D.domain_size(phi)
    assert np.abs(got[:3] - want).max() <= 1e-12 * max(want)
    t2, m2 = D.spectrum_moments(phi)
    assert abs(t2 - tot) <= 1e-12 * tot and np.abs(np.array(m2) - mom).max() <= 1e-12 * max(mom)


def test_invariances():
    """A constant offset, a periodic translation, a rescaling and a sign
    flip leave L unchanged; transposing two axes swaps their components."""
    rng = np.random.default_rng(4)
    phi = rng.normal(size=(6, 10, 8))
    L0 = D.domain_size(phi)
    for other in (phi + 3.7, np.roll(phi, (2, -3, 5), axis=(0, 1, 2)), 0.01 * phi, -phi):
        assert np.abs(D.domain_size(other) - L0).max() <= 1e-12 * L0.max()
    Lt = D.domain_size(np.transpose(phi, (0, 2, 1)))  # swaps the x and y axes
    assert abs(Lt[0] - L0[1]) <= 1e-12 * L0.max() and abs(Lt[1] - L0[0]) <= 1e-12 * L0.max()
    assert abs(Lt[2] - L0[2]) <= 1e-12 * L0.max()


def test_uniform_field_has_no_domain_size():
    assert np.isnan(D.domain_size(np.full((4, 4, 4), 0.3))).all()


def test_line_transform_identity():
    """The identity a line-by-line evaluation rests on: by Parseval over the
    other two axes, sum_k k_x^2 |phi'_k|^2 = n_y n_z sum over x-lines of
    sum_{k_x} k_x^2 |A(k_x)|^2, A the 1-D transform of the line; and
    sum_k |phi'_k|^2 = N sum |phi'|^2."""
    rng = np.random.default_rng(9)
    nz, ny, nx = 6, 5, 12
    phi = rng.normal(size=(nz, ny, nx))
    N = phi.size
    f = phi - phi.mean()
    tot, mom = D.spectrum_moments(phi)
    kx = 2 * math.pi * np.fft.fftfreq(nx)
    A = np.fft.fft(f, axis=2)
    lines = (np.abs(A) ** 2 * kx ** 2).sum()
    assert abs(mom[0] - lines * ny * nz / N) <= 1e-12 * mom[0]
    assert abs(tot - (f * f).sum()) <= 1e-12 * tot


def test_order_parameter_masks_solid_nodes():
    dims = (3, 2, 2)
    ra = np.arange(12, dtype=float)
    rb = np.full(12, 0.5)
    own = np.full(12, -1, dtype=np.int32)
    own[4], own[7] = 3, -2  # a particle node and a wall node
    phi = D.order_parameter(ra, rb, own, dims).ravel()
    want = ra - rb
    want[4] = want[7] = 0.0
    assert np.array_equal(phi, want)
