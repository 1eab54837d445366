"""Pins of the oracle's stencil and Cahn-Hilliard routines against
mathematics that does not come from the oracle: scipy's correlate, Fourier
symbols of the difference operators, the FFT solution of the implicit part,
the exact linear amplification factor of a small single mode, the continuous
growth rate D k^2 (1 - gamma k^2), mass conservation, free-energy decay and
closed forms of the diagnostics."""
import math

import numpy as np
import pytest
from scipy import ndimage

from paper_2101_06550_amd import inputs

L = 2 * math.pi


def kappa2(n, length):
    """Symbol of minus the 1D second difference, (4/h^2) sin^2(pi m / n)."""
    h = length / n
    m = np.fft.fftfreq(n, d=1.0 / n)
    return (4.0 / h ** 2) * np.sin(np.pi * m / n) ** 2


def spectral_rhs(c, D, gamma, dt):
    ny, nx = c.shape
    kx2 = kappa2(nx, L)[None, :]
    ky2 = kappa2(ny, L)[:, None]
    mu = c ** 3 - c
    lap_mu = np.real(np.fft.ifft2(-(kx2 + ky2) * np.fft.fft2(mu)))
    cross = np.real(np.fft.ifft2(kx2 * ky2 * np.fft.fft2(c)))
    return c + D * dt * lap_mu - 2 * D * gamma * dt * cross


def spectral_implicit(r, D, gamma, dt):
    ny, nx = r.shape
    kx2 = kappa2(nx, L)[None, :]
    ky2 = kappa2(ny, L)[:, None]
    den = (1 + D * gamma * dt * kx2 ** 2) * (1 + D * gamma * dt * ky2 ** 2)
    return np.real(np.fft.ifft2(np.fft.fft2(r) / den))


# ---------------------------------------------------------------- stencils
@pytest.mark.parametrize("shape,ext", [((16, 20), (1, 1, 1, 1)), ((12, 9), (2, 1, 0, 3)),
                                       ((7, 33), (0, 4, 2, 2)), ((5, 5), (2, 2, 2, 2))])
@pytest.mark.parametrize("premap", [0, 1])
def test_stencil_periodic_vs_scipy(orc, shape, ext, premap):
    left, right, top, bottom = ext
    rng = np.random.default_rng(sum(shape) + premap)
    x = rng.uniform(-1, 1, shape)
    w = rng.uniform(-1, 1, (top + bottom + 1, left + right + 1))
    out = orc.stencil2d(x, w, left, right, top, bottom, periodic=True, premap=premap)
    src = x ** 3 - x if premap else x
    ref = np.zeros_like(x)
    for q in range(-top, bottom + 1):
        for p in range(-left, right + 1):
            ref += w[q + top, p + left] * np.roll(np.roll(src, -q, axis=0), -p, axis=1)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13)
    if (left, right) == (right, left) and (top, bottom) == (bottom, top):
        lib = ndimage.correlate(src, w, mode="wrap")
        np.testing.assert_allclose(out, lib, rtol=0, atol=1e-13)


def test_stencil_nonperiodic_leaves_boundary(orc):
    x = inputs.uniform(3, (10, 14), -1, 1)
    w = inputs.uniform(4, (3, 5), -1, 1)
    init = np.full_like(x, 7.0)
    out = orc.stencil2d(x, w, 2, 2, 1, 1, periodic=False, out=init)
    lib = ndimage.correlate(x, w, mode="constant")
    np.testing.assert_allclose(out[1:-1, 2:-2], lib[1:-1, 2:-2], rtol=0, atol=1e-13)
    mask = np.ones_like(x, dtype=bool)
    mask[1:-1, 2:-2] = False
    assert np.all(out[mask] == 7.0)


def test_stencil_eighth_order_second_derivative_of_sin(orc):
    """Ch.3 "Standard Weights": 8th-order central second difference of sin(x)
    on 1024 x 512 over (0, 2 pi), compared with the closed form -sin(x)."""
    nx, ny = 1024, 512
    dx = L / nx
    x = np.arange(nx) * dx
    data = np.tile(np.sin(x), (ny, 1))
    w = np.array([-1 / 560, 8 / 315, -1 / 5, 8 / 5, -205 / 72, 8 / 5, -1 / 5, 8 / 315,
                  -1 / 560]) / dx ** 2
    out = orc.stencil2d(data, w[None, :], 4, 4, 0, 0, periodic=False)
    err = np.abs(out[:, 4:-4] + np.sin(x)[None, 4:-4]).max()
    assert err < 1e-9
    assert np.all(out[:, :4] == 0) and np.all(out[:, -4:] == 0)


# ---------------------------------------------------------------- CH step
@pytest.mark.parametrize("n,seed", [(32, 1), (64, 2), (48, 9)])
def test_rhs_vs_fourier_symbols(orc, n, seed):
    c = inputs.noise_field(n, n, seed)
    D, gamma, dt = 1.0, 0.01, 1e-4
    r = orc.ch_rhs(c, L, L, D, gamma, dt)
    np.testing.assert_allclose(r, spectral_rhs(c, D, gamma, dt), rtol=0, atol=1e-12)


def test_rhs_rectangular_box(orc):
    ny, nx = 24, 40
    c = inputs.noise_field(ny, nx, 4)
    r = orc.ch_rhs(c, L, L, 1.0, 0.01, 1e-4)
    np.testing.assert_allclose(r, spectral_rhs(c, 1.0, 0.01, 1e-4), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,dt,gamma", [(32, 1e-4, 0.01), (64, 1e-3, 0.01), (128, 1e-5, 0.01),
                                        (64, 1e-6, 0.001)])
def test_step_vs_fft_implicit(orc, n, dt, gamma):
    c = inputs.noise_field(n, n, 17)
    ref = spectral_implicit(spectral_rhs(c, 1.0, gamma, dt), 1.0, gamma, dt)
    out = orc.ch_step(c, L, L, 1.0, gamma, dt)
    assert np.max(np.abs(out - ref)) / np.max(np.abs(ref)) < 1e-13


def test_step_non_square(orc):
    ny, nx = 20, 36
    c = inputs.noise_field(ny, nx, 8)
    ref = spectral_implicit(spectral_rhs(c, 1.0, 0.01, 1e-4), 1.0, 0.01, 1e-4)
    out = orc.ch_step(c, L, L, 1.0, 0.01, 1e-4)
    assert np.max(np.abs(out - ref)) / np.max(np.abs(ref)) < 1e-13


@pytest.mark.parametrize("mx,my", [(3, 4), (5, 0), (2, 7)])
def test_linear_amplification_single_mode(orc, mx, my):
    """A 1e-9 mode grows by the discrete factor
    G = (1 + D dt (kx2 + ky2) - 2 D gamma dt kx2 ky2) /
        ((1 + D gamma dt kx2^2)(1 + D gamma dt ky2^2))."""
    n, D, gamma, dt = 64, 1.0, 0.01, 1e-4
    h = L / n
    x = np.arange(n) * h
    c = 1e-9 * np.cos(mx * x[None, :] + my * x[:, None])
    kx2 = (4 / h ** 2) * math.sin(mx * h / 2) ** 2
    ky2 = (4 / h ** 2) * math.sin(my * h / 2) ** 2
    G = (1 + D * dt * (kx2 + ky2) - 2 * D * gamma * dt * kx2 * ky2) / \
        ((1 + D * gamma * dt * kx2 ** 2) * (1 + D * gamma * dt * ky2 ** 2))
    out = orc.ch_step(c, L, L, D, gamma, dt)
    assert np.max(np.abs(out - G * c)) < 1e-12 * 1e-9


def test_linear_growth_rate_matches_continuum(orc):
    """Continuous growth rate D k^2 (1 - gamma k^2) of a small mode; the
    scheme is first order in dt and second order in h, so at h = 2 pi / 256,
    dt = 1e-5 the measured rate agrees to well under 1%."""
    n, D, gamma, dt, steps = 256, 1.0, 0.01, 1e-5, 20
    h = L / n
    x = np.arange(n) * h
    mx, my = 3, 4
    amp0 = 1e-10
    c = amp0 * np.cos(mx * x[None, :] + my * x[:, None])
    out = orc.ch_step(c, L, L, D, gamma, dt, nsteps=steps)
    amp = np.sum(out * np.cos(mx * x[None, :] + my * x[:, None])) * 2 / (n * n)
    rate = math.log(amp / amp0) / (steps * dt)
    k2 = mx * mx + my * my
    sigma = D * k2 * (1 - gamma * k2)
    assert abs(rate - sigma) / sigma < 5e-3, (rate, sigma)


@pytest.mark.parametrize("n,dt,seed", [(128, 1e-4, 1), (64, 1e-3, 3)])
def test_mass_conservation_and_energy_decay(orc, n, dt, seed):
    c = inputs.noise_field(n, n, seed)
    m0 = orc.ch_mass(c, L, L)
    l1 = np.sum(np.abs(c)) * (L / n) ** 2
    F = orc.ch_energy(c, L, L, 0.01)
    for _ in range(60):
        c = orc.ch_step(c, L, L, 1.0, 0.01, dt)
        m = orc.ch_mass(c, L, L)
        assert abs(m - m0) / l1 < 1e-12
        Fn = orc.ch_energy(c, L, L, 0.01)
        assert Fn <= F + 1e-12 * abs(F)
        F = Fn


def test_diagnostics_closed_forms(orc):
    n, s, k = 64, 0.3, 5
    h = L / n
    x = np.arange(n) * h
    c = 0.2 + s * np.sin(k * x)[None, :] * np.ones((n, 1))
    assert abs(orc.ch_mass(c, L, L) - 0.2 * L * L) < 1e-12
    gamma = 0.01
    c0 = np.tile(s * np.sin(k * x), (n, 1))
    # bulk: sum (s^2 sin^2 - 1)^2 / 4 with sum sin^2 = n/2, sum sin^4 = 3n/8
    bulk = 0.25 * (s ** 4 * 3 * n / 8 - 2 * s ** 2 * n / 2 + n) * n
    # gradient: sum ((s sin(k(x+h)) - s sin(kx)) / h)^2 = s^2 4 sin^2(kh/2) (n/2) / h^2
    grad = s ** 2 * 4 * math.sin(k * h / 2) ** 2 * (n / 2) / h ** 2 * n
    F = (bulk + 0.5 * gamma * grad) * h * h
    assert abs(orc.ch_energy(c0, L, L, gamma) - F) < 1e-12 * F


def test_simpson_average_against_scipy(orc):
    """Ch.3 s(t) = 1/(1 - <C^2>), the average by Simpson's rule: on the
    periodic extension (first row and column appended) it is scipy's
    composite Simpson integral over (0, 2 pi)^2 divided by the area."""
    from scipy.integrate import simpson
    n_y, n_x = 48, 64
    c = inputs.noise_field(n_y, n_x, 17)
    ext = np.concatenate([c, c[:1]], axis=0)
    ext = np.concatenate([ext, ext[:, :1]], axis=1)
    x = np.linspace(0, 2 * np.pi, n_x + 1)
    y = np.linspace(0, 2 * np.pi, n_y + 1)
    for power in (1, 2):
        ref = simpson(simpson(ext ** power, x=x, axis=1), x=y) / (2 * np.pi) ** 2
        assert abs(orc.simpson_mean(c, power) - ref) < 1e-15 * max(1.0, abs(ref)) + 1e-17
    # closed forms: a constant, and a mode whose doubled frequency avoids n/2
    assert abs(orc.simpson_mean(np.full((8, 8), 0.3), 2) - 0.09) < 1e-16
    xx = np.arange(64) * 2 * np.pi / 64
    m = np.tile(0.7 * np.sin(3 * xx), (16, 1))
    assert abs(orc.simpson_mean(m, 2) - 0.245) < 1e-15
    assert abs(orc.ch_s(m) - 1 / (1 - 0.245)) < 1e-14


def test_k1_closed_forms(orc):
    """k1 of a single Fourier mode is its wavenumber; of two modes with
    amplitudes a, b it is (a^2 + b^2) / (a^2/|k_a| + b^2/|k_b|); the mean
    does not enter."""
    n = 64
    x = np.arange(n) * 2 * np.pi / n
    X, Y = np.meshgrid(x, x)
    assert abs(orc.ch_k1(0.3 + np.cos(3 * X + 4 * Y), L, L) - 5.0) < 1e-12
    a, b = 0.7, 0.2
    c = a * np.sin(2 * X) + b * np.cos(6 * X + 8 * Y)
    ref = (a ** 2 + b ** 2) / (a ** 2 / 2 + b ** 2 / 10)
    assert abs(orc.ch_k1(c, L, L) - ref) < 1e-12
    # a rectangular box rescales the wavenumbers
    assert abs(orc.ch_k1(np.cos(3 * X), 4 * np.pi, L) - 1.5) < 1e-12


def test_energy_decay_rate_pins(orc):
    """Ch.7 eq. 7:betaN, beta = -(t/F) dF/dt of a sampled F(t): exact for a
    quadratic F (the second-order differences are exact there), the LSW value
    1/3 for F = A t^(-1/3) (Ch.7's late-time proposition) to O(dt^2), and too
    few samples refused."""
    t0, dt = 2.0, 0.01
    t = t0 + dt * np.arange(50)
    F = 3.0 * t ** (-1.0 / 3.0)
    beta = orc.energy_decay_rate(F, t0, dt)
    assert np.max(np.abs(beta - 1.0 / 3.0)) < 1e-5
    a, b, c = 2.0, 0.3, -0.01
    F = a + b * t + c * t ** 2
    assert np.allclose(orc.energy_decay_rate(F, t0, dt), -t * (b + 2 * c * t) / F,
                       rtol=0, atol=1e-12)
    with pytest.raises(ValueError):
        orc.energy_decay_rate([1.0, 2.0], 0.0, 0.1)
