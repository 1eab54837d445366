"""Pins of the oracle's Cahn-Hilliard-Cook forcing (Ch.7): the counter-based
SplitMix64 stream against the independent implementation of the inputs
module, Box-Muller normals (moments), a conservative increment (sum zero,
variance from the forward-difference divergence), and the forced step equal
to the unforced step plus the solved increment (Fourier-space solve)."""
import math

import numpy as np
import pytest

from paper_2101_06550_amd import inputs

L = 2 * math.pi


def test_generator_matches_published_splitmix64(orc):
    """u = ((out >> 11) + 1/2) 2^-53: the inputs module's stream (same
    published generator, written independently) shifted by half a unit of
    2^-53."""
    for seed in (0, 5, 123456789):
        ref = inputs.uniform01(seed, 2000)
        got = np.array([orc.sm_uniform(seed, k) for k in range(2000)])
        # the same float64 operations on the inputs module's m = u 2^53
        assert np.array_equal(got, (ref * 2.0 ** 53 + 0.5) * 2.0 ** -53)
        assert got.min() > 0.0 and got.max() < 1.0


def test_rho_is_standard_normal(orc):
    rx, ry = orc.cook_rho(512, 512, 7, 3)
    n = rx.size
    for r in (rx, ry):
        assert abs(r.mean()) < 5 / math.sqrt(n)
        assert abs(r.var() - 1.0) < 5 * math.sqrt(2.0 / n)
        assert abs(np.mean(r ** 4) - 3.0) < 0.05        # Gaussian fourth moment
    assert abs(np.mean(rx * ry)) < 5 / math.sqrt(n)
    rx2, _ = orc.cook_rho(512, 512, 7, 4)               # the next step draws anew
    assert abs(np.mean(rx * rx2)) < 5 / math.sqrt(n)


def test_increment_is_conservative_with_the_divergence_variance(orc):
    nx, ny, dt, sigma = 256, 192, 1e-4, 1e-10
    dx, dy = L / nx, L / ny
    q = orc.cook_increment(nx, ny, L, L, dt, sigma, 11, 0)
    assert abs(q.sum()) < 1e-12 * np.abs(q).sum()
    # var(dt eta) = dt^2 sigma / (dx dy dt) (2 / dx^2 + 2 / dy^2)
    var = dt * sigma / (dx * dy) * (2 / dx ** 2 + 2 / dy ** 2)
    assert abs(q.var() / var - 1.0) < 0.03


def test_forced_step_is_unforced_step_plus_solved_increment(orc):
    n, D, g, dt, sigma = 64, 1.0, 0.01, 1e-4, 1e-12
    c = inputs.noise_field(n, n, 12)
    q = orc.cook_increment(n, n, L, L, dt, sigma, 3, 7)
    k2 = (4.0 / (L / n) ** 2) * np.sin(np.pi * np.fft.fftfreq(n, d=1.0 / n) / n) ** 2
    a = D * g * dt
    vq = np.real(np.fft.ifft2(np.fft.fft2(q) / ((1 + a * k2[None, :] ** 2) *
                                                (1 + a * k2[:, None] ** 2))))
    forced = orc.ch_step_cook(c, L, L, D, g, dt, sigma, 3, step0=7)
    plain = orc.ch_step(c, L, L, D, g, dt)
    assert np.max(np.abs(forced - plain - vq)) < 1e-13 * np.max(np.abs(c))
    assert np.array_equal(orc.ch_step_cook(c, L, L, D, g, dt, 0.0, 3), plain)
