"""Pins of the oracle's second scheme, the thesis's own delta-form ADI step
with 2/3 factors (Ch.3 eq. 3:ch_adi): a Fourier-space solution of one step,
single Fourier modes against the exact two-step recurrence of the discrete
symbols, mass conservation, the start C^{-1} = C^0, and the first-order time
accuracy the thesis reports for it (Table 3.1)."""
import math

import numpy as np
import pytest

from paper_2101_06550_amd import inputs

L = 2 * math.pi


def kappa2(n):
    return (4.0 / (L / n) ** 2) * np.sin(np.pi * np.fft.fftfreq(n, d=1.0 / n) / n) ** 2


def fft_step(c, cp, D, g, dt):
    ny, nx = c.shape
    k2x, k2y = kappa2(nx)[None, :], kappa2(ny)[:, None]
    a, b = 2.0 / 3.0 * D * g * dt, 2.0 / 3.0 * D * dt
    cbar = 2 * c - cp
    r = -2.0 / 3.0 * (c - cp) - a * np.real(np.fft.ifft2((k2x + k2y) ** 2 * np.fft.fft2(cbar))) \
        + b * np.real(np.fft.ifft2(-(k2x + k2y) * np.fft.fft2(c ** 3 - c)))
    v = np.real(np.fft.ifft2(np.fft.fft2(r) / ((1 + a * k2x ** 2) * (1 + a * k2y ** 2))))
    return cbar + v


@pytest.mark.parametrize("ny,nx,D,g,dt,seed", [(32, 32, 1.0, 0.01, 1e-3, 1),
                                               (24, 40, 0.7, 0.02, 5e-4, 2),
                                               (64, 64, 1.0, 0.01, 1e-5, 3)])
def test_one_step_matches_fourier_solution(orc, ny, nx, D, g, dt, seed):
    c = inputs.noise_field(ny, nx, seed)
    cp = inputs.noise_field(ny, nx, seed + 100)
    out, prev = orc.ch2_step(c, cp, L, L, D, g, dt)
    ref = fft_step(c, cp, D, g, dt)
    assert np.max(np.abs(out - ref)) / np.max(np.abs(ref)) < 1e-13
    assert np.array_equal(prev, c)


def test_single_mode_two_step_recurrence(orc):
    """A 1e-9 mode is linear to rounding (c^3 ~ 1e-27): its amplitude follows
    A_{n+1} = Cbar + [-2/3 (A_n - A_{n-1}) - a Lam^2 Cbar + b Lam A_n] /
    ((1 + a kx^4)(1 + a ky^4)), Cbar = 2 A_n - A_{n-1}, Lam = kx^2 + ky^2."""
    n, D, g, dt = 32, 1.0, 0.01, 2e-3
    h = L / n
    x = np.arange(n) * h
    kx_i, ky_i = 3, 5
    mode = np.cos(kx_i * x[None, :] + ky_i * x[:, None])
    eps = 1e-9
    kx2 = (4 / h ** 2) * math.sin(kx_i * h / 2) ** 2
    ky2 = (4 / h ** 2) * math.sin(ky_i * h / 2) ** 2
    a, b = 2 / 3 * D * g * dt, 2 / 3 * D * dt
    lam = kx2 + ky2
    A_prev = A = eps
    c, cp = eps * mode, eps * mode
    for _ in range(6):
        cbar = 2 * A - A_prev
        v = (-2 / 3 * (A - A_prev) - a * lam ** 2 * cbar + b * lam * A) / \
            ((1 + a * kx2 ** 2) * (1 + a * ky2 ** 2))
        A_prev, A = A, cbar + v
        c, cp = orc.ch2_step(c, cp, L, L, D, g, dt)
    assert np.max(np.abs(c - A * mode)) < 1e-12 * abs(A)


def test_first_step_from_equal_states_has_no_difference_term(orc):
    c = inputs.noise_field(32, 32, 9)
    r_same = orc.ch2_rhs(c, c, L, L, 1.0, 0.01, 1e-3)
    r_shift = orc.ch2_rhs(c, c - 1e-3, L, L, 1.0, 0.01, 1e-3)
    # C_prev = C - d: the difference term gives -2/3 d, the extrapolation
    # 2C - C_prev = C + d changes the biharmonic of a constant by nothing
    assert np.max(np.abs(r_shift - (r_same - 2 / 3 * 1e-3))) < 1e-15


def test_mass_conserved(orc):
    c = inputs.noise_field(48, 32, 11)
    m0 = orc.ch_mass(c, L, L)
    cn, cp = orc.ch2_step(c, c, L, L, 1.0, 0.01, 1e-3, nsteps=20)
    assert abs(orc.ch_mass(cn, L, L) - m0) <= 1e-13 * np.sum(np.abs(c)) * (L / 32) * (L / 48)


def test_first_order_in_time(orc):
    """Table 3.1 reports first-order convergence for this scheme (the explicit
    non-linear term); at a fixed 32^2 grid and in the asymptotic range of dt,
    halving dt halves the error at T = 0.2 against a reference with dt / 8."""
    n, D, g, T = 32, 1.0, 0.01, 0.2
    c0 = inputs.noise_field(n, n, 13)

    def run(dt):
        k = int(round(T / dt))
        c, _ = orc.ch2_step(c0, c0, L, L, D, g, dt, nsteps=k)
        return c

    ref = run(T / 5120)
    errs = [np.max(np.abs(run(T / m) - ref)) for m in (160, 320, 640)]
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(0.85 < r < 1.2 for r in rates), rates
