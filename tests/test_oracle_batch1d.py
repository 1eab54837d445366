"""Pins of the oracle's batched 1D periodic schemes: Crank-Nicolson
hyperdiffusion (Ch.4 eq. disc), Crank-Nicolson diffusion (Ch.5
eq. 5:1ddiffscheme) and the 1D Cahn-Hilliard scheme (Ch.6 eq. 6:1Dnumerical):
exact per-mode amplification factors, the Fourier-space solution of one step
for arbitrary data, conservation of the mean, and the thesis's second-order
convergence of the hyperdiffusion validation (fitted slope -2.0162)."""
import math
import os

import numpy as np
import pytest

from paper_2101_06550_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
L2PI = 2 * math.pi


def symbols(n, L):
    """Discrete symbols of the second and fourth central differences (times
    dx^2 and dx^4): 4 sin^2(theta/2) and 16 sin^4(theta/2), theta = 2 pi m / n."""
    th = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / n
    return 4 * np.sin(th / 2) ** 2, 16 * np.sin(th / 2) ** 4


def fft_step(kind, x, L, dt, a, D):
    n = x.shape[0]
    dx = L / n
    s2, s4 = symbols(n, L)
    s2, s4 = s2[:, None], s4[:, None]
    X = np.fft.fft(x, axis=0)
    if kind == 0:
        s = a * dt / (2 * dx ** 4)
        Y = X * (1 - s * s4) / (1 + s * s4)
    elif kind == 1:
        s = a * dt / (2 * dx ** 2)
        Y = X * (1 - s * s2) / (1 + s * s2)
    else:
        s, al = a * D * dt / dx ** 4, D * dt / dx ** 2
        Nf = np.fft.fft(x ** 3 - x, axis=0)
        Y = (X - al * s2 * Nf) / (1 + s * s4)
    return np.real(np.fft.ifft(Y, axis=0))


@pytest.mark.parametrize("kind,n,L,dt,a,D", [(0, 64, 1.0, 1e-8, 1.0, 1.0),
                                            (1, 50, 1.0, 1e-4, 1.0, 1.0),
                                            (2, 256, L2PI, 1e-3, 0.01, 1.0),
                                            (2, 96, L2PI, 5e-4, 0.02, 0.7)])
def test_one_step_matches_fourier_solution(orc, kind, n, L, dt, a, D):
    x = inputs.uniform(21 + kind, (n, 7), -0.1, 0.1)
    out = orc.batch1d_step(kind, x, L, dt, a, D)
    ref = fft_step(kind, x, L, dt, a, D)
    assert np.max(np.abs(out - ref)) / np.max(np.abs(ref)) < 1e-13


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_single_modes_follow_exact_amplification(orc, kind):
    n, L = 64, (1.0 if kind < 2 else L2PI)
    dt, a, D = {0: (1e-7, 1.0, 1.0), 1: (1e-4, 1.0, 1.0), 2: (1e-3, 0.01, 1.0)}[kind]
    dx = L / n
    i = np.arange(n)[:, None]
    modes = np.array([1, 2, 5, 11, 31])[None, :]
    eps = 1e-9 if kind == 2 else 1.0
    x = eps * np.cos(2 * np.pi * modes * i / n)
    th = 2 * np.pi * modes / n
    s2, s4 = 4 * np.sin(th / 2) ** 2, 16 * np.sin(th / 2) ** 4
    if kind == 0:
        s = a * dt / (2 * dx ** 4)
        G = (1 - s * s4) / (1 + s * s4)
    elif kind == 1:
        s = a * dt / (2 * dx ** 2)
        G = (1 - s * s2) / (1 + s * s2)
    else:
        s, al = a * D * dt / dx ** 4, D * dt / dx ** 2
        G = (1 + al * s2) / (1 + s * s4)   # small amplitude: C^3 - C ~ -C
    steps = 5
    out = orc.batch1d_step(kind, x, L, dt, a, D, nsteps=steps)
    assert np.max(np.abs(out - x * G ** steps)) < 1e-12 * eps


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_mean_is_conserved(orc, kind):
    L = 1.0 if kind < 2 else L2PI
    x = inputs.uniform(30, (128, 4), -0.1, 0.1)
    out = orc.batch1d_step(kind, x, L, 1e-4 if kind else 1e-8, 0.01 if kind == 2 else 1.0,
                           nsteps=10)
    assert np.max(np.abs(out.mean(axis=0) - x.mean(axis=0))) < 1e-15


def test_hyperdiffusion_second_order_against_exact_solution(orc):
    g = {}
    for ln in open(os.path.join(GOLDEN, "hyperdiffusion_cn_convergence.txt")):
        if ln.strip() and not ln.startswith("#"):
            k, v = ln.split()
            g[k] = float(v)
    dt, T, nmode = g["dt"], g["T"], int(g["n_mode"])
    steps = int(round(T / dt))
    k = 2 * math.pi * nmode
    Ns = [16, 24, 32, 48, 64]
    x0 = np.zeros((64, len(Ns)))
    errs = []
    for N in Ns:
        xs = np.arange(N) / N
        c = orc.batch1d_step(0, np.cos(k * xs)[:, None], 1.0, dt, 1.0, nsteps=steps)[:, 0]
        exact = math.exp(-k ** 4 * T) * np.cos(k * xs)
        errs.append(math.sqrt(np.mean((c - exact) ** 2)))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert abs(slope - g["slope"]) < 0.05, slope
