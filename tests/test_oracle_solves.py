"""Pins of the oracle's banded solvers against mathematics that does not come
from the oracle: dense LU (numpy.linalg.solve), the circulant closed form via
FFT, exact Fourier modes, residuals, and the thesis's own hyperdiffusion
validation (Ch.4 "Validation of Scheme")."""
import math
import os

import numpy as np
import pytest

from paper_2101_06550_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_cyclic(n, coefs):
    """Dense cyclic banded matrix: row i has coefs[k] at column i + k - w
    (mod n), w = len(coefs) // 2."""
    w = len(coefs) // 2
    A = np.zeros((n, n))
    for i in range(n):
        for k, v in enumerate(coefs):
            A[i, (i + k - w) % n] += v
    return A


def penta_config(sigma):
    return (sigma, -4 * sigma, 1 + 6 * sigma, -4 * sigma, sigma)


def circulant_solve(f, coefs):
    """x = A^{-1} f for a circulant A, by the convolution theorem."""
    n = f.shape[0]
    w = len(coefs) // 2
    m = np.arange(n)
    lam = sum(v * np.exp(2j * np.pi * (k - w) * m / n) for k, v in enumerate(coefs))
    return np.real(np.fft.ifft(np.fft.fft(f) / lam))


def rel_inf(x, ref):
    return np.max(np.abs(x - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("n", list(range(5, 41)) + [64, 97, 128])
def test_cyclic_penta_vs_dense_lu_nonsymmetric(orc, n):
    rng = np.random.default_rng(n)
    a, b, d, e = rng.uniform(-0.9, 0.9, 4)
    c = 4.0 + rng.uniform(0, 1)
    f = rng.uniform(-1, 1, n)
    A = dense_cyclic(n, (a, b, c, d, e))
    ref = np.linalg.solve(A, f)
    x = orc.cyclic_penta_solve((a, b, c, d, e), f)
    assert rel_inf(x, ref) < 1e-13


@pytest.mark.parametrize("sigma", [0.17224, 0.5, 2.7558, 44.092, 70.547, 2889.6])
@pytest.mark.parametrize("n", [5, 6, 7, 16, 33, 128])
def test_cyclic_penta_vs_dense_lu_config_operators(orc, n, sigma):
    f = inputs.uniform(7, (n,), -1, 1)
    A = dense_cyclic(n, penta_config(sigma))
    ref = np.linalg.solve(A, f)
    x = orc.cyclic_penta_solve(penta_config(sigma), f)
    # kappa(A) = 1 + 16 sigma bounds the forward error
    assert rel_inf(x, ref) < 1e-15 * (1 + 16 * sigma) * 20


@pytest.mark.parametrize("n,sigma", [(128, 0.17224), (1024, 0.5), (1024, 70.547),
                                     (512, 44.092), (8192, 2889.6)])
def test_cyclic_penta_vs_circulant_fft(orc, n, sigma):
    f = inputs.uniform(11, (n,), -1, 1)
    x = orc.cyclic_penta_solve(penta_config(sigma), f)
    ref = circulant_solve(f, penta_config(sigma))
    assert rel_inf(x, ref) < 1e-16 * (1 + 16 * sigma) * 50
    # residual, computed with shifts (no matrix, no solver)
    co = penta_config(sigma)
    Ax = sum(v * np.roll(x, -(k - 2)) for k, v in enumerate(co))
    res = np.max(np.abs(Ax - f)) / (np.sum(np.abs(co)) * np.max(np.abs(x)))
    assert res < 4e-16


@pytest.mark.parametrize("n,mode", [(64, 1), (64, 7), (96, 5), (1024, 100), (30, 15)])
def test_cyclic_penta_single_mode_exact(orc, n, mode):
    sigma = 3.3
    j = np.arange(n)
    f = np.cos(2 * np.pi * mode * j / n)
    lam = 1 + 16 * sigma * math.sin(math.pi * mode / n) ** 4
    x = orc.cyclic_penta_solve(penta_config(sigma), f)
    assert np.max(np.abs(x - f / lam)) < 2e-15 * (1 + 16 * sigma)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 17, 64])
def test_general_penta_lr_vs_dense(orc, n):
    rng = np.random.default_rng(100 + n)
    a, b, d, e = (rng.uniform(-1, 1, n) for _ in range(4))
    c = 5 + rng.uniform(0, 1, n)
    A = np.diag(c)
    for i in range(n):
        if i >= 2: A[i, i - 2] = a[i]
        if i >= 1: A[i, i - 1] = b[i]
        if i + 1 < n: A[i, i + 1] = d[i]
        if i + 2 < n: A[i, i + 2] = e[i]
    f = rng.uniform(-1, 1, n)
    x = orc.penta_lr_solve(a, b, c, d, e, f)
    assert rel_inf(x, np.linalg.solve(A, f)) < 1e-14


@pytest.mark.parametrize("n", [3, 4, 5, 9, 31, 64, 257])
def test_cyclic_tri_vs_dense_lu_nonsymmetric(orc, n):
    rng = np.random.default_rng(1000 + n)
    a, c = rng.uniform(-0.9, 0.9, 2)
    b = 2.5 + rng.uniform(0, 1)
    f = rng.uniform(-1, 1, n)
    ref = np.linalg.solve(dense_cyclic(n, (a, b, c)), f)
    x = orc.cyclic_tri_solve((a, b, c), f)
    assert rel_inf(x, ref) < 1e-13


@pytest.mark.parametrize("n,beta", [(1024, 0.5), (64, 3.0), (7, 0.1), (4096, 200.0)])
def test_cyclic_tri_vs_circulant_fft(orc, n, beta):
    co = (-beta, 1 + 2 * beta, -beta)
    f = inputs.uniform(3, (n,), -1, 1)
    x = orc.cyclic_tri_solve(co, f)
    assert rel_inf(x, circulant_solve(f, co)) < 1e-16 * (1 + 4 * beta) * 50


@pytest.mark.parametrize("n", [3, 4, 6, 50])
def test_general_tri_vs_dense(orc, n):
    rng = np.random.default_rng(n)
    a, c = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    b = 3 + rng.uniform(0, 1, n)
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    f = rng.uniform(-1, 1, n)
    assert rel_inf(orc.tri_solve(a, b, c, f), np.linalg.solve(A, f)) < 1e-14


def test_lines_match_single_solves(orc):
    ny, nx = 9, 12
    data = inputs.uniform(5, (ny, nx), -1, 1)
    co = penta_config(1.7)
    rows = orc.cpenta_lines(data, 0, co)
    cols = orc.cpenta_lines(data, 1, co)
    for j in range(ny):
        np.testing.assert_allclose(rows[j], np.linalg.solve(dense_cyclic(nx, co), data[j]),
                                   rtol=0, atol=1e-14)
    for i in range(nx):
        np.testing.assert_allclose(cols[:, i], np.linalg.solve(dense_cyclic(ny, co), data[:, i]),
                                   rtol=0, atol=1e-14)


def test_bad_sizes_rejected(orc):
    with pytest.raises(ValueError):
        orc.cyclic_penta_solve(penta_config(1.0), np.ones(4))
    with pytest.raises(ValueError):
        orc.cyclic_tri_solve((-1, 2.5, -1), np.ones(2))


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_hyperdiffusion_crank_nicolson_validation(orc):
    """Ch.4 "Validation of Scheme": CN hyperdiffusion with the cyclic penta
    solver converges at second order in space against the exact decay
    A exp(-k^4 t) cos(kx); the thesis prints a fitted slope of -2.0162.
    Each step is also checked against the exact amplification factor of the
    discrete CN scheme for a single mode."""
    g = _read_golden("hyperdiffusion_cn_convergence.txt")
    dt, T, nmode = g["dt"], g["T"], int(g["n_mode"])
    steps = int(round(T / dt))
    k = 2 * math.pi * nmode
    errs, Ns = [], [16, 24, 32, 48, 64]
    for N in Ns:
        dx = 1.0 / N
        s = dt / (2 * dx ** 4)
        x = np.arange(N) * dx
        C = np.cos(k * x)
        lhs = (s, -4 * s, 1 + 6 * s, -4 * s, s)
        # discrete CN amplification for this mode
        lam = 16 * math.sin(k * dx / 2) ** 4
        G = (1 - s * lam) / (1 + s * lam)
        for _ in range(steps):
            rhs = -s * np.roll(C, 2) + 4 * s * np.roll(C, 1) + (1 - 6 * s) * C \
                  + 4 * s * np.roll(C, -1) - s * np.roll(C, -2)
            C = orc.cyclic_penta_solve(lhs, rhs)
        assert np.max(np.abs(C - G ** steps * np.cos(k * x))) < 1e-12
        exact = math.exp(-k ** 4 * T) * np.cos(k * x)
        errs.append(math.sqrt(np.mean((C - exact) ** 2)))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert abs(slope - g["slope"]) < 0.08, (slope, errs)
