"""Oracle pins for batches with one banded matrix per system (Ch.4
"Implementation on GPU": five diagonals and a right-hand side per system,
interleaved; Ch.5 for the tridiagonal case), periodic or not."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


def _dense(coefs, offsets, s, periodic):
    n = coefs[0].shape[0]
    A = np.zeros((n, n))
    for i in range(n):
        for off, co in zip(offsets, coefs):
            j = i + off
            if periodic:
                A[i, j % n] += co[i, s]
            elif 0 <= j < n:
                A[i, j] += co[i, s]
    return A


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("n", [5, 7, 64])
def test_penta_rows_vs_dense(orc, periodic, n):
    rng = np.random.default_rng(100 + n)
    B = 6
    a, b, d, e = (rng.uniform(-1, 1, (n, B)) for _ in range(4))
    c = 4.5 + rng.uniform(0, 1, (n, B))
    f = rng.uniform(-1, 1, (n, B))
    x = orc.penta_rows_batch(a, b, c, d, e, f, periodic)
    for s in range(B):
        ref = np.linalg.solve(_dense((a, b, c, d, e), (-2, -1, 0, 1, 2), s, periodic), f[:, s])
        assert np.max(np.abs(x[:, s] - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("n", [3, 4, 64])
def test_tri_rows_vs_dense(orc, periodic, n):
    rng = np.random.default_rng(200 + n)
    B = 6
    a, c = (rng.uniform(-1, 1, (n, B)) for _ in range(2))
    b = 2.5 + rng.uniform(0, 1, (n, B))
    f = rng.uniform(-1, 1, (n, B))
    x = orc.tri_rows_batch(a, b, c, f, periodic)
    for s in range(B):
        ref = np.linalg.solve(_dense((a, b, c), (-1, 0, 1), s, periodic), f[:, s])
        assert np.max(np.abs(x[:, s] - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


def test_constant_rows_match_circulant_closed_form(orc):
    """Equal rows give the Ch.4 hyperdiffusion matrix, whose inverse acts on
    Fourier mode m by 1/(1 + 16 s sin^4(pi m / n))."""
    n, B, sig = 48, 3, 2.5
    rng = np.random.default_rng(7)
    f = rng.uniform(-1, 1, (n, B))
    one = np.ones((n, B))
    x = orc.penta_rows_batch(sig * one, -4 * sig * one, (1 + 6 * sig) * one,
                             -4 * sig * one, sig * one, f, True)
    lam = 1 + 16 * sig * np.sin(np.pi * np.arange(n) / n) ** 4
    ref = np.real(np.fft.ifft(np.fft.fft(f, axis=0) / lam[:, None], axis=0))
    assert np.max(np.abs(x - ref)) < 1e-14
    beta = 0.75
    y = orc.tri_rows_batch(-beta * one, (1 + 2 * beta) * one, -beta * one, f, True)
    lam3 = 1 + 4 * beta * np.sin(np.pi * np.arange(n) / n) ** 2
    ref3 = np.real(np.fft.ifft(np.fft.fft(f, axis=0) / lam3[:, None], axis=0))
    assert np.max(np.abs(y - ref3)) < 1e-14


def test_systems_are_independent(orc):
    """Changing one system's matrix leaves the others' solutions untouched."""
    n, B = 16, 5
    rng = np.random.default_rng(9)
    a, b, d, e = (rng.uniform(-1, 1, (n, B)) for _ in range(4))
    c = 5 + rng.uniform(0, 1, (n, B))
    f = rng.uniform(-1, 1, (n, B))
    x0 = orc.penta_rows_batch(a, b, c, d, e, f, True)
    c2 = c.copy()
    c2[:, 2] += 1.0
    x1 = orc.penta_rows_batch(a, b, c2, d, e, f, True)
    keep = [0, 1, 3, 4]
    assert np.array_equal(x0[:, keep], x1[:, keep])
    assert not np.allclose(x0[:, 2], x1[:, 2])


def test_zero_pivot_is_reported(orc):
    n, B = 8, 3
    z = np.zeros((n, B))
    c = np.ones((n, B))
    c[0, 1] = 0.0  # system 1 has a zero first pivot
    with pytest.raises(ValueError, match="-3"):
        orc.penta_rows_batch(z, z, c, z, z, np.ones((n, B)), False)
    with pytest.raises(ValueError, match="-3"):
        orc.tri_rows_batch(z, c, z, np.ones((n, B)), False)
