"""Seeded synthetic inputs shared by the tests, the smoke entry point and the
benchmark.  This module holds none of the method's arithmetic: it only turns
a seed into numbers and shapes them like the thesis's workloads (uniform
noise initial conditions on the periodic box (0, 2*pi)^2, uniform right-hand
sides for batched solves).

Generator: the k-th output of the SplitMix64 sequence (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) whose state
starts at mix(seed):

    state_k = mix(seed) + (k + 1) * 0x9E3779B97F4A7C15      (mod 2^64)
    u_k     = (mix(state_k) >> 11) * 2^-53                   in [0, 1)

with mix(z) = the SplitMix64 finaliser (xor-shift 30/27/31 with the
multipliers 0xBF58476D1CE4E5B9 and 0x94D049BB133111EB).  For a field c[j][i]
the counter is k = j * nx + i.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """u_k for k = start .. start+count-1, as float64 in [0, 1)."""
    with np.errstate(over="ignore"):
        s0 = _mix(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
        out = np.empty(count, dtype=np.float64)
        step = 1 << 22
        for lo in range(0, count, step):
            hi = min(count, lo + step)
            k = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            st = s0 + k * _GOLDEN
            out[lo:hi] = (_mix(st) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return out


def uniform(seed: int, shape, lo: float, hi: float) -> np.ndarray:
    """lo + (hi - lo) * u, laid out row-major in ``shape``."""
    n = int(np.prod(shape))
    return (lo + (hi - lo) * uniform01(seed, n)).reshape(shape)


def noise_field(n_y: int, n_x: int, seed: int, amp: float = 0.1) -> np.ndarray:
    """c0 ~ U[-amp, amp] iid on an (n_y, n_x) grid (the thesis's symmetric
    quench, U[-0.1, 0.1])."""
    return uniform(seed, (n_y, n_x), -amp, amp)


def asymmetric_mixture(n_y: int, n_x: int, seed: int, lo: float = 0.4,
                       hi: float = 0.6) -> np.ndarray:
    """c0 ~ U[lo, hi] iid: the thesis's asymmetric (off-critical) mixture of
    the Ch.7 ensembles, U[0.4, 0.6], whose minority phase coarsens by
    Ostwald ripening."""
    return uniform(seed, (n_y, n_x), lo, hi)


def mode_plus_noise(n: int, seed: int, amp: float = 0.05, kx: int = 3, ky: int = 5,
                    noise: float = 0.01, length: float = 2 * math.pi) -> np.ndarray:
    """c0 = amp sin(kx x) sin(ky y) + U[-noise, noise] on an n x n grid of
    (0, length)^2 with x_i = i * length / n (the large-run initial state)."""
    x = np.arange(n) * (length / n)
    field = amp * np.outer(np.sin(ky * x), np.sin(kx * x))
    return field + uniform(seed, (n, n), -noise, noise)


def batch_rhs(seed: int, n: int, batch: int, lo: float = -1.0, hi: float = 1.0,
              interleaved: bool = True) -> np.ndarray:
    """Right-hand sides for ``batch`` systems of size ``n``.  Interleaved
    layout returns shape (n, batch) (entry i of every system contiguous);
    otherwise (batch, n)."""
    u = uniform(seed, (n, batch) if interleaved else (batch, n), lo, hi)
    return u


# Parameters of the thesis's workloads (see the benchmark and tests).
TWO_PI = 2.0 * math.pi
