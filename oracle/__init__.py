"""Plain serial FP64 CPU oracle for the Cahn-Hilliard ADI hot path.

TEST INFRASTRUCTURE ONLY: only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the HIP library (``paper_2101_06550_amd``) and never imports it;
the library never imports this package.

The arithmetic lives in ``oracle.c`` (gcc -O2 -ffp-contract=off); this module
only marshals numpy arrays through ctypes.  Each wrapper names the passage of
the thesis (arXiv 2101.06550) that the C routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.POINTER(ctypes.c_double)


def build(out: str = _LIB, src: str = _SRC, extra: tuple = ()) -> str:
    """Compile the oracle with gcc (no FMA contraction); returns the path."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-fPIC", "-shared", "-I", _HERE, *extra, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def load(path: str | None = None):
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB
    if not os.path.exists(p):
        build(p)
    lib = ctypes.CDLL(p)
    lib.orc_penta_lr_factor.restype = _I
    lib.orc_penta_lr_factor.argtypes = [_I] + [_P] * 10
    lib.orc_penta_lr_solve.restype = None
    lib.orc_penta_lr_solve.argtypes = [_I] + [_P] * 7
    lib.orc_tri_prefactor.restype = _I
    lib.orc_tri_prefactor.argtypes = [_I] + [_P] * 5
    lib.orc_tri_solve.restype = None
    lib.orc_tri_solve.argtypes = [_I] + [_P] * 5
    lib.orc_cyclic_penta_solve.restype = _I
    lib.orc_cyclic_penta_solve.argtypes = [_I, _D, _D, _D, _D, _D, _P, _P]
    lib.orc_cyclic_tri_solve.restype = _I
    lib.orc_cyclic_tri_solve.argtypes = [_I, _D, _D, _D, _P, _P]
    lib.orc_penta_rows_batch.restype = _I
    lib.orc_penta_rows_batch.argtypes = [_I, _I, ctypes.c_long, _I] + [_P] * 6
    lib.orc_tri_rows_batch.restype = _I
    lib.orc_tri_rows_batch.argtypes = [_I, _I, ctypes.c_long, _I] + [_P] * 4
    lib.orc_cpenta_lines.restype = _I
    lib.orc_cpenta_lines.argtypes = [_I, _I, _I, _D, _D, _D, _D, _D, _P]
    lib.orc_ctri_lines.restype = _I
    lib.orc_ctri_lines.argtypes = [_I, _I, _I, _D, _D, _D, _P]
    lib.orc_stencil2d.restype = _I
    lib.orc_stencil2d.argtypes = [_P, _P, _I, _I, _P, _I, _I, _I, _I, _I, _I]
    lib.orc_ch_rhs.restype = None
    lib.orc_ch_rhs.argtypes = [_P, _P, _I, _I, _D, _D, _D, _D, _D]
    lib.orc_ch_step.restype = _I
    lib.orc_ch_step.argtypes = [_P, _I, _I, _D, _D, _D, _D, _D]
    _U64 = ctypes.c_uint64
    lib.orc_sm_uniform.restype = _D
    lib.orc_sm_uniform.argtypes = [_U64, _U64]
    lib.orc_cook_rho.restype = None
    lib.orc_cook_rho.argtypes = [_P, _P, _I, _I, _U64, _U64]
    lib.orc_cook_increment.restype = None
    lib.orc_cook_increment.argtypes = [_P, _I, _I, _D, _D, _D, _D, _U64, _U64]
    lib.orc_ch_step_cook.restype = _I
    lib.orc_ch_step_cook.argtypes = [_P, _I, _I, _D, _D, _D, _D, _D, _D, _U64, _U64]
    lib.orc_simpson_mean.restype = _D
    lib.orc_simpson_mean.argtypes = [_P, _I, _I, _I]
    lib.orc_batch1d_step.restype = _I
    lib.orc_batch1d_step.argtypes = [_I, _P, _I, _I, _D, _D, _D, _D]
    lib.orc_ch2_rhs.restype = None
    lib.orc_ch2_rhs.argtypes = [_P, _P, _P, _I, _I, _D, _D, _D, _D, _D]
    lib.orc_ch2_step.restype = _I
    lib.orc_ch2_step.argtypes = [_P, _P, _I, _I, _D, _D, _D, _D, _D]
    lib.orc_ch_mass.restype = _D
    lib.orc_ch_mass.argtypes = [_P, _I, _I, _D, _D]
    lib.orc_ch_energy.restype = _D
    lib.orc_ch_energy.argtypes = [_P, _I, _I, _D, _D, _D]
    lib.orc_energy_decay_rate.restype = _I
    lib.orc_energy_decay_rate.argtypes = [_P, _I, _D, _D, _P]
    if path is None:
        _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Bound view of one compiled oracle library (the default one, or a
    mutant build made by a test)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # Ch.4 "Solution of the pentadiagonal system" (general LR, non-cyclic)
    def penta_lr_solve(self, a, b, c, d, e, f):
        a, b, c, d, e, f = map(_f64, (a, b, c, d, e, f))
        n = f.shape[0]
        fac = [np.zeros(n) for _ in range(5)]
        rc = self.lib.orc_penta_lr_factor(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d),
                                          _ptr(e), *[_ptr(x) for x in fac])
        if rc:
            raise ValueError("zero or non-finite pivot")
        x = np.zeros(n)
        self.lib.orc_penta_lr_solve(n, *[_ptr(v) for v in fac], _ptr(f), _ptr(x))
        return x

    # Ch.5 "Tridiagonal Inversion Algorithm" (general Thomas, non-cyclic)
    def tri_solve(self, a, b, c, f):
        a, b, c, f = map(_f64, (a, b, c, f))
        n = f.shape[0]
        chat, den = np.zeros(n), np.zeros(n)
        if self.lib.orc_tri_prefactor(n, _ptr(a), _ptr(b), _ptr(c), _ptr(chat),
                                      _ptr(den)):
            raise ValueError("zero or non-finite pivot")
        x = np.zeros(n)
        self.lib.orc_tri_solve(n, _ptr(a), _ptr(chat), _ptr(den), _ptr(f), _ptr(x))
        return x

    # Ch.4 "The pentadiagonal matrix system" (Navon bordering) + LR
    def cyclic_penta_solve(self, coefs, f):
        f = _f64(f)
        x = np.zeros_like(f)
        rc = self.lib.orc_cyclic_penta_solve(f.shape[0], *map(float, coefs), _ptr(f),
                                             _ptr(x))
        if rc:
            raise ValueError(f"cyclic penta solve failed ({rc})")
        return x

    # Ch.5 "Periodic Tridiagonal Matrix" (Sherman-Morrison) + Thomas
    def cyclic_tri_solve(self, coefs, f):
        f = _f64(f)
        x = np.zeros_like(f)
        rc = self.lib.orc_cyclic_tri_solve(f.shape[0], *map(float, coefs), _ptr(f),
                                           _ptr(x))
        if rc:
            raise ValueError(f"cyclic tri solve failed ({rc})")
        return x

    # Ch.4 "Implementation on GPU" / Ch.5: batches with one matrix per system
    def penta_rows_batch(self, a, b, c, d, e, f, periodic):
        """Every argument is an (n, batch) array (entry i of system s at
        [i, s]); row i of system s is a x_{i-2} + b x_{i-1} + c x_i + d x_{i+1}
        + e x_{i+2} = f_i, wrapping mod n when ``periodic``.  Returns x."""
        a, b, c, d, e = map(_f64, (a, b, c, d, e))
        x = _f64(f).copy()
        n, batch = x.shape
        rc = self.lib.orc_penta_rows_batch(n, batch, batch, int(bool(periodic)),
                                           *[_ptr(v) for v in (a, b, c, d, e, x)])
        if rc:
            raise ValueError(f"batched penta solve failed ({rc})")
        return x

    def tri_rows_batch(self, a, b, c, f, periodic):
        """As ``penta_rows_batch`` for rows a x_{i-1} + b x_i + c x_{i+1}."""
        a, b, c = map(_f64, (a, b, c))
        x = _f64(f).copy()
        n, batch = x.shape
        rc = self.lib.orc_tri_rows_batch(n, batch, batch, int(bool(periodic)),
                                         *[_ptr(v) for v in (a, b, c, x)])
        if rc:
            raise ValueError(f"batched tri solve failed ({rc})")
        return x

    def cpenta_lines(self, data2d, direction, coefs):
        """Solve every row (direction 0) or column (direction 1) of a
        row-major (ny, nx) array with one cyclic penta matrix; returns a copy."""
        out = _f64(data2d).copy()
        ny, nx = out.shape
        rc = self.lib.orc_cpenta_lines(nx, ny, direction, *map(float, coefs), _ptr(out))
        if rc:
            raise ValueError(f"cyclic penta lines failed ({rc})")
        return out

    def ctri_lines(self, data2d, direction, coefs):
        out = _f64(data2d).copy()
        ny, nx = out.shape
        rc = self.lib.orc_ctri_lines(nx, ny, direction, *map(float, coefs), _ptr(out))
        if rc:
            raise ValueError(f"cyclic tri lines failed ({rc})")
        return out

    # Ch.3 "Software API" (cuSten-style stencil, xy direction)
    def stencil2d(self, x2d, weights, left, right, top, bottom, periodic=True,
                  premap=0, out=None):
        x2d = _f64(x2d)
        ny, nx = x2d.shape
        w = _f64(weights).ravel()
        assert w.size == (left + right + 1) * (top + bottom + 1)
        o = np.zeros_like(x2d) if out is None else _f64(out).copy()
        rc = self.lib.orc_stencil2d(_ptr(x2d), _ptr(o), nx, ny, _ptr(w), left, right,
                                    top, bottom, int(bool(periodic)), int(premap))
        if rc:
            raise ValueError("bad stencil arguments")
        return o

    # Ch.2 eq. 2:ch / Ch.3 eq. 3:ch_adi (first-order ADI right-hand side)
    def ch_rhs(self, c2d, lx, ly, D, gamma, dt):
        c = _f64(c2d)
        ny, nx = c.shape
        r = np.zeros_like(c)
        self.lib.orc_ch_rhs(_ptr(c), _ptr(r), nx, ny, lx, ly, D, gamma, dt)
        return r

    def ch_step(self, c2d, lx, ly, D, gamma, dt, nsteps=1):
        c = _f64(c2d).copy()
        ny, nx = c.shape
        for _ in range(nsteps):
            rc = self.lib.orc_ch_step(_ptr(c), nx, ny, lx, ly, D, gamma, dt)
            if rc:
                raise ValueError(f"ch step failed ({rc})")
        return c

    # Ch.3 eq. 3:ch_adi (the thesis's delta-form scheme with 2/3 factors)
    def ch2_rhs(self, c2d, cprev2d, lx, ly, D, gamma, dt):
        c, cp = _f64(c2d), _f64(cprev2d)
        ny, nx = c.shape
        r = np.zeros_like(c)
        self.lib.orc_ch2_rhs(_ptr(c), _ptr(cp), _ptr(r), nx, ny, lx, ly, D, gamma, dt)
        return r

    def ch2_step(self, c2d, cprev2d, lx, ly, D, gamma, dt, nsteps=1):
        """Advance (C^n, C^{n-1}) by nsteps; returns the new (C, C_prev)."""
        c, cp = _f64(c2d).copy(), _f64(cprev2d).copy()
        ny, nx = c.shape
        for _ in range(nsteps):
            rc = self.lib.orc_ch2_step(_ptr(c), _ptr(cp), nx, ny, lx, ly, D, gamma, dt)
            if rc:
                raise ValueError(f"ch2 step failed ({rc})")
        return c, cp

    # Ch.4 eq. disc / Ch.5 eq. 5:1ddiffscheme / Ch.6 eq. 6:1Dnumerical
    def batch1d_step(self, kind, x2d, L, dt, a, D=1.0, nsteps=1):
        """x2d: (n, batch) interleaved systems; returns the state nsteps later."""
        x = _f64(x2d).copy()
        n, batch = x.shape
        for _ in range(nsteps):
            rc = self.lib.orc_batch1d_step(int(kind), _ptr(x), n, batch, L, dt, a, D)
            if rc:
                raise ValueError(f"batch1d step failed ({rc})")
        return x

    # Ch.7 Cahn-Hilliard-Cook forcing
    def sm_uniform(self, seed, k):
        return self.lib.orc_sm_uniform(seed, k)

    def cook_rho(self, nx, ny, seed, step):
        rx, ry = np.zeros((ny, nx)), np.zeros((ny, nx))
        self.lib.orc_cook_rho(_ptr(rx), _ptr(ry), nx, ny, seed, step)
        return rx, ry

    def cook_increment(self, nx, ny, lx, ly, dt, sigma, seed, step):
        out = np.zeros((ny, nx))
        self.lib.orc_cook_increment(_ptr(out), nx, ny, lx, ly, dt, sigma, seed, step)
        return out

    def ch_step_cook(self, c2d, lx, ly, D, gamma, dt, sigma, seed, step0=0, nsteps=1):
        """nsteps Cook steps; step k of the call draws with counter step0 + k."""
        c = _f64(c2d).copy()
        ny, nx = c.shape
        for k in range(nsteps):
            rc = self.lib.orc_ch_step_cook(_ptr(c), nx, ny, lx, ly, D, gamma, dt, sigma, seed,
                                           step0 + k)
            if rc:
                raise ValueError(f"cook step failed ({rc})")
        return c

    # Ch.3 "Numerical Results": Simpson averages and s(t) = 1 / (1 - <C^2>)
    def simpson_mean(self, c2d, power=1):
        c = _f64(c2d)
        ny, nx = c.shape
        return self.lib.orc_simpson_mean(_ptr(c), nx, ny, int(power))

    def ch_s(self, c2d):
        return 1.0 / (1.0 - self.simpson_mean(c2d, 2))

    @staticmethod
    def ch_k1(c2d, lx, ly):
        """Ch.3 "Numerical Results": k1 = sum |C^|^2 / sum |k|^-1 |C^|^2 over
        the discrete wavevectors k = (2 pi m / lx, 2 pi l / ly) other than
        k = 0 (where |k|^-1 is undefined), C^ the discrete Fourier transform
        (a library FFT, numpy's)."""
        c = _f64(c2d)
        ny, nx = c.shape
        C = np.fft.fft2(c)
        kx = 2 * np.pi * np.fft.fftfreq(nx, d=lx / nx)
        ky = 2 * np.pi * np.fft.fftfreq(ny, d=ly / ny)
        k = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
        p = np.abs(C) ** 2
        p[0, 0] = 0.0
        k[0, 0] = 1.0
        return float(np.sum(p) / np.sum(p / k))

    def ch_mass(self, c2d, lx, ly):
        c = _f64(c2d)
        ny, nx = c.shape
        return self.lib.orc_ch_mass(_ptr(c), nx, ny, lx, ly)

    def ch_energy(self, c2d, lx, ly, gamma):
        c = _f64(c2d)
        ny, nx = c.shape
        return self.lib.orc_ch_energy(_ptr(c), nx, ny, lx, ly, gamma)

    def energy_decay_rate(self, F, t0, dt):
        """beta_k = -(t_k / F_k) dF/dt at t_k = t0 + k dt (Ch.7 eq. 7:betaN)."""
        f = _f64(np.asarray(F, dtype=np.float64)).copy()
        out = np.empty_like(f)
        if self.lib.orc_energy_decay_rate(_ptr(f), f.size, float(t0), float(dt), _ptr(out)):
            raise ValueError("energy_decay_rate needs at least three samples and dt > 0")
        return out


_default = None


def oracle() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
