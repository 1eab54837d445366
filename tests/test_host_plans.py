"""CPU tests of the library's host side: the shared library loads without a
GPU, exports every symbol that include/chx.h declares, rejects bad arguments
before touching a device, and its factorisation tables (read back through the
host-inspection calls) reproduce the oracle's cyclic solves when the chunked
and whole-system algorithms are replayed with them in numpy."""
import os
import re

import numpy as np
import pytest

from paper_2101_06550_amd import chx, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chx.h")


def penta(sigma):
    return (sigma, -4 * sigma, 1 + 6 * sigma, -4 * sigma, sigma)


@pytest.fixture(scope="module")
def lib():
    return chx.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_library_exports_every_declared_symbol(lib):
    declared = header_functions()
    assert "penta_solve_batch" in declared and "ch_adi_step" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(chx.EXPORTED) == declared


def test_status_strings(lib):
    assert chx.chx_status_string(0) == "ok"
    assert "pivot" in chx.chx_status_string(-3)
    assert chx.chx_version() >= 100


def test_bad_arguments_rejected_on_host(lib):
    import ctypes
    h = ctypes.c_void_p()
    assert lib.penta_factor(4, 1, -4, 7, -4, 1, 1, ctypes.byref(h)) == chx.CHX_EUNSUPPORTED_N
    assert lib.tri_factor(2, -1, 3, -1, 1, ctypes.byref(h)) == chx.CHX_EUNSUPPORTED_N
    assert lib.penta_factor(8, 1, -4, 7, -4, 1, 1, None) == chx.CHX_EINVAL
    # NaN coefficient
    assert lib.penta_factor(8, float("nan"), -4, 7, -4, 1, 1, ctypes.byref(h)) == chx.CHX_EINVAL
    # null plan / pointers
    assert lib.penta_solve_batch(None, 4, None, 4, 0, 0, 0, None, 0, None) == chx.CHX_EINVAL
    w = (ctypes.c_double * 9)(*([0.0] * 9))
    assert lib.stencil2d_apply(None, None, 8, 8, 8, 0, w, 1, 1, 1, 1, 1, 0, None) == chx.CHX_EINVAL
    # stencil extent beyond 4
    p = ctypes.c_void_p(1 << 20)
    q = ctypes.c_void_p(1 << 30)
    big = (ctypes.c_double * 121)(*([0.0] * 121))
    assert lib.stencil2d_apply(p, q, 64, 64, 64, 0, big, 5, 5, 0, 0, 1, 0, None) == chx.CHX_EINVAL
    # overlapping in/out, for either element size (FP32 arrays 4 B apart per
    # element: 8 x 8 FP32 at p and p + 128 B overlap, FP64 at p + 256 B too)
    assert lib.stencil2d_apply(p, p, 8, 8, 8, 0, w, 1, 1, 1, 1, 1, 0, None) == chx.CHX_EINVAL
    p2 = ctypes.c_void_p((1 << 20) + 128)
    assert lib.stencil2d_apply(p, p2, 8, 8, 8, chx.CHX_F32, w, 1, 1, 1, 1, 1, 0,
                               None) == chx.CHX_EINVAL
    # unknown dtype (CHX_F32_REFINED is not an array type)
    assert lib.stencil2d_apply(p, q, 8, 8, 8, chx.CHX_F32_REFINED, w, 1, 1, 1, 1, 1, 0,
                               None) == chx.CHX_EINVAL
    prm = chx.ChParams(4, 64, 6.28, 6.28, 1.0, 0.01, 1e-4, 0, 0)
    assert lib.ch_create(ctypes.byref(prm), ctypes.byref(h)) == chx.CHX_EUNSUPPORTED_N
    prm = chx.ChParams(64, 64, 6.28, 6.28, 1.0, 0.01, -1.0, 0, 0)
    assert lib.ch_create(ctypes.byref(prm), ctypes.byref(h)) == chx.CHX_EINVAL
    assert lib.batch1d_create(7, 64, 1.0, 1e-3, 1.0, 1.0, ctypes.byref(h)) == chx.CHX_EINVAL
    assert lib.batch1d_create(0, 4, 1.0, 1e-3, 1.0, 1.0, ctypes.byref(h)) == chx.CHX_EUNSUPPORTED_N
    assert lib.batch1d_create(1, 2, 1.0, 1e-3, 1.0, 1.0, ctypes.byref(h)) == chx.CHX_EUNSUPPORTED_N
    assert lib.batch1d_create(2, 64, 1.0, -1.0, 1.0, 1.0, ctypes.byref(h)) == chx.CHX_EINVAL
    assert lib.batch1d_create(2, 64, 1.0, 1e-3, 1.0, 1.0, None) == chx.CHX_EINVAL
    assert lib.batch1d_step(None, 4, None, 4, 1, None, 0, None) == chx.CHX_EINVAL
    assert lib.batch1d_ws_bytes(None, 4) == 0
    assert lib.ch_set_noise(None, 1e-10, 1, 0) == chx.CHX_EINVAL
    assert lib.ch_moments(None, None, 8, None, None) == chx.CHX_EINVAL
    assert lib.ch_k1(None, None, 8, None, None) == chx.CHX_EINVAL
    assert lib.ch_get_noise_step(None, None) == chx.CHX_EINVAL
    v = ctypes.c_int()
    assert lib.ch_get_tuning(None, 0, ctypes.byref(v)) == chx.CHX_EINVAL
    assert lib.ch_set_tuning(None, 0, 0) == chx.CHX_EINVAL


def test_shape_count_matches_header():
    text = open(HEADER).read()
    for name in ("CHX_NUM_REDUCED_SHAPES", "CHX_TUNE_REDUCED_SHAPE", "CHX_TUNE_SMALL_PATH",
                 "CHX_TUNE_ROW_SPLIT", "CHX_NUM_SPLIT_SHAPES", "CHX_SCHEME_P1", "CHX_SCHEME_P2",
                 "CHX_TUNE_COLUMN_ORDER", "CHX_NUM_COLUMN_ORDERS", "CHX_NOALLOC_SCRATCH_BYTES",
                 "CHX_TUNE_GRAPH", "CHX_TUNE_COLUMN_CHUNK", "CHX_TUNE_ROW_CHUNK",
                 "CHX_NUM_ENS_REDUCED_SHAPES",
                 "CHX_1D_HYPERDIFFUSION_CN", "CHX_1D_DIFFUSION_CN", "CHX_1D_CAHN_HILLIARD"):
        m = re.search(r"#define\s+" + name + r"\s+\(?(\d+)(u << (\d+)\))?", text)
        value = int(m.group(1)) << int(m.group(3) or 0) if m else None
        assert value == getattr(chx, name), name
    m = re.search(r"#define\s+CHX_ROW_SPLIT_OVERLAP\s+\((-?\d+)\)", text)
    assert m and int(m.group(1)) == chx.CHX_ROW_SPLIT_OVERLAP


def test_non_positive_pivot_is_reported():
    # a matrix with a negative diagonal fails the alpha_i > 0 check
    rec = None
    with pytest.raises(chx.ChxError) as ei:
        chx.chx_host_whole_tables(2, (0.1, 0.2, -3.0, 0.2, 0.1), 16, True)
    assert ei.value.status == chx.CHX_EPIVOT
    del rec


# ---------------------------------------------------------------- replays
def replay_chunked(P, coef, f, m):
    """Replay of the chunked solve (chunk sweeps, reduced system, correction)
    with the library's tables; f has shape (n, batch)."""
    rec, blocks, dlo = chx.chx_host_chunk_tables(P, coef, f.shape[0], m)
    n = f.shape[0]
    S, mi = n // m, m - P
    y = np.zeros_like(f)
    pa = np.zeros((S, P, f.shape[1]))
    pb = np.zeros((S, P, f.shape[1]))
    for k in range(S):
        ch = f[k * m:(k + 1) * m].copy()
        g = np.zeros((mi, f.shape[1]))
        for p in range(mi):
            v = ch[p].copy()
            if P == 2 and p >= 2:
                v -= coef[0] * g[p - 2]
            if p >= 1:
                v -= rec[p, 1] * g[p - 1]
            g[p] = v * rec[p, 0]
        yy = np.zeros_like(g)
        for p in range(mi - 1, -1, -1):
            v = g[p].copy()
            if P == 2 and p + 2 < mi:
                v -= rec[p, 3] * yy[p + 2]
            if p + 1 < mi:
                v -= rec[p, 2] * yy[p + 1]
            yy[p] = v
        y[k * m:k * m + mi] = yy
        for a in range(P):
            v = ch[mi + a].copy()
            for p in range(mi + a - P, mi):
                v -= coef[(p - mi - a) + P] * yy[p]
            pa[k, a] = v
            w = np.zeros(f.shape[1])
            for q in range(a + 1):
                w += coef[(q + P - a) + P] * yy[q]
            pb[k, a] = w
    sep = np.zeros((S, P, f.shape[1]))
    for k in range(S):
        for t in range(blocks.shape[0]):
            j = (k + dlo + t) % S
            r = pa[j] - pb[(j + 1) % S]
            sep[k] += blocks[t, :P, :P] @ r
    x = y.copy()
    for k in range(S):
        sp, so = sep[(k - 1) % S], sep[k]
        for p in range(mi):
            x[k * m + p] -= rec[p, 4:4 + P] @ sp + rec[p, 6:6 + P] @ so
        x[k * m + mi:k * m + m] = so
    return x


@pytest.mark.parametrize("n,sigma", [(32, 0.5), (64, 0.17224), (128, 2.7558), (256, 44.092),
                                     (1024, 70.547), (512, 2889.6)])
def test_chunked_replay_matches_oracle_penta(orc, n, sigma):
    f = inputs.uniform(21, (n, 6), -1, 1)
    co = penta(sigma)
    x = replay_chunked(2, co, f, 32)
    ref = np.stack([orc.cyclic_penta_solve(co, f[:, s]) for s in range(f.shape[1])], axis=1)
    # two FP64 direct solvers differ by at most ~ kappa * eps; kappa = 1 + 16 sigma
    tol = max(1e-13, 20 * 2.2e-16 * (1 + 16 * sigma))
    assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) < tol


@pytest.mark.parametrize("n,coef", [(64, (-0.5, 2.0, -0.5)), (96, (-3.0, 7.0, -3.0)),
                                    (32, (0.3, 2.2, -0.6)), (256, (-200.0, 401.0, -200.0))])
def test_chunked_replay_matches_oracle_tri(orc, n, coef):
    f = inputs.uniform(22, (n, 5), -1, 1)
    x = replay_chunked(1, coef, f, 32)
    ref = np.stack([orc.cyclic_tri_solve(coef, f[:, s]) for s in range(f.shape[1])], axis=1)
    assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) < 1e-13


def test_chunked_replay_nonsymmetric_penta(orc):
    co = (0.21, -0.7, 3.9, 0.45, -0.33)
    f = inputs.uniform(23, (96, 4), -1, 1)
    x = replay_chunked(2, co, f, 32)
    ref = np.stack([orc.cyclic_penta_solve(co, f[:, s]) for s in range(4)], axis=1)
    assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) < 1e-13


def replay_whole(P, coef, f, periodic=True):
    rec, minv = chx.chx_host_whole_tables(P, coef, f.shape[0], periodic)
    n = f.shape[0]
    mi = rec.shape[0]
    g = np.zeros(mi)
    q = np.zeros(2)
    for i in range(mi):
        if periodic:
            q += rec[i, 4:6] * f[i]
        v = f[i]
        if P == 2 and i >= 2:
            v -= coef[0] * g[i - 2]
        if i >= 1:
            v -= rec[i, 1] * g[i - 1]
        g[i] = v * rec[i, 0]
    t = np.zeros(2)
    if periodic:
        r = np.array([f[mi] - q[0], (f[mi + 1] - q[1]) if P == 2 else 0.0])
        t = minv @ r
    x = np.zeros(n)
    y1 = y2 = 0.0
    for i in range(mi - 1, -1, -1):
        v = g[i]
        if P == 2:
            v -= rec[i, 3] * y2
        v -= rec[i, 2] * y1
        y2, y1 = y1, v
        x[i] = v - (rec[i, 6] * t[0] + rec[i, 7] * t[1] if periodic else 0.0)
    if periodic:
        x[mi:] = t[:P]
    return x


@pytest.mark.parametrize("n", [5, 6, 7, 13, 100])
def test_whole_replay_matches_oracle(orc, n):
    co = (0.21, -0.7, 3.9, 0.45, -0.33)
    f = inputs.uniform(24, (n,), -1, 1)
    assert np.max(np.abs(replay_whole(2, co, f) - orc.cyclic_penta_solve(co, f))) < 1e-13
    tco = (0.4, 2.5, -0.7)
    assert np.max(np.abs(replay_whole(1, tco, f) - orc.cyclic_tri_solve(tco, f))) < 1e-13


def test_reduced_blocks_are_truncated_below_rounding():
    rec, blocks, dlo = chx.chx_host_chunk_tables(2, penta(2889.6), 8192, 32)
    norms = np.abs(blocks).reshape(blocks.shape[0], -1).max(axis=1)
    assert blocks.shape[0] < 8192 // 32          # truncated
    assert norms.max() == norms[-dlo]              # B_0 is the largest
    assert min(norms[0], norms[-1]) < 1e-12 * norms.max()


def test_per_system_batch_workspace_and_argument_checks(lib):
    """Workspace sizes and host-side rejections of the per-system batched
    solves (no device work is enqueued on any of these paths)."""
    import ctypes
    F, R = chx.CHX_BATCH_FACTOR, chx.CHX_BATCH_REWRITE
    ldw = 128  # 100 systems, rows padded to 32 entries (256 bytes)
    assert chx.penta_batch_ws_bytes(5, 100, True, F) == (4 * 3 + 4) * ldw * 8
    assert chx.penta_batch_ws_bytes(5, 100, True, R) == 4 * 3 * ldw * 8
    assert chx.penta_batch_ws_bytes(5, 100, False, F) == 0
    assert chx.penta_batch_ws_bytes(5, 100, False, R) == 2 * 5 * ldw * 8
    assert chx.tri_batch_ws_bytes(9, 100, True, F) == (2 * 9 + 1) * ldw * 8
    assert chx.tri_batch_ws_bytes(9, 100, True, R) == 2 * 9 * ldw * 8
    assert chx.tri_batch_ws_bytes(9, 100, False, R) == 9 * ldw * 8
    assert chx.penta_batch_ws_bytes(4, 100, True, F) == 0      # below the minimum size
    assert chx.penta_batch_ws_bytes(8, 100, True, 7) == 0      # unknown mode
    p = [ctypes.c_void_p((k + 1) << 20) for k in range(6)]
    ws = ctypes.c_void_p(1 << 32)
    # sizes below the minimum
    assert lib.penta_batch_factor(4, 8, 1, *p[:5], 8, ws, 1 << 20, None) == chx.CHX_EUNSUPPORTED_N
    assert lib.penta_batch_rewrite(2, 8, 0, *p[:5], 8, p[5], ws, 1 << 20, None) == \
        chx.CHX_EUNSUPPORTED_N
    assert lib.tri_batch_rewrite(2, 8, 1, *p[:3], 8, p[5], ws, 1 << 20, None) == \
        chx.CHX_EUNSUPPORTED_N
    assert lib.tri_batch_solve(1, 8, 0, *p[:3], 8, ws, 1 << 20, p[5], None) == \
        chx.CHX_EUNSUPPORTED_N
    # ld < batch, periodic flag not 0/1, NULL arrays
    assert lib.penta_batch_solve(8, 8, 1, *p[:5], 7, ws, 1 << 20, p[5], None) == chx.CHX_EINVAL
    assert lib.penta_batch_solve(8, 8, 2, *p[:5], 8, ws, 1 << 20, p[5], None) == chx.CHX_EINVAL
    assert lib.penta_batch_rewrite(8, 8, 1, *p[:4], None, 8, p[5], ws, 1 << 20, None) == \
        chx.CHX_EINVAL
    assert lib.tri_batch_factor(8, 8, 1, p[0], None, p[2], 8, ws, 1 << 20, None) == chx.CHX_EINVAL
    # workspace missing, misaligned or short
    assert lib.penta_batch_factor(8, 8, 1, *p[:5], 8, None, 1 << 20, None) == chx.CHX_EINVAL
    assert lib.penta_batch_factor(8, 8, 1, *p[:5], 8, ctypes.c_void_p((1 << 32) + 8), 1 << 20,
                                  None) == chx.CHX_EINVAL
    need = chx.penta_batch_ws_bytes(8, 8, True, R)
    assert lib.penta_batch_rewrite(8, 8, 1, *p[:5], 8, p[5], ws, need - 8, None) == chx.CHX_ENOMEM
    need = chx.tri_batch_ws_bytes(8, 8, True, F)
    assert lib.tri_batch_solve(8, 8, 1, *p[:3], 8, ws, need - 8, p[5], None) == chx.CHX_ENOMEM


def test_ensemble_extras_reject_bad_arguments_on_host(lib):
    """The ensemble's forcing and per-run measures check their arguments before
    any device work."""
    import ctypes
    u = ctypes.c_uint64()
    d = (ctypes.c_double * 3)()
    assert lib.ch_ensemble_set_noise(None, 1e-10, None, 0) == chx.CHX_EINVAL
    assert lib.ch_ensemble_get_noise_step(None, ctypes.byref(u)) == chx.CHX_EINVAL
    assert lib.ch_ensemble_moments(None, None, None, d, None) == chx.CHX_EINVAL
    assert lib.ch_ensemble_k1(None, None, None, d, None) == chx.CHX_EINVAL
    assert lib.ch_ensemble_step(None, None, None, 1, None, None, 0, 0, None) == chx.CHX_EINVAL
    v = ctypes.c_int()
    assert lib.ch_ensemble_get_tuning(None, 0, ctypes.byref(v)) == chx.CHX_EINVAL
    assert lib.ch_ensemble_set_tuning(None, 0, 0) == chx.CHX_EINVAL


def test_decay_rate_rejects_bad_arguments_on_host(lib):
    """Too few states, a non-positive dt and overlapping buffers are refused
    before anything is launched (the pointers are never dereferenced)."""
    import ctypes
    p = ctypes.c_void_p(1 << 20)
    q = ctypes.c_void_p(1 << 30)
    assert lib.ch_energy_decay_rate(p, 1, 2, 0.0, 0.1, q, None) == chx.CHX_EINVAL
    assert lib.ch_energy_decay_rate(p, 1, 8, 0.0, 0.0, q, None) == chx.CHX_EINVAL
    assert lib.ch_energy_decay_rate(p, 1, 8, 0.0, 0.1, None, None) == chx.CHX_EINVAL
    inside = ctypes.c_void_p((1 << 20) + 64)  # within the 16 doubles of diag
    assert lib.ch_energy_decay_rate(p, 1, 8, 0.0, 0.1, inside, None) == chx.CHX_EINVAL


def test_stencil_binding_rejects_mismatched_layouts():
    """One leading dimension serves input and output: a padded input with a
    packed output (or any other mismatch) is refused before the library is
    called."""
    import torch
    from paper_2101_06550_amd import chx
    big = torch.zeros((8, 16), dtype=torch.float64)
    w = [1.0] * 9
    with pytest.raises(chx.ChxError, match="leading dimension"):
        chx.stencil2d_apply(big[:, :10], torch.zeros((8, 10), dtype=torch.float64), w, 1, 1, 1, 1)
    with pytest.raises(chx.ChxError, match="leading dimension"):
        chx.stencil2d_apply(torch.zeros((8, 10), dtype=torch.float64), big[:, :10], w, 1, 1, 1, 1)
    with pytest.raises(chx.ChxError, match="shape of inp"):
        chx.stencil2d_apply(torch.zeros((8, 10), dtype=torch.float64),
                            torch.zeros((8, 11), dtype=torch.float64), w, 1, 1, 1, 1)
    with pytest.raises(chx.ChxError, match="leading dimension"):  # column-strided view
        chx.stencil2d_apply(big[:, ::2], torch.zeros((8, 8), dtype=torch.float64), w, 1, 1, 1, 1)
    with pytest.raises(chx.ChxError, match="float64 or both float32"):
        chx.stencil2d_apply(torch.zeros((8, 10), dtype=torch.float64),
                            torch.zeros((8, 10), dtype=torch.float32), w, 1, 1, 1, 1)


class _FakeHandle:
    """Stand-in for a CH handle: the binding's argument checks read only the
    grid shape; every call below is refused before the library is reached."""

    def __init__(self, nx, ny):
        from paper_2101_06550_amd import chx
        self.params = chx.ChParams(nx, ny, 1.0, 1.0, 1.0, 0.01, 1e-4, 0, 0, 0)
        self.handle = None
        self._ws = None


@pytest.mark.parametrize("call", ["ch_adi_step", "ch_adi_step_timed", "ch_diagnostics",
                                  "ch_moments", "ch_k1"])
def test_step_binding_rejects_fields_that_do_not_fit(call):
    """A field whose rows (ny of them, ld apart, nx used) do not lie inside the
    tensor, or that is not row-major, is refused before any kernel could read
    or write past it."""
    import torch
    from paper_2101_06550_amd import chx
    h = _FakeHandle(64, 32)
    fn = getattr(chx, call)
    f64 = torch.float64
    with pytest.raises(chx.ChxError, match=r"\(32, >= 64\)"):  # too few rows
        fn(h, torch.zeros((31, 64), dtype=f64))
    with pytest.raises(chx.ChxError, match=r"\(32, >= 64\)"):  # too few columns
        fn(h, torch.zeros((32, 63), dtype=f64))
    with pytest.raises(chx.ChxError, match=r"\(32, >= 64\)"):  # flat buffer
        fn(h, torch.zeros(64 * 32, dtype=f64))
    with pytest.raises(chx.ChxError, match="unit column stride"):
        fn(h, torch.zeros((32, 128), dtype=f64)[:, ::2])
    with pytest.raises(chx.ChxError, match="leading dimension"):  # ld below nx
        fn(h, torch.zeros((32, 64), dtype=f64), ld=32)
    with pytest.raises(chx.ChxError, match="leading dimension"):  # ld not the row stride
        fn(h, torch.zeros((32, 64), dtype=f64), ld=80)
    with pytest.raises(chx.ChxError, match="device tensor"):  # shape fine: only the device
        fn(h, torch.zeros((32, 80), dtype=f64))


def test_step_binding_rejects_short_diagnostics_and_bad_pairs():
    import torch
    from paper_2101_06550_amd import chx
    h = _FakeHandle(64, 32)
    c = torch.zeros((32, 64), dtype=torch.float64)
    for call in (chx.ch_adi_step, chx.ch_adi_step_timed):
        with pytest.raises(chx.ChxError, match=">= 8 values"):  # 3 steps: 2 * 4 values
            call(h, c, nsteps=3, diag_out=torch.zeros(7, dtype=torch.float64))
        with pytest.raises(chx.ChxError, match="contiguous"):
            call(h, c, nsteps=1, diag_out=torch.zeros(8, dtype=torch.float64)[::2])
    with pytest.raises(chx.ChxError, match=r"cprev must be a \(32, >= 64\)"):
        chx.ch_adi_step_p2(h, c, torch.zeros((16, 64), dtype=torch.float64))
    with pytest.raises(chx.ChxError, match="one leading dimension"):
        chx.ch_adi_step_p2(h, c, torch.zeros((32, 72), dtype=torch.float64))
    with pytest.raises(chx.ChxError, match=">= 6 values"):
        chx.ch_adi_step_p2(h, c, c.clone(), nsteps=2, diag_out=torch.zeros(5, dtype=torch.float64))


def test_ensemble_binding_checks_every_run():
    import torch
    from paper_2101_06550_amd import chx
    e = chx.Ensemble.__new__(chx.Ensemble)  # shapes only; the library is never reached
    e.handle, e.nruns, e.shapes, e._ws = None, 2, [(64, 32), (128, 64)], None
    ok0 = torch.zeros((32, 64), dtype=torch.float64)
    with pytest.raises(chx.ChxError, match=r"field 1 must be a \(64, >= 128\)"):
        chx.ch_ensemble_step(e, [ok0, torch.zeros((64, 64), dtype=torch.float64)])
    with pytest.raises(chx.ChxError, match="one field per run"):
        chx.ch_ensemble_step(e, [ok0])
    with pytest.raises(chx.ChxError, match=r"field 1 must be a"):
        chx.ch_ensemble_moments(e, [ok0, ok0])
    e.handle = None


def test_solve_binding_rejects_short_buffers():
    import torch
    from paper_2101_06550_amd import chx

    class P:
        handle, n = None, 64

    x = torch.zeros(64 * 100 - 1, dtype=torch.float64)  # one element short of (n - 1) 100 + 100
    with pytest.raises(chx.ChxError, match="storage holds fewer"):
        chx.penta_solve_batch(P(), 100, x, ld=100, layout=chx.CHX_INTERLEAVED)
    with pytest.raises(chx.ChxError, match="storage holds fewer"):
        chx.tri_solve_batch(P(), 100, x, ld=64, layout=chx.CHX_CONTIGUOUS)
    with pytest.raises(chx.ChxError, match="unit last stride"):
        chx.penta_solve_batch(P(), 10, torch.zeros((64, 40), dtype=torch.float64)[:, ::2],
                              ld=40)
