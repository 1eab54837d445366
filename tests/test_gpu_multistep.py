"""GPU parity of several ADI steps in one call on the multi-kernel path
against the oracle's time loop (Ch.3 eq. 3:ch_adi advanced step after step).

Every step after the first of such a call applies the previous step's
column-chunk correction while it reads the state (the deferred correction of
the chunked column solve, Ch.4 bordering across 32-row chunks), and the call
ends with the correction written into the caller's array.  These cases cover
grids with several chunks and several 256-column blocks of the column pass,
a ragged last block of one wave, two chunks (the wrap chunk is both
neighbours), the benchmark's 8192^2 launch configuration, the forced step,
and the per-step diagnostics of every state against the oracle's."""
import math

import numpy as np
import pytest

from paper_2101_06550_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
L = 2 * math.pi


@pytest.fixture(scope="module")
def chx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_06550_amd import chx as m
    m.load()
    return m


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def oracle_states(orc, c0, g, dt, k):
    """The oracle's states after 0, 1, ..., k steps."""
    out = [c0]
    for _ in range(k):
        out.append(orc.ch_step(out[-1], L, L, 1.0, g, dt))
    return out


# (ny, nx, gamma, dt, steps, seed): chunks = ny / 32, column blocks = nx / 256 (ragged: nx % 256)
CASES = [(1024, 1024, 0.01, 1e-5, 3, 61),   # 32 chunks x 4 blocks
         (96, 320, 0.01, 1e-4, 3, 62),      # 3 chunks, last block one wave
         (160, 576, 0.01, 1e-4, 4, 63),     # 5 chunks, last block one wave
         (64, 2048, 0.01, 1e-5, 3, 64),     # 2 chunks: the wrap chunk is both neighbours
         (256, 448, 0.01, 1e-4, 5, 65)]     # 8 chunks, last block three waves


@pytest.mark.parametrize("ny,nx,g,dt,k,seed", CASES)
def test_steps_in_one_call_match_oracle(chx, orc, ny, nx, g, dt, k, seed):
    c0 = inputs.noise_field(ny, nx, seed)
    h = chx.ch_create(nx, ny, L, L, 1.0, g, dt)
    chx.ch_set_tuning(h, 0, what=chx.CHX_TUNE_SMALL_PATH)  # the multi-kernel path
    c = torch.tensor(c0, device="cuda")
    d = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
    print(f"[case] {k} steps in one call {ny}x{nx}", flush=True)
    chx.ch_adi_step(h, c, nsteps=k, diag_out=d)
    torch.cuda.synchronize()
    ref = oracle_states(orc, c0, g, dt, k)
    err = rel(c.cpu().numpy(), ref[k])
    assert err < k * 1e-12, f"{k} steps: {err:.3e}"
    dd = d.cpu().numpy().reshape(k + 1, 2)
    l1 = np.sum(np.abs(c0)) * (L / nx) * (L / ny)
    for j in range(k + 1):  # mass and free energy of every state of the call
        m, e = orc.ch_mass(ref[j], L, L), orc.ch_energy(ref[j], L, L, g)
        assert abs(dd[j, 0] - m) <= 1e-12 * l1, (j, dd[j, 0], m)
        assert abs(dd[j, 1] - e) <= max(j, 1) * 1e-12 * abs(e), (j, dd[j, 1], e)


def test_every_row_order_matches_oracle_over_steps(chx, orc):
    """Rows of 8192 points (the benchmark's row length): every row-pass order
    the tuner may pick, three steps in one call, against the oracle."""
    ny, nx, g, dt, k = 96, 8192, 0.001, 1e-6, 3
    c0 = inputs.noise_field(ny, nx, 66)
    h = chx.ch_create(nx, ny, L, L, 1.0, g, dt)
    for w in (chx.CHX_TUNE_COLUMN_CHUNK, chx.CHX_TUNE_ROW_CHUNK):  # split forms need 32
        chx.ch_set_tuning(h, 32, what=w)
    ref = oracle_states(orc, c0, g, dt, k)[k]
    for split in [-1, chx.CHX_ROW_SPLIT_OVERLAP] + list(range(chx.CHX_NUM_SPLIT_SHAPES)):
        print(f"[case] row order {split}, {k} steps {ny}x{nx}", flush=True)
        chx.ch_set_tuning(h, split, what=chx.CHX_TUNE_ROW_SPLIT)
        c = torch.tensor(c0, device="cuda")
        chx.ch_adi_step(h, c, nsteps=k)
        torch.cuda.synchronize()
        err = rel(c.cpu().numpy(), ref)
        assert err < k * 1e-12, f"row order {split}: {err:.3e}"


@pytest.mark.parametrize("mchunk", [32, 16])
def test_forced_steps_in_one_call_match_oracle(chx, orc, mchunk):
    """Cahn-Hilliard-Cook forcing drawn inside the column pass of every step,
    three steps in one call on the multi-kernel path, with 32- and 16-point
    chunks in both directions."""
    ny = nx = 1024
    dt, sigma, k = 1e-5, 1e-12, 3
    c0 = inputs.noise_field(ny, nx, 67)
    h = chx.ch_create(nx, ny, L, L, 1.0, 0.01, dt)
    chx.ch_set_tuning(h, -1, what=chx.CHX_TUNE_ROW_SPLIT)
    for w in (chx.CHX_TUNE_COLUMN_CHUNK, chx.CHX_TUNE_ROW_CHUNK):
        chx.ch_set_tuning(h, mchunk, what=w)
    chx.ch_set_noise(h, sigma, seed=91, step0=4)
    c = torch.tensor(c0, device="cuda")
    print(f"[case] forced 3 steps 1024x1024 chunks {mchunk}", flush=True)
    chx.ch_adi_step(h, c, nsteps=k)
    torch.cuda.synchronize()
    ref = orc.ch_step_cook(c0, L, L, 1.0, 0.01, dt, sigma, 91, step0=4, nsteps=k)
    err = rel(c.cpu().numpy(), ref)
    assert err < k * 1e-12, f"forced {k} steps: {err:.3e}"
    assert rel(orc.ch_step(c0, L, L, 1.0, 0.01, dt, nsteps=k), ref) > 1e-9  # forcing matters


def test_large_run_two_steps_in_one_call(chx, orc):
    """8192 x 8192 in the benchmark's configuration (gamma = 0.001, dt = 1e-6,
    c0 = 0.05 sin 3x sin 5y + noise, tuned kernel shapes): two steps in one
    call, every point against the oracle's two steps, and both states'
    diagnostics."""
    n, g, dt, k = 8192, 0.001, 1e-6, 2
    c0 = inputs.mode_plus_noise(n, 5)
    h = chx.ch_create(n, n, L, L, 1.0, g, dt)
    c = torch.tensor(c0, device="cuda")
    d = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
    print("[case] 8192x8192 two steps in one call", flush=True)
    chx.ch_adi_step(h, c, nsteps=k, diag_out=d)
    torch.cuda.synchronize()
    out = c.cpu().numpy()
    del c
    ref = oracle_states(orc, c0, g, dt, k)
    err = rel(out, ref[k])
    print(f"8192^2 two-step error {err:.3e}", flush=True)
    assert err < k * 1e-12, f"two steps: {err:.3e}"
    dd = d.cpu().numpy().reshape(k + 1, 2)
    l1 = np.sum(np.abs(c0)) * (L / n) ** 2
    for j in range(k + 1):
        m, e = orc.ch_mass(ref[j], L, L), orc.ch_energy(ref[j], L, L, g)
        assert abs(dd[j, 0] - m) <= 1e-12 * l1, (j, dd[j, 0], m)
        assert abs(dd[j, 1] - e) <= 1e-12 * abs(e), (j, dd[j, 1], e)


@pytest.mark.parametrize("ny,nx", [(1024, 1024), (96, 320), (160, 576)])
def test_column_orders_bitwise_and_match_oracle(chx, orc, ny, nx):
    """Every tile order of the column pass (and of the pass that writes the
    final state): the same sums in the same order, so bitwise identical
    states and diagnostics, including tile counts that are not a multiple of
    the 8 XCDs (96 x 320: 2 x 3 tiles; 160 x 576: 3 x 5)."""
    g, dt, k = 0.01, 1e-5, 3
    c0 = inputs.noise_field(ny, nx, 68)
    h = chx.ch_create(nx, ny, L, L, 1.0, g, dt)
    chx.ch_set_tuning(h, 0, what=chx.CHX_TUNE_SMALL_PATH)
    outs = []
    for order in range(chx.CHX_NUM_COLUMN_ORDERS):
        print(f"[case] column order {order}, {k} steps {ny}x{nx}", flush=True)
        chx.ch_set_tuning(h, order, what=chx.CHX_TUNE_COLUMN_ORDER)
        assert chx.ch_get_tuning(h, chx.CHX_TUNE_COLUMN_ORDER) == order
        c = torch.tensor(c0, device="cuda")
        d = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
        chx.ch_adi_step(h, c, nsteps=k, diag_out=d)
        torch.cuda.synchronize()
        outs.append((c.cpu().numpy(), d.cpu().numpy()))
    for c, d in outs[1:]:
        assert np.array_equal(c, outs[0][0]) and np.array_equal(d, outs[0][1])
    ref = oracle_states(orc, c0, g, dt, k)
    assert rel(outs[0][0], ref[k]) < k * 1e-12
    with pytest.raises(chx.ChxError):
        chx.ch_set_tuning(h, chx.CHX_NUM_COLUMN_ORDERS, what=chx.CHX_TUNE_COLUMN_ORDER)


# (ny, nx): 16-point chunks = ny / 16 down the columns, nx / 16 along the rows
# (gamma dt / dx^4 kept moderate: the row systems of 4096 points at gamma =
# 0.01, dt = 1e-5 have condition numbers near 3e5, and either chunk length
# then misses the 1e-12 bound by rounding alone)
CHUNK_CASES = [(1024, 1024, 0.01, 1e-5, 3, 71),   # 64 x 64 short chunks, 4 column blocks
               (96, 320, 0.01, 1e-5, 3, 72),      # 6 x 20, last column block one wave
               (64, 2048, 0.01, 1e-5, 2, 73),     # 4 x 128
               (160, 576, 0.01, 1e-5, 4, 74),     # 10 x 36, last block one wave
               (288, 4096, 0.001, 1e-6, 2, 75)]   # 18 x 256: the longest row of 16-point chunks


@pytest.mark.parametrize("ny,nx,g,dt,k,seed", CHUNK_CASES)
def test_chunk_lengths_match_oracle(chx, orc, ny, nx, g, dt, k, seed):
    """CHX_TUNE_COLUMN_CHUNK / CHX_TUNE_ROW_CHUNK: 32- and 16-point chunks in
    each direction (the 16-point separator system has twice the separators
    and its own decay window), several steps in one call with the deferred
    column correction and the per-step diagnostics, against the oracle; the
    four choices agree to rounding."""
    c0 = inputs.noise_field(ny, nx, seed)
    h = chx.ch_create(nx, ny, L, L, 1.0, g, dt)
    chx.ch_set_tuning(h, 0, what=chx.CHX_TUNE_SMALL_PATH)
    chx.ch_set_tuning(h, -1, what=chx.CHX_TUNE_ROW_SPLIT)
    ref = oracle_states(orc, c0, g, dt, k)
    l1 = np.sum(np.abs(c0)) * (L / nx) * (L / ny)
    for mc in (32, 16):
        for mr in (32, 16):
            print(f"[case] chunks {mc}/{mr}, {k} steps {ny}x{nx}", flush=True)
            chx.ch_set_tuning(h, mc, what=chx.CHX_TUNE_COLUMN_CHUNK)
            chx.ch_set_tuning(h, mr, what=chx.CHX_TUNE_ROW_CHUNK)
            assert chx.ch_get_tuning(h, chx.CHX_TUNE_COLUMN_CHUNK) == mc
            assert chx.ch_get_tuning(h, chx.CHX_TUNE_ROW_CHUNK) == mr
            c = torch.tensor(c0, device="cuda")
            d = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
            chx.ch_adi_step(h, c, nsteps=k, diag_out=d)
            torch.cuda.synchronize()
            err = rel(c.cpu().numpy(), ref[k])
            assert err < k * 1e-12, f"chunks {mc}/{mr}: {err:.3e}"
            dd = d.cpu().numpy().reshape(k + 1, 2)
            for j in range(k + 1):
                m, e = orc.ch_mass(ref[j], L, L), orc.ch_energy(ref[j], L, L, g)
                assert abs(dd[j, 0] - m) <= 1e-12 * l1, (mc, mr, j, dd[j, 0], m)
                assert abs(dd[j, 1] - e) <= max(j, 1) * 1e-12 * abs(e), (mc, mr, j)


@pytest.mark.parametrize("ny,nx,seed", [(1024, 1024, 81), (96, 320, 82), (160, 576, 83),
                                        (64, 2048, 84)])
def test_overlapped_row_order_any_chunk_lengths(chx, orc, ny, nx, seed):
    """CHX_ROW_SPLIT_OVERLAP for every chunk-length pair: the separator rows on
    the handle's second stream beside the interior rows, in row groups that
    span column chunks (groups of R = 256 / S rows of the 14- or 30-row
    interiors, ragged last groups); bitwise equal to the plain order, three
    steps with diagnostics, and against the oracle."""
    g, dt, k = 0.01, 1e-5, 3
    c0 = inputs.noise_field(ny, nx, seed)
    h = chx.ch_create(nx, ny, L, L, 1.0, g, dt)
    chx.ch_set_tuning(h, 0, what=chx.CHX_TUNE_SMALL_PATH)
    ref = oracle_states(orc, c0, g, dt, k)[k]
    for mc in (32, 16):
        for mr in (32, 16):
            outs = []
            for split in (-1, chx.CHX_ROW_SPLIT_OVERLAP):
                print(f"[case] row order {split} chunks {mc}/{mr} {ny}x{nx}", flush=True)
                chx.ch_set_tuning(h, -1, what=chx.CHX_TUNE_ROW_SPLIT)
                chx.ch_set_tuning(h, mc, what=chx.CHX_TUNE_COLUMN_CHUNK)
                chx.ch_set_tuning(h, mr, what=chx.CHX_TUNE_ROW_CHUNK)
                chx.ch_set_tuning(h, split, what=chx.CHX_TUNE_ROW_SPLIT)
                c = torch.tensor(c0, device="cuda")
                d = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
                chx.ch_adi_step(h, c, nsteps=k, diag_out=d)
                torch.cuda.synchronize()
                outs.append((c.cpu().numpy(), d.cpu().numpy()))
            assert np.array_equal(outs[0][0], outs[1][0]), (mc, mr)
            assert np.array_equal(outs[0][1], outs[1][1]), (mc, mr)
            assert rel(outs[1][0], ref) < k * 1e-12, (mc, mr)


def test_chunk_length_choices_refused_where_they_do_not_apply(chx):
    """16-point rows need at most 256 chunks (4096 points); any chunk other
    than 16 or 32 is refused; 16 and the fused split row forms exclude each
    other (the overlapped order takes either)."""
    h = chx.ch_create(8192, 96, L, L, 1.0, 0.001, 1e-6)
    for w in (chx.CHX_TUNE_COLUMN_CHUNK, chx.CHX_TUNE_ROW_CHUNK):
        chx.ch_set_tuning(h, 32, what=w)
    with pytest.raises(chx.ChxError):
        chx.ch_set_tuning(h, 16, what=chx.CHX_TUNE_ROW_CHUNK)  # 512 chunks a row
    for bad in (0, 8, 24, 64):
        for w in (chx.CHX_TUNE_COLUMN_CHUNK, chx.CHX_TUNE_ROW_CHUNK):
            with pytest.raises(chx.ChxError):
                chx.ch_set_tuning(h, bad, what=w)
    chx.ch_set_tuning(h, 0, what=chx.CHX_TUNE_ROW_SPLIT)
    with pytest.raises(chx.ChxError):
        chx.ch_set_tuning(h, 16, what=chx.CHX_TUNE_COLUMN_CHUNK)
    chx.ch_set_tuning(h, -1, what=chx.CHX_TUNE_ROW_SPLIT)
    chx.ch_set_tuning(h, 16, what=chx.CHX_TUNE_COLUMN_CHUNK)
    with pytest.raises(chx.ChxError):
        chx.ch_set_tuning(h, 0, what=chx.CHX_TUNE_ROW_SPLIT)
    chx.ch_set_tuning(h, chx.CHX_ROW_SPLIT_OVERLAP, what=chx.CHX_TUNE_ROW_SPLIT)  # any length


@pytest.mark.parametrize("ny,nx,dtype,passes", [(1024, 1024, 0, 0), (96, 320, 0, 0),
                                                (256, 448, 1, 2)])
def test_graph_replays_match_eager(chx, ny, nx, dtype, passes):
    """CHX_TUNE_GRAPH: the call captured once and replayed several times, with
    eager calls of another handle and synchronisations between the replays;
    every replay bitwise equal to the eager handle's result, the diagnostics
    too; a new field pointer is re-captured and the old field left alone."""
    g, dt, k = 0.01, 1e-5, 3
    c0 = inputs.noise_field(ny, nx, 69)
    hg = chx.ch_create(nx, ny, L, L, 1.0, g, dt, dtype=dtype, refine_passes=passes)
    he = chx.ch_create(nx, ny, L, L, 1.0, g, dt, dtype=dtype, refine_passes=passes)
    for h in (hg, he):  # the multi-kernel path, same choices on both
        if dtype == 0:
            chx.ch_set_tuning(h, 0, what=chx.CHX_TUNE_SMALL_PATH)
    chx.ch_set_tuning(hg, 1, what=chx.CHX_TUNE_GRAPH)
    assert chx.ch_get_tuning(hg, chx.CHX_TUNE_GRAPH) == 1
    ws = torch.empty(chx.ch_ws_bytes(hg), dtype=torch.uint8, device="cuda")
    cg = torch.tensor(c0, device="cuda")
    ce = torch.tensor(c0, device="cuda")
    dg = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
    de = torch.zeros_like(dg)
    for rep in range(4):
        print(f"[case] graph replay {rep} {ny}x{nx} dtype={dtype}", flush=True)
        chx.ch_adi_step(hg, cg, nsteps=k, diag_out=dg, ws=ws)
        chx.ch_adi_step(he, ce, nsteps=k, diag_out=de)
        torch.cuda.synchronize()
        assert torch.equal(cg, ce), rep
        assert torch.equal(dg, de), rep
    other = torch.tensor(c0, device="cuda")
    keep = cg.clone()
    chx.ch_adi_step(hg, other, nsteps=k, diag_out=dg, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(cg, keep)
    ref = torch.tensor(c0, device="cuda")
    chx.ch_adi_step(he, ref, nsteps=k)
    torch.cuda.synchronize()
    assert torch.equal(other, ref)


def test_tuning_cache_file_is_reused_across_processes(tmp_path):
    """The autotuned choices of a size go to the tuning cache file once; a
    second process reads them back (the file keeps one line) and picks the
    same choices; results are bitwise identical whatever was chosen."""
    import os
    import subprocess
    import sys
    cache = tmp_path / "tuning.txt"
    code = ("import math, sys; sys.path.insert(0, %r); "
            "from paper_2101_06550_amd import chx; chx.load(); "
            "h = chx.ch_create(2048, 1024, 2 * math.pi, 2 * math.pi, 1.0, 0.01, 1e-5); "
            "print([chx.ch_get_tuning(h, w) for w in (0, 2, 3, 5, 6)])") % os.getcwd()
    env = dict(os.environ, CHX_TUNE_CACHE=str(cache))
    env.pop("CHX_AUTOTUNE", None)
    outs = []
    for run in range(2):
        print(f"[case] tuning cache process {run}", flush=True)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(r.stdout.strip().splitlines()[-1])
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and lines[0].startswith("chx-tune-3 gfx"), lines
        assert " 2048 1024 " in lines[0]
    assert outs[0] == outs[1]
    assert lines[0].split()[-5:] == [v.strip() for v in outs[0].strip("[]").split(",")]
