"""GPU parity of the Cahn-Hilliard-Cook forcing (Ch.7) against the oracle:
the same counter-based draws on both sides, the forced step, the counter
carried across calls, mass conservation, and sigma = 0 equal to the unforced
step."""
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


@pytest.mark.parametrize("ny,nx,dt,sigma", [(128, 128, 1e-4, 1e-10), (256, 128, 1e-4, 1e-8),
                                            (96, 192, 1e-4, 1e-10), (1024, 1024, 1e-5, 1e-12)])
def test_forced_steps_match_oracle(chx, orc, ny, nx, dt, sigma):
    c0 = inputs.noise_field(ny, nx, 31)
    h = chx.ch_create(nx, ny, L, L, 1.0, 0.01, dt)
    chx.ch_set_noise(h, sigma, seed=77, step0=5)
    c = torch.tensor(c0, device="cuda")
    print(f"[case] cook {ny}x{nx} sigma={sigma}", flush=True)
    chx.ch_adi_step(h, c, nsteps=1)
    torch.cuda.synchronize()
    ref = orc.ch_step_cook(c0, L, L, 1.0, 0.01, dt, sigma, 77, step0=5)
    assert rel(c.cpu().numpy(), ref) < 1e-12
    assert chx.ch_get_noise_step(h) == 6
    # the forcing is not negligible in this test
    assert rel(orc.ch_step(c0, L, L, 1.0, 0.01, dt), ref) > 1e-9


def test_counter_carries_across_calls(chx, orc):
    c0 = inputs.noise_field(128, 128, 32)
    h = chx.ch_create(128, 128, L, L, 1.0, 0.01, 1e-4)
    chx.ch_set_noise(h, 1e-10, seed=3)
    a = torch.tensor(c0, device="cuda")
    d = torch.zeros(12, dtype=torch.float64, device="cuda")
    chx.ch_adi_step(h, a, nsteps=5, diag_out=d)
    chx.ch_set_noise(h, 1e-10, seed=3, step0=0)
    b = torch.tensor(c0, device="cuda")
    chx.ch_adi_step(h, b, nsteps=2)
    chx.ch_adi_step(h, b, nsteps=3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref = orc.ch_step_cook(c0, L, L, 1.0, 0.01, 1e-4, 1e-10, 3, step0=0, nsteps=5)
    assert rel(a.cpu().numpy(), ref) < 1e-11
    dd = d.cpu().numpy().reshape(6, 2)
    l1 = np.sum(np.abs(c0)) * (L / 128) ** 2
    assert np.max(np.abs(dd[:, 0] - dd[0, 0])) < 1e-12 * l1


def test_zero_intensity_is_the_unforced_step(chx):
    c0 = inputs.noise_field(256, 256, 33)
    h = chx.ch_create(256, 256, L, L, 1.0, 0.01, 1e-4)
    plain = torch.tensor(c0, device="cuda")
    chx.ch_adi_step(h, plain, nsteps=3)
    w0 = chx.ch_ws_bytes(h)
    chx.ch_set_noise(h, 1e-10, seed=1)
    assert chx.ch_ws_bytes(h) == w0  # the draws are made inside the kernels
    chx.ch_set_noise(h, 0.0)
    assert chx.ch_ws_bytes(h) == w0
    again = torch.tensor(c0, device="cuda")
    chx.ch_adi_step(h, again, nsteps=3)
    torch.cuda.synchronize()
    assert torch.equal(plain, again)


def test_noise_arguments_rejected(chx):
    h = chx.ch_create(128, 128, L, L, 1.0, 0.01, 1e-4)
    with pytest.raises(chx.ChxError):
        chx.ch_set_noise(h, -1.0)
    for bad in (chx.ch_create(80, 72, L, L, 1.0, 0.01, 1e-4),
                chx.ch_create(128, 128, L, L, 1.0, 0.01, 1e-4, scheme=chx.CHX_SCHEME_P2),
                chx.ch_create(128, 128, L, L, 1.0, 0.01, 1e-4, dtype=chx.CHX_F32_REFINED,
                              refine_passes=1)):
        with pytest.raises(chx.ChxError):
            chx.ch_set_noise(bad, 1e-10)


# runs of an ensemble: single-workgroup sizes and multi-kernel sizes
ENS_RUNS = [(64, 64, 1.0, 0.01, 1e-4), (128, 128, 1.0, 0.01, 1e-4), (256, 256, 1.0, 0.01, 1e-4),
            (256, 128, 1.0, 0.02, 5e-5), (512, 256, 1.0, 0.01, 1e-4)]
SIGMA = 1e-10


def _ens(chx):
    return chx.ch_ensemble_create([(nx, ny, L, L, D, g, dt) for (nx, ny, D, g, dt) in ENS_RUNS])


def test_ensemble_forcing_matches_oracle_and_single_runs(chx, orc):
    """Every run of a forced ensemble gets the draws of a single handle with
    its seed: one step against the oracle, and several steps (graph replays,
    the counter carried across calls) bit for bit against single handles."""
    seeds = [101, 202, 303, 404, 505]
    c0 = [inputs.noise_field(ny, nx, 60 + r) for r, (nx, ny, *_) in enumerate(ENS_RUNS)]
    ens = _ens(chx)
    chx.ch_ensemble_set_noise(ens, SIGMA, seeds, step0=7)
    f = [torch.tensor(c, device="cuda") for c in c0]
    print("[case] forced ensemble one step", flush=True)
    chx.ch_ensemble_step(ens, f, nsteps=1, use_graph=False)
    torch.cuda.synchronize()
    assert chx.ch_ensemble_get_noise_step(ens) == 8
    for (nx, ny, D, g, dt), c, t, sd in zip(ENS_RUNS, c0, f, seeds):
        ref = orc.ch_step_cook(c, L, L, D, g, dt, SIGMA, sd, step0=7)
        assert rel(t.cpu().numpy(), ref) < 1e-12, (nx, ny)
        assert rel(orc.ch_step(c, L, L, D, g, dt), ref) > 1e-10, (nx, ny)  # forcing visible
    print("[case] forced ensemble graph replays vs single handles", flush=True)
    for rep in range(3):
        chx.ch_ensemble_step(ens, f, nsteps=2, use_graph=True)
    torch.cuda.synchronize()
    assert chx.ch_ensemble_get_noise_step(ens) == 14
    for r, ((nx, ny, D, g, dt), c) in enumerate(zip(ENS_RUNS, c0)):
        h = chx.ch_create(nx, ny, L, L, D, g, dt)
        for w in (chx.CHX_TUNE_COLUMN_CHUNK, chx.CHX_TUNE_ROW_CHUNK):  # the ensemble's chunks
            chx.ch_set_tuning(h, 32, what=w)
        chx.ch_set_noise(h, SIGMA, seed=seeds[r], step0=7)
        s = torch.tensor(c, device="cuda")
        chx.ch_adi_step(h, s, nsteps=1)
        for rep in range(3):
            chx.ch_adi_step(h, s, nsteps=2)
        torch.cuda.synchronize()
        assert torch.equal(s, f[r]), (nx, ny)


def test_ensemble_forcing_off_equals_unforced(chx):
    c0 = [inputs.noise_field(ny, nx, 70 + r) for r, (nx, ny, *_) in enumerate(ENS_RUNS)]
    a = _ens(chx)
    b = _ens(chx)
    chx.ch_ensemble_set_noise(b, SIGMA, [1] * len(ENS_RUNS))
    chx.ch_ensemble_set_noise(b, 0.0)
    fa = [torch.tensor(c, device="cuda") for c in c0]
    fb = [torch.tensor(c, device="cuda") for c in c0]
    print("[case] ensemble forcing switched off", flush=True)
    chx.ch_ensemble_step(a, fa, nsteps=3)
    chx.ch_ensemble_step(b, fb, nsteps=3)
    torch.cuda.synchronize()
    for x, y in zip(fa, fb):
        assert torch.equal(x, y)
    with pytest.raises(chx.ChxError):
        chx.ch_ensemble_set_noise(a, -1.0, [1] * len(ENS_RUNS))


def test_forced_ensemble_conserves_mass(chx, orc):
    c0 = [inputs.noise_field(ny, nx, 80 + r) for r, (nx, ny, *_) in enumerate(ENS_RUNS)]
    ens = _ens(chx)
    chx.ch_ensemble_set_noise(ens, 1e-8, [9, 8, 7, 6, 5])
    f = [torch.tensor(c, device="cuda") for c in c0]
    n = 20
    d = torch.zeros(len(ENS_RUNS) * 2 * (n + 1), dtype=torch.float64, device="cuda")
    print("[case] forced ensemble mass", flush=True)
    chx.ch_ensemble_step(ens, f, nsteps=n, diag_out=d)
    torch.cuda.synchronize()
    dd = d.cpu().numpy().reshape(len(ENS_RUNS), n + 1, 2)
    for r, c in enumerate(c0):
        scale = np.sum(np.abs(c)) * (L / c.shape[1]) * (L / c.shape[0])
        assert abs(dd[r, -1, 0] - dd[r, 0, 0]) < 1e-12 * scale, r


def test_forced_large_run_one_step(chx, orc):
    """The benchmark's forced workload (8192^2, gamma = 0.001, dt = 1e-6,
    sigma = 1e-14, seed 2021) for one step against the oracle."""
    n = 8192
    c0 = inputs.mode_plus_noise(n, 5)
    h = chx.ch_create(n, n, L, L, 1.0, 0.001, 1e-6)
    chx.ch_set_noise(h, 1e-14, seed=2021)
    c = torch.tensor(c0, device="cuda")
    print("[case] cook 8192 one step", flush=True)
    chx.ch_adi_step(h, c, nsteps=1)
    torch.cuda.synchronize()
    ref = orc.ch_step_cook(c0, L, L, 1.0, 0.001, 1e-6, 1e-14, 2021)
    assert rel(c.cpu().numpy(), ref) < 1e-12
