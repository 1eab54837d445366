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
    assert chx.ch_ws_bytes(h) > w0
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
