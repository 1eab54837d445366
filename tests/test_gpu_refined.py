"""GPU parity of the FP32-sweep, FP64-residual refinement path: every result
is compared with the FP64 oracle; the per-solve target is 1e-10 (normwise
relative, infinity norm) with the solution held in FP64."""
import math

import numpy as np
import pytest

from paper_2101_06550_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
L = 2 * math.pi
TARGET = 1e-10


@pytest.fixture(scope="module")
def chx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_06550_amd import chx as m
    m.load()
    return m


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def penta(s):
    return (s, -4 * s, 1 + 6 * s, -4 * s, s)


def solve_refined(chx, kind, co, f, layout, passes, periodic=True):
    n, batch = (f.shape[0], f.shape[1]) if layout == 0 else (f.shape[1], f.shape[0])
    x = torch.tensor(f, device="cuda")
    print(f"[case] refined {kind} n={n} batch={batch} layout={layout} passes={passes}", flush=True)
    if kind == "penta":
        plan = chx.penta_factor(n, *co, periodic=periodic)
        chx.penta_solve_batch(plan, batch, x, layout=layout, dtype=chx.CHX_F32_REFINED,
                              refine_passes=passes)
    else:
        plan = chx.tri_factor(n, *co, periodic=periodic)
        chx.tri_solve_batch(plan, batch, x, layout=layout, dtype=chx.CHX_F32_REFINED,
                            refine_passes=passes)
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("passes", [1, 2])
def test_penta_standalone_workload(chx, orc, layout, passes):
    """1024 systems of N = 1024, alpha = 0.5 (kappa = 9)."""
    f = inputs.uniform(2, (1024, 1024), -1, 1)
    out = solve_refined(chx, "penta", penta(0.5), f, layout, passes)
    ref = orc.cpenta_lines(f, 1 if layout == 0 else 0, penta(0.5))
    assert rel(out, ref) < TARGET


@pytest.mark.parametrize("layout", [0, 1])
def test_tri_standalone_workload(chx, orc, layout):
    co = (-0.5, 2.0, -0.5)
    f = inputs.uniform(2, (1024, 1024), -1, 1)
    out = solve_refined(chx, "tri", co, f, layout, 1)
    assert rel(out, orc.ctri_lines(f, 1 if layout == 0 else 0, co)) < TARGET


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("n,batch,sigma,passes", [(256, 128, 44.092, 2), (1024, 64, 70.547, 2),
                                                  (1000, 40, 3.0, 1), (13, 20, 0.8, 1),
                                                  (512, 64, 2889.6, 3)])
def test_penta_ill_conditioned_and_fallback(chx, orc, n, batch, sigma, passes, layout):
    shape = (n, batch) if layout == 0 else (batch, n)
    f = inputs.uniform(8, shape, -1, 1)
    out = solve_refined(chx, "penta", penta(sigma), f, layout, passes)
    ref = orc.cpenta_lines(f, 1 if layout == 0 else 0, penta(sigma))
    assert rel(out, ref) < TARGET


@pytest.mark.parametrize("layout", [0, 1])
def test_non_periodic_refined(chx, orc, layout):
    co = penta(1.5)
    n, batch = 64, 16
    f = inputs.uniform(9, (n, batch) if layout == 0 else (batch, n), -1, 1)
    out = solve_refined(chx, "penta", co, f, layout, 2, periodic=False)
    sys_ = f.T if layout == 0 else f
    ref = np.stack([orc.penta_lr_solve(*(np.full(n, v) for v in co), sys_[s]) for s in range(batch)])
    ref = ref.T if layout == 0 else ref
    assert rel(out, ref) < TARGET


def test_refine_passes_validated(chx):
    x = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    plan = chx.penta_factor(64, *penta(1.0))
    for bad in (0, 4):
        with pytest.raises(chx.ChxError):
            chx.penta_solve_batch(plan, 64, x, layout=0, dtype=chx.CHX_F32_REFINED,
                                  refine_passes=bad)


@pytest.mark.parametrize("n,dt,passes", [(128, 1e-4, 1), (256, 1e-4, 2), (1024, 1e-5, 2)])
def test_adi_step_refined(chx, orc, n, dt, passes):
    c0 = inputs.noise_field(n, n, 3)
    h = chx.ch_create(n, n, L, L, 1.0, 0.01, dt, dtype=chx.CHX_F32_REFINED,
                      refine_passes=passes)
    c = torch.tensor(c0, device="cuda")
    print(f"[case] refined ADI {n} passes={passes}", flush=True)
    chx.ch_adi_step(h, c, nsteps=1)
    torch.cuda.synchronize()
    assert rel(c.cpu().numpy(), orc.ch_step(c0, L, L, 1.0, 0.01, dt)) < TARGET


def test_adi_refined_large_run_one_step(chx, orc):
    n = 8192
    c0 = inputs.mode_plus_noise(n, 5)
    h = chx.ch_create(n, n, L, L, 1.0, 0.001, 1e-6, dtype=chx.CHX_F32_REFINED, refine_passes=3)
    c = torch.tensor(c0, device="cuda")
    print("[case] refined ADI 8192 passes=3", flush=True)
    chx.ch_adi_step(h, c, nsteps=1)
    torch.cuda.synchronize()
    err = rel(c.cpu().numpy(), orc.ch_step(c0, L, L, 1.0, 0.001, 1e-6))
    print(f"refined 8192 one-step error {err:.3e}")
    assert err < TARGET
