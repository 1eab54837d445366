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


# (ny, nx, dt, passes, steps, seed): several 32-row chunks, 60-column wave
# segments with a ragged last one (nx % 60 != 0), exact segments (960), two
# chunks (the wrap chunk is both neighbours), one chunk
# (64, 64): one 64-column wave per row, whose halo lanes wrap onto its own
# columns
STEP_CASES = [(1024, 1024, 1e-5, 2, 3, 81), (96, 320, 1e-4, 1, 3, 82), (160, 576, 1e-4, 3, 2, 83),
              (64, 2048, 1e-5, 2, 2, 84), (256, 960, 1e-4, 2, 2, 85), (32, 128, 1e-4, 1, 4, 86),
              (64, 64, 1e-4, 2, 3, 87)]


@pytest.mark.parametrize("ny,nx,dt,passes,k,seed", STEP_CASES)
def test_refined_steps_in_one_call(chx, orc, ny, nx, dt, passes, k, seed):
    """k refined steps in one call against the oracle's k FP64 steps, and the
    diagnostics of every state of the call."""
    g = 0.01
    c0 = inputs.noise_field(ny, nx, seed)
    h = chx.ch_create(nx, ny, L, L, 1.0, g, dt, dtype=chx.CHX_F32_REFINED, refine_passes=passes)
    c = torch.tensor(c0, device="cuda")
    d = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
    print(f"[case] refined {k} steps {ny}x{nx} passes={passes}", flush=True)
    chx.ch_adi_step(h, c, nsteps=k, diag_out=d)
    torch.cuda.synchronize()
    out = c.cpu().numpy()
    ref = [c0]
    for _ in range(k):
        ref.append(orc.ch_step(ref[-1], L, L, 1.0, g, dt))
    err = rel(out, ref[k])
    print(f"refined {ny}x{nx} p={passes}: {k}-step error {err:.3e}", flush=True)
    assert err < k * TARGET, err
    dd = d.cpu().numpy().reshape(k + 1, 2)
    l1 = np.sum(np.abs(c0)) * (L / nx) * (L / ny)
    # the last state's diagnostics are those of the returned field
    assert abs(dd[k, 0] - orc.ch_mass(out, L, L)) <= 1e-12 * l1
    assert abs(dd[k, 1] - orc.ch_energy(out, L, L, g)) <= 1e-12 * abs(dd[k, 1])
    for j in range(k + 1):
        m, e = orc.ch_mass(ref[j], L, L), orc.ch_energy(ref[j], L, L, g)
        assert abs(dd[j, 0] - m) <= 1e-10 * l1, (j, dd[j, 0], m)
        assert abs(dd[j, 1] - e) <= max(j, 1) * 1e-9 * abs(e), (j, dd[j, 1], e)


def test_refined_step_error_falls_with_passes(chx, orc):
    """kappa = 1130 (1024^2, dt = 1e-5): each pass gains log10(1 / (kappa 2^-24))
    digits, so one pass stays above 1e-10 and two reach the FP64 level."""
    n, dt = 1024, 1e-5
    c0 = inputs.noise_field(n, n, 3)
    ref = orc.ch_step(c0, L, L, 1.0, 0.01, dt)
    errs = []
    for passes in (1, 2, 3):
        h = chx.ch_create(n, n, L, L, 1.0, 0.01, dt, dtype=chx.CHX_F32_REFINED,
                          refine_passes=passes)
        c = torch.tensor(c0, device="cuda")
        print(f"[case] refined 1024 passes={passes}", flush=True)
        chx.ch_adi_step(h, c, nsteps=1)
        torch.cuda.synchronize()
        errs.append(rel(c.cpu().numpy(), ref))
    print("refined 1024 errors by passes", errs, flush=True)
    assert errs[0] > 1e-11 and errs[1] < 1e-12 and errs[2] < 1e-12, errs


def test_refinement_that_cannot_converge_is_refused(chx):
    """CHX_EREFINE when FP32 sweeps cannot contract the error
    (4 kappa 2^-24 >= 1; kappa = 1 + 16 sigma for the periodic penta matrix):
    sigma = 1e9 is refused before anything is enqueued, sigma = 0.5 runs; the
    FP64 solve of the same stiff matrix is unaffected.  A refined ADI handle
    whose directions sum to such a kappa is refused at creation."""
    n, batch = 1024, 64
    f = inputs.uniform(11, (n, batch), -1, 1)
    x = torch.tensor(f, device="cuda")
    stiff = chx.penta_factor(n, *penta(1e9))
    with pytest.raises(chx.ChxError) as ei:
        chx.penta_solve_batch(stiff, batch, x, layout=0, dtype=chx.CHX_F32_REFINED,
                              refine_passes=3)
    assert ei.value.status == chx.CHX_EREFINE
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), f)  # nothing was enqueued
    chx.penta_solve_batch(stiff, batch, x, layout=0)  # FP64: fine
    mild = chx.penta_factor(n, *penta(0.5))
    y = torch.tensor(f, device="cuda")
    chx.penta_solve_batch(mild, batch, y, layout=0, dtype=chx.CHX_F32_REFINED, refine_passes=1)
    torch.cuda.synchronize()
    tri = chx.tri_factor(n, -1e9, 1 + 2e9, -1e9)
    with pytest.raises(chx.ChxError) as ei:
        chx.tri_solve_batch(tri, batch, x, layout=0, dtype=chx.CHX_F32_REFINED, refine_passes=1)
    assert ei.value.status == chx.CHX_EREFINE
    with pytest.raises(chx.ChxError) as ei:  # 1024^2, dt = 1: kappa ~ 1.1e7 per direction
        chx.ch_create(1024, 1024, L, L, 1.0, 0.001, 1.0, dtype=chx.CHX_F32_REFINED,
                      refine_passes=3)
    assert ei.value.status == chx.CHX_EREFINE


@pytest.mark.parametrize("ny,nx", [(1024, 1024), (96, 320)])
def test_refined_separator_shapes_bitwise(chx, orc, ny, nx):
    """Refined handles tune the FP32 separator kernel's tile shape too: every
    shape sums the same terms in the same order, so two refined steps are
    bitwise identical whatever the shape, and match the oracle."""
    g, dt, k = 0.01, 1e-5, 2
    c0 = inputs.noise_field(ny, nx, 77)
    h = chx.ch_create(nx, ny, L, L, 1.0, g, dt, dtype=chx.CHX_F32_REFINED, refine_passes=2)
    assert 0 <= chx.ch_get_tuning(h) < chx.CHX_NUM_REDUCED_SHAPES
    ref = None
    for shape in range(chx.CHX_NUM_REDUCED_SHAPES):
        print(f"[case] refined separator shape {shape} {ny}x{nx}", flush=True)
        chx.ch_set_tuning(h, shape)
        c = torch.tensor(c0, device="cuda")
        d = torch.zeros(2 * (k + 1), dtype=torch.float64, device="cuda")
        chx.ch_adi_step(h, c, nsteps=k, diag_out=d)
        torch.cuda.synchronize()
        out = (c.cpu().numpy(), d.cpu().numpy())
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), shape
    assert rel(ref[0], orc.ch_step(c0, L, L, 1.0, g, dt, nsteps=k)) < k * TARGET
