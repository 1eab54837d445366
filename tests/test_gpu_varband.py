"""GPU parity of the batched solves with one matrix per system (Ch.4
cuPentBatch design with its factor-once and "Rewrite" modes; Ch.5 for the
tridiagonal case) against the oracle, periodic and not, through the C-ABI.

Tolerance: the matrices are diagonally dominant with diagonal in [4.5, 5.5]
and off-diagonals in [-1, 1] (tridiagonal: [2.5, 3.5] against [-1, 1]), so
kappa_inf <= 19; a backward-stable sweep then gives a normwise relative error
of a few units of n * eps * kappa, far below the 1e-12 used here.  The
hyperdiffusion matrices of Ch.4 use kappa-scaled bounds."""
import numpy as np
import pytest

from paper_2101_06550_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def chx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_06550_amd import chx as m
    m.load()
    return m


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle.Oracle()


def _penta_system(n, batch, seed):
    u = [inputs.uniform(seed + k, (n, batch), -1.0, 1.0) for k in range(4)]
    c = inputs.uniform(seed + 4, (n, batch), 4.5, 5.5)
    f = inputs.uniform(seed + 5, (n, batch), -1.0, 1.0)
    return u[0], u[1], c, u[2], u[3], f


def _tri_system(n, batch, seed):
    a = inputs.uniform(seed, (n, batch), -1.0, 1.0)
    b = inputs.uniform(seed + 1, (n, batch), 2.5, 3.5)
    c = inputs.uniform(seed + 2, (n, batch), -1.0, 1.0)
    f = inputs.uniform(seed + 3, (n, batch), -1.0, 1.0)
    return a, b, c, f


def _dev(arr, ld):
    """(n, batch) host array -> device (n, ld) tensor, padding columns NaN so
    that any read past `batch` would show."""
    n, batch = arr.shape
    t = torch.full((n, ld), float("nan"), dtype=torch.float64, device="cuda")
    t[:, :batch] = torch.from_numpy(arr).cuda()
    return t


def _err(x, ref):
    return np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300)


CASES = [(5, 1), (6, 63), (7, 64), (8, 65), (33, 300), (257, 129), (1024, 64)]


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("n,batch", CASES)
def test_penta_rewrite_and_factor_solve(chx, orc, periodic, n, batch):
    print(f"[penta per-system] n={n} batch={batch} periodic={periodic}", flush=True)
    a, b, c, d, e, f = _penta_system(n, batch, 31 * n + batch)
    ref = orc.penta_rows_batch(a, b, c, d, e, f, periodic)
    ld = batch + 3
    A = [_dev(v, ld) for v in (a, b, c, d, e)]
    x = _dev(f, ld)
    chx.penta_batch_rewrite(*A, x, periodic=periodic, batch=batch)
    torch.cuda.synchronize()
    xr = x[:, :batch].cpu().numpy()
    assert _err(xr, ref) < 1e-12
    assert torch.isnan(x[:, batch:]).all()  # padding untouched
    for v, t in zip((a, b, c, d, e), A):    # rewrite leaves the matrix alone
        assert np.array_equal(t[:, :batch].cpu().numpy(), v)
    ws = chx.penta_batch_factor(*A, periodic=periodic, batch=batch)
    for rep in range(2):  # the factors serve repeated solves
        x2 = _dev(f, ld)
        chx.penta_batch_solve(*A, x2, ws=ws, periodic=periodic, batch=batch)
        torch.cuda.synchronize()
        assert _err(x2[:, :batch].cpu().numpy(), ref) < 1e-12
        assert torch.isnan(x2[:, batch:]).all()


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("n,batch", [(3, 1), (4, 63), (5, 65), (33, 300), (1024, 64)])
def test_tri_rewrite_and_factor_solve(chx, orc, periodic, n, batch):
    print(f"[tri per-system] n={n} batch={batch} periodic={periodic}", flush=True)
    a, b, c, f = _tri_system(n, batch, 17 * n + batch)
    ref = orc.tri_rows_batch(a, b, c, f, periodic)
    ld = batch + 5
    A = [_dev(v, ld) for v in (a, b, c)]
    x = _dev(f, ld)
    chx.tri_batch_rewrite(*A, x, periodic=periodic, batch=batch)
    torch.cuda.synchronize()
    assert _err(x[:, :batch].cpu().numpy(), ref) < 1e-12
    for v, t in zip((a, b, c), A):
        assert np.array_equal(t[:, :batch].cpu().numpy(), v)
    ws = chx.tri_batch_factor(*A, periodic=periodic, batch=batch)
    for rep in range(2):
        x2 = _dev(f, ld)
        chx.tri_batch_solve(*A, x2, ws=ws, periodic=periodic, batch=batch)
        torch.cuda.synchronize()
        assert _err(x2[:, :batch].cpu().numpy(), ref) < 1e-12


def test_hyperdiffusion_rows_match_shared_matrix_path(chx, orc):
    """Equal rows (the Ch.4 Crank-Nicolson hyperdiffusion matrix with
    sigma = dt / (2 dx^4), n = 256, dt = 1e-6 on (0, 1)) solved per system
    agree with the oracle and with the shared-matrix solver."""
    n, batch = 256, 512
    sig = 1e-6 / (2 * (1.0 / n) ** 4)
    kappa = 1 + 16 * sig
    one = np.ones((n, batch))
    diag = [sig * one, -4 * sig * one, (1 + 6 * sig) * one, -4 * sig * one, sig * one]
    f = inputs.batch_rhs(77, n, batch)
    ref = orc.penta_rows_batch(*diag, f, True)
    A = [_dev(v, batch) for v in diag]
    x = _dev(f, batch)
    chx.penta_batch_rewrite(*A, x, periodic=True)
    plan = chx.penta_factor(n, sig, -4 * sig, 1 + 6 * sig, -4 * sig, sig, True)
    y = _dev(f, batch)
    chx.penta_solve_batch(plan, batch, y)
    torch.cuda.synchronize()
    tol = 64 * n * np.finfo(float).eps * kappa
    assert _err(x.cpu().numpy(), ref) < tol
    assert _err(y.cpu().numpy(), x.cpu().numpy()) < tol
    chx.penta_plan_destroy(plan)


def test_systems_are_independent_and_batch_zero(chx, orc):
    n, batch = 40, 70
    a, b, c, d, e, f = _penta_system(n, batch, 5)
    A = [_dev(v, batch) for v in (a, b, c, d, e)]
    x0 = _dev(f, batch)
    chx.penta_batch_rewrite(*A, x0, periodic=True)
    c2 = c.copy()
    c2[:, 13] += 0.5
    A[2] = _dev(c2, batch)
    x1 = _dev(f, batch)
    chx.penta_batch_rewrite(*A, x1, periodic=True)
    torch.cuda.synchronize()
    keep = [k for k in range(batch) if k != 13]
    assert torch.equal(x0[:, keep], x1[:, keep])
    # batch = 0: nothing is touched
    x2 = _dev(f, batch)
    chx.penta_batch_rewrite(*A, x2, periodic=True, batch=0)
    chx.tri_batch_rewrite(*A[:3], x2, periodic=True, batch=0)
    torch.cuda.synchronize()
    assert np.array_equal(x2.cpu().numpy(), f)


def test_large_batch_sampled(chx, orc):
    """The benchmark's shape (n = 1024, 65536 systems, periodic) on sampled
    systems against the oracle."""
    n, batch = 1024, 65536
    print(f"[penta per-system large] n={n} batch={batch}", flush=True)
    dev = dict(dtype=torch.float64, device="cuda")
    A = [torch.from_numpy(inputs.uniform(900 + k, (n, batch), -1.0, 1.0)).to(**dev)
         for k in range(5)]
    A[2] = A[2] * 0.5 + 5.0
    f = torch.from_numpy(inputs.uniform(905, (n, batch), -1.0, 1.0)).to(**dev)
    x = f.clone()
    chx.penta_batch_rewrite(*A, x, periodic=True)
    torch.cuda.synchronize()
    pick = [0, 1, 63, 64, 4095, 32768, batch - 1]
    host = [t[:, pick].cpu().numpy() for t in A]
    ref = orc.penta_rows_batch(*host, f[:, pick].cpu().numpy(), True)
    assert _err(x[:, pick].cpu().numpy(), ref) < 1e-12


def test_penta_rewrite_argument_errors_leave_the_arrays_untouched(chx, orc):
    """Through the C-ABI itself: a null band or right-hand side, batch < 0,
    ld < batch, periodic other than 0/1, n below the periodic minimum, a
    workspace that is missing, misaligned or too small are refused with their
    codes before any launch and batch = 0 is a no-op; bands and right-hand
    sides stay bitwise as they were and a valid call afterwards still matches
    the oracle."""
    lib = chx.load()
    n, batch = 33, 70
    print(f"[penta per-system] argument errors n={n} batch={batch}", flush=True)
    host = _penta_system(n, batch, 77)
    A = [torch.tensor(v, device="cuda") for v in host[:5]]
    x = torch.tensor(host[5], device="cuda")
    need = lib.penta_batch_ws_bytes(n, batch, 1, getattr(chx, "CHX_BATCH_REWRITE", 1))
    assert need > 0
    ws = torch.zeros(need + 512, dtype=torch.uint8, device="cuda")
    aligned = (ws.data_ptr() + 255) // 256 * 256
    st = chx._stream(None)
    bad = [
        (dict(a=None), chx.CHX_EINVAL),
        (dict(x=None), chx.CHX_EINVAL),
        (dict(batch=-1), chx.CHX_EINVAL),
        (dict(ld=batch - 1), chx.CHX_EINVAL),
        (dict(periodic=2), chx.CHX_EINVAL),
        (dict(n=4), chx.CHX_EUNSUPPORTED_N),
        (dict(ws=None), chx.CHX_EINVAL),
        (dict(ws=aligned + 8), chx.CHX_EINVAL),
        (dict(avail=need - 8), chx.CHX_ENOMEM),
        (dict(batch=0), chx.CHX_OK),
    ]
    for over, code in bad:
        g = dict(n=n, batch=batch, periodic=1, a=A[0].data_ptr(), ld=batch, x=x.data_ptr(),
                 ws=aligned, avail=need)
        g.update(over)
        rc = lib.penta_batch_rewrite(g["n"], g["batch"], g["periodic"], g["a"],
                                     *[t.data_ptr() for t in A[1:]], g["ld"], g["x"], g["ws"],
                                     g["avail"], st)
        assert rc == code, (over, rc)
    torch.cuda.synchronize()
    for v, t in zip(host, A + [x]):
        assert np.array_equal(t.cpu().numpy(), v)
    rc = lib.penta_batch_rewrite(n, batch, 1, *[t.data_ptr() for t in A], batch, x.data_ptr(),
                                 aligned, need, st)
    assert rc == chx.CHX_OK
    torch.cuda.synchronize()
    ref = orc.penta_rows_batch(*host, True)
    assert _err(x.cpu().numpy(), ref) < 1e-12
