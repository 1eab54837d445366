"""Thin ctypes binding of ``libchx.so`` (the C-ABI in ``include/chx.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C-ABI.  PyTorch provides device memory (tensors) and
streams; functions accept CUDA/HIP ``torch.Tensor`` objects (float64) and use
the current torch stream unless one is given.  There is no CPU fallback: if
the library is missing, loading raises ``ChxError``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CHX_LIBRARY", os.path.join(HERE, "libchx.so"))

CHX_OK = 0
CHX_EINVAL = -1
CHX_EUNSUPPORTED_N = -2
CHX_EPIVOT = -3
CHX_EHIP = -4
CHX_ENONFINITE = -5
CHX_ENOMEM = -6
CHX_EREFINE = -7
CHX_ESCRATCH = -8
CHX_NOALLOC_SCRATCH_BYTES = 32 << 20

CHX_SCHEME_P1 = 0
CHX_SCHEME_P2 = 1
CHX_F64 = 0
CHX_F32_REFINED = 1
CHX_F32 = 2
CHX_INTERLEAVED = 0
CHX_CONTIGUOUS = 1
CHX_BATCH_FACTOR = 0
CHX_BATCH_REWRITE = 1

# Every symbol that include/chx.h declares.
EXPORTED = [
    "chx_version", "chx_status_string", "chx_stream_copy",
    "penta_factor", "penta_plan_destroy", "penta_solve_ws_bytes", "penta_solve_batch",
    "penta_solve_batch_noalloc",
    "tri_factor", "tri_plan_destroy", "tri_solve_ws_bytes", "tri_solve_batch",
    "penta_batch_ws_bytes", "penta_batch_factor", "penta_batch_solve", "penta_batch_rewrite",
    "tri_batch_ws_bytes", "tri_batch_factor", "tri_batch_solve", "tri_batch_rewrite",
    "stencil2d_apply",
    "ch_create", "ch_destroy", "ch_ws_bytes", "ch_adi_step", "ch_adi_step_p2",
    "ch_adi_step_timed",
    "ch_get_tuning", "ch_set_tuning", "ch_set_noise", "ch_get_noise_step", "ch_diagnostics",
    "ch_moments", "ch_k1", "ch_energy_decay_rate",
    "batch1d_create", "batch1d_destroy", "batch1d_ws_bytes", "batch1d_step",
    "batch1d_rewrite_ws_bytes", "batch1d_step_rewrite",
    "ch_ensemble_create", "ch_ensemble_destroy", "ch_ensemble_ws_bytes", "ch_ensemble_step",
    "ch_ensemble_moments", "ch_ensemble_k1", "ch_ensemble_set_noise",
    "ch_ensemble_get_noise_step", "ch_ensemble_get_tuning", "ch_ensemble_set_tuning",
    "chx_host_chunk_tables", "chx_host_whole_tables",
]


class ChxError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _status_string(status) if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class ChParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("D", ctypes.c_double), ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
                ("dtype", ctypes.c_int), ("refine_passes", ctypes.c_int),
                ("scheme", ctypes.c_int)]


_lib = None
_V = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_long
_D = ctypes.c_double
_S = ctypes.c_size_t
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def load(path: str | None = None):
    """Load libchx.so (raises ChxError(CHX_EHIP) if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ChxError(CHX_EHIP, f"HIP library not built ({p}); run "
                       "python -m paper_2101_06550_amd.csrc.build")
    lib = ctypes.CDLL(p)
    sig = {
        "chx_version": (_I, []),
        "chx_status_string": (ctypes.c_char_p, [_I]),
        "chx_stream_copy": (_I, [_V, _V, _S, _V]),
        "penta_factor": (_I, [_I, _D, _D, _D, _D, _D, _I, ctypes.POINTER(_V)]),
        "penta_plan_destroy": (_I, [_V]),
        "penta_solve_ws_bytes": (_S, [_V, _I, _I, _I, _I]),
        "penta_solve_batch": (_I, [_V, _I, _V, _L, _I, _I, _I, _V, _S, _V]),
        "penta_solve_batch_noalloc": (_I, [_V, _I, _V, _L, _I, _I, _I, _V]),
        "tri_factor": (_I, [_I, _D, _D, _D, _I, ctypes.POINTER(_V)]),
        "tri_plan_destroy": (_I, [_V]),
        "tri_solve_ws_bytes": (_S, [_V, _I, _I, _I, _I]),
        "tri_solve_batch": (_I, [_V, _I, _V, _L, _I, _I, _I, _V, _S, _V]),
        "penta_batch_ws_bytes": (_S, [_I, _I, _I, _I]),
        "penta_batch_factor": (_I, [_I, _I, _I] + [_V] * 5 + [_L, _V, _S, _V]),
        "penta_batch_solve": (_I, [_I, _I, _I] + [_V] * 5 + [_L, _V, _S, _V, _V]),
        "penta_batch_rewrite": (_I, [_I, _I, _I] + [_V] * 5 + [_L, _V, _V, _S, _V]),
        "tri_batch_ws_bytes": (_S, [_I, _I, _I, _I]),
        "tri_batch_factor": (_I, [_I, _I, _I] + [_V] * 3 + [_L, _V, _S, _V]),
        "tri_batch_solve": (_I, [_I, _I, _I] + [_V] * 3 + [_L, _V, _S, _V, _V]),
        "tri_batch_rewrite": (_I, [_I, _I, _I] + [_V] * 3 + [_L, _V, _V, _S, _V]),
        "stencil2d_apply": (_I, [_V, _V, _I, _I, _L, _I, _DP, _I, _I, _I, _I, _I, _I, _V]),
        "ch_create": (_I, [ctypes.POINTER(ChParams), ctypes.POINTER(_V)]),
        "ch_destroy": (_I, [_V]),
        "ch_ws_bytes": (_S, [_V]),
        "ch_adi_step": (_I, [_V, _V, _L, _I, _V, _V, _S, _V]),
        "ch_adi_step_timed": (_I, [_V, _V, _L, _I, _V, _V, _S, _V, _I, _DP, _IP]),
        "ch_adi_step_p2": (_I, [_V, _V, _V, _L, _I, _V, _V, _S, _V]),
        "ch_set_noise": (_I, [_V, _D, ctypes.c_uint64, ctypes.c_uint64]),
        "ch_get_noise_step": (_I, [_V, ctypes.POINTER(ctypes.c_uint64)]),
        "ch_get_tuning": (_I, [_V, _I, _IP]),
        "ch_set_tuning": (_I, [_V, _I, _I]),
        "ch_diagnostics": (_I, [_V, _V, _L, _DP, _DP, _V]),
        "ch_moments": (_I, [_V, _V, _L, _DP, _V]),
        "ch_energy_decay_rate": (_I, [_V, _I, _I, _D, _D, _V, _V]),
        "ch_k1": (_I, [_V, _V, _L, _DP, _V]),
        "batch1d_create": (_I, [_I, _I, _D, _D, _D, _D, ctypes.POINTER(_V)]),
        "batch1d_destroy": (_I, [_V]),
        "batch1d_ws_bytes": (_S, [_V, _I]),
        "batch1d_step": (_I, [_V, _I, _V, _L, _I, _V, _S, _V]),
        "batch1d_rewrite_ws_bytes": (_S, [_V, _I]),
        "batch1d_step_rewrite": (_I, [_V, _I, _V, _L, _I, _V, _S, _V]),
        "ch_ensemble_create": (_I, [_I, ctypes.POINTER(ChParams), ctypes.POINTER(_V)]),
        "ch_ensemble_destroy": (_I, [_V]),
        "ch_ensemble_ws_bytes": (_S, [_V]),
        "ch_ensemble_step": (_I, [_V, ctypes.POINTER(_V), ctypes.POINTER(_L), _I, _V, _V, _S,
                                  _I, _V]),
        "ch_ensemble_set_noise": (_I, [_V, _D, ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64]),
        "ch_ensemble_get_noise_step": (_I, [_V, ctypes.POINTER(ctypes.c_uint64)]),
        "ch_ensemble_get_tuning": (_I, [_V, _I, ctypes.POINTER(_I)]),
        "ch_ensemble_set_tuning": (_I, [_V, _I, _I]),
        "ch_ensemble_moments": (_I, [_V, ctypes.POINTER(_V), ctypes.POINTER(_L), _DP, _V]),
        "ch_ensemble_k1": (_I, [_V, ctypes.POINTER(_V), ctypes.POINTER(_L), _DP, _V]),
        "chx_host_chunk_tables": (_I, [_I, _DP, _I, _I, _DP, _I, _DP, _I, _IP]),
        "chx_host_whole_tables": (_I, [_I, _DP, _I, _I, _DP, _I, _DP, _IP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _status_string(st: int) -> str:
    return _lib.chx_status_string(st).decode()


def _check(st: int, what: str):
    if st != CHX_OK:
        raise ChxError(st, what)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _devptr(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ChxError(CHX_EINVAL, f"{what} must be a device tensor")
    if t.dtype != torch.float64:
        raise ChxError(CHX_EINVAL, f"{what} must be float64")
    return ctypes.c_void_p(t.data_ptr())


def _storage_elems(t) -> int:
    """Elements of t's dtype from t's first element to the end of its storage."""
    return t.untyped_storage().nbytes() // t.element_size() - t.storage_offset()


def _field_ld(t, nx: int, ny: int, ld, what: str) -> int:
    """Leading dimension of a (ny, >= nx) field with unit column stride whose
    rows, ld apart, lie inside its storage (the kernels read and write
    (ny - 1) * ld + nx elements from its start); ChxError otherwise."""
    if t.dim() != 2 or t.shape[0] != ny or t.shape[1] < nx:
        raise ChxError(CHX_EINVAL, f"{what} must be a ({ny}, >= {nx}) tensor, got "
                                   f"{tuple(t.shape)}")
    if nx > 1 and t.stride(1) != 1:
        raise ChxError(CHX_EINVAL, f"{what} must have unit column stride")
    ld = t.stride(0) if ld is None else int(ld)
    if (ny > 1 and t.stride(0) != ld) or ld < nx:
        raise ChxError(CHX_EINVAL, f"{what}: leading dimension {ld} must be its row stride "
                                   f"and >= {nx}")
    if (ny - 1) * ld + nx > _storage_elems(t):
        raise ChxError(CHX_EINVAL, f"{what}: rows run past the end of its storage")
    return ld


def _field(t, nx: int, ny: int, ld, what: str):
    """Device pointer and leading dimension of a float64 device field that
    passes _field_ld."""
    ld = _field_ld(t, nx, ny, ld, what)
    return _devptr(t, what), ld


def _diag(diag_out, count: int, what: str = "diag_out"):
    """Device pointer of an optional float64 diagnostics buffer of >= count
    contiguous values (null when diag_out is None)."""
    if diag_out is None:
        return ctypes.c_void_p(0)
    if not diag_out.is_contiguous() or diag_out.numel() < count:
        raise ChxError(CHX_EINVAL, f"{what} must be contiguous with >= {count} values")
    return _devptr(diag_out, what)


def _workspace(nbytes: int, ws, device):
    import torch
    if nbytes == 0:
        return None, ctypes.c_void_p(0), 0
    if ws is None:
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = ws.data_ptr()
    aligned = (base + 255) & ~255
    avail = ws.numel() * ws.element_size() - (aligned - base)
    return ws, ctypes.c_void_p(aligned), avail


# ----------------------------------------------------------------------- version
def chx_version() -> int:
    return load().chx_version()


def chx_status_string(status: int) -> str:
    return load().chx_status_string(status).decode()


# ------------------------------------------------------------------------- plans
class _Plan:
    _destroy = None

    def __init__(self, handle, n, P, periodic):
        self.handle = handle
        self.n = n
        self.P = P
        self.periodic = periodic

    def close(self):
        if self.handle:
            getattr(load(), self._destroy)(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PentaPlan(_Plan):
    _destroy = "penta_plan_destroy"


class TriPlan(_Plan):
    _destroy = "tri_plan_destroy"


def penta_factor(n: int, a: float, b: float, c: float, d: float, e: float,
                 periodic: bool = True) -> PentaPlan:
    h = ctypes.c_void_p()
    _check(load().penta_factor(n, a, b, c, d, e, int(bool(periodic)), ctypes.byref(h)),
           "penta_factor")
    return PentaPlan(h, n, 2, periodic)


def penta_plan_destroy(plan: PentaPlan) -> None:
    plan.close()


def tri_factor(n: int, a: float, b: float, c: float, periodic: bool = True) -> TriPlan:
    h = ctypes.c_void_p()
    _check(load().tri_factor(n, a, b, c, int(bool(periodic)), ctypes.byref(h)), "tri_factor")
    return TriPlan(h, n, 1, periodic)


def tri_plan_destroy(plan: TriPlan) -> None:
    plan.close()


def penta_solve_ws_bytes(plan, batch, layout=CHX_INTERLEAVED, dtype=CHX_F64, refine_passes=0):
    return load().penta_solve_ws_bytes(plan.handle, batch, layout, dtype, refine_passes)


def tri_solve_ws_bytes(plan, batch, layout=CHX_INTERLEAVED, dtype=CHX_F64, refine_passes=0):
    return load().tri_solve_ws_bytes(plan.handle, batch, layout, dtype, refine_passes)


def _solve_ld(kind, plan, batch, x, ld, layout):
    """Leading dimension of x, checked against x's storage."""
    if ld is None:
        ld = x.stride(0) if x.dim() == 2 else (batch if layout == CHX_INTERLEAVED else plan.n)
    if batch > 0:  # element (s, i) at i * ld + s (interleaved) or s * ld + i (contiguous)
        span = (plan.n - 1) * ld + batch if layout == CHX_INTERLEAVED else (batch - 1) * ld + plan.n
        if x.dim() == 2 and x.stride(-1) != 1:
            raise ChxError(CHX_EINVAL, f"{kind}_solve_batch: x must have unit last stride")
        if ld >= 1 and span > _storage_elems(x):
            raise ChxError(CHX_EINVAL, f"{kind}_solve_batch: {span} elements needed from x's "
                                       "start, its storage holds fewer")
    return ld


def _solve(kind, plan, batch, x, ld, layout, dtype, refine_passes, ws, stream):
    lib = load()
    ld = _solve_ld(kind, plan, batch, x, ld, layout)
    xp = _devptr(x, "x")
    nbytes = getattr(lib, f"{kind}_solve_ws_bytes")(plan.handle, batch, layout, dtype,
                                                    refine_passes)
    keep, wsp, avail = _workspace(nbytes, ws, x.device)
    st = getattr(lib, f"{kind}_solve_batch")(plan.handle, batch, xp, ld, layout,
                                             dtype, refine_passes, wsp, avail, _stream(stream))
    _check(st, f"{kind}_solve_batch")
    return keep


def penta_solve_batch(plan: PentaPlan, batch: int, x, ld: int | None = None,
                      layout: int = CHX_INTERLEAVED, dtype: int = CHX_F64,
                      refine_passes: int = 0, ws=None, stream=None):
    """Solve in place: x (float64 device tensor) holds the right-hand sides
    and receives the solutions.  Returns the workspace tensor used (keep it
    alive until the stream has finished if it was allocated here)."""
    return _solve("penta", plan, batch, x, ld, layout, dtype, refine_passes, ws, stream)


def penta_solve_batch_noalloc(plan: PentaPlan, batch: int, x, ld: int | None = None,
                              layout: int = CHX_INTERLEAVED, dtype: int = CHX_F64,
                              refine_passes: int = 0, stream=None) -> None:
    """penta_solve_batch with the library's static device scratch as its
    workspace: allocates nothing.  Raises ChxError(CHX_ESCRATCH) when the
    solve needs more than CHX_NOALLOC_SCRATCH_BYTES."""
    lib = load()
    ld = _solve_ld("penta", plan, batch, x, ld, layout)
    st = lib.penta_solve_batch_noalloc(plan.handle, batch, _devptr(x, "x"), ld, layout, dtype,
                                       refine_passes, _stream(stream))
    _check(st, "penta_solve_batch_noalloc")


def tri_solve_batch(plan: TriPlan, batch: int, x, ld: int | None = None,
                    layout: int = CHX_INTERLEAVED, dtype: int = CHX_F64,
                    refine_passes: int = 0, ws=None, stream=None):
    return _solve("tri", plan, batch, x, ld, layout, dtype, refine_passes, ws, stream)


# ----------------------------------------------------------------------- stencil
# ------------------------------------------ batches with one matrix per system
def _band_args(arrays, names, x=None, batch=None):
    """Common (n, ld, batch) of interleaved (n, >= batch) arrays sharing one
    row stride."""
    ref = arrays[0]
    if ref.dim() != 2:
        raise ChxError(CHX_EINVAL, f"{names[0]} must be a 2D (n, batch) tensor")
    n, ld = ref.shape[0], ref.stride(0)
    for t, nm in zip(list(arrays) + ([x] if x is not None else []),
                     list(names) + (["x"] if x is not None else [])):
        if t.dim() != 2 or t.shape[0] != n or t.stride(1) != 1 or t.stride(0) != ld:
            raise ChxError(CHX_EINVAL, f"{nm} must be (n, batch) with the common row stride")
    b = ref.shape[1] if batch is None else int(batch)
    if b > ref.shape[1]:
        raise ChxError(CHX_EINVAL, "batch exceeds the arrays' width")
    return n, ld, b


def penta_batch_ws_bytes(n: int, batch: int, periodic: bool = True,
                         mode: int = CHX_BATCH_FACTOR) -> int:
    return load().penta_batch_ws_bytes(n, batch, int(bool(periodic)), int(mode))


def tri_batch_ws_bytes(n: int, batch: int, periodic: bool = True,
                       mode: int = CHX_BATCH_FACTOR) -> int:
    return load().tri_batch_ws_bytes(n, batch, int(bool(periodic)), int(mode))


def penta_batch_factor(a, b, c, d, e, periodic: bool = True, ws=None, batch=None, stream=None):
    """Factor every system in place (b, c, d, e are overwritten); returns the
    workspace tensor that penta_batch_solve must be given (None if unused)."""
    n, ld, bt = _band_args((a, b, c, d, e), "abcde", batch=batch)
    ws, wsp, avail = _workspace(penta_batch_ws_bytes(n, bt, periodic), ws, a.device)
    _check(load().penta_batch_factor(n, bt, int(bool(periodic)),
                                     *[_devptr(t, nm) for t, nm in zip((a, b, c, d, e), "abcde")],
                                     ld, wsp, avail, _stream(stream)), "penta_batch_factor")
    return ws


def penta_batch_solve(a, b, c, d, e, x, ws=None, periodic: bool = True, batch=None, stream=None):
    """Solve with the factors left by penta_batch_factor; x in place."""
    n, ld, bt = _band_args((a, b, c, d, e), "abcde", x=x, batch=batch)
    need = penta_batch_ws_bytes(n, bt, periodic)
    if need and ws is None:
        raise ChxError(CHX_EINVAL, "periodic systems need the workspace of penta_batch_factor")
    ws, wsp, avail = _workspace(need, ws, a.device)
    _check(load().penta_batch_solve(n, bt, int(bool(periodic)),
                                    *[_devptr(t, nm) for t, nm in zip((a, b, c, d, e), "abcde")],
                                    ld, wsp, avail, _devptr(x, "x"), _stream(stream)),
           "penta_batch_solve")


def penta_batch_rewrite(a, b, c, d, e, x, periodic: bool = True, ws=None, batch=None,
                        stream=None):
    """Factor and solve in one pass (the diagonals are left as they are)."""
    n, ld, bt = _band_args((a, b, c, d, e), "abcde", x=x, batch=batch)
    ws, wsp, avail = _workspace(penta_batch_ws_bytes(n, bt, periodic, CHX_BATCH_REWRITE), ws,
                                a.device)
    _check(load().penta_batch_rewrite(n, bt, int(bool(periodic)),
                                      *[_devptr(t, nm) for t, nm in zip((a, b, c, d, e), "abcde")],
                                      ld, _devptr(x, "x"), wsp, avail, _stream(stream)),
           "penta_batch_rewrite")
    return ws


def tri_batch_factor(a, b, c, periodic: bool = True, ws=None, batch=None, stream=None):
    n, ld, bt = _band_args((a, b, c), "abc", batch=batch)
    ws, wsp, avail = _workspace(tri_batch_ws_bytes(n, bt, periodic), ws, a.device)
    _check(load().tri_batch_factor(n, bt, int(bool(periodic)),
                                   *[_devptr(t, nm) for t, nm in zip((a, b, c), "abc")],
                                   ld, wsp, avail, _stream(stream)), "tri_batch_factor")
    return ws


def tri_batch_solve(a, b, c, x, ws=None, periodic: bool = True, batch=None, stream=None):
    n, ld, bt = _band_args((a, b, c), "abc", x=x, batch=batch)
    need = tri_batch_ws_bytes(n, bt, periodic)
    if need and ws is None:
        raise ChxError(CHX_EINVAL, "periodic systems need the workspace of tri_batch_factor")
    ws, wsp, avail = _workspace(need, ws, a.device)
    _check(load().tri_batch_solve(n, bt, int(bool(periodic)),
                                  *[_devptr(t, nm) for t, nm in zip((a, b, c), "abc")],
                                  ld, wsp, avail, _devptr(x, "x"), _stream(stream)),
           "tri_batch_solve")


def tri_batch_rewrite(a, b, c, x, periodic: bool = True, ws=None, batch=None, stream=None):
    n, ld, bt = _band_args((a, b, c), "abc", x=x, batch=batch)
    ws, wsp, avail = _workspace(tri_batch_ws_bytes(n, bt, periodic, CHX_BATCH_REWRITE), ws,
                                a.device)
    _check(load().tri_batch_rewrite(n, bt, int(bool(periodic)),
                                    *[_devptr(t, nm) for t, nm in zip((a, b, c), "abc")],
                                    ld, _devptr(x, "x"), wsp, avail, _stream(stream)),
           "tri_batch_rewrite")
    return ws


def stencil2d_apply(inp, out, weights, left: int, right: int, top: int, bottom: int,
                    periodic: bool = True, premap: int = 0, ld: int | None = None,
                    stream=None) -> None:
    ny, nx = inp.shape
    ld = inp.stride(0) if ld is None else ld
    if tuple(out.shape) != (ny, nx):
        raise ChxError(CHX_EINVAL, "stencil2d_apply: out must have the shape of inp")
    for t in (inp, out):  # one leading dimension serves both arrays
        if ny > 1 and t.stride(0) != ld or nx > 1 and t.stride(1) != 1:
            raise ChxError(CHX_EINVAL, "stencil2d_apply: inp and out must be row-major with "
                                       "leading dimension ld")
    import torch
    if inp.dtype not in (torch.float64, torch.float32) or out.dtype != inp.dtype:
        raise ChxError(CHX_EINVAL, "stencil2d_apply: inp and out must both be float64 or "
                                   "both float32")
    dtype = CHX_F32 if inp.dtype == torch.float32 else CHX_F64
    for t, what in ((inp, "in"), (out, "out")):
        if not t.is_cuda:
            raise ChxError(CHX_EINVAL, f"{what} must be a device tensor")
    w = (ctypes.c_double * len(weights))(*[float(v) for v in weights])
    _check(load().stencil2d_apply(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  nx, ny, ld, dtype, w, left, right, top, bottom,
                                  int(bool(periodic)), premap, _stream(stream)),
           "stencil2d_apply")


# ----------------------------------------------------------------- Cahn-Hilliard
class CH:
    """Handle of ch_create (factored operators for one grid and time step)."""

    def __init__(self, nx, ny, lx, ly, D, gamma, dt, dtype=CHX_F64, refine_passes=0,
                 scheme=CHX_SCHEME_P1):
        self.params = ChParams(nx, ny, lx, ly, D, gamma, dt, dtype, refine_passes, scheme)
        h = ctypes.c_void_p()
        _check(load().ch_create(ctypes.byref(self.params), ctypes.byref(h)), "ch_create")
        self.handle = h
        self._ws = None

    def close(self):
        if self.handle:
            load().ch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ch_create(nx, ny, lx, ly, D, gamma, dt, dtype=CHX_F64, refine_passes=0,
              scheme=CHX_SCHEME_P1) -> CH:
    return CH(nx, ny, lx, ly, D, gamma, dt, dtype, refine_passes, scheme)


def ch_destroy(h: CH) -> None:
    h.close()


def ch_ws_bytes(h: CH) -> int:
    return load().ch_ws_bytes(h.handle)


def _handle_ws(h, lib, ws, device):
    """The caller's workspace, else one allocated on first use and cached on
    the handle (reallocated when too small or on another device)."""
    nbytes = lib.ch_ws_bytes(h.handle)
    if ws is None:
        if h._ws is None or h._ws.numel() < nbytes + 256 or h._ws.device != device:
            import torch
            h._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ws = h._ws
    return _workspace(nbytes, ws, device)


def ch_adi_step(h: CH, c, nsteps: int = 1, diag_out=None, ws=None, ld: int | None = None,
                stream=None):
    """Advance the float64 device field c (ny, nx) by nsteps in place.  The
    workspace is allocated on first use and cached on the handle unless
    given.  diag_out: optional float64 device tensor of 2*(nsteps+1)."""
    lib = load()
    ld = _field_ld(c, h.params.nx, h.params.ny, ld, "c")
    dptr = _diag(diag_out, 2 * (int(nsteps) + 1))
    cp_ = _devptr(c, "c")
    _, wsp, avail = _handle_ws(h, lib, ws, c.device)
    _check(lib.ch_adi_step(h.handle, cp_, ld, nsteps, dptr, wsp, avail, _stream(stream)),
           "ch_adi_step")


def ch_adi_step_p2(h: CH, c, cprev, nsteps: int = 1, diag_out=None, ws=None,
                   ld: int | None = None, stream=None):
    """Advance the two float64 device states of a CHX_SCHEME_P2 handle in
    place: c = C^n, cprev = C^{n-1} on entry (a copy of C^0 to start), the
    states nsteps later on exit."""
    lib = load()
    ld = _field_ld(c, h.params.nx, h.params.ny, ld, "c")
    if _field_ld(cprev, h.params.nx, h.params.ny, None, "cprev") != ld:
        raise ChxError(CHX_EINVAL, "ch_adi_step_p2: c and cprev need one leading dimension")
    dptr = _diag(diag_out, 2 * (int(nsteps) + 1))
    cp_, pp_ = _devptr(c, "c"), _devptr(cprev, "cprev")
    _, wsp, avail = _handle_ws(h, lib, ws, c.device)
    _check(lib.ch_adi_step_p2(h.handle, cp_, pp_, ld, nsteps, dptr, wsp, avail,
                              _stream(stream)), "ch_adi_step_p2")


def ch_adi_step_timed(h: CH, c, nsteps: int = 1, diag_out=None, ws=None,
                      ld: int | None = None, stream=None, sample_every: int = 1):
    """ch_adi_step with per-phase HIP-event kernel timing of every
    sample_every-th step; returns (phase_ms[4], phase_launches[4]) for phases
    column pass, column separators, row solves, finalize/diagnostics.
    Synchronises."""
    lib = load()
    ld = _field_ld(c, h.params.nx, h.params.ny, ld, "c")
    dptr = _diag(diag_out, 2 * (int(nsteps) + 1))
    cp_ = _devptr(c, "c")
    _, wsp, avail = _handle_ws(h, lib, ws, c.device)
    ms = (ctypes.c_double * 4)()
    cnt = (ctypes.c_int * 4)()
    _check(lib.ch_adi_step_timed(h.handle, cp_, ld, nsteps, dptr, wsp, avail,
                                 _stream(stream), int(sample_every), ms, cnt),
           "ch_adi_step_timed")
    return list(ms), list(cnt)


def chx_stream_copy(src, dst, stream=None):
    """dst[:] = src[:] (float64 device tensors of equal size) with the
    library's plain streaming copy kernel (a measurement reference)."""
    if src.numel() != dst.numel():
        raise ChxError(CHX_EINVAL, "chx_stream_copy: sizes differ")
    _check(load().chx_stream_copy(_devptr(src, "src"), _devptr(dst, "dst"), src.numel(),
                                  _stream(stream)), "chx_stream_copy")


CHX_1D_HYPERDIFFUSION_CN = 0
CHX_1D_DIFFUSION_CN = 1
CHX_1D_CAHN_HILLIARD = 2


class Batch1D:
    """Handle of batch1d_create (one factored cyclic matrix for a batched 1D
    periodic scheme)."""

    def __init__(self, kind, n, L, dt, a, D=1.0):
        h = ctypes.c_void_p()
        _check(load().batch1d_create(int(kind), int(n), float(L), float(dt), float(a), float(D),
                                     ctypes.byref(h)), "batch1d_create")
        self.handle, self.n, self._ws = h, n, None

    def close(self):
        if self.handle:
            load().batch1d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch1d_create(kind, n, L, dt, a, D=1.0) -> Batch1D:
    return Batch1D(kind, n, L, dt, a, D)


def batch1d_step(b: Batch1D, x, nsteps: int = 1, ws=None, ld: int | None = None, stream=None):
    """Advance the interleaved float64 device batch x (n, batch) in place."""
    lib = load()
    if x.dim() != 2 or x.shape[0] != b.n or (x.shape[1] > 1 and x.stride(1) != 1):
        raise ChxError(CHX_EINVAL, "batch1d_step: x must be (n, batch) with unit column stride")
    batch = x.shape[1]
    ld = x.stride(0) if ld is None else ld
    if (b.n > 1 and x.stride(0) != ld) or ld < batch:
        raise ChxError(CHX_EINVAL, "batch1d_step: ld must be x's row stride")
    nbytes = lib.batch1d_ws_bytes(b.handle, batch)
    if ws is None:
        if b._ws is None or b._ws.numel() < nbytes + 256 or b._ws.device != x.device:
            import torch
            b._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=x.device)
        ws = b._ws
    _, wsp, avail = _workspace(nbytes, ws, x.device)
    _check(lib.batch1d_step(b.handle, batch, _devptr(x, "x"), ld, nsteps, wsp, avail,
                            _stream(stream)), "batch1d_step")


def batch1d_step_rewrite(b: Batch1D, x, nsteps: int = 1, ws=None, ld: int | None = None,
                         stream=None):
    """The same steps in the rewrite mode (diagonals written and every system
    factored and solved afresh each step)."""
    lib = load()
    if x.dim() != 2 or x.shape[0] != b.n or (x.shape[1] > 1 and x.stride(1) != 1):
        raise ChxError(CHX_EINVAL, "batch1d_step_rewrite: x must be (n, batch) with unit "
                                   "column stride")
    batch = x.shape[1]
    ld = x.stride(0) if ld is None else ld
    if (b.n > 1 and x.stride(0) != ld) or ld < batch:
        raise ChxError(CHX_EINVAL, "batch1d_step_rewrite: ld must be x's row stride")
    nbytes = lib.batch1d_rewrite_ws_bytes(b.handle, batch)
    ws, wsp, avail = _workspace(nbytes, ws, x.device)
    _check(lib.batch1d_step_rewrite(b.handle, batch, _devptr(x, "x"), ld, nsteps, wsp, avail,
                                    _stream(stream)), "batch1d_step_rewrite")
    return ws


CHX_TUNE_REDUCED_SHAPE = 0
CHX_TUNE_SMALL_PATH = 1
CHX_TUNE_ROW_SPLIT = 2
CHX_NUM_REDUCED_SHAPES = 15
CHX_ROW_SPLIT_OVERLAP = -2
CHX_NUM_SPLIT_SHAPES = 3
CHX_TUNE_COLUMN_ORDER = 3
CHX_NUM_COLUMN_ORDERS = 3
CHX_TUNE_GRAPH = 4
CHX_NUM_ENS_REDUCED_SHAPES = 4
CHX_TUNE_COLUMN_CHUNK = 5
CHX_TUNE_ROW_CHUNK = 6


def ch_get_tuning(h: CH, what: int = CHX_TUNE_REDUCED_SHAPE) -> int:
    """Current kernel choice `what` of the handle (separator tile shape, or
    1/0 for the single-workgroup small-grid path)."""
    v = ctypes.c_int()
    _check(load().ch_get_tuning(h.handle, int(what), ctypes.byref(v)), "ch_get_tuning")
    return v.value


def ch_set_tuning(h: CH, value: int, what: int = CHX_TUNE_REDUCED_SHAPE):
    """Set kernel choice `what` of the handle to value from now on."""
    _check(load().ch_set_tuning(h.handle, int(what), int(value)), "ch_set_tuning")


def ch_set_noise(h: CH, sigma: float, seed: int = 0, step0: int = 0):
    """Cahn-Hilliard-Cook forcing of intensity sigma (0 turns it off)."""
    _check(load().ch_set_noise(h.handle, float(sigma), int(seed) & 0xFFFFFFFFFFFFFFFF,
                               int(step0)), "ch_set_noise")


def ch_get_noise_step(h: CH) -> int:
    v = ctypes.c_uint64()
    _check(load().ch_get_noise_step(h.handle, ctypes.byref(v)), "ch_get_noise_step")
    return v.value


def ch_diagnostics(h: CH, c, ld: int | None = None, stream=None):
    """(mass, free energy) of the device field c; synchronises the stream."""
    cp_, ld = _field(c, h.params.nx, h.params.ny, ld, "c")
    m, e = ctypes.c_double(), ctypes.c_double()
    st = load().ch_diagnostics(h.handle, cp_, ld, ctypes.byref(m), ctypes.byref(e),
                               _stream(stream))
    if st not in (CHX_OK, CHX_ENONFINITE):
        _check(st, "ch_diagnostics")
    return m.value, e.value, st


def ch_energy_decay_rate(diag, nruns: int, nstates: int, t0: float, dt: float, stream=None):
    """beta = -(t / F) dF/dt (Ch.7) of every run and state from a stepping
    call's diagnostics (float64 device tensor of nruns * 2 * nstates values);
    returns a new device tensor of nruns * nstates values."""
    import torch
    if diag.numel() < nruns * 2 * nstates:
        raise ChxError(CHX_EINVAL, "ch_energy_decay_rate: diag holds fewer than "
                                   "nruns * 2 * nstates values")
    beta = torch.empty(nruns * nstates, dtype=torch.float64, device=diag.device)
    _check(load().ch_energy_decay_rate(_devptr(diag, "diag"), nruns, nstates, float(t0),
                                       float(dt), _devptr(beta, "beta"), _stream(stream)),
           "ch_energy_decay_rate")
    return beta


def ch_moments(h: CH, c, ld: int | None = None, stream=None):
    """(<C>, <C^2>, s = 1/(1 - <C^2>)) by Simpson's rule; synchronises."""
    cp_, ld = _field(c, h.params.nx, h.params.ny, ld, "c")
    out = (ctypes.c_double * 3)()
    st = load().ch_moments(h.handle, cp_, ld, out, _stream(stream))
    if st not in (CHX_OK, CHX_ENONFINITE):
        _check(st, "ch_moments")
    return out[0], out[1], out[2]


def ch_k1(h: CH, c, ld: int | None = None, stream=None) -> float:
    """k1 = sum |C^|^2 / sum |k|^-1 |C^|^2 (k != 0); synchronises."""
    cp_, ld = _field(c, h.params.nx, h.params.ny, ld, "c")
    v = ctypes.c_double()
    _check(load().ch_k1(h.handle, cp_, ld, ctypes.byref(v), _stream(stream)), "ch_k1")
    return v.value


# ------------------------------------------------------------- host inspection
def chx_host_chunk_tables(P: int, coef, n: int, m: int):
    """Host-only: (rec[mi,8], blocks[dcount,2,2], dlo) of the chunk tables."""
    import numpy as np
    lib = load()
    cf = (ctypes.c_double * 5)(*[float(v) for v in coef])
    info = (ctypes.c_int * 4)()
    _check(lib.chx_host_chunk_tables(P, cf, n, m, None, 0, None, 0, info), "chunk tables")
    mi, S, dlo, dcount = list(info)
    rec = np.zeros(mi * 8)
    blocks = np.zeros(dcount * 4)
    _check(lib.chx_host_chunk_tables(P, cf, n, m, rec.ctypes.data_as(_DP), rec.size,
                                     blocks.ctypes.data_as(_DP), blocks.size, info),
           "chunk tables")
    return rec.reshape(mi, 8), blocks.reshape(dcount, 2, 2), dlo


def chx_host_whole_tables(P: int, coef, n: int, periodic: bool = True):
    import numpy as np
    lib = load()
    cf = (ctypes.c_double * 5)(*[float(v) for v in coef])
    mi = ctypes.c_int()
    _check(lib.chx_host_whole_tables(P, cf, n, int(periodic), None, 0, None, ctypes.byref(mi)),
           "whole tables")
    rec = np.zeros(mi.value * 8)
    minv = np.zeros(4)
    _check(lib.chx_host_whole_tables(P, cf, n, int(periodic), rec.ctypes.data_as(_DP), rec.size,
                                     minv.ctypes.data_as(_DP), ctypes.byref(mi)), "whole tables")
    return rec.reshape(mi.value, 8), minv.reshape(2, 2)


# --------------------------------------------------------------------- ensembles
class Ensemble:
    """Handle of ch_ensemble_create: many independent runs (each a tuple
    (nx, ny, lx, ly, D, gamma, dt)) advanced together, all in FP64 or all
    FP32-refined with ``refine_passes`` passes (one number, or one per run)."""

    def __init__(self, runs, dtype: int = CHX_F64, refine_passes=0):
        lib = load()
        passes = (list(refine_passes) if hasattr(refine_passes, "__len__")
                  else [refine_passes] * len(runs))
        if len(passes) != len(runs):
            raise ChxError(CHX_EINVAL, "ch_ensemble_create: one refine_passes per run")
        arr = (ChParams * len(runs))(*[ChParams(nx, ny, lx, ly, D, g, dt, dtype, int(p))
                                       for (nx, ny, lx, ly, D, g, dt), p in zip(runs, passes)])
        h = ctypes.c_void_p()
        _check(lib.ch_ensemble_create(len(runs), arr, ctypes.byref(h)), "ch_ensemble_create")
        self.handle = h
        self.nruns = len(runs)
        self.shapes = [(int(r[0]), int(r[1])) for r in runs]  # (nx, ny) per run
        self._ws = None

    def close(self):
        if self.handle:
            load().ch_ensemble_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ch_ensemble_create(runs, dtype: int = CHX_F64, refine_passes=0) -> Ensemble:
    return Ensemble(runs, dtype, refine_passes)


def ch_ensemble_destroy(e: Ensemble) -> None:
    e.close()


def ch_ensemble_ws_bytes(e: Ensemble) -> int:
    return load().ch_ensemble_ws_bytes(e.handle)


def ch_ensemble_get_tuning(ens, what: int = 0) -> int:
    """The FP64 ensemble's separator tile shape (what = CHX_TUNE_REDUCED_SHAPE)."""
    v = ctypes.c_int()
    _check(load().ch_ensemble_get_tuning(ens.handle, int(what), ctypes.byref(v)),
           "ch_ensemble_get_tuning")
    return v.value


def ch_ensemble_set_tuning(ens, value: int, what: int = 0):
    """Set the FP64 ensemble's separator tile shape from now on."""
    _check(load().ch_ensemble_set_tuning(ens.handle, int(what), int(value)),
           "ch_ensemble_set_tuning")


def ch_ensemble_step(e: Ensemble, fields, nsteps: int = 1, diag_out=None, use_graph: bool = True,
                     ws=None, stream=None):
    """Advance every run's float64 device field (list of (ny, nx) tensors) by
    nsteps in place.  diag_out: optional float64 device tensor of
    nruns * 2 * (nsteps + 1) values."""
    import torch
    lib = load()
    ptrs, lds = _ens_fields(e, fields)
    dptr = _diag(diag_out, e.nruns * 2 * (int(nsteps) + 1))
    nbytes = lib.ch_ensemble_ws_bytes(e.handle)
    if ws is None:
        if (e._ws is None or e._ws.numel() < nbytes + 256 or
                e._ws.device != fields[0].device):
            e._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=fields[0].device)
        ws = e._ws
    _, wsp, avail = _workspace(nbytes, ws, fields[0].device)
    _check(lib.ch_ensemble_step(e.handle, ptrs, lds, nsteps, dptr, wsp, avail, int(use_graph),
                                _stream(stream)), "ch_ensemble_step")


def _ens_fields(e: Ensemble, fields):
    if len(fields) != e.nruns:
        raise ChxError(CHX_EINVAL, "one field per run")
    lds = [_field_ld(f, nx, ny, None, f"field {r}")
           for r, (f, (nx, ny)) in enumerate(zip(fields, e.shapes))]
    ptrs = (ctypes.c_void_p * e.nruns)(*[_devptr(f, f"field {r}").value
                                         for r, f in enumerate(fields)])
    return ptrs, (ctypes.c_long * e.nruns)(*lds)


def ch_ensemble_moments(e: Ensemble, fields, stream=None):
    """Per run (<C>, <C^2>, s) as an (nruns, 3) numpy array (synchronises)."""
    import numpy as np
    ptrs, lds = _ens_fields(e, fields)
    out = np.zeros(3 * e.nruns)
    _check(load().ch_ensemble_moments(e.handle, ptrs, lds, out.ctypes.data_as(_DP),
                                      _stream(stream)), "ch_ensemble_moments")
    return out.reshape(e.nruns, 3)


def ch_ensemble_k1(e: Ensemble, fields, stream=None):
    """Per run k1 as a numpy array of nruns values (synchronises)."""
    import numpy as np
    ptrs, lds = _ens_fields(e, fields)
    out = np.zeros(e.nruns)
    _check(load().ch_ensemble_k1(e.handle, ptrs, lds, out.ctypes.data_as(_DP), _stream(stream)),
           "ch_ensemble_k1")
    return out


def ch_ensemble_set_noise(e: Ensemble, sigma: float, seeds=None, step0: int = 0):
    """Cahn-Hilliard-Cook forcing for every run; seeds: one per run."""
    if seeds is None:
        seeds = [0] * e.nruns
    if len(seeds) != e.nruns:
        raise ChxError(CHX_EINVAL, "one seed per run")
    arr = (ctypes.c_uint64 * e.nruns)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in seeds])
    _check(load().ch_ensemble_set_noise(e.handle, float(sigma), arr,
                                        int(step0) & 0xFFFFFFFFFFFFFFFF),
           "ch_ensemble_set_noise")


def ch_ensemble_get_noise_step(e: Ensemble) -> int:
    v = ctypes.c_uint64()
    _check(load().ch_ensemble_get_noise_step(e.handle, ctypes.byref(v)),
           "ch_ensemble_get_noise_step")
    return v.value
