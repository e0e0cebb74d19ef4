"""ctypes binding of libfld.so (include/fld.h), same names as the C ABI.

Argument marshalling only: torch tensors are checked (device, dtype,
contiguity, size) and passed as device pointers; every step of the update
runs in the HIP kernels of the library.  There is no CPU fallback: if the
library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libfld.so")

FLD_OK = 0
FLD_ERR_INVALID_ARG = 1
FLD_ERR_WORKSPACE = 2
FLD_ERR_DEVICE = 3
FLD_ERR_NONPHYSICAL = 4
FLD_ERR_NOT_CONVERGED = 5
FLD_ERR_MODEL = 6

FLD_BC_PERIODIC = 0
FLD_BC_NEUMANN = 1
FLD_BC_DIRICHLET = 2
FLD_LIMITER_LP = 0
FLD_LIMITER_MINERBO = 2
FLD_LIMITER_DIFFUSION = 1
FLD_FACE_ARITH = 0
FLD_FACE_HARMONIC = 1
FLD_PREC_FP64 = 0
FLD_PREC_FP32_IR = 1
FLD_GUESS_PREV = 0
FLD_GUESS_ZERO = 1
FLD_GUESS_LEARNED = 2
FLD_GUESS_ADAPTIVE = 0
FLD_GUESS_EVERY_STEP = 1

EXPORTED = [
    "fld_params_default", "fld_workspace_bytes", "fld_setup", "fld_step",
    "fld_step_noalloc", "fld_exchange", "fld_opacity_powerlaw",
    "fld_explicit_sources", "fld_set_held",
    "fld_kernel_timing_enable",
    "fld_kernel_timing_read", "fld_destroy", "fld_status_str",
    "fld_last_error", "fld_autotune", "fld_tile_shape_name",
]


class fld_params(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double * 3),
        ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
        ("c", ctypes.c_double), ("a_rad", ctypes.c_double),
        ("gamma", ctypes.c_double), ("gas_const", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("face_mean", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("guess", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("max_cycles", ctypes.c_int32),
        ("pre_smooth", ctypes.c_int32), ("post_smooth", ctypes.c_int32),
        ("ir_inner", ctypes.c_int32),
        ("coarse_pre_smooth", ctypes.c_int32),
        ("coarse_post_smooth", ctypes.c_int32),
        ("guess_policy", ctypes.c_int32), ("krylov", ctypes.c_int32),
        ("bc_value_lo", ctypes.c_double * 3),
        ("bc_value_hi", ctypes.c_double * 3),
        ("held_cells", ctypes.c_int32),
    ]


class fld_stats(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
        ("guess_rejected", ctypes.c_int32), ("guess_skipped", ctypes.c_int32),
        ("precond_fp64", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("flagged_cells", ctypes.c_int64),
        ("rel_res_initial", ctypes.c_double),
        ("rel_res_final", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FldError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load libfld.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with "
            "`python -m paper_2503_02764_amd.build` (there is no fallback)")
    # Import torch first: its HIP runtime then serves this library too
    # (same SONAME), so device pointers and streams are shared.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, V, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_double
    lib.fld_params_default.argtypes = [P(fld_params)]
    lib.fld_params_default.restype = None
    lib.fld_workspace_bytes.argtypes = [P(fld_params)]
    lib.fld_workspace_bytes.restype = ctypes.c_size_t
    lib.fld_setup.argtypes = [P(fld_params), V, ctypes.c_size_t, V, P(V)]
    lib.fld_setup.restype = ctypes.c_int
    lib.fld_step.argtypes = [V, D, V, V, V, V, P(fld_stats)]
    lib.fld_step.restype = ctypes.c_int
    lib.fld_step_noalloc.argtypes = [P(fld_params), D, V, V, V, V,
                                     P(fld_stats), V]
    lib.fld_step_noalloc.restype = ctypes.c_int
    lib.fld_explicit_sources.argtypes = [V, V, V, V, V, V, V, V, V]
    lib.fld_explicit_sources.restype = ctypes.c_int
    lib.fld_set_held.argtypes = [V, V, V]
    lib.fld_set_held.restype = ctypes.c_int
    lib.fld_exchange.argtypes = [V, D, V, V, V, V]
    lib.fld_exchange.restype = ctypes.c_int
    lib.fld_opacity_powerlaw.argtypes = [V, V, V, D, D, D, D, D, V]
    lib.fld_opacity_powerlaw.restype = ctypes.c_int
    lib.fld_kernel_timing_enable.argtypes = [V, ctypes.c_int32]
    lib.fld_kernel_timing_enable.restype = ctypes.c_int
    lib.fld_kernel_timing_read.argtypes = [V, P(D), P(ctypes.c_int64), P(D),
                                           P(ctypes.c_char_p)]
    lib.fld_kernel_timing_read.restype = ctypes.c_int
    lib.fld_destroy.argtypes = [V]
    lib.fld_destroy.restype = None
    lib.fld_status_str.argtypes = [ctypes.c_int32]
    lib.fld_status_str.restype = ctypes.c_char_p
    lib.fld_last_error.argtypes = [V]
    lib.fld_last_error.restype = ctypes.c_char_p
    lib.fld_autotune.argtypes = [V, P(ctypes.c_int32), ctypes.c_int32]
    lib.fld_autotune.restype = ctypes.c_int
    lib.fld_tile_shape_name.argtypes = [ctypes.c_int32]
    lib.fld_tile_shape_name.restype = ctypes.c_char_p
    _batch_argtypes(lib)
    _lib = lib
    return lib


def status_str(status):
    return load().fld_status_str(status).decode()


def _check(ctx_ptr, status):
    if status != FLD_OK:
        msg = load().fld_last_error(ctx_ptr).decode()
        raise FldError(status, msg)


def fld_params_default(**overrides):
    p = fld_params()
    load().fld_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if k in ("n", "dx", "bc_lo", "bc_hi", "bc_value_lo", "bc_value_hi"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


def fld_workspace_bytes(params):
    return int(load().fld_workspace_bytes(ctypes.byref(params)))


def _ptr(t, name, numel=None, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Ctx:
    """An fld_ctx* with the workspace tensor it borrows and its stream."""

    def __init__(self, ptr, params, workspace, stream):
        self.ptr = ptr
        self.params = params
        self.workspace = workspace
        self.stream = stream
        self.cells = int(params.n[0] * params.n[1] * params.n[2])

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.fld_destroy(self.ptr)
            self.ptr = None


def fld_setup(params, workspace=None, stream=None):
    """Create a context; allocates the workspace tensor if none is given."""
    import torch
    lib = load()
    need = fld_workspace_bytes(params)
    if need == 0:
        out = ctypes.c_void_p()
        st = lib.fld_setup(ctypes.byref(params), None, 0, None,
                           ctypes.byref(out))
        _check(None, st)
        raise FldError(FLD_ERR_INVALID_ARG, "invalid parameters")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    if stream is None:
        stream = torch.cuda.current_stream()
    out = ctypes.c_void_p()
    st = lib.fld_setup(ctypes.byref(params),
                       _ptr(workspace, "workspace", dtype=torch.uint8),
                       workspace.numel(), ctypes.c_void_p(stream.cuda_stream),
                       ctypes.byref(out))
    _check(None, st)
    return Ctx(out, params, workspace, stream)


def fld_step(ctx, dt, rho, kappa, E_in, E_out, stats=True, check=True):
    """Diffusion step; returns (status, stats dict or None)."""
    import torch
    n = ctx.cells
    s = fld_stats() if stats else None
    st = load().fld_step(ctx.ptr, float(dt),
                         _ptr(rho, "rho", n, torch.float64),
                         _ptr(kappa, "kappa", n, torch.float64),
                         _ptr(E_in, "E_in", n, torch.float64),
                         _ptr(E_out, "E_out", n, torch.float64),
                         ctypes.byref(s) if s is not None else None)
    if check:
        _check(ctx.ptr, st)
    return st, (s.as_dict() if s is not None else None)


def fld_step_noalloc(params, dt, rho, kappa, E_in, E_out, stats=True,
                     check=True, stream=None):
    """fld_step without a context or workspace (the library's static
    scratch); returns (status, stats dict or None)."""
    import torch
    n = int(params.n[0] * params.n[1] * params.n[2])
    if stream is None:
        stream = torch.cuda.current_stream()
    s = fld_stats() if stats else None
    st = load().fld_step_noalloc(ctypes.byref(params), float(dt),
                                 _ptr(rho, "rho", n, torch.float64),
                                 _ptr(kappa, "kappa", n, torch.float64),
                                 _ptr(E_in, "E_in", n, torch.float64),
                                 _ptr(E_out, "E_out", n, torch.float64),
                                 ctypes.byref(s) if s is not None else None,
                                 ctypes.c_void_p(stream.cuda_stream))
    if check:
        _check(None, st)
    return st, (s.as_dict() if s is not None else None)


def fld_explicit_sources(ctx, rho, kappa, E, v=None, f_r=None, work=None,
                         tiring=None, fedd=None, check=True):
    """Explicit source terms; v and f_r are lists of ndim device tensors (or
    None), work / tiring / fedd device tensors or None."""
    import torch
    n = ctx.cells
    nd = int(ctx.params.ndim)

    def arr(ts, name):
        if ts is None:
            return None, None
        if len(ts) != nd:
            raise ValueError(f"{name} needs {nd} components")
        a = (ctypes.c_void_p * nd)(*[_ptr(t, f"{name}[{i}]", n, torch.float64)
                                     for i, t in enumerate(ts)])
        return ctypes.cast(a, ctypes.c_void_p), a

    vp, _va = arr(v, "v")
    fp, _fa = arr(f_r, "f_r")

    def opt(t, name):
        return None if t is None else _ptr(t, name, n, torch.float64)

    st = load().fld_explicit_sources(
        ctx.ptr, _ptr(rho, "rho", n, torch.float64),
        _ptr(kappa, "kappa", n, torch.float64), _ptr(E, "E", n, torch.float64),
        vp, fp, opt(work, "work"), opt(tiring, "tiring"), opt(fedd, "fedd"))
    if check:
        _check(ctx.ptr, st)
    return st


def fld_set_held(ctx, mask, E_hold, check=True):
    """Held cells of a context set up with held_cells = 1: `mask` a uint8
    device tensor (nonzero = held), `E_hold` a float64 device tensor of the
    same cells, or both None to clear.  The library keeps the pointers, so
    the context keeps the tensors alive until the next call."""
    import torch
    n = ctx.cells
    if mask is None and E_hold is None:
        mp = hp = None
    else:
        mp = _ptr(mask, "mask", n, torch.uint8)
        hp = _ptr(E_hold, "E_hold", n, torch.float64)
    st = load().fld_set_held(ctx.ptr, mp, hp)
    if check:
        _check(ctx.ptr, st)
    if st == FLD_OK:
        ctx.held = (mask, E_hold)
    return st


def fld_exchange(ctx, dt, rho, kappa, E, e_int, check=True):
    import torch
    n = ctx.cells
    st = load().fld_exchange(ctx.ptr, float(dt),
                             _ptr(rho, "rho", n, torch.float64),
                             _ptr(kappa, "kappa", n, torch.float64),
                             _ptr(E, "E", n, torch.float64),
                             _ptr(e_int, "e_int", n, torch.float64))
    if check:
        _check(ctx.ptr, st)
    return st


def fld_opacity_powerlaw(ctx, rho, e_int, k0, a, b, kmin, kmax, kappa,
                         check=True):
    import torch
    n = ctx.cells
    st = load().fld_opacity_powerlaw(ctx.ptr,
                                     _ptr(rho, "rho", n, torch.float64),
                                     _ptr(e_int, "e_int", n, torch.float64),
                                     float(k0), float(a), float(b),
                                     float(kmin), float(kmax),
                                     _ptr(kappa, "kappa", n, torch.float64))
    if check:
        _check(ctx.ptr, st)
    return st


def fld_kernel_timing_enable(ctx, on=True):
    _check(ctx.ptr, load().fld_kernel_timing_enable(ctx.ptr, 1 if on else 0))


def fld_kernel_timing_read(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    by = ctypes.c_double()
    name = ctypes.c_char_p()
    _check(ctx.ptr, load().fld_kernel_timing_read(
        ctx.ptr, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by),
        ctypes.byref(name)))
    return dict(ms=ms.value, launches=n.value, bytes=by.value,
                kernel=name.value.decode())


def fld_autotune(ctx, max_levels=24):
    """Tune the tile shapes; returns [(down, up) shape name per level]."""
    lib = load()
    arr = (ctypes.c_int32 * (2 * max_levels))()
    _check(ctx.ptr, lib.fld_autotune(ctx.ptr, arr, max_levels))
    return [(lib.fld_tile_shape_name(arr[2 * l]).decode(),
             lib.fld_tile_shape_name(arr[2 * l + 1]).decode())
            for l in range(max_levels)]


def fld_destroy(ctx):
    if ctx.ptr:
        load().fld_destroy(ctx.ptr)
        ctx.ptr = None


# ---- batched grids -----------------------------------------------------------

EXPORTED += ["fld_workspace_bytes_batch", "fld_setup_batch", "fld_step_batch",
             "fld_exchange_batch", "fld_opacity_powerlaw_batch",
             "fld_batch_set_graph"]


# ---- block-adaptive 2D grids -------------------------------------------

EXPORTED += ["fld_amr_workspace_bytes", "fld_amr_setup", "fld_amr_step",
             "fld_amr_last_error", "fld_amr_destroy",
             "fld_amr_kernel_timing_enable", "fld_amr_kernel_timing_read",
             "fld_amr_exchange", "fld_amr_opacity_powerlaw",
             "fld_amr_workspace_bytes_levels", "fld_amr_setup_levels"]


def _amr_argtypes(lib):
    if getattr(lib, "_amr_ready", False):
        return
    P, V, D, I32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32
    lib.fld_amr_workspace_bytes.argtypes = [P(fld_params), I32, V, I32]
    lib.fld_amr_workspace_bytes.restype = ctypes.c_size_t
    lib.fld_amr_setup.argtypes = [P(fld_params), I32, V, I32, V,
                                  ctypes.c_size_t, V, P(V)]
    lib.fld_amr_setup.restype = ctypes.c_int
    lib.fld_amr_workspace_bytes_levels.argtypes = [P(fld_params), I32, I32,
                                                   V, V]
    lib.fld_amr_workspace_bytes_levels.restype = ctypes.c_size_t
    lib.fld_amr_setup_levels.argtypes = [P(fld_params), I32, I32, V, V, V,
                                         ctypes.c_size_t, V, P(V)]
    lib.fld_amr_setup_levels.restype = ctypes.c_int
    lib.fld_amr_step.argtypes = [V, D, V, V, V, V, V, V, V, V, V]
    lib.fld_amr_step.restype = ctypes.c_int
    lib.fld_amr_last_error.argtypes = [V]
    lib.fld_amr_last_error.restype = ctypes.c_char_p
    lib.fld_amr_destroy.argtypes = [V]
    lib.fld_amr_destroy.restype = None
    lib.fld_amr_exchange.argtypes = [V, D, V, V, V, V, V, V, V, V]
    lib.fld_amr_exchange.restype = ctypes.c_int
    lib.fld_amr_opacity_powerlaw.argtypes = [V, V, V, V, V, D, D, D, D, D, V,
                                             V]
    lib.fld_amr_opacity_powerlaw.restype = ctypes.c_int
    lib.fld_amr_kernel_timing_enable.argtypes = [V, I32]
    lib.fld_amr_kernel_timing_enable.restype = ctypes.c_int
    lib.fld_amr_kernel_timing_read.argtypes = [V, P(D), P(ctypes.c_int64),
                                               P(D), P(ctypes.c_char_p)]
    lib.fld_amr_kernel_timing_read.restype = ctypes.c_int
    lib._amr_ready = True


def _amrlib():
    lib = load()
    _amr_argtypes(lib)
    return lib


def _blocks_arr(blocks):
    flat = [int(v) for xy in blocks for v in xy]
    return (ctypes.c_int32 * max(1, len(flat)))(*flat), len(blocks)


class AmrCtx:
    """An fld_amr_ctx* with its workspace, stream and sizes."""

    def __init__(self, ptr, params, block, nblocks, workspace, stream):
        self.ptr = ptr
        self.params = params
        self.block = block
        self.nblocks = nblocks
        self.workspace = workspace
        self.stream = stream
        self.base_cells = int(params.n[0] * params.n[1])
        self.fine_cells = nblocks * 4 * block * block

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.fld_amr_destroy(self.ptr)
            self.ptr = None


def _levels(blocks):
    """A list of (bx, by) is one level; a list of such lists, several."""
    if blocks and isinstance(blocks[0][0], (list, tuple)):
        return [list(b) for b in blocks]
    return [list(blocks)]


def _levels_arr(levels):
    counts = (ctypes.c_int32 * max(1, len(levels)))(*[len(b) for b in levels])
    flat = [int(v) for bl in levels for xy in bl for v in xy]
    return counts, (ctypes.c_int32 * max(1, len(flat)))(*flat)


def fld_amr_workspace_bytes(params, block, blocks):
    levels = _levels(blocks)
    counts, arr = _levels_arr(levels)
    return int(_amrlib().fld_amr_workspace_bytes_levels(
        ctypes.byref(params), block, len(levels), counts, arr))


def fld_amr_setup(params, block, blocks, workspace=None, stream=None):
    """Context of a block-adaptive 2D grid: `blocks` lists the refined
    base blocks as (bx, by), or is a list of such lists, one per refined
    level (level l's corners in units of `block` level-(l-1) cells)."""
    import torch
    lib = _amrlib()
    levels = _levels(blocks)
    counts, arr = _levels_arr(levels)
    need = fld_amr_workspace_bytes(params, block, blocks)
    out = ctypes.c_void_p()
    if need == 0:
        st = lib.fld_amr_setup_levels(ctypes.byref(params), block,
                                      len(levels), counts, arr, None, 0, None,
                                      ctypes.byref(out))
        raise FldError(st, lib.fld_amr_last_error(None).decode())
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib.fld_amr_setup_levels(
        ctypes.byref(params), block, len(levels), counts, arr,
        _ptr(workspace, "workspace", dtype=torch.uint8), workspace.numel(),
        ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
    if st != FLD_OK:
        raise FldError(st, lib.fld_amr_last_error(None).decode())
    return AmrCtx(out, params, block, sum(len(b) for b in levels), workspace,
                  stream)


def _amr_fine(ctx, t, name):
    import torch
    return _ptr(t, name, ctx.fine_cells, torch.float64) if ctx.fine_cells \
        else None


def fld_amr_exchange(ctx, dt, rho_b, kappa_b, E_b, e_b, rho_f, kappa_f, E_f,
                     e_f, check=True):
    """The exchange quartic on the base and fine arrays (in place)."""
    import torch
    lib = _amrlib()
    nb = ctx.base_cells
    f64 = torch.float64
    st = lib.fld_amr_exchange(ctx.ptr, float(dt),
                              _ptr(rho_b, "rho_b", nb, f64),
                              _ptr(kappa_b, "kappa_b", nb, f64),
                              _ptr(E_b, "E_b", nb, f64),
                              _ptr(e_b, "e_b", nb, f64),
                              _amr_fine(ctx, rho_f, "rho_f"),
                              _amr_fine(ctx, kappa_f, "kappa_f"),
                              _amr_fine(ctx, E_f, "E_f"),
                              _amr_fine(ctx, e_f, "e_f"))
    if check and st != FLD_OK:
        raise FldError(st, lib.fld_amr_last_error(ctx.ptr).decode())
    return st


def fld_amr_opacity_powerlaw(ctx, rho_b, e_b, rho_f, e_f, k0, a, b, kmin,
                             kmax, kappa_b, kappa_f, check=True):
    import torch
    lib = _amrlib()
    nb = ctx.base_cells
    f64 = torch.float64
    st = lib.fld_amr_opacity_powerlaw(
        ctx.ptr, _ptr(rho_b, "rho_b", nb, f64), _ptr(e_b, "e_b", nb, f64),
        _amr_fine(ctx, rho_f, "rho_f"), _amr_fine(ctx, e_f, "e_f"),
        float(k0), float(a), float(b), float(kmin), float(kmax),
        _ptr(kappa_b, "kappa_b", nb, f64), _amr_fine(ctx, kappa_f, "kappa_f"))
    if check and st != FLD_OK:
        raise FldError(st, lib.fld_amr_last_error(ctx.ptr).decode())
    return st


def fld_amr_kernel_timing_enable(ctx, on=True):
    _amrlib().fld_amr_kernel_timing_enable(ctx.ptr, int(bool(on)))


def fld_amr_kernel_timing_read(ctx):
    """dict(kernel, ms, launches, bytes) since the last read."""
    ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    name = ctypes.c_char_p()
    _amrlib().fld_amr_kernel_timing_read(ctx.ptr, ctypes.byref(ms),
                                         ctypes.byref(n), ctypes.byref(by),
                                         ctypes.byref(name))
    return {"kernel": name.value.decode() if name.value else "none",
            "ms": ms.value, "launches": n.value, "bytes": by.value}


def fld_amr_step(ctx, dt, rho_b, kappa_b, E_b_in, E_b_out, rho_f, kappa_f,
                 E_f_in, E_f_out, check=True):
    """Block-adaptive diffusion step; returns (status, stats dict)."""
    import torch
    lib = _amrlib()
    nb, nf = ctx.base_cells, ctx.fine_cells
    f64 = torch.float64

    def fine(t, name):
        return _ptr(t, name, nf, f64) if nf else None
    s = fld_stats()
    st = lib.fld_amr_step(ctx.ptr, float(dt), _ptr(rho_b, "rho_b", nb, f64),
                          _ptr(kappa_b, "kappa_b", nb, f64),
                          _ptr(E_b_in, "E_b_in", nb, f64),
                          _ptr(E_b_out, "E_b_out", nb, f64),
                          fine(rho_f, "rho_f"), fine(kappa_f, "kappa_f"),
                          fine(E_f_in, "E_f_in"), fine(E_f_out, "E_f_out"),
                          ctypes.byref(s))
    if check and st != FLD_OK:
        raise FldError(st, lib.fld_amr_last_error(ctx.ptr).decode())
    return st, s.as_dict()


def _batch_argtypes(lib):
    P, V, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_double
    VP = P(ctypes.c_void_p)
    lib.fld_workspace_bytes_batch.argtypes = [ctypes.c_int32, P(fld_params)]
    lib.fld_workspace_bytes_batch.restype = ctypes.c_size_t
    lib.fld_setup_batch.argtypes = [ctypes.c_int32, P(fld_params), V,
                                    ctypes.c_size_t, V, P(V)]
    lib.fld_setup_batch.restype = ctypes.c_int
    lib.fld_step_batch.argtypes = [V, P(D), VP, VP, VP, VP, P(fld_stats)]
    lib.fld_step_batch.restype = ctypes.c_int
    lib.fld_exchange_batch.argtypes = [V, P(D), VP, VP, VP, VP]
    lib.fld_exchange_batch.restype = ctypes.c_int
    lib.fld_opacity_powerlaw_batch.argtypes = [V, VP, VP, D, D, D, D, D, VP]
    lib.fld_opacity_powerlaw_batch.restype = ctypes.c_int
    lib.fld_batch_set_graph.argtypes = [V, ctypes.c_int32]
    lib.fld_batch_set_graph.restype = ctypes.c_int


class BatchCtx:
    """A batched fld_ctx* over `count` grids and the workspace it borrows."""

    def __init__(self, ptr, params_list, workspace, stream):
        self.ptr = ptr
        self.params = params_list
        self.workspace = workspace
        self.stream = stream
        self.count = len(params_list)
        self.cells = [int(p.n[0] * p.n[1] * p.n[2]) for p in params_list]

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.fld_destroy(self.ptr)
            self.ptr = None


def _params_array(params_list):
    arr = (fld_params * len(params_list))()
    for i, p in enumerate(params_list):
        arr[i] = p
    return arr


def fld_workspace_bytes_batch(params_list):
    lib = load()
    _batch_argtypes(lib)
    arr = _params_array(params_list)
    return int(lib.fld_workspace_bytes_batch(len(params_list), arr))


def fld_setup_batch(params_list, workspace=None, stream=None):
    import torch
    lib = load()
    _batch_argtypes(lib)
    arr = _params_array(params_list)
    need = int(lib.fld_workspace_bytes_batch(len(params_list), arr))
    out = ctypes.c_void_p()
    if need == 0:
        st = lib.fld_setup_batch(len(params_list), arr, None, 0, None,
                                 ctypes.byref(out))
        _check(None, st)
        raise FldError(FLD_ERR_INVALID_ARG, "invalid parameters")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib.fld_setup_batch(len(params_list), arr,
                             _ptr(workspace, "workspace", dtype=torch.uint8),
                             workspace.numel(),
                             ctypes.c_void_p(stream.cuda_stream),
                             ctypes.byref(out))
    _check(None, st)
    return BatchCtx(out, params_list, workspace, stream)


def _ptr_array(ctx, tensors, name):
    import torch
    if len(tensors) != ctx.count:
        raise ValueError(f"{name}: expected {ctx.count} tensors")
    arr = (ctypes.c_void_p * ctx.count)()
    for i, t in enumerate(tensors):
        arr[i] = _ptr(t, f"{name}[{i}]", ctx.cells[i], torch.float64).value
    return arr


def fld_step_batch(ctx, dts, rho, kappa, E_in, E_out, check=True):
    """Diffusion step of every grid; returns (status, list of stats dicts)."""
    lib = load()
    dt = (ctypes.c_double * ctx.count)(*[float(v) for v in dts])
    stats = (fld_stats * ctx.count)()
    st = lib.fld_step_batch(ctx.ptr, dt, _ptr_array(ctx, rho, "rho"),
                            _ptr_array(ctx, kappa, "kappa"),
                            _ptr_array(ctx, E_in, "E_in"),
                            _ptr_array(ctx, E_out, "E_out"), stats)
    if check:
        _check(ctx.ptr, st)
    return st, [s.as_dict() for s in stats]


def fld_exchange_batch(ctx, dts, rho, kappa, E, e_int, check=True):
    lib = load()
    dt = (ctypes.c_double * ctx.count)(*[float(v) for v in dts])
    st = lib.fld_exchange_batch(ctx.ptr, dt, _ptr_array(ctx, rho, "rho"),
                                _ptr_array(ctx, kappa, "kappa"),
                                _ptr_array(ctx, E, "E"),
                                _ptr_array(ctx, e_int, "e_int"))
    if check:
        _check(ctx.ptr, st)
    return st


def fld_opacity_powerlaw_batch(ctx, rho, e_int, k0, a, b, kmin, kmax, kappa,
                               check=True):
    lib = load()
    st = lib.fld_opacity_powerlaw_batch(
        ctx.ptr, _ptr_array(ctx, rho, "rho"), _ptr_array(ctx, e_int, "e_int"),
        float(k0), float(a), float(b), float(kmin), float(kmax),
        _ptr_array(ctx, kappa, "kappa"))
    if check:
        _check(ctx.ptr, st)
    return st


def fld_batch_set_graph(ctx, on=True):
    lib = load()
    _check(ctx.ptr, lib.fld_batch_set_graph(ctx.ptr, 1 if on else 0))


# ---- learned initial guess (include/fldnn.h) --------------------------------

EXPORTED_NN = ["fldnn_param_count", "fldnn_workspace_bytes", "fldnn_create",
               "fldnn_set_params", "fldnn_get_params", "fldnn_forward",
               "fldnn_gradients", "fldnn_train_step", "fldnn_destroy",
               "fldnn_set_loss", "fldnn_last_error",
               "fld_features", "fld_set_model"]


def _nn_argtypes(lib):
    if getattr(lib, "_nn_ready", False):
        return
    P, V, F = ctypes.POINTER, ctypes.c_void_p, ctypes.c_float
    I32, SZ = ctypes.c_int32, ctypes.c_size_t
    lib.fldnn_param_count.argtypes = []
    lib.fldnn_param_count.restype = SZ
    lib.fldnn_workspace_bytes.argtypes = [I32, I32, I32, I32]
    lib.fldnn_workspace_bytes.restype = SZ
    lib.fldnn_create.argtypes = [I32, I32, I32, I32, V, SZ, V, P(V)]
    lib.fldnn_create.restype = ctypes.c_int
    lib.fldnn_set_params.argtypes = [V, P(F), SZ]
    lib.fldnn_set_params.restype = ctypes.c_int
    lib.fldnn_get_params.argtypes = [V, P(F), SZ]
    lib.fldnn_get_params.restype = ctypes.c_int
    lib.fldnn_forward.argtypes = [V, V, V]
    lib.fldnn_forward.restype = ctypes.c_int
    lib.fldnn_gradients.argtypes = [V, V, V, P(F), P(F), SZ]
    lib.fldnn_gradients.restype = ctypes.c_int
    lib.fldnn_train_step.argtypes = [V, V, V, F, I32, P(F)]
    lib.fldnn_train_step.restype = ctypes.c_int
    lib.fldnn_last_error.argtypes = []
    lib.fldnn_last_error.restype = ctypes.c_char_p
    lib.fldnn_set_loss.argtypes = [V, I32]
    lib.fldnn_set_loss.restype = ctypes.c_int
    lib.fldnn_destroy.argtypes = [V]
    lib.fldnn_destroy.restype = None
    lib.fld_features.argtypes = [V, ctypes.c_double, V, V, V, V]
    lib.fld_features.restype = ctypes.c_int
    lib.fld_set_model.argtypes = [V, P(F), SZ]
    lib.fld_set_model.restype = ctypes.c_int
    lib._nn_ready = True


def _nnlib():
    lib = load()
    _nn_argtypes(lib)
    return lib


def _check_nn(status):
    if status != FLD_OK:
        raise FldError(status, _nnlib().fldnn_last_error().decode())


def _f32_host(arr, count):
    import numpy as np
    a = np.ascontiguousarray(arr, dtype=np.float32).reshape(-1)
    if a.size != count:
        raise ValueError(f"expected {count} parameters, got {a.size}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def fldnn_param_count():
    return int(_nnlib().fldnn_param_count())


def fldnn_workspace_bytes(N, H, W, training):
    return int(_nnlib().fldnn_workspace_bytes(N, H, W, 1 if training else 0))


class Net:
    """An fldnn* with the workspace tensor it borrows and its stream."""

    def __init__(self, ptr, shape, training, workspace, stream):
        self.ptr = ptr
        self.shape = shape
        self.training = training
        self.workspace = workspace
        self.stream = stream
        self.count = fldnn_param_count()

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.fldnn_destroy(self.ptr)
            self.ptr = None


def fldnn_create(N, H, W, training=False, workspace=None, stream=None):
    import torch
    lib = _nnlib()
    need = fldnn_workspace_bytes(N, H, W, training)
    if need == 0:
        raise FldError(FLD_ERR_INVALID_ARG,
                       f"invalid network shape N={N} H={H} W={W}")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    if stream is None:
        stream = torch.cuda.current_stream()
    out = ctypes.c_void_p()
    st = lib.fldnn_create(N, H, W, 1 if training else 0,
                          _ptr(workspace, "workspace", dtype=torch.uint8),
                          workspace.numel(),
                          ctypes.c_void_p(stream.cuda_stream),
                          ctypes.byref(out))
    _check_nn(st)
    return Net(out, (N, H, W), training, workspace, stream)


def fldnn_set_params(net, flat):
    a, p = _f32_host(flat, net.count)
    _check_nn(_nnlib().fldnn_set_params(net.ptr, p, a.size))


def fldnn_get_params(net):
    import numpy as np
    a = np.empty(net.count, dtype=np.float32)
    _check_nn(_nnlib().fldnn_get_params(
        net.ptr, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
    return a


def fldnn_forward(net, inputs, delta):
    import torch
    N, H, W = net.shape
    _check_nn(_nnlib().fldnn_forward(
        net.ptr, _ptr(inputs, "inputs", N * H * W * 4, torch.float32),
        _ptr(delta, "delta", N * H * W, torch.float32)))


def fldnn_gradients(net, inputs, targets):
    """Returns (loss, FP32 gradient array in the parameter layout)."""
    import numpy as np
    import torch
    N, H, W = net.shape
    g = np.empty(net.count, dtype=np.float32)
    loss = ctypes.c_float()
    _check_nn(_nnlib().fldnn_gradients(
        net.ptr, _ptr(inputs, "inputs", N * H * W * 4, torch.float32),
        _ptr(targets, "targets", N * H * W, torch.float32),
        ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
        g.size))
    return float(loss.value), g


def fldnn_train_step(net, inputs, targets, lr, step, want_loss=False):
    import torch
    N, H, W = net.shape
    loss = ctypes.c_float()
    _check_nn(_nnlib().fldnn_train_step(
        net.ptr, _ptr(inputs, "inputs", N * H * W * 4, torch.float32),
        _ptr(targets, "targets", N * H * W, torch.float32), float(lr),
        int(step), ctypes.byref(loss) if want_loss else None))
    return float(loss.value) if want_loss else None


FLDNN_LOSS_MSE = 0
FLDNN_LOSS_ENERGY = 1


def fldnn_set_loss(net, kind):
    """kind: "mse" or "energy" (see include/fldnn.h)."""
    code = {"mse": FLDNN_LOSS_MSE, "energy": FLDNN_LOSS_ENERGY}[kind]
    _check_nn(_nnlib().fldnn_set_loss(net.ptr, code))


def fldnn_destroy(net):
    if net.ptr:
        _nnlib().fldnn_destroy(net.ptr)
        net.ptr = None


def fld_features(ctx, dt, rho, kappa, E, out):
    import torch
    n = ctx.cells
    _check(ctx.ptr, _nnlib().fld_features(
        ctx.ptr, float(dt), _ptr(rho, "rho", n, torch.float64),
        _ptr(kappa, "kappa", n, torch.float64),
        _ptr(E, "E", n, torch.float64),
        _ptr(out, "out", 4 * n, torch.float32)))


def fld_set_model(ctx, flat):
    lib = _nnlib()
    a, p = _f32_host(flat, fldnn_param_count())
    _check(ctx.ptr, lib.fld_set_model(ctx.ptr, p, a.size))
