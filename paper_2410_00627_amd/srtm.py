"""Python binding of libsrtm (argument marshalling only).

Every function here validates tensor placement, allocates outputs and workspace with
torch on the current device and stream, and calls the C-ABI entry point of the same
name in libsrtm.so. All arithmetic runs in the HIP kernels; there is no fallback. A
missing library or a non-GPU tensor raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsrtm.so")

SRTM_F32, SRTM_F64 = 0, 1
INFO_BITS = {1: "innovation covariance not positive definite", 2: "I + D_i J_j singular in the filter combine",
             4: "smoother prediction covariance singular", 8: "non-finite output"}


class SrtmError(RuntimeError):
    pass


class Shape(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("L", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("N", ctypes.c_int64)]


class SeqC(ctypes.Structure):
    """srtm_seq: one sequence of a batch (device pointers)."""
    _fields_ = ([(n, ctypes.c_void_p) for n in ("F", "Q", "H", "R", "m0", "P0", "y",
                                                 "ms_fast", "Ps_fast", "ms_slow", "Ps_slow")] +
                [("N", ctypes.c_int64), ("L", ctypes.c_int32), ("reserved", ctypes.c_int32)])


class SeqExC(ctypes.Structure):
    """srtm_seq_ex: one sequence of a mixed batch (its own nx, ny; optional inputs or per-window model)."""
    _fields_ = ([("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("L", ctypes.c_int32), ("per_window", ctypes.c_int32),
                 ("N", ctypes.c_int64)] +
                [(n, ctypes.c_void_p) for n in ("F", "Q", "H", "R", "m0", "P0", "y", "B", "u")] +
                [("nu", ctypes.c_int32), ("reserved", ctypes.c_int32)] +
                [(n, ctypes.c_void_p) for n in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow")])


class InputsC(ctypes.Structure):
    """srtm_inputs: known inputs B [nx][nu] and u [N][L][nu] (device pointers)."""
    _fields_ = [("B", ctypes.c_void_p), ("u", ctypes.c_void_p), ("nu", ctypes.c_int32), ("reserved", ctypes.c_int32)]


MAX_NU = 4
_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded libsrtm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SrtmError(f"{LIB_PATH} not found: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    L.srtm_workspace_size.argtypes = [ctypes.POINTER(Shape), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.srtm_workspace_size.restype = ctypes.c_int
    L.srtm_workspace_size_inputs.argtypes = L.srtm_workspace_size.argtypes
    L.srtm_workspace_size_inputs.restype = ctypes.c_int
    L.srtm_workspace_size_tv.argtypes = L.srtm_workspace_size.argtypes
    L.srtm_workspace_size_tv.restype = ctypes.c_int
    L.srtm_supported.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.srtm_supported.restype = ctypes.c_int32
    L.srtm_filter.argtypes = [ctypes.POINTER(Shape)] + [_vp] * 12 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_filter.restype = ctypes.c_int
    L.srtm_smooth.argtypes = [ctypes.POINTER(Shape)] + [_vp] * 16 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_smooth.restype = ctypes.c_int
    L.srtm_filter_tv.argtypes = L.srtm_filter.argtypes
    L.srtm_filter_tv.restype = ctypes.c_int
    L.srtm_smooth_tv.argtypes = L.srtm_smooth.argtypes
    L.srtm_smooth_tv.restype = ctypes.c_int
    L.srtm_smooth_lag1.argtypes = [ctypes.POINTER(Shape)] + [_vp] * 13 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_smooth_lag1.restype = ctypes.c_int
    L.srtm_smooth_sequential.argtypes = [ctypes.POINTER(Shape)] + [_vp] * 12 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_smooth_sequential.restype = ctypes.c_int
    L.srtm_smooth_noalloc.argtypes = [ctypes.POINTER(Shape)] + [_vp] * 17
    L.srtm_smooth_noalloc.restype = ctypes.c_int
    L.srtm_smooth_profiled.argtypes = ([ctypes.POINTER(Shape)] + [_vp] * 16 +
                                       [ctypes.c_size_t, _vp, _vp, ctypes.POINTER(_vp), ctypes.c_int32])
    L.srtm_smooth_profiled.restype = ctypes.c_int
    L.srtm_batch_plan.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(SeqC),
                                  ctypes.c_int32, _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t),
                                  ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int32)]
    L.srtm_batch_plan.restype = ctypes.c_int
    L.srtm_smooth_batch.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp, _vp]
    L.srtm_smooth_batch.restype = ctypes.c_int
    L.srtm_loglik_grad_batch.argtypes = L.srtm_smooth_batch.argtypes
    L.srtm_loglik_grad_batch.restype = ctypes.c_int
    L.srtm_batch_plan_ex.argtypes = [ctypes.c_int32, ctypes.POINTER(SeqExC), ctypes.c_int32, _vp, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
    L.srtm_batch_plan_ex.restype = ctypes.c_int
    L.srtm_smooth_batch_ex.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
    L.srtm_smooth_batch_ex.restype = ctypes.c_int
    L.srtm_graph_begin.argtypes = [_vp]
    L.srtm_graph_begin.restype = ctypes.c_int
    L.srtm_graph_end.argtypes = [_vp, ctypes.POINTER(_vp)]
    L.srtm_graph_end.restype = ctypes.c_int
    L.srtm_graph_launch.argtypes = [_vp, _vp]
    L.srtm_graph_launch.restype = ctypes.c_int
    L.srtm_graph_destroy.argtypes = [_vp]
    L.srtm_graph_destroy.restype = ctypes.c_int
    L.srtm_loglik.argtypes = [ctypes.POINTER(Shape)] + [_vp] * 9 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_loglik.restype = ctypes.c_int
    L.srtm_loglik_grad.argtypes = [ctypes.POINTER(Shape)] + [_vp] * 12 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_loglik_grad.restype = ctypes.c_int
    _si = [ctypes.POINTER(Shape), ctypes.POINTER(InputsC)]
    L.srtm_filter_inputs.argtypes = _si + [_vp] * 12 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_filter_inputs.restype = ctypes.c_int
    L.srtm_smooth_inputs.argtypes = _si + [_vp] * 16 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_smooth_inputs.restype = ctypes.c_int
    L.srtm_loglik_inputs.argtypes = _si + [_vp] * 9 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_loglik_inputs.restype = ctypes.c_int
    L.srtm_loglik_grad_inputs.argtypes = _si + [_vp] * 12 + [ctypes.c_size_t, _vp, _vp]
    L.srtm_loglik_grad_inputs.restype = ctypes.c_int
    L.srtm_kernel_count.argtypes = [ctypes.c_int32]
    L.srtm_kernel_count.restype = ctypes.c_int32
    L.srtm_kernel_name.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.srtm_kernel_name.restype = ctypes.c_char_p
    L.srtm_status_string.argtypes = [ctypes.c_int32]
    L.srtm_status_string.restype = ctypes.c_char_p
    L.srtm_version.argtypes = []
    L.srtm_version.restype = ctypes.c_int32
    _lib = L
    return L


def status_string(code: int) -> str:
    return lib().srtm_status_string(code).decode()


def _check(code: int, what: str):
    if code != 0:
        raise SrtmError(f"{what}: status {code} ({status_string(code)})")


def _dtype_code(dtype: torch.dtype) -> int:
    if dtype == torch.float64:
        return SRTM_F64
    if dtype == torch.float32:
        return SRTM_F32
    raise SrtmError(f"unsupported dtype {dtype}; use torch.float32 or torch.float64")


def shape_of(nx: int, ny: int, L: int, N: int, dtype: torch.dtype) -> Shape:
    return Shape(nx, ny, L, _dtype_code(dtype), N)


def workspace_size(nx: int, ny: int, L: int, N: int, dtype: torch.dtype, smoother: bool,
                   inputs: bool = False, tv: bool = False) -> int:
    """Workspace bytes of srtm_filter (smoother False) or srtm_smooth, or of their *_inputs or
    per-window (*_tv) forms."""
    out = ctypes.c_size_t(0)
    sh = shape_of(nx, ny, L, N, dtype)
    fn = (lib().srtm_workspace_size_tv if tv else
          lib().srtm_workspace_size_inputs if inputs else lib().srtm_workspace_size)
    _check(fn(ctypes.byref(sh), int(smoother), ctypes.byref(out)), "srtm_workspace_size")
    return int(out.value)


def kernel_names(smoother: bool):
    L = lib()
    return [L.srtm_kernel_name(int(smoother), j).decode() for j in range(L.srtm_kernel_count(int(smoother)))]


def _prep(F, Q, H, R, L, m0, P0, y):
    ts = dict(F=F, Q=Q, H=H, R=R, m0=m0, P0=P0, y=y)
    dev, dt = y.device, y.dtype
    for k, t in ts.items():
        if not isinstance(t, torch.Tensor):
            raise SrtmError(f"{k} must be a torch tensor")
        if t.device.type != "cuda":
            raise SrtmError(f"{k} must be on a GPU (got {t.device}); there is no CPU path")
        if t.device != dev or t.dtype != dt:
            raise SrtmError(f"{k} must share device {dev} and dtype {dt}")
    tv = F.dim() == 3  # per-window (time-varying) model: F, Q, H, R are [N, ...]
    nx, ny = F.shape[-1], H.shape[-2]
    N = y.shape[0]
    w = (N,) if tv else ()
    exp = dict(F=w + (nx, nx), Q=w + (nx, nx), H=w + (ny, nx), R=w + (ny, ny), m0=(nx,), P0=(nx, nx), y=(N, ny))
    for k, s in exp.items():
        if tuple(ts[k].shape) != s:
            raise SrtmError(f"{k} has shape {tuple(ts[k].shape)}, expected {s}")
    ts = {k: v.contiguous() for k, v in ts.items()}
    return ts, nx, ny, N


def _prep_inputs(B, u, nx: int, L: int, N: int, y: torch.Tensor):
    """Validated (contiguous B, contiguous u, srtm_inputs) for known inputs, or None without."""
    if B is None and u is None:
        return None
    if B is None or u is None:
        raise SrtmError("known inputs need both B [nx, nu] and u [N, L, nu]")
    for k, t in (("B", B), ("u", u)):
        if not isinstance(t, torch.Tensor) or t.device != y.device or t.dtype != y.dtype:
            raise SrtmError(f"{k} must be a tensor on {y.device} of dtype {y.dtype}")
    nu = B.shape[1] if B.dim() == 2 else -1
    if tuple(B.shape) != (nx, nu) or tuple(u.shape) != (N, L, nu) or not 1 <= nu <= MAX_NU:
        raise SrtmError(f"inputs: B {tuple(B.shape)} and u {tuple(u.shape)} must be [{nx}, nu] and "
                        f"[{N}, {L}, nu] with 1 <= nu <= {MAX_NU}")
    B, u = B.contiguous(), u.contiguous()
    return B, u, InputsC(B.data_ptr(), u.data_ptr(), nu, 0)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _raise_info(info: torch.Tensor, what: str):
    v = int(info.item())
    if v:
        msgs = [m for b, m in INFO_BITS.items() if v & b]
        raise SrtmError(f"{what}: numerical failure, info={v} ({'; '.join(msgs)})")


def filter(F, Q, H, R, L: int, m0, P0, y, *, fast: bool = True, slow: bool = True,
           workspace: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None,
           check: bool = True, B=None, u=None) -> Dict[str, torch.Tensor]:
    """p(x_{k,i} | y_{1:k}) as m_fast [N,L,nx], P_fast [N,L,nx,nx]; p(x_{k,L} | y_{1:k}) as m_slow, P_slow.

    B [nx, nu] and u [N, L, nu] add known inputs (u[k-1, i-1] drives x_{k,i}). F, Q, H, R given
    per window ([N, ...]) select the time-varying form (srtm_filter_tv)."""
    ts, nx, ny, N = _prep(F, Q, H, R, L, m0, P0, y)
    inp = _prep_inputs(B, u, nx, L, N, y)
    tv = F.dim() == 3
    if tv and inp is not None:
        raise SrtmError("a per-window model takes no inputs")
    dev, dt = y.device, y.dtype
    out = {}
    if fast:
        out["m_fast"] = torch.empty((N, L, nx), device=dev, dtype=dt)
        out["P_fast"] = torch.empty((N, L, nx, nx), device=dev, dtype=dt)
    if slow:
        out["m_slow"] = torch.empty((N, nx), device=dev, dtype=dt)
        out["P_slow"] = torch.empty((N, nx, nx), device=dev, dtype=dt)
    nbytes = workspace_size(nx, ny, L, N, dt, False, inp is not None, tv)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, device=dev, dtype=torch.uint8)
    if info is None:
        info = torch.zeros(1, device=dev, dtype=torch.int32)
    sh = shape_of(nx, ny, L, N, dt)
    stream = torch.cuda.current_stream(dev).cuda_stream
    args = ([_ptr(ts[k]) for k in ("F", "Q", "H", "R", "m0", "P0", "y")] +
            [_ptr(out.get(k)) for k in ("m_fast", "P_fast", "m_slow", "P_slow")] +
            [_ptr(workspace), workspace.numel(), _ptr(info), ctypes.c_void_p(stream)])
    if tv:
        _check(lib().srtm_filter_tv(ctypes.byref(sh), *args), "srtm_filter_tv")
    elif inp is None:
        _check(lib().srtm_filter(ctypes.byref(sh), *args), "srtm_filter")
    else:
        _check(lib().srtm_filter_inputs(ctypes.byref(sh), ctypes.byref(inp[2]), *args), "srtm_filter_inputs")
    if check:
        _raise_info(info, "srtm_filter")
    out["info"] = info
    return out


def _smooth_args(ts, out, workspace, info):
    return ([_ptr(ts[k]) for k in ("F", "Q", "H", "R", "m0", "P0", "y")] +
            [_ptr(out.get(k)) for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow",
                                        "mf_fast", "Pf_fast", "mf_slow", "Pf_slow")] +
            [_ptr(workspace), workspace.numel(), _ptr(info)])


def smooth(F, Q, H, R, L: int, m0, P0, y, *, fast: bool = True, slow: bool = True, with_filter: bool = False,
           workspace: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None,
           out: Optional[Dict[str, torch.Tensor]] = None, check: bool = True,
           events=None, B=None, u=None, lag1: bool = False) -> Dict[str, torch.Tensor]:
    """p(x_{k,i} | y_{1:N}) as ms_fast [N,L,nx], Ps_fast [N,L,nx,nx]; p(x_{k,1} | y_{1:N}) as ms_slow, Ps_slow.

    with_filter also returns the filter outputs (mf_fast, Pf_fast, mf_slow, Pf_slow). `out` may
    supply preallocated output tensors; `events` (a ctypes array of hipEvent_t) selects the
    profiling entry point. B [nx, nu] and u [N, L, nu] add known inputs (u[k-1, i-1] drives x_{k,i}).
    lag1 also returns Cs_fast [N,L,nx,nx] = Cov(x_{k,i}, x_{k,i-1} | y_{1:N}) (x_{k,0} = x_{k-1,L},
    x_{1,0} = x_0) through srtm_smooth_lag1 (time-invariant model, no inputs or filter outputs).
    """
    ts, nx, ny, N = _prep(F, Q, H, R, L, m0, P0, y)
    inp = _prep_inputs(B, u, nx, L, N, y)
    tv = F.dim() == 3
    if (inp is not None or tv) and events is not None:
        raise SrtmError("the profiling entry point takes neither inputs nor a per-window model")
    if tv and inp is not None:
        raise SrtmError("a per-window model takes no inputs")
    if lag1 and (tv or inp is not None or events is not None or with_filter):
        raise SrtmError("lag-one cross-covariances: time-invariant model, no inputs, filter outputs or events")
    dev, dt = y.device, y.dtype
    if out is None:
        out = {}
        if fast:
            out["ms_fast"] = torch.empty((N, L, nx), device=dev, dtype=dt)
            out["Ps_fast"] = torch.empty((N, L, nx, nx), device=dev, dtype=dt)
        if slow:
            out["ms_slow"] = torch.empty((N, nx), device=dev, dtype=dt)
            out["Ps_slow"] = torch.empty((N, nx, nx), device=dev, dtype=dt)
        if with_filter:
            out["mf_fast"] = torch.empty((N, L, nx), device=dev, dtype=dt)
            out["Pf_fast"] = torch.empty((N, L, nx, nx), device=dev, dtype=dt)
            out["mf_slow"] = torch.empty((N, nx), device=dev, dtype=dt)
            out["Pf_slow"] = torch.empty((N, nx, nx), device=dev, dtype=dt)
        if lag1:
            out["Cs_fast"] = torch.empty((N, L, nx, nx), device=dev, dtype=dt)
    nbytes = workspace_size(nx, ny, L, N, dt, True, inp is not None, tv)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, device=dev, dtype=torch.uint8)
    if info is None:
        info = torch.zeros(1, device=dev, dtype=torch.int32)
    sh = shape_of(nx, ny, L, N, dt)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    args = _smooth_args(ts, out, workspace, info)
    if lag1:
        lag_args = ([_ptr(ts[k]) for k in ("F", "Q", "H", "R", "m0", "P0", "y")] +
                    [_ptr(out.get(k)) for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow", "Cs_fast")] +
                    [_ptr(workspace), workspace.numel(), _ptr(info)])
        _check(lib().srtm_smooth_lag1(ctypes.byref(sh), *lag_args, stream), "srtm_smooth_lag1")
    elif tv:
        _check(lib().srtm_smooth_tv(ctypes.byref(sh), *args, stream), "srtm_smooth_tv")
    elif inp is not None:
        code = lib().srtm_smooth_inputs(ctypes.byref(sh), ctypes.byref(inp[2]), *args, stream)
        _check(code, "srtm_smooth_inputs")
    elif events is None:
        code = lib().srtm_smooth(ctypes.byref(sh), *args, stream)
        _check(code, "srtm_smooth")
    else:
        code = lib().srtm_smooth_profiled(ctypes.byref(sh), *args, stream, events, len(events))
        _check(code, "srtm_smooth_profiled")
    if check:
        _raise_info(info, "srtm_smooth")
    out["info"] = info
    return out


def smooth_sequential(F, Q, H, R, L: int, m0, P0, y, *, out: Optional[Dict[str, torch.Tensor]] = None,
                      workspace: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None,
                      check: bool = True) -> Dict[str, torch.Tensor]:
    """srtm_smooth_sequential: the same smoothed outputs as `smooth` by the sequential IMKF and
    smoother on one GPU lane (the paper's sequential comparison method; no scan)."""
    ts, nx, ny, N = _prep(F, Q, H, R, L, m0, P0, y)
    dev, dt = y.device, y.dtype
    if out is None:
        out = {"ms_fast": torch.empty((N, L, nx), device=dev, dtype=dt),
               "Ps_fast": torch.empty((N, L, nx, nx), device=dev, dtype=dt),
               "ms_slow": torch.empty((N, nx), device=dev, dtype=dt),
               "Ps_slow": torch.empty((N, nx, nx), device=dev, dtype=dt)}
    nbytes = workspace_size(nx, ny, L, N, dt, True)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, device=dev, dtype=torch.uint8)
    if info is None:
        info = torch.zeros(1, device=dev, dtype=torch.int32)
    sh = shape_of(nx, ny, L, N, dt)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    args = ([_ptr(ts[k]) for k in ("F", "Q", "H", "R", "m0", "P0", "y")] +
            [_ptr(out.get(k)) for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow")] +
            [_ptr(workspace), workspace.numel(), _ptr(info), stream])
    _check(lib().srtm_smooth_sequential(ctypes.byref(sh), *args), "srtm_smooth_sequential")
    if check:
        _raise_info(info, "srtm_smooth_sequential")
    out["info"] = info
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def smooth_noalloc(F, Q, H, R, L: int, m0, P0, y, out: Dict[str, torch.Tensor], info: torch.Tensor) -> int:
    """srtm_smooth_noalloc: the smoother with the library's fixed per-GPU scratch as workspace.

    `out` holds the caller's preallocated outputs (keys of `smooth`, each optional) and `info`
    a zeroed device int32. Nothing is allocated here or in the library. Returns the status
    code (0 = ok; SRTM_E_SCRATCH = 8 when the problem needs more than NOALLOC_SCRATCH_BYTES)
    without raising, so callers can test the limit."""
    ts, nx, ny, N = _prep(F, Q, H, R, L, m0, P0, y)
    sh = shape_of(nx, ny, L, N, y.dtype)
    stream = ctypes.c_void_p(torch.cuda.current_stream(y.device).cuda_stream)
    args = ([_ptr(ts[k]) for k in ("F", "Q", "H", "R", "m0", "P0", "y")] +
            [_ptr(out.get(k)) for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow",
                                        "mf_fast", "Pf_fast", "mf_slow", "Pf_slow")] +
            [_ptr(info), stream])
    return int(lib().srtm_smooth_noalloc(ctypes.byref(sh), *args))


def _lik(F, Q, H, R, L, m0, P0, y, grad: bool, check: bool, B=None, u=None):
    ts, nx, ny, N = _prep(F, Q, H, R, L, m0, P0, y)
    inp = _prep_inputs(B, u, nx, L, N, y)
    if F.dim() == 3:
        raise SrtmError("the log-likelihood entry points take a time-invariant model")
    dev, dt = y.device, y.dtype
    ll = torch.empty(1, device=dev, dtype=dt)
    dF = torch.empty((nx, nx), device=dev, dtype=dt) if grad else None
    dQ = torch.empty((nx, nx), device=dev, dtype=dt) if grad else None
    dR = torch.empty((ny, ny), device=dev, dtype=dt) if grad else None
    ws = torch.empty(workspace_size(nx, ny, L, N, dt, grad, inp is not None), device=dev, dtype=torch.uint8)
    info = torch.zeros(1, device=dev, dtype=torch.int32)
    sh = shape_of(nx, ny, L, N, dt)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    ins = [_ptr(ts[k]) for k in ("F", "Q", "H", "R", "m0", "P0", "y")]
    if grad and inp is not None:
        code = lib().srtm_loglik_grad_inputs(ctypes.byref(sh), ctypes.byref(inp[2]), *ins, _ptr(ll), _ptr(dF),
                                             _ptr(dQ), _ptr(dR), _ptr(ws), ws.numel(), _ptr(info), stream)
        _check(code, "srtm_loglik_grad_inputs")
    elif grad:
        code = lib().srtm_loglik_grad(ctypes.byref(sh), *ins, _ptr(ll), _ptr(dF), _ptr(dQ), _ptr(dR), _ptr(ws),
                                      ws.numel(), _ptr(info), stream)
        _check(code, "srtm_loglik_grad")
    elif inp is not None:
        code = lib().srtm_loglik_inputs(ctypes.byref(sh), ctypes.byref(inp[2]), *ins, _ptr(ll), _ptr(ws), ws.numel(),
                                        _ptr(info), stream)
        _check(code, "srtm_loglik_inputs")
    else:
        code = lib().srtm_loglik(ctypes.byref(sh), *ins, _ptr(ll), _ptr(ws), ws.numel(), _ptr(info), stream)
        _check(code, "srtm_loglik")
    if check:
        _raise_info(info, "srtm_loglik_grad" if grad else "srtm_loglik")
    return ll[0], dF, dQ, dR


def loglik(F, Q, H, R, L: int, m0, P0, y, *, check: bool = True, B=None, u=None) -> torch.Tensor:
    """log p(y_{1:N}) (a 0-d tensor on the device); B, u: optional known inputs as in filter()."""
    return _lik(F, Q, H, R, L, m0, P0, y, False, check, B, u)[0]


def loglik_grad(F, Q, H, R, L: int, m0, P0, y, *, check: bool = True, B=None, u=None):
    """(log p(y_{1:N}), d/dF, d/dQ, d/dR); the Q and R gradients are symmetric-matrix gradients.
    B, u: optional known inputs as in filter() (the gradient stays with respect to F, Q, R)."""
    return _lik(F, Q, H, R, L, m0, P0, y, True, check, B, u)


class LogLikelihood(torch.autograd.Function):
    """log p(y_{1:N}) as a differentiable function of F, Q and R (known inputs B, u, if given, are
    constants). The forward pass runs the filter scan only; the backward pass runs both scans
    again (nothing from the forward pass is stored) and returns the gradient from the library."""

    @staticmethod
    def forward(ctx, F, Q, R, H, m0, P0, y, L, B=None, u=None):
        ctx.save_for_backward(F, Q, R, H, m0, P0, y)
        ctx.L = int(L)
        ctx.inputs = None if B is None else (B.detach(), u.detach())
        inp = {} if B is None else dict(B=B.detach(), u=u.detach())
        return loglik(F.detach(), Q.detach(), H.detach(), R.detach(), int(L), m0.detach(), P0.detach(), y.detach(),
                      **inp)

    @staticmethod
    def backward(ctx, g):
        F, Q, R, H, m0, P0, y = ctx.saved_tensors
        inp = {} if ctx.inputs is None else dict(B=ctx.inputs[0], u=ctx.inputs[1])
        _, dF, dQ, dR = loglik_grad(F.detach(), Q.detach(), H.detach(), R.detach(), ctx.L, m0.detach(),
                                    P0.detach(), y.detach(), **inp)
        return g * dF, g * dQ, g * dR, None, None, None, None, None, None, None


def log_likelihood(F, Q, R, H, L: int, m0, P0, y, B=None, u=None) -> torch.Tensor:
    """Differentiable log p(y_{1:N}) with respect to F, Q and R (see LogLikelihood); B [nx, nu]
    and u [N, L, nu] are optional known inputs."""
    return LogLikelihood.apply(F, Q, R, H, m0, P0, y, L, B, u)


class Batch:
    """A planned batch: the host and device copies of the plan's table, the workspace, the
    per-sequence status words and output tensors. Reusable for repeated calls (and graph
    capture) on the same inputs."""

    def __init__(self, problems, *, fast: bool = True, slow: bool = True, outputs=None, alloc=None,
                 grad: bool = False):
        items = []
        for pr in problems:
            F, Q, H, R, L, m0, P0, y = pr
            ts, nx, ny, N = _prep(F, Q, H, R, L, m0, P0, y)
            items.append((ts, int(L), N, nx, ny))
        if not items:
            raise SrtmError("empty batch")
        nx, ny = items[0][3], items[0][4]
        dev, dt = items[0][0]["y"].device, items[0][0]["y"].dtype
        for ts, L, N, a, b in items:
            if (a, b) != (nx, ny) or ts["y"].device != dev or ts["y"].dtype != dt:
                raise SrtmError("all sequences of a batch share nx, ny, device and dtype")
        self.nx, self.ny, self.dtype, self.device = nx, ny, dt, dev
        self.inputs = [it[0] for it in items]
        self.outputs = []
        arr = (SeqC * len(items))()
        self.grad = grad
        if grad:   # per sequence: ll, dF, dQ, dR in the four output slots
            outputs = [{"ll": torch.empty(1, device=dev, dtype=dt), "dF": torch.empty((nx, nx), device=dev, dtype=dt),
                        "dQ": torch.empty((nx, nx), device=dev, dtype=dt),
                        "dR": torch.empty((ny, ny), device=dev, dtype=dt)} for _ in items]
        for j, (ts, L, N, _, _) in enumerate(items):
            out = {} if outputs is None else outputs[j]
            if outputs is not None and not grad:
                for k, shp in (("ms_fast", (N, L, nx)), ("Ps_fast", (N, L, nx, nx)), ("ms_slow", (N, nx)),
                               ("Ps_slow", (N, nx, nx))):
                    t = out.get(k)
                    if t is not None and (tuple(t.shape) != shp or t.dtype != dt or t.device != dev or
                                          not t.is_contiguous()):
                        raise SrtmError(f"sequence {j}: output {k} must be a contiguous {shp} tensor")
            elif fast:
                out["ms_fast"] = torch.empty((N, L, nx), device=dev, dtype=dt)
                out["Ps_fast"] = torch.empty((N, L, nx, nx), device=dev, dtype=dt)
            if outputs is None and slow:
                out["ms_slow"] = torch.empty((N, nx), device=dev, dtype=dt)
                out["Ps_slow"] = torch.empty((N, nx, nx), device=dev, dtype=dt)
            self.outputs.append(out)
            e = arr[j]
            for k in ("F", "Q", "H", "R", "m0", "P0", "y"):
                setattr(e, k, ts[k].data_ptr())
            slots = dict(zip(("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"), ("ll", "dF", "dQ", "dR"))) if grad else {}
            for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
                src = slots.get(k, k)
                setattr(e, k, out[src].data_ptr() if src in out else None)
            e.N, e.L, e.reserved = N, L, 0
        self.nseq = len(items)
        tsz, wsz = ctypes.c_size_t(0), ctypes.c_size_t(0)
        ntiles, max_L = ctypes.c_int64(0), ctypes.c_int32(0)
        code = _dtype_code(dt)
        _check(lib().srtm_batch_plan(nx, ny, code, arr, self.nseq, None, 0, ctypes.byref(tsz), ctypes.byref(wsz),
                                     ctypes.byref(ntiles), ctypes.byref(max_L)), "srtm_batch_plan")
        self.table_host = torch.empty(tsz.value, dtype=torch.uint8, pin_memory=True)
        _check(lib().srtm_batch_plan(nx, ny, code, arr, self.nseq, _ptr(self.table_host), tsz.value,
                                     ctypes.byref(tsz), ctypes.byref(wsz), ctypes.byref(ntiles),
                                     ctypes.byref(max_L)), "srtm_batch_plan")
        # device buffers: from `alloc(nbytes) -> uint8 device tensor` when given (an arena), else torch
        get = alloc if alloc is not None else (lambda n: torch.empty(n, device=dev, dtype=torch.uint8))
        self.table_dev = get(tsz.value)
        self.table_dev.copy_(self.table_host, non_blocking=True)
        self.workspace = get(max(wsz.value, 256))
        self.info = get(4 * self.nseq).view(torch.int32)
        self.info.zero_()
        self.ntiles, self.max_L = int(ntiles.value), int(max_L.value)

    def launch(self, stream=None):
        """Enqueue the batch on `stream` (default: the current stream); no allocation, no sync."""
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        fn = lib().srtm_loglik_grad_batch if self.grad else lib().srtm_smooth_batch
        _check(fn(self.nx, self.ny, _dtype_code(self.dtype), self.nseq, _ptr(self.table_host), _ptr(self.table_dev),
                  _ptr(self.workspace), self.workspace.numel(), _ptr(self.info), ctypes.c_void_p(stream)),
               "srtm_loglik_grad_batch" if self.grad else "srtm_smooth_batch")

    def check(self):
        v = self.info.cpu()
        bad = [(j, int(x)) for j, x in enumerate(v.tolist()) if x]
        if bad:
            raise SrtmError(f"srtm_smooth_batch: numerical failure in sequences {bad[:8]}")


class BatchEx:
    """A planned mixed batch (srtm_batch_plan_ex / srtm_smooth_batch_ex): sequences of any
    supported (nx, ny), each with a time-invariant model, with known inputs (problem tuples
    (F, Q, H, R, L, m0, P0, y, B, u)) or with a per-window model (F, Q, H, R of shape [N, ...]),
    smoothed by one set of six launches. Same members as Batch."""

    LAUNCHES = 6

    def __init__(self, problems, *, fast: bool = True, slow: bool = True, outputs=None, alloc=None):
        problems = list(problems)
        if not problems:
            raise SrtmError("empty batch")
        arr = (SeqExC * len(problems))()
        self.inputs, self.outputs = [], []
        dev, dt = problems[0][7].device, problems[0][7].dtype
        for j, pr in enumerate(problems):
            if len(pr) not in (8, 10):
                raise SrtmError(f"sequence {j}: expected (F, Q, H, R, L, m0, P0, y[, B, u])")
            F, Q, H, R, L, m0, P0, y = pr[:8]
            ts, nx, ny, N = _prep(F, Q, H, R, L, m0, P0, y)
            if ts["y"].device != dev or ts["y"].dtype != dt:
                raise SrtmError("all sequences of a batch share device and dtype")
            tv = F.dim() == 3
            inp = _prep_inputs(pr[8], pr[9], nx, int(L), N, ts["y"]) if len(pr) == 10 else None
            if tv and inp is not None:
                raise SrtmError(f"sequence {j}: a per-window model takes no inputs")
            if inp is not None:
                ts["B"], ts["u"] = inp[0], inp[1]
            self.inputs.append(ts)
            out = {} if outputs is None else outputs[j]
            if outputs is None:
                if fast:
                    out["ms_fast"] = torch.empty((N, L, nx), device=dev, dtype=dt)
                    out["Ps_fast"] = torch.empty((N, L, nx, nx), device=dev, dtype=dt)
                if slow:
                    out["ms_slow"] = torch.empty((N, nx), device=dev, dtype=dt)
                    out["Ps_slow"] = torch.empty((N, nx, nx), device=dev, dtype=dt)
            else:
                for k, shp in (("ms_fast", (N, L, nx)), ("Ps_fast", (N, L, nx, nx)), ("ms_slow", (N, nx)),
                               ("Ps_slow", (N, nx, nx))):
                    t = out.get(k)
                    if t is not None and (tuple(t.shape) != shp or t.dtype != dt or t.device != dev or
                                          not t.is_contiguous()):
                        raise SrtmError(f"sequence {j}: output {k} must be a contiguous {shp} tensor")
            self.outputs.append(out)
            e = arr[j]
            e.nx, e.ny, e.L, e.per_window, e.N = nx, ny, int(L), int(tv), N
            for k in ("F", "Q", "H", "R", "m0", "P0", "y", "B", "u"):
                setattr(e, k, ts[k].data_ptr() if k in ts else None)
            e.nu, e.reserved = (inp[2].nu if inp is not None else 0), 0
            for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
                setattr(e, k, out[k].data_ptr() if k in out else None)
        self.nseq, self.dtype, self.device = len(problems), dt, dev
        tsz, wsz = ctypes.c_size_t(0), ctypes.c_size_t(0)
        ntiles, max_L = ctypes.c_int64(0), ctypes.c_int32(0)
        code = _dtype_code(dt)
        refs = (ctypes.byref(tsz), ctypes.byref(wsz), ctypes.byref(ntiles), ctypes.byref(max_L))
        _check(lib().srtm_batch_plan_ex(code, arr, self.nseq, None, 0, *refs), "srtm_batch_plan_ex")
        self.table_host = torch.empty(tsz.value, dtype=torch.uint8, pin_memory=True)
        _check(lib().srtm_batch_plan_ex(code, arr, self.nseq, _ptr(self.table_host), tsz.value, *refs),
               "srtm_batch_plan_ex")
        get = alloc if alloc is not None else (lambda n: torch.empty(n, device=dev, dtype=torch.uint8))
        self.table_dev = get(tsz.value)
        self.table_dev.copy_(self.table_host, non_blocking=True)
        self.workspace = get(max(wsz.value, 256))
        self.info = get(4 * self.nseq).view(torch.int32)
        self.info.zero_()
        self.ntiles, self.max_L = int(ntiles.value), int(max_L.value)

    def launch(self, stream=None):
        """Enqueue the six launches on `stream` (default: the current stream); no allocation, no sync."""
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().srtm_smooth_batch_ex(_dtype_code(self.dtype), self.nseq, _ptr(self.table_host),
                                          _ptr(self.table_dev), _ptr(self.workspace), self.workspace.numel(),
                                          _ptr(self.info), ctypes.c_void_p(stream)), "srtm_smooth_batch_ex")

    def check(self):
        v = self.info.cpu()
        bad = [(j, int(x)) for j, x in enumerate(v.tolist()) if x]
        if bad:
            raise SrtmError(f"srtm_smooth_batch_ex: numerical failure in sequences {bad[:8]}")


class Graph:
    """A HIP graph recorded from calls enqueued on one capture stream (and streams joined to it by
    events) through srtm_graph_begin / srtm_graph_end; `replay` enqueues it on a stream."""

    def __init__(self, device):
        self.device = device
        self.stream = torch.cuda.Stream(device)
        self.exec = None

    def record(self, enqueue):
        """Runs enqueue() with the capture stream current, capturing what it enqueues."""
        torch.cuda.synchronize(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(lib().srtm_graph_begin(ctypes.c_void_p(self.stream.cuda_stream)), "srtm_graph_begin")
            try:
                enqueue()
            except BaseException:
                # end the capture so that the stream is usable again, and drop what it recorded
                if lib().srtm_graph_end(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)) == 0 and h.value:
                    lib().srtm_graph_destroy(h)
                raise
            code = lib().srtm_graph_end(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(code, "srtm_graph_end")
        if self.exec is not None:
            lib().srtm_graph_destroy(self.exec)
        self.exec = h
        torch.cuda.synchronize(self.device)

    def replay(self, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().srtm_graph_launch(self.exec, ctypes.c_void_p(stream)), "srtm_graph_launch")

    def __del__(self):
        if getattr(self, "exec", None) is not None and _lib is not None:
            _lib.srtm_graph_destroy(self.exec)
            self.exec = None


def smooth_batch(problems, *, fast: bool = True, slow: bool = True, check: bool = True):
    """Smooths many independent sequences (tuples (F, Q, H, R, L, m0, P0, y) of device tensors
    sharing nx, ny and dtype) with one set of launches; returns one output dict per sequence."""
    b = Batch(problems, fast=fast, slow=slow)
    b.info.zero_()
    b.launch()
    if check:
        b.check()
    return [dict(o, info=b.info[j:j + 1]) for j, o in enumerate(b.outputs)]


def model_tensors(model, device="cuda", dtype=torch.float64):
    """(F, Q, H, R, m0, P0) of a workloads.Model as device tensors."""
    conv = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device=device, dtype=dtype).contiguous()  # noqa: E731
    return conv(model.A), conv(model.Q), conv(model.C), conv(model.R), conv(model.m0), conv(model.P0)
