"""C-ABI library checks that need no GPU: symbols, sizing and argument validation.

Every call here fails validation on the host, so nothing is ever enqueued (the
pointers passed are not valid device memory and must never reach a kernel).
"""
import ctypes
import os
import re

import pytest

from paper_2410_00627_amd import srtm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srtm.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(srtm.LIB_PATH):
        pytest.skip("libsrtm.so not built")
    return srtm.lib()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srtm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert "srtm_filter" in names and "srtm_smooth" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/srtm.h but not exported"


def test_version_and_kernel_names(L):
    assert L.srtm_version() >= 100
    assert srtm.kernel_names(False)[0] == "k_constants"
    assert len(srtm.kernel_names(True)) == L.srtm_kernel_count(1)
    assert L.srtm_kernel_name(1, 99) is None
    for c in range(8):
        assert isinstance(srtm.status_string(c), str)


def _ws(nx, ny, Lw, N, dtype=1, smoother=1):
    sh = srtm.Shape(nx, ny, Lw, dtype, N)
    out = ctypes.c_size_t(0)
    code = srtm.lib().srtm_workspace_size(ctypes.byref(sh), smoother, ctypes.byref(out))
    return code, out.value


def test_workspace_size_valid(L):
    code, b = _ws(4, 2, 20, 1 << 17)
    assert code == 0
    # the slow-filter carry alone is N (nx + nx^2) float64 scalars
    assert b >= (1 << 17) * 20 * 8
    c32, b32 = _ws(4, 2, 20, 1 << 17, dtype=0)
    assert c32 == 0 and b32 < b
    cf, bf = _ws(4, 2, 20, 1 << 17, smoother=0)
    assert cf == 0 and bf < b


@pytest.mark.parametrize("nx,ny,Lw,N,dtype,code", [
    (0, 1, 10, 5, 1, 2), (2, 0, 10, 5, 1, 2), (2, 1, 0, 5, 1, 2), (2, 1, 10, 0, 1, 2),
    (2, 1, 10, 5, 7, 3), (5, 3, 10, 5, 1, 4), (2, 1, 100000, 5, 1, 4), (2, 1, 10, 1 << 40, 1, 4),
])
def test_workspace_size_errors(L, nx, ny, Lw, N, dtype, code):
    assert _ws(nx, ny, Lw, N, dtype)[0] == code


def test_supported_pairs(L):
    for nx, ny in [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (4, 2)]:
        assert L.srtm_supported(nx, ny) == 1
    assert L.srtm_supported(9, 9) == 0


def _call(fn, sh, ptrs, ws_bytes, n_out):
    P = [ctypes.c_void_p(p) if p else None for p in ptrs]
    args = [ctypes.byref(sh)] + P[:7] + [None] * n_out + [P[7], ws_bytes, None, None]
    return fn(*args)


FAKE = [0x1000 * (i + 1) for i in range(8)]   # 16-byte aligned, never dereferenced


def test_filter_rejects_null_inputs(L):
    sh = srtm.Shape(2, 1, 10, 1, 5)
    for i in range(8):
        ptrs = list(FAKE)
        ptrs[i] = 0
        assert _call(L.srtm_filter, sh, ptrs, 1 << 30, 4) == 1


def test_smooth_rejects_small_workspace(L):
    sh = srtm.Shape(2, 1, 10, 1, 5)
    assert _call(L.srtm_smooth, sh, FAKE, 16, 8) == 6


def test_rejects_misaligned(L):
    sh = srtm.Shape(2, 1, 10, 1, 5)
    ptrs = list(FAKE)
    ptrs[6] = 0x1008          # y misaligned
    assert _call(L.srtm_smooth, sh, ptrs, 1 << 30, 8) == 5
    ptrs = list(FAKE)
    ptrs[7] = 0x1010          # workspace not 256-aligned
    assert _call(L.srtm_filter, sh, ptrs, 1 << 30, 4) == 5


def test_rejects_bad_shape_and_dtype(L):
    assert _call(L.srtm_smooth, srtm.Shape(2, 1, 10, 9, 5), FAKE, 1 << 30, 8) == 3
    assert _call(L.srtm_smooth, srtm.Shape(2, 1, 10, 1, 0), FAKE, 1 << 30, 8) == 2
    assert _call(L.srtm_smooth, srtm.Shape(7, 1, 10, 1, 5), FAKE, 1 << 30, 8) == 4
    assert L.srtm_smooth(None, *([None] * 16), 0, None, None) == 1


def test_profiled_requires_events(L):
    sh = srtm.Shape(2, 1, 10, 1, 5)
    P = [ctypes.c_void_p(p) for p in FAKE]
    assert L.srtm_smooth_profiled(ctypes.byref(sh), *P[:7], *([None] * 8), P[7], 1 << 30, None, None,
                                  None, 0) == 1


def test_python_binding_refuses_cpu_tensors():
    import torch
    from paper_2410_00627_amd import workloads as wl
    m = wl.wna_model()
    t = [torch.as_tensor(a) for a in (m.A, m.Q, m.C, m.R, m.m0, m.P0)]
    y = torch.zeros(5, 1, dtype=torch.float64)
    with pytest.raises(srtm.SrtmError, match="GPU"):
        srtm.smooth(*t[:4], m.L, t[4], t[5], y)
