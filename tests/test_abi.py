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
    for c in range(9):
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


def test_window_length_limits(L):
    """L = 128, the build's maximum, is accepted for every pair (the constants kernel's float64
    tables then still fit in 160 KiB of LDS for nx = 6); L = 129 is not."""
    for nx, ny in [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (4, 2), (6, 1)]:
        assert _ws(nx, ny, 128, 1000)[0] == 0
        assert _ws(nx, ny, 129, 1000)[0] == 4


def test_supported_pairs(L):
    for nx, ny in [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (4, 2), (6, 1)]:
        assert L.srtm_supported(nx, ny) == 1
    assert L.srtm_supported(9, 9) == 0 and L.srtm_supported(5, 1) == 0


def _no_gpu():
    # These calls pass fake device addresses: they must fail validation on the host, and as a
    # second line of defence they never run where a GPU could execute a launch.
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-validation test with fake device pointers; skipped where a GPU is visible")


def _call(fn, sh, ptrs, ws_bytes, n_out):
    _no_gpu()
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


def _call_inputs(fn, sh, inp, ptrs, ws_bytes, n_out):
    _no_gpu()
    P = [ctypes.c_void_p(p) if p else None for p in ptrs]
    args = [ctypes.byref(sh), None if inp is None else ctypes.byref(inp)] + P[:7] + [None] * n_out
    return fn(*args, P[7], ws_bytes, None, None)


@pytest.mark.parametrize("name,n_out", [("srtm_filter_inputs", 4), ("srtm_smooth_inputs", 8)])
def test_inputs_entry_points_validate(L, name, n_out):
    fn = getattr(L, name)
    sh = srtm.Shape(2, 1, 10, 1, 5)
    ok = srtm.InputsC(0x9000, 0xA000, 2, 0)
    assert _call_inputs(fn, sh, None, FAKE, 1 << 30, n_out) == 1                                # no inputs struct
    assert _call_inputs(fn, sh, srtm.InputsC(0, 0xA000, 2, 0), FAKE, 1 << 30, n_out) == 1       # B missing
    assert _call_inputs(fn, sh, srtm.InputsC(0x9000, 0, 2, 0), FAKE, 1 << 30, n_out) == 1       # u missing
    assert _call_inputs(fn, sh, srtm.InputsC(0x9000, 0xA000, 0, 0), FAKE, 1 << 30, n_out) == 2  # nu = 0
    assert _call_inputs(fn, sh, srtm.InputsC(0x9000, 0xA000, 5, 0), FAKE, 1 << 30, n_out) == 2  # nu > max
    assert _call_inputs(fn, sh, srtm.InputsC(0x9000, 0xA000, 2, 1), FAKE, 1 << 30, n_out) == 2  # reserved
    assert _call_inputs(fn, sh, srtm.InputsC(0x9008, 0xA000, 2, 0), FAKE, 1 << 30, n_out) == 5  # misaligned B
    assert _call_inputs(fn, sh, ok, FAKE, 16, n_out) == 6                                        # workspace
    assert _call_inputs(fn, srtm.Shape(7, 1, 10, 1, 5), ok, FAKE, 1 << 30, n_out) == 4          # pair


def test_loglik_inputs_validates(L):
    _no_gpu()
    sh = srtm.Shape(2, 1, 10, 1, 5)
    P = [ctypes.c_void_p(p) for p in FAKE]
    ll = ctypes.c_void_p(0xB000)
    assert L.srtm_loglik_inputs(ctypes.byref(sh), None, *P[:7], ll, P[7], 1 << 30, None, None) == 1
    bad = srtm.InputsC(0x9000, 0xA000, 9, 0)
    assert L.srtm_loglik_inputs(ctypes.byref(sh), ctypes.byref(bad), *P[:7], ll, P[7], 1 << 30, None, None) == 2
    ok = srtm.InputsC(0x9000, 0xA000, 1, 0)
    assert L.srtm_loglik_inputs(ctypes.byref(sh), ctypes.byref(ok), *P[:7], ll, P[7], 16, None, None) == 6


def test_profiled_requires_events(L):
    sh = srtm.Shape(2, 1, 10, 1, 5)
    P = [ctypes.c_void_p(p) for p in FAKE]
    assert L.srtm_smooth_profiled(ctypes.byref(sh), *P[:7], *([None] * 8), P[7], 1 << 30, None, None,
                                  None, 0) == 1


def test_noalloc_validates_before_touching_the_device(L):
    """srtm_smooth_noalloc: shape and null checks, and the scratch limit, all on the host."""
    P = [ctypes.c_void_p(p) for p in FAKE]
    sh = srtm.Shape(4, 2, 20, 1, 5)
    assert L.srtm_smooth_noalloc(ctypes.byref(sh), None, *P[1:7], *([None] * 8), None, None) == 1
    assert L.srtm_smooth_noalloc(ctypes.byref(srtm.Shape(4, 2, 0, 1, 5)), *P[:7], *([None] * 8), None, None) == 2
    big = srtm.Shape(4, 2, 20, 1, 1 << 18)   # workspace above SRTM_NOALLOC_SCRATCH_BYTES
    code, need = _ws(4, 2, 20, 1 << 18)
    assert code == 0 and need > srtm.NOALLOC_SCRATCH_BYTES
    assert L.srtm_smooth_noalloc(ctypes.byref(big), *P[:7], *([None] * 8), None, None) == 8
    assert "SCRATCH" in srtm.status_string(8).upper()


def test_sequential_validates(L):
    P = [ctypes.c_void_p(p) for p in FAKE]
    sh = srtm.Shape(4, 2, 20, 1, 50)
    assert L.srtm_smooth_sequential(ctypes.byref(sh), *P[:7], *([None] * 4), None, 1 << 30, None, None) == 1
    assert L.srtm_smooth_sequential(ctypes.byref(sh), *P[:7], *([None] * 4), P[7], 16, None, None) == 6
    assert L.srtm_smooth_sequential(ctypes.byref(srtm.Shape(5, 2, 20, 1, 50)), *P[:7], *([None] * 4), P[7],
                                    1 << 30, None, None) == 4


def test_python_binding_refuses_cpu_tensors():
    import torch
    from paper_2410_00627_amd import workloads as wl
    m = wl.wna_model()
    t = [torch.as_tensor(a) for a in (m.A, m.Q, m.C, m.R, m.m0, m.P0)]
    y = torch.zeros(5, 1, dtype=torch.float64)
    with pytest.raises(srtm.SrtmError, match="GPU"):
        srtm.smooth(*t[:4], m.L, t[4], t[5], y)


# ----------------------------------------------------------------------------- batch plan (host only)
def _seqs(specs, base=0x100000):
    """srtm_seq entries with fake, 16-byte aligned addresses (never dereferenced on the host)."""
    arr = (srtm.SeqC * len(specs))()
    a = base
    for j, (N, Lw) in enumerate(specs):
        e = arr[j]
        for k in ("F", "Q", "H", "R", "m0", "P0", "y", "ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            setattr(e, k, a)
            a += 4096
        e.N, e.L, e.reserved = N, Lw, 0
    return arr


def _plan(arr, nx=4, ny=2, dtype=1, table=None, nbytes=0):
    t, w = ctypes.c_size_t(0), ctypes.c_size_t(0)
    nt, ml = ctypes.c_int64(0), ctypes.c_int32(0)
    code = srtm.lib().srtm_batch_plan(nx, ny, dtype, arr, len(arr), table, nbytes, ctypes.byref(t), ctypes.byref(w),
                                      ctypes.byref(nt), ctypes.byref(ml))
    return code, t.value, w.value, nt.value, ml.value


def test_batch_plan_sizes_and_tile_map(L):
    specs = [(1, 20), (300, 5), (256, 10), (257, 20), (5000, 3)]
    arr = _seqs(specs)
    code, tsz, wsz, nt, ml = _plan(arr)
    assert code == 0 and ml == 20
    assert nt == sum((N + 255) // 256 for N, _ in specs)
    # the workspace is the sum of the per-sequence smoother workspaces (256-byte aligned blocks)
    assert wsz == sum(((_ws(4, 2, Lw, N)[1] + 255) // 256) * 256 for N, Lw in specs)
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    tile_map = (ctypes.c_int32 * nt).from_buffer(buf, tsz - 4 * nt)
    expect = [j for j, (N, _) in enumerate(specs) for _ in range((N + 255) // 256)]
    assert list(tile_map) == expect
    # a table that is too small is not written, and the sizes are still returned
    small = (ctypes.c_uint8 * 8)()
    assert _plan(arr, table=ctypes.cast(small, ctypes.c_void_p), nbytes=8)[:2] == (0, tsz)
    assert bytes(small) == bytes(8)


@pytest.mark.parametrize("mutate,code", [
    (lambda a: setattr(a[1], "N", 0), 2),
    (lambda a: setattr(a[0], "L", 0), 2),
    (lambda a: setattr(a[2], "reserved", 1), 2),
    (lambda a: setattr(a[1], "y", None), 1),
    (lambda a: setattr(a[0], "Ps_fast", 0x100008), 5),
    (lambda a: setattr(a[2], "L", 1000), 4),
])
def test_batch_plan_errors(L, mutate, code):
    arr = _seqs([(10, 4), (20, 5), (30, 6)])
    mutate(arr)
    assert _plan(arr)[0] == code


def test_batch_plan_unsupported_pair(L):
    assert _plan(_seqs([(10, 4)]), nx=9, ny=9)[0] == 4


def test_smooth_batch_rejects_small_workspace_and_bad_table(L):
    _no_gpu()
    specs = [(300, 5), (600, 7)]
    arr = _seqs(specs)
    _, tsz, wsz, nt, _ = _plan(arr)
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    fake_dev = ctypes.c_void_p(0x4000000)
    fake_ws = ctypes.c_void_p(0x8000000)
    host = ctypes.cast(buf, ctypes.c_void_p)
    # workspace smaller than planned: rejected before anything is enqueued
    assert L.srtm_smooth_batch(4, 2, 1, 2, host, fake_dev, fake_ws, wsz - 256, None, None) == 6
    # a tile map that does not match the descriptors
    tile_map = (ctypes.c_int32 * nt).from_buffer(buf, tsz - 4 * nt)
    tile_map[0] = 1
    assert L.srtm_smooth_batch(4, 2, 1, 2, host, fake_dev, fake_ws, wsz, None, None) == 2
    assert L.srtm_smooth_batch(4, 2, 1, 2, None, fake_dev, fake_ws, wsz, None, None) == 1
    assert L.srtm_smooth_batch(4, 2, 1, 2, host, ctypes.c_void_p(0x4000008), fake_ws, wsz, None, None) == 5


def test_smooth_batch_rejects_descriptors_with_inputs(L):
    """The per-pair batch entry point takes no inputs (srtm_smooth_batch_ex does): a table whose
    descriptor names inputs is refused."""
    _no_gpu()
    arr = _seqs([(300, 5)])
    _, tsz, wsz, nt, _ = _plan(arr)
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    # descriptor layout: 15 pointers, N, tile0, ws_off (8 bytes each), L, smoother (4 each), then B
    off_B = 15 * 8 + 3 * 8 + 2 * 4
    assert bytes(buf[off_B:off_B + 8]) == bytes(8)
    ctypes.c_uint64.from_buffer(buf, off_B).value = 0x9000
    host = ctypes.cast(buf, ctypes.c_void_p)
    assert L.srtm_smooth_batch(4, 2, 1, 1, host, ctypes.c_void_p(0x4000000), ctypes.c_void_p(0x8000000), wsz,
                               None, None) == 2


def test_smooth_batch_rejects_descriptors_with_cross_covariances(L):
    """Batch descriptors carry no lag-one cross-covariance output (single calls only)."""
    _no_gpu()
    arr = _seqs([(300, 5)])
    _, tsz, wsz, nt, _ = _plan(arr)
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    # after B, u (8 bytes each) and nu, tv (4 each): the cross-covariance output pointer
    off_cs = 15 * 8 + 3 * 8 + 2 * 4 + 2 * 8 + 2 * 4
    assert bytes(buf[off_cs:off_cs + 8]) == bytes(8)
    ctypes.c_uint64.from_buffer(buf, off_cs).value = 0x9000
    host = ctypes.cast(buf, ctypes.c_void_p)
    assert L.srtm_smooth_batch(4, 2, 1, 1, host, ctypes.c_void_p(0x4000000), ctypes.c_void_p(0x8000000), wsz,
                               None, None) == 2


def test_workspace_size_with_inputs(L):
    """The *_inputs entry points need one more per-window record of nx + ny scalars."""
    for dtype, esz in ((1, 8), (0, 4)):
        for smoother in (0, 1):
            sh = srtm.Shape(4, 2, 20, dtype, 1000)
            a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
            assert L.srtm_workspace_size(ctypes.byref(sh), smoother, ctypes.byref(a)) == 0
            assert L.srtm_workspace_size_inputs(ctypes.byref(sh), smoother, ctypes.byref(b)) == 0
            assert b.value >= a.value + 1000 * 6 * esz
            assert b.value - a.value < 1000 * 6 * esz + 512


def test_inputs_call_rejects_plain_workspace_size(L):
    sh = srtm.Shape(2, 1, 10, 1, 5)
    plain = _ws(2, 1, 10, 5)[1]
    ok = srtm.InputsC(0x9000, 0xA000, 1, 0)
    assert _call_inputs(L.srtm_smooth_inputs, sh, ok, FAKE, plain, 8) == 6


def test_time_varying_entry_points_validate(L):
    """Per-window models: nx <= 4 only; a larger workspace than the plain one: per window the
    element (3 nx^2) and, for every other fast step, the two backward factors A^s, C Sig_s
    (nx^2 + ny nx)."""
    sh = srtm.Shape(4, 2, 20, 1, 1000)
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.srtm_workspace_size(ctypes.byref(sh), 1, ctypes.byref(a)) == 0
    assert L.srtm_workspace_size_tv(ctypes.byref(sh), 1, ctypes.byref(b)) == 0
    assert b.value > a.value + 1000 * (3 * 16 + 10 * (16 + 8)) * 8
    assert L.srtm_workspace_size_tv(ctypes.byref(srtm.Shape(6, 1, 20, 1, 1000)), 1, ctypes.byref(b)) == 4
    small = srtm.Shape(2, 1, 10, 1, 5)
    assert _call(L.srtm_smooth_tv, small, FAKE, _ws(2, 1, 10, 5)[1], 8) == 6   # plain size is too small
    assert _call(L.srtm_filter_tv, small, FAKE, 16, 4) == 6
    assert _call(L.srtm_smooth_tv, srtm.Shape(6, 1, 10, 1, 5), FAKE, 1 << 30, 8) == 4
    ptrs = list(FAKE)
    ptrs[0] = 0
    assert _call(L.srtm_smooth_tv, small, ptrs, 1 << 30, 8) == 1


def test_binding_declares_every_signature(L):
    """The Python binding gives every C entry point its argument and result types (a missing
    declaration would pass 64-bit sizes as C ints)."""
    for n in _declared_functions():
        fn = getattr(L, n)
        assert fn.argtypes is not None, f"{n}: argtypes not set"
        assert fn.restype is not None, f"{n}: restype not set"


def test_lag1_entry_point_validates(L):
    """srtm_smooth_lag1: the cross-covariance array is required and aligned; the other checks are
    srtm_smooth's (unsupported pair, small workspace). No kernel is launched on these paths."""
    _no_gpu()
    sh = srtm.Shape(2, 1, 10, 1, 5)
    _, need = _ws(2, 1, 10, 5)

    def call(shape, cs, ws_bytes, nulled=None):
        P = [ctypes.c_void_p(p) for p in FAKE]
        if nulled is not None:
            P[nulled] = None
        return L.srtm_smooth_lag1(ctypes.byref(shape), *P[:7], None, None, None, None,
                                  None if cs is None else ctypes.c_void_p(cs), P[7], ws_bytes, None, None)

    assert call(sh, None, need) == 1                      # Cs_fast is required
    assert call(sh, 0x9008, need) == 5                    # misaligned Cs_fast
    assert call(sh, 0x9000, need, nulled=0) == 1          # null model array
    assert call(sh, 0x9000, need - 256) == 6              # workspace too small
    assert call(srtm.Shape(5, 1, 10, 1, 5), 0x9000, need) == 4   # pair not compiled


# ----------------------------------------------------------------------------- mixed batches (host only)
DESC_BYTES = 192   # srtm::SeqDesc: 15 pointers, N, tile0, ws_off, L, smoother, B, u, nu, tv, Cs_fast, nx, ny
OFF_NX = 184


def _seqs_ex(specs, base=0x200000):
    """srtm_seq_ex entries (nx, ny, L, N, kind) with fake, 16-byte aligned addresses."""
    arr = (srtm.SeqExC * len(specs))()
    a = base
    for j, (nx, ny, Lw, N, kind) in enumerate(specs):
        e = arr[j]
        for k in ("F", "Q", "H", "R", "m0", "P0", "y", "ms_fast", "Ps_fast", "ms_slow", "Ps_slow"):
            setattr(e, k, a)
            a += 4096
        e.nx, e.ny, e.L, e.N, e.reserved = nx, ny, Lw, N, 0
        e.per_window = 1 if kind == "tv" else 0
        if kind == "inputs":
            e.B, e.u, e.nu = a, a + 4096, 2
            a += 8192
    return arr


def _plan_ex(arr, dtype=1, table=None, nbytes=0):
    t, w = ctypes.c_size_t(0), ctypes.c_size_t(0)
    nt, ml = ctypes.c_int64(0), ctypes.c_int32(0)
    code = srtm.lib().srtm_batch_plan_ex(dtype, arr, len(arr), table, nbytes, ctypes.byref(t), ctypes.byref(w),
                                         ctypes.byref(nt), ctypes.byref(ml))
    return code, t.value, w.value, nt.value, ml.value


MIXED = [(2, 1, 5, 300, "plain"), (4, 2, 10, 700, "inputs"), (6, 1, 20, 1, "plain"), (3, 2, 7, 257, "tv"),
         (1, 1, 3, 5000, "plain")]


def test_batch_plan_ex_sizes_descriptors_and_tile_map(L):
    arr = _seqs_ex(MIXED)
    code, tsz, wsz, nt, ml = _plan_ex(arr)
    assert code == 0 and ml == 20
    assert nt == sum((N + 255) // 256 for *_, N, _ in MIXED)
    want = 0
    for nx, ny, Lw, N, kind in MIXED:
        sh = srtm.Shape(nx, ny, Lw, 1, N)
        b = ctypes.c_size_t(0)
        fn = {"plain": L.srtm_workspace_size, "inputs": L.srtm_workspace_size_inputs,
              "tv": L.srtm_workspace_size_tv}[kind]
        assert fn(ctypes.byref(sh), 1, ctypes.byref(b)) == 0
        want += (b.value + 255) // 256 * 256
    assert wsz == want
    assert tsz == (len(MIXED) * DESC_BYTES + 15) // 16 * 16 + 4 * nt
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan_ex(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    for j, (nx, ny, *_rest) in enumerate(MIXED):
        assert ctypes.c_int32.from_buffer(buf, j * DESC_BYTES + OFF_NX).value == nx
        assert ctypes.c_int32.from_buffer(buf, j * DESC_BYTES + OFF_NX + 4).value == ny
    tile_map = (ctypes.c_int32 * nt).from_buffer(buf, tsz - 4 * nt)
    assert list(tile_map) == [j for j, (*_, N, _) in enumerate(MIXED) for _ in range((N + 255) // 256)]


@pytest.mark.parametrize("mutate,code", [
    (lambda a: setattr(a[2], "per_window", 1), 4),                # per-window models: nx <= 4
    (lambda a: setattr(a[1], "per_window", 1), 2),                # per-window model with inputs
    (lambda a: setattr(a[1], "nu", 0), 2),
    (lambda a: setattr(a[1], "nu", 5), 2),
    (lambda a: setattr(a[1], "u", None), 1),
    (lambda a: setattr(a[0], "nx", 5), 4),                        # pair not compiled
    (lambda a: setattr(a[0], "reserved", 3), 2),
    (lambda a: setattr(a[3], "per_window", 2), 2),
    (lambda a: setattr(a[4], "N", 0), 2),
    (lambda a: setattr(a[1], "B", 0x200008), 5),
    (lambda a: setattr(a[0], "F", None), 1),
])
def test_batch_plan_ex_errors(L, mutate, code):
    arr = _seqs_ex(MIXED)
    mutate(arr)
    assert _plan_ex(arr)[0] == code
    assert _plan_ex(_seqs_ex(MIXED), dtype=7)[0] == 3


def test_smooth_batch_ex_host_validation(L):
    _no_gpu()
    arr = _seqs_ex(MIXED)
    _, tsz, wsz, nt, _ = _plan_ex(arr)
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan_ex(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    host = ctypes.cast(buf, ctypes.c_void_p)
    dev, ws = ctypes.c_void_p(0x4000000), ctypes.c_void_p(0x8000000)
    n = len(MIXED)
    assert L.srtm_smooth_batch_ex(1, n, host, dev, ws, wsz - 256, None, None) == 6
    assert L.srtm_smooth_batch_ex(1, n, None, dev, ws, wsz, None, None) == 1
    assert L.srtm_smooth_batch_ex(1, n, host, ctypes.c_void_p(0x4000008), ws, wsz, None, None) == 5
    assert L.srtm_smooth_batch_ex(5, n, host, dev, ws, wsz, None, None) == 3
    # a per-window descriptor whose nx the per-window path does not take
    ctypes.c_int32.from_buffer(buf, 3 * DESC_BYTES + OFF_NX).value = 6
    assert L.srtm_smooth_batch_ex(1, n, host, dev, ws, wsz, None, None) in (2, 4, 6)
    ctypes.c_int32.from_buffer(buf, 3 * DESC_BYTES + OFF_NX).value = 3
    tile_map = (ctypes.c_int32 * nt).from_buffer(buf, tsz - 4 * nt)
    tile_map[0] = 2
    assert L.srtm_smooth_batch_ex(1, n, host, dev, ws, wsz, None, None) == 2


@pytest.mark.parametrize("field,value,code", [(0, 0, 1), (6, 0, 1), (6, 0x200008, 5), (8, 0x200004, 5)],
                         ids=["F-null", "y-null", "y-misaligned", "Ps_fast-misaligned"])
def test_batch_launch_rechecks_descriptor_arrays(L, field, value, code):
    """Both batch entry points check each descriptor's arrays again at launch: a table edited
    after planning (a required array removed, an array moved off 16-byte alignment) is refused
    before anything is enqueued. Descriptor pointer j sits at byte 8 j (F, Q, H, R, m0, P0, y, then
    the outputs)."""
    _no_gpu()
    dev, ws = ctypes.c_void_p(0x4000000), ctypes.c_void_p(0x8000000)
    # per-pair batch
    arr = _seqs([(300, 5), (600, 7)])
    _, tsz, wsz, _, _ = _plan(arr)
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    ctypes.c_uint64.from_buffer(buf, 8 * field).value = value
    assert L.srtm_smooth_batch(4, 2, 1, 2, ctypes.cast(buf, ctypes.c_void_p), dev, ws, wsz, None, None) == code
    # mixed batch: the second descriptor
    arr = _seqs_ex(MIXED)
    _, tsz, wsz, _, _ = _plan_ex(arr)
    buf = (ctypes.c_uint8 * tsz)()
    assert _plan_ex(arr, table=ctypes.cast(buf, ctypes.c_void_p), nbytes=tsz)[0] == 0
    ctypes.c_uint64.from_buffer(buf, DESC_BYTES + 8 * field).value = value
    assert L.srtm_smooth_batch_ex(1, len(MIXED), ctypes.cast(buf, ctypes.c_void_p), dev, ws, wsz, None, None) == code


def test_graph_entry_points_validate(L):
    h = ctypes.c_void_p()
    assert L.srtm_graph_begin(None) == 1
    assert L.srtm_graph_end(None, ctypes.byref(h)) == 1
    assert L.srtm_graph_launch(None, None) == 1
    assert L.srtm_graph_destroy(None) == 1


def test_loglik_grad_inputs_requires_inputs(L):
    _no_gpu()
    sh = srtm.Shape(4, 2, 5, 1, 100)
    fake = [ctypes.c_void_p(0x100000 + 4096 * j) for j in range(11)]
    assert L.srtm_loglik_grad_inputs(ctypes.byref(sh), None, *fake, ctypes.c_void_p(0x800000), 1 << 30, None,
                                     None) == 1
    bad = srtm.InputsC(0x300000, 0x310000, 0, 0)  # nu = 0
    assert L.srtm_loglik_grad_inputs(ctypes.byref(sh), ctypes.byref(bad), *fake, ctypes.c_void_p(0x800000),
                                     1 << 30, None, None) == 2
