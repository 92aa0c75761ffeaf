"""GPU parity: the HIP path (through the C ABI) against the float64 CPU reference.

Tolerances (relative, per fast state, metric of conftest.rel_errors): 1e-8 for the
float64 path, 1e-3 for the float32 path. The float32 path is compared with the
reference evaluated on the float32-rounded inputs.
"""
import numpy as np
import pytest

import oracle
from paper_2410_00627_amd import workloads as wl
from conftest import assert_close_states, rel_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-8, torch.float32: 1e-3}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_00627_amd import srtm
    srtm.lib()
    return srtm


def _rounded(model, y, dtype):
    if dtype == torch.float64:
        return model, y
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    m = wl.Model(r(model.A), r(model.Q), r(model.C), r(model.R), model.L, r(model.m0), r(model.P0), model.name)
    return m, r(y)


def _args(m):
    return (m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0)


def run_gpu(model, y, dtype, *, filter_only=False, with_filter=True):
    srtm = _need_gpu()
    F, Q, H, R, m0, P0 = srtm.model_tensors(model, "cuda", dtype)
    yt = torch.as_tensor(y, dtype=torch.float64).to("cuda", dtype)
    print(f"[gpu] {'filter' if filter_only else 'smooth'} nx={model.nx} ny={model.ny} L={model.L} "
          f"N={y.shape[0]} dtype={dtype}", flush=True)
    if filter_only:
        out = srtm.filter(F, Q, H, R, model.L, m0, P0, yt)
    else:
        out = srtm.smooth(F, Q, H, R, model.L, m0, P0, yt, with_filter=with_filter)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in out.items()}


def check_smoother(model, y, dtype, what=""):
    out = run_gpu(model, y, dtype)
    mr, yr = _rounded(model, y, dtype)
    ref = oracle.srtm_smoother(*_args(mr), yr, with_filter=True)
    tol = TOL[dtype]
    assert int(out["info"][0]) == 0
    assert_close_states(out["ms_fast"], out["Ps_fast"], ref["ms_fast"], ref["Ps_fast"], tol, what + " smoothed fast")
    assert_close_states(out["ms_slow"], out["Ps_slow"], ref["ms_slow"], ref["Ps_slow"], tol, what + " smoothed slow")
    assert_close_states(out["mf_fast"], out["Pf_fast"], ref["m_fast"], ref["P_fast"], tol, what + " filtered fast")
    assert_close_states(out["mf_slow"], out["Pf_slow"], ref["m_slow"], ref["P_slow"], tol, what + " filtered slow")
    for k in ("Ps_fast", "Pf_fast", "Ps_slow", "Pf_slow"):
        assert np.array_equal(out[k], np.swapaxes(out[k], -1, -2)), f"{k} not exactly symmetric"
    return out, ref


# ----------------------------------------------------------------------------- tiny case
@pytest.mark.parametrize("dtype", [torch.float64])
def test_wna_tiny(dtype):
    """Position/velocity model, l = 10, N = 100 (the tiny float64 case)."""
    m = wl.wna_model()
    y = wl.simulate(m, wl.WNA_N, seed=1)
    check_smoother(m, y, dtype, "wna")


# ----------------------------------------------------------------------------- shapes
CASES = [
    # nx, ny, L, N, seed  -- N spans several 256-window tiles with a ragged tail
    (4, 2, 20, 845, 1),
    (2, 1, 10, 600, 2),
    (3, 2, 7, 300, 3),
    (4, 1, 5, 1100, 4),
    (1, 1, 3, 513, 5),
    (2, 2, 1, 700, 6),      # l = 1: Kalman filter + RTS smoother
    (3, 1, 16, 257, 7),
    (6, 1, 5, 300, 8),      # nx > 4: Gaussian elimination instead of the adjugate
    (4, 2, 2, 400, 9),      # l = 2: one power of A and one cross term per window
]


@pytest.mark.parametrize("nx,ny,L,N,seed", CASES, ids=[f"nx{c[0]}ny{c[1]}L{c[2]}N{c[3]}" for c in CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_parity_shapes(nx, ny, L, N, seed, dtype):
    m = wl.random_stable_model(nx, ny, L, seed)
    y = wl.simulate(m, N, seed + 50)
    check_smoother(m, y, dtype, f"nx{nx} ny{ny} L{L} N{N}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_parity_one_tile_per_scan_lane(dtype):
    """201 tiles (the last one ragged): one tile per lane of the tile-level scans and all eight of
    their steps, the early ones with wave 0's vector runs kept by wave 1; every window against the
    reference."""
    m = wl.random_stable_model(2, 1, 2, 11)
    y = wl.simulate(m, 200 * 256 + 37, 12)
    check_smoother(m, y, dtype, "201 tiles")


def test_parity_chunk_fold_float32():
    """514 tiles in float32: past 512 tiles each lane of the tile-level scans first folds a chunk of
    four tiles with full element combines; every window against the reference (float64:
    test_many_tiles_general_paths)."""
    m = wl.random_stable_model(1, 1, 1, 13)
    y = wl.simulate(m, 512 * 256 + 300, 14)
    check_smoother(m, y, torch.float32, "514 tiles")


@pytest.mark.parametrize("N", [1, 2, 3, 255, 256, 257, 512, 513])
def test_edge_lengths(N):
    m = wl.random_general_model(3, 2, 4, 11)
    y = wl.simulate(m, N, 12)
    check_smoother(m, y, torch.float64, f"N={N}")


def test_many_tiles_general_paths():
    """N = 140000 windows (547 tiles of 256): each lane of the tile-level scans folds a chunk of
    four tiles with full element combines first (float64)."""
    m = wl.random_stable_model(2, 1, 3, 61)
    y = wl.simulate(m, 140000, 62)
    check_smoother(m, y, torch.float64, "N=140000")


def test_general_model_nonzero_prior():
    """Non-orthogonal A, full Q, R, P0 and nonzero m0."""
    m = wl.random_general_model(4, 2, 6, 21)
    y = wl.simulate(m, 400, 22)
    check_smoother(m, y, torch.float64, "general")


def test_filter_entry_point_matches_smoother_filter_outputs():
    m = wl.random_stable_model(4, 2, 20, 31)
    y = wl.simulate(m, 300, 32)
    f = run_gpu(m, y, torch.float64, filter_only=True)
    ref = oracle.srtm_filter(*_args(m), y)
    assert_close_states(f["m_fast"], f["P_fast"], ref["m_fast"], ref["P_fast"], 1e-8, "srtm_filter fast")
    assert_close_states(f["m_slow"], f["P_slow"], ref["m_slow"], ref["P_slow"], 1e-8, "srtm_filter slow")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_bitwise_deterministic(dtype):
    m = wl.random_stable_model(4, 2, 20, 41)
    y = wl.simulate(m, 1000, 42)
    a = run_gpu(m, y, dtype)
    b = run_gpu(m, y, dtype)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_profiled_call_times_each_kernel_and_keeps_the_outputs(dtype):
    """srtm_smooth with per-kernel events (the profiled entry point bench.py times with) gives
    bitwise the outputs of the plain call; every stage's interval is positive, each starts no
    earlier than the previous one ends, and the call's span covers their sum."""
    srtm = _need_gpu()
    from paper_2410_00627_amd.hip_events import EventArray
    import ctypes
    m = wl.random_stable_model(4, 2, 20, 77)
    y = wl.simulate(m, 2000, 78)
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", dtype)
    yt = torch.as_tensor(y, dtype=torch.float64).to("cuda", dtype)
    plain = srtm.smooth(F, Q, H, R, 20, m0, P0, yt)
    names = srtm.kernel_names(True)
    ev = EventArray(2 * len(names))
    print(f"[gpu] profiled call, {len(names)} stages, dtype={dtype}", flush=True)
    prof = srtm.smooth(F, Q, H, R, 20, m0, P0, yt, events=(ctypes.c_void_p * len(ev))(*ev.arr))
    torch.cuda.synchronize()
    for k in plain:
        assert torch.equal(plain[k], prof[k]), k
    dur = [ev.elapsed_ms(2 * j, 2 * j + 1) for j in range(len(names))]
    gaps = [ev.elapsed_ms(2 * j - 1, 2 * j) for j in range(1, len(names))]
    span = ev.elapsed_ms(0, 2 * len(names) - 1)
    ev.close()
    print(f"[gpu]   stages (ms) {dict(zip(names, [round(d, 4) for d in dur]))}, span {span:.4f}", flush=True)
    assert all(d > 0 for d in dur)
    assert all(g >= -1e-3 for g in gaps)
    assert span >= sum(dur) - 1e-3


def test_info_flags_forced_from_host():
    """Conditions forced through the inputs (kernels still exit normally)."""
    srtm = _need_gpu()
    m = wl.random_stable_model(2, 1, 4, 51)
    y = wl.simulate(m, 300, 52)
    y[100, 0] = np.nan
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", torch.float64)
    yt = torch.as_tensor(y, device="cuda")
    out = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, check=False)
    torch.cuda.synchronize()
    assert int(out["info"].item()) & 8
    with pytest.raises(srtm.SrtmError):
        srtm.smooth(F, Q, H, R, m.L, m0, P0, yt)
    # zero measurement noise and a zero measurement matrix: innovation covariance is 0
    Z = torch.zeros_like(R)
    out = srtm.smooth(F, Q, torch.zeros_like(H), Z, m.L, m0, P0, torch.zeros_like(yt), check=False)
    torch.cuda.synchronize()
    assert int(out["info"].item()) & 1


# ----------------------------------------------------------------------------- full size
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_headline_full_size(dtype):
    """One long sequence, nx=4, ny=2, L=20, N=2^17 (2,621,440 fast states), in the benchmark's
    launch configuration: every window of every output (smoothed and filtered, fast and slow
    rate) against the reference's sequential smoother over the whole sequence, element by
    element, at 1e-8 (float64) or 1e-3 (float32, reference on the rounded inputs). This is the
    float32 path with more than 256 tiles (the chunked tile-level scans)."""
    from threadpoolctl import threadpool_limits
    m = wl.headline_model()
    N = wl.HEADLINE_N
    y = wl.simulate(m, N, seed=2024)
    out = run_gpu(m, y, dtype)
    assert int(out["info"][0]) == 0
    mr, yr = _rounded(m, y, dtype)
    with threadpool_limits(limits=1):
        ref = oracle.srtm_smoother(*_args(mr), yr, with_filter=True)
    tol = TOL[dtype]
    worst = {}
    for mk, pk, rm, rp in (("ms_fast", "Ps_fast", "ms_fast", "Ps_fast"), ("ms_slow", "Ps_slow", "ms_slow", "Ps_slow"),
                           ("mf_fast", "Pf_fast", "m_fast", "P_fast"), ("mf_slow", "Pf_slow", "m_slow", "P_slow")):
        worst[mk] = assert_close_states(out[mk], out[pk], ref[rm], ref[rp], tol, f"headline {mk}/{pk}, all windows")
    print(f"[gpu] headline {dtype}: max errors (mean, cov) over all windows {worst}", flush=True)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_filter_entry_point_full_size(dtype):
    """srtm_filter on the long-sequence shape (nx=4, ny=2, L=20, N=2^17): every window of the
    fast- and slow-rate filter outputs against the reference filter (IMKF and dense window
    filter) over the whole sequence."""
    from threadpoolctl import threadpool_limits
    m = wl.headline_model()
    N = wl.HEADLINE_N
    y = wl.simulate(m, N, seed=2031)
    out = run_gpu(m, y, dtype, filter_only=True)
    assert int(out["info"][0]) == 0
    mr, yr = _rounded(m, y, dtype)
    tol = TOL[dtype]
    with threadpool_limits(limits=1):
        ref = oracle.srtm_filter(*_args(mr), yr)
    assert_close_states(out["m_slow"], out["P_slow"], ref["m_slow"], ref["P_slow"], tol, "srtm_filter slow, all windows")
    assert_close_states(out["m_fast"], out["P_fast"], ref["m_fast"], ref["P_fast"], tol, "srtm_filter fast, all windows")


@pytest.mark.parametrize("nx,ny,L,N", [(4, 2, 128, 12), (6, 1, 128, 10), (1, 1, 128, 300)],
                         ids=["nx4ny2L128", "nx6ny1L128", "nx1ny1L128N300"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_longest_windows(nx, ny, L, N, dtype):
    """The longest window the build accepts (L = 128; for nx = 6 the constants kernel's LDS tables
    are then within 3 KiB of the 160 KiB limit)."""
    m = wl.random_stable_model(nx, ny, L, 70 + nx)
    y = wl.simulate(m, N, 71 + nx)
    check_smoother(m, y, dtype, f"nx{nx} ny{ny} L{L} N{N}")


def test_largest_sequence():
    """N = 2^26 windows (the build's maximum; l = 1, nx = ny = 1, float64): the chunked tile
    scans at their deepest (1024 tiles per Kogge-Stone lane). Checked: the first 2000 windows'
    filter against the sequential IMKF from the prior; at sampled windows one IMKF step from the
    GPU's carry of the previous window and one smoother step from the GPU's smoothed state of
    the next; the last 16 windows against the smoother started from the GPU's carry."""
    srtm = _need_gpu()
    N = 1 << 26
    m = wl.random_stable_model(1, 1, 1, 91)
    y = wl.simulate(m, N, 92)
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", torch.float64)
    yt = torch.as_tensor(y, device="cuda")
    out = {"ms_fast": torch.empty(N, 1, 1, device="cuda", dtype=torch.float64)}
    out["Ps_fast"] = torch.empty(N, 1, 1, 1, device="cuda", dtype=torch.float64)
    out["mf_slow"] = torch.empty(N, 1, device="cuda", dtype=torch.float64)
    out["Pf_slow"] = torch.empty(N, 1, 1, device="cuda", dtype=torch.float64)
    print(f"[gpu] largest sequence N={N}", flush=True)
    o = srtm.smooth(F, Q, H, R, 1, m0, P0, yt, out=out)
    torch.cuda.synchronize()
    assert int(o["info"][0]) == 0
    ms, Ps = o["ms_fast"][:, 0].cpu().numpy(), o["Ps_fast"][:, 0].cpu().numpy()
    mf, Pf = o["mf_slow"].cpu().numpy(), o["Pf_slow"].cpu().numpy()
    head_m, head_P, _ = oracle.imkf(m.A, m.Q, m.C, m.R, 1, m.m0, m.P0, y[:2000])
    assert_close_states(mf[:2000], Pf[:2000], head_m, head_P, 1e-8, "filter head")
    rng = np.random.default_rng(93)
    for k in sorted(set(rng.integers(1, N - 1, 40).tolist()) | {1 << 18, (1 << 26) - 2}):
        one_m, one_P, _ = oracle.imkf(m.A, m.Q, m.C, m.R, 1, mf[k - 1], Pf[k - 1], y[k:k + 1])
        assert_close_states(mf[k:k + 1], Pf[k:k + 1], one_m, one_P, 1e-8, f"filter step {k}")
        # RTS step (l = 1): G = P A^T (A P A^T + Q)^{-1}
        Pp = m.A @ Pf[k] @ m.A.T + m.Q
        G = Pf[k] @ m.A.T @ np.linalg.inv(Pp)
        m_s = mf[k] + G @ (ms[k + 1] - m.A @ mf[k])
        P_s = Pf[k] + G @ (Ps[k + 1] - Pp) @ G.T
        assert_close_states(ms[k:k + 1], Ps[k:k + 1], m_s[None], P_s[None], 1e-8, f"smoother step {k}")
    n = 16
    tail = oracle.srtm_smoother(m.A, m.Q, m.C, m.R, 1, mf[N - n - 1], Pf[N - n - 1], y[N - n:])
    assert_close_states(ms[N - n:], Ps[N - n:], tail["ms_fast"][:, 0], tail["Ps_fast"][:, 0], 1e-8, "tail")
