"""srtm_smooth_noalloc (the smoother with the library's fixed per-GPU scratch as its workspace)
against srtm_smooth with a caller workspace: the same kernels on the same tiles, so every output
must be bitwise equal. Two calls in a row, the second on a smaller problem (the scratch keeps the
first call's contents), in both precisions; a problem above the scratch limit is refused before
anything is enqueued.
"""
import numpy as np
import pytest

from paper_2410_00627_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow", "mf_fast", "Pf_fast", "mf_slow", "Pf_slow")


def _srtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_00627_amd import srtm
    srtm.lib()
    return srtm


def _outputs(N, L, nx, dt):
    dev = "cuda"
    o = {}
    for p in ("s", "f"):
        o[f"m{p}_fast"] = torch.full((N, L, nx), np.nan, device=dev, dtype=dt)
        o[f"P{p}_fast"] = torch.full((N, L, nx, nx), np.nan, device=dev, dtype=dt)
        o[f"m{p}_slow"] = torch.full((N, nx), np.nan, device=dev, dtype=dt)
        o[f"P{p}_slow"] = torch.full((N, nx, nx), np.nan, device=dev, dtype=dt)
    return o


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_noalloc_equals_smooth_two_calls(dtype):
    srtm = _srtm()
    for N, seed in ((3000, 1), (700, 2)):   # the second call is smaller than the first
        m = wl.random_stable_model(4, 2, 20, 300 + seed)
        y = wl.simulate(m, N, 310 + seed)
        F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", dtype)
        yt = torch.as_tensor(y, dtype=torch.float64).to("cuda", dtype)
        print(f"[gpu] noalloc N={N} dtype={dtype}", flush=True)
        ref = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt, with_filter=True)
        out = _outputs(N, m.L, m.nx, dtype)
        info = torch.zeros(1, device="cuda", dtype=torch.int32)
        code = srtm.smooth_noalloc(F, Q, H, R, m.L, m0, P0, yt, out, info)
        torch.cuda.synchronize()
        assert code == 0, srtm.status_string(code)
        assert int(info.item()) == 0
        for k in KEYS:
            assert torch.equal(out[k], ref[k]), f"N={N}: {k} differs from srtm_smooth"


def test_noalloc_largest_headline_shape_and_limit():
    """The long-sequence shape (nx=4, ny=2, L=20, N=2^17, float64) fits the scratch; a problem
    whose workspace exceeds it is refused with SRTM_E_SCRATCH and leaves the outputs untouched."""
    srtm = _srtm()
    m = wl.headline_model()
    N = wl.HEADLINE_N
    assert srtm.workspace_size(4, 2, 20, N, torch.float64, True) <= srtm.NOALLOC_SCRATCH_BYTES
    y = wl.simulate(m, N, seed=2024)
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", torch.float64)
    yt = torch.as_tensor(y, device="cuda")
    print(f"[gpu] noalloc headline N={N}", flush=True)
    ref = srtm.smooth(F, Q, H, R, m.L, m0, P0, yt)
    out = {k: torch.empty_like(ref[k]) for k in ("ms_fast", "Ps_fast", "ms_slow", "Ps_slow")}
    info = torch.zeros(1, device="cuda", dtype=torch.int32)
    assert srtm.smooth_noalloc(F, Q, H, R, m.L, m0, P0, yt, out, info) == 0
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    for k in out:
        assert torch.equal(out[k], ref[k]), k
    big = 2 * N
    assert srtm.workspace_size(4, 2, 20, big, torch.float64, True) > srtm.NOALLOC_SCRATCH_BYTES
    yb = torch.zeros((big, 2), device="cuda", dtype=torch.float64)
    ob = {"ms_slow": torch.full((big, 4), 7.0, device="cuda", dtype=torch.float64)}
    info.zero_()
    assert srtm.smooth_noalloc(F, Q, H, R, m.L, m0, P0, yb, ob, info) == 8   # SRTM_E_SCRATCH
    torch.cuda.synchronize()
    assert bool((ob["ms_slow"] == 7.0).all()) and int(info.item()) == 0
